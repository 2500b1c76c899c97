"""Parity at the full n=12, d=6 size (N = k = 18,564, M = 2,704,156), in the
launch configuration the benchmark times (BF16X3 plan, single-product
backward), through the C ABI.

* Coefficients: a seeded sample of coefficient positions (plus the extreme
  ones: x1^12, with one pair, and the constant, with one pair), each summed
  pair by pair by the oracle, against c = r + p from the fast forward
  (split-bf16 bound) and from the exact forward (1e-10).
* Gradient: the oracle cannot form a full gradient row at this size in
  reasonable time (every row needs ~18,564 coefficients, each from ~127
  pair dot products of length 18,564), so the gradient is checked through
  two properties that hold at any size:
    - the directional derivative along g: L(W + hU) - L(W - hU) (exact FP64
      forward, with the FP32-rounded perturbations measured exactly) against
      <g, Wp - Wm>; L is quartic along the line, so the central difference
      is exact to O(h^2);
    - Euler's identity <grad L, W> = 4 <r, c>, since sum_ij R_ij G_ij =
      sum_b r_b c_b.
  The single-product backward rounds R and W to 8 significant bits; its
  per-term errors are random in sign, so inner products with g itself agree
  to ~2^-9 relative; the tests allow 1e-2.
"""
import math

import numpy as np
import pytest

import oracle as O
from workloads import CONFIGS, gaussian

torch = pytest.importorskip("torch")
S = pytest.importorskip("paper_2410_19844_amd")

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def gamma(n):
    return n * U32 / (1 - n * U32)


@pytest.fixture(scope="module")
def full():
    c = CONFIGS["n12d6"]
    dev = torch.device("cuda")
    Wd = torch.tensor(c.W_init(), dtype=torch.float32, device=dev)
    p = gaussian(c.M, 7)
    pd = torch.tensor(p, dtype=torch.float64, device=dev)
    pl = S.Plan(c.n, c.d, c.rank, "bf16x3")
    L_fast, g, r_fast = pl.loss_grad(Wd, pd, grad=True, want_r=True, single_backward=True)
    L_ex, _, r_ex = pl.loss_grad(Wd, pd, grad=False, want_r=True, exact=True)
    torch.cuda.synchronize()
    return dict(c=c, pl=pl, W=Wd, p=p, pd=pd, g=g, r_fast=r_fast, r_ex=r_ex,
                L_fast=float(L_fast.item()), L_ex=float(L_ex.item()))


def sample_betas(M, count=96, seed=21):
    rng = np.random.default_rng(seed)
    return np.unique(np.concatenate([[0, M - 1], rng.choice(M, count, replace=False)]))


def test_fullsize_sampled_coefficients(full):
    c, W = full["c"], full["W"]
    betas = sample_betas(c.M)
    W64 = W.double().cpu().numpy()
    basis = O.monomials(c.n, c.d)
    bidx, cidx = O.MonomialIndex(c.n, c.d), O.MonomialIndex(c.n, 2 * c.d)
    want = O.sample_coefficients(W64, c.n, c.d, betas, basis, bidx, cidx)
    cabs = O.sample_coefficients(np.abs(W64), c.n, c.d, betas, basis, bidx, cidx)
    p = full["p"][betas]
    got_fast = full["r_fast"][torch.as_tensor(betas, device=W.device)].cpu().numpy() + p
    got_ex = full["r_ex"][torch.as_tensor(betas, device=W.device)].cpu().numpy() + p
    tol_fast = 3.1 * 2.0 ** -16 + gamma(3 * c.rank) + U32
    slack = 1e-15 * np.abs(p)                       # adding p back to r
    err = np.abs(got_fast - want) / (tol_fast * cabs + slack)
    assert err.max() <= 1.0, f"fast forward: max |err|/bound {err.max():.3g}"
    err = np.abs(got_ex - want) / (1e-10 * cabs + slack)
    assert err.max() <= 1.0, f"exact forward: max |err|/bound {err.max():.3g}"


def test_fullsize_loss_matches_residual(full):
    # L is the sum of squares of the r that the same call returns (FP64, fixed order)
    for key_L, key_r in (("L_fast", "r_fast"), ("L_ex", "r_ex")):
        r = full[key_r]
        want = float(torch.dot(r, r))
        assert abs(full[key_L] - want) <= 1e-12 * want, key_L


def test_fullsize_gradient_directional_derivative(full):
    pl, W, g, pd = full["pl"], full["W"], full["g"], full["pd"]
    U = g.double() / g.abs().max().double()
    h = 1e-5
    Wp = (W.double() + h * U).float()
    Wm = (W.double() - h * U).float()
    D = Wp.double() - Wm.double()                   # exact: the perturbation actually applied
    Lp = float(pl.loss_grad(Wp, pd, grad=False, exact=True)[0].item())
    Lm = float(pl.loss_grad(Wm, pd, grad=False, exact=True)[0].item())
    fd = Lp - Lm
    lin = float(torch.sum(g.double() * D))
    assert fd > 0 and lin > 0
    assert abs(fd - lin) <= 1e-2 * abs(fd), (fd, lin)


def test_fullsize_gradient_euler_identity(full):
    W, g, r, pd = full["W"], full["g"], full["r_fast"], full["pd"]
    lhs = float(torch.sum(g.double() * W.double()))
    rhs = 4.0 * float(torch.dot(r, r + pd))
    assert abs(lhs - rhs) <= 1e-2 * abs(rhs), (lhs, rhs)


def test_fullsize_pair_ranks_sample(full):
    c, pl = full["c"], full["pl"]
    ranks = pl.pair_ranks()
    rows = np.array([0, 1, 777, c.N // 2, c.N - 2, c.N - 1])
    want = O.pair_ranks(c.n, c.d, rows=rows)
    got = ranks[torch.as_tensor(rows, device=ranks.device)].cpu().numpy()
    assert np.array_equal(got, want)
