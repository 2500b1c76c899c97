"""sos_loss_grad_noalloc (the library's static device workspace, no
allocation) against sos_loss_grad (a caller workspace), through the C ABI.

Both run the same kernels on the same W and p.  Each result is checked
against the FP64 oracle under the parity bounds of the plan's precision
(relative to cabs = coeff(|W||W|^T) and gabs = 4 |R| |W|, as in the parity
tests), and the two entry points against each other under the sum of their
two bounds (they may differ only in the order of the forward's FP64 atomic
adds and what that order does to later roundings).  Two calls in a row,
the second on a smaller problem, check that the shared workspace keeps
nothing from the previous call that a later call would read.
"""
import math
from math import comb

import numpy as np
import pytest

import oracle as O
from workloads import gaussian

torch = pytest.importorskip("torch")
S = pytest.importorskip("paper_2410_19844_amd")

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def gamma(n):
    return n * U32 / (1 - n * U32)


def tol_for(prec, K, single=False):
    if prec == "fp64":
        return 1e-10
    if prec == "fp32":
        return gamma(K + 1) + U32
    if single:
        return 2.0 ** -7 + 2.0 ** -16 + gamma(K) + U32
    return 3.1 * 2.0 ** -16 + gamma(3 * K) + U32


def case(n, d, k, prec, seed):
    N, M = comb(n + d, d), comb(n + 2 * d, 2 * d)
    W = gaussian((N, k), 300 + seed, 1.0 / math.sqrt(k))
    wdt = torch.float64 if prec == "fp64" else torch.float32
    Wd = torch.tensor(W, dtype=wdt, device="cuda")
    p = gaussian(M, 400 + seed)
    return Wd, Wd.double().cpu().numpy(), p, torch.tensor(p, dtype=torch.float64, device="cuda")


def bounds(W64, p, n, d, prec, exact, single):
    pr = O.pair_ranks(n, d)
    L_o, g_o, r_o = O.loss_grad(W64, p, n, d, pr)
    cabs = O.coefficients_abs(W64, n, d, pr)
    N, k = W64.shape
    tf = 1e-10 if exact else tol_for(prec, k)
    tb = tol_for(prec, N, single)
    dc = tf * cabs
    dL = 2.0 * np.sum(np.abs(r_o) * dc) + np.sum(dc * dc) + 1e-12 * L_o
    Wa = np.abs(W64)
    dg = tb * 4.0 * (np.abs(r_o)[pr] @ Wa) + 4.0 * (dc[pr] @ Wa) + 1e-300
    return L_o, g_o, r_o, dc + 1e-300, dL, dg


def run_pair(n, d, k, prec, seed, exact=False, single=False):
    Wd, W64, p, pd = case(n, d, k, prec, seed)
    free = S.Plan(n, d, k, prec, bind=False)
    assert free.ws is None
    loss_a = torch.empty(1, dtype=torch.float64, device="cuda")
    g_a = torch.empty_like(Wd)
    r_a = torch.empty(free.M, dtype=torch.float64, device="cuda")
    free.loss_grad_noalloc(Wd, pd, loss_a, g_a, r_a, exact=exact, single_backward=single)
    bound = S.Plan(n, d, k, prec)
    loss_b, g_b, r_b = bound.loss_grad(Wd, pd, grad=True, want_r=True, exact=exact, single_backward=single)
    torch.cuda.synchronize()
    L_o, g_o, r_o, dc, dL, dg = bounds(W64, p, n, d, prec, exact, single)
    got = {"a": (loss_a.item(), g_a.double().cpu().numpy(), r_a.cpu().numpy()),
           "b": (loss_b.item(), g_b.double().cpu().numpy(), r_b.cpu().numpy())}
    for name, (L, g, r) in got.items():
        assert abs(L - L_o) <= dL, (name, L, L_o)
        assert np.max(np.abs(r - r_o) / dc) <= 1.0, (name, "residual")
        assert np.max(np.abs(g - g_o) / dg) <= 1.0, (name, "gradient")
    La, ga, ra = got["a"]
    Lb, gb, rb = got["b"]
    assert abs(La - Lb) <= 2 * dL
    assert np.max(np.abs(ra - rb) / (2 * dc)) <= 1.0
    assert np.max(np.abs(ga - gb) / (2 * dg)) <= 1.0
    return free


@pytest.mark.parametrize("prec,exact,single", [("fp32", False, False), ("bf16x3", False, True),
                                               ("bf16x3", True, True), ("fp64", False, False)])
def test_noalloc_matches_bound_entry_point_twice(prec, exact, single):
    # a larger problem, then a smaller one on the same static workspace
    run_pair(6, 4, 420, prec, seed=1, exact=exact, single=single)
    run_pair(4, 3, 37, prec, seed=2, exact=exact, single=single)


def test_noalloc_rejects_bound_plan_and_forward_only():
    n, d, k = 3, 2, 20
    Wd, W64, p, pd = case(n, d, k, "fp32", 5)
    bound = S.Plan(n, d, k, "fp32")
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    with pytest.raises(S.SosError) as e:
        bound.loss_grad_noalloc(Wd, pd, loss)
    assert e.value.code == S.EINVAL
    # forward only (no gradient, no residual): the loss alone
    free = S.Plan(n, d, k, "fp32", bind=False)
    free.loss_grad_noalloc(Wd, pd, loss)
    L_o, _, _ = O.loss_grad(W64, p, n, d)
    assert abs(loss.item() - L_o) <= 1e-4 * L_o
