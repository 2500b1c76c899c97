"""SOS_FP16X3: the split engine with fp16 halves, against the FP64 oracle.

Bounds.  The W copies hold 2^sW w with 2^sW max|W| < 2^12, and R holds
2^sR fp32(r) with 2^sR max|r| < 2^14 (exponents recomputed here with NumPy's
frexp from the same definitions).  A scaled operand x is split as
hi = fp16(x), lo = fp16(x - hi); in fp16's normal range each rounding loses
at most 2^-11 relative, below it at most 2^-25 absolute (half the subnormal
spacing), so |x - hi - lo| <= 2^-22 |x| + 2^-25.  The three kept products
leave out lo lo' and the split errors:

  per product, unscaled:  3.1 2^-22 |w w'| + 2^-24 (2^-s |w'| + 2^-s' |w|),

and the FP32 accumulation of 3K products adds gamma(3K) of the absolute
sum.  Per coefficient that is (3.1 2^-22 + gamma(3K) + u) coeff(|W||W|^T)
plus 2^-24 2^-sW times the pair sum of the row sums of |W|.  The single
product backward (hi * hi) has 2^-10 + 2^-22 relative per term (both
operands rounded to 11 bits) instead of 3.1 2^-22, and the forward's error
reaches the gradient through 4 |dR| |W|.
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


def scale_exp(m, top):
    """s with m 2^s < 2^top (0 for m = 0), clamped like the library."""
    if not m > 0:
        return 0
    _, e = math.frexp(m)
    return max(-100, min(100, top - e))


def pair_sum(v, pr):
    """coefficient-wise sum over ordered pairs (i, j) of v_i + v_j."""
    return np.bincount(pr.ravel(), weights=(v[:, None] + v[None, :]).ravel(), minlength=int(pr.max()) + 1)


CASES = [(3, 2, 20), (4, 3, 37), (6, 3, 168), (6, 4, 420), (10, 5, 300), (17, 2, 40), (40, 2, 130)]


@pytest.mark.parametrize("single", [False, True])
@pytest.mark.parametrize("n,d,k", CASES)
def test_fp16x3_loss_grad_parity(n, d, k, single):
    N, M = comb(n + d, d), comb(n + 2 * d, 2 * d)
    Wd = torch.tensor(gaussian((N, k), 900 + n, 1 / math.sqrt(k)), dtype=torch.float32, device="cuda")
    p = gaussian(M, 910 + n)
    pd = torch.tensor(p, dtype=torch.float64, device="cuda")
    pl = S.Plan(n, d, k, "fp16x3")
    loss, g, r = pl.loss_grad(Wd, pd, grad=True, want_r=True, single_backward=single)
    W64 = Wd.double().cpu().numpy()
    pr = O.pair_ranks(n, d)
    L_o, g_o, r_o = O.loss_grad(W64, p, n, d, pr)
    cabs = O.coefficients_abs(W64, n, d, pr)
    Wa = np.abs(W64)
    sW = scale_exp(float(Wa.max()), 12)
    dc = ((3.1 * 2.0 ** -22 + gamma(3 * k) + U32) * cabs + 2.0 ** (-24 - sW) * pair_sum(Wa.sum(1), pr)
          + 1e-15 * np.abs(p) + 1e-300)
    err = np.abs(r.cpu().numpy() - r_o)
    assert np.max(err / dc) <= 1.0, np.max(err / dc)
    # far inside that bound: the split keeps ~22 bits, the FP32 sums ~1e-7 relative
    assert np.max(err / (1e-5 * cabs + 1e-15 * np.abs(p) + 1e-300)) <= 1.0
    dL = 2.0 * np.sum(np.abs(r_o) * dc) + np.sum(dc * dc)
    assert abs(loss.item() - L_o) <= dL + 1e-12 * L_o
    # backward
    R = np.abs(r_o)[pr]
    sR = scale_exp(float(np.abs(r_o).max()) * (1 + 1e-6), 14) - 1   # one binade of slack for r's rounding
    tb = (2.0 ** -10 + 2.0 ** -22 + gamma(N) + 2 * U32) if single else (3.1 * 2.0 ** -22 + gamma(3 * N) + 2 * U32)
    bound = 4.0 * (tb * (R @ Wa) + 2.0 ** (-24 - sR) * Wa.sum(0)[None, :]
                   + 2.0 ** (-24 - sW) * R.sum(1)[:, None]) + 4.0 * (dc[pr] @ Wa) + 1e-300
    gerr = np.abs(g.double().cpu().numpy() - g_o)
    assert np.max(gerr / bound) <= 1.0, np.max(gerr / bound)


def test_fp16x3_backward_more_accurate_than_bf16():
    """One fp16 product per term keeps 11 bits of each operand against
    bf16's 8: the single-product gradient's error shrinks about 8x."""
    n, d, k = 6, 4, 420
    N, M = comb(n + d, d), comb(n + 2 * d, 2 * d)
    Wd = torch.tensor(gaussian((N, k), 5, 1 / math.sqrt(k)), dtype=torch.float32, device="cuda")
    p = gaussian(M, 6)
    pd = torch.tensor(p, dtype=torch.float64, device="cuda")
    _, g_o, _ = O.loss_grad(Wd.double().cpu().numpy(), p, n, d)
    errs = {}
    for prec in ("bf16x3", "fp16x3"):
        _, g, _ = S.Plan(n, d, k, prec).loss_grad(Wd, pd, grad=True, single_backward=True)
        errs[prec] = float(np.linalg.norm(g.double().cpu().numpy() - g_o) / np.linalg.norm(g_o))
    assert errs["fp16x3"] * 4 <= errs["bf16x3"], errs


def test_fp16x3_fused_steps_track_unfused():
    """The single-product step runs Adam in the backward's epilogue and writes
    the next step's scaled fp16 copies there; a run of such steps must follow
    the unfused steps (fresh copies every step) to rounding."""
    n, d, k = 6, 4, 420
    N, M = comb(n + d, d), comb(n + 2 * d, 2 * d)
    pr = O.pair_ranks(n, d)
    p = O.coefficients(gaussian((N, 50), 0) / math.sqrt(50), n, d, pr)
    pd = torch.tensor(p, dtype=torch.float64, device="cuda")
    W0 = torch.tensor(gaussian((N, k), 1, 1 / math.sqrt(k)), dtype=torch.float32, device="cuda")
    adam = S.Adam(lr=3e-3)
    runs = []
    for copies in (True, False):
        pl = S.Plan(n, d, k, "fp16x3")
        W, st = W0.clone(), pl.new_state()
        L = []
        for t in range(1, 41):
            fl = S.FLAG_SINGLE_BACKWARD | (S.FLAG_COPIES_VALID if copies else 0)
            L.append(pl.step(W, st, t, pd, adam, flags=fl).item())
        runs.append((np.array(L), W))
    (La, Wa), (Lb, Wb) = runs
    assert La[-1] < 0.1 * La[0]
    assert np.max(np.abs(La - Lb) / Lb) <= 1e-3
    assert float((Wa - Wb).abs().max()) <= 1e-4 * float(Wb.abs().max())


def test_fp16x3_solve_certified_by_the_oracle():
    n, d = 6, 4
    N = comb(n + d, d)
    k = 2 * N
    pr = O.pair_ranks(n, d)
    p = O.coefficients(gaussian((N, N // 2), 0) / math.sqrt(N // 2), n, d, pr)
    pl = S.Plan(n, d, k, "fp16x3")
    Wd = torch.tensor(gaussian((N, k), 1, 1 / math.sqrt(k)), dtype=torch.float32, device="cuda")
    res = pl.solve(Wd, torch.tensor(p, dtype=torch.float64, device="cuda"), S.Adam(lr=3e-3), tol=1e-8,
                   max_steps=20000, check_every=10, ladder=True, stall_checks=6, stall_ratio=0.8,
                   switch_rel=3e-6, lr_exact=1e-3, rollback_ratio=10.0, single_backward=True)
    assert res["status"] == S.OK, res
    rel_o = float(np.linalg.norm(O.residual(Wd.double().cpu().numpy(), p, n, d, pr)) / np.linalg.norm(p))
    assert rel_o <= 1e-8 and abs(rel_o - res["rel"]) <= 1e-6 * rel_o


def test_fp16x3_scale_keeps_tiny_and_huge_rows():
    """W scaled by 2^-40 (and by 2^+40): the plan's scale exponent moves the
    copies back into fp16's range, so the relative accuracy is unchanged."""
    n, d, k = 4, 3, 37
    N, M = comb(n + d, d), comb(n + 2 * d, 2 * d)
    base = gaussian((N, k), 3, 1 / math.sqrt(k))
    pl = S.Plan(n, d, k, "fp16x3")
    for e in (-40, 40):
        W64 = base * 2.0 ** e
        Wd = torch.tensor(W64, dtype=torch.float32, device="cuda")
        W64 = Wd.double().cpu().numpy()
        p = O.coefficients(gaussian((N, 5), 4) * 2.0 ** e, n, d)
        pd = torch.tensor(p, dtype=torch.float64, device="cuda")
        _, _, r = pl.loss_grad(Wd, pd, grad=False, want_r=True)
        r_o = O.residual(W64, p, n, d)
        cabs = O.coefficients_abs(W64, n, d)
        assert np.max(np.abs(r.cpu().numpy() - r_o) / (1e-5 * cabs + 1e-300)) <= 1.0, e
