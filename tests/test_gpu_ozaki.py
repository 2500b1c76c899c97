"""The Ozaki-split forward (SOS_FLAG_OZAKI_FORWARD: an FP64-accurate Gram
from int8 MFMA) against the FP64 oracle, through the C ABI.

Bound.  Row i of W is scaled by 2^e_i, the least power of two above its
largest magnitude, and cut into S = 6 signed 7-bit digits.  Per product
W_il W_jl the digits left out and the slice levels dropped (s + t >= S)
amount to at most (S + 1.05) 2^-7S 2^(e_i + e_j), so each Gram entry is off
by at most (S + 1.05) 2^-7S k 2^(e_i + e_j), and coefficient b by the
ordered-pair sum of that over the pairs of b:

    |c_b - c~_b| <= (S + 1.05) 2^-7S k coeff(s s^T)_b,   s_i = 2^e_i,

plus FP64 rounding (the levels are combined and the tiles scattered in
FP64 into r = -p: 1e-13 of cabs = coeff(|W||W|^T) + |p| covers it, at most
a few hundred atomic adds per coefficient here).  The exponents come from
numpy's frexp on the host, independently of the library.  The digit errors
are independent and of both signs, so the actual error is far inside this
worst case: the tests also hold it to 1e-10 of cabs, the bar of the FP64
path.

Five slices (SOS_FLAG_OZAKI_FIVE_SLICES, S = 5) keep the levels s + t < 5:
the same bound with S = 5, about 128 times the six-slice one, and a
statistical bar of 2e-9 of cabs (a CPU emulation of the split puts the
largest error on these shapes at 2.3e-10 of cabs; dropping one more level
would give ~4e-8).  Four slices (SOS_FLAG_OZAKI_FOUR_SLICES): the bound with
S = 4 and a bar of 5e-7 (emulated largest error 6.6e-8).
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
BAR = {6: 1e-10, 5: 2e-9, 4: 5e-7}  # statistical bars (of cabs) per slice count


def gamma(n):
    return n * U32 / (1 - n * U32)


def row_scales(W64):
    """2^e_i with max_l |W_il| < 2^e_i (1 for a zero row)."""
    m = np.abs(W64).max(axis=1)
    _, e = np.frexp(m)          # m = f 2^e with 0.5 <= f < 1; frexp(0) = (0, 0)
    return np.ldexp(1.0, e)


def ozaki_bound(W64, p, n, d, pr, slices=6):
    k = W64.shape[1]
    s = row_scales(W64)[:, None]
    worst = (slices + 1.05) * 2.0 ** (-7 * slices) * k * O.coefficients(s, n, d, pr)
    return worst + 1e-13 * (O.coefficients_abs(W64, n, d, pr) + np.abs(p))


def make(n, d, k, seed, row_exp=None):
    N, M = comb(n + d, d), comb(n + 2 * d, 2 * d)
    W = gaussian((N, k), 500 + seed, 1.0 / math.sqrt(k))
    if row_exp is not None:
        W = W * np.ldexp(1.0, row_exp)[:, None]
    p = gaussian(M, 600 + seed)
    return W, p


CASES = [(3, 2, 20), (4, 3, 37), (6, 3, 168), (6, 4, 420), (10, 5, 300), (17, 2, 40), (40, 2, 130)]


@pytest.mark.parametrize("slices", [6, 5, 4])
@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("n,d,k", CASES)
def test_ozaki_forward_matches_oracle(prec, n, d, k, slices):
    W, p = make(n, d, k, seed=n * 10 + d)
    Wd = torch.tensor(W, dtype=torch.float32, device="cuda")
    W64 = Wd.double().cpu().numpy()
    pd = torch.tensor(p, dtype=torch.float64, device="cuda")
    pl = S.Plan(n, d, k, prec)
    loss, g, r = pl.loss_grad(Wd, pd, grad=True, want_r=True, ozaki=slices)
    torch.cuda.synchronize()
    pr = O.pair_ranks(n, d)
    L_o, g_o, r_o = O.loss_grad(W64, p, n, d, pr)
    cabs = O.coefficients_abs(W64, n, d, pr)
    dc = ozaki_bound(W64, p, n, d, pr, slices)
    got = r.cpu().numpy() + p
    err = np.abs(got - (r_o + p))
    assert np.max(err / (dc + 1e-300)) <= 1.0
    assert np.max(err / (BAR[slices] * cabs + 1e-300)) <= 1.0
    dL = 2.0 * np.sum(np.abs(r_o) * dc) + np.sum(dc * dc)
    assert abs(loss.item() - L_o) <= dL + 1e-13 * L_o
    # the plan's own backward on the Ozaki residual
    N = W64.shape[0]
    tb = gamma(N + 1) + U32 if prec == "fp32" else 3.1 * 2.0 ** -16 + gamma(3 * N) + U32
    Wa = np.abs(W64)
    bound = tb * 4.0 * (np.abs(r_o)[pr] @ Wa) + 4.0 * (dc[pr] @ Wa) + 1e-300
    assert np.max(np.abs(g.double().cpu().numpy() - g_o) / bound) <= 1.0


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_ozaki_rows_of_very_different_scales(prec):
    """Rows scaled by 2^u, u in [-30, 30], and one zero row: each row gets its
    own exponent, so the bound scales with each row."""
    n, d, k = 6, 4, 420
    N = comb(n + d, d)
    u = np.random.default_rng(9).integers(-30, 31, size=N)
    W, p = make(n, d, k, seed=3, row_exp=u)
    W[17] = 0.0
    Wd = torch.tensor(W, dtype=torch.float32, device="cuda")
    W64 = Wd.double().cpu().numpy()
    pl = S.Plan(n, d, k, prec)
    pd = torch.tensor(p, dtype=torch.float64, device="cuda")
    _, _, r = pl.loss_grad(Wd, pd, grad=False, want_r=True, ozaki=True)
    pr = O.pair_ranks(n, d)
    r_o = O.residual(W64, p, n, d, pr)
    dc = ozaki_bound(W64, p, n, d, pr)
    err = np.abs(r.cpu().numpy() - r_o)
    assert np.max(err / (dc + 1e-300)) <= 1.0


@pytest.mark.parametrize("n,d,k", [(6, 4, 420), (40, 2, 130)])
def test_five_slices_are_five(n, d, k):
    """The five-slice forward really drops the sixth digit: its error is
    well above the six-slice one (an emulation gives ~50-130x in norm), and
    the four-slice one well above that; each stays inside its bound."""
    W, p = make(n, d, k, seed=n * 10 + d)
    Wd = torch.tensor(W, dtype=torch.float32, device="cuda")
    W64 = Wd.double().cpu().numpy()
    pd = torch.tensor(p, dtype=torch.float64, device="cuda")
    pl = S.Plan(n, d, k, "bf16x3")
    pr = O.pair_ranks(n, d)
    r_o = O.residual(W64, p, n, d, pr)
    e = {}
    for sl in (4, 5, 6):
        _, _, r = pl.loss_grad(Wd, pd, grad=False, want_r=True, ozaki=sl)
        err = r.cpu().numpy() - r_o
        assert np.all(np.abs(err) <= ozaki_bound(W64, p, n, d, pr, sl)), sl
        e[sl] = np.linalg.norm(err)
    assert e[5] >= 10.0 * e[6] and e[4] >= 10.0 * e[5], e


def test_ozaki_forward_agrees_with_exact_forward_at_a_fit():
    """Near a fit (W from p's own factor) the residual is ~1e3 times smaller
    than the coefficients; both FP64-accurate forwards must see the same
    residual far below the FP32 level."""
    n, d, k = 6, 4, 420
    N = comb(n + d, d)
    W0 = gaussian((N, k), 11, 1.0 / math.sqrt(k))
    Wd = torch.tensor(W0, dtype=torch.float32, device="cuda")
    W64 = Wd.double().cpu().numpy()
    pr = O.pair_ranks(n, d)
    p = O.coefficients(W64, n, d, pr)
    pd = torch.tensor(p, dtype=torch.float64, device="cuda")
    pl = S.Plan(n, d, k, "bf16x3")
    L_oz, _, r_oz = pl.loss_grad(Wd, pd, grad=False, want_r=True, ozaki=True)
    L_ex, _, r_ex = pl.loss_grad(Wd, pd, grad=False, want_r=True, exact=True)
    # p is the exact image of this W: the exact forward's residual is FP64
    # rounding only, the Ozaki forward's also its digit truncation (a CPU
    # emulation of the split gives 2.3e-12 here), both far below FP32's ~1e-7
    rel_oz = math.sqrt(L_oz.item()) / np.linalg.norm(p)
    rel_ex = math.sqrt(L_ex.item()) / np.linalg.norm(p)
    dc = ozaki_bound(W64, p, n, d, pr)
    assert rel_ex <= 1e-14, rel_ex
    assert rel_oz <= np.linalg.norm(dc) / np.linalg.norm(p) and rel_oz <= 1e-10, rel_oz
    assert np.all(np.abs(r_oz.cpu().numpy()) <= dc)


@pytest.mark.parametrize("prec,finisher,four_rel", [("bf16x3", "ozaki", 0.0), ("bf16x3", "ozaki5", 0.0),
                                                    ("bf16x3", "ozaki5", 1e-7), ("fp32", "ozaki5", 1e-7)])
def test_ozaki_finisher_solve_certified_by_the_oracle(prec, finisher, four_rel):
    """The ladder with the Ozaki forward (six or five slices) in its exact
    phase reaches an FP64-verified 1e-8 (the certificate is the FP64-MFMA
    forward), and the oracle agrees on the returned W."""
    n, d = 6, 4
    N = comb(n + d, d)
    k = 2 * N
    pr = O.pair_ranks(n, d)
    p = O.coefficients(gaussian((N, N // 2), 0) / math.sqrt(N // 2), n, d, pr)
    pl = S.Plan(n, d, k, prec)
    Wd = torch.tensor(gaussian((N, k), 1, 1 / math.sqrt(k)), dtype=torch.float32, device="cuda")
    res = pl.solve(Wd, torch.tensor(p, dtype=torch.float64, device="cuda"), S.Adam(lr=3e-3), tol=1e-8,
                   max_steps=20000, check_every=10, ladder=True, stall_checks=6, stall_ratio=0.8,
                   switch_rel=3e-6, lr_exact=1e-3, rollback_ratio=10.0, single_backward=True, finisher=finisher,
                   four_rel=four_rel)
    assert res["status"] == S.OK and res["phase"] == 2 and res["exact_steps"] > 0, res
    W64 = Wd.double().cpu().numpy()
    rel_o = float(np.linalg.norm(O.residual(W64, p, n, d, pr)) / np.linalg.norm(p))
    assert rel_o <= 1e-8 and abs(rel_o - res["rel"]) <= 1e-6 * rel_o, (rel_o, res)


def test_ozaki_fused_step_matches_unfused():
    """sos_step with the Ozaki forward and the single-product backward runs
    Adam in the backward GEMM's epilogue; the loss it reports must be the
    Ozaki loss of sos_loss_grad at the same W, and a second step reusing the
    transposed copy the epilogue wrote must see the loss of the updated W."""
    n, d, k = 6, 4, 420
    W, p = make(n, d, k, seed=7)
    Wd = torch.tensor(W, dtype=torch.float32, device="cuda")
    pd = torch.tensor(p, dtype=torch.float64, device="cuda")
    pl = S.Plan(n, d, k, "bf16x3")
    fl = S.FLAG_OZAKI_FORWARD | S.FLAG_SINGLE_BACKWARD
    L0 = pl.loss_grad(Wd, pd, grad=False, ozaki=True)[0].item()
    st = pl.new_state()
    L1 = pl.step(Wd, st, 1, pd, S.Adam(lr=1e-3), flags=fl).item()
    assert abs(L1 - L0) <= 1e-12 * L0
    W1 = Wd.clone()
    L2 = pl.step(Wd, st, 2, pd, S.Adam(lr=1e-3), flags=fl | S.FLAG_COPIES_VALID).item()
    L_ref = pl.loss_grad(W1, pd, grad=False, ozaki=True)[0].item()
    assert abs(L2 - L_ref) <= 1e-12 * L_ref
    assert L2 < L0


def test_ozaki_nonfinite_and_errors():
    n, d, k = 4, 3, 37
    W, p = make(n, d, k, seed=2)
    W[5, 3] = np.nan
    Wd = torch.tensor(W, dtype=torch.float32, device="cuda")
    pd = torch.tensor(p, dtype=torch.float64, device="cuda")
    pl = S.Plan(n, d, k, "fp32")
    loss, _, _ = pl.loss_grad(Wd, pd, grad=False, ozaki=True)
    assert not math.isfinite(loss.item())
    p64 = S.Plan(n, d, k, "fp64")
    with pytest.raises(S.SosError) as e:
        p64.loss_grad(Wd.double(), pd, grad=False, ozaki=True)
    assert e.value.code == S.EINVAL
    # five slices is a modifier of the Ozaki forward only
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    rc = S._lib.sos_loss_grad(pl._h, S._ptr(Wd), S._ptr(pd), S._ptr(loss), S._ptr(None), S._ptr(None),
                              S.FLAG_OZAKI_FIVE_SLICES, S._stream())
    assert rc == S.EINVAL
    with pytest.raises(S.SosError) as e:
        pl.step(Wd, pl.new_state(), 1, pd, S.Adam(lr=1e-3), flags=S.FLAG_OZAKI_FIVE_SLICES)
    assert e.value.code == S.EINVAL
    with pytest.raises(ValueError):
        pl.loss_grad(Wd, pd, grad=False, ozaki=3)
    both = S.FLAG_OZAKI_FORWARD | S.FLAG_OZAKI_FIVE_SLICES | S.FLAG_OZAKI_FOUR_SLICES
    for fl in (S.FLAG_OZAKI_FOUR_SLICES, both):
        rc = S._lib.sos_loss_grad(pl._h, S._ptr(Wd), S._ptr(pd), S._ptr(loss), S._ptr(None), S._ptr(None), fl,
                                  S._stream())
        assert rc == S.EINVAL, fl
