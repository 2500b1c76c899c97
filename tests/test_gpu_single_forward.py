"""The single-product fast forward (SOS_FLAG_SINGLE_FORWARD: the gram takes
hi hi^T only) against the FP64 oracle, through the C ABI.

Bound.  Each operand is rounded once: bf16 keeps 8 significant bits, so
hi = w (1 + e) with |e| <= 2^-8 and a product of two is off by at most
(2^-7 + 2^-16) |w w'|; the FP32 sum of K such products adds gamma(K) of the
absolute sum.  Per coefficient that is (2^-7 + 2^-16 + gamma(K) + u) of
coeff(|W||W|^T), plus 1e-15 |p| for adding p back.  fp16 keeps 11 bits of
the scaled copy 2^sW w (2^sW max|W| < 2^12); below its normal range a
rounding loses at most 2^-25 absolute, which adds 2^-24 2^-sW times the pair
sum of the row sums of |W| (as for the split fp16 forward).  The same
plans' merge maps serve both forms (the epilogue does not depend on how the
tile was summed).
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
    if not m > 0:
        return 0
    _, e = math.frexp(m)
    return max(-100, min(100, top - e))


def pair_sum(v, pr):
    return np.bincount(pr.ravel(), weights=(v[:, None] + v[None, :]).ravel(), minlength=int(pr.max()) + 1)


def single_bound(W64, p, n, d, pr, prec):
    k = W64.shape[1]
    cabs = O.coefficients_abs(W64, n, d, pr)
    if prec == "bf16x3":
        return (2.0 ** -7 + 2.0 ** -16 + gamma(k) + U32) * cabs + 1e-15 * np.abs(p) + 1e-300
    Wa = np.abs(W64)
    sW = scale_exp(float(Wa.max()), 12)
    return ((2.0 ** -10 + 2.0 ** -22 + gamma(k) + U32) * cabs + 2.0 ** (-24 - sW) * pair_sum(Wa.sum(1), pr)
            + 1e-15 * np.abs(p) + 1e-300)


CASES = [(3, 2, 20), (4, 3, 37), (6, 4, 420), (10, 5, 300), (12, 4, 64), (40, 2, 130)]


@pytest.mark.parametrize("prec", ["bf16x3", "fp16x3"])
@pytest.mark.parametrize("n,d,k", CASES)
def test_single_forward_matches_oracle(prec, n, d, k):
    N, M = comb(n + d, d), comb(n + 2 * d, 2 * d)
    Wd = torch.tensor(gaussian((N, k), 700 + n + d, 1 / math.sqrt(k)), dtype=torch.float32, device="cuda")
    p = gaussian(M, 710 + n + d)
    pd = torch.tensor(p, dtype=torch.float64, device="cuda")
    pl = S.Plan(n, d, k, prec)
    W64 = Wd.double().cpu().numpy()
    pr = O.pair_ranks(n, d)
    L_o, _, r_o = O.loss_grad(W64, p, n, d, pr)
    dc = single_bound(W64, p, n, d, pr, prec)
    loss, _, r = pl.loss_grad(Wd, pd, grad=False, want_r=True, single_forward=True)
    err = np.abs(r.cpu().numpy() - r_o)
    assert np.max(err / dc) <= 1.0, np.max(err / dc)
    dL = 2.0 * np.sum(np.abs(r_o) * dc) + np.sum(dc * dc)
    assert abs(loss.item() - L_o) <= dL + 1e-12 * L_o
    # the flag has its effect: the three-product forward is far closer
    _, _, r3 = pl.loss_grad(Wd, pd, grad=False, want_r=True)
    e3 = np.linalg.norm(r3.cpu().numpy() - r_o)
    assert np.linalg.norm(err) >= 20.0 * e3, (np.linalg.norm(err), e3)


def test_single_forward_tail_split():
    """n = 13, d = 5: 595 upper tiles, so the last round runs in K ranges of
    whole two-block stages; every coefficient inside the bound."""
    n, d, k = 13, 5, 64
    N, M = comb(n + d, d), comb(n + 2 * d, 2 * d)
    Wd = torch.tensor(gaussian((N, k), 731, 1 / math.sqrt(k)), dtype=torch.float32, device="cuda")
    p = gaussian(M, 732)
    pd = torch.tensor(p, dtype=torch.float64, device="cuda")
    pl = S.Plan(n, d, k, "bf16x3")
    W64 = Wd.double().cpu().numpy()
    pr = O.pair_ranks(n, d)
    r_o = O.residual(W64, p, n, d, pr)
    _, _, r = pl.loss_grad(Wd, pd, grad=False, want_r=True, single_forward=True)
    assert np.max(np.abs(r.cpu().numpy() - r_o) / single_bound(W64, p, n, d, pr, "bf16x3")) <= 1.0


def test_single_forward_fused_step():
    """sos_step with the single-product forward and backward reports the
    single forward's loss at the same W, and a second step from the copies
    its epilogue wrote sees the loss of the updated W."""
    n, d, k = 6, 4, 420
    N, M = comb(n + d, d), comb(n + 2 * d, 2 * d)
    Wd = torch.tensor(gaussian((N, k), 741, 1 / math.sqrt(k)), dtype=torch.float32, device="cuda")
    pd = torch.tensor(gaussian(M, 742), dtype=torch.float64, device="cuda")
    pl = S.Plan(n, d, k, "bf16x3")
    fl = S.FLAG_SINGLE_FORWARD | S.FLAG_SINGLE_BACKWARD
    L0 = pl.loss_grad(Wd, pd, grad=False, single_forward=True)[0].item()
    st = pl.new_state()
    L1 = pl.step(Wd, st, 1, pd, S.Adam(lr=1e-3), flags=fl).item()
    assert abs(L1 - L0) <= 1e-12 * L0
    W1 = Wd.clone()
    L2 = pl.step(Wd, st, 2, pd, S.Adam(lr=1e-3), flags=fl | S.FLAG_COPIES_VALID).item()
    L_ref = pl.loss_grad(W1, pd, grad=False, single_forward=True)[0].item()
    assert abs(L2 - L_ref) <= 1e-12 * L_ref
    assert L2 < L0


@pytest.mark.parametrize("prec", ["bf16x3", "fp16x3"])
def test_fast_start_solve_certified_by_the_oracle(prec):
    """The ladder starting with the single-product forward (single_rel) goes
    on to the three products and the finisher (four, then five int8 slices),
    and reaches an FP64-verified 1e-8 that the oracle confirms."""
    n, d = 6, 4
    N = comb(n + d, d)
    k = 2 * N
    pr = O.pair_ranks(n, d)
    p = O.coefficients(gaussian((N, N // 2), 0) / math.sqrt(N // 2), n, d, pr)
    pl = S.Plan(n, d, k, prec)
    Wd = torch.tensor(gaussian((N, k), 1, 1 / math.sqrt(k)), dtype=torch.float32, device="cuda")
    res = pl.solve(Wd, torch.tensor(p, dtype=torch.float64, device="cuda"), S.Adam(lr=3e-3), tol=1e-8,
                   max_steps=20000, check_every=10, ladder=True, stall_checks=6, stall_ratio=0.8,
                   switch_rel=3e-6, lr_exact=1e-3, rollback_ratio=10.0, single_backward=True, finisher="ozaki5",
                   single_rel=1e-2, four_rel=1e-7)
    assert res["status"] == S.OK and res["phase"] == 2 and res["exact_steps"] > 0, res
    W64 = Wd.double().cpu().numpy()
    rel_o = float(np.linalg.norm(O.residual(W64, p, n, d, pr)) / np.linalg.norm(p))
    assert rel_o <= 1e-8 and abs(rel_o - res["rel"]) <= 1e-6 * rel_o, (rel_o, res)


def test_single_forward_errors():
    n, d, k = 4, 3, 37
    N, M = comb(n + d, d), comb(n + 2 * d, 2 * d)
    Wd = torch.tensor(gaussian((N, k), 5, 1 / math.sqrt(k)), dtype=torch.float32, device="cuda")
    pd = torch.tensor(gaussian(M, 6), dtype=torch.float64, device="cuda")
    bf = S.Plan(n, d, k, "bf16x3")
    f32 = S.Plan(n, d, k, "fp32")
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    fs = S.FLAG_SINGLE_FORWARD
    for pl, fl in [(f32, fs), (bf, fs | S.FLAG_UNMERGED_SCATTER), (bf, fs | S.FLAG_UNFUSED_SCATTER)]:
        rc = S._lib.sos_loss_grad(pl._h, S._ptr(Wd), S._ptr(pd), S._ptr(loss), S._ptr(None), S._ptr(None), fl,
                                  S._stream())
        assert rc == S.EINVAL, (pl.prec, fl, rc)
    with pytest.raises(S.SosError) as e:
        bf.solve(Wd, pd, S.Adam(lr=1e-3), single_rel=-1.0)
    assert e.value.code == S.EINVAL
