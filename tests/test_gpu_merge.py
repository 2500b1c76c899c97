"""The split plans' gram epilogue with merge maps (the default for bound plans
where merging saves atomics) and without them (SOS_FLAG_UNMERGED_SCATTER),
against the FP64 oracle through the C ABI.

Merging changes only the order of the FP64 additions into r (a segment's
pairs of one coefficient are summed in an LDS slot first), so both forms keep
the split-bf16 bound of the parity tests: 3.1 2^-16 + gamma(3K) + u of
coeff(|W||W|^T) per coefficient (the FP64 additions far inside it), plus
1e-15 |p| for adding p back.  The shapes bind with merging on (pairs per
atomic after merging: (6, 4) 4.5, (10, 5) 3.8, (12, 4) 3.0, (20, 3) 2.2,
(24, 3) 2.0, (40, 2) 1.6), and (20, 3), (24, 3) and (40, 2) have segments
with more than 8,192 distinct coefficients, whose remaining pairs take the
direct path.  Both 16-bit formats.
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


def n_basis(n, d):
    return comb(n + d, d)


CASES = [(3, 2, 20), (6, 4, 420), (8, 4, 1000), (10, 5, 300), (12, 4, 64), (20, 3, 100), (24, 3, 64),
         (40, 2, 130)]


@pytest.mark.parametrize("prec", ["bf16x3", "fp16x3"])
@pytest.mark.parametrize("n,d,k", CASES)
def test_merged_and_unmerged_scatter_match_oracle(prec, n, d, k):
    N, M = n_basis(n, d), comb(n + 2 * d, 2 * d)
    Wd = torch.tensor(gaussian((N, k), 40 + n + d, 1 / math.sqrt(k)), dtype=torch.float32, device="cuda")
    p = gaussian(M, 50 + n + d)
    pd = torch.tensor(p, dtype=torch.float64, device="cuda")
    pl = S.Plan(n, d, k, prec)
    W64 = Wd.double().cpu().numpy()
    pr = O.pair_ranks(n, d)
    L_o, _, r_o = O.loss_grad(W64, p, n, d, pr)
    cabs = O.coefficients_abs(W64, n, d, pr)
    tf = 3.1 * 2.0 ** -16 + gamma(3 * k) + U32
    dc = tf * cabs + 1e-15 * np.abs(p) + 1e-300
    dL = 2.0 * np.sum(np.abs(r_o) * tf * cabs) + np.sum((tf * cabs) ** 2)
    for unmerged in (False, True):
        loss, _, r = pl.loss_grad(Wd, pd, grad=False, want_r=True, unmerged_scatter=unmerged)
        worst = float(np.max(np.abs(r.cpu().numpy() - r_o) / dc))
        assert worst <= 1.0, (unmerged, worst)
        assert abs(loss.item() - L_o) <= dL + 1e-12 * L_o, unmerged


def test_merged_scatter_in_the_fused_step():
    """sos_step (single-product backward, Adam in its epilogue) on the merged
    forward reports the forward's loss at the same W, and a second step from
    the copies the epilogue wrote sees the loss of the updated W."""
    n, d, k = 10, 5, 300
    N, M = n_basis(n, d), comb(n + 2 * d, 2 * d)
    Wd = torch.tensor(gaussian((N, k), 61, 1 / math.sqrt(k)), dtype=torch.float32, device="cuda")
    pd = torch.tensor(gaussian(M, 62), dtype=torch.float64, device="cuda")
    pl = S.Plan(n, d, k, "bf16x3")
    L0 = pl.loss_grad(Wd, pd, grad=False, unmerged_scatter=True)[0].item()
    st = pl.new_state()
    L1 = pl.step(Wd, st, 1, pd, S.Adam(lr=1e-3), flags=S.FLAG_SINGLE_BACKWARD).item()
    assert abs(L1 - L0) <= 1e-9 * L0
    W1 = Wd.clone()
    L2 = pl.step(Wd, st, 2, pd, S.Adam(lr=1e-3), flags=S.FLAG_SINGLE_BACKWARD | S.FLAG_COPIES_VALID).item()
    L_ref = pl.loss_grad(W1, pd, grad=False)[0].item()
    assert abs(L2 - L_ref) <= 1e-9 * L_ref
    assert L2 < L0


def test_unmerged_flag_errors():
    n, d, k = 4, 3, 37
    N, M = n_basis(n, d), comb(n + 2 * d, 2 * d)
    Wd = torch.tensor(gaussian((N, k), 5, 1 / math.sqrt(k)), dtype=torch.float32, device="cuda")
    pd = torch.tensor(gaussian(M, 6), dtype=torch.float64, device="cuda")
    bf = S.Plan(n, d, k, "bf16x3")
    f32 = S.Plan(n, d, k, "fp32")
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    fu = S.FLAG_UNMERGED_SCATTER
    bad = [(bf, fu | S.FLAG_EXACT_FORWARD), (bf, fu | S.FLAG_OZAKI_FORWARD), (bf, fu | S.FLAG_FP32_FORWARD),
           (bf, fu | S.FLAG_UNFUSED_SCATTER), (f32, fu)]
    for pl, fl in bad:
        rc = S._lib.sos_loss_grad(pl._h, S._ptr(Wd), S._ptr(pd), S._ptr(loss), S._ptr(None), S._ptr(None), fl,
                                  S._stream())
        assert rc == S.EINVAL, (pl.prec, fl, rc)
        with pytest.raises(S.SosError) as e:
            pl.step(Wd, pl.new_state(), 1, pd, S.Adam(lr=1e-3), flags=fl)
        assert e.value.code == S.EINVAL, (pl.prec, fl)
