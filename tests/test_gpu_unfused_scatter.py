"""SOS_FLAG_UNFUSED_SCATTER (split plans): the gram stores its FP32 tiles and a
separate kernel ranks and scatters them.  It must give the coefficients of
the fused forward: every coefficient within the split-bf16 bound of the
parity tests (3.1 2^-16 + gamma(3K) + u of coeff(|W||W|^T)) against the
FP64 oracle, and the loss within the bound carried from it."""
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


@pytest.mark.parametrize("n,d,k", [(3, 2, 20), (6, 4, 420), (10, 5, 300), (40, 2, 130)])
def test_unfused_scatter_matches_oracle(n, d, k):
    N, M = comb(n + d, d), comb(n + 2 * d, 2 * d)
    Wd = torch.tensor(gaussian((N, k), 70 + n, 1 / math.sqrt(k)), dtype=torch.float32, device="cuda")
    p = gaussian(M, 80 + n)
    pd = torch.tensor(p, dtype=torch.float64, device="cuda")
    pl = S.Plan(n, d, k, "bf16x3")
    loss_u, _, r_u = pl.loss_grad(Wd, pd, grad=False, want_r=True, unfused_scatter=True)
    loss_f, _, r_f = pl.loss_grad(Wd, pd, grad=False, want_r=True)
    W64 = Wd.double().cpu().numpy()
    pr = O.pair_ranks(n, d)
    L_o, _, r_o = O.loss_grad(W64, p, n, d, pr)
    cabs = O.coefficients_abs(W64, n, d, pr)
    tf = 3.1 * 2.0 ** -16 + gamma(3 * k) + U32
    dc = tf * cabs + 1e-15 * np.abs(p) + 1e-300
    for r in (r_u, r_f):
        assert np.max(np.abs(r.cpu().numpy() - r_o) / dc) <= 1.0
    dL = 2.0 * np.sum(np.abs(r_o) * tf * cabs) + np.sum((tf * cabs) ** 2)
    assert abs(loss_u.item() - L_o) <= dL + 1e-12 * L_o
    # same tiles, same FP32 sums: the two forwards differ only in the order of the FP64 adds
    assert abs(loss_u.item() - loss_f.item()) <= 1e-12 * loss_f.item()
