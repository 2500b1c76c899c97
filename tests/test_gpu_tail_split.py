"""The split-bf16 gram where its tail split runs: n = 13, d = 5 has 595 upper
tiles of 256 rows (N = 8,568), so on a 256-CU MI355X the last 83 tiles run
in K ranges, each scattering its partial sum.  Every one of the 1,144,066
coefficients is checked against the FP64 oracle under the split-bf16 bound
of the parity tests (3.1 2^-16 + gamma(3K) + u of coeff(|W||W|^T), plus
1e-15 |p| for adding p back), with the merged epilogue and without it, in
both 16-bit formats, and the loss under the bound carried from it.  The
ranges change only how the FP32 tile sums are cut before their FP64
additions, which the bound already covers.  (On a device with another CU
count the tail differs, or no split runs; the checks hold either way.)
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
n, d, k = 13, 5, 64


def gamma(m):
    return m * U32 / (1 - m * U32)


@pytest.fixture(scope="module")
def case():
    N, M = comb(n + d, d), comb(n + 2 * d, 2 * d)
    assert (N + 255) // 256 == 34  # 595 upper tiles
    Wd = torch.tensor(gaussian((N, k), 71, 1 / math.sqrt(k)), dtype=torch.float32, device="cuda")
    W64 = Wd.double().cpu().numpy()
    p = gaussian(M, 72)
    pr = O.pair_ranks(n, d)
    L_o, _, r_o = O.loss_grad(W64, p, n, d, pr)
    cabs = O.coefficients_abs(W64, n, d, pr)
    return dict(Wd=Wd, p=p, pd=torch.tensor(p, dtype=torch.float64, device="cuda"), L_o=L_o, r_o=r_o, cabs=cabs)


@pytest.mark.parametrize("prec", ["bf16x3", "fp16x3"])
def test_tail_split_coefficients(case, prec):
    pl = S.Plan(n, d, k, prec)
    tf = 3.1 * 2.0 ** -16 + gamma(3 * k) + U32
    dc = tf * case["cabs"] + 1e-15 * np.abs(case["p"]) + 1e-300
    dL = 2.0 * np.sum(np.abs(case["r_o"]) * tf * case["cabs"]) + np.sum((tf * case["cabs"]) ** 2)
    for unmerged in (False, True):
        loss, _, r = pl.loss_grad(case["Wd"], case["pd"], grad=False, want_r=True, unmerged_scatter=unmerged)
        worst = float(np.max(np.abs(r.cpu().numpy() - case["r_o"]) / dc))
        assert worst <= 1.0, (prec, unmerged, worst)
        assert abs(loss.item() - case["L_o"]) <= dL + 1e-12 * case["L_o"], (prec, unmerged)
