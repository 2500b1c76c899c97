"""An independent FP64 certificate of the full-size solve (n = 12, d = 6:
N = k = 18,564, M = 2,704,156).

The GPU runs the mixed-precision ladder (single-product forward to 3e-3,
split-BF16 bulk steps to 3e-6, both with the single-product backward, then
the int8 Ozaki forward with four slices to 2e-7 and five after) to an
FP64-verified relative residual of 1e-8, in the configuration the
time-to-target benchmark uses.  The oracle then checks the W the GPU returned on the host, in its own
way: its own p from the same FP32-rounded W0, its own pair map (dictionary
lookup of exponent codes), a plain matmul for W W^T and a bincount over the
ordered pairs (eq. nonconvex).  Its relative residual ||r|| / ||p||
(Section 3) must be <= 1e-8 and agree with the GPU's own certificate.

Host work: about 10 GB of memory and one to two minutes of CPU.
"""
import numpy as np
import pytest

import oracle as O
from workloads import CONFIGS

torch = pytest.importorskip("torch")
S = pytest.importorskip("paper_2410_19844_amd")

pytestmark = pytest.mark.gpu


def test_fullsize_solve_certified_by_the_oracle(pair_ranks_n12d6):
    c = CONFIGS["n12d6"]
    dev = torch.device("cuda")
    W0_32 = c.W0().astype(np.float32)
    # p on the GPU: the exact FP64 forward of the FP32-rounded W0
    pl0 = S.Plan(c.n, c.d, c.w0_rank, "fp32")
    zeros = torch.zeros(c.M, dtype=torch.float64, device=dev)
    _, _, p = pl0.loss_grad(torch.tensor(W0_32, device=dev), zeros, grad=False, want_r=True, exact=True)
    del pl0, zeros
    W = torch.tensor(c.W_init(), dtype=torch.float32, device=dev)
    pl = S.Plan(c.n, c.d, c.rank, "bf16x3")
    res = pl.solve(W, p, S.Adam(lr=3e-3), tol=1e-8, max_steps=3000, check_every=10, ladder=True,
                   stall_checks=6, stall_ratio=0.8, switch_rel=3e-6, lr_exact=1e-3, rollback_ratio=10.0,
                   single_backward=True, finisher="ozaki5", single_rel=3e-3, four_rel=2e-7)
    assert res["status"] == S.OK, res
    assert res["rel"] <= 1e-8, res
    Wf = W.double().cpu().numpy()
    del pl, W, p
    torch.cuda.empty_cache()

    pr = pair_ranks_n12d6
    p_o = O.coefficients(W0_32.astype(np.float64), c.n, c.d, pr)
    r_o = O.residual(Wf, p_o, c.n, c.d, pr)
    rel_o = float(np.linalg.norm(r_o) / np.linalg.norm(p_o))
    # both sides sum exact products of the same FP32 values in FP64; they differ
    # only in summation order (~1e-16 of coeff(|W||W|^T) per coefficient)
    assert rel_o <= 1e-8 * (1 + 1e-4), (rel_o, res["rel"])
    assert abs(rel_o - res["rel"]) <= 1e-4 * res["rel"], (rel_o, res["rel"])
