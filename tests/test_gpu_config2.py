"""The n = 6, d = 4 workload and its non-SOS control, end to end on the GPU.

* SOS by construction (N = 210, M = 3,003): p = coeff(W0 W0^T) with W0
  210 x 50, N(0, 1) entries (not normalised, diag G0 ~ 50), computed by the
  oracle in FP64.  The plain FP32 form (FP32 plan, FP32 MFMA for both
  contractions, no ladder) runs sos_solve from W 210 x 420, N(0, 0.05^2), to
  an FP64-verified relative residual <= 1e-6 (the FP32 floor is ~1e-7);
  the oracle then re-certifies the returned W on the host with its own pair
  map, matmul and bincount (Section 1.1, eq. nonconvex and eq. basicsos).
* The Motzkin form padded into n = 6, d = 3 (N = 84, M = 924, rank
  k = 2N = 168): non-negative but not a sum of squares (Section 1.1), so no
  W reaches it.  The smallest achievable loss is the squared distance from p
  to the SOS cone, which the oracle computes by a convex method (FISTA with
  PSD projection, independent of the factored objective).  Every step's
  loss must stay at or above it, and Adam's best loss must come within 5%
  of it.  Step sizes: 3e-3 for 10,000 steps, then 1e-3 for 10,000 (an
  oracle sweep over four starts comes within 0.02% with this schedule,
  while constant step sizes oscillate).
"""
import math

import numpy as np
import pytest

import oracle as O
from workloads import CONFIGS, motzkin_terms

torch = pytest.importorskip("torch")
S = pytest.importorskip("paper_2410_19844_amd")

pytestmark = pytest.mark.gpu


def test_n6d4_fp32_solve_certified_by_the_oracle():
    c = CONFIGS["n6d4"]
    pr = O.pair_ranks(c.n, c.d)
    p = O.coefficients(c.W0(), c.n, c.d, pr)
    dev = torch.device("cuda")
    pd = torch.tensor(p, dtype=torch.float64, device=dev)
    W = torch.tensor(c.W_init(), dtype=torch.float32, device=dev)
    pl = S.Plan(c.n, c.d, c.rank, "fp32")
    res = pl.solve(W, pd, S.Adam(lr=1e-2), tol=1e-6, max_steps=20000, check_every=10, ladder=False,
                   rollback_ratio=10.0)
    assert res["status"] == S.OK, res
    assert res["rel"] <= 1e-6
    Wf = W.double().cpu().numpy()
    rel_o = float(np.linalg.norm(O.residual(Wf, p, c.n, c.d, pr)) / np.linalg.norm(p))
    # both sides: exact products of the same FP32 entries summed in FP64
    assert rel_o <= 1e-6 * (1 + 1e-6), (rel_o, res)
    assert abs(rel_o - res["rel"]) <= 1e-6 * res["rel"], (rel_o, res["rel"])


@pytest.fixture(scope="module")
def motzkin():
    c = CONFIGS["motzkin_n6d3"]
    p = O.poly_vector(motzkin_terms(c.n), c.n, c.d)
    dist2 = O.psd_distance(p, c.n, c.d).dist2
    return c, p, dist2


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_motzkin_n6d3_stays_at_the_cone_distance(motzkin, prec):
    c, p, dist2 = motzkin
    dev = torch.device("cuda")
    pl = S.Plan(c.n, c.d, c.rank, prec)
    wdt = torch.float64 if prec == "fp64" else torch.float32
    W = torch.tensor(c.W_init(), dtype=wdt, device=dev)
    pd = torch.tensor(p, dtype=torch.float64, device=dev)
    st = pl.new_state()
    flags = S.FLAG_EXACT_FORWARD if prec == "fp32" else 0
    sched = [(3e-3, 10000), (1e-3, 10000)]
    losses = torch.empty(sum(n for _, n in sched), dtype=torch.float64, device=dev)
    t = 0
    for lr, n in sched:
        adam = S.Adam(lr=lr)
        for _ in range(n):
            pl.step(W, st, t + 1, pd, adam, loss=losses[t:t + 1], flags=flags)
            t += 1
    L = losses.cpu().numpy()
    assert np.isfinite(L).all()
    # no W reaches below the distance to the SOS cone (the losses are FP64 sums of exact products)
    assert L.min() >= dist2 * (1 - 1e-9), (L.min(), dist2)
    assert L.min() <= dist2 * 1.05, (L.min() / dist2)
    rel = pl.verify(W, pd)
    assert rel >= math.sqrt(dist2) / np.linalg.norm(p) * (1 - 1e-9)
