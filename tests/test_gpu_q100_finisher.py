"""The hundred-variable quartic (n = 99, d = 2: N = k = 5,050, M = 4,421,275)
reaches an FP64-verified relative residual of 1e-8 at the benchmark's step
sizes, with the exact-forward finisher's step size inside a stable band.

Above that band the finisher's step count depends on the rounding order of
the forward's FP64 sums. At 3e-3, two tile orders of the gram gave 500 and
2190 steps, each reproducibly. From 1.5e-3 to 2.5e-3 both orders gave 440
to 450 steps. The test runs the band's ends and the default, and bounds
the step count well below the unstable regime's.
"""
import pytest

from workloads import CONFIGS

torch = pytest.importorskip("torch")
S = pytest.importorskip("paper_2410_19844_amd")

pytestmark = pytest.mark.gpu

BAND = (1.5e-3, 2e-3, 2.5e-3)


@pytest.fixture(scope="module")
def q100():
    c = CONFIGS["q100"]
    dev = torch.device("cuda")
    W0 = torch.tensor(c.W0(), dtype=torch.float32, device=dev)
    pl0 = S.Plan(c.n, c.d, c.w0_rank, "fp32")
    zeros = torch.zeros(c.M, dtype=torch.float64, device=dev)
    _, _, p = pl0.loss_grad(W0, zeros, grad=False, want_r=True, exact=True)
    del pl0, W0, zeros
    pl = S.Plan(c.n, c.d, c.rank, "bf16x3")
    yield c, pl, p
    del pl, p
    torch.cuda.empty_cache()


def test_default_finisher_step_is_inside_the_band():
    import bench
    lr_bulk, lr_fin = bench.LR_DEFAULTS["q100"]
    assert lr_bulk == 3e-3
    assert min(BAND) < lr_fin < max(BAND)


@pytest.mark.parametrize("lr_exact", BAND)
def test_q100_reaches_1e8_in_few_steps(q100, lr_exact):
    c, pl, p = q100
    W = torch.tensor(c.W_init(), dtype=torch.float32, device="cuda")
    res = pl.solve(W, p, S.Adam(lr=3e-3), tol=1e-8, max_steps=3000, check_every=10, ladder=True,
                   stall_checks=6, stall_ratio=0.8, switch_rel=3e-6, lr_exact=lr_exact, rollback_ratio=10.0,
                   single_backward=True)
    print(f"q100 lr_exact {lr_exact}: {res}", flush=True)
    assert res["status"] == S.OK, res
    assert res["rel"] <= 1e-8, res
    assert res["steps"] <= 700, res
