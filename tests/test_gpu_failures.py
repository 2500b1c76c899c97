"""Failure detection, forced from the host: a non-finite loss is reported as
SOS_ENUMERIC by the solvers when no finite check came before it; after a
finite check the solvers roll back to the best iterate with fresh Adam
moments and half the step size, and recover; a serving request that goes
non-finite retires "not certified" without touching the other requests'
results.

(The NaN only flows through the arithmetic: no index, size or control flow
depends on it.)"""
import dataclasses

import pytest

torch = pytest.importorskip("torch")
S = pytest.importorskip("paper_2410_19844_amd")
from paper_2410_19844_amd import serve  # noqa: E402

from test_gpu_serving import build_requests  # noqa: E402

pytestmark = pytest.mark.gpu


def _problem(prec):
    pl = S.Plan(3, 2, 20, prec)
    g = torch.Generator(device="cuda").manual_seed(5)
    W = (0.1 * torch.randn((pl.N, pl.rank), device="cuda", generator=g)).to(pl.wdtype)
    p = torch.randn(pl.M, device="cuda", dtype=torch.float64, generator=g)
    return pl, W, p


@pytest.mark.parametrize("prec", ["fp32", "fp64", "bf16x3"])
def test_solve_reports_a_nonfinite_loss(prec):
    pl, W, p = _problem(prec)
    W[0, 0] = float("nan")
    with pytest.raises(S.SosError) as e:
        pl.solve(W, p, S.Adam(lr=1e-2), tol=1e-8, max_steps=100, check_every=10)
    assert e.value.code == S.ENUMERIC


def test_net_solve_reports_a_nonfinite_loss():
    net = S.Net(4, 4, 6, "fp64")
    net.At.copy_(torch.eye(4, 4, device="cuda"))
    net.Bt.normal_(0, 0.3)
    net.Bt[0, 0] = float("nan")
    p = torch.ones(net.plan.M, dtype=torch.float64, device="cuda")
    with pytest.raises(S.SosError) as e:
        net.solve(p, S.Adam(lr=1e-2), tol=1e-8, max_steps=100, check_every=10, ladder=False)
    assert e.value.code == S.ENUMERIC


@pytest.mark.parametrize("prec,single", [("fp32", False), ("bf16x3", True), ("bf16x3", False)])
def test_solve_recovers_from_a_nonfinite_loss_after_a_finite_check(prec, single):
    """A step size of 2^66 makes the first update overflow the FP32 Gram (the
    loss at the second check is Inf, the first one was finite).  The solver
    must roll back to the best W with zeroed moments and half the step size,
    again on each divergence, until the step size is workable, and then make
    progress: moments that kept the non-finite gradient would leave W NaN at
    every later check and the best iterate at the start."""
    pl = S.Plan(3, 2, 20, prec)
    g = torch.Generator(device="cuda").manual_seed(11)
    W0 = torch.randn((pl.N, 6), device="cuda", generator=g, dtype=torch.float64)
    zeros = torch.zeros(pl.M, dtype=torch.float64, device="cuda")
    pl64 = S.Plan(3, 2, 6, "fp64")
    _, _, p = pl64.loss_grad(W0.contiguous(), zeros, grad=False, want_r=True)
    W = (0.1 * torch.randn((pl.N, pl.rank), device="cuda", generator=g)).to(pl.wdtype)
    rel0 = pl.verify(W, p)
    res = pl.solve(W, p, S.Adam(lr=2.0 ** 66), tol=1e-12, max_steps=3000, check_every=1, ladder=False,
                   rollback_ratio=10.0, single_backward=single)
    assert bool(torch.isfinite(W).all())
    assert res["rel"] <= 0.1 * rel0, (res, rel0)


def test_net_solve_recovers_from_a_nonfinite_loss_after_a_finite_check():
    net = S.Net(4, 4, 6, "fp32")
    g = torch.Generator(device="cuda").manual_seed(12)
    net.At.copy_(torch.randn((4, 4), device="cuda", generator=g) * 0.5)
    net.Bt.copy_(torch.randn((16, 6), device="cuda", generator=g) * 0.3)
    W_t = net.weights().clone()                    # target: p from the starting network, perturbed below
    zeros = torch.zeros(net.plan.M, dtype=torch.float64, device="cuda")
    _, _, p = net.plan.loss_grad(W_t, zeros, grad=False, want_r=True, exact=True)
    net.Bt.add_(0.1 * torch.randn((16, 6), device="cuda", generator=g))
    rel0 = net.plan.verify(net.weights(), p)
    res = net.solve(p, S.Adam(lr=2.0 ** 66), tol=1e-12, max_steps=3000, check_every=1, ladder=False,
                    single_backward=False, rollback_ratio=10.0)
    assert bool(torch.isfinite(net.At).all()) and bool(torch.isfinite(net.Bt).all())
    assert res["rel"] <= 0.1 * rel0, (res, rel0)


def test_server_isolates_a_nonfinite_request():
    specs = [(0, 5, 3, "sos", 0.0), (1, 4, 2, "sos", 0.0), (2, 3, 3, "non", 0.0)]
    good = build_requests(specs)
    bad = build_requests([(3, 4, 3, "sos", 0.0)])[0]
    Wb = bad.W_init.clone()
    Wb[1, 2] = float("nan")
    bad = dataclasses.replace(bad, W_init=Wb)
    mk = lambda: serve.Server(max_active=8, check_every=50, tol=1e-6, max_steps=1500, keep_W=True)
    alone = mk().run(good)
    mixed = mk().run(good + [bad])
    r_bad = next(r for r in mixed if r.id == 3)
    assert (r_bad.verdict, r_bad.reason) == ("not certified", "nonfinite")
    assert r_bad.steps == 50                       # retired at its first check
    for a in alone:
        b = next(r for r in mixed if r.id == a.id)
        assert (a.verdict, a.reason, a.steps) == (b.verdict, b.reason, b.steps), a.id
        assert torch.equal(a.W, b.W), a.id
