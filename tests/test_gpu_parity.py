"""GPU parity: libsos (HIP, gfx950) against the FP64 oracle, through the C ABI.

Tolerances (per coefficient / gradient entry, relative to the absolute-value
scale cabs = coeff(|W||W|^T) and gabs = 4 |R| |W|):
  * FP64 plans and the exact forward: 1e-10.
  * FP32: gamma(K+1) + 2^-24, gamma(n) = n u / (1 - n u), u = 2^-24 (the
    standard bound for a K-term FP32 dot product, plus the FP64 -> FP32
    rounding of R).
  * BF16X3: 3.1 * 2^-16 + gamma(3K) + 2^-24: each operand w = hi + lo + e with
    |e| <= 2^-16 |w| and |lo| <= 2^-8 |w|; the three kept products leave out
    lo*lo' and the e terms (<= 3 * 2^-16 |w w'| together), and the FP32
    accumulation runs over 3K products.
The loss error follows from the coefficient error: |dL| <= 2 sum |r| |dc| + |dc|^2.
"""
import math
from math import comb

import numpy as np
import pytest

import oracle as O
from workloads import CONFIGS, gaussian, motzkin_terms

torch = pytest.importorskip("torch")
S = pytest.importorskip("paper_2410_19844_amd")

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def gamma(n):
    return n * U32 / (1 - n * U32)


def tol_for(prec, K):
    if prec == "fp64":
        return 1e-10
    if prec == "fp32":
        return gamma(K + 1) + U32
    if prec == "bf16x1":   # one bf16 product: both operands rounded to 8 significant bits
        return 2.0 ** -7 + 2.0 ** -16 + gamma(K) + U32
    return 3.1 * 2.0 ** -16 + gamma(3 * K) + U32


def dev():
    return torch.device("cuda")


def to_dev(x, dtype):
    return torch.tensor(np.ascontiguousarray(x), dtype=dtype, device=dev())


def make_case(n, d, k, prec, seed=0, p_kind="random", wstd=None):
    N, M = comb(n + d, d), comb(n + 2 * d, 2 * d)
    W = gaussian((N, k), 100 + seed, wstd if wstd is not None else 1.0 / math.sqrt(k))
    wdt = torch.float64 if prec == "fp64" else torch.float32
    Wd = to_dev(W, wdt)
    W64 = Wd.double().cpu().numpy()           # exactly the values the GPU sees
    if p_kind == "random":
        p = gaussian(M, 200 + seed)
    else:
        p = O.poly_vector(motzkin_terms(n), n, d)
    return W64, Wd, p, to_dev(p, torch.float64)


def assert_close_scaled(got, want, scale, tol, what):
    err = np.abs(got - want)
    bound = tol * scale + 1e-300
    worst = float(np.max(err / bound))
    assert worst <= 1.0, f"{what}: max |err|/bound = {worst:.3g} (tol {tol:.3g})"


# ---------------------------------------------------------------------------
# Ranking: bit-exact
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,d", [(1, 1), (1, 7), (2, 7), (3, 2), (4, 3), (6, 3), (6, 4), (16, 1), (8, 4), (10, 5),
                                 (17, 1), (17, 2), (20, 3), (40, 2), (24, 3)])
def test_pair_ranks_bit_exact(n, d):
    pl = S.Plan(n, d, 4, "fp32")
    got = pl.pair_ranks().cpu().numpy()
    want = O.pair_ranks(n, d)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("n,d", [(18, 4), (99, 2)])
def test_pair_ranks_many_variables_sampled_rows(n, d):
    """Variable-list ranking at the longest merged lists (2d = 8) and at the
    paper's hundred-variable quartic, on sampled rows of the N x N map."""
    pl = S.Plan(n, d, 8, "bf16x3")
    got = pl.pair_ranks()
    rows = np.unique(np.r_[0, 1, pl.N - 1, pl.N // 2, np.random.default_rng(6).integers(0, pl.N, 40)])
    want = O.pair_ranks_sparse(n, d, rows=rows)
    assert np.array_equal(got[torch.tensor(rows, device=dev())].cpu().numpy(), want)


def test_pair_ranks_n12d6_sampled_rows():
    n, d = 12, 6
    pl = S.Plan(n, d, 8, "bf16x3")
    got = pl.pair_ranks()
    rows = np.unique(np.r_[0, 1, pl.N - 1, pl.N // 2, np.random.default_rng(5).integers(0, pl.N, 60)])
    want = O.pair_ranks(n, d, rows=rows)
    assert np.array_equal(got[torch.tensor(rows, device=dev())].cpu().numpy(), want)
    del got
    torch.cuda.empty_cache()


# ---------------------------------------------------------------------------
# Loss / gradient parity at sizes that span several tiles and ragged tails
# ---------------------------------------------------------------------------

# (17, 2) and (40, 2) take the variable-list ranking (n > 16)
CASES = [(1, 1, 1), (3, 2, 20), (4, 3, 37), (6, 3, 168), (6, 4, 420), (10, 5, 300), (17, 2, 40), (40, 2, 130)]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("n,d,k", CASES)
def test_loss_grad_parity(prec, n, d, k):
    W64, Wd, p, pd = make_case(n, d, k, prec, seed=n * 10 + d)
    pl = S.Plan(n, d, k, prec)
    loss, g, r = pl.loss_grad(Wd, pd, grad=True, want_r=True)
    torch.cuda.synchronize()
    pr = O.pair_ranks(n, d)
    L_o, g_o, r_o = O.loss_grad(W64, p, n, d, pr)
    c_o = r_o + p
    cabs = O.coefficients_abs(W64, n, d, pr)
    tf = tol_for(prec, k)
    c_gpu = r.cpu().numpy() + p
    assert_close_scaled(c_gpu, c_o, cabs, tf, "coefficients")
    dL = 2.0 * np.sum(np.abs(r_o) * tf * cabs) + np.sum((tf * cabs) ** 2)
    assert abs(float(loss.item()) - L_o) <= dL + 1e-12 * L_o
    N = W64.shape[0]
    tb = tol_for(prec, N)
    gabs = 4.0 * (np.abs(r_o)[pr] @ np.abs(W64))
    # the backward sees r with the forward's error, which moves g by at most 4 |dR| |W|
    gabs_fwd = 4.0 * ((tf * cabs + 0.0)[pr] @ np.abs(W64))
    err = np.abs(g.double().cpu().numpy() - g_o)
    assert np.all(err <= tb * gabs + gabs_fwd + 1e-300), f"gradient: max ratio {np.max(err / (tb * gabs + gabs_fwd + 1e-300)):.3g}"


@pytest.mark.parametrize("n,d,k", [(3, 2, 20), (6, 4, 420), (10, 5, 300)])
def test_single_product_backward(n, d, k):
    """SOS_FLAG_SINGLE_BACKWARD: split-bf16 forward, one bf16 product in R W."""
    W64, Wd, p, pd = make_case(n, d, k, "bf16x3", seed=n + d)
    pl = S.Plan(n, d, k, "bf16x3")
    loss, g, r = pl.loss_grad(Wd, pd, grad=True, want_r=True, single_backward=True)
    pr = O.pair_ranks(n, d)
    L_o, g_o, r_o = O.loss_grad(W64, p, n, d, pr)
    cabs = O.coefficients_abs(W64, n, d, pr)
    tf = tol_for("bf16x3", k)
    assert_close_scaled(r.cpu().numpy() + p, r_o + p, cabs, tf, "coefficients")
    N = W64.shape[0]
    tb = tol_for("bf16x1", N)
    gabs = 4.0 * (np.abs(r_o)[pr] @ np.abs(W64))
    gabs_fwd = 4.0 * ((tf * cabs)[pr] @ np.abs(W64))
    err = np.abs(g.double().cpu().numpy() - g_o)
    assert np.all(err <= tb * gabs + gabs_fwd + 1e-300)


def test_fp32_forward_rung_in_split_plan():
    """SOS_FLAG_FP32_FORWARD in a split-bf16 plan: FP32 MFMA on the FP32 master."""
    n, d, k = 6, 4, 420
    W64, Wd, p, pd = make_case(n, d, k, "bf16x3", seed=8)
    pl = S.Plan(n, d, k, "bf16x3")
    loss, _, r = pl.loss_grad(Wd, pd, grad=False, want_r=True, fp32_forward=True)
    pr = O.pair_ranks(n, d)
    L_o, _, r_o = O.loss_grad(W64, p, n, d, pr)
    cabs = O.coefficients_abs(W64, n, d, pr)
    assert_close_scaled(r.cpu().numpy() + p, r_o + p, cabs, tol_for("fp32", k), "fp32-rung coefficients")


def test_solve_three_rung_ladder():
    n, d = 4, 3
    N = comb(n + d, d)
    p = O.coefficients(gaussian((N, N // 2), 0), n, d)
    pl = S.Plan(n, d, 2 * N, "bf16x3")
    Wd = to_dev(gaussian((N, 2 * N), 1, 1 / math.sqrt(2 * N)), torch.float32)
    res = pl.solve(Wd, to_dev(p, torch.float64), S.Adam(lr=3e-3), tol=1e-8, max_steps=30000, check_every=20,
                   ladder=True, stall_checks=8, stall_ratio=0.8, switch_rel=1e-5, mid_rel=3e-7,
                   lr_exact=1e-3, rollback_ratio=10.0, single_backward=True)
    assert res["status"] == S.OK and res["phase"] == 2, res
    L_o, _, _ = O.loss_grad(Wd.double().cpu().numpy(), p, n, d)
    assert math.sqrt(L_o) / np.linalg.norm(p) <= 1e-8


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_exact_forward_is_fp64(prec):
    n, d, k = 6, 4, 420
    W64, Wd, p, pd = make_case(n, d, k, prec, seed=3)
    pl = S.Plan(n, d, k, prec)
    loss, _, r = pl.loss_grad(Wd, pd, grad=False, want_r=True, exact=True)
    pr = O.pair_ranks(n, d)
    L_o, _, r_o = O.loss_grad(W64, p, n, d, pr)
    cabs = O.coefficients_abs(W64, n, d, pr)
    assert_close_scaled(r.cpu().numpy() + p, r_o + p, cabs, 1e-10, "exact coefficients")
    assert abs(loss.item() - L_o) <= 1e-10 * L_o


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_verify_matches_oracle(prec):
    n, d, k = 4, 3, 50
    W64, Wd, p, pd = make_case(n, d, k, prec, seed=4)
    pl = S.Plan(n, d, k, prec)
    rel, r = pl.verify(Wd, pd, want_r=True)
    L_o, _, r_o = O.loss_grad(W64, p, n, d)
    assert abs(rel - math.sqrt(L_o) / np.linalg.norm(p)) <= 1e-10 * rel


# ---------------------------------------------------------------------------
# Adam steps and trajectories (FP64)
# ---------------------------------------------------------------------------

def test_adam_steps_fp64():
    n, d, k = 4, 3, 40
    W64, Wd, p, pd = make_case(n, d, k, "fp64", seed=5, wstd=0.3)
    pl = S.Plan(n, d, k, "fp64")
    st = pl.new_state()
    adam = S.Adam(lr=1e-2)
    pr = O.pair_ranks(n, d)
    ost = O.AdamState(np.zeros_like(W64), np.zeros_like(W64))
    Wo = W64.copy()
    for t in range(1, 6):
        loss = pl.step(Wd, st, t, pd, adam)
        L_o, g_o, _ = O.loss_grad(Wo, p, n, d, pr)
        Wo = O.adam_step(Wo, g_o, ost, 1e-2)
        assert abs(loss.item() - L_o) <= 1e-10 * L_o
        assert np.max(np.abs(Wd.cpu().numpy() - Wo)) <= 1e-9 * np.max(np.abs(Wo))


def test_trajectory_fp64_config_n3d2():
    c = CONFIGS["n3d2"]
    W0 = c.W0()
    p = O.coefficients(W0, c.n, c.d)
    pl = S.Plan(c.n, c.d, c.rank, "fp64")
    Wd = to_dev(c.W_init(), torch.float64)
    pd = to_dev(p, torch.float64)
    st = pl.new_state()
    adam = S.Adam(lr=0.1)
    res = O.solve(p, c.n, c.d, c.W_init(), 50, 0.1)
    for t in range(1, 51):
        loss = pl.step(Wd, st, t, pd, adam)
        assert abs(loss.item() - res.losses[t - 1]) <= 1e-9 * res.losses[t - 1], t


def test_solve_config_n3d2_fp64():
    c = CONFIGS["n3d2"]
    p = O.coefficients(c.W0(), c.n, c.d)
    ores = O.solve(p, c.n, c.d, c.W_init(), 2000, 0.1)
    o_rel = math.sqrt(ores.best_loss) / np.linalg.norm(p)
    pl = S.Plan(c.n, c.d, c.rank, "fp64")
    Wd = to_dev(c.W_init(), torch.float64)
    res = pl.solve(Wd, to_dev(p, torch.float64), S.Adam(lr=0.1), tol=1e-30, max_steps=2000, check_every=1)
    assert res["steps"] == 2000 and res["status"] == S.NOT_CONVERGED
    assert res["best_rel"] <= 1e-3
    # Adam at this step size on this sublinear problem amplifies rounding-level
    # differences over 2000 steps: the oracle's own best residual moves by
    # several percent when its start is perturbed at 1e-15, and the GPU sums
    # in another order (FP64 atomics).  The per-step parity is pinned by the
    # 50-step trajectory test; here the GPU must land inside the oracle's
    # spread under such perturbations (with 10% slack on either side).
    rng = np.random.default_rng(11)
    pn = np.linalg.norm(p)
    spread = [o_rel]
    for _ in range(6):
        Wp = c.W_init() * (1 + 1e-15 * rng.standard_normal((c.N, c.rank)))
        spread.append(math.sqrt(O.solve(p, c.n, c.d, Wp, 2000, 0.1).best_loss) / pn)
    assert 0.9 * min(spread) <= res["best_rel"] <= 1.1 * max(spread), (res["best_rel"], spread)
    L_o, _, _ = O.loss_grad(Wd.cpu().numpy(), p, c.n, c.d)
    assert abs(res["rel"] - math.sqrt(L_o) / np.linalg.norm(p)) <= 1e-9 * res["rel"]


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_solve_reaches_1e8_with_ladder(prec):
    n, d = 3, 2
    N = comb(n + d, d)
    W0 = gaussian((N, N), 0)
    p = O.coefficients(W0, n, d)
    pl = S.Plan(n, d, 2 * N, prec)
    Wd = to_dev(gaussian((N, 2 * N), 1, 0.1), torch.float32)
    res = pl.solve(Wd, to_dev(p, torch.float64), S.Adam(lr=0.03), tol=1e-8, max_steps=20000,
                   check_every=50, ladder=True, stall_checks=4, stall_ratio=0.7)
    assert res["status"] == S.OK, res
    L_o, _, _ = O.loss_grad(Wd.double().cpu().numpy(), p, n, d)
    assert math.sqrt(L_o) / np.linalg.norm(p) <= 1e-8


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_motzkin_stays_away_from_zero(prec):
    n, d = 3, 3
    p = O.poly_vector(motzkin_terms(n), n, d)
    dist2 = O.psd_distance(p, n, d).dist2
    N = comb(n + d, d)
    pl = S.Plan(n, d, 2 * N, prec)
    wdt = torch.float64 if prec == "fp64" else torch.float32
    Wd = to_dev(gaussian((N, 2 * N), 1, 0.3), wdt)
    pd = to_dev(p, torch.float64)
    st = pl.new_state()
    adam = S.Adam(lr=1e-2)
    steps = 20000     # the oracle's Adam needs ~2e4 steps at this lr to come within 1% of dist^2
    losses = torch.empty(steps, dtype=torch.float64, device=dev())
    for t in range(1, steps + 1):
        pl.step(Wd, st, t, pd, adam, loss=losses[t - 1:t], flags=S.FLAG_EXACT_FORWARD if prec != "fp64" else 0)
    L = losses.cpu().numpy()
    assert L.min() >= dist2 * (1 - 1e-9)
    assert L.min() <= dist2 * 1.05
    assert pl.verify(Wd, pd) >= math.sqrt(dist2) / np.linalg.norm(p) * (1 - 1e-9)


# ---------------------------------------------------------------------------
# Differentiation: autograd.Function vs central differences and the oracle
# ---------------------------------------------------------------------------

def test_sosloss_autograd_matches_fd_and_oracle():
    n, d, k = 10, 5, 3003
    N = comb(n + d, d)
    c = CONFIGS["n10d5"]
    W0 = gaussian((N, 300), 0, 1 / math.sqrt(300))
    p = O.coefficients(W0, n, d)
    pl = S.Plan(n, d, k, "bf16x3")
    W = to_dev(gaussian((N, k), 1, 1 / math.sqrt(k)), torch.float32).requires_grad_(True)
    pd = to_dev(p, torch.float64)
    L = S.SosLoss.apply(W, pd, pl)
    L.backward()
    g = W.grad.double().cpu().numpy()
    Wn = W.detach().double().cpu().numpy()
    pr = O.pair_ranks(n, d)
    L_o, g_o, r_o = O.loss_grad(Wn, p, n, d, pr)
    gabs = 4.0 * (np.abs(r_o)[pr] @ np.abs(Wn))
    cabs = O.coefficients_abs(Wn, n, d, pr)
    tf, tb = tol_for("bf16x3", k), tol_for("bf16x3", N)
    gabs_fwd = 4.0 * ((tf * cabs)[pr] @ np.abs(Wn))
    assert np.all(np.abs(g - g_o) <= tb * gabs + gabs_fwd)
    # central differences of the exact FP64 forward on 64 random entries (seed 2)
    rng = np.random.default_rng(2)
    idx = [(int(rng.integers(0, N)), int(rng.integers(0, k))) for _ in range(64)]
    Wd = W.detach().clone()
    for i, j in idx:
        x0 = Wd[i, j].item()
        vals = {}
        for s in (+1, -1):
            Wd[i, j] = x0 + s * 2.0 ** -7
            h = Wd[i, j].item() - x0
            lo, _, _ = pl.loss_grad(Wd, pd, grad=False, exact=True)
            vals[s] = (lo.item(), h)
        Wd[i, j] = x0
        fd = (vals[1][0] - vals[-1][0]) / (vals[1][1] - vals[-1][1])
        # curvature term of an O(h^2) central difference, bounded by the oracle's exact value
        assert abs(fd - g_o[i, j]) <= 1e-3 * abs(g_o).max() + 1e-6, (i, j, fd, g_o[i, j])
        assert abs(g[i, j] - g_o[i, j]) <= tb * gabs[i, j] + gabs_fwd[i, j]




# ---------------------------------------------------------------------------
# Fused backward + Adam: the copies its epilogue leaves for the next step
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("exact", [False, True])
@pytest.mark.parametrize("n,d,k", [(6, 4, 420), (10, 5, 300)])
def test_fused_step_leaves_the_copies_the_next_step_needs(n, d, k, exact):
    """A split plan's single-product step updates W in the backward GEMM's
    epilogue and writes there the operand copies of the new W; the next step
    with SOS_FLAG_COPIES_VALID uses them instead of preparing its own.  That
    step's loss and gradient must equal those from freshly prepared copies of
    the same W (sos_loss_grad), and its update must be the Adam formula."""
    _, Wd, _, pd = make_case(n, d, k, "bf16x3", seed=9)
    pl = S.Plan(n, d, k, "bf16x3")
    N = pl.N
    st = pl.new_state()
    base = S.FLAG_SINGLE_BACKWARD | (S.FLAG_EXACT_FORWARD if exact else 0)
    adam = S.Adam(lr=1e-3)
    for t in (1, 2):
        pl.step(Wd, st, t, pd, adam, flags=base | S.FLAG_COPIES_VALID)
    W_before = Wd.clone()
    adam0 = S.Adam(lr=1e-3, beta1=0.0)                 # first moment = this step's gradient
    L3 = pl.step(Wd, st, 3, pd, adam0, flags=base | S.FLAG_COPIES_VALID).item()
    torch.cuda.synchronize()
    slot = pl.state_bytes // 4
    g3 = st[: N * k * 4].view(torch.float32).reshape(N, k).clone()
    v3 = st[slot: slot + N * k * 4].view(torch.float32).reshape(N, k).clone()
    L_ref, g_ref, _ = pl.loss_grad(W_before, pd, grad=True, exact=exact, single_backward=True)
    assert abs(L3 - L_ref.item()) <= 1e-12 * L_ref.item(), (L3, L_ref.item())
    assert torch.equal(g3, g_ref)
    want = W_before.double() - 1e-3 * g3.double() / (torch.sqrt(v3.double() / (1 - 0.999 ** 3)) + 1e-8)
    assert bool(((Wd.double() - want).abs() <= 1e-6 * want.abs() + 1e-8).all())
