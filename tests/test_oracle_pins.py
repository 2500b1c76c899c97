"""Pins for the FP64 oracle: checks against what the paper and mathematics fix.

None of these re-types an oracle formula: each compares the oracle with an
independent route (a printed example, brute force, symbolic expansion, a
different derivation, a closed form, an invariant or a second algorithm).
"""
import itertools
import os
from math import comb, factorial, sqrt

import numpy as np
import pytest

import oracle as O
from workloads import CONFIGS, gaussian, motzkin_terms

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_rows(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


# --- ordering and counts (Section 1.1, Section 1.2, Section 3.1 table) ---------

def test_order_matches_paper_example():
    want = np.array([[int(a) for a in r] for r in _golden_rows("order_n2d2.txt")])
    assert (O.monomials(2, 2) == want).all()


@pytest.mark.parametrize("n,D", [(1, 5), (2, 4), (3, 4), (4, 3), (3, 6), (5, 2)])
def test_enumeration_matches_bruteforce(n, D):
    assert (O.monomials(n, D) == O.monomials_bruteforce(n, D)).all()


@pytest.mark.parametrize("n,D", [(3, 2), (6, 4), (6, 8), (10, 5), (4, 11)])
def test_counts_are_binomials(n, D):
    assert O.monomials(n, D).shape[0] == comb(n + D, D)


def test_quartic_form_counts_from_table():
    for n_forms, m in _golden_rows("quartic_counts.txt"):
        n_forms, m = int(n_forms), int(m)
        # homogenisation: quartic forms in n variables <-> degree <= 4 in n-1 variables
        if n_forms <= 30:
            assert O.monomials(n_forms - 1, 4).shape[0] == m
        else:
            assert comb(n_forms - 1 + 4, 4) == m


def test_burer_monteiro_numbers():
    g = {k: float(v) for k, v in _golden_rows("bm_numbers.txt")}
    l = comb(99 + 2, 2)
    m = comb(99 + 4, 4)
    assert l == g["l"] and m == g["m"]
    assert int(sqrt(2 * m)) == g["sqrt2m"]          # the paper truncates 2973.6
    assert abs(l * sqrt(2 * m) - g["lp"]) / g["lp"] < 1e-3
    assert abs(l * (l + 1) / 2 - g["sym"]) / g["sym"] < 1e-3


def test_pair_ranks_match_dictionary():
    for n, d in [(2, 2), (3, 2), (3, 3), (4, 2), (2, 5)]:
        basis = [tuple(r) for r in O.monomials_bruteforce(n, d)]
        coeffs = {tuple(r): k for k, r in enumerate(O.monomials_bruteforce(n, 2 * d))}
        want = np.array([[coeffs[tuple(a + b for a, b in zip(x, y))] for y in basis] for x in basis])
        assert (O.pair_ranks(n, d) == want).all()


# --- coefficients: symbolic expansion and evaluation identity (eq. basicsos) ---

@pytest.mark.parametrize("n,d,k", [(1, 2, 2), (2, 1, 3), (2, 2, 3), (3, 2, 4), (3, 1, 2)])
def test_coefficients_match_sympy_expansion(n, d, k):
    sympy = pytest.importorskip("sympy")
    xs = sympy.symbols(f"x1:{n + 1}")
    rng = np.random.default_rng(7 + n + 10 * d)
    W = rng.integers(-3, 4, size=(comb(n + d, d), k))
    basis = O.monomials(n, d)
    mono = [sympy.Mul(*[x ** int(e) for x, e in zip(xs, a)]) for a in basis]
    poly = sympy.expand(sum((sum(int(W[i, l]) * mono[i] for i in range(len(mono)))) ** 2
                            for l in range(k)))
    P = sympy.Poly(poly, *xs)
    cidx = O.MonomialIndex(n, 2 * d)
    want = np.zeros(len(cidx))
    for expo, val in P.terms():
        want[int(cidx.lookup(np.array([expo]))[0])] = int(val)
    got = O.coefficients(W.astype(float), n, d)
    assert np.array_equal(got, want)          # integers below 2^53: exact


@pytest.mark.parametrize("n,d", [(3, 2), (2, 4), (4, 3)])
def test_evaluation_identity(n, d):
    N = comb(n + d, d)
    W = gaussian((N, N + 3), 11)
    c = O.coefficients(W, n, d)
    rng = np.random.default_rng(3)
    for _ in range(5):
        x = rng.uniform(-1.2, 1.2, size=n)
        lhs = O.evaluate_poly(c, n, 2 * d, x)
        rhs = O.evaluate_sos(W, n, d, x)
        assert abs(lhs - rhs) <= 1e-12 * abs(rhs)
    # at x = 1 every monomial is 1: sum of all coefficients = ||W^T 1||^2
    assert abs(c.sum() - np.sum(W.sum(axis=0) ** 2)) <= 1e-12 * np.sum(W.sum(axis=0) ** 2)


@pytest.mark.parametrize("n,m,k", [(2, 2, 3), (3, 3, 5), (4, 6, 7), (5, 5, 4)])
def test_network_pairing_identities(n, m, k):
    """Quartic coefficients from the paper's 4th-derivative pairing identities
    (Section 2) equal the oracle's gram-scatter on the network's factor."""
    rng = np.random.default_rng(100 + n)
    A = rng.standard_normal((m, n))
    B = rng.standard_normal((k, n * m))
    W = O.network_factor(A, B)
    c = O.coefficients(W, n, 2)
    cidx = O.MonomialIndex(n, 4)
    want = O.network_quartic_coefficients(A, B)
    got = {}
    for pos, e in enumerate(cidx.exps):
        if e.sum() == 4:
            got[tuple(int(v) for v in e)] = c[pos]
        else:
            assert abs(c[pos]) < 1e-12      # a quartic form has no lower-degree terms
    assert set(got) == set(want)
    scale = max(abs(v) for v in want.values())
    for key, v in want.items():
        assert abs(got[key] - v) <= 1e-12 * scale


# --- gradient: Richardson-extrapolated central differences -------------------

@pytest.mark.parametrize("n,d,k", [(3, 2, 7), (2, 3, 5)])
def test_gradient_matches_finite_differences(n, d, k):
    """L is a quartic polynomial in each single entry of W, so the Richardson
    combination (4 D(h) - D(2h)) / 3 of central differences is exact up to
    rounding (it cancels the only truncation term, h^2 f'''/6)."""
    N = comb(n + d, d)
    W = gaussian((N, k), 5, 0.5)
    p = gaussian(comb(n + 2 * d, 2 * d), 6)
    L, g, _ = O.loss_grad(W, p, n, d)

    def Lat(i, j, h):
        Wp = W.copy()
        Wp[i, j] += h
        return O.loss_grad(Wp, p, n, d)[0]

    rng = np.random.default_rng(9)
    for _ in range(12):
        i, j = rng.integers(0, N), rng.integers(0, k)
        h = 1e-3
        D1 = (Lat(i, j, h) - Lat(i, j, -h)) / (2 * h)
        D2 = (Lat(i, j, 2 * h) - Lat(i, j, -2 * h)) / (4 * h)
        fd = (4 * D1 - D2) / 3
        assert abs(fd - g[i, j]) <= 1e-8 * max(abs(g).max(), 1.0)


# --- invariants ---------------------------------------------------------------

def test_orthogonal_and_scaling_invariance():
    n, d, k = 3, 3, 25
    N = comb(n + d, d)
    W = gaussian((N, k), 21)
    p = gaussian(comb(n + 2 * d, 2 * d), 22)
    Q, _ = np.linalg.qr(gaussian((k, k), 23))
    L, g, _ = O.loss_grad(W, p, n, d)
    L2, g2, _ = O.loss_grad(W @ Q, p, n, d)
    assert abs(L - L2) <= 1e-12 * L
    assert np.abs(g @ Q - g2).max() <= 1e-11 * np.abs(g).max()
    s = 1.7
    assert np.allclose(O.coefficients(s * W, n, d), s * s * O.coefficients(W, n, d), rtol=1e-13)


def test_sampled_coefficients_match_full():
    n, d = 4, 3
    N = comb(n + d, d)
    W = gaussian((N, 30), 31)
    p = gaussian(comb(n + 2 * d, 2 * d), 32)
    c = O.coefficients(W, n, d)
    betas = np.arange(0, len(c), 7)
    assert np.allclose(O.sample_coefficients(W, n, d, betas), c[betas], rtol=1e-12, atol=1e-12)
    _, g, _ = O.loss_grad(W, p, n, d)
    rows = [0, 5, N - 1]
    assert np.allclose(O.sample_gradient_rows(W, p, n, d, rows), g[rows], rtol=1e-11, atol=1e-11)


# --- Adam (Section 3): a library implementation and a closed-form case --------

def test_adam_matches_torch_adam():
    torch = pytest.importorskip("torch")
    W = gaussian((6, 4), 41)
    gs = [gaussian((6, 4), 42 + t) for t in range(5)]
    st = O.AdamState(np.zeros_like(W), np.zeros_like(W))
    Wo = W.copy()
    for g in gs:
        Wo = O.adam_step(Wo, g, st, lr=0.01, beta1=0.9, beta2=0.999, eps=1e-8)
    P = torch.nn.Parameter(torch.tensor(W, dtype=torch.float64))
    opt = torch.optim.Adam([P], lr=0.01, betas=(0.9, 0.999), eps=1e-8)
    for g in gs:
        P.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
    assert np.allclose(P.detach().numpy(), Wo, rtol=1e-14, atol=1e-15)


def test_adam_constant_gradient_moves_by_lr():
    # with a constant gradient the bias-corrected moments are exactly g and g^2
    W = np.zeros(3)
    g = np.array([2.0, -0.5, 1e-3])
    st = O.AdamState(np.zeros(3), np.zeros(3))
    for _ in range(7):
        W = O.adam_step(W, g, st, lr=0.1, eps=0.0)
    assert np.allclose(W, -0.7 * np.sign(g), rtol=1e-12)


# --- convergence: SOS by construction, Motzkin bounded away from 0 ------------

def test_sos_by_construction_converges():
    n, d = 3, 2
    N = comb(n + d, d)
    W0 = gaussian((N, N), 0)
    p = O.coefficients(W0, n, d)
    res = O.solve(p, n, d, gaussian((N, 2 * N), 1, 0.1), 3000, 0.03)
    assert sqrt(res.best_loss) / np.linalg.norm(p) < 1e-9


def test_config_n3d2_rank3_target():
    """The n=3, d=2 workload (W0 rank 3) converges only sublinearly: it must
    still drop by orders of magnitude within 2000 steps."""
    c = CONFIGS["n3d2"]
    p = O.coefficients(c.W0(), c.n, c.d)
    res = O.solve(p, c.n, c.d, c.W_init(), 2000, 0.1)
    rel = sqrt(res.best_loss) / np.linalg.norm(p)
    assert rel < 1e-3
    assert res.losses[0] > 1e4 * res.best_loss


def test_motzkin_distance_two_ways():
    """Motzkin is not SOS: its distance to the SOS cone is positive.  The convex
    solver (with its KKT certificate) and Adam on a full-rank factor agree, and
    no iterate of the factored method goes below the convex minimum."""
    n, d = 3, 3
    p = O.poly_vector(motzkin_terms(n), n, d)
    assert abs(p @ p - 12.0) < 1e-15
    cv = O.psd_distance(p, n, d)
    assert cv.dist2 > 1e-4
    assert cv.kkt_min_eig > -1e-8 and abs(cv.kkt_gap) < 1e-8
    N = comb(n + d, d)
    res = O.solve(p, n, d, gaussian((N, 2 * N), 1, 0.3), 40000, 1e-2)
    assert min(res.losses) >= cv.dist2 * (1 - 1e-9)
    assert res.best_loss <= cv.dist2 * (1 + 1e-2)


@pytest.mark.parametrize("n", [4, 5])
def test_motzkin_padding_keeps_distance(n):
    """Variables the Motzkin form does not use cannot lower its distance (Gram
    entries of monomials holding those variables feed no coefficient of p)."""
    p3 = O.poly_vector(motzkin_terms(3), 3, 3)
    base = O.psd_distance(p3, 3, 3).dist2
    pn = O.poly_vector(motzkin_terms(n), n, 3)
    assert abs(O.psd_distance(pn, n, 3, iters=6000).dist2 - base) <= 1e-6 * base


# ---------------------------------------------------------------------------
# Sparse (variable-list) representation for many variables
# ---------------------------------------------------------------------------

def _dense_of(lists, n):
    out = np.zeros((lists.shape[0], n), dtype=np.int64)
    for q in range(lists.shape[1]):
        v = lists[:, q]
        ok = v >= 0
        np.add.at(out, (np.nonzero(ok)[0], v[ok]), 1)
    return out


@pytest.mark.parametrize("n,D", [(1, 3), (3, 4), (5, 4), (20, 3)])
def test_sparse_order_is_the_basis_order(n, D):
    """Lexicographic ascending variable lists, degree by degree, reproduce the
    dense basis order (itself pinned to the Section 1.1 example)."""
    assert np.array_equal(_dense_of(O.monomials_sparse(n, D), n), O.monomials(n, D))


@pytest.mark.parametrize("n,d", [(2, 2), (4, 2), (6, 3), (3, 5)])
def test_sparse_pair_ranks_equal_dense(n, d):
    assert np.array_equal(O.pair_ranks_sparse(n, d), O.pair_ranks(n, d))


def test_sparse_counts_of_the_hundred_variable_quartic():
    """Section 1.2: quartics in 100 variables have l = 5,050 basis monomials and
    m = 4,421,275 coefficients; as forms in n = 100 they are our (99, 2)."""
    assert len(O.monomials_sparse(99, 2)) == 5050
    assert len(O.SparseIndex(99, 4)) == 4421275


def test_sparse_evaluation_identity_many_variables():
    """sum_b c_b x^b = ||W^T m_d(x)||^2 with the sparse ranks (n = 40, d = 2)."""
    n, d, k = 40, 2, 3
    rng = np.random.default_rng(3)
    basis = O.monomials_sparse(n, d)
    coeffs = O.monomials_sparse(n, 2 * d)
    W = rng.standard_normal((len(basis), k))
    c = O.coefficients(W, n, d, O.pair_ranks_sparse(n, d))
    for _ in range(3):
        x = rng.uniform(-1, 1, n)
        xe = np.append(x, 1.0)                         # index -1 (padding) reads 1
        m = np.prod(xe[basis], axis=1)
        xb = np.prod(xe[coeffs], axis=1)
        lhs = float(c @ xb)
        rhs = float(np.sum((W.T @ m) ** 2))
        assert abs(lhs - rhs) <= 1e-12 * (np.abs(c) @ np.abs(xb))


def test_network_gradient_matches_finite_differences():
    """dL/dA and dL/dB of the two-layer network (chain rule through 4 R W)
    against Richardson central differences (L is a polynomial in each weight)."""
    from oracle.sos import MonomialIndex
    n, m, k = 3, 4, 5
    rng = np.random.default_rng(11)
    A = rng.standard_normal((m, n)) * 0.5
    B = rng.standard_normal((k, n * m)) * 0.5
    p = rng.standard_normal(len(MonomialIndex(n, 4)))
    L, dA, dB = O.network_loss_grad(A, B, p)

    def fd(M, i, j):
        def Lat(h):
            M2 = M.copy()
            M2[i, j] += h
            args = (M2, B) if M is A else (A, M2)
            return O.network_loss_grad(*args, p)[0]
        D = lambda h: (Lat(h) - Lat(-h)) / (2 * h)
        return (4 * D(1e-4) - D(2e-4)) / 3
    for (i, j) in [(0, 0), (3, 2), (1, 1)]:
        assert abs(fd(A, i, j) - dA[i, j]) <= 1e-6 * max(1.0, abs(dA[i, j]))
    for (i, j) in [(0, 0), (4, 11), (2, 5)]:
        assert abs(fd(B, i, j) - dB[i, j]) <= 1e-6 * max(1.0, abs(dB[i, j]))
