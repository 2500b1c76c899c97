"""The paper's largest workload at full size: quartic forms in 100 variables
(Section 1.2, Section 3.1 table), i.e. (n, d) = (99, 2) in the degree-<=d
basis: N = 5,050, M = 4,421,275, full rank k = N.  The ranking takes the
variable-list encoding (n > 16).  The oracle forms the whole coefficient
vector here (25.5 M pairs, row blocks of 505), so the comparison is
element by element, for the coefficients and for sampled gradient rows
(including the ragged last tile row, 4,864 .. 5,049).
"""
import math

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


@pytest.fixture(scope="module")
def case():
    n, d = 99, 2
    N = math.comb(n + d, d)
    k = N
    W = gaussian((N, k), 41, 1.0 / math.sqrt(k))
    Wd = torch.tensor(W, dtype=torch.float32, device="cuda")
    W64 = Wd.double().cpu().numpy()
    M = math.comb(n + 2 * d, 2 * d)
    p = gaussian(M, 42)
    # oracle coefficients, row block by row block
    G = W64 @ W64.T
    Ga = np.abs(W64) @ np.abs(W64).T
    c = np.zeros(M)
    cabs = np.zeros(M)
    basis, cidx = O.monomials_sparse(n, d), O.SparseIndex(n, 2 * d)
    for r0 in range(0, N, 505):
        rows = np.arange(r0, min(N, r0 + 505))
        pr = O.pair_ranks_sparse(n, d, rows=rows, basis=basis, cidx=cidx)
        c += np.bincount(pr.ravel(), weights=G[rows].ravel(), minlength=M)
        cabs += np.bincount(pr.ravel(), weights=Ga[rows].ravel(), minlength=M)
    return dict(n=n, d=d, N=N, M=M, k=k, Wd=Wd, W64=W64, p=p, c=c, cabs=cabs, basis=basis, cidx=cidx)


@pytest.mark.parametrize("prec,exact", [("bf16x3", False), ("bf16x3", True), ("fp32", False)])
def test_quartic100_coefficients(case, prec, exact):
    pl = S.Plan(case["n"], case["d"], case["k"], prec)
    pd = torch.tensor(case["p"], dtype=torch.float64, device="cuda")
    L, _, r = pl.loss_grad(case["Wd"], pd, grad=False, want_r=True, exact=exact)
    got = r.cpu().numpy() + case["p"]
    K = case["k"]
    tol = 1e-10 if exact else (gamma(K + 1) + U32 if prec == "fp32" else 3.1 * 2.0 ** -16 + gamma(3 * K) + U32)
    bound = tol * case["cabs"] + 1e-15 * np.abs(case["p"])
    err = np.abs(got - case["c"]) / bound
    assert err.max() <= 1.0, f"max |err|/bound {err.max():.3g}"
    want_L = float(np.sum((case["c"] - case["p"]) ** 2))
    dc = tol * case["cabs"]
    assert abs(L.item() - want_L) <= 2 * np.sum(np.abs(case["c"] - case["p"]) * dc) + np.sum(dc * dc) + 1e-12 * want_L


def test_quartic100_ozaki_coefficients(case):
    """The int8 Ozaki forward on all 4,421,275 coefficients: within its
    truncation bound (7.05 2^-42 K 2^(e_i + e_j) per Gram entry, 2^e_i the
    least power of two above row i's largest magnitude, pair-summed by the
    oracle's own map) and within 1e-10 of coeff(|W||W|^T)."""
    n, d, N, M, K = case["n"], case["d"], case["N"], case["M"], case["k"]
    pl = S.Plan(n, d, K, "bf16x3")
    pd = torch.tensor(case["p"], dtype=torch.float64, device="cuda")
    _, _, r = pl.loss_grad(case["Wd"], pd, grad=False, want_r=True, ozaki=True)
    got = r.cpu().numpy() + case["p"]
    _, e = np.frexp(np.abs(case["W64"]).max(axis=1))
    sc = np.ldexp(1.0, e)
    cs = np.zeros(M)
    for r0 in range(0, N, 505):
        rows = np.arange(r0, min(N, r0 + 505))
        pr = O.pair_ranks_sparse(n, d, rows=rows, basis=case["basis"], cidx=case["cidx"])
        cs += np.bincount(pr.ravel(), weights=np.outer(sc[rows], sc).ravel(), minlength=M)
    slack = 1e-13 * (case["cabs"] + np.abs(case["p"]))
    err = np.abs(got - case["c"])
    assert np.max(err / (7.05 * 2.0 ** -42 * K * cs + slack)) <= 1.0
    assert np.max(err / (1e-10 * case["cabs"] + 1e-15 * np.abs(case["p"]))) <= 1.0


@pytest.mark.parametrize("prec,exact,single", [("bf16x3", False, True), ("bf16x3", True, False), ("fp32", False, False)])
def test_quartic100_gradient_rows(case, prec, exact, single):
    """Rows of 4 R W against the oracle's r (bound: the backward's own error
    relative to 4 |R| |W|, plus the forward's carried through 4 |dR| |W|)."""
    n, d, N, K = case["n"], case["d"], case["N"], case["k"]
    pl = S.Plan(n, d, K, prec)
    pd = torch.tensor(case["p"], dtype=torch.float64, device="cuda")
    _, g, _ = pl.loss_grad(case["Wd"], pd, grad=True, exact=exact, single_backward=single)
    rng = np.random.default_rng(57)
    rows = np.unique(np.concatenate([[0, 255, 256, 4863, 4864, 4865, N - 2, N - 1],
                                     rng.choice(N, 12, replace=False)]))
    got = g[torch.as_tensor(rows, device="cuda")].double().cpu().numpy()
    P = O.pair_ranks_sparse(n, d, rows=rows, basis=case["basis"], cidx=case["cidx"])
    r = case["c"] - case["p"]
    W64 = case["W64"]
    want = 4.0 * (r[P] @ W64)
    Wa = np.abs(W64)
    if prec == "fp32":
        tol_f, tol_b = gamma(K + 1) + U32, gamma(N + 1) + U32
    else:
        tol_f = 1e-10 if exact else 3.1 * 2.0 ** -16 + gamma(3 * K) + U32
        tol_b = (2.0 ** -7 + 2.0 ** -16 + gamma(N) + U32) if single else (3.1 * 2.0 ** -16 + gamma(3 * N) + U32)
    bound = tol_b * 4.0 * (np.abs(r[P]) @ Wa) + 4.0 * ((tol_f * case["cabs"])[P] @ Wa) + 1e-30
    worst = np.abs(got - want) / bound
    assert worst.max() <= 1.0, f"max |err|/bound {worst.max():.3g} at row {rows[np.argmax(worst.max(1))]}"
