"""FP64 oracle: monomial bases, coefficient extraction, loss, gradient, Adam.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain NumPy in FP64;
no blocking, fusion or reordering beyond the definitions.

Conventions (readings of the paper, each listed in the design doc):

* Basis (Section 1.1, eq. basicsos and its n=d=2 example): m_d holds all
  monomials of total degree <= d in n variables, ordered with higher total
  degree first and, within one degree, the lexicographically larger exponent
  vector first (x1 most significant) -- the order of the worked example
  (x1^2, x1 x2, x2^2, x1, x2, 1).
* Coefficients (Section 1.1, eq. nonconvex): the polynomial m_d^T G m_d of a
  Gram matrix G has coefficient c_beta = sum of G_ij over all ORDERED pairs
  (i, j) with alpha_i + alpha_j = beta.  Coefficient monomials (degree <= 2d)
  use the same order as the basis.
* Loss (eq. nonconvex, "un-normalized", Section 3): L(W) = ||c(W W^T) - p||^2,
  no factor 1/2 and no division by the number of coefficients.
* Gradient: dL = <2R, dW W^T + W dW^T> with R_ij = r[rank(alpha_i+alpha_j)]
  symmetric, so grad_W L = 4 R W.  (The paper differentiates automatically;
  this is the same derivative written out.)
* Optimiser (Section 3): Adam (Kingma and Ba, bias-corrected) from a random
  start; success is judged on the minimum error over all iterations.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field
from math import comb

import numpy as np


# ---------------------------------------------------------------------------
# Monomial enumeration and ordering (Section 1.1, eq. basicsos example)
# ---------------------------------------------------------------------------

def _grlex_desc_order(exps: np.ndarray) -> np.ndarray:
    """Permutation sorting exponent rows by (-|a|, -a_1, -a_2, ..., -a_n)."""
    deg = exps.sum(axis=1)
    keys = [-exps[:, v] for v in range(exps.shape[1] - 1, -1, -1)] + [-deg]
    return np.lexsort(keys)


def monomials_bruteforce(n: int, D: int) -> np.ndarray:
    """All alpha in {0..D}^n with |alpha| <= D by exhaustive product, sorted.

    Exponential in n; used only to pin ``monomials`` on tiny cases.
    """
    exps = [a for a in itertools.product(range(D + 1), repeat=n) if sum(a) <= D]
    exps.sort(key=lambda a: (-sum(a), tuple(-x for x in a)))
    return np.array(exps, dtype=np.int64).reshape(len(exps), n)


def monomials(n: int, D: int) -> np.ndarray:
    """Exponent vectors of all monomials of degree <= D in n variables.

    Built one variable at a time (each partial row is extended by every
    exponent that keeps the total <= D), then sorted into the basis order.
    Returns an int64 array of shape (C(n+D, D), n).
    """
    rows = np.zeros((1, 0), dtype=np.int64)
    for _ in range(n):
        tot = rows.sum(axis=1)
        parts = []
        for e in range(D + 1):
            keep = rows[tot + e <= D]
            if keep.shape[0] == 0:
                continue
            parts.append(np.hstack([keep, np.full((keep.shape[0], 1), e, dtype=np.int64)]))
        rows = np.vstack(parts)
    return rows[_grlex_desc_order(rows)]


class MonomialIndex:
    """Dictionary exponent-vector -> position in the degree-<=D list.

    Each exponent vector is encoded as the integer sum_v a_v * (D+1)^(n-1-v)
    (a base-(D+1) numeral; injective since every a_v <= D).  Lookups sort the
    codes once and binary-search them.
    """

    def __init__(self, n: int, D: int):
        self.n, self.D = n, D
        self.base = D + 1
        if (D + 1) ** n >= 2 ** 62:
            raise ValueError("exponent codes would overflow int64")
        self.exps = monomials(n, D)
        self.weights = np.array([self.base ** (n - 1 - v) for v in range(n)], dtype=np.int64)
        self.codes = self.exps @ self.weights
        self._sorter = np.argsort(self.codes, kind="stable")
        self._sorted = self.codes[self._sorter]

    def __len__(self) -> int:
        return self.exps.shape[0]

    def encode(self, exps: np.ndarray) -> np.ndarray:
        return np.asarray(exps, dtype=np.int64) @ self.weights

    def lookup_codes(self, codes: np.ndarray) -> np.ndarray:
        """Positions of encoded exponent vectors; -1 where absent."""
        codes = np.asarray(codes, dtype=np.int64)
        pos = np.searchsorted(self._sorted, codes)
        pos = np.clip(pos, 0, len(self._sorted) - 1)
        hit = self._sorted[pos] == codes
        return np.where(hit, self._sorter[pos], -1)

    def lookup(self, exps: np.ndarray) -> np.ndarray:
        exps = np.asarray(exps, dtype=np.int64)
        ok = (exps >= 0).all(axis=-1) & (exps <= self.D).all(axis=-1) & (exps.sum(axis=-1) <= self.D)
        out = self.lookup_codes(self.encode(np.where(ok[..., None], exps, 0)))
        return np.where(ok, out, -1)


def pair_ranks(n: int, d: int, rows=None) -> np.ndarray:
    """R-index matrix: entry (i, j) = position of alpha_i + alpha_j among the
    degree-<=2d monomials (eq. nonconvex: the monomial a Gram entry feeds).

    ``rows`` restricts i to a subset (for large bases).  Uses the fact that the
    base-(2d+1) code of a sum of two exponent vectors whose entries are <= d is
    the sum of their codes (no digit exceeds 2d, so nothing carries).  When
    those codes would overflow (many variables), the sparse variable-list
    index gives the same map (``pair_ranks_sparse``).
    """
    if (2 * d + 1) ** n >= 2 ** 62:
        return pair_ranks_sparse(n, d, rows)
    basis = monomials(n, d)
    cidx = MonomialIndex(n, 2 * d)
    bcode = cidx.encode(basis)
    ri = bcode if rows is None else bcode[np.asarray(rows)]
    out = cidx.lookup_codes(ri[:, None] + bcode[None, :])
    assert (out >= 0).all()
    return out


# ---------------------------------------------------------------------------
# The same order for many variables and low degree (sparse representation)
# ---------------------------------------------------------------------------
#
# With n ~ 100 and degree <= 4 (the paper's largest quartic workload, Section
# 1.2 and the Section 3.1 table), dense exponent vectors are wasteful (99
# entries, at most 4 nonzero) and their base-(D+1) codes overflow.  A monomial
# of degree t is also the multiset of its variables, written as the
# ascending list v_1 <= ... <= v_t.  Within one degree, the lexicographically
# larger exponent vector is exactly the lexicographically smaller list: at
# the first position where two lists differ, the one with the smaller
# variable has one more factor of that variable and the same count of every
# earlier one.  So each degree block of the basis order is the lexicographic
# enumeration of ascending lists, which is the order in which
# itertools.combinations_with_replacement produces them.

def monomials_sparse(n: int, D: int) -> np.ndarray:
    """Monomials of degree <= D in n variables, in the basis order, as
    ascending variable lists padded with -1: shape (C(n+D, D), D)."""
    rows = []
    for t in range(D, -1, -1):
        for c in itertools.combinations_with_replacement(range(n), t):
            rows.append(c + (-1,) * (D - t))
    return np.array(rows, dtype=np.int64).reshape(len(rows), D)


class SparseIndex:
    """Dictionary variable-list -> position in the degree-<=D list.

    A padded ascending list (v_1, .., v_t, -1, ..) is encoded as the integer
    sum_p (v_p + 1) (n + 1)^(D - 1 - p) (absent entries contribute 0), which
    is injective; lookups sort the codes once and binary-search them.
    """

    def __init__(self, n: int, D: int):
        self.n, self.D = n, D
        if (n + 1) ** D >= 2 ** 62:
            raise ValueError("variable-list codes would overflow int64")
        self.lists = monomials_sparse(n, D)
        self.weights = np.array([(n + 1) ** (D - 1 - q) for q in range(D)], dtype=np.int64)
        self.codes = self.encode(self.lists)
        self._sorter = np.argsort(self.codes, kind="stable")
        self._sorted = self.codes[self._sorter]

    def __len__(self) -> int:
        return self.lists.shape[0]

    def encode(self, lists: np.ndarray) -> np.ndarray:
        return (np.asarray(lists, dtype=np.int64) + 1) @ self.weights

    def lookup(self, lists: np.ndarray) -> np.ndarray:
        """Positions of padded ascending lists; -1 where absent."""
        codes = self.encode(lists)
        pos = np.clip(np.searchsorted(self._sorted, codes), 0, len(self._sorted) - 1)
        return np.where(self._sorted[pos] == codes, self._sorter[pos], -1)


def merge_lists(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Variable list of the product of two monomials given as padded lists
    (broadcasting over leading axes): the sorted union with multiplicity,
    padding moved to the end."""
    a, b = np.broadcast_arrays(np.asarray(a), np.asarray(b))
    both = np.concatenate([a, b], axis=-1)
    big = np.iinfo(np.int64).max
    both = np.sort(np.where(both < 0, big, both), axis=-1)
    return np.where(both == big, -1, both)


def pair_ranks_sparse(n: int, d: int, rows=None, basis=None, cidx=None) -> np.ndarray:
    """``pair_ranks`` through the sparse representation: entry (i, j) is the
    position of the merged list of basis monomials i and j among the
    degree-<=2d lists.  ``basis`` and ``cidx`` (from ``monomials_sparse`` and
    ``SparseIndex``) may be passed in when calling block by block."""
    basis = monomials_sparse(n, d) if basis is None else basis
    cidx = SparseIndex(n, 2 * d) if cidx is None else cidx
    bi = basis if rows is None else basis[np.asarray(rows)]
    out = cidx.lookup(merge_lists(bi[:, None, :], basis[None, :, :]))
    assert (out >= 0).all()
    return out


# ---------------------------------------------------------------------------
# Coefficients, loss and gradient (eq. nonconvex)
# ---------------------------------------------------------------------------

def coefficients(W: np.ndarray, n: int, d: int, pr=None) -> np.ndarray:
    """c = coeff(m_d^T W W^T m_d): FP64 Gram, summed over ordered pairs."""
    W = np.asarray(W, dtype=np.float64)
    if pr is None:
        pr = pair_ranks(n, d)
    G = W @ W.T
    return np.bincount(pr.ravel(), weights=G.ravel(), minlength=comb(n + 2 * d, 2 * d))


def coefficients_abs(W: np.ndarray, n: int, d: int, pr=None) -> np.ndarray:
    """coeff(|W| |W|^T): the per-coefficient scale used for error bounds."""
    return coefficients(np.abs(np.asarray(W, dtype=np.float64)), n, d, pr)


def residual(W, p, n, d, pr=None) -> np.ndarray:
    """r = c(W W^T) - p (the error vector of Section 3)."""
    return coefficients(W, n, d, pr) - np.asarray(p, dtype=np.float64)


def loss_grad(W, p, n, d, pr=None):
    """L = ||r||^2 and grad_W L = 4 R W with R_ij = r[rank(alpha_i+alpha_j)].

    Returns (L, g, r).
    """
    W = np.asarray(W, dtype=np.float64)
    if pr is None:
        pr = pair_ranks(n, d)
    r = residual(W, p, n, d, pr)
    L = float(r @ r)
    R = r[pr]
    g = 4.0 * (R @ W)
    return L, g, r


# ---------------------------------------------------------------------------
# Polynomials given as term lists; evaluation identities (eq. basicsos)
# ---------------------------------------------------------------------------

def poly_vector(terms, n: int, d: int) -> np.ndarray:
    """Coefficient vector (degree <= 2d order) of a list of (exponents, coef)."""
    cidx = MonomialIndex(n, 2 * d)
    p = np.zeros(len(cidx))
    for e, v in terms:
        k = int(cidx.lookup(np.array([e]))[0])
        if k < 0:
            raise ValueError(f"monomial {e} has degree above {2 * d}")
        p[k] += v
    return p


def evaluate_poly(c: np.ndarray, n: int, D: int, x: np.ndarray) -> float:
    """sum_beta c_beta x^beta over the degree-<=D list."""
    exps = monomials(n, D)
    return float(np.sum(c * np.prod(np.asarray(x, dtype=np.float64) ** exps, axis=1)))


def evaluate_sos(W: np.ndarray, n: int, d: int, x: np.ndarray) -> float:
    """||W^T m_d(x)||^2: the value of the sum of squares with factor W."""
    md = np.prod(np.asarray(x, dtype=np.float64) ** monomials(n, d), axis=1)
    q = np.asarray(W, dtype=np.float64).T @ md
    return float(q @ q)


# ---------------------------------------------------------------------------
# Adam (Section 3: "basic ADAM ... w/o any parameter optimization")
# ---------------------------------------------------------------------------

@dataclass
class AdamState:
    m: np.ndarray
    v: np.ndarray
    t: int = 0


def adam_step(W, g, st: AdamState, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One bias-corrected Adam update (Kingma and Ba 2015), FP64.

    m <- b1 m + (1-b1) g;  v <- b2 v + (1-b2) g^2;  t <- t+1;
    W <- W - lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps).
    """
    st.t += 1
    st.m = beta1 * st.m + (1.0 - beta1) * g
    st.v = beta2 * st.v + (1.0 - beta2) * g * g
    mhat = st.m / (1.0 - beta1 ** st.t)
    vhat = st.v / (1.0 - beta2 ** st.t)
    return W - lr * mhat / (np.sqrt(vhat) + eps)


@dataclass
class SolveResult:
    W: np.ndarray
    best_W: np.ndarray
    losses: list = field(default_factory=list)
    best_loss: float = float("inf")
    best_step: int = -1


def solve(p, n, d, W0, steps, lr, beta1=0.9, beta2=0.999, eps=1e-8, pr=None):
    """Adam on L(W) from W0 for a fixed number of steps (Section 3).

    losses[t] is L at the iterate before update t+1; the best (minimum) loss
    over all iterates and its W are kept, since the paper judges success by
    the minimal error over the iterations.
    """
    if pr is None:
        pr = pair_ranks(n, d)
    W = np.array(W0, dtype=np.float64)
    st = AdamState(np.zeros_like(W), np.zeros_like(W))
    res = SolveResult(W=W, best_W=W.copy())
    for t in range(steps):
        L, g, _ = loss_grad(W, p, n, d, pr)
        res.losses.append(L)
        if L < res.best_loss:
            res.best_loss, res.best_step, res.best_W = L, t, W.copy()
        W = adam_step(W, g, st, lr, beta1, beta2, eps)
    L, _, _ = loss_grad(W, p, n, d, pr)
    res.losses.append(L)
    if L < res.best_loss:
        res.best_loss, res.best_step, res.best_W = L, steps, W.copy()
    res.W = W
    return res


# ---------------------------------------------------------------------------
# One-by-one evaluation for bases too large for the full Gram matrix
# ---------------------------------------------------------------------------

def _pairs_of(beta: np.ndarray, basis: np.ndarray, bidx: MonomialIndex):
    """All ordered (i, j) with alpha_i + alpha_j = beta."""
    gam = beta[None, :] - basis
    j = bidx.lookup(gam)
    i = np.nonzero(j >= 0)[0]
    return i, j[i]


def sample_coefficients(W, n, d, beta_ranks, basis=None, bidx=None, cidx=None):
    """c_beta for selected coefficient positions, each summed pair by pair.

    c_beta = sum over ordered (i, j) with alpha_i + alpha_j = beta of
    <W_i, W_j> (eq. nonconvex), with the pair set found by testing every
    basis monomial alpha_i for beta - alpha_i in the basis.
    """
    W = np.asarray(W, dtype=np.float64)
    basis = monomials(n, d) if basis is None else basis
    bidx = MonomialIndex(n, d) if bidx is None else bidx
    cidx = MonomialIndex(n, 2 * d) if cidx is None else cidx
    out = np.empty(len(beta_ranks))
    for q, b in enumerate(beta_ranks):
        i, j = _pairs_of(cidx.exps[int(b)], basis, bidx)
        out[q] = float(np.einsum("ij,ij->", W[i], W[j]))
    return out


def sample_gradient_rows(W, p, n, d, rows):
    """Rows i of grad L = 4 R W, with every needed r entry computed one by one.

    Row i needs r at beta = alpha_i + alpha_j for all j; each such c_beta is
    summed pair by pair as in ``sample_coefficients``.
    """
    W = np.asarray(W, dtype=np.float64)
    basis = monomials(n, d)
    bidx = MonomialIndex(n, d)
    cidx = MonomialIndex(n, 2 * d)
    out = np.empty((len(rows), W.shape[1]))
    for q, i in enumerate(rows):
        betas = cidx.lookup(basis[int(i)][None, :] + basis)
        c = sample_coefficients(W, n, d, betas, basis, bidx, cidx)
        r = c - np.asarray(p, dtype=np.float64)[betas]
        out[q] = 4.0 * (r @ W)
    return out
