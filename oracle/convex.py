"""Distance from p to the cone of SOS polynomials, by a convex method.

TEST INFRASTRUCTURE ONLY.  Solves  min_{G PSD} ||coeff(G) - p||^2  (the
convex problem behind eq. basicsos) with FISTA: a gradient step on the
squared coefficient error followed by projection onto the PSD cone
(eigen-decomposition, negative eigenvalues clipped).  This is independent of
the factored, non-convex objective of eq. nonconvex, so the two can check
each other: for full-rank factors the factored minimum equals this one, and
no factor can do better.

Optimality check (KKT for a convex cone program): at the minimiser G*, with
r* = coeff(G*) - p and R*_ij = r*[rank(alpha_i+alpha_j)], R* is PSD and
<R*, G*> = 0.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .sos import pair_ranks


@dataclass
class PsdDistance:
    dist2: float          # min ||coeff(G) - p||^2 over PSD G
    G: np.ndarray
    r: np.ndarray
    kkt_min_eig: float    # smallest eigenvalue of R* (>= -tol at optimum)
    kkt_gap: float        # <R*, G*> (0 at optimum)
    iters: int


def _project_psd(S: np.ndarray) -> np.ndarray:
    S = 0.5 * (S + S.T)
    w, V = np.linalg.eigh(S)
    w = np.maximum(w, 0.0)
    return (V * w) @ V.T


def psd_distance(p, n, d, iters=20000, tol=1e-13) -> PsdDistance:
    pr = pair_ranks(n, d)
    p = np.asarray(p, dtype=np.float64)
    M = p.shape[0]
    mult = np.bincount(pr.ravel(), minlength=M)
    lip = 2.0 * mult.max()          # ||coeff||^2 = max number of ordered pairs per monomial
    N = pr.shape[0]
    G = np.zeros((N, N))
    Y = G.copy()
    tk = 1.0
    fprev = np.inf
    it = 0
    for it in range(1, iters + 1):
        r = np.bincount(pr.ravel(), weights=Y.ravel(), minlength=M) - p
        Gn = _project_psd(Y - (2.0 * r[pr]) / lip)
        tn = 0.5 * (1.0 + np.sqrt(1.0 + 4.0 * tk * tk))
        Y = Gn + ((tk - 1.0) / tn) * (Gn - G)
        G, tk = Gn, tn
        if it % 200 == 0:
            rg = np.bincount(pr.ravel(), weights=G.ravel(), minlength=M) - p
            f = float(rg @ rg)
            if abs(fprev - f) <= tol * max(f, 1e-300):
                break
            fprev = f
    r = np.bincount(pr.ravel(), weights=G.ravel(), minlength=M) - p
    R = r[pr]
    return PsdDistance(
        dist2=float(r @ r), G=G, r=r,
        kkt_min_eig=float(np.linalg.eigvalsh(0.5 * (R + R.T)).min()),
        kkt_gap=float(np.sum(R * G)), iters=it,
    )
