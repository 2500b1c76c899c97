"""Quartic forms from the paper's two-layer network ||B Z A x||^2 (Section 2).

TEST INFRASTRUCTURE ONLY.  Two independent routes to the coefficients of the
same quartic form, used to pin the oracle's coefficient extraction for d=2:

* ``network_quartic_coefficients``: the paper's derivative route.  With
  f = B Z A x (a vector of quadratic forms), the second derivative is the
  constant vector f_ij = B Z_i A e_j + B Z_j A e_i, where B Z_i A e_j is the
  i-th column block of B times column j of A (Section 2, eq. NN and the
  augmentation Z).  A coefficient of ||f||^2 is the sum, over the ways to
  split the monomial's four variables into two pairs, of the inner products
  of the matching second derivatives, times 2 and divided by the product of
  the factorials of the exponents (Section 2, the pairing identities for
  x_i^4, x_i^3 x_j, x_i^2 x_j^2, x_i^2 x_j x_k and x_i x_j x_k x_l).
* ``network_factor``: the factor W whose columns hold each f_k's coefficients
  over the degree-<=2 basis, so that ||f||^2 = m_2^T W W^T m_2 and the
  oracle's ``coefficients(W)`` applies.
"""
from __future__ import annotations

from itertools import combinations_with_replacement
from math import factorial

import numpy as np

from .sos import MonomialIndex


def _second_derivatives(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """F[i, j] = f_{x_i x_j} = B Z_i A e_j + B Z_j A e_i (length-k vectors)."""
    m, n = A.shape
    k = B.shape[0]
    assert B.shape[1] == n * m
    BZA = np.empty((n, n, k))          # BZA[i, j] = B[:, i-th block] @ A[:, j]
    for i in range(n):
        blk = B[:, i * m:(i + 1) * m]
        for j in range(n):
            BZA[i, j] = blk @ A[:, j]
    return BZA + BZA.transpose(1, 0, 2)


def network_quartic_coefficients(A: np.ndarray, B: np.ndarray) -> dict:
    """{exponent tuple: coefficient} of ||B Z A x||^2 via the pairing identities."""
    n = A.shape[1]
    F = _second_derivatives(np.asarray(A, float), np.asarray(B, float))
    out = {}
    for vars4 in combinations_with_replacement(range(n), 4):
        a, b, c, e = vars4
        # the three ways to split four (possibly repeated) variables into two pairs
        s = (F[a, b] @ F[c, e]) + (F[a, c] @ F[b, e]) + (F[a, e] @ F[b, c])
        expo = [0] * n
        for v in vars4:
            expo[v] += 1
        denom = 1
        for x in expo:
            denom *= factorial(x)
        out[tuple(expo)] = 2.0 * s / denom
    return out


def network_factor(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """W (C(n+2,2) x k) with column l = coefficients of f_l on the degree-<=2 basis."""
    A = np.asarray(A, float)
    B = np.asarray(B, float)
    m, n = A.shape
    k = B.shape[0]
    idx = MonomialIndex(n, 2)
    W = np.zeros((len(idx), k))
    for a in range(n):
        blk = B[:, a * m:(a + 1) * m]
        for c in range(n):
            # f_l contains sum_b B[l, a m + b] A[b, c] x_a x_c
            e = [0] * n
            e[a] += 1
            e[c] += 1
            row = int(idx.lookup(np.array([e]))[0])
            W[row] += blk @ A[:, c]
    return W


def network_loss_grad(A: np.ndarray, B: np.ndarray, p: np.ndarray):
    """L(A, B) = ||coeff(W W^T) - p||^2 for W = network_factor(A, B), and its
    gradient with respect to A and B (Section 2's network trained as in
    Section 3).  p is indexed like MonomialIndex(n, 4) (all monomials of
    degree <= 4 in the n variables; a quartic form has zeros below degree 4).

    Chain rule: column l of W holds f_l = sum_{a,c} P[l,a,c] x_a x_c with
    P[l,a,c] = sum_b B[l, a m + b] A[b, c]; the row of x_a x_c receives
    P[l,a,c] + P[l,c,a] (a != c) or P[l,a,a], so dL/dP[l,a,c] is the
    gradient dL/dW = 4 R W at that row, for both orders of (a, c).
    """
    from .sos import loss_grad, pair_ranks
    W = network_factor(A, B)
    n = np.asarray(A).shape[1]
    L, gW, _ = loss_grad(W, p, n, 2, pair_ranks(n, 2))
    dA, dB = network_chain(A, B, gW)
    return L, dA, dB


def network_chain(A: np.ndarray, B: np.ndarray, gW: np.ndarray):
    """dL/dA and dL/dB from dL/dW (rows of the degree-<=2 basis in n
    variables) by the chain rule through W = network_factor(A, B): the row of
    x_a x_c holds P[l,a,c] + P[l,c,a] (a != c) or P[l,a,a], so
    dL/dP[l,a,c] = gW[row of x_a x_c, l] for both orders of (a, c), and
    P[l,a,c] = sum_b B[l, a m + b] A[b, c]."""
    A = np.asarray(A, float)
    B = np.asarray(B, float)
    gW = np.asarray(gW, float)
    m, n = A.shape
    k = B.shape[0]
    idx = MonomialIndex(n, 2)
    dP = np.zeros((k, n, n))
    for a in range(n):
        for c in range(n):
            e = [0] * n
            e[a] += 1
            e[c] += 1
            dP[:, a, c] = gW[int(idx.lookup(np.array([e]))[0])]
    dB = np.zeros_like(B)
    dA = np.zeros_like(A)
    for a in range(n):
        blk = B[:, a * m:(a + 1) * m]            # k x m
        dB[:, a * m:(a + 1) * m] = dP[:, a, :] @ A.T
        dA += blk.T @ dP[:, a, :]
    return dA, dB
