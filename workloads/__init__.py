"""Seeded synthetic inputs shared by the FP64 oracle and the GPU path.

This module holds no arithmetic of the SOS method itself: no monomial
ordering, no ranking, no coefficient extraction.  It only draws random
numbers and describes polynomials as lists of (exponent tuple, coefficient)
terms; each consumer maps those onto its own coefficient vector.

The paper builds its test polynomials from a random PSD Gram matrix B B^T
with B uniform in [-1, 1] (Section 3.1).  The workloads below keep that idea
(p is the coefficient vector of W0 W0^T for a random factor W0) with a
Gaussian W0, at the sizes listed in ``CONFIGS``.
"""
from __future__ import annotations

from dataclasses import dataclass
from math import comb

import numpy as np

__all__ = [
    "Workload",
    "CONFIGS",
    "gaussian",
    "uniform",
    "motzkin_terms",
    "basis_size",
    "coeff_size",
    "serving_stream",
]


def basis_size(n: int, d: int) -> int:
    """Number of monomials of degree <= d in n variables."""
    return comb(n + d, d)


def coeff_size(n: int, d: int) -> int:
    """Number of monomials of degree <= 2d in n variables."""
    return comb(n + 2 * d, 2 * d)


def gaussian(shape, seed: int, std: float = 1.0) -> np.ndarray:
    """i.i.d. N(0, std^2) in FP64 from numpy's PCG64 stream ``seed``."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) * std


def uniform(shape, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """i.i.d. U[lo, hi) in FP64 from numpy's PCG64 stream ``seed``."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=shape)


def motzkin_terms(n: int):
    """Motzkin form x^4 y^2 + x^2 y^4 - 3 x^2 y^2 z^2 + z^6 on x1, x2, x3.

    Returned as (exponent tuple of length n, coefficient) terms; variables
    x4..xn do not occur.  The form is non-negative but not a sum of squares,
    which makes it the standard negative control for an SOS test.
    """
    if n < 3:
        raise ValueError("Motzkin form needs n >= 3")

    def e(a, b, c):
        return (a, b, c) + (0,) * (n - 3)

    return [(e(4, 2, 0), 1.0), (e(2, 4, 0), 1.0), (e(2, 2, 2), -3.0), (e(0, 0, 6), 1.0)]


@dataclass(frozen=True)
class Workload:
    """One synthetic problem: sizes, seeds and scales (no arithmetic)."""

    name: str
    n: int
    d: int
    rank: int            # k: columns of the trained factor W
    w0_rank: int         # columns of the generating factor W0 (0: p is not generated from W0)
    w0_std: float        # standard deviation of W0's entries
    w_std: float         # standard deviation of W's initial entries
    w0_seed: int = 0
    w_seed: int = 1
    w0_uniform: bool = False   # W0 entries uniform in [-w0_std, w0_std] instead of normal

    @property
    def N(self) -> int:
        return basis_size(self.n, self.d)

    @property
    def M(self) -> int:
        return coeff_size(self.n, self.d)

    def W0(self) -> np.ndarray:
        if self.w0_uniform:
            return uniform((self.N, self.w0_rank), self.w0_seed, -self.w0_std, self.w0_std)
        return gaussian((self.N, self.w0_rank), self.w0_seed, self.w0_std)

    def W_init(self) -> np.ndarray:
        return gaussian((self.N, self.rank), self.w_seed, self.w_std)


# Sizes of the five workloads: (n, d) pairs, W0 shape and scale, W shape and scale.
CONFIGS = {
    # n=3, d=2: N=10, M=35.  W0 10x3 N(0,1); W 10x20 N(0, 0.1^2).
    "n3d2": Workload("n3d2", 3, 2, rank=20, w0_rank=3, w0_std=1.0, w_std=0.1),
    # n=6, d=4: N=210, M=3003.  W0 210x50 N(0,1); W 210x420 N(0, 0.05^2).
    "n6d4": Workload("n6d4", 6, 4, rank=420, w0_rank=50, w0_std=1.0, w_std=0.05),
    # Motzkin control padded into n=6, d=3: N=84, M=924; W 84x168.
    "motzkin_n6d3": Workload("motzkin_n6d3", 6, 3, rank=168, w0_rank=0, w0_std=0.0, w_std=0.05),
    # n=10, d=5: N=3003, M=184,756.  W0 3003x300 N(0,1)/sqrt(300); W 3003x3003 N(0, 1/k).
    "n10d5": Workload("n10d5", 10, 5, rank=3003, w0_rank=300, w0_std=300 ** -0.5,
                      w_std=3003 ** -0.5),
    # n=12, d=6: N=18,564, M=2,704,156.  W0 18564x2000 N(0,1)/sqrt(2000); W 18564^2 N(0, 1/k).
    "n12d6": Workload("n12d6", 12, 6, rank=18564, w0_rank=2000, w0_std=2000 ** -0.5,
                      w_std=18564 ** -0.5),
    # The paper's largest problem (Sections 1.2 and 3.1): quartic forms in 100
    # variables = degree <= 2 in n=99: N=5,050, M=4,421,275, full rank k = N.
    # p = m^T B B^T m with B uniform as in Section 3.1, here N x N and scaled
    # by 1/sqrt(N) (p scaled by 1/N: the relative residual is unchanged);
    # W 5050^2 N(0, 1/k).
    "q100": Workload("q100", 99, 2, rank=5050, w0_rank=5050, w0_std=5050 ** -0.5,
                     w_std=5050 ** -0.5, w0_uniform=True),
}


def serving_stream(count: int, seed: int = 12345, rate: float = 1.0):
    """Request stream for the serving workload.

    Each request draws n uniform in {3..8} and d uniform in {2,3,4}; half are
    SOS by construction (W0 of rank ceil(N/4), N(0,1) entries) and half are the
    Motzkin form plus 1e-3 times a unit-norm random SOS (those draw d in {3,4},
    since the degree-6 Motzkin form needs 2d >= 6).  Arrival times follow a
    Poisson process of the given rate.  Returns a list of dicts holding sizes,
    seeds and arrival times only; each consumer builds its coefficient vectors.
    """
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    arrivals = np.cumsum(gaps) - gaps[0]
    out = []
    for i in range(count):
        sos = bool(rng.integers(0, 2) == 0)
        n = int(rng.integers(3, 9))
        d = int(rng.integers(2, 5)) if sos else int(rng.integers(3, 5))
        N = basis_size(n, d)
        out.append(dict(
            id=i, n=n, d=d, sos=sos, N=N, M=coeff_size(n, d), rank=2 * N,
            w0_rank=-(-N // 4), w0_seed=2 * i, w_seed=2 * i + 1,
            arrival=float(arrivals[i]),
        ))
    return out
