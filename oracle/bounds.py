"""Relative error bounds of the paper's algorithms -- TEST INFRASTRUCTURE ONLY.

Evaluated with mpmath at high precision, in multiples of the unit roundoff eps
(eps_D = 2^-53, eps_S = 2^-24, Sect. 1):

* ``ub_L(n)`` -- Theorem 1, Eq. (13): the single-accumulator fma sum of squares,
  1 + eta_i^+ = (1 + eta_{i-1}^+)(1 + eps) with eta_1 = 0 (the first square is taken
  as exact, which is what reproduces Table 3), and ub = sqrt(1 + eta_n^+)(1 + eps) - 1.
* ``ub_R(n, node)`` -- Theorem 3, Eq. (8) evaluated recursively over R's ceil split
  (Listing 1).  Reading of Eq. (8): 1 + eps_/ is the ratio of the smaller to the
  larger child factor, hence <= 1, so the square-root factor of the upper bound is at
  most 1 and the bound is 1 + eps_[n]^+ = max(1 + eps_[p]^+, 1 + eps_[q]^+)(1 + eps'^+).
  Taken literally (ratio of an upper to a lower bound) Eq. (8) gives about 4 at n = 4,
  while Table 3 prints 2.00000000000000011; the reading reproduces every printed digit.
* node factors 1 + eps'^+: cr_hypot: 1 + eps; v1_hypot (Listing 2): Eq. (reH),
  (1 + eps)^(5/2) sqrt(1 + eps(2 + eps)/2).
"""
from __future__ import annotations

import functools
import math

import mpmath

mpmath.mp.prec = 512

EPS = {"f64": mpmath.mpf(2) ** -53, "f32": mpmath.mpf(2) ** -24}


def node_factor(node: str, fmt: str = "f64"):
    e = EPS[fmt]
    if node == "cr":
        return 1 + e
    if node == "v1":
        return (1 + e) ** mpmath.mpf(2.5) * mpmath.sqrt(1 + e * (2 + e) / 2)
    raise ValueError(node)


def ub_L(n: int, fmt: str = "f64"):
    e = EPS[fmt]
    eta = mpmath.mpf(1)  # 1 + eta_1^+ = 1
    eta *= (1 + e) ** (n - 1)
    return (mpmath.sqrt(eta) * (1 + e) - 1) / e


def ub_R(n: int, node: str = "cr", fmt: str = "f64"):
    """Upper bound on relerr / eps of the recursion R with the given node."""
    f = node_factor(node, fmt)

    @functools.lru_cache(maxsize=None)
    def up(m):
        if m == 1:
            return mpmath.mpf(1)
        if m == 2:
            return f
        p = (m >> 1) + (m & 1)
        return max(up(p), up(m - p)) * f

    return (up(n) - 1) / EPS[fmt]


def ub_R_literal(n: int, node: str = "cr", fmt: str = "f64"):
    """Eq. (8) taken literally (ratio of the larger upper to the smaller lower bound)."""
    e = EPS[fmt]
    f = node_factor(node, fmt)
    fm = 2 - f  # lower node factor 1 - eps'

    @functools.lru_cache(maxsize=None)
    def bnd(m):
        if m == 1:
            return mpmath.mpf(1), mpmath.mpf(1)
        if m == 2:
            return fm, f
        p = (m >> 1) + (m & 1)
        (lp, hp), (lq, hq) = bnd(p), bnd(m - p)
        k_hi = max(hp, hq)
        k_lo = min(lp, lq)
        ratio_hi = max(hp, hq) / min(lp, lq)
        up = mpmath.sqrt(1 + (ratio_hi - 1) * (1 + ratio_hi)) * k_hi * f
        return k_lo * fm, up

    return (bnd(n)[1] - 1) / e


def tol_parity(n: int, fmt: str = "f64") -> float:
    """GPU-versus-oracle tolerance |G - O| / O <= 2 (ceil(log2 n) + 1) eps."""
    k = 0 if n <= 1 else math.ceil(math.log2(n))
    return 2.0 * (k + 1) * float(EPS[fmt])


def depth_R(n: int) -> int:
    """Depth (number of nodes on the longest root-leaf path) of R's tree."""
    if n <= 1:
        return 0
    if n == 2:
        return 1
    p = (n >> 1) + (n & 1)
    return 1 + depth_R(p)
