"""Angular-momentum algebra for the oracle.

Test infrastructure only (see ``oracle/__init__.py``).

Paper anchors: Eq. D1 (Clebsch-Gordan coefficients, associated Legendre
functions P_lambda^mu of the collision angle), Eq. K1 (Wigner rotation
d^l_{m q}(theta)), Eq. K2 (associated Legendre functions at the spheroidal
arguments, Bessel J_{q-q'}).  The paper calls P_lambda^mu "Legendre
polynomials"; they are the associated Legendre functions with the
Condon-Shortley phase (P_1^1(x) = -sqrt(1-x^2)).
"""
from __future__ import annotations

import math
from fractions import Fraction
from functools import lru_cache

import numpy as np
from scipy.special import jv


def _f(n: int) -> int:
    return math.factorial(n)


@lru_cache(maxsize=None)
def clebsch_gordan(j1: int, m1: int, j2: int, m2: int, J: int, M: int) -> float:
    """C^{J M}_{j1 m1 j2 m2} = <j1 m1 j2 m2 | J M> by Racah's formula (exact rationals)."""
    if m1 + m2 != M or abs(m1) > j1 or abs(m2) > j2 or abs(M) > J:
        return 0.0
    if J < abs(j1 - j2) or J > j1 + j2:
        return 0.0
    pre = Fraction((2 * J + 1) * _f(J + j1 - j2) * _f(J - j1 + j2) * _f(j1 + j2 - J),
                   _f(j1 + j2 + J + 1))
    pre *= (_f(J + M) * _f(J - M) * _f(j1 - m1) * _f(j1 + m1) * _f(j2 - m2) * _f(j2 + m2))
    s = Fraction(0)
    for k in range(0, j1 + j2 - J + 1):
        a = (k, j1 + j2 - J - k, j1 - m1 - k, j2 + m2 - k, J - j2 + m1 + k, J - j1 - m2 + k)
        if min(a) < 0:
            continue
        den = 1
        for x in a:
            den *= _f(x)
        s += Fraction((-1) ** k, den)
    if s == 0:
        return 0.0
    sign = 1.0 if s > 0 else -1.0
    return sign * math.sqrt(float(pre * s * s))


def assoc_legendre(l: int, m: int, x):
    """P_l^m(x) with the Condon-Shortley phase; negative m through
    P_l^{-m} = (-1)^m (l-m)!/(l+m)! P_l^m."""
    x = np.asarray(x, dtype=np.float64)
    if abs(m) > l:
        return np.zeros_like(x)
    if m < 0:
        mm = -m
        return (-1) ** mm * _f(l - mm) / _f(l + mm) * assoc_legendre(l, mm, x)
    s = np.sqrt(np.maximum(0.0, 1.0 - x * x))
    pmm = np.ones_like(x)
    for i in range(1, m + 1):
        pmm = -pmm * (2 * i - 1) * s
    if l == m:
        return pmm
    pm1 = x * (2 * m + 1) * pmm
    if l == m + 1:
        return pm1
    p0, p1 = pmm, pm1
    for ll in range(m + 1, l):
        p2 = ((2 * ll + 1) * x * p1 - (ll + m) * p0) / (ll - m + 1)
        p0, p1 = p1, p2
    return p1


def wigner_small_d(l: int, m: int, q: int, theta: float) -> float:
    """Wigner's d^l_{m q}(theta) by his explicit sum (convention: d^1_{10} = -sin(theta)/sqrt(2))."""
    if abs(m) > l or abs(q) > l:
        return 0.0
    c = math.cos(theta / 2.0)
    s = math.sin(theta / 2.0)
    pre = math.sqrt(_f(l + m) * _f(l - m) * _f(l + q) * _f(l - q))
    tot = 0.0
    for k in range(max(0, q - m), min(l + q, l - m) + 1):
        den = _f(l + q - k) * _f(k) * _f(m - q + k) * _f(l - m - k)
        tot += (-1) ** (m - q + k) * c ** (2 * l + q - m - 2 * k) * s ** (m - q + 2 * k) / den
    return pre * tot


def bessel_j(n: int, x):
    """Bessel function of the first kind J_n(x) (library routine; J_{-n} = (-1)^n J_n)."""
    return jv(n, np.asarray(x, dtype=np.float64))
