"""Pins of the oracle's angular algebra against sympy (exact), scipy and closed forms."""
import math

import numpy as np
import pytest
from scipy.special import jv, lpmv
from sympy import S
from sympy.physics.quantum.cg import CG

from oracle.angular import assoc_legendre, bessel_j, clebsch_gordan, wigner_small_d


def test_clebsch_gordan_against_sympy():
    for j1 in range(0, 4):
        for j2 in range(0, 4):
            for J in range(abs(j1 - j2), j1 + j2 + 1):
                for m1 in range(-j1, j1 + 1):
                    for m2 in range(-j2, j2 + 1):
                        M = m1 + m2
                        if abs(M) > J:
                            continue
                        ref = float(CG(S(j1), S(m1), S(j2), S(m2), S(J), S(M)).doit())
                        assert abs(clebsch_gordan(j1, m1, j2, m2, J, M) - ref) < 1e-14


def test_clebsch_gordan_selection():
    assert clebsch_gordan(1, 0, 1, 0, 1, 0) == 0.0      # parity-odd
    assert clebsch_gordan(1, 1, 1, 0, 1, 0) == 0.0      # M mismatch
    assert clebsch_gordan(2, 0, 1, 0, 4, 0) == 0.0      # triangle


@pytest.mark.parametrize("l", range(0, 9))
def test_assoc_legendre_against_scipy(l):
    x = np.linspace(-0.999, 0.999, 37)
    for m in range(0, l + 1):
        assert np.allclose(assoc_legendre(l, m, x), lpmv(m, l, x), rtol=1e-12, atol=1e-12)
    for m in range(1, l + 1):
        ref = (-1) ** m * math.factorial(l - m) / math.factorial(l + m) * lpmv(m, l, x)
        assert np.allclose(assoc_legendre(l, -m, x), ref, rtol=1e-12, atol=1e-14)


def test_condon_shortley_phase():
    x = 0.3
    assert abs(assoc_legendre(1, 1, x) + math.sqrt(1 - x * x)) < 1e-15


def test_wigner_d_closed_forms():
    for th in (0.0, 0.4, 1.3, 2.9):
        c, s = math.cos(th), math.sin(th)
        assert abs(wigner_small_d(1, 1, 1, th) - (1 + c) / 2) < 1e-15
        assert abs(wigner_small_d(1, 1, 0, th) + s / math.sqrt(2)) < 1e-15
        assert abs(wigner_small_d(1, 0, 1, th) - s / math.sqrt(2)) < 1e-15
        assert abs(wigner_small_d(1, 1, -1, th) - (1 - c) / 2) < 1e-15
        assert abs(wigner_small_d(1, 0, 0, th) - c) < 1e-15


@pytest.mark.parametrize("l", range(0, 6))
def test_wigner_d_orthogonal_and_m0_column(l):
    th = 0.77
    d = np.array([[wigner_small_d(l, m, q, th) for q in range(-l, l + 1)]
                  for m in range(-l, l + 1)])
    assert np.abs(d @ d.T - np.eye(2 * l + 1)).max() < 1e-13
    # d^l_{m0}(theta) = sqrt((l-m)!/(l+m)!) P_l^m(cos theta)
    for m in range(-l, l + 1):
        ref = math.sqrt(math.factorial(l - m) / math.factorial(l + m)) * assoc_legendre(l, m, math.cos(th))
        assert abs(d[m + l, l] - ref) < 1e-13
    # composition d(a) d(b) = d(a + b)
    da = np.array([[wigner_small_d(l, m, q, 0.3) for q in range(-l, l + 1)] for m in range(-l, l + 1)])
    db = np.array([[wigner_small_d(l, m, q, 0.47) for q in range(-l, l + 1)] for m in range(-l, l + 1)])
    assert np.abs(da @ db - d).max() < 1e-13


def test_bessel_jacobi_anger():
    # (1/2pi) int exp(i n phi) exp(i x cos phi) dphi = i^n J_n(x)
    phi = np.linspace(0, 2 * np.pi, 4096, endpoint=False)
    for n in range(-4, 5):
        for x in (0.3, 2.5, 9.0):
            val = np.mean(np.exp(1j * n * phi) * np.exp(1j * x * np.cos(phi)))
            assert abs(val - (1j) ** n * bessel_j(n, x)) < 1e-13
    assert abs(bessel_j(-3, 1.7) + jv(3, 1.7)) < 1e-15
