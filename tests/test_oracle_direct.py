"""Pins of the oracle's Eq. D1/D2 direct couplings (no GPU).

The angular algebra of Eq. D1 is pinned against a brute-force angular
quadrature of Y*_{l'm'} P_lambda(r^.R^) Y_{lm} with scipy's spherical
harmonics (the multipole expansion of 1/|r-R|), which is independent of the
Clebsch-Gordan / associated-Legendre route the oracle takes.
"""
import math

import numpy as np
import pytest
from scipy.special import sph_harm_y

from oracle.direct import (direct_matrix, direct_spatial, multipole_kernel,
                           radial_integrals)
from oracle.radial import BasisSpec, build_basis


@pytest.fixture(scope="module")
def bound_raw():
    """Bound-only hydrogen basis n <= 3 without Gram-Schmidt (closed-form functions)."""
    return build_basis(BasisSpec(n_max=3, l_max=2, n_bins=0, k_max=1.0, n_r=1500),
                       orthonormalise=False)


def _legendre(lam, x):
    from numpy.polynomial import legendre
    c = np.zeros(lam + 1)
    c[lam] = 1.0
    return legendre.legval(x, c)


def _angular_bruteforce(lp, mp, l, m, lam, theta_R):
    """int Y*_{l'm'} P_lam(r^ . R^) Y_lm dOmega, R^ = (sin T, 0, cos T), by a
    Gauss-Legendre x uniform-phi product rule exact for these polynomials."""
    x, wx = np.polynomial.legendre.leggauss(24)
    nphi = 32
    phi = np.arange(nphi) * (2 * np.pi / nphi)
    th = np.arccos(x)
    TH, PH = np.meshgrid(th, phi, indexing="ij")
    W = np.outer(wx, np.full(nphi, 2 * np.pi / nphi))
    cosg = np.sin(TH) * np.cos(PH) * math.sin(theta_R) + np.cos(TH) * math.cos(theta_R)
    f = np.conj(sph_harm_y(lp, mp, TH, PH)) * _legendre(lam, cosg) * sph_harm_y(l, m, TH, PH)
    return (W * f).sum()


@pytest.mark.parametrize("R,theta", [(0.7, 0.4), (3.0, 2.2), (15.0, 1.1), (140.0, 0.05)])
def test_d1_against_multipole_bruteforce(basis_small, R, theta):
    b = basis_small
    D = direct_spatial(b, R, math.cos(theta))
    F = [radial_integrals(b, R, lam) for lam in range(5)]
    ref = np.zeros_like(D)
    N = b.n_states
    cache = {}
    for i in range(N):
        for j in range(N):
            lp, mp, l, m = b.st_l[i], b.st_m[i], b.st_l[j], b.st_m[j]
            tot = 0.0
            for lam in range(abs(l - lp), l + lp + 1):
                key = (lp, mp, l, m, lam)
                if key not in cache:
                    cache[key] = _angular_bruteforce(lp, mp, l, m, lam, theta)
                a = cache[key]
                assert abs(a.imag) < 1e-13
                tot += -F[lam][b.st_a[i], b.st_a[j]] * a.real
            ref[i, j] = tot
    scale = np.abs(ref).max()
    assert np.abs(D - ref).max() <= 1e-12 * scale


def test_d1_real_symmetric_and_hermitian(basis_c1):
    b = basis_c1
    Dsp = direct_spatial(b, 2.3, 0.6)
    assert np.abs(Dsp - Dsp.T).max() <= 1e-14 * np.abs(Dsp).max()
    D = direct_matrix(b, 1.0, 1.7, 1.0)
    assert np.abs(D - D.conj().T).max() <= 1e-14 * np.abs(D).max()


def test_d1_axial_field_conserves_m(basis_small):
    # R along z (Theta = 0): only mu = 0 survives, so m' = m
    b = basis_small
    D = direct_spatial(b, 2.0, 1.0)
    mm = np.subtract.outer(b.st_m, b.st_m)
    assert np.abs(D[mm != 0]).max() < 1e-15


def test_dp_is_parity_transform(basis_small):
    b = basis_small
    DT = direct_spatial(b, 1.4, -0.35)
    DP = direct_spatial(b, 1.4, -0.35, parity=-1)
    s = (-1.0) ** b.st_l
    assert np.abs(DP - s[:, None] * DT * s[None, :]).max() < 1e-14 * np.abs(DT).max()


def test_f0_1s_closed_form(bound_raw):
    # potential of the 1s cloud: F_0^{1s1s}(R) = 1/R - (1 + 1/R) exp(-2R)
    for R in (0.5, 2.0, 7.0):
        F0 = radial_integrals(bound_raw, R, 0)[0, 0]
        ref = 1 / R - (1 + 1 / R) * math.exp(-2 * R)
        assert abs(F0 - ref) < 1e-5


def test_multipole_outside_grid(bound_raw):
    # R >= r_max: F_lambda(R) R^(lambda+1) is the multipole moment, e.g. the dipole
    b = bound_raw
    i1s, i2p = 0, b.rad_off[1]
    for R in (100.0, 173.0, 1e4):
        F1 = radial_integrals(b, R, 1)[i1s, i2p]
        assert abs(F1 * R * R - 128 * math.sqrt(6) / 243) < 1e-12


def test_d_asymptotics(basis_c1):
    # monopole: D -> -I/R (orthonormal basis); remainder falls like R^-2 (dipole)
    b = basis_c1
    th = 0.8
    rem = []
    for R in (200.0, 400.0):
        D = direct_spatial(b, R, math.cos(th))
        assert np.abs(np.diag(D) + 1 / R).max() < 5e-3 / R
        rem.append(np.abs(D + np.eye(b.n_states) / R).max())
    assert 3.6 < rem[0] / rem[1] < 4.4


def test_kernel_continuous_at_R():
    r = np.array([1.999999, 2.0, 2.000001])
    g = multipole_kernel(3, r, 2.0)
    assert abs(g[0] - g[1]) < 1e-5 and abs(g[2] - g[1]) < 1e-5
