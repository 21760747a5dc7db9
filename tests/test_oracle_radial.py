"""Pins of the oracle's radial part against closed forms and mpmath (no GPU)."""
import math

import mpmath
import numpy as np
import pytest

from oracle.radial import (BasisSpec, build_basis, coulomb_norm, coulomb_psi,
                           coulomb_u, gram_schmidt, hydrogen_radial, radial_grid,
                           wave_packets)


def test_grid_simpson_exact_for_low_degree():
    # In x the integrands of int dr and int r dr are x and x^3: Simpson is exact.
    r, w = radial_grid(1500, 100.0)
    assert r[0] == 0.0 and r[-1] == 100.0
    assert w[0] == 0.0
    assert abs(w.sum() - 100.0) < 1e-12
    assert abs((w * r).sum() - 100.0 ** 2 / 2) < 1e-9


def test_grid_rejects_odd():
    with pytest.raises(ValueError):
        radial_grid(1501, 100.0)


def test_hydrogen_closed_forms():
    r = np.linspace(0.0, 30.0, 301)
    Z = 1.0
    assert np.allclose(hydrogen_radial(1, 0, Z, r), 2.0 * np.exp(-r), rtol=0, atol=1e-15)
    assert np.allclose(hydrogen_radial(2, 0, Z, r),
                       (1 / math.sqrt(2)) * (1 - r / 2) * np.exp(-r / 2), rtol=0, atol=1e-15)
    assert np.allclose(hydrogen_radial(2, 1, Z, r),
                       r * np.exp(-r / 2) / (2 * math.sqrt(6)), rtol=0, atol=1e-15)
    # Z scaling: R_nl(Z; r) = Z^(3/2) R_nl(1; Z r)
    assert np.allclose(hydrogen_radial(3, 1, 2.0, r),
                       2.0 ** 1.5 * hydrogen_radial(3, 1, 1.0, 2.0 * r), rtol=1e-13, atol=1e-15)


def test_hydrogen_orthonormal_on_grid():
    r, w = radial_grid(1500, 100.0)
    m = w * r * r
    s1 = hydrogen_radial(1, 0, 1.0, r)
    s2 = hydrogen_radial(2, 0, 1.0, r)
    p2 = hydrogen_radial(2, 1, 1.0, r)
    assert abs((m * s1 * s1).sum() - 1.0) < 1e-13
    assert abs((m * s1 * s2).sum()) < 1e-13
    assert abs((m * p2 * p2).sum() - 1.0) < 1e-13


def test_dipole_closed_form():
    # int r^3 R_10 R_21 dr = 128 sqrt(6) / 243 (the radial part of <1s|r|2p>)
    r, w = radial_grid(1500, 100.0)
    val = (w * r ** 3 * hydrogen_radial(1, 0, 1.0, r) * hydrogen_radial(2, 1, 1.0, r)).sum()
    assert abs(val - 128 * math.sqrt(6) / 243) < 1e-12


@pytest.mark.parametrize("l", [0, 1, 2, 4])
@pytest.mark.parametrize("k", [0.0008, 0.05, 0.7, 2.9])
def test_coulomb_regular_against_mpmath(l, k):
    r, _ = radial_grid(1500, 100.0)
    u = coulomb_u(l, np.array([k]), 1.0, r)[0]
    eta = -1.0 / k
    C = coulomb_norm(l, np.array([eta]))[0]
    mine = C * k ** (l + 1) * u
    scale = np.abs(mine).max()
    for i in (1, 7, 150, 600, 1100, 1500):
        ref = float(mpmath.coulombf(l, eta, k * r[i]))
        assert abs(mine[i] - ref) <= 1e-12 * max(abs(ref), scale), (i, mine[i], ref)


def test_coulomb_norm_limits():
    # eta -> 0: C_0 -> 1; C_1(0) = 1/3.
    assert abs(coulomb_norm(0, np.array([1e-12]))[0] - 1.0) < 1e-10
    assert abs(coulomb_norm(1, np.array([1e-12]))[0] - 1.0 / 3.0) < 1e-10


def test_coulomb_psi_origin_limit():
    r, _ = radial_grid(600, 100.0)
    psi0 = coulomb_psi(0, np.array([0.5]), 1.0, r)[0]
    # l = 0: psi(0) equals the limit of psi at the first grid points
    assert abs(psi0[0] - psi0[1]) < 1e-3 * abs(psi0[0])
    psi1 = coulomb_psi(1, np.array([0.5]), 1.0, r)[0]
    assert psi1[0] == 0.0


def test_wave_packet_energies_and_near_orthogonality():
    r, w = radial_grid(1500, 100.0)
    m = w * r * r
    f, eps = wave_packets(0, 8, 3.0, 1.0, r)
    dk = 3.0 / 8
    for i in range(8):
        lo, hi = i * dk, (i + 1) * dk
        assert abs(eps[i] - (lo * lo + lo * hi + hi * hi) / 6) < 1e-15
    # continuum packets are orthogonal to the bound states up to grid truncation
    s1 = hydrogen_radial(1, 0, 1.0, r)
    ov = np.abs(f @ (m * s1))
    assert ov.max() < 2e-3
    # higher bins are well contained in 100 a.u.: norm close to 1
    nrm = (f * f * m).sum(axis=1)
    assert np.all(np.abs(nrm[2:] - 1.0) < 2e-2)


def test_gram_schmidt_orthonormal():
    r, w = radial_grid(600, 50.0)
    m = w * r * r
    rng = np.random.default_rng(0)
    f = rng.standard_normal((5, r.size))
    q = gram_schmidt(f, m)
    G = (q * m) @ q.T
    assert np.abs(G - np.eye(5)).max() < 1e-13


def test_basis_shapes_and_order(basis_c1):
    b = basis_c1
    assert b.n_per_l == [11, 10, 9]
    assert b.n_radial == 30 and b.n_states == 86
    assert b.st_l[0] == 0 and b.st_m[0] == 0 and b.eps[0] == -0.5
    m = b.w * b.r * b.r
    for l in range(3):
        o, n = b.rad_off[l], b.n_per_l[l]
        G = (b.phi[o:o + n] * m) @ b.phi[o:o + n].T
        assert np.abs(G - np.eye(n)).max() < 1e-13
    # Gram-Schmidt barely touches the bound states
    assert np.abs(b.phi[0] - hydrogen_radial(1, 0, 1.0, b.r)).max() < 1e-10


def test_basis_counts_large():
    # N_l = n_max - l + n_bins, all m: 580 states for n<=6, 20 bins, l<=4.
    spec = BasisSpec(n_max=6, l_max=4, n_bins=20, k_max=3.0, n_r=400)
    b = build_basis(spec)
    assert b.n_per_l == [26, 25, 24, 23, 22]
    assert b.n_states == 580 and b.n_radial == 120
