"""Pins of the oracle's paper-production form of the radial integrals: F
tabulated on the r-grid and interpolated at R with a five-point polynomial
(Sec. II), and the propagation that uses it.

* The Lagrange weights reproduce every polynomial of degree <= 4 in r
  exactly (a wrong sign, index or missing factor fails at once), sum to 1,
  and are (1, 0, ...) at a node.
* At a grid node the interpolated F is the table entry itself (the quadrature
  of Eq. D2 at R = r_k).
* The stencil is centred on the node nearest to R and clamped at both ends.
* Off the nodes, F_0^{1s1s}(R) = 1/R - (1 + 1/R) e^{-2R} (the potential of the
  1s cloud) holds to the same 1e-5 as the exact-R quadrature.
* Interpolated and exact-R integrals approach each other as the grid is
  refined: the quadrature's F(R) has a kink at every node (the r-grid term
  moves from the r^lam/R^(lam+1) side to the R^lam/r^(lam+1) side), so the
  difference falls like h^2: by at least 3x per halving of h.
* Beyond r_max the interpolated form is the multipole form, the exact value.
* A whole one-centre path with the interpolated couplings approaches the
  exact-R path as the grid is refined, and conserves the norm as well.
"""
import math

import numpy as np
import pytest

from oracle.direct import (direct_matrix, lagrange5, radial_integrals, radial_integrals_interp,
                           stencil_start)
from oracle.propagate import probabilities, propagate_one_centre
from oracle.radial import BasisSpec, build_basis


@pytest.fixture(scope="module")
def bound_raw():
    return build_basis(BasisSpec(n_max=3, l_max=2, n_bins=0, k_max=1.0, n_r=1500), orthonormalise=False)


def test_lagrange_reproduces_quartics():
    rng = np.random.default_rng(9)
    nodes = np.sort(rng.uniform(0.1, 3.0, 5))
    for deg in range(5):
        c = rng.standard_normal(deg + 1)
        for x in (0.05, 0.7, 1.9, 3.4):
            w = lagrange5(nodes, x)
            assert abs(w @ np.polyval(c, nodes) - np.polyval(c, x)) < 1e-11 * (1 + abs(np.polyval(c, x)))
    assert abs(lagrange5(nodes, 1.234).sum() - 1.0) < 1e-13
    assert np.array_equal(lagrange5(nodes, nodes[2]), np.array([0.0, 0.0, 1.0, 0.0, 0.0]))


def test_stencil_nearest_and_clamped(bound_raw):
    b = bound_raw
    n_r = b.spec.n_r
    for k in (2, 3, 700, n_r - 2):
        assert stencil_start(b, float(b.r[k])) == k - 2
    assert stencil_start(b, 1e-9) == 0 and stencil_start(b, float(b.r[1])) == 0
    assert stencil_start(b, float(b.r[n_r - 1])) == n_r - 4
    # halfway in x between nodes 700 and 701 rounds to the nearer one
    x = (700.3 / n_r) ** 2 * b.spec.r_max
    assert stencil_start(b, x) == 698


def test_nodes_are_table_entries(bound_raw):
    b = bound_raw
    for k in (5, 333, 1200):
        R = float(b.r[k])
        for lam in (0, 2, 4):
            assert np.array_equal(radial_integrals_interp(b, R, lam), radial_integrals(b, R, lam) * 1.0) or \
                np.abs(radial_integrals_interp(b, R, lam) - radial_integrals(b, R, lam)).max() == 0.0


def test_f0_1s_closed_form_interp(bound_raw):
    for R in (0.5, 2.0, 7.0, 0.0123):
        F0 = radial_integrals_interp(bound_raw, R, 0)[0, 0]
        ref = 1 / R - (1 + 1 / R) * math.exp(-2 * R)
        assert abs(F0 - ref) < 1e-5, (R, F0 - ref)


def test_interp_converges_to_exact_as_h2():
    diffs = []
    Rs = (0.61, 1.37, 3.3, 8.05)
    for n_r in (400, 800, 1600):
        b = build_basis(BasisSpec(n_max=3, l_max=2, n_bins=0, k_max=1.0, n_r=n_r), orthonormalise=False)
        d = 0.0
        for R in Rs:
            for lam in (0, 1, 2):
                d = max(d, np.abs(radial_integrals_interp(b, R, lam) - radial_integrals(b, R, lam)).max())
        diffs.append(d)
    assert diffs[0] / diffs[1] > 3.0 and diffs[1] / diffs[2] > 3.0, diffs


def test_beyond_grid_is_multipole(bound_raw):
    b = bound_raw
    i1s, i2p = 0, b.rad_off[1]
    for R in (100.0, 250.0):
        F1 = radial_integrals_interp(b, R, 1)[i1s, i2p]
        assert abs(F1 * R * R - 128 * math.sqrt(6) / 243) < 1e-12


def test_interp_path_converges_to_exact():
    """Whole path (160 steps): the interpolated-F probabilities approach the
    exact-R ones as the grid is refined (interpolation error ~ h^2), and the
    interpolated couplings stay Hermitian (the table and the weights are real,
    F symmetric in the radial pair)."""
    zg = np.linspace(-8.0, 8.0, 161)
    dPs = []
    for n_r in (300, 600):
        bas = build_basis(BasisSpec(n_max=2, l_max=1, n_bins=3, k_max=2.0, n_r=n_r, r_max=60.0))
        Xe = propagate_one_centre(bas, 0.9, 1.2, zg)
        Xi = propagate_one_centre(bas, 0.9, 1.2, zg, radial="interp")
        dPs.append(np.abs(probabilities(Xi) - probabilities(Xe)).max())
        assert abs(np.vdot(Xi, Xi).real - np.vdot(Xe, Xe).real) < 1e-6
    assert dPs[0] / dPs[1] > 3.0, dPs
    Di = direct_matrix(bas, 0.9, 0.37, 1.2, radial="interp")
    assert np.abs(Di - Di.conj().T).max() < 1e-15 * np.abs(Di).max()
