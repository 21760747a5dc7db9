"""Pins of the oracle's Algorithm 1 (RK4) and of the 1C propagation (no GPU)."""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle.direct import direct_spatial
from oracle.propagate import (initial_state, probabilities, propagate_one_centre,
                              rk4_propagate, z_grid_geometric)
from oracle.radial import BasisSpec, build_basis


def test_rk4_constant_matrix_is_taylor_polynomial():
    rng = np.random.default_rng(1)
    A = rng.standard_normal((6, 6)) + 1j * rng.standard_normal((6, 6))
    x0 = rng.standard_normal(6) + 1j * rng.standard_normal(6)
    h = 0.13
    X = rk4_propagate(lambda z: A, x0, np.array([0.4, 0.4 + h]))
    ref = x0.copy()
    term = x0.copy()
    for k in range(1, 5):
        term = (h * A) @ term / k
        ref = ref + term
    assert np.abs(X - ref).max() <= 1e-14 * np.abs(ref).max()


def test_rk4_fourth_order_on_known_solution():
    # dX/dz = i z X  ->  X = exp(i z^2 / 2)
    errs = []
    for n in (20, 40, 80):
        zg = np.linspace(0.0, 2.0, n + 1)
        X = rk4_propagate(lambda z: np.array([[1j * z]]), np.array([1.0 + 0j]), zg)
        errs.append(abs(X[0] - np.exp(1j * 2.0)))
    assert 12 < errs[0] / errs[1] < 20 and 12 < errs[1] / errs[2] < 20


def test_geometric_zgrid():
    zg = z_grid_geometric(1e-3, 100.0, 500)
    assert zg.size == 1001 and zg[500] == 0.0
    assert abs(zg[-1] - 100.0) < 1e-12 and abs(zg[0] + 100.0) < 1e-12
    assert abs(zg[501] - 1e-3 * (1e5) ** (1 / 500)) < 1e-15
    assert np.all(np.diff(zg) > 0)


@pytest.fixture(scope="module")
def tiny():
    return build_basis(BasisSpec(n_max=2, l_max=1, n_bins=2, k_max=1.5, n_r=400, r_max=60.0))


def test_norm_conservation_fourth_order(tiny):
    devs = []
    for n in (100, 200, 400):
        zg = np.linspace(-20, 20, n + 1)
        X = propagate_one_centre(tiny, 1.0, 1.0, zg)
        devs.append(abs(probabilities(X).sum() - 1.0))
    assert devs[0] / devs[1] > 12 and devs[1] / devs[2] > 12


def test_phase_origin_invariance(tiny):
    zg = np.linspace(-20, 20, 201)
    P0 = probabilities(propagate_one_centre(tiny, 1.3, 0.8, zg))
    P1 = probabilities(propagate_one_centre(tiny, 1.3, 0.8, zg, z_phase=3.7))
    assert np.abs(P0 - P1).max() < 1e-13


def test_large_b_no_transition(tiny):
    zg = np.linspace(-20, 20, 201)
    P = probabilities(propagate_one_centre(tiny, 500.0, 1.0, zg))
    assert P[0] > 1 - 1e-5


def test_interaction_picture_matches_schroedinger_picture():
    # i v dc/dz = (E + V(z)) c in the Schroedinger picture has no phase
    # convention to choose; |c|^2 must equal the oracle's |X|^2.
    b = build_basis(BasisSpec(n_max=2, l_max=1, n_bins=0, k_max=1.0, n_r=800, r_max=60.0))
    bb, v = 1.0, 1.0
    E = np.diag(b.eps)

    def rhs(z, c):
        R = math.hypot(bb, z)
        V = direct_spatial(b, R, z / R)
        return (-1j / v) * ((E + V) @ c)

    zg = np.linspace(-15.0, 15.0, 1501)
    sol = solve_ivp(rhs, (zg[0], zg[-1]), initial_state(b.n_states), method="DOP853",
                    rtol=1e-12, atol=1e-13)
    Pref = np.abs(sol.y[:, -1]) ** 2
    P = probabilities(propagate_one_centre(b, bb, v, zg))
    assert np.abs(P - Pref).max() < 1e-6
    # the same run with the projectile charge flipped differs by far more:
    # the test can tell the two phase conventions apart
    P_flip = probabilities(propagate_one_centre(b, bb, v, zg, Zp=-1.0))
    assert np.abs(P_flip - Pref).max() > 1e-4
