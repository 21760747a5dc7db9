"""Pins of the oracle's model potential and tangent-linear sensitivities (no GPU).

* <1s| e^{-c r}/r |1s> = 4 / (2 + c)^2 and its c-derivative -8 / (2 + c)^3
  (closed forms) for the model-potential matrix and its c-derivative;
* dP_l^m/dx, dF_lambda/dR and dD_T/db against central differences of the
  undifferentiated oracle functions (R kept between grid nodes, where the
  quadrature is smooth in R);
* the tangent-linear gradients of a probability loss against central
  differences of the full oracle propagation in a, c and b.
"""
import math

import numpy as np
import pytest

from oracle.angular import assoc_legendre
from oracle.direct import direct_spatial, radial_integrals
from oracle.propagate import initial_state, rk4_propagate
from oracle.radial import BasisSpec, build_basis
from oracle.sensitivity import (assoc_legendre_dx, direct_spatial_db, dm_model, loss_gradient,
                                m_model, model_potential, model_potential_dc, radial_integrals_dR,
                                rk4_tangent)


@pytest.fixture(scope="module")
def fine():
    return build_basis(BasisSpec(n_max=2, l_max=1, n_bins=0, k_max=1.0, n_r=4000, r_max=60.0))


@pytest.fixture(scope="module")
def small():
    return build_basis(BasisSpec(n_max=2, l_max=1, n_bins=2, k_max=2.0, n_r=600, r_max=60.0))


@pytest.mark.parametrize("c", [0.5, 1.3, 2.0])
def test_model_potential_closed_form_1s(fine, c):
    a = 0.7
    dv = model_potential(fine, a, c)
    assert abs(dv[0, 0] - (-a * 4.0 / (2.0 + c) ** 2)) < 1e-10
    dc = model_potential_dc(fine, a, c)
    assert abs(dc[0, 0] - a * 8.0 / (2.0 + c) ** 3) < 1e-10
    # block structure: no coupling between different l or m
    l, m = fine.st_l, fine.st_m
    off = (l[:, None] != l[None, :]) | (m[:, None] != m[None, :])
    assert np.all(dv[off] == 0.0)
    assert np.allclose(dv, dv.T, rtol=0, atol=1e-16)


@pytest.mark.parametrize("l,m", [(1, 0), (2, 1), (3, -2), (4, 3), (6, -5), (5, 0)])
def test_legendre_derivative_fd(l, m):
    for x in [-0.83, -0.2, 0.31, 0.77]:
        h = 1e-6
        fd = (float(assoc_legendre(l, m, x + h)) - float(assoc_legendre(l, m, x - h))) / (2 * h)
        an = assoc_legendre_dx(l, m, x)
        assert abs(an - fd) <= 1e-7 * max(1.0, abs(fd)), (l, m, x, an, fd)


@pytest.mark.parametrize("lam", [0, 1, 2, 3])
def test_radial_integral_R_derivative_fd(small, lam):
    r = small.r
    for R in [0.7, 3.3, 17.9]:
        i = np.searchsorted(r, R)
        h = 1e-3 * min(R - r[i - 1], r[i] - R)
        fd = (radial_integrals(small, R + h, lam) - radial_integrals(small, R - h, lam)) / (2 * h)
        an = radial_integrals_dR(small, R, lam)
        assert np.abs(an - fd).max() <= 1e-6 * max(np.abs(an).max(), 1e-3), (lam, R)


def test_direct_db_fd(small):
    r = small.r
    for b, z in [(1.3, -2.2), (0.6, 0.9), (4.0, 7.5)]:
        R = math.hypot(b, z)
        i = np.searchsorted(r, R)
        h = 1e-3 * min(R - r[i - 1], r[i] - R) * R / b
        Dp = direct_spatial(small, math.hypot(b + h, z), z / math.hypot(b + h, z))
        Dm = direct_spatial(small, math.hypot(b - h, z), z / math.hypot(b - h, z))
        fd = (Dp - Dm) / (2 * h)
        an = direct_spatial_db(small, b, z)
        assert np.abs(an - fd).max() <= 1e-6 * np.abs(an).max(), (b, z)


def test_tangent_gradients_match_finite_differences(small):
    b, v, a, c = 1.3, 1.0, 0.6, 1.1
    zg = np.linspace(-5.0, 5.0, 41)
    X0 = initial_state(small.n_states)
    rng = np.random.default_rng(11)
    wts = rng.uniform(0.0, 1.0, small.n_states)
    X, dX = rk4_tangent(m_model(small, b, v, a, c), dm_model(small, b, v, a, c), X0, zg)
    L, g = loss_gradient(X, dX, wts)
    # the undifferentiated propagation reproduces X
    Xr = rk4_propagate(m_model(small, b, v, a, c), X0, zg)
    assert np.abs(X - Xr).max() < 1e-15

    def loss(aa, cc, bb):
        Xf = rk4_propagate(m_model(small, bb, v, aa, cc), X0, zg)
        return float(np.sum(wts * np.abs(Xf) ** 2))

    for k, (da, dc, db) in enumerate([(1e-5, 0, 0), (0, 1e-5, 0), (0, 0, 1e-5)]):
        fd = (loss(a + da, c + dc, b + db) - loss(a - da, c - dc, b - db)) / (2 * (da + dc + db))
        assert abs(g[k] - fd) <= 1e-7 * max(1.0, abs(fd)), (k, g[k], fd)
