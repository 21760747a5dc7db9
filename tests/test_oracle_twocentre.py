"""Pins of the oracle's two-centre couplings (no GPU).

* closed forms at v = 0: the 1s-1s overlap e^{-R}(1 + R + R^2/3) and the
  transfer integral <1s_T| -1/r_T |1s_P> = -(1 + R) e^{-R};
* a lab-frame quadrature of phi_T^* exp(i v.r_c) phi_P (and with -Z_T/r_T)
  over the same spheroidal nodes but with an explicit trapezoidal rule in the
  azimuth, lab-frame spherical harmonics from scipy and the lab geometry of
  each point: it uses none of the Wigner rotation, the Bessel-function phi
  integral, the i^(q-q') factor or the Eq. K2 prefactor, so it pins all the
  frame conventions of Eq. K1/K2;
* Gauss-Laguerre weights against their defining moments.
"""
import math

import numpy as np
import pytest
from scipy.special import roots_laguerre, sph_harm_y

from oracle.propagate import initial_state, rk4_propagate
from oracle.radial import BasisSpec, build_basis
from oracle.twocentre import (Q_DAGGER, Q_PRIOR, gauss_legendre, interpolate_radial, lab_matrix,
                              laguerre_scaled_weights, m_two_centre, m_two_centre_symmetric,
                              spheroidal_quadrature, symmetric_matrices, two_centre_matrices)


@pytest.fixture(scope="module")
def bound2():
    """Bound hydrogen states n <= 2 (1s, 2s, 2p) on a fine grid, both centres."""
    return build_basis(BasisSpec(n_max=2, l_max=1, n_bins=0, k_max=1.0, n_r=3000, r_max=60.0))


@pytest.fixture(scope="module")
def mixed():
    """n <= 3 bound + 1 bin per l, l <= 2: covers l up to 2 and every m."""
    return build_basis(BasisSpec(n_max=3, l_max=2, n_bins=1, k_max=1.0, n_r=1200, r_max=60.0))


def test_laguerre_scaled_weights_moments():
    x, W = laguerre_scaled_weights(40)
    for k in range(0, 12):
        # int_0^inf x^k e^{-x} dx = k!
        val = np.sum(W * np.exp(-x) * x ** k)
        assert abs(val - math.factorial(k)) < 1e-11 * math.factorial(k)
    xr, wr = roots_laguerre(40)
    assert np.allclose(W * np.exp(-x), wr, rtol=1e-11, atol=0)


def test_laguerre_scaled_weights_large_n_finite():
    x, W = laguerre_scaled_weights(256)
    assert np.all(np.isfinite(W)) and np.all(W > 0)
    # the integral of e^{-x} (weight function times 1) with the scaled weights
    assert abs(np.sum(W * np.exp(-x)) - 1.0) < 1e-11


@pytest.mark.parametrize("n", [32, 512])
def test_gauss_legendre_moments_and_extended_precision(n):
    """tau rule of the spheroidal quadrature: exact for x^k, k <= 2n - 1
    (int_-1^1 x^k = 2/(k+1) for even k, 0 for odd), and equal to the rule
    recomputed by Newton's method in extended precision."""
    x, w = gauss_legendre(n)
    assert np.all(np.diff(x) > 0) and np.all(w > 0)
    for k in [0, 1, 2, 7, 10, 100, 500, 1000]:
        if k > 2 * n - 1:
            continue
        exact = 2.0 / (k + 1) if k % 2 == 0 else 0.0
        assert abs(np.sum(w * x ** k) - exact) <= 1e-13 * max(exact, 1e-3), k
    L = np.longdouble
    t = np.cos(np.pi * (np.arange(n, dtype=L) + L(0.75)) / (L(n) + L(0.5)))
    for _ in range(8):
        p0, p1 = np.ones_like(t), t.copy()
        for k in range(1, n):
            p0, p1 = p1, ((2 * k + 1) * t * p1 - k * p0) / (k + 1)
        t = t - p1 / (n * (t * p1 - p0) / (t * t - 1))
    p0, p1 = np.ones_like(t), t.copy()
    for k in range(1, n):
        p0, p1 = p1, ((2 * k + 1) * t * p1 - k * p0) / (k + 1)
    wl = (2 * (1 - t * t) / (n * n * p0 * p0))[::-1]
    assert np.abs(x - t[::-1].astype(np.float64)).max() <= 2e-16
    assert np.abs(w / wl.astype(np.float64) - 1.0).max() <= 1e-11


def test_interpolation_reproduces_grid_and_smooth_function(bound2):
    b = bound2
    # at grid nodes the interpolant returns the node values
    idx = np.array([3, 100, 1500, 2990])
    assert np.allclose(interpolate_radial(b, b.r[idx]), b.phi[:, idx], rtol=0, atol=1e-14)
    # off-grid: close to the closed form 1s function 2 exp(-r)
    r = np.array([0.0123, 0.77, 3.3, 10.1])
    f = interpolate_radial(b, r)[0]
    assert np.abs(f - 2 * np.exp(-r)).max() < 1e-9
    assert np.all(interpolate_radial(b, np.array([60.5, 100.0])) == 0.0)


@pytest.mark.parametrize("R", [0.8, 2.0, 5.0])
def test_overlap_and_transfer_closed_forms(bound2, R):
    b = bound2
    K = lab_matrix(b, b, R, 0.0, 0.0, 128, 128, "overlap")
    Q = lab_matrix(b, b, R, 0.0, 0.0, 128, 128, "target", 1.0)
    assert abs(K[0, 0] - math.exp(-R) * (1 + R + R * R / 3)) < 1e-8
    assert abs(Q[0, 0] + (1 + R) * math.exp(-R)) < 1e-8
    # arbitrary orientation (z != 0) at v = 0: the s-s overlap depends on R only
    K2 = lab_matrix(b, b, R * 0.6, R * 0.8, 0.0, 128, 128, "overlap")
    assert abs(K2[0, 0] - K[0, 0]) < 1e-9


def _lab_quadrature(tb, pb, bb, z, v, n_eta, n_tau, n_phi, weight):
    """phi_T^* exp(i v.r_c) [W] phi_P by direct summation on spheroidal nodes x phi."""
    R = math.hypot(bb, z)
    th = math.acos(z / R)
    eta, tau, om = spheroidal_quadrature(n_eta, n_tau, R)
    rA = R * (eta + tau) / 2
    rB = R * (eta - tau) / 2
    keep = np.maximum(rA, rB) <= 60.0 + 1e-9
    eta, tau, om, rA, rB = eta[keep], tau[keep], om[keep], rA[keep], rB[keep]
    cA = (1 + eta * tau) / (eta + tau)
    rho = rA * np.sqrt(np.maximum(0.0, 1 - cA * cA))
    zp = rA * cA
    phi = np.arange(n_phi) * (2 * np.pi / n_phi)
    # molecular-frame point (origin at the target) -> lab by a rotation of th about y
    X = rho[:, None] * np.cos(phi)[None, :]
    Y = rho[:, None] * np.sin(phi)[None, :]
    Z = np.broadcast_to(zp[:, None], X.shape)
    xl = math.cos(th) * X + math.sin(th) * Z
    yl = Y
    zl = -math.sin(th) * X + math.cos(th) * Z
    Rv = np.array([bb, 0.0, z])
    rT = np.sqrt(xl ** 2 + yl ** 2 + zl ** 2)
    xp, yp, zpp = xl - Rv[0], yl - Rv[1], zl - Rv[2]
    rP = np.sqrt(xp ** 2 + yp ** 2 + zpp ** 2)
    assert np.allclose(rT, rA[:, None], atol=1e-9) and np.allclose(rP, rB[:, None], atol=1e-9)
    thT, phT = np.arccos(np.clip(zl / rT, -1, 1)), np.arctan2(yl, xl)
    thP, phP = np.arccos(np.clip(zpp / rP, -1, 1)), np.arctan2(yp, xp)
    trans = np.exp(1j * v * (zl - z / 2))
    jac = (R / 2) ** 3 * (eta * eta - tau * tau) * om * (2 * np.pi / n_phi)
    if weight == "target":
        wgt = -1.0 / rT
    else:
        wgt = 1.0
    fA = interpolate_radial(tb, rA)
    fB = interpolate_radial(pb, rB)
    out = np.zeros((tb.n_states, pb.n_states), dtype=np.complex128)
    ylm_T = {}
    ylm_P = {}
    for i in range(tb.n_states):
        l, m, a = tb.st_l[i], tb.st_m[i], tb.st_a[i]
        if (l, m) not in ylm_T:
            ylm_T[(l, m)] = np.conj(sph_harm_y(l, m, thT, phT))
        left = fA[a][:, None] * ylm_T[(l, m)] * trans * wgt * jac[:, None]
        for j in range(pb.n_states):
            lb, mb, bidx = pb.st_l[j], pb.st_m[j], pb.st_a[j]
            if (lb, mb) not in ylm_P:
                ylm_P[(lb, mb)] = sph_harm_y(lb, mb, thP, phP)
            out[i, j] = np.sum(left * (fB[bidx][:, None] * ylm_P[(lb, mb)]))
    return out


@pytest.mark.parametrize("bb,z,v", [(1.3, 0.7, 1.0), (0.6, -1.9, 2.0), (2.5, 0.0, 0.5)])
def test_k1_k2_conventions_against_lab_frame(mixed, bb, z, v):
    nE, nT = 40, 48
    for weight in ("overlap", "target"):
        ref = _lab_quadrature(mixed, mixed, bb, z, v, nE, nT, 96, weight)
        got = lab_matrix(mixed, mixed, bb, z, v, nE, nT, weight, 1.0)
        # the lab quadrature drops nodes beyond r_max where both vanish; the
        # azimuthal rule is spectrally accurate for these smooth integrands
        scale = np.abs(ref).max()
        assert np.abs(got - ref).max() <= 1e-9 * scale, (weight, np.abs(got - ref).max(), scale)


def test_overlap_block_structure(bound2):
    b = bound2
    S, H = two_centre_matrices(b, b, 1.1, 0.4, 1.0, 48, 64)
    n = b.n_states
    assert np.abs(S - S.conj().T).max() < 1e-15
    assert np.linalg.eigvalsh(S).min() > 0
    # D_T, D_P blocks Hermitian; with Q^dagger the whole H is Hermitian
    assert np.abs(H - H.conj().T).max() < 1e-14 * np.abs(H).max()
    S2, H2 = two_centre_matrices(b, b, 1.1, 0.4, 1.0, 48, 64, q_lower=Q_PRIOR)
    assert np.array_equal(S, S2) and np.array_equal(H[:n, :], H2[:n, :])
    assert np.abs(H2[n:, :n] - H[n:, :n]).max() > 1e-6


def test_prior_form_conserves_norm_on_bound_basis(bound2):
    """With the prior lower-left block and exact eigenstates (bound hydrogen
    states on a fine grid) X^dag S X is constant along the path; RK4 leaves a
    drift that falls by more than 10x when h halves and is below 1e-8 at h = 0.05."""
    b = bound2
    M = m_two_centre(b, b, 1.5, 1.0, 24, 32, q_lower=Q_PRIOR)
    drift = []
    for h in (0.1, 0.05):
        zg = np.linspace(-4.0, 4.0, int(round(8.0 / h)) + 1)
        S0, _ = two_centre_matrices(b, b, 1.5, zg[0], 1.0, 24, 32, q_lower=Q_PRIOR)
        X0 = initial_state(2 * b.n_states)
        X0 = X0 / np.sqrt((X0.conj() @ S0 @ X0).real)
        X = rk4_propagate(M, X0, zg)
        S1, _ = two_centre_matrices(b, b, 1.5, zg[-1], 1.0, 24, 32, q_lower=Q_PRIOR)
        drift.append(abs((X.conj() @ S1 @ X).real - 1.0))
    assert drift[1] < 1e-8 and drift[0] > 10 * drift[1], drift


def test_dagger_form_balance_law(bound2):
    """With the printed Q^dagger block H stays Hermitian while S changes, so
    d(X^dag S X)/dz = X^dag (dS/dz) X: the change of X^dag S X over the path
    equals the integral of X^dag (dS/dz) X (dS/dz by central differences,
    Simpson's rule on the grid), up to an error of high order in h, while the
    change itself is of order 1e-3."""
    b = bound2
    n = b.n_states

    def S_of(z):
        K = lab_matrix(b, b, 1.5, z, 1.0, 24, 32, "overlap") * np.exp(
            1j * np.subtract.outer(b.eps, b.eps) * z)
        return np.block([[np.eye(n), K], [K.conj().T, np.eye(n)]])

    M = m_two_centre(b, b, 1.5, 1.0, 24, 32, q_lower=Q_DAGGER)
    gaps = []
    for h in (0.2, 0.1):
        zg = np.linspace(-3.0, 3.0, int(round(6.0 / h)) + 1)
        X, hist = rk4_propagate(M, initial_state(2 * n), zg, keep=True)
        change = (X.conj() @ S_of(zg[-1]) @ X).real - 1.0
        d = 1e-4
        f = np.array([(x.conj() @ ((S_of(z + d) - S_of(z - d)) / (2 * d)) @ x).real for z, x in zip(zg, hist)])
        integral = h / 3 * (f[0] + f[-1] + 4 * f[1:-1:2].sum() + 2 * f[2:-1:2].sum())
        gaps.append(abs(change - integral))
        assert abs(change) > 1e-3
    assert gaps[1] < 2e-7 and gaps[0] > 10 * gaps[1], gaps


def test_symmetric_form_conserves_norm(bound2):
    """The S-norm-conserving form built from the printed Q^dagger block (which
    itself changes X^dag S X by ~1e-3 over this path, above): X^dag S X stays
    at 1 up to RK4's error, which falls by more than 10x when h halves, and
    the central difference of S.  A sign or factor slip in the -(i v/2) dS/dz
    term, or dS/dz transposed, leaves a drift of the dagger form's size."""
    b = bound2
    n2 = 2 * b.n_states
    M = m_two_centre_symmetric(b, b, 1.5, 1.0, 24, 32, q_lower=Q_DAGGER)
    drift = []
    for h in (0.1, 0.05):
        zg = np.linspace(-3.0, 3.0, int(round(6.0 / h)) + 1)
        S0, _ = two_centre_matrices(b, b, 1.5, zg[0], 1.0, 24, 32)
        X0 = initial_state(n2) / math.sqrt((S0[0, 0]).real)
        X = rk4_propagate(M, X0, zg)
        S1, _ = two_centre_matrices(b, b, 1.5, zg[-1], 1.0, 24, 32)
        drift.append(abs((X.conj() @ S1 @ X).real - (X0.conj() @ S0 @ X0).real))
    assert drift[1] < 1e-8 and drift[0] > 10 * drift[1], drift


@pytest.mark.parametrize("z", [-1.1, 0.4])
def test_symmetric_form_reproduces_prior_form_on_eigenstates(bound2, z):
    """On exact eigenstates the prior and post transfer blocks differ by the
    overlap's derivative, Q - L^dag = -i v dK/dz, so the prior form already
    has the anti-Hermitian part the symmetric form imposes: H~ built from the
    prior form is the prior H itself, while H~ built from the dagger form
    differs from that H by (v/2)|dK/dz|.  The bound states on the fine grid
    are eigenstates to ~1e-6 (hence the bar)."""
    b = bound2
    v = 1.0
    S, Hp = two_centre_matrices(b, b, 1.5, z, v, 24, 32, q_lower=Q_PRIOR)
    _, Hs_prior = symmetric_matrices(b, b, 1.5, z, v, 24, 32, q_lower=Q_PRIOR)
    _, Hs_dag = symmetric_matrices(b, b, 1.5, z, v, 24, 32, q_lower=Q_DAGGER)
    _, Hd = two_centre_matrices(b, b, 1.5, z, v, 24, 32, q_lower=Q_DAGGER)
    scale = np.abs(Hp).max()
    assert np.abs(Hs_prior - Hp).max() <= 1e-5 * scale
    # the dagger form's H~ has the same anti-Hermitian part ...
    assert np.abs((Hs_dag - Hs_dag.conj().T) - (Hp - Hp.conj().T)).max() <= 1e-5 * scale
    # ... and is not the dagger H: their difference is the K-block term
    n = b.n_states
    Sp, _ = two_centre_matrices(b, b, 1.5, z + 1e-3, v, 24, 32)
    Sm, _ = two_centre_matrices(b, b, 1.5, z - 1e-3, v, 24, 32)
    dK = (Sp - Sm)[:n, n:] / 2e-3
    assert np.abs((Hs_dag - Hd)[:n, n:] + 0.5j * v * dK).max() <= 1e-6 * scale
    assert np.abs(dK).max() > 1e-2


def test_prior_block_mirrors_q_on_one_basis(mixed):
    """With one basis on both centres the spheroidal quadrature is symmetric
    under tau -> -tau, which exchanges the centres, turns the target
    potential's weight into the projectile's and conjugates the translation
    phase: the prior lower-left block is then (-1)^(l_i + l_j) Q_ij (the same
    indices), to rounding.  With the dagger form the block is Q^dagger, which
    differs."""
    b = mixed
    par = np.concatenate([np.full((2 * l + 1) * b.n_per_l[l], (-1.0) ** l) for l in range(b.spec.l_max + 1)])
    n = b.n_states
    for bb, z, v in ((1.3, -0.7, 1.0), (0.6, 2.1, 0.5)):
        _, H = two_centre_matrices(b, b, bb, z, v, 24, 32, q_lower=Q_PRIOR)
        Q, L = H[:n, n:], H[n:, :n]
        assert np.abs(L - par[:, None] * Q * par[None, :]).max() <= 1e-14 * np.abs(Q).max()
        assert np.abs(L - Q.conj().T).max() > 1e-3 * np.abs(Q).max()
