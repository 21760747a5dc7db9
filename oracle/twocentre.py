"""Two-centre couplings: Eq. K1/K2 overlaps, transfer couplings, S and H of Eq. 1.

Test infrastructure only (see ``oracle/__init__.py``).

Geometry and conventions (the paper's Eq. K1/K2 with its index typos read as
below; every convention here is pinned by the lab-frame quadrature in the
tests, which uses none of the molecular-frame algebra):

* Target nucleus T at the origin, projectile P at R = (b, 0, z), b > 0,
  v = v z^.  Prolate spheroidal coordinates with foci A = T and B = P:
  r_A = R (eta + tau)/2, r_B = R (eta - tau)/2, cos theta_A = (1 + eta tau)/(eta + tau),
  cos theta_B = (eta tau - 1)/(eta - tau), volume (R/2)^3 (eta^2 - tau^2).
* Target states phi_alpha(r) = f_a(r) Y_{l m}(r^) and projectile states
  phi_beta(r) = f_b(|r - R|) Y_{l m}((r - R)^), both quantised along the lab z.
  Translation factors exp(-+ i v.r_c / 2), r_c measured from the midpoint of
  T and P, so every target-projectile element carries exp(i v.r_c).
* The molecular frame is the lab frame turned by theta = arccos(z/R) about y
  (its x' axis is (cos theta, 0, -sin theta)); then
  Y_{lm}(r^) = sum_q d^l_{mq}(theta) Y_{lq}(r'^) with Wigner's d (real), so
  K_{alpha beta} = sum_{q' q} d^{l_a}_{m_a q'} d^{l_b}_{m_b q} S_{(a q'), (b q)}   (Eq. K1,
  read with d^{l_alpha}_{m_alpha q} in the second factor).
* In that frame v.r_c = (v z / 2) eta tau - X cos(phi), X = (v b / 2)
  sqrt((eta^2 - 1)(1 - tau^2)), and the phi integral gives
  2 pi (-i)^(q - q') J_{q - q'}(X).  The paper prints i^(q - q'): that is the
  same integral with the molecular x' axis reversed, which the d-matrices of
  Eq. K1 do not carry; the sign used here is the one the lab-frame quadrature
  confirms.
* Transfer couplings (Q) use the same integral with the weight of the
  target's potential acting between the two centres:
  (eta^2 - tau^2) -> -(2 Z_T / R)(eta - tau)  (= (eta^2 - tau^2) (-Z_T / r_A)).
  The lower-left block of H is Q^dagger as printed in Eq. 1 (default); the
  prior form <phi_P | -Z_P/r_B | phi_T> is available as an option.
* Interaction-picture phases exp(i (eps_row - eps_col) z / v) on every block.
* Radial functions at r_A, r_B: 5-point Lagrange interpolation in r on the
  grid nodes j-2..j+2, j the node nearest in x = sqrt(r / r_max) (clamped to
  2..n_r-2); f = 0 beyond r_max.
* eta: Gauss-Laguerre in x = R (eta - 1) with weights w_i e^{x_i} formed from
  the scaled Laguerre recurrence (no underflow at 256 nodes); tau:
  Gauss-Legendre.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import roots_laguerre

from .angular import assoc_legendre, bessel_j, wigner_small_d
from .direct import direct_spatial, interaction_phases
from .radial import Basis

Q_DAGGER = "dagger"
Q_PRIOR = "prior"


def laguerre_scaled_weights(n: int):
    """Gauss-Laguerre nodes x_i and weights w_i e^{x_i} = x_i / ((n+1)^2 l(x_i)^2),
    l(x) = e^{-x/2} L_{n+1}(x) by the three-term recurrence (bounded, no underflow)."""
    x, _ = roots_laguerre(n)
    # polish the nodes by Newton steps on L_n: L_n' = n (L_n - L_{n-1}) / x
    for _ in range(3):
        p0 = np.exp(-x / 2.0)
        p1 = (1.0 - x) * p0
        for k in range(1, n):
            p0, p1 = p1, ((2 * k + 1 - x) * p1 - k * p0) / (k + 1)
        x = x - x * p1 / (n * (p1 - p0))
    l0 = np.exp(-x / 2.0)
    l1 = (1.0 - x) * l0
    for k in range(1, n + 1):
        l0, l1 = l1, ((2 * k + 1 - x) * l1 - k * l0) / (k + 1)
    return x, x / ((n + 1) ** 2 * l1 * l1)


def gauss_legendre(n: int):
    """Gauss-Legendre nodes and weights on [-1, 1] (ascending).

    Nodes: numpy's, polished by two Newton steps on P_n.  Weights:
    2 / ((1 - x^2) P_n'(x)^2) with P_n' = n (x P_n - P_(n-1)) / (x^2 - 1) from the
    three-term recurrence; this form keeps ~1e-12 relative accuracy up to
    n = 512 near x = +-1, where numpy's own weights drift to ~1e-10."""
    x, _ = np.polynomial.legendre.leggauss(n)

    def p_n(t):
        p0, p1 = np.ones_like(t), t.copy()
        for k in range(1, n):
            p0, p1 = p1, ((2 * k + 1) * t * p1 - k * p0) / (k + 1)
        return p1, p0

    for _ in range(2):
        p1, p0 = p_n(x)
        x = x - p1 / (n * (x * p1 - p0) / (x * x - 1.0))
    p1, p0 = p_n(x)
    dp = n * (x * p1 - p0) / (x * x - 1.0)
    return x, 2.0 / ((1.0 - x * x) * dp * dp)


def spheroidal_quadrature(n_eta: int, n_tau: int, R: float):
    """Nodes (eta, tau) and weights omega for int_1^inf d eta int_-1^1 d tau.

    eta = 1 + x / R with Gauss-Laguerre x (d eta = dx / R), tau Gauss-Legendre.
    Returns flattened arrays eta, tau, omega of length n_eta * n_tau."""
    x, wx = laguerre_scaled_weights(n_eta)
    t, wt = gauss_legendre(n_tau)
    eta = 1.0 + x / R
    E, T = np.meshgrid(eta, t, indexing="ij")
    Wt = np.outer(wx / R, wt)
    return E.ravel(), T.ravel(), Wt.ravel()


def interpolate_radial(basis: Basis, r: np.ndarray) -> np.ndarray:
    """Five-point Lagrange interpolation of every radial function at r: [N_f, len(r)]."""
    n_r = basis.spec.n_r
    r_max = basis.spec.r_max
    grid = basis.r
    r = np.asarray(r, dtype=np.float64)
    out = np.zeros((basis.phi.shape[0], r.size))
    inside = r <= r_max
    ri = r[inside]
    j = np.rint(n_r * np.sqrt(ri / r_max)).astype(np.int64)
    j = np.clip(j, 2, n_r - 2)
    nodes = j[:, None] + np.arange(-2, 3)[None, :]          # [n, 5]
    rn = grid[nodes]                                        # [n, 5]
    L = np.ones((ri.size, 5))
    for i in range(5):
        for mm in range(5):
            if mm != i:
                L[:, i] *= (ri - rn[:, mm]) / (rn[:, i] - rn[:, mm])
    vals = basis.phi[:, nodes]                              # [N_f, n, 5]
    out[:, inside] = (vals * L[None, :, :]).sum(axis=2)
    return out


def _pair_norm(la, qa, lb, qb):
    """sqrt((2l_a+1)(2l_b+1)) sqrt((l_a-q')!(l_b-q)!/((l_a+q')!(l_b+q)!)) of Eq. K2."""
    f = math.factorial
    return math.sqrt((2 * la + 1) * (2 * lb + 1)) * math.sqrt(
        f(la - qa) * f(lb - qb) / (f(la + qa) * f(lb + qb)))


def molecular_matrix(tb: Basis, pb: Basis, b: float, z: float, v: float, n_eta: int, n_tau: int,
                     weight: str = "overlap", Z: float = 1.0) -> np.ndarray:
    """S_{(a q'), (b q)} of Eq. K2 in the molecular frame, for every target
    radial function a (l_a) with |q'| <= l_a and projectile function b with
    |q| <= l_b.  Index order: target (l, q', n) blocks as in the state order
    with q' in place of m; same for the projectile.

    weight: "overlap" (eta^2 - tau^2), "target" (-(2Z/R)(eta - tau)),
    "projectile" (-(2Z/R)(eta + tau))."""
    R = math.hypot(b, z)
    eta, tau, om = spheroidal_quadrature(n_eta, n_tau, R)
    rA = R * (eta + tau) / 2.0
    rB = R * (eta - tau) / 2.0
    cA = (1.0 + eta * tau) / (eta + tau)
    cB = (eta * tau - 1.0) / (eta - tau)
    X = (v * b / 2.0) * np.sqrt(np.maximum(0.0, (eta * eta - 1.0) * (1.0 - tau * tau)))
    if weight == "overlap":
        W = eta * eta - tau * tau
    elif weight == "target":
        W = -(2.0 * Z / R) * (eta - tau)
    elif weight == "projectile":
        W = -(2.0 * Z / R) * (eta + tau)
    else:
        raise ValueError(weight)
    base = om * W * np.exp(1j * (v * z / 2.0) * eta * tau)
    fA = interpolate_radial(tb, rA)
    fB = interpolate_radial(pb, rB)
    LA, LB = tb.spec.l_max, pb.spec.l_max
    nA, nB = tb.n_states, pb.n_states
    S = np.zeros((nA, nB), dtype=np.complex128)
    # state offsets (l, q) in each basis
    def offs(basis):
        o, pos = {}, 0
        for l in range(basis.spec.l_max + 1):
            for q in range(-l, l + 1):
                o[(l, q)] = pos
                pos += basis.n_per_l[l]
        return o
    oA, oB = offs(tb), offs(pb)
    for la in range(LA + 1):
        sa = slice(tb.rad_off[la], tb.rad_off[la] + tb.n_per_l[la])
        for qa in range(-la, la + 1):
            PA = assoc_legendre(la, qa, cA)
            Arow = fA[sa] * PA[None, :]
            for lb in range(LB + 1):
                sb = slice(pb.rad_off[lb], pb.rad_off[lb] + pb.n_per_l[lb])
                for qb in range(-lb, lb + 1):
                    PB = assoc_legendre(lb, qb, cB)
                    n = qb - qa
                    w = base * bessel_j(n, X) * PB
                    blk = (Arow * w[None, :]) @ fB[sb].T
                    pref = (R ** 3 / 16.0) * _pair_norm(la, qa, lb, qb) * (-1j) ** n
                    i0, j0 = oA[(la, qa)], oB[(lb, qb)]
                    S[i0:i0 + tb.n_per_l[la], j0:j0 + pb.n_per_l[lb]] = pref * blk
    return S


def rotation_matrix(basis: Basis, theta: float) -> np.ndarray:
    """U[(l m n), (l q n)] = d^l_{m q}(theta): lab states from molecular ones."""
    N = basis.n_states
    U = np.zeros((N, N))
    pos = 0
    for l in range(basis.spec.l_max + 1):
        nl = basis.n_per_l[l]
        d = np.array([[wigner_small_d(l, m, q, theta) for q in range(-l, l + 1)]
                      for m in range(-l, l + 1)])
        for im in range(2 * l + 1):
            for iq in range(2 * l + 1):
                U[pos + im * nl: pos + (im + 1) * nl, pos + iq * nl: pos + (iq + 1) * nl] = \
                    d[im, iq] * np.eye(nl)
        pos += (2 * l + 1) * nl
    return U


def lab_matrix(tb: Basis, pb: Basis, b: float, z: float, v: float, n_eta: int, n_tau: int,
               weight: str = "overlap", Z: float = 1.0) -> np.ndarray:
    """Eq. K1: the spatial target-projectile block in the lab frame (no time phases)."""
    R = math.hypot(b, z)
    theta = math.acos(z / R)
    Smol = molecular_matrix(tb, pb, b, z, v, n_eta, n_tau, weight, Z)
    return rotation_matrix(tb, theta) @ Smol @ rotation_matrix(pb, theta).T


def two_centre_matrices(tb: Basis, pb: Basis, b: float, z: float, v: float, n_eta: int,
                        n_tau: int, q_lower: str = Q_DAGGER):
    """S and H of Eq. 1 at (b, z): S = [[I, K], [K^dag, I]], H = [[D_T, Q], [L, D_P]],
    with interaction-picture phases.  Z_T = target basis Z, Z_P = projectile basis Z.
    L = Q^dagger (paper) or the prior form <phi_P | -Z_P/r_B | phi_T>."""
    R = math.hypot(b, z)
    ZT, ZP = tb.spec.Z, pb.spec.Z
    nA, nB = tb.n_states, pb.n_states
    phTP = interaction_phases(tb.eps, pb.eps, z, v)
    K = lab_matrix(tb, pb, b, z, v, n_eta, n_tau, "overlap") * phTP
    Q = lab_matrix(tb, pb, b, z, v, n_eta, n_tau, "target", ZT) * phTP
    DT = direct_spatial(tb, R, z / R, Zp=ZP) * interaction_phases(tb.eps, tb.eps, z, v)
    DP = direct_spatial(pb, R, z / R, Zp=ZT, parity=-1) * interaction_phases(pb.eps, pb.eps, z, v)
    if q_lower == Q_DAGGER:
        L = Q.conj().T
    elif q_lower == Q_PRIOR:
        L = (lab_matrix(tb, pb, b, z, v, n_eta, n_tau, "projectile", ZP) * phTP).conj().T
    else:
        raise ValueError(q_lower)
    S = np.block([[np.eye(nA), K], [K.conj().T, np.eye(nB)]])
    H = np.block([[DT, Q], [L, DP]])
    return S, H


def m_two_centre(tb: Basis, pb: Basis, b: float, v: float, n_eta: int, n_tau: int,
                 q_lower: str = Q_DAGGER):
    """z -> M(z) = -(i/v) S^{-1} H, S^{-1} H by LAPACK ZGESV (numpy.linalg.solve)."""
    def M(z: float) -> np.ndarray:
        S, H = two_centre_matrices(tb, pb, b, z, v, n_eta, n_tau, q_lower)
        return (-1j / v) * np.linalg.solve(S, H)
    return M


def symmetric_matrices(tb: Basis, pb: Basis, b: float, z: float, v: float, n_eta: int, n_tau: int,
                       q_lower: str = Q_DAGGER, dz: float = 1e-4):
    """S and the S-norm-conserving form of H at (b, z) (not in the paper; a
    variant of Eq. 1): H~ = (H + H^dag)/2 - (i v / 2) dS/dz.

    For i v S X' = H X the rate d(X^dag S X)/dz is X^dag [(i/v)(H^dag - H) +
    dS/dz] X, so X^dag S X is constant exactly when H - H^dag = -i v dS/dz, a
    relation the complete-basis matrices satisfy and the truncated ones do
    not.  H~ keeps the Hermitian part of H and takes the anti-Hermitian part
    the relation prescribes.  dS/dz is the central difference of the phased S
    at z +- dz (only its K blocks vary)."""
    S, H = two_centre_matrices(tb, pb, b, z, v, n_eta, n_tau, q_lower)
    Sp, _ = two_centre_matrices(tb, pb, b, z + dz, v, n_eta, n_tau, q_lower)
    Sm, _ = two_centre_matrices(tb, pb, b, z - dz, v, n_eta, n_tau, q_lower)
    dS = (Sp - Sm) / (2.0 * dz)
    return S, 0.5 * (H + H.conj().T) - 0.5j * v * dS


def m_two_centre_symmetric(tb: Basis, pb: Basis, b: float, v: float, n_eta: int, n_tau: int,
                           q_lower: str = Q_DAGGER, dz: float = 1e-4):
    """z -> M(z) = -(i/v) S^{-1} H~ of the S-norm-conserving form (ZGESV)."""
    def M(z: float) -> np.ndarray:
        S, Hs = symmetric_matrices(tb, pb, b, z, v, n_eta, n_tau, q_lower, dz)
        return (-1j / v) * np.linalg.solve(S, Hs)
    return M
