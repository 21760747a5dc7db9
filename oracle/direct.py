"""Direct couplings: Eq. D2 radial multipole integrals and Eq. D1 assembly.

Test infrastructure only (see ``oracle/__init__.py``).

Readings (the paper is garbled or silent here)
----------------------------------------------
* Eq. D1's angular factor sqrt((lambda-mu)/(lambda+mu)) is read as the
  factorial ratio sqrt((lambda-mu)!/(lambda+mu)!): this is what the multipole
  expansion of 1/|r-R| with R = (b, 0, z) and the Gaunt integral give, and the
  literal form vanishes for mu = lambda.  mu = m' - m.
* The overall minus sign is the attractive electron-projectile potential
  -Z_P/|r - R|; the couplings are scaled by the projectile charge Z_P.
* Amplitudes are in the interaction picture (Eq. 1 has no energy term), so
  every element carries exp(i (eps_row - eps_col) z / v).
* The projectile-centred block D_P is the same expression about the
  projectile, where the other nucleus sits at -R: P_lambda^mu picks up
  (-1)^lambda.
"""
from __future__ import annotations

import math
from functools import lru_cache

import numpy as np

from .angular import assoc_legendre, clebsch_gordan
from .radial import Basis


def multipole_kernel(lam: int, r: np.ndarray, R: float) -> np.ndarray:
    """min(r,R)^lambda / max(r,R)^(lambda+1) (Eq. D2)."""
    lo = np.minimum(r, R)
    hi = np.maximum(r, R)
    out = lo ** lam / hi ** (lam + 1)
    return out


def radial_integrals(basis: Basis, R: float, lam: int) -> np.ndarray:
    """F_{a b lambda}(R) of Eq. D2 for all radial pairs, by the grid quadrature.

    F = Phi diag(w r^2 g_lambda(r; R)) Phi^T, the r = 0 node excluded (its
    weight is zero).  Returns [N_f, N_f].
    """
    r = basis.r[1:]
    w = basis.w[1:]
    phi = basis.phi[:, 1:]
    g = w * r * r * multipole_kernel(lam, r, R)
    return (phi * g) @ phi.T


def lagrange5(nodes: np.ndarray, x: float) -> np.ndarray:
    """Weights of the Lagrange polynomial through five nodes evaluated at x:
    L_i(x) = prod_{k != i} (x - x_k) / (x_i - x_k)."""
    w = np.ones(5)
    for i in range(5):
        for k in range(5):
            if k != i:
                w[i] *= (x - nodes[k]) / (nodes[i] - nodes[k])
    return w


def stencil_start(basis: Basis, R: float) -> int:
    """First node of the five-point stencil at R < r_max: the node j nearest
    to R in x = sqrt(r / r_max) (the grid is uniform in x), nodes j-2..j+2,
    clamped to the grid."""
    n_r = basis.spec.n_r
    j = int(round(n_r * math.sqrt(R / basis.spec.r_max)))
    return min(max(j, 2), n_r - 2) - 2


def radial_integrals_interp(basis: Basis, R: float, lam: int) -> np.ndarray:
    """F_{a b lambda}(R) as the paper's production code evaluates it (Sec. II):
    F tabulated on the r-grid (R = r_k, the quadrature of Eq. D2 at each node)
    and interpolated at R by the five-point Lagrange polynomial in r.  For R at
    or beyond the grid's end the quadrature is the multipole form
    R^-(lam+1) sum_i w_i r_i^(2+lam) f_a f_b, evaluated directly (reading: the
    table ends at r_max).  Returns [N_f, N_f]."""
    if R >= basis.spec.r_max:
        return radial_integrals(basis, R, lam)
    j0 = stencil_start(basis, R)
    nodes = basis.r[j0:j0 + 5]
    w = lagrange5(nodes, R)
    out = np.zeros((basis.n_radial, basis.n_radial))
    for i in range(5):
        out += w[i] * radial_integrals(basis, float(nodes[i]), lam)
    return out


@lru_cache(maxsize=None)
def d1_coefficient(lp: int, mp: int, l: int, m: int, lam: int) -> float:
    """The lambda-term of Eq. D1 without P and F:
    -sqrt((2l+1)(lam-mu)!/((2l'+1)(lam+mu)!)) C^{l'0}_{lam 0 l 0} C^{l'm'}_{lam mu l m},
    mu = m' - m (zero when |mu| > lambda or a coefficient vanishes)."""
    mu = mp - m
    if abs(mu) > lam:
        return 0.0
    c1 = clebsch_gordan(lam, 0, l, 0, lp, 0)
    c2 = clebsch_gordan(lam, mu, l, m, lp, mp)
    if c1 == 0.0 or c2 == 0.0:
        return 0.0
    fac = math.sqrt((2 * l + 1) * math.factorial(lam - mu)
                    / ((2 * lp + 1) * math.factorial(lam + mu)))
    return -fac * c1 * c2


def d1_angular(lp: int, mp: int, l: int, m: int, lam: int, cos_theta: float) -> float:
    """The full lambda-term of Eq. D1 without F (coefficient times P_lam^mu(cos Theta))."""
    c = d1_coefficient(lp, mp, l, m, lam)
    if c == 0.0:
        return 0.0
    return c * float(assoc_legendre(lam, mp - m, cos_theta))


def direct_spatial(basis: Basis, R: float, cos_theta: float, Zp: float = 1.0,
                   parity: int = 1, radial: str = "exact") -> np.ndarray:
    """Real spatial part of D (Eq. D1) at (R, Theta): [N, N] float64.

    ``parity`` = -1 gives the projectile-centred form (factor (-1)^lambda).
    ``radial``: "exact" (Eq. D2's quadrature at R) or "interp" (the tabulated
    F interpolated at R, ``radial_integrals_interp``).
    """
    lmax = basis.spec.l_max
    rad = radial_integrals_interp if radial == "interp" else radial_integrals
    F = [rad(basis, R, lam) for lam in range(2 * lmax + 1)]
    P = {(lam, mu): float(assoc_legendre(lam, mu, cos_theta))
         for lam in range(2 * lmax + 1) for mu in range(-lam, lam + 1)}
    N = basis.n_states
    D = np.zeros((N, N))
    # state offsets of each (l, m) block
    start = {}
    pos = 0
    for l in range(lmax + 1):
        for m in range(-l, l + 1):
            start[(l, m)] = pos
            pos += basis.n_per_l[l]
    for lp in range(lmax + 1):
        nlp = basis.n_per_l[lp]
        ap = slice(basis.rad_off[lp], basis.rad_off[lp] + nlp)
        for l in range(lmax + 1):
            nl = basis.n_per_l[l]
            a = slice(basis.rad_off[l], basis.rad_off[l] + nl)
            for mp in range(-lp, lp + 1):
                for m in range(-l, l + 1):
                    blk = np.zeros((nlp, nl))
                    for lam in range(abs(l - lp), l + lp + 1):
                        c = d1_coefficient(lp, mp, l, m, lam)
                        if c != 0.0:
                            blk += (c * P[(lam, mp - m)] * parity ** lam) * F[lam][ap, a]
                    i0 = start[(lp, mp)]
                    j0 = start[(l, m)]
                    D[i0:i0 + nlp, j0:j0 + nl] = Zp * blk
    return D


def interaction_phases(eps_row: np.ndarray, eps_col: np.ndarray, z: float, v: float) -> np.ndarray:
    """exp(i (eps_row - eps_col) z / v) as an [N_row, N_col] array."""
    return np.exp(1j * np.subtract.outer(eps_row, eps_col) * (z / v))


def direct_matrix(basis: Basis, b: float, z: float, v: float, Zp: float = 1.0,
                  parity: int = 1, z_phase: float = 0.0, radial: str = "exact") -> np.ndarray:
    """D_T(b, z) of Eq. D1 with interaction-picture phases: complex [N, N].

    R = sqrt(b^2 + z^2), cos Theta = z / R (the straight-line path R = (b, 0, z)).
    ``z_phase`` shifts the origin of the phases only (probabilities must not
    depend on it).
    """
    R = math.hypot(b, z)
    if R <= 0.0:
        raise ValueError("R must be positive")
    Dsp = direct_spatial(basis, R, z / R, Zp=Zp, parity=parity, radial=radial)
    return Dsp * interaction_phases(basis.eps, basis.eps, z + z_phase, v)
