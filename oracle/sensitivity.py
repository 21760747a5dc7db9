"""Screened target potential and the tangent-linear sensitivities of the
one-centre propagation (reference gradients for the adjoint).

Test infrastructure only (see ``oracle/__init__.py``).

Model potential (reading of the screened form V(r) = -(1 + a e^{-c r})/r on
the fixed hydrogen + wave-packet basis): the target Hamiltonian gains
DeltaV = -a e^{-c r}/r, whose matrix on the basis is block diagonal in
(l, m) with the radial block
    DeltaV_{a' a} = -a sum_i w_i r_i f_a'(r_i) f_a(r_i) e^{-c r_i}
(the r^2 of the measure times 1/r).  The amplitudes stay in the interaction
picture of the unperturbed energies eps, so DeltaV enters M like D_T:
M(z) = -(i/v) [D_T(z) + DeltaV] with both carrying exp(i(eps_row - eps_col) z / v).

Sensitivities are the derivatives of the discrete scheme itself (Algorithm 1
on the given grid): every RK4 step is differentiated exactly (forward mode),
with dM/dtheta from
    dDeltaV/da = DeltaV / a,
    dDeltaV/dc = +a sum_i w_i r_i^2 f f e^{-c r_i},
    dD_T/db   = sum_lambda c(...) [P'(x) dx/db F_lambda(R) + P(x) F'_lambda(R) dR/db]
at fixed z, with R = sqrt(b^2 + z^2), x = z / R, dR/db = b / R,
dx/db = -z b / R^3, F'_lambda the R-derivative of the Eq. D2 quadrature
(sum_i w_i r_i^2 f f dg_lambda/dR, g = r_<^lambda / r_>^(lambda+1)) and P' from
(x^2 - 1) dP_l^m/dx = l x P_l^m - (l + m) P_(l-1)^m.
"""
from __future__ import annotations

import math

import numpy as np

from .angular import assoc_legendre
from .direct import d1_coefficient, direct_spatial, interaction_phases, radial_integrals
from .radial import Basis


def _blocks(basis: Basis):
    """(l, m, state offset) of every (l, m) block in the canonical order."""
    out, pos = [], 0
    for l in range(basis.spec.l_max + 1):
        for m in range(-l, l + 1):
            out.append((l, m, pos))
            pos += basis.n_per_l[l]
    return out


def _radial_block_diag(basis: Basis, radial: np.ndarray) -> np.ndarray:
    """Spread a [N_f, N_f] radial matrix (used within equal l only) over the states."""
    N = basis.n_states
    out = np.zeros((N, N))
    for l, m, pos in _blocks(basis):
        nl = basis.n_per_l[l]
        a = slice(basis.rad_off[l], basis.rad_off[l] + nl)
        out[pos:pos + nl, pos:pos + nl] = radial[a, a]
    return out


def model_potential(basis: Basis, a: float, c: float) -> np.ndarray:
    """DeltaV = -a e^{-c r}/r on the basis: real [N, N]."""
    r, w, phi = basis.r[1:], basis.w[1:], basis.phi[:, 1:]
    rad = -a * (phi * (w * r * np.exp(-c * r))) @ phi.T
    return _radial_block_diag(basis, rad)


def model_potential_dc(basis: Basis, a: float, c: float) -> np.ndarray:
    """d DeltaV / dc = +a sum w r^2 f f e^{-c r}: real [N, N]."""
    r, w, phi = basis.r[1:], basis.w[1:], basis.phi[:, 1:]
    rad = a * (phi * (w * r * r * np.exp(-c * r))) @ phi.T
    return _radial_block_diag(basis, rad)


def multipole_kernel_dR(lam: int, r: np.ndarray, R: float) -> np.ndarray:
    """d/dR of min(r,R)^lambda / max(r,R)^(lambda+1): -(lambda+1) r^lambda / R^(lambda+2)
    for r < R, lambda R^(lambda-1) / r^(lambda+1) for r > R."""
    inner = -(lam + 1) * r ** lam / R ** (lam + 2)
    outer = lam * R ** (lam - 1) / r ** (lam + 1) if lam > 0 else np.zeros_like(r)
    return np.where(r < R, inner, outer)


def radial_integrals_dR(basis: Basis, R: float, lam: int) -> np.ndarray:
    """dF_{ab lambda}/dR of the Eq. D2 grid quadrature: [N_f, N_f]."""
    r, w, phi = basis.r[1:], basis.w[1:], basis.phi[:, 1:]
    g = w * r * r * multipole_kernel_dR(lam, r, R)
    return (phi * g) @ phi.T


def assoc_legendre_dx(l: int, m: int, x: float) -> float:
    """dP_l^m/dx from (x^2 - 1) P' = l x P_l^m - (l + m) P_(l-1)^m, |x| < 1."""
    p = float(assoc_legendre(l, m, x))
    q = float(assoc_legendre(l - 1, m, x)) if l >= 1 else 0.0
    return (l * x * p - (l + m) * q) / (x * x - 1.0)


def direct_spatial_db(basis: Basis, b: float, z: float, Zp: float = 1.0) -> np.ndarray:
    """d D_T^spatial / db at fixed z (Eq. D1 differentiated term by term)."""
    R = math.hypot(b, z)
    x = z / R
    dR, dx = b / R, -z * b / R ** 3
    lmax = basis.spec.l_max
    F = [radial_integrals(basis, R, lam) for lam in range(2 * lmax + 1)]
    dF = [radial_integrals_dR(basis, R, lam) for lam in range(2 * lmax + 1)]
    N = basis.n_states
    out = np.zeros((N, N))
    blocks = _blocks(basis)
    for lp, mp, i0 in blocks:
        nlp = basis.n_per_l[lp]
        ap = slice(basis.rad_off[lp], basis.rad_off[lp] + nlp)
        for l, m, j0 in blocks:
            nl = basis.n_per_l[l]
            aa = slice(basis.rad_off[l], basis.rad_off[l] + nl)
            blk = np.zeros((nlp, nl))
            for lam in range(abs(l - lp), l + lp + 1):
                cf = d1_coefficient(lp, mp, l, m, lam)
                if cf == 0.0:
                    continue
                P = float(assoc_legendre(lam, mp - m, x))
                dP = assoc_legendre_dx(lam, mp - m, x)
                blk += cf * (dP * dx * F[lam][ap, aa] + P * dR * dF[lam][ap, aa])
            out[i0:i0 + nlp, j0:j0 + nl] = Zp * blk
    return out


def m_model(basis: Basis, b: float, v: float, a: float, c: float, Zp: float = 1.0):
    """z -> M(z) = -(i/v) [D_T(b, z) + DeltaV] with interaction phases."""
    dv = model_potential(basis, a, c)

    def M(z: float) -> np.ndarray:
        R = math.hypot(b, z)
        sp = direct_spatial(basis, R, z / R, Zp=Zp) + dv
        return (-1j / v) * sp * interaction_phases(basis.eps, basis.eps, z, v)
    return M


def dm_model(basis: Basis, b: float, v: float, a: float, c: float, Zp: float = 1.0):
    """z -> [dM/da, dM/dc, dM/db] at fixed z."""
    dva = model_potential(basis, 1.0, c)          # DeltaV / a
    dvc = model_potential_dc(basis, a, c)

    def dM(z: float):
        ph = (-1j / v) * interaction_phases(basis.eps, basis.eps, z, v)
        return [ph * dva, ph * dvc, ph * direct_spatial_db(basis, b, z, Zp=Zp)]
    return dM


def rk4_tangent(M, dM, X0: np.ndarray, zgrid: np.ndarray):
    """Algorithm 1 with forward-mode derivatives of every step.

    M(z) -> [N, N]; dM(z) -> list of dM/dtheta_k.  Returns X at the last point
    and the list of dX/dtheta_k (dX0/dtheta = 0)."""
    X = np.array(X0, dtype=np.complex128, copy=True)
    M_new, dM_new = M(zgrid[0]), dM(zgrid[0])
    nth = len(dM_new)
    dX = [np.zeros_like(X) for _ in range(nth)]
    for i in range(len(zgrid) - 1):
        z, zn = zgrid[i], zgrid[i + 1]
        h = zn - z
        M1, dM1 = M_new, dM_new
        M2, dM2 = M(0.5 * (z + zn)), dM(0.5 * (z + zn))
        M_new, dM_new = M(zn), dM(zn)
        M3, dM3 = M_new, dM_new
        k1 = M1 @ X
        u2 = X + 0.5 * h * k1
        k2 = M2 @ u2
        u3 = X + 0.5 * h * k2
        k3 = M2 @ u3
        u4 = X + h * k3
        k4 = M3 @ u4
        for t in range(nth):
            d = dX[t]
            dk1 = dM1[t] @ X + M1 @ d
            du2 = d + 0.5 * h * dk1
            dk2 = dM2[t] @ u2 + M2 @ du2
            du3 = d + 0.5 * h * dk2
            dk3 = dM2[t] @ u3 + M2 @ du3
            du4 = d + h * dk3
            dk4 = dM3[t] @ u4 + M3 @ du4
            dX[t] = d + (h / 6.0) * (dk1 + 2.0 * dk2 + 2.0 * dk3 + dk4)
        X = X + (h / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
    return X, dX


def loss_gradient(X: np.ndarray, dX: list, weights: np.ndarray):
    """L = sum_i w_i |X_i|^2 and dL/dtheta_k = sum_i w_i 2 Re(conj(X_i) dX_i/dtheta_k)."""
    L = float(np.sum(weights * np.abs(X) ** 2))
    g = [float(np.sum(weights * 2.0 * np.real(np.conj(X) * d))) for d in dX]
    return L, g
