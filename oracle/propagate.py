"""Algorithm 1 of the paper: fourth-order Runge-Kutta along the z-grid.

Test infrastructure only (see ``oracle/__init__.py``).

dX/dz = M X (Eq. DIFFEQ).  One-centre: M = -(i/v) D_T (Eq. NOINV read as Eq.
INV with K = Q = 0; the literal "M = D_T" drops the -i/v of Eq. INV).
Two-centre: M = -(i/v) S^{-1} H with S = [[I, K], [K^dagger, I]] obtained by
solving S M' = H with LAPACK's ZGESV (``numpy.linalg.solve``), as the paper
does, rather than by inverting S.

Initial condition: X = 0 except the target ground state (state 0) = 1.
M is evaluated once at the first grid point and then at z_mid and z_new of
every step; M at z of a step is M at z_new of the step before.
"""
from __future__ import annotations

import math
from typing import Callable

import numpy as np

from .direct import direct_matrix
from .radial import Basis


def z_grid_geometric(z_min: float, z_max: float, n_z: int) -> np.ndarray:
    """The paper's z-grid: zgrid[i] = z_min (z_max/z_min)^(i/n_z), zgrid[0] = 0,
    zgrid[-i] = -zgrid[i]; returned ascending, 2 n_z + 1 points."""
    pos = z_min * (z_max / z_min) ** (np.arange(1, n_z + 1) / n_z)
    return np.concatenate([-pos[::-1], [0.0], pos])


def rk4_propagate(M: Callable[[float], np.ndarray], X0: np.ndarray, zgrid: np.ndarray,
                  keep: bool = False):
    """Algorithm 1 with the slopes written as in the paper:
    K1 = M_z X, K2 = M_mid X + h/2 M_mid K1, K3 = M_mid X + h/2 M_mid K2,
    K4 = M_new X + h M_new K3, X <- X + h/6 (K1 + 2 K2 + 2 K3 + K4).

    Returns X at the last grid point (and the list of X at every grid point if
    ``keep``)."""
    X = np.array(X0, dtype=np.complex128, copy=True)
    hist = [X.copy()] if keep else None
    M_new = M(zgrid[0])
    for i in range(len(zgrid) - 1):
        z = zgrid[i]
        z_new = zgrid[i + 1]
        z_mid = 0.5 * (z + z_new)
        h = z_new - z
        h2 = h / 2.0
        h6 = h / 6.0
        M_z = M_new
        M_mid = M(z_mid)
        M_new = M(z_new)
        K1 = M_z @ X
        K2 = M_mid @ X + h2 * (M_mid @ K1)
        K3 = M_mid @ X + h2 * (M_mid @ K2)
        K4 = M_new @ X + h * (M_new @ K3)
        X = X + h6 * (K1 + 2.0 * K2 + 2.0 * K3 + K4)
        if keep:
            hist.append(X.copy())
    return (X, hist) if keep else X


def initial_state(n: int) -> np.ndarray:
    """X[:] = 0, X[first] = 1: the target in its ground state."""
    X = np.zeros(n, dtype=np.complex128)
    X[0] = 1.0
    return X


def m_one_centre(basis: Basis, b: float, v: float, Zp: float = 1.0, z_phase: float = 0.0,
                 radial: str = "exact"):
    """z -> M(z) = -(i/v) D_T(b, z); ``radial`` as in ``direct_spatial``."""
    def M(z: float) -> np.ndarray:
        return (-1j / v) * direct_matrix(basis, b, z, v, Zp=Zp, z_phase=z_phase, radial=radial)
    return M


def propagate_one_centre(basis: Basis, b: float, v: float, zgrid: np.ndarray,
                         Zp: float = 1.0, X0: np.ndarray | None = None,
                         z_phase: float = 0.0, radial: str = "exact") -> np.ndarray:
    """X at the end of the z-grid for one straight-line path (1C)."""
    if X0 is None:
        X0 = initial_state(basis.n_states)
    return rk4_propagate(m_one_centre(basis, b, v, Zp, z_phase, radial), X0, zgrid)


def probabilities(X: np.ndarray) -> np.ndarray:
    """P_i = |X_i|^2."""
    return (X.conj() * X).real
