"""Radial part of the oracle: r-grid, quadrature weights and the basis.

Test infrastructure only (see ``oracle/__init__.py``).

Paper anchors
-------------
* Sec. II (end): the radial integrals and the radial functions live on one
  r-grid from 0 to 100 a.u., up to 10,000 points, denser near the origin.
* Sec. II (start): the expansion functions are bound eigenstates plus
  wave-packet pseudostates of the target (and, in 2C, of the projectile).

Readings taken where the paper is silent
----------------------------------------
* Grid: r_i = r_max (i / n_r)^2, i = 0..n_r (n_r even), composite Simpson in
  x = i / n_r with the Jacobian dr = 2 r_max x dx.  The i = 0 weight is 0.
* Bound states: hydrogen-like R_nl(r) with nuclear charge Z, energies
  -Z^2 / (2 n^2); f = R_nl so that Eq. D2's r^2 f f measure is the norm.
* Wave packets: bins uniform in k on [0, k_max];
  f_i(r) = Delta_k^{-1/2} * int_{bin} psi_kl(r) dk with the momentum-normalised
  Coulomb wave psi_kl(r) = sqrt(2/pi) F_l(-Z/k, k r) / r, the k-integral by
  16-point Gauss-Legendre per bin; energy (k_lo^2 + k_lo k_hi + k_hi^2)/6,
  the exact expectation of k^2/2 over a flat bin.
* Per l, modified Gram-Schmidt on the grid (bound states by n, then bins by
  k) so that the identity blocks of Eq. 1 hold on the grid.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
from scipy.special import eval_genlaguerre

N_GAUSS_K = 16


def radial_grid(n_r: int, r_max: float):
    """Quadratic grid and Simpson weights (reading above).  Returns (r, w)."""
    if n_r < 2 or n_r % 2:
        raise ValueError("n_r must be even and >= 2")
    x = np.arange(n_r + 1, dtype=np.float64) / n_r
    r = r_max * x * x
    s = np.ones(n_r + 1)
    s[1:-1:2] = 4.0
    s[2:-1:2] = 2.0
    w = s * (1.0 / n_r) / 3.0 * (2.0 * r_max * x)
    return r, w


def hydrogen_radial(n: int, l: int, Z: float, r: np.ndarray) -> np.ndarray:
    """Hydrogen-like bound radial function R_nl(r), normalised int r^2 R^2 dr = 1."""
    rho = 2.0 * Z * r / n
    norm = math.sqrt((2.0 * Z / n) ** 3 * math.factorial(n - l - 1)
                     / (2.0 * n * math.factorial(n + l)))
    return norm * np.exp(-rho / 2.0) * rho ** l * eval_genlaguerre(n - l - 1, 2 * l + 1, rho)


def coulomb_norm(l: int, eta: np.ndarray) -> np.ndarray:
    """Coulomb normalisation C_l(eta): F_l(eta, rho) ~ C_l rho^(l+1) as rho -> 0.

    C_0^2 = 2 pi eta / (exp(2 pi eta) - 1) and C_l = C_(l-1) sqrt(l^2+eta^2)/(l(2l+1)).
    """
    x = 2.0 * np.pi * eta
    c = np.sqrt(x / np.expm1(x))
    for ll in range(1, l + 1):
        c = c * np.sqrt(ll * ll + eta * eta) / (ll * (2 * ll + 1))
    return c


def coulomb_u(l: int, k: np.ndarray, Z: float, r: np.ndarray,
              r_switch: float = 0.5, n_series: int = 80, n_taylor: int = 30) -> np.ndarray:
    """Regular solution of u'' + (k^2 + 2Z/r - l(l+1)/r^2) u = 0, u ~ r^(l+1) at 0.

    Below ``r_switch`` the power series about the origin is summed
    (j (j+2l+1) a_j = -2Z a_(j-1) - k^2 a_(j-2), a_0 = 1); beyond it the solution
    is carried from grid point to grid point by its Taylor series about the
    current point, whose coefficients follow from r^2 u'' = (l(l+1) - 2Zr -
    k^2 r^2) u.  Returns an array (len(k), len(r)); ``r`` must be ascending.
    """
    k = np.atleast_1d(np.asarray(k, dtype=np.float64))
    nk = k.size
    k2 = k * k
    L = float(l * (l + 1))
    out = np.zeros((nk, r.size))
    # origin series coefficients
    a = np.zeros((n_series + 1, nk))
    a[0] = 1.0
    for j in range(1, n_series + 1):
        prev2 = a[j - 2] if j >= 2 else 0.0
        a[j] = (-2.0 * Z * a[j - 1] - k2 * prev2) / (j * (j + 2 * l + 1))
    inner = np.nonzero(r <= r_switch)[0]
    if inner.size == 0:
        raise ValueError("the grid must start at or below r_switch")
    last = inner[-1]
    for i in inner:
        ri = r[i]
        s = np.zeros(nk)
        for j in range(n_series, -1, -1):
            s = s * ri + a[j]
        out[:, i] = ri ** (l + 1) * s
    # value and derivative at the last series point
    r0 = r[last]
    du = np.zeros(nk)
    for j in range(n_series, -1, -1):
        du = du * r0 + (j + l + 1) * a[j]
    u = out[:, last].copy()
    up = du * r0 ** l
    for i in range(last + 1, r.size):
        t = r[i] - r0
        A = L - 2.0 * Z * r0 - k2 * r0 * r0
        B = -(2.0 * Z + 2.0 * k2 * r0)
        c = [u, up]
        for n in range(0, n_taylor - 1):
            cn = c[n]
            cn1 = c[n + 1]
            cm1 = c[n - 1] if n >= 1 else 0.0
            cm2 = c[n - 2] if n >= 2 else 0.0
            num = A * cn + B * cm1 - k2 * cm2 - 2.0 * r0 * n * (n + 1) * cn1 - n * (n - 1) * cn
            c.append(num / (r0 * r0 * (n + 1) * (n + 2)))
        val = np.zeros(nk)
        der = np.zeros(nk)
        for n in range(len(c) - 1, -1, -1):
            val = val * t + c[n]
        for n in range(len(c) - 1, 0, -1):
            der = der * t + n * c[n]
        u, up, r0 = val, der, r[i]
        out[:, i] = u
    return out


def coulomb_psi(l: int, k: np.ndarray, Z: float, r: np.ndarray) -> np.ndarray:
    """Momentum-normalised Coulomb wave sqrt(2/pi) F_l(-Z/k, kr)/r on the grid.

    Shape (len(k), len(r)); the r = 0 entry is the limit (non-zero only for l = 0).
    """
    k = np.atleast_1d(np.asarray(k, dtype=np.float64))
    eta = -Z / k
    u = coulomb_u(l, k, Z, r)
    pref = math.sqrt(2.0 / math.pi) * coulomb_norm(l, eta) * k ** (l + 1)
    psi = np.zeros_like(u)
    pos = r > 0
    psi[:, pos] = u[:, pos] / r[pos]
    if not pos[0]:
        psi[:, 0] = 1.0 if l == 0 else 0.0
    return pref[:, None] * psi


def wave_packets(l: int, n_bins: int, k_max: float, Z: float, r: np.ndarray):
    """Wave-packet bins for one l: returns (f[n_bins, len(r)], eps[n_bins])."""
    edges = np.arange(n_bins + 1, dtype=np.float64) * (k_max / n_bins)
    xg, wg = np.polynomial.legendre.leggauss(N_GAUSS_K)
    kk = []
    ww = []
    for i in range(n_bins):
        lo, hi = edges[i], edges[i + 1]
        half = 0.5 * (hi - lo)
        kk.append(0.5 * (hi + lo) + half * xg)
        ww.append(half * wg)
    kk = np.concatenate(kk)
    ww = np.concatenate(ww)
    psi = coulomb_psi(l, kk, Z, r)
    f = np.zeros((n_bins, r.size))
    eps = np.zeros(n_bins)
    for i in range(n_bins):
        lo, hi = edges[i], edges[i + 1]
        sl = slice(i * N_GAUSS_K, (i + 1) * N_GAUSS_K)
        f[i] = (ww[sl, None] * psi[sl]).sum(axis=0) / math.sqrt(hi - lo)
        eps[i] = (lo * lo + lo * hi + hi * hi) / 6.0
    return f, eps


def gram_schmidt(f: np.ndarray, measure: np.ndarray) -> np.ndarray:
    """Modified Gram-Schmidt of the rows of f under <a, b> = sum_i measure_i a_i b_i."""
    q = np.array(f, dtype=np.float64, copy=True)
    for j in range(q.shape[0]):
        for i in range(j):
            q[j] -= np.dot(measure * q[i], q[j]) * q[i]
        q[j] /= math.sqrt(np.dot(measure * q[j], q[j]))
    return q


@dataclass
class BasisSpec:
    """One centre's basis recipe: bound n <= n_max (l <= l_max) plus n_bins bins per l."""
    n_max: int
    l_max: int
    n_bins: int
    k_max: float
    n_r: int
    r_max: float = 100.0
    Z: float = 1.0


@dataclass
class Basis:
    spec: BasisSpec
    r: np.ndarray
    w: np.ndarray
    phi: np.ndarray            # [N_f, n_r+1] orthonormal radial functions
    rad_l: np.ndarray          # [N_f] l of each radial function
    rad_eps: np.ndarray        # [N_f] energy of each radial function
    n_per_l: list              # N_l for l = 0..l_max
    rad_off: list              # first radial index of each l
    st_l: np.ndarray = field(default=None)   # [N] per state
    st_m: np.ndarray = field(default=None)
    st_a: np.ndarray = field(default=None)   # radial index
    eps: np.ndarray = field(default=None)    # [N] energies

    @property
    def n_states(self) -> int:
        return int(self.st_l.size)

    @property
    def n_radial(self) -> int:
        return int(self.rad_l.size)


def build_basis(spec: BasisSpec, orthonormalise: bool = True) -> Basis:
    """Bound states + wave packets per l, orthonormalised; canonical state order.

    Radial functions are ordered by l, then bound n ascending, then bins by k.
    States are ordered by l, then m = -l..l, then radial index, so the target
    ground state (1s) is state 0 (the paper's X[1] = 1).
    """
    r, w = radial_grid(spec.n_r, spec.r_max)
    measure = w * r * r
    phis, ls, epss, n_per_l, off = [], [], [], [], []
    for l in range(spec.l_max + 1):
        rows, e = [], []
        for n in range(l + 1, spec.n_max + 1):
            rows.append(hydrogen_radial(n, l, spec.Z, r))
            e.append(-spec.Z * spec.Z / (2.0 * n * n))
        if spec.n_bins > 0:
            fw, ew = wave_packets(l, spec.n_bins, spec.k_max, spec.Z, r)
            rows.extend(list(fw))
            e.extend(list(ew))
        block = np.array(rows)
        if orthonormalise and block.size:
            block = gram_schmidt(block, measure)
        off.append(sum(n_per_l))
        n_per_l.append(block.shape[0])
        phis.append(block)
        ls.extend([l] * block.shape[0])
        epss.extend(e)
    phi = np.concatenate(phis, axis=0)
    b = Basis(spec, r, w, phi, np.array(ls), np.array(epss), n_per_l, off)
    st_l, st_m, st_a = [], [], []
    for l in range(spec.l_max + 1):
        for m in range(-l, l + 1):
            for i in range(n_per_l[l]):
                st_l.append(l)
                st_m.append(m)
                st_a.append(off[l] + i)
    b.st_l = np.array(st_l)
    b.st_m = np.array(st_m)
    b.st_a = np.array(st_a)
    b.eps = b.rad_eps[b.st_a]
    return b
