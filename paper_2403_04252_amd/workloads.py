"""Seeded synthetic workloads (inputs only: basis recipes, impact parameters,
speeds and z-grids).  No coupling, solver or propagation arithmetic lives here;
both the HIP library and the oracle receive these plain values.

The shapes follow the paper's proton + hydrogen workload: bound hydrogen
states plus Coulomb wave-packet bins per l (all m), an r-grid to 100 a.u.,
straight-line paths at fixed v, batched over impact parameters b.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class Recipe:
    n_max: int
    l_max: int
    n_bins: int
    k_max: float
    n_r: int
    r_max: float = 100.0
    Z: float = 1.0


@dataclass
class Workload:
    name: str
    description: str
    basis: Recipe
    b: np.ndarray
    v: np.ndarray
    zgrid: np.ndarray
    extra: dict = field(default_factory=dict)

    @property
    def n_steps(self) -> int:
        return int(self.zgrid.size - 1)


def z_uniform(z0: float, z1: float, dz: float) -> np.ndarray:
    n = int(round((z1 - z0) / dz))
    return np.linspace(z0, z1, n + 1)


def z_geometric(z_min: float, z_max: float, n_z: int) -> np.ndarray:
    """zgrid[i] = z_min (z_max/z_min)^(i/n_z), zgrid[0] = 0, zgrid[-i] = -zgrid[i]."""
    pos = z_min * (z_max / z_min) ** (np.arange(1, n_z + 1) / n_z)
    return np.concatenate([-pos[::-1], [0.0], pos])


def single_centre_small() -> Workload:
    """n <= 3 bound + 8 bins/l, l <= 2 (N = 86), 1500-point grid; one path b = 1,
    v = 1, z from -40 to 40 with dz = 0.1 (800 RK4 steps)."""
    return Workload("p+H 1C N=86 b=1 v=1", "single-centre, FP64, one path",
                    Recipe(3, 2, 8, 3.0, 1500), np.array([1.0]), np.array([1.0]),
                    z_uniform(-40.0, 40.0, 0.1))


def single_centre_batched() -> Workload:
    """n <= 6 bound + 20 bins/l, l <= 4 (N = 580), 4000-point grid; 32 paths with
    b log-spaced 0.05..20, v = 1, z from -40 to 40 with dz = 0.1."""
    j = np.arange(32)
    b = 0.05 * 400.0 ** (j / 31.0)
    return Workload("p+H 1C N=580 x32 b", "single-centre, FP64, 32 paths in one batch",
                    Recipe(6, 4, 20, 3.0, 4000), b, np.ones(32), z_uniform(-40.0, 40.0, 0.1))


def single_centre_seeded(n_paths: int = 64, seed: int = 4) -> Workload:
    """The N = 580 basis with b drawn log-uniform in [0.05, 20] (numpy default_rng(seed)), sorted."""
    rng = np.random.default_rng(seed)
    b = np.sort(np.exp(rng.uniform(np.log(0.05), np.log(20.0), n_paths)))
    return Workload(f"p+H 1C N=580 x{n_paths} seeded b", "single-centre, seeded impact parameters",
                    Recipe(6, 4, 20, 3.0, 4000), b, np.ones(n_paths), z_uniform(-40.0, 40.0, 0.1))


def reduced(w: Workload, n_paths: int | None = None, n_steps: int | None = None,
            n_r: int | None = None) -> Workload:
    """A cheaper cut of a workload for oracle comparisons: the first n_steps steps
    of the z-grid, a spread subset of the paths, or a coarser grid."""
    b, v, z = w.b, w.v, w.zgrid
    if n_paths is not None and n_paths < b.size:
        idx = np.unique(np.linspace(0, b.size - 1, n_paths).round().astype(int))
        b, v = b[idx], v[idx]
    if n_steps is not None:
        z = z[: n_steps + 1]
    rec = w.basis
    if n_r is not None:
        rec = Recipe(rec.n_max, rec.l_max, rec.n_bins, rec.k_max, n_r, rec.r_max, rec.Z)
    return Workload(w.name + " (reduced)", w.description, rec, b.copy(), v.copy(), z.copy())


def random_state(n_paths: int, n_states: int, seed: int) -> np.ndarray:
    """A normalised random complex amplitude vector per path (for single-step checks)."""
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n_paths, n_states)) + 1j * rng.standard_normal((n_paths, n_states))
    return X / np.linalg.norm(X, axis=1, keepdims=True)


@dataclass
class TwoCentreWorkload:
    """Paths of a two-centre batch: path j expands in the basis pair
    (targets[set_of[j]], projectiles[set_of[j]])."""
    name: str
    description: str
    targets: list
    projectiles: list
    set_of: np.ndarray
    b: np.ndarray
    v: np.ndarray
    zgrid: np.ndarray
    n_eta: int = 256
    n_tau: int = 512
    q_lower: str = "prior"   # lower-left block of H: "prior" or "dagger" (Q^dagger as printed)

    @property
    def n_steps(self) -> int:
        return int(self.zgrid.size - 1)


def two_centre_batched(v: float = 1.0) -> TwoCentreWorkload:
    """p + H with capture, the same recipe on both centres (bound n <= 6 plus 20
    Coulomb bins per l, 4000-point grid) at three sizes, l <= 1, 2, 3: 101, 221
    and 382 states per centre (N = 202, 442, 764).  8 impact parameters b
    log-spaced 0.2..10 for each size, 24 paths in one batch at speed v (0.5, 1
    or 2 a.u.), 256 x 512 spheroidal nodes, z from -40 to 40 with dz = 0.1."""
    recs = [Recipe(6, l, 20, 3.0, 4000) for l in (1, 2, 3)]
    k = np.arange(24) % 8
    s = np.arange(24) // 8
    b = 0.2 * 50.0 ** (k / 7.0)
    return TwoCentreWorkload(f"p+H 2C N=202/442/764 x24 b v={v:g}", "two-centre with capture, FP64, uneven bases",
                             recs, recs, s.astype(np.int32), b, np.full(24, float(v)), z_uniform(-40.0, 40.0, 0.1))


def two_centre_small() -> TwoCentreWorkload:
    """A two-centre batch the oracle finishes in seconds: target bound n <= 2 plus
    one bin (l <= 1) or n <= 3 plus one bin (l <= 2), projectile n <= 2 plus two
    bins (l <= 1), 600-point grid to 40 a.u.; three paths (b = 0.8, 1.5, 3, v = 0.5,
    1, 2), 24 x 32 nodes, z from -4 to 4 with dz = 0.5."""
    t0 = Recipe(2, 1, 1, 1.5, 600, 40.0)
    t1 = Recipe(3, 2, 1, 1.5, 600, 40.0)
    p0 = Recipe(2, 1, 2, 1.5, 600, 40.0)
    return TwoCentreWorkload("p+H 2C small", "two-centre, FP64, oracle-sized",
                             [t0, t1], [p0, p0], np.array([0, 1, 0], dtype=np.int32),
                             np.array([0.8, 1.5, 3.0]), np.array([0.5, 1.0, 2.0]),
                             z_uniform(-4.0, 4.0, 0.5), n_eta=24, n_tau=32)


@dataclass
class AdjointWorkload:
    """Screened-potential gradients: one (a, c) for the batch, paths b, loss weights."""
    name: str
    basis: Recipe
    a: float
    c: float
    b: np.ndarray
    v: np.ndarray
    weights: np.ndarray
    zgrid: np.ndarray


def adjoint_batch(n_states: int = 86) -> AdjointWorkload:
    """The N = 86 single-path basis with the screened potential -(1 + a e^{-c r})/r:
    numpy default_rng(5) draws a ~ U[0.2, 1.0], c ~ U[0.5, 2.0], 16 b log-uniform
    in [0.3, 8] (sorted) and the loss weights w_i ~ U[0, 1], in that order;
    v = 1, z from -40 to 40 with dz = 0.1."""
    rng = np.random.default_rng(5)
    a = float(rng.uniform(0.2, 1.0))
    c = float(rng.uniform(0.5, 2.0))
    b = np.sort(np.exp(rng.uniform(np.log(0.3), np.log(8.0), 16)))
    w = rng.uniform(0.0, 1.0, n_states)
    return AdjointWorkload("p+H 1C N=86 screened potential x16 b", Recipe(3, 2, 8, 3.0, 1500), a, c, b,
                           np.ones(16), w, z_uniform(-40.0, 40.0, 0.1))
