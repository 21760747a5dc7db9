"""Write the stored oracle results used by the full-size GPU parity tests.

Every value here comes from ``oracle/`` only (FP64, numpy):

* ``c2_paths.npz``: the batched one-centre workload (N = 580, 4000-point
  grid, v = 1, z from -40 to 40 with dz = 0.1, all 800 RK4 steps) for three
  of its 32 impact parameters (the first, middle and last): final
  probabilities P_i = |X_i|^2.
* ``c4_paths.npz``: the seeded one-centre workload (the N = 580 basis, 64
  impact parameters drawn log-uniform in [0.05, 20] by default_rng(4), v = 1,
  all 800 RK4 steps) for four of its paths (the first, two inner and the
  last): final probabilities; the reference of the reduced-precision form.
* ``c3_couplings.npz``: the two-centre workload (v = 1) at one position on a
  path of the smallest basis pair (101 states per centre) and one on a path
  of the largest (382): 4096 seeded sampled elements of S and H (rows,
  columns, values) from the oracle's Eq. 1 blocks at 256 x 512 nodes.
* ``c3_path101.npz``: one path of the two-centre workload with 101 states
  per centre (b = 0.2 * 50^(3/7), v = 1, lower-left block in the prior form)
  over all 800 RK4 steps of z from -40 to 40 on 64 x 128 spheroidal nodes:
  final probabilities.
* ``c3_spot382.npz``: a path with 382 states per centre (b = 0.2 * 50^(3/7),
  v = 1) on the full 256 x 512 nodes, 4 RK4 steps from z = -0.2 through
  closest approach starting from the target ground state: final amplitudes.

Usage: python tests/golden/make_golden.py [c2] [c4] [c3] [c3p] [c3s]   (minutes of CPU each)
"""
from __future__ import annotations

import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle.propagate import probabilities, propagate_one_centre  # noqa: E402
from oracle.radial import BasisSpec, build_basis  # noqa: E402
from paper_2403_04252_amd import workloads as WL  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
C2_PATHS = [0, 15, 31]
C4_PATHS = [0, 21, 42, 63]
C3_POSITIONS = [(7, -2.35), (19, 0.65)]   # (path index, z): paths 0-7 have 101 states per centre, 16-23 have 382


def make_c2():
    w = WL.single_centre_batched()
    r = w.basis
    ob = build_basis(BasisSpec(r.n_max, r.l_max, r.n_bins, r.k_max, r.n_r, r.r_max, r.Z))
    P = []
    for j in C2_PATHS:
        t0 = time.time()
        X = propagate_one_centre(ob, float(w.b[j]), float(w.v[j]), w.zgrid)
        P.append(probabilities(X))
        print(f"c2 path {j} b={w.b[j]:.4g}: {time.time() - t0:.0f} s", flush=True)
    np.savez(os.path.join(HERE, "c2_paths.npz"), paths=np.array(C2_PATHS), b=w.b[C2_PATHS], P=np.array(P))


def make_c4():
    w = WL.single_centre_seeded()
    r = w.basis
    ob = build_basis(BasisSpec(r.n_max, r.l_max, r.n_bins, r.k_max, r.n_r, r.r_max, r.Z))
    P = []
    for j in C4_PATHS:
        t0 = time.time()
        X = propagate_one_centre(ob, float(w.b[j]), float(w.v[j]), w.zgrid)
        P.append(probabilities(X))
        print(f"c4 path {j} b={w.b[j]:.4g}: {time.time() - t0:.0f} s", flush=True)
    np.savez(os.path.join(HERE, "c4_paths.npz"), paths=np.array(C4_PATHS), b=w.b[C4_PATHS], P=np.array(P))


def make_c3():
    from oracle.twocentre import two_centre_matrices
    w = WL.two_centre_batched(1.0)
    rng = np.random.default_rng(7)
    out = {}
    for k, (j, z) in enumerate(C3_POSITIONS):
        rec = w.targets[w.set_of[j]]
        ob = build_basis(BasisSpec(rec.n_max, rec.l_max, rec.n_bins, rec.k_max, rec.n_r, rec.r_max, rec.Z))
        t0 = time.time()
        S, H = two_centre_matrices(ob, ob, float(w.b[j]), z, float(w.v[j]), w.n_eta, w.n_tau, w.q_lower)
        N = S.shape[0]
        rows = rng.integers(0, N, 4096)
        cols = rng.integers(0, N, 4096)
        out[f"path{k}"] = np.array([j])
        out[f"z{k}"] = np.array([z])
        out[f"rows{k}"] = rows
        out[f"cols{k}"] = cols
        out[f"S{k}"] = S[rows, cols]
        out[f"H{k}"] = H[rows, cols]
        out[f"Smax{k}"] = np.array([np.abs(S).max()])
        out[f"Hmax{k}"] = np.array([np.abs(H).max()])
        print(f"c3 path {j} z={z}: N={N}, {time.time() - t0:.0f} s", flush=True)
    np.savez(os.path.join(HERE, "c3_couplings.npz"), **out)


C3_PATH = 3          # of the 8 impact parameters of each basis size
C3_SPOT_Z = (-0.2, 0.2, 4)


def _c3_basis(l_max):
    rec = WL.Recipe(6, l_max, 20, 3.0, 4000)
    return build_basis(BasisSpec(rec.n_max, rec.l_max, rec.n_bins, rec.k_max, rec.n_r, rec.r_max, rec.Z))


def make_c3_path():
    from oracle.propagate import initial_state, rk4_propagate
    from oracle.twocentre import m_two_centre
    w = WL.two_centre_batched(1.0)
    j = C3_PATH           # basis set 0: 101 states per centre
    ob = _c3_basis(1)
    t0 = time.time()
    X = rk4_propagate(m_two_centre(ob, ob, float(w.b[j]), float(w.v[j]), 64, 128, w.q_lower),
                      initial_state(2 * ob.n_states), w.zgrid)
    print(f"c3 path {j} (101 + 101 states, 64 x 128 nodes, 800 steps): {time.time() - t0:.0f} s", flush=True)
    np.savez(os.path.join(HERE, "c3_path101.npz"), path=np.array([j]), b=w.b[[j]], n_eta=np.array([64]),
             n_tau=np.array([128]), P=probabilities(X), X=X)


def make_c3_spot():
    from oracle.propagate import initial_state, rk4_propagate
    from oracle.twocentre import m_two_centre
    w = WL.two_centre_batched(1.0)
    j = 16 + C3_PATH      # basis set 2: 382 states per centre
    ob = _c3_basis(3)
    X0 = initial_state(2 * ob.n_states)
    zg = np.linspace(C3_SPOT_Z[0], C3_SPOT_Z[1], C3_SPOT_Z[2] + 1)
    t0 = time.time()
    X = rk4_propagate(m_two_centre(ob, ob, float(w.b[j]), float(w.v[j]), w.n_eta, w.n_tau, w.q_lower), X0, zg)
    print(f"c3 spot path {j} (382 + 382 states, 256 x 512 nodes, 4 steps): {time.time() - t0:.0f} s", flush=True)
    np.savez(os.path.join(HERE, "c3_spot382.npz"), path=np.array([j]), b=w.b[[j]], zgrid=zg, X0=X0, X=X)


if __name__ == "__main__":
    which = sys.argv[1:] or ["c2", "c4", "c3"]
    if "c2" in which:
        make_c2()
    if "c4" in which:
        make_c4()
    if "c3" in which:
        make_c3()
    if "c3p" in which:
        make_c3_path()
    if "c3s" in which:
        make_c3_spot()
