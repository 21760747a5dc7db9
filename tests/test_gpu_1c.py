"""GPU parity of the one-centre path against the FP64 oracle (through the C ABI).

Tolerances
----------
* couplings: element-wise |H_gpu - H_oracle| <= 1e-12 max|H|.  The two sides
  sum the same n_r quadrature terms in different orders (prefix moments vs a
  direct sum), which moves each element by a few units of n_r^(1/2) eps of
  the largest term.
* amplitudes after one step: |dX| <= 1e-13 (unit-norm X).
* probabilities after a whole path: |P_gpu - P_oracle| <= 1e-10 max(P, 1e-6),
  the 1e-10 relative target with a floor at P = 1e-6 (below it the
  amplitude rounding of ~1e-14 dominates any relative measure).
"""
import math

import numpy as np
import pytest
import torch

import paper_2403_04252_amd as W
from paper_2403_04252_amd import workloads as WL
from oracle.direct import direct_matrix
from oracle.propagate import (initial_state, m_one_centre, probabilities, propagate_one_centre,
                              rk4_propagate)
from oracle.radial import BasisSpec as OSpec, build_basis

pytestmark = pytest.mark.gpu

P_FLOOR = 1e-6


def lib_basis(rec):
    return W.wpccc_basis(W.BasisSpec(rec.n_max, rec.l_max, rec.n_bins, rec.k_max, rec.n_r, rec.r_max, rec.Z))


def oracle_basis(rec):
    return build_basis(OSpec(rec.n_max, rec.l_max, rec.n_bins, rec.k_max, rec.n_r, rec.r_max, rec.Z))


def prob_ok(P, Pref):
    return np.abs(P - Pref) <= 1e-10 * np.maximum(Pref, P_FLOOR)


@pytest.fixture(scope="module")
def small():
    rec = WL.single_centre_small().basis
    return rec, lib_basis(rec), oracle_basis(rec)


@pytest.fixture(scope="module")
def large():
    rec = WL.single_centre_batched().basis
    return rec, lib_basis(rec), oracle_basis(rec)


def test_device_present():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    print("device:", torch.cuda.get_device_name(0), flush=True)


@pytest.mark.parametrize("which", ["small", "large"])
def test_couplings_parity(which, request):
    rec, lb, ob = request.getfixturevalue(which)
    bs = [0.3, 1.0, 7.5] if which == "small" else [0.05, 2.4]
    zs = [-40.0, -3.3, -0.05, 0.0, 1.234, 40.0] if which == "small" else [-17.0, 0.0, 0.61]
    v = 1.0
    plan = W.wpccc_plan_create(lb, bs, v)
    N = plan.n_states
    H = torch.empty((N, N), dtype=torch.complex128, device="cuda")
    worst = 0.0
    for j, b in enumerate(bs):
        for z in zs:
            print(f"couplings {which} b={b} z={z}", flush=True)
            W.wpccc_couplings(plan, j, z, H)
            torch.cuda.synchronize()
            Hg = H.cpu().numpy()
            Ho = direct_matrix(ob, b, z, v)
            err = np.abs(Hg - Ho).max() / np.abs(Ho).max()
            worst = max(worst, err)
            assert err <= 1e-12, (b, z, err)
    print("worst relative coupling error", worst)


def test_couplings_outside_grid(small):
    rec, lb, ob = small
    plan = W.wpccc_plan_create(lb, [150.0], [1.3])
    N = plan.n_states
    H = torch.empty((N, N), dtype=torch.complex128, device="cuda")
    for z in (0.0, 90.0):
        W.wpccc_couplings(plan, 0, z, H)
        torch.cuda.synchronize()
        Ho = direct_matrix(ob, 150.0, z, 1.3)
        assert np.abs(H.cpu().numpy() - Ho).max() <= 1e-12 * np.abs(Ho).max()


def test_couplings_hermitian(large):
    rec, lb, ob = large
    plan = W.wpccc_plan_create(lb, [0.7], [1.0])
    N = plan.n_states
    H = torch.empty((N, N), dtype=torch.complex128, device="cuda")
    W.wpccc_couplings(plan, 0, -2.2, H)
    torch.cuda.synchronize()
    Hg = H.cpu().numpy()
    assert np.abs(Hg - Hg.conj().T).max() <= 1e-14 * np.abs(Hg).max()


def test_step_parity(small):
    rec, lb, ob = small
    bs, vs = [0.4, 1.0, 3.0], [1.0, 0.5, 2.0]
    plan = W.wpccc_plan_create(lb, bs, vs)
    N, npad = plan.n_states, plan.n_pad
    X0 = WL.random_state(3, N, seed=11)
    X = torch.zeros((3, npad), dtype=torch.complex128, device="cuda")
    X[:, :N] = torch.from_numpy(X0).cuda()
    z, h = -0.37, 0.1
    W.wpccc_step(plan, X, z, h)
    torch.cuda.synchronize()
    Xg = X.cpu().numpy()[:, :N]
    for j in range(3):
        Xo = rk4_propagate(m_one_centre(ob, bs[j], vs[j]), X0[j], np.array([z, z + h]))
        assert np.abs(Xg[j] - Xo).max() <= 1e-13, (j, np.abs(Xg[j] - Xo).max())


def _propagate_gpu(lb, b, v, zgrid, Zp=1.0, batched=True, stage_rows=0):
    plan = W.wpccc_plan_create(lb, b, v, Zp=Zp, batched=batched, stage_rows=stage_rows)
    X = torch.zeros((plan.n_traj, plan.n_pad), dtype=torch.complex128, device="cuda")
    X[:, 0] = 1.0
    P = torch.zeros((plan.n_traj, plan.n_pad), dtype=torch.float64, device="cuda")
    nrm = torch.zeros(plan.n_traj, dtype=torch.float64, device="cuda")
    W.wpccc_propagate(plan, zgrid, X, P, nrm)
    W.wpccc_plan_status(plan)
    torch.cuda.synchronize()
    N = plan.n_states
    return X.cpu().numpy()[:, :N], P.cpu().numpy()[:, :N], nrm.cpu().numpy()


def test_propagate_single_path_full(small):
    """The N = 86 single-path workload, all 800 steps, against the oracle."""
    rec, lb, ob = small
    w = WL.single_centre_small()
    print("propagate N=86 full path on GPU", flush=True)
    X, P, nrm = _propagate_gpu(lb, w.b, w.v, w.zgrid)
    print("oracle", flush=True)
    Xo = propagate_one_centre(ob, w.b[0], w.v[0], w.zgrid)
    Po = probabilities(Xo)
    ok = prob_ok(P[0], Po)
    print("max |dP|", np.abs(P[0] - Po).max(), "max |dX|", np.abs(X[0] - Xo).max())
    assert ok.all(), np.abs(P[0] - Po).max()
    assert abs(nrm[0] - P[0].sum()) < 1e-13
    assert abs(nrm[0] - 1.0) < 1e-4


def test_propagate_large_basis_reduced(large):
    """N = 580 basis, two paths, the first 40 steps."""
    rec, lb, ob = large
    w = WL.reduced(WL.single_centre_batched(), n_paths=2, n_steps=40)
    X, P, _ = _propagate_gpu(lb, w.b, w.v, w.zgrid)
    for j in range(2):
        Xo = propagate_one_centre(ob, w.b[j], w.v[j], w.zgrid)
        assert np.abs(X[j] - Xo).max() <= 1e-12
        assert prob_ok(P[j], probabilities(Xo)).all()


def test_batched_equals_sequential(small):
    rec, lb, ob = small
    b = [0.2, 0.9, 2.5, 6.0]
    zg = WL.z_uniform(-10.0, 5.0, 0.1)
    # the same stage tiling for both (the timed choice may differ between plans)
    Xb, Pb, _ = _propagate_gpu(lb, b, 1.0, zg, batched=True, stage_rows=8)
    Xs, Ps, _ = _propagate_gpu(lb, b, 1.0, zg, batched=False, stage_rows=8)
    assert np.array_equal(Xb, Xs)


def test_negative_projectile(small):
    rec, lb, ob = small
    zg = WL.z_uniform(-15.0, 15.0, 0.1)
    X, P, _ = _propagate_gpu(lb, [1.2], 1.0, zg, Zp=-1.0)
    Xo = propagate_one_centre(ob, 1.2, 1.0, zg, Zp=-1.0)
    assert prob_ok(P[0], probabilities(Xo)).all()


def test_geometric_grid(small):
    """The paper's geometric z-grid (z_min = 1e-3, z_max = 20, n_z = 60)."""
    rec, lb, ob = small
    zg = WL.z_geometric(1e-3, 20.0, 60)
    X, P, _ = _propagate_gpu(lb, [0.8], 1.5, zg)
    Xo = propagate_one_centre(ob, 0.8, 1.5, zg)
    assert prob_ok(P[0], probabilities(Xo)).all()


def test_single_step_grid_and_errors(small):
    rec, lb, ob = small
    zg = np.array([-1.0, -0.9])
    X, P, _ = _propagate_gpu(lb, [1.0], 1.0, zg)
    Xo = propagate_one_centre(ob, 1.0, 1.0, zg)
    assert np.abs(X[0] - Xo).max() <= 1e-14
    plan = W.wpccc_plan_create(lb, [1.0], [1.0])
    Xd = torch.zeros((1, plan.n_pad), dtype=torch.complex128, device="cuda")
    with pytest.raises(W.WpcccError) as e1:
        W.wpccc_propagate(plan, np.array([0.0, 0.0]), Xd)
    assert e1.value.code == -1
    with pytest.raises(W.WpcccError) as e2:
        W.wpccc_step(plan, Xd, 0.0, 0.0)
    assert e2.value.code == -1
    H = torch.empty((plan.n_states, plan.n_states), dtype=torch.complex128, device="cuda")
    with pytest.raises(W.WpcccError) as e3:
        W.wpccc_couplings(plan, 1, 0.0, H)
    assert e3.value.code == -1
    with pytest.raises(W.WpcccError) as e4:
        W.wpccc_plan_create(lb, [0.0], [1.0])
    assert e4.value.code == -1


def test_stage_rows_variants_agree(large):
    """k_stage with 4, 5, 6, 7, 8, 10, 12 or 16 output rows per workgroup (and
    the timed choice) runs the same arithmetic per output up to the order of
    its final reduction: results agree to rounding."""
    rec, lb, _ = large
    w = WL.reduced(WL.single_centre_batched(), n_paths=5, n_steps=10)
    outs = {}
    for rows in (4, 5, 6, 7, 8, 10, 12, 16, 0):
        print(f"stage rows {rows}", flush=True)
        plan = W.wpccc_plan_create(lb, w.b, w.v, stage_rows=rows, stage_launch=W.WPCCC_LAUNCH_STAGES)
        if rows:
            assert W.wpccc_plan_stage_rows(plan) == rows
        else:
            assert W.wpccc_plan_stage_rows(plan) in (4, 5, 6, 7, 8, 10, 12, 16)
        assert W.wpccc_plan_stage_launch(plan) == W.WPCCC_LAUNCH_STAGES
        X = torch.zeros((plan.n_traj, plan.n_pad), dtype=torch.complex128, device="cuda")
        X[:, 0] = 1.0
        W.wpccc_propagate(plan, w.zgrid, X)
        torch.cuda.synchronize()
        outs[rows] = X.cpu().numpy()
    for rows in (4, 5, 6, 7, 10, 12, 16, 0):
        assert np.abs(outs[rows] - outs[8]).max() <= 1e-13


def test_large_l_basis_parity():
    """l_max = 6 (multipoles to 12, Pbar_12^mu, 13 values of m' per output
    row, angular factors of 13 x 252 per l' block): two paths, 10 steps,
    against the oracle.  Larger l_max is refused with WPCCC_ENOTSUP: the
    angular factors of the largest l' block (21 x 946 at l_max = 10) no
    longer fit the stage workgroup's LDS."""
    rec = WL.Recipe(2, 6, 1, 2.0, 300, 60.0)
    lb, ob = lib_basis(rec), oracle_basis(rec)
    w = WL.reduced(WL.single_centre_batched(), n_paths=2, n_steps=10)
    print("l_max = 6 basis, 2 paths x 10 steps", flush=True)
    X, P, _ = _propagate_gpu(lb, w.b, w.v, w.zgrid)
    for j in range(2):
        Xo = propagate_one_centre(ob, w.b[j], w.v[j], w.zgrid)
        assert np.abs(X[j] - Xo).max() <= 1e-12, (j, np.abs(X[j] - Xo).max())
        assert prob_ok(P[j], probabilities(Xo)).all()
    # l_max = 10: no regular tiling fits the LDS, the large-basis form is
    # used (tilings of 1, 2 or 4 rows only)
    big = lib_basis(WL.Recipe(2, 10, 1, 2.0, 300, 60.0))
    assert W.wpccc_plan_stage_rows(W.wpccc_plan_create(big, [1.0], [1.0])) in (1, 2, 4)
    with pytest.raises(W.WpcccError) as e:
        W.wpccc_plan_create(big, [1.0], [1.0], stage_rows=8)
    assert e.value.code == -6


@pytest.mark.parametrize("l_max,n_states,n_steps", [(6, 1855, 6), (7, 2380, 3)])
def test_paper_shape_smaller_tiles(l_max, n_states, n_steps):
    """The paper's basis shape at l_max = 6 and 7 (N_l = 42 - l radial
    functions per l, N = 1855 and 2380, the largest the stage kernel takes):
    a stage tile of 8 rows no longer fits the LDS, so the plan times the
    smaller tilings that do (the adjoint's operator kernel takes 4 rows here,
    tested in the adjoint tests).  One path against the oracle; 8 rows
    explicitly are refused with WPCCC_ENOTSUP; every admissible smaller
    tiling agrees with the timed one to rounding (the order of the final
    reductions differs)."""
    rec = WL.Recipe(10, l_max, 32, 3.0, 300, 100.0)
    lb, ob = lib_basis(rec), oracle_basis(rec)
    zg = np.linspace(-3.0, -3.0 + 0.1 * n_steps, n_steps + 1)
    print(f"paper shape l_max = {l_max} (N = {n_states}), 1 path x {n_steps} steps", flush=True)
    plan = W.wpccc_plan_create(lb, [1.5], [2.0])
    assert plan.n_states == n_states
    rows = W.wpccc_plan_stage_rows(plan)
    print(f"  timed tiling: {rows} rows", flush=True)
    assert rows < 8
    X, P, _ = _propagate_gpu(lb, [1.5], [2.0], zg)
    Xo = propagate_one_centre(ob, 1.5, 2.0, zg)
    assert np.abs(X[0] - Xo).max() <= 1e-12, np.abs(X[0] - Xo).max()
    assert prob_ok(P[0], probabilities(Xo)).all()
    with pytest.raises(W.WpcccError) as e:
        W.wpccc_plan_create(lb, [1.5], [2.0], stage_rows=8)
    assert e.value.code == -6
    for r in (4, 5, 6, 7):
        if r == rows:
            continue
        try:
            Xr, _, _ = _propagate_gpu(lb, [1.5], [2.0], zg, stage_rows=r)
        except W.WpcccError as err:
            assert err.code in (-1, -6), str(err)   # does not fit this basis
            continue
        print(f"  tiling {r} rows vs timed: {np.abs(Xr - X).max():.1e}", flush=True)
        assert np.abs(Xr - X).max() <= 1e-13


def test_nonfinite_amplitude_latched(small):
    """A non-finite input amplitude propagates to the RK4 update, whose
    watchdog latches WPCCC_ENUMERIC for wpccc_plan_status (no device fault,
    every kernel ends normally); the latch clears after it is read."""
    rec, lb, _ = small
    plan = W.wpccc_plan_create(lb, [1.0, 2.0], [1.0, 1.0])
    X = torch.zeros((2, plan.n_pad), dtype=torch.complex128, device="cuda")
    X[:, 0] = 1.0
    X[1, 3] = float("nan")
    W.wpccc_propagate(plan, WL.z_uniform(-2.0, 2.0, 0.1), X)
    with pytest.raises(W.WpcccError) as e:
        W.wpccc_plan_status(plan)
    assert e.value.code == -5
    W.wpccc_plan_status(plan)   # cleared
    assert torch.isfinite(X[0]).all()


def test_smem_limit_only_raised():
    """The dynamic-LDS limit of the stage kernels is process-wide: a plan with
    a smaller basis created after a larger one must not lower it under the
    larger plan, which propagates correctly afterwards."""
    big = WL.Recipe(10, 6, 32, 3.0, 300, 100.0)
    lbig = lib_basis(big)
    zg = np.linspace(-3.0, -2.8, 3)
    ref, _, _ = _propagate_gpu(lbig, [1.5], [2.0], zg, stage_rows=4)
    mid = lib_basis(WL.Recipe(6, 4, 20, 3.0, 300, 100.0))
    pmid = W.wpccc_plan_create(mid, [1.0], [1.0], stage_rows=4)
    assert pmid.n_states == 580
    again, _, _ = _propagate_gpu(lbig, [1.5], [2.0], zg, stage_rows=4)
    assert np.array_equal(again, ref)


def test_stage_rows_limit():
    """Every output of a stage workgroup needs a lane of the phase-3
    reduction: rows x (2 l_max + 1) <= 256, so 16 rows are refused for
    l_max = 8 while the timed choice stays within the limit."""
    lb = lib_basis(WL.Recipe(2, 8, 1, 2.0, 300, 60.0))
    with pytest.raises(W.WpcccError) as e:
        W.wpccc_plan_create(lb, [1.0], [1.0], stage_rows=16)
    assert e.value.code == -1
    plan = W.wpccc_plan_create(lb, [1.0, 2.0], [1.0, 1.0])
    assert W.wpccc_plan_stage_rows(plan) * 17 <= 256


def _run_plan(plan, zg):
    X = torch.zeros((plan.n_traj, plan.n_pad), dtype=torch.complex128, device="cuda")
    X[:, 0] = 1.0
    W.wpccc_propagate(plan, zg, X)
    torch.cuda.synchronize()
    W.wpccc_plan_status(plan)
    return X.cpu().numpy()


def test_persistent_chunk_matches_stages(large):
    """The persistent chunk kernel (all workgroups resident for a 64-step
    chunk, per-path barriers between stages) runs the stage kernel's
    arithmetic: bitwise the kernel-by-kernel result, for all 32 paths of the
    N = 580 batch over 2 full chunks and a ragged one, for every row tiling
    whose grid fits, and for one path per launch (batched = 0)."""
    rec, lb, _ = large
    w = WL.reduced(WL.single_centre_batched(), n_steps=150)
    assert w.b.size == 32
    fitted = []
    for rows in (10, 12, 16, 8):
        print(f"persistent vs stages, 32 paths x 150 steps, rows {rows}", flush=True)
        try:
            pp = W.wpccc_plan_create(lb, w.b, w.v, stage_rows=rows, stage_launch=W.WPCCC_LAUNCH_PERSISTENT)
        except W.WpcccError as e:
            assert e.code == -6, str(e)   # grid larger than what can be resident at once
            print(f"  rows {rows}: {e}", flush=True)
            continue
        fitted.append(rows)
        assert W.wpccc_plan_stage_launch(pp) == W.WPCCC_LAUNCH_PERSISTENT
        ps = W.wpccc_plan_create(lb, w.b, w.v, stage_rows=rows, stage_launch=W.WPCCC_LAUNCH_STAGES)
        Xp, Xs = _run_plan(pp, w.zgrid), _run_plan(ps, w.zgrid)
        assert np.array_equal(Xp, Xs), (rows, np.abs(Xp - Xs).max())
        # a second call on the same plan (barrier counters start again from zero)
        assert np.array_equal(_run_plan(pp, w.zgrid[:70]), _run_plan(ps, w.zgrid[:70]))
    assert 10 in fitted
    # one path per launch sequence
    sub = WL.reduced(WL.single_centre_batched(), n_paths=3, n_steps=70)
    pp = W.wpccc_plan_create(lb, sub.b, sub.v, batched=False, stage_rows=8,
                             stage_launch=W.WPCCC_LAUNCH_PERSISTENT)
    ps = W.wpccc_plan_create(lb, sub.b, sub.v, stage_rows=8, stage_launch=W.WPCCC_LAUNCH_STAGES)
    assert np.array_equal(_run_plan(pp, sub.zgrid), _run_plan(ps, sub.zgrid))


def test_timed_launch_choice_is_valid(large):
    """The default plan times both launch forms and keeps one; either gives the
    kernel-by-kernel amplitudes of its row tiling bitwise."""
    rec, lb, _ = large
    w = WL.reduced(WL.single_centre_batched(), n_steps=70)
    auto = W.wpccc_plan_create(lb, w.b, w.v)
    rows, launch = W.wpccc_plan_stage_rows(auto), W.wpccc_plan_stage_launch(auto)
    print(f"timed choice: rows {rows}, launch {launch}", flush=True)
    assert launch in (W.WPCCC_LAUNCH_STAGES, W.WPCCC_LAUNCH_PERSISTENT)
    ref = W.wpccc_plan_create(lb, w.b, w.v, stage_rows=rows, stage_launch=W.WPCCC_LAUNCH_STAGES)
    assert np.array_equal(_run_plan(auto, w.zgrid), _run_plan(ref, w.zgrid))


def test_graph_replay_matches_eager(large):
    """wpccc_propagate replaying a captured 64-step graph (positions and step
    lengths from device memory) gives the kernel-by-kernel result bitwise, on
    every call, with eager work and synchronisation between the calls."""
    rec, lb, _ = large
    w = WL.reduced(WL.single_centre_batched(), n_paths=5, n_steps=200)   # 3 full chunks + 8 steps
    zg = w.zgrid
    eager = W.wpccc_plan_create(lb, w.b, w.v, stage_rows=8)
    graph = W.wpccc_plan_create(lb, w.b, w.v, stage_rows=8, graph=True)

    def run(plan, z):
        X = torch.zeros((plan.n_traj, plan.n_pad), dtype=torch.complex128, device="cuda")
        X[:, 0] = 1.0
        W.wpccc_propagate(plan, z, X)
        torch.cuda.synchronize()
        return X

    ref = run(eager, zg).cpu().numpy()
    Xg = torch.zeros((graph.n_traj, graph.n_pad), dtype=torch.complex128, device="cuda")
    for rep in range(3):
        print(f"graph replay call {rep}", flush=True)
        Xg.zero_()
        Xg[:, 0] = 1.0
        W.wpccc_propagate(graph, zg, Xg)
        torch.cuda.synchronize()
        assert np.array_equal(Xg.cpu().numpy(), ref), rep
        # eager work in between, on the same stream
        other = run(eager, zg[:20])
        assert other.abs().sum().item() > 0
    # a different grid (geometric step lengths) through the same graph
    zg2 = np.concatenate([zg[:1], zg[0] + np.cumsum(np.linspace(0.05, 0.15, 150))])
    ref2 = run(eager, zg2).cpu().numpy()
    Xg.zero_()
    Xg[:, 0] = 1.0
    W.wpccc_propagate(graph, zg2, Xg)
    torch.cuda.synchronize()
    assert np.array_equal(Xg.cpu().numpy(), ref2)


def test_interpolated_radial_form(small):
    """The paper's production form of the radial integrals (F on the grid
    nodes, five-point interpolation at R, multipole form beyond the grid):
    couplings element-wise and a 200-step path against the oracle's
    interpolated form at the FP64 bars; it differs from the exact-R form by
    the interpolation error only."""
    rec, lb, ob = small
    bs = [0.3, 1.0, 150.0]
    plan = W.wpccc_plan_create(lb, bs, 1.0, interp=True)
    N = plan.n_states
    H = torch.empty((N, N), dtype=torch.complex128, device="cuda")
    for j, b in enumerate(bs):
        for z in (-30.0, -0.05, 0.0, 1.234):
            W.wpccc_couplings(plan, j, z, H)
            torch.cuda.synchronize()
            Ho = direct_matrix(ob, b, z, 1.0, radial="interp")
            err = np.abs(H.cpu().numpy() - Ho).max() / np.abs(Ho).max()
            assert err <= 1e-12, (b, z, err)
    zg = WL.z_uniform(-10.0, 10.0, 0.1)
    pi = W.wpccc_plan_create(lb, [1.0], [1.0], interp=True)
    X = torch.zeros((1, pi.n_pad), dtype=torch.complex128, device="cuda")
    X[:, 0] = 1.0
    W.wpccc_propagate(pi, zg, X)
    W.wpccc_plan_status(pi)
    Pg = (X.abs() ** 2).cpu().numpy()[0, :N]
    Po = probabilities(propagate_one_centre(ob, 1.0, 1.0, zg, radial="interp"))
    assert prob_ok(Pg, Po).all(), np.abs(Pg - Po).max()
    _, Pe, _ = _propagate_gpu(lb, [1.0], [1.0], zg)
    d = np.abs(Pg - Pe[0]).max()
    print(f"interpolated vs exact-R F over 200 steps: max|dP| {d:.2e}", flush=True)
    assert 0.0 < d < 1e-3
    with pytest.raises(W.WpcccError) as e:
        W.wpccc_plan_create(lb, [1.0], [1.0], interp=True, mixed=True)
    assert e.value.code == -6


@pytest.mark.parametrize("l_max,n_states", [(8, 2958), (10, 4257)])
def test_paper_shape_large_basis_form(l_max, n_states):
    """The paper's one-centre basis shape beyond l_max = 7 (N_l = 42 - l; at
    l_max = 10, N = 4257, the largest one-centre system of the paper's
    scaling runs): no tiling of the stage kernel fits the LDS with the
    angular factors staged there, so the plan reads them from global memory
    (1, 2 or 4 rows per workgroup).  Two paths, 2 steps, against the oracle
    on a 300-point grid."""
    rec = WL.Recipe(10, l_max, 32, 3.0, 300, 100.0)
    lb, ob = lib_basis(rec), oracle_basis(rec)
    zg = np.array([-3.0, -2.9, -2.8])
    bs, vs = [1.5, 4.0], [2.0, 2.0]
    print(f"paper shape l_max = {l_max} (N = {n_states}), large-basis form", flush=True)
    X, P, _ = _propagate_gpu(lb, bs, vs, zg)
    assert X.shape[1] == n_states
    for j in range(2):
        Xo = propagate_one_centre(ob, bs[j], vs[j], zg)
        err = np.abs(X[j] - Xo).max()
        print(f"  path {j}: max|dX| {err:.2e}", flush=True)
        assert err <= 1e-12
        assert prob_ok(P[j], probabilities(Xo)).all()
    with pytest.raises(W.WpcccError) as e:
        W.wpccc_plan_create(lb, [1.0], [1.0], stage_launch=W.WPCCC_LAUNCH_PERSISTENT)
    assert e.value.code == -6


def test_stage_cache_forms_bitwise(large):
    """Stage kernels with the radial-integral cache (F formed at the two new
    points of a step and read back) and without it (F formed from the moment
    table in every stage) run the same arithmetic: bitwise the same
    amplitudes over two chunks and a ragged one; the timed choice is one of
    the two; the forms that need the cache refuse WPCCC_CACHE_OFF."""
    rec, lb, _ = large
    w = WL.reduced(WL.single_centre_batched(), n_paths=6, n_steps=150)
    outs = {}
    for c in (W.WPCCC_CACHE_ON, W.WPCCC_CACHE_OFF):
        plan = W.wpccc_plan_create(lb, w.b, w.v, stage_rows=6, stage_launch=W.WPCCC_LAUNCH_STAGES, stage_cache=c)
        assert W.wpccc_plan_stage_cache(plan) == (c == W.WPCCC_CACHE_ON)
        outs[c] = _run_plan(plan, w.zgrid)
    assert np.array_equal(outs[W.WPCCC_CACHE_ON], outs[W.WPCCC_CACHE_OFF])
    auto = W.wpccc_plan_create(lb, w.b, w.v)
    print("timed choice: rows", W.wpccc_plan_stage_rows(auto), "cache", W.wpccc_plan_stage_cache(auto), flush=True)
    with pytest.raises(W.WpcccError) as e:
        W.wpccc_plan_create(lb, w.b, w.v, interp=True, stage_cache=W.WPCCC_CACHE_OFF)
    assert e.value.code == -6
