"""GPU checks of the reduced-precision one-centre form (WPCCC_MIXED): the
moment tables of Eq. D2 stored in FP32 in scaled form, everything else FP64.

Bars
----
* couplings: |H_mixed - H_oracle| <= 1e-6 max|H| element-wise.  Each stored
  integral carries one FP32 rounding (2^-24 relative to the larger of its two
  scaled moments, both of the size of the integral); Eq. D1 sums at most
  l + l' + 1 of them per element with angular factors of modulus <= 1.
* probabilities: every |P_mixed - P_ref| <= 1e-6 absolute or <= 1e-4
  relative (the reduced-precision bar), against the FP64 oracle where it is
  run and against the FP64 GPU path (itself at 1e-10 of the oracle) for the
  paths the oracle is not run on.
"""
import numpy as np
import pytest
import torch

import paper_2403_04252_amd as W
from paper_2403_04252_amd import workloads as WL
from oracle.direct import direct_matrix
from oracle.propagate import probabilities, propagate_one_centre
from oracle.radial import BasisSpec as OSpec, build_basis

pytestmark = pytest.mark.gpu


def lib_basis(rec):
    return W.wpccc_basis(W.BasisSpec(rec.n_max, rec.l_max, rec.n_bins, rec.k_max, rec.n_r, rec.r_max, rec.Z))


def oracle_basis(rec):
    return build_basis(OSpec(rec.n_max, rec.l_max, rec.n_bins, rec.k_max, rec.n_r, rec.r_max, rec.Z))


def mixed_ok(P, Pref):
    d = np.abs(P - Pref)
    return (d <= 1e-6) | (d <= 1e-4 * np.abs(Pref))


def run(plan, zg):
    X = torch.zeros((plan.n_traj, plan.n_pad), dtype=torch.complex128, device="cuda")
    X[:, 0] = 1.0
    P = torch.zeros((plan.n_traj, plan.n_pad), dtype=torch.float64, device="cuda")
    W.wpccc_propagate(plan, zg, X, P)
    W.wpccc_plan_status(plan)
    torch.cuda.synchronize()
    return X.cpu().numpy()[:, :plan.n_states], P.cpu().numpy()[:, :plan.n_states]


@pytest.fixture(scope="module")
def small():
    rec = WL.single_centre_small().basis
    return rec, lib_basis(rec), oracle_basis(rec)


@pytest.fixture(scope="module")
def large():
    rec = WL.single_centre_batched().basis
    return rec, lib_basis(rec), oracle_basis(rec)


@pytest.mark.parametrize("which", ["small", "large"])
def test_mixed_couplings(which, request):
    rec, lb, ob = request.getfixturevalue(which)
    bs = [0.05, 1.0, 7.5, 150.0]
    zs = [-40.0, -0.05, 0.0, 1.234] if which == "small" else [-17.0, 0.0, 0.61]
    plan = W.wpccc_plan_create(lb, bs, 1.0, mixed=True)
    ref = W.wpccc_plan_create(lb, bs, 1.0)
    N = plan.n_states
    H = torch.empty((N, N), dtype=torch.complex128, device="cuda")
    H64 = torch.empty_like(H)
    worst = worst64 = 0.0
    for j, b in enumerate(bs):
        for z in zs:
            print(f"mixed couplings {which} b={b} z={z}", flush=True)
            W.wpccc_couplings(plan, j, z, H)
            W.wpccc_couplings(ref, j, z, H64)
            torch.cuda.synchronize()
            Ho = direct_matrix(ob, b, z, 1.0)
            scale = np.abs(Ho).max()
            err = np.abs(H.cpu().numpy() - Ho).max() / scale
            worst = max(worst, err)
            worst64 = max(worst64, np.abs(H64.cpu().numpy() - Ho).max() / scale)
            assert err <= 1e-6, (b, z, err)
    print(f"worst relative coupling error: mixed {worst:.2e}, FP64 {worst64:.2e}")
    assert worst > worst64   # the reduced form is in use


def test_mixed_full_single_path(small):
    """The N = 86 single-path workload, all 800 steps, against the oracle."""
    rec, lb, ob = small
    w = WL.single_centre_small()
    plan = W.wpccc_plan_create(lb, w.b, w.v, mixed=True)
    X, P = run(plan, w.zgrid)
    Po = probabilities(propagate_one_centre(ob, w.b[0], w.v[0], w.zgrid))
    d = np.abs(P[0] - Po)
    print(f"mixed N=86 full path: max|dP| {d.max():.2e}, max rel {(d / np.maximum(Po, 1e-300)).max():.2e}")
    assert mixed_ok(P[0], Po).all()


def test_mixed_tilings_and_graph(large):
    """Row tilings and graph replay of the mixed form: the same arithmetic up
    to the order of the final reductions (tilings), bitwise (graph)."""
    rec, lb, _ = large
    w = WL.reduced(WL.single_centre_batched(), n_paths=5, n_steps=130)
    outs = {}
    for rows in (4, 6, 8):
        plan = W.wpccc_plan_create(lb, w.b, w.v, stage_rows=rows, stage_launch=W.WPCCC_LAUNCH_STAGES, mixed=True)
        outs[rows] = run(plan, w.zgrid)[0]
    for rows in (4, 6):
        assert np.abs(outs[rows] - outs[8]).max() <= 1e-13
    gp = W.wpccc_plan_create(lb, w.b, w.v, stage_rows=8, stage_launch=W.WPCCC_LAUNCH_STAGES, graph=True, mixed=True)
    for rep in range(2):
        assert np.array_equal(run(gp, w.zgrid)[0], outs[8]), rep


def test_mixed_cache_forms(large):
    """The reduced-precision form with and without the radial-integral cache
    (FP32 F in the cache: one more rounding): both within the reduced-
    precision bar of the FP64 run over 150 steps of six paths."""
    rec, lb, _ = large
    w = WL.reduced(WL.single_centre_batched(), n_paths=6, n_steps=150)
    ref = run(W.wpccc_plan_create(lb, w.b, w.v, stage_rows=6, stage_launch=W.WPCCC_LAUNCH_STAGES), w.zgrid)[1]
    for c in (W.WPCCC_CACHE_ON, W.WPCCC_CACHE_OFF):
        plan = W.wpccc_plan_create(lb, w.b, w.v, stage_rows=6, stage_launch=W.WPCCC_LAUNCH_STAGES, mixed=True,
                                   stage_cache=c)
        P = run(plan, w.zgrid)[1]
        print(f"mixed cache {c}: max|dP| vs FP64 {np.abs(P - ref).max():.2e}", flush=True)
        assert mixed_ok(P, ref).all()


def test_mixed_refusals(small):
    rec, lb, _ = small
    with pytest.raises(W.WpcccError) as e:
        W.wpccc_plan_create(lb, [1.0], [1.0], mixed=True, stage_launch=W.WPCCC_LAUNCH_PERSISTENT)
    assert e.value.code == -6
    plan = W.wpccc_plan_create(lb, [1.0], [1.0], mixed=True)
    assert W.wpccc_plan_stage_launch(plan) == W.WPCCC_LAUNCH_STAGES
    zg = WL.z_uniform(-2.0, 2.0, 0.1)
    X0 = torch.zeros((1, plan.n_pad), dtype=torch.complex128, device="cuda")
    X0[:, 0] = 1.0
    grad = torch.empty((1, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(W.WpcccError) as e:
        W.wpccc_adjoint(plan, zg, X0, X0.clone(), grad)
    assert e.value.code == -6


@pytest.mark.parametrize("v", [0.5, 1.0, 2.0])
def test_mixed_two_centre_full_paths(v):
    """Two-centre reduced-precision form (FP32 contraction products) at the
    two-centre workload's quadrature (256 x 512 nodes) over all 800 steps of
    z from -40 to 40, from the target ground state, for two paths of the
    101-states-per-centre pair at each of the workload's speeds: every
    probability within the reduced-precision bar of the FP64 run."""
    rec = WL.Recipe(6, 1, 20, 3.0, 4000)
    lb = lib_basis(rec)
    b = np.array([0.2, 2.3])
    zg = WL.z_uniform(-40.0, 40.0, 0.1)
    out = {}
    for mixed in (False, True):
        print(f"2C full paths v={v} mixed={mixed}", flush=True)
        plan = W.wpccc_plan_create_2c([lb], [lb], [0, 0], b, v, q_lower=W.WPCCC_Q_PRIOR, n_eta=256, n_tau=512,
                                      mixed=mixed)
        out[mixed] = run(plan, zg)[1]
    d = np.abs(out[True] - out[False])
    print(f"  v={v}: max|dP| {d.max():.2e}, sum P {out[False].sum(axis=1)}", flush=True)
    assert mixed_ok(out[True], out[False]).all(), d.max()
