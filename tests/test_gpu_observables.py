"""Channel probabilities and cross sections on the GPU (wpccc_observables)
against the oracle's definitions applied to the same probabilities.

The GPU sums P per channel and integrates over b in a fixed order; the oracle
sums in index order and applies the trapezoidal rule in b order, so the two
agree to rounding: |d| <= 1e-14 of the total probability (channels) and of
the cross section of the total (cross sections).
"""
import numpy as np
import pytest
import torch

import paper_2403_04252_amd as W
from paper_2403_04252_amd import workloads as WL
from oracle import observables as O
from oracle.radial import BasisSpec as OSpec, build_basis

pytestmark = pytest.mark.gpu


def lib_basis(rec):
    return W.wpccc_basis(W.BasisSpec(rec.n_max, rec.l_max, rec.n_bins, rec.k_max, rec.n_r, rec.r_max, rec.Z))


def oracle_basis(rec):
    return build_basis(OSpec(rec.n_max, rec.l_max, rec.n_bins, rec.k_max, rec.n_r, rec.r_max, rec.Z))


def _observe(plan, zg):
    X = torch.zeros((plan.n_traj, plan.n_pad), dtype=torch.complex128, device="cuda")
    X[:, 0] = 1.0
    P = torch.zeros((plan.n_traj, plan.n_pad), dtype=torch.float64, device="cuda")
    W.wpccc_propagate(plan, zg, X, P)
    n_groups, group_of = W.wpccc_plan_groups(plan)
    chan = torch.full((plan.n_traj, W.WPCCC_N_CHANNELS), float("nan"), dtype=torch.float64, device="cuda")
    sigma = torch.full((n_groups, W.WPCCC_N_CHANNELS), float("nan"), dtype=torch.float64, device="cuda")
    W.wpccc_observables(plan, P, chan, sigma)
    torch.cuda.synchronize()
    W.wpccc_plan_status(plan)
    return P.cpu().numpy(), chan.cpu().numpy(), sigma.cpu().numpy(), group_of


def _check(P, chan, sigma, group_of, b, v, eps_of, n_of):
    for j in range(P.shape[0]):
        N = n_of(j)
        ref = O.channel_probabilities(P[j, :N], *eps_of(j))
        assert np.abs(chan[j] - ref).max() <= 1e-14 * ref[O.TOTAL], (j, chan[j], ref)
    for g in range(sigma.shape[0]):
        idx = np.nonzero(group_of == g)[0]
        assert np.unique(v[idx]).size == 1
        for c in range(W.WPCCC_N_CHANNELS):
            ref = O.cross_section(b[idx], chan[idx, c])
            scale = O.cross_section(b[idx], chan[idx, O.TOTAL])
            assert abs(sigma[g, c] - ref) <= 1e-14 * scale, (g, c, sigma[g, c], ref)


def test_observables_one_centre():
    rec = WL.single_centre_small().basis
    lb, ob = lib_basis(rec), oracle_basis(rec)
    b = np.array([2.0, 0.3, 1.1, 5.0, 0.7, 0.3])     # unsorted; the last path at another speed
    v = np.array([1.0, 1.0, 1.0, 1.0, 1.0, 2.0])
    plan = W.wpccc_plan_create(lb, b, v)
    P, chan, sigma, group_of = _observe(plan, WL.z_uniform(-6.0, 6.0, 0.1))
    assert list(group_of) == [0, 0, 0, 0, 0, 1]
    _check(P, chan, sigma, group_of, b, v, lambda j: (ob.eps,), lambda j: ob.n_states)
    assert np.all(chan[:, O.CAPTURE] == 0.0) and np.all(chan[:, O.PROJ_CONT] == 0.0)
    print("1C channels of path 1:", dict(zip(W.CHANNELS, chan[1].round(6))))


def test_observables_two_centre():
    wl = WL.two_centre_small()
    lt = [lib_basis(r) for r in wl.targets]
    lp = [lib_basis(r) for r in wl.projectiles]
    ot = [oracle_basis(r) for r in wl.targets]
    op = [oracle_basis(r) for r in wl.projectiles]
    plan = W.wpccc_plan_create_2c(lt, lp, wl.set_of, wl.b, wl.v, n_eta=wl.n_eta, n_tau=wl.n_tau,
                                  q_lower=W.WPCCC_Q_PRIOR)
    P, chan, sigma, group_of = _observe(plan, wl.zgrid)
    s = wl.set_of
    _check(P, chan, sigma, group_of, wl.b, wl.v,
           lambda j: (ot[s[j]].eps, op[s[j]].eps), lambda j: ot[s[j]].n_states + op[s[j]].n_states)
    assert np.all(chan[:, O.CAPTURE] > 0.0)
    print("2C channels:", chan.round(6))
