"""The allocation-free couplings entry point (wpccc_couplings_noalloc) against
wpccc_couplings, through the C ABI.

Both run the same two kernels on the same inputs, so the dense couplings must
agree bit for bit (integer-exact comparison of the FP64 words).  Two calls in a
row on the shared per-device scratch array, the second on a smaller basis
(fewer radial integrals, angular factors and phases than the first left
behind), show that a call reads nothing the previous one wrote.  A two-centre
plan is refused with WPCCC_ENOTSUP.  The dense matrix is also checked against
the oracle on the small basis, so the comparison is not between two equal
wrong answers.
"""
import numpy as np
import pytest
import torch

import paper_2403_04252_amd as W
from paper_2403_04252_amd import workloads as WL
from oracle.direct import direct_matrix
from oracle.radial import BasisSpec as OSpec, build_basis

pytestmark = pytest.mark.gpu


def lib_basis(rec):
    return W.wpccc_basis(W.BasisSpec(rec.n_max, rec.l_max, rec.n_bins, rec.k_max, rec.n_r, rec.r_max, rec.Z))


def _pair(plan, j, z):
    N = plan.n_states
    Ha = torch.full((N, N), float("nan"), dtype=torch.complex128, device="cuda")
    Hb = torch.full((N, N), float("nan"), dtype=torch.complex128, device="cuda")
    W.wpccc_couplings_noalloc(plan, j, z, Hb)
    W.wpccc_couplings(plan, j, z, Ha)
    torch.cuda.synchronize()
    return Ha.cpu().numpy(), Hb.cpu().numpy()


def test_noalloc_matches_couplings_twice():
    big = WL.single_centre_batched().basis           # N = 580
    small = WL.single_centre_small().basis           # a smaller basis for the second call
    lb_big, lb_small = lib_basis(big), lib_basis(small)
    plan_big = W.wpccc_plan_create(lb_big, [0.05, 2.4], [1.0, 1.0])
    plan_small = W.wpccc_plan_create(lb_small, [0.3, 7.5], [1.0, 0.5])
    assert plan_small.n_states < plan_big.n_states
    for plan, j, z in ((plan_big, 1, -3.7), (plan_small, 0, 0.61), (plan_small, 1, -12.0)):
        print(f"noalloc N={plan.n_states} j={j} z={z}", flush=True)
        Ha, Hb = _pair(plan, j, z)
        assert np.isfinite(Ha).all()
        assert np.array_equal(Ha.view(np.int64), Hb.view(np.int64)), (plan.n_states, j, z)
    # the small basis against the oracle (the tolerance of the couplings parity tests)
    ob = build_basis(OSpec(small.n_max, small.l_max, small.n_bins, small.k_max, small.n_r, small.r_max, small.Z))
    Ho = direct_matrix(ob, 7.5, -12.0, 0.5)
    assert np.abs(Hb - Ho).max() <= 1e-12 * np.abs(Ho).max()


def test_noalloc_refuses_two_centre():
    rec = WL.Recipe(2, 1, 1, 1.5, 200, 40.0)
    lb = lib_basis(rec)
    plan = W.wpccc_plan_create_2c([lb], [lb], [0], [1.0], [1.0], n_eta=8, n_tau=8)
    N = plan.n_states
    H = torch.empty((N, N), dtype=torch.complex128, device="cuda")
    with pytest.raises(W.WpcccError) as e:
        W.wpccc_couplings_noalloc(plan, 0, 0.5, H)
    assert e.value.code == -6
