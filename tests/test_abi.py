"""Host-side checks of the C ABI library (no GPU needed).

* every function declared in include/wpccc.h is exported by libwpccc.so;
* the library's host basis builder (independent code) reproduces the oracle's
  basis: grid, weights, radial functions, energies and state order;
* invalid specifications are rejected with WPCCC_EINVAL.
"""
import os
import re

import numpy as np
import pytest

import paper_2403_04252_amd as W
from oracle.radial import BasisSpec, build_basis

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    src = open(os.path.join(ROOT, "include", "wpccc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(wpccc_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(W.library_path()):
        from paper_2403_04252_amd.build import build_library
        build_library()
    return W.load_library()


def test_header_symbols_exported(lib):
    names = _declared_symbols()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n


def test_version(lib):
    assert re.match(r"^\d+\.\d+\.\d+$", W.wpccc_version())


@pytest.mark.parametrize("spec", [BasisSpec(3, 2, 8, 3.0, 1500), BasisSpec(2, 3, 5, 2.0, 800, 60.0)])
def test_library_basis_matches_oracle(lib, spec):
    hb = W.wpccc_basis(W.BasisSpec(spec.n_max, spec.l_max, spec.n_bins, spec.k_max, spec.n_r,
                                   spec.r_max, spec.Z))
    ex = W.wpccc_basis_export(hb)
    ob = build_basis(spec)
    assert W.wpccc_basis_info(hb) == (ob.n_states, ob.n_radial, spec.n_r)
    assert np.array_equal(ex["r"], ob.r)
    assert np.abs(ex["w"] - ob.w).max() <= 1e-15 * np.abs(ob.w).max()
    assert np.abs(ex["phi"] - ob.phi).max() <= 1e-13 * np.abs(ob.phi).max()
    assert np.abs(ex["eps"] - ob.eps).max() <= 1e-15
    assert np.array_equal(ex["l"], ob.st_l)
    assert np.array_equal(ex["m"], ob.st_m)
    assert np.array_equal(ex["a"], ob.st_a)


@pytest.mark.parametrize("bad", [dict(n_r=1501), dict(l_max=11), dict(n_max=0), dict(Z=0.0),
                                 dict(k_max=0.0), dict(r_max=-1.0)])
def test_invalid_spec_rejected(lib, bad):
    kw = dict(n_max=2, l_max=1, n_bins=2, k_max=1.0, n_r=100, r_max=50.0, Z=1.0)
    kw.update(bad)
    with pytest.raises(W.WpcccError) as ei:
        W.wpccc_basis(W.BasisSpec(**kw))
    assert ei.value.code == -1


def test_plan_without_gpu_fails_loudly(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present: plan creation is exercised by the GPU tests")
    hb = W.wpccc_basis(W.BasisSpec(2, 1, 2, 1.0, 100, 50.0))
    with pytest.raises(W.WpcccError) as ei:
        W.wpccc_plan_create(hb, [1.0], [1.0], stream=0)
    assert ei.value.code == -3


@pytest.mark.parametrize("bad", [dict(q_lower=2), dict(n_eta=2), dict(n_tau=5000), dict(sets=[1]),
                                 dict(b=[0.0]), dict(v=[-1.0]), dict(b=[], v=[], sets=[]), dict(solve=2),
                                 dict(batched=3), dict(symmetric=True, dz_sym=0.5),
                                 dict(symmetric=True, dz_sym=-1e-4)])
def test_two_centre_plan_arguments_rejected(lib, bad):
    """Argument checks of wpccc_plan_create_2c run on the host, before any device call."""
    hb = W.wpccc_basis(W.BasisSpec(2, 1, 2, 1.0, 100, 50.0))
    kw = dict(q_lower=0, n_eta=8, n_tau=8, sets=[0], b=[1.0], v=[1.0], solve=0, batched=True,
              symmetric=False, dz_sym=0.0)
    kw.update(bad)
    with pytest.raises(W.WpcccError) as ei:
        W.wpccc_plan_create_2c([hb], [hb], kw["sets"], kw["b"], kw["v"], q_lower=kw["q_lower"],
                               n_eta=kw["n_eta"], n_tau=kw["n_tau"], solve=kw["solve"], batched=kw["batched"],
                               symmetric=kw["symmetric"], dz_sym=kw["dz_sym"], stream=0)
    assert ei.value.code == -1


def test_two_centre_symmetric_refusals_on_host(lib):
    """The symmetric form with reduced precision or graph replay is refused on the host."""
    hb = W.wpccc_basis(W.BasisSpec(2, 1, 2, 1.0, 100, 50.0))
    for kw in (dict(mixed=True), dict(graph=True)):
        with pytest.raises(W.WpcccError) as ei:
            W.wpccc_plan_create_2c([hb], [hb], [0], [1.0], [1.0], n_eta=8, n_tau=8, symmetric=True, stream=0, **kw)
        assert ei.value.code == -6


def test_zgesv_arguments_rejected_on_host(lib):
    """wpccc_zgesv_batched checks its sizes and pointers before any device call."""
    assert lib.wpccc_zgesv_batched(0, 1, None, None, None, None) == -1
    assert lib.wpccc_zgesv_batched(4, 0, None, None, None, None) == -1
    assert lib.wpccc_zgesv_batched(4097, 1, 1, 1, 1, None) == -1
    assert b"wpccc_zgesv_batched" in lib.wpccc_last_error()


def test_two_centre_plan_without_gpu_fails_loudly(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present: plan creation is exercised by the GPU tests")
    hb = W.wpccc_basis(W.BasisSpec(2, 1, 2, 1.0, 100, 50.0))
    with pytest.raises(W.WpcccError) as ei:
        W.wpccc_plan_create_2c([hb], [hb], [0], [1.0], [1.0], n_eta=8, n_tau=8, stream=0)
    assert ei.value.code == -3
