"""Python binding of the MI355X WP-CCC propagation library (``libwpccc.so``).

A thin ctypes layer over the C ABI in ``include/wpccc.h``: the functions keep
the C names and only marshal arguments (PyTorch tensors supply device memory
and streams).  Every computation runs in the HIP library; if the library is
not built or no GPU is usable the calls raise, there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

__all__ = [
    "WpcccError", "BasisSpec", "load_library", "library_path",
    "wpccc_version", "wpccc_basis", "wpccc_basis_info", "wpccc_basis_export",
    "wpccc_basis_destroy", "wpccc_plan_create", "wpccc_plan_create_2c", "wpccc_plan_info",
    "wpccc_plan_path_info", "wpccc_plan_destroy", "WPCCC_Q_DAGGER", "WPCCC_Q_PRIOR",
    "wpccc_plan_status", "wpccc_couplings", "wpccc_couplings_noalloc", "wpccc_step", "wpccc_propagate",
    "wpccc_plan_timing", "wpccc_plan_kernel_time", "wpccc_adjoint", "wpccc_plan_stage_rows",
    "wpccc_plan_stage_launch", "wpccc_plan_stage_cache", "wpccc_measure_mfma", "wpccc_zgesv_batched", "wpccc_plan_groups", "wpccc_observables", "WPCCC_SOLVE_FACTORED", "WPCCC_SOLVE_EXPLICIT", "WPCCC_LAUNCH_AUTO", "WPCCC_LAUNCH_STAGES", "WPCCC_LAUNCH_PERSISTENT",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libwpccc.so")
_lib = None

WPCCC_OK = 0
WPCCC_Q_DAGGER = 0
WPCCC_Q_PRIOR = 1
WPCCC_FP64 = 0
WPCCC_MIXED = 1
WPCCC_LAUNCH_AUTO = 0
WPCCC_LAUNCH_STAGES = 1
WPCCC_LAUNCH_PERSISTENT = 2
WPCCC_CACHE_AUTO = 0
WPCCC_CACHE_ON = 1
WPCCC_CACHE_OFF = 2
WPCCC_SOLVE_FACTORED = 0
WPCCC_SOLVE_EXPLICIT = 1
WPCCC_N_CHANNELS = 6
CHANNELS = ("elastic", "excitation", "target_continuum", "capture", "projectile_continuum", "total")
_STATUS = {-1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ESINGULAR", -5: "ENUMERIC", -6: "ENOTSUP"}


class WpcccError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"WPCCC_{_STATUS.get(code, code)}: {msg}")
        self.code = code


class _Spec(ctypes.Structure):
    _fields_ = [("n_max", ctypes.c_int), ("l_max", ctypes.c_int), ("n_bins", ctypes.c_int),
                ("k_max", ctypes.c_double), ("n_r", ctypes.c_int), ("r_max", ctypes.c_double),
                ("Z", ctypes.c_double)]


class _PlanOpts(ctypes.Structure):
    _fields_ = [("Zp", ctypes.c_double), ("batched", ctypes.c_int), ("two_centre", ctypes.c_int),
                ("q_lower", ctypes.c_int), ("n_eta", ctypes.c_int), ("n_tau", ctypes.c_int),
                ("model_a", ctypes.c_double), ("model_c", ctypes.c_double),
                ("checkpoint_every", ctypes.c_int), ("stage_rows", ctypes.c_int),
                ("precision", ctypes.c_int), ("graph", ctypes.c_int), ("stage_launch", ctypes.c_int),
                ("radial", ctypes.c_int), ("stage_cache", ctypes.c_int), ("solve", ctypes.c_int),
                ("symmetric", ctypes.c_int), ("dz_sym", ctypes.c_double)]


@dataclass
class BasisSpec:
    """One centre's basis recipe (see ``wpccc_basis_spec`` in include/wpccc.h)."""
    n_max: int
    l_max: int
    n_bins: int
    k_max: float
    n_r: int
    r_max: float = 100.0
    Z: float = 1.0


def library_path() -> str:
    return _LIB_PATH


def load_library():
    """Load libwpccc.so (built in-tree by ``paper_2403_04252_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"{_LIB_PATH} is missing: build it with "
                           "`python -m paper_2403_04252_amd.build` (there is no CPU fallback)")
    lib = ctypes.CDLL(_LIB_PATH)
    vp, i, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    pi, pd = ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)
    sig = {
        "wpccc_last_error": ([], ctypes.c_char_p),
        "wpccc_version": ([], ctypes.c_char_p),
        "wpccc_basis": ([ctypes.POINTER(_Spec), ctypes.POINTER(vp)], i),
        "wpccc_basis_info": ([vp, pi, pi, pi], i),
        "wpccc_basis_export": ([vp, pd, pd, pd, pd, pi], i),
        "wpccc_basis_destroy": ([vp], i),
        "wpccc_plan_create": ([vp, i, pd, pd, ctypes.POINTER(_PlanOpts), vp, ctypes.POINTER(vp)], i),
        "wpccc_plan_create_2c": ([ctypes.POINTER(vp), ctypes.POINTER(vp), i, i, pi, pd, pd,
                                  ctypes.POINTER(_PlanOpts), vp, ctypes.POINTER(vp)], i),
        "wpccc_plan_info": ([vp, pi, pi, pi, ctypes.POINTER(ctypes.c_longlong)], i),
        "wpccc_plan_path_info": ([vp, i, pi, pi], i),
        "wpccc_plan_destroy": ([vp], i),
        "wpccc_plan_status": ([vp, vp], i),
        "wpccc_couplings": ([vp, i, d, vp, vp, vp], i),
        "wpccc_couplings_noalloc": ([vp, i, d, vp, vp, vp], i),
        "wpccc_step": ([vp, vp, d, d, vp], i),
        "wpccc_propagate": ([vp, pd, i, vp, vp, vp, vp], i),
        "wpccc_adjoint": ([vp, pd, i, vp, vp, vp, vp, vp], i),
        "wpccc_plan_stage_rows": ([vp, pi], i),
        "wpccc_plan_stage_launch": ([vp, pi], i),
        "wpccc_plan_stage_cache": ([vp, pi], i),
        "wpccc_plan_timing": ([vp, i], i),
        "wpccc_plan_kernel_time": ([vp, ctypes.c_char_p, pd, ctypes.POINTER(ctypes.c_longlong)], i),
        "wpccc_measure_mfma": ([pd, pd, vp], i),
        "wpccc_zgesv_batched": ([i, i, vp, vp, vp, vp], i),
        "wpccc_plan_groups": ([vp, pi, pi], i),
        "wpccc_observables": ([vp, vp, vp, vp, vp], i),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _check(rc: int):
    if rc != WPCCC_OK:
        msg = load_library().wpccc_last_error().decode()
        raise WpcccError(rc, msg)


def _stream_ptr(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_ptr(t, dtype_name, shape=None, name="tensor"):
    if t is None:
        return None
    import torch
    want = {"complex128": torch.complex128, "float64": torch.float64}[dtype_name]
    if t.dtype != want or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {dtype_name} CUDA tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return ctypes.c_void_p(t.data_ptr())


class Basis:
    def __init__(self, handle):
        self.handle = handle

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.wpccc_basis_destroy(self.handle)
            self.handle = None


class Plan:
    def __init__(self, handle, basis, n_traj, n_states, n_pad):
        self.handle = handle
        self.basis = basis          # keeps the basis alive as long as the plan
        self.n_traj = n_traj
        self.n_states = n_states
        self.n_pad = n_pad

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.wpccc_plan_destroy(self.handle)
            self.handle = None


def wpccc_version() -> str:
    return load_library().wpccc_version().decode()


def wpccc_basis(spec) -> Basis:
    """Build one centre's basis on the host (see BasisSpec)."""
    lib = load_library()
    s = _Spec(int(spec.n_max), int(spec.l_max), int(spec.n_bins), float(spec.k_max),
              int(spec.n_r), float(spec.r_max), float(spec.Z))
    h = ctypes.c_void_p()
    _check(lib.wpccc_basis(ctypes.byref(s), ctypes.byref(h)))
    return Basis(h)


def wpccc_basis_info(basis: Basis):
    """(n_states, n_radial, n_r)."""
    a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(load_library().wpccc_basis_info(basis.handle, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return a.value, b.value, c.value


def wpccc_basis_export(basis: Basis) -> dict:
    """Grid, weights, radial functions, energies and (l, m, radial index) per state."""
    n, nf, nr = wpccc_basis_info(basis)
    r = np.zeros(nr + 1)
    w = np.zeros(nr + 1)
    phi = np.zeros((nf, nr + 1))
    eps = np.zeros(n)
    lmi = np.zeros((n, 3), dtype=np.int32)
    dp = lambda x: x.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    _check(load_library().wpccc_basis_export(basis.handle, dp(r), dp(w), dp(phi), dp(eps),
                                             lmi.ctypes.data_as(ctypes.POINTER(ctypes.c_int))))
    return {"r": r, "w": w, "phi": phi, "eps": eps, "l": lmi[:, 0], "m": lmi[:, 1], "a": lmi[:, 2]}


def wpccc_basis_destroy(basis: Basis):
    if basis.handle:
        _check(load_library().wpccc_basis_destroy(basis.handle))
        basis.handle = None


def wpccc_plan_create(basis: Basis, b, v, Zp: float = 1.0, batched: bool = True,
                      two_centre: bool = False, model_a: float = 0.0, model_c: float = 0.0,
                      checkpoint_every: int = 0, stage_rows: int = 0, graph: bool = False,
                      stage_launch: int = WPCCC_LAUNCH_AUTO, mixed: bool = False, interp: bool = False,
                      stage_cache: int = 0, stream=None) -> Plan:
    """Plan for len(b) straight-line paths in one basis; b, v in a.u.  model_a,
    model_c: screened target potential -(1 + a e^{-c r})/r on the fixed basis;
    stage_launch: WPCCC_LAUNCH_AUTO / _STAGES / _PERSISTENT; mixed: the scaled
    FP32 moment tables (WPCCC_MIXED); interp: F tabulated on the grid and
    interpolated at R (WPCCC_RADIAL_INTERP)."""
    lib = load_library()
    b = np.ascontiguousarray(np.atleast_1d(b), dtype=np.float64)
    v = np.ascontiguousarray(np.broadcast_to(np.atleast_1d(v), b.shape), dtype=np.float64)
    opts = _PlanOpts(float(Zp), 1 if batched else 0, 1 if two_centre else 0, 0, 0, 0,
                     float(model_a), float(model_c), int(checkpoint_every), int(stage_rows),
                     WPCCC_MIXED if mixed else WPCCC_FP64, 1 if graph else 0, int(stage_launch),
                     1 if interp else 0, int(stage_cache))
    h = ctypes.c_void_p()
    dp = lambda x: x.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    _check(lib.wpccc_plan_create(basis.handle, int(b.size), dp(b), dp(v), ctypes.byref(opts),
                                 _stream_ptr(stream), ctypes.byref(h)))
    nt, ns, npad, nb = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_longlong()
    _check(lib.wpccc_plan_info(h, ctypes.byref(nt), ctypes.byref(ns), ctypes.byref(npad), ctypes.byref(nb)))
    p = Plan(h, basis, nt.value, ns.value, npad.value)
    p.device_bytes = nb.value
    return p


def wpccc_plan_stage_rows(plan: Plan) -> int:
    """Rows per workgroup of the plan's RK4 stage kernel (set or chosen by timing)."""
    r = ctypes.c_int()
    _check(load_library().wpccc_plan_stage_rows(plan.handle, ctypes.byref(r)))
    return r.value


def wpccc_plan_stage_launch(plan: Plan) -> int:
    """WPCCC_LAUNCH_STAGES or WPCCC_LAUNCH_PERSISTENT: how the plan runs its RK4 stages."""
    r = ctypes.c_int()
    _check(load_library().wpccc_plan_stage_launch(plan.handle, ctypes.byref(r)))
    return r.value


def wpccc_plan_stage_cache(plan: Plan) -> bool:
    """True when the plan's stage kernels read F from the radial-integral cache."""
    r = ctypes.c_int()
    _check(load_library().wpccc_plan_stage_cache(plan.handle, ctypes.byref(r)))
    return bool(r.value)


def wpccc_plan_create_2c(targets, projectiles, set_of_traj, b, v, q_lower: int = WPCCC_Q_DAGGER,
                         n_eta: int = 0, n_tau: int = 0, batched: bool = True, mixed: bool = False,
                         solve: int = WPCCC_SOLVE_FACTORED, graph: bool = False, symmetric: bool = False,
                         dz_sym: float = 0.0, stream=None) -> Plan:
    """Two-centre plan: path j uses the basis pair (targets[s], projectiles[s]), s = set_of_traj[j].
    batched: True/1 all paths of a basis-size group per coupling launch and every path in one
    launch per RK4 stage; 2 the stages per group too; False/0 one path at a time.
    solve: WPCCC_SOLVE_FACTORED (triangular solves per stage) or WPCCC_SOLVE_EXPLICIT
    (M = S^-1 H per coupling point, the paper's form); graph: replay wpccc_propagate's
    steps from captured HIP graphs; symmetric: the S-norm-conserving form of H with dS/dz
    by central differences of step dz_sym (0: 1e-4)."""
    lib = load_library()
    b = np.ascontiguousarray(np.atleast_1d(b), dtype=np.float64)
    v = np.ascontiguousarray(np.broadcast_to(np.atleast_1d(v), b.shape), dtype=np.float64)
    sets = np.ascontiguousarray(np.broadcast_to(np.atleast_1d(set_of_traj), b.shape), dtype=np.int32)
    ns = len(targets)
    if len(projectiles) != ns:
        raise ValueError("targets and projectiles must pair up")
    T = (ctypes.c_void_p * ns)(*[t.handle for t in targets])
    P = (ctypes.c_void_p * ns)(*[q.handle for q in projectiles])
    nb = int(batched) if not isinstance(batched, bool) else (1 if batched else 0)
    opts = _PlanOpts(0.0, nb, 1, int(q_lower), int(n_eta), int(n_tau), 0.0, 0.0, 0, 0,
                     WPCCC_MIXED if mixed else WPCCC_FP64, 1 if graph else 0, 0, 0, 0, int(solve),
                     1 if symmetric else 0, float(dz_sym))
    h = ctypes.c_void_p()
    dp = lambda x: x.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    _check(lib.wpccc_plan_create_2c(T, P, ns, int(b.size), sets.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                    dp(b), dp(v), ctypes.byref(opts), _stream_ptr(stream), ctypes.byref(h)))
    nt, nst, npad, nb = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_longlong()
    _check(lib.wpccc_plan_info(h, ctypes.byref(nt), ctypes.byref(nst), ctypes.byref(npad), ctypes.byref(nb)))
    p = Plan(h, (list(targets), list(projectiles)), nt.value, nst.value, npad.value)
    p.device_bytes = nb.value
    p.two_centre = True
    return p


def wpccc_plan_path_info(plan: Plan, j: int):
    """(n_states, n_target) of path j."""
    a, t = ctypes.c_int(), ctypes.c_int()
    _check(load_library().wpccc_plan_path_info(plan.handle, int(j), ctypes.byref(a), ctypes.byref(t)))
    return a.value, t.value


def wpccc_plan_info(plan: Plan):
    """(n_traj, n_states, n_pad, device_bytes)."""
    nt, ns, npad, nb = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_longlong()
    _check(load_library().wpccc_plan_info(plan.handle, ctypes.byref(nt), ctypes.byref(ns),
                                          ctypes.byref(npad), ctypes.byref(nb)))
    return nt.value, ns.value, npad.value, nb.value


def wpccc_plan_destroy(plan: Plan):
    if plan.handle:
        _check(load_library().wpccc_plan_destroy(plan.handle))
        plan.handle = None


def wpccc_plan_status(plan: Plan, stream=None):
    _check(load_library().wpccc_plan_status(plan.handle, _stream_ptr(stream)))


def wpccc_couplings(plan: Plan, j: int, z: float, H, S=None, stream=None):
    """H (complex128 CUDA [N_j, N_j]) <- couplings of path j at z with phases;
    S: None for a one-centre plan, the [N_j, N_j] overlap matrix for a two-centre plan."""
    N = wpccc_plan_path_info(plan, j)[0]
    _check(load_library().wpccc_couplings(plan.handle, int(j), float(z),
                                          _dev_ptr(H, "complex128", (N, N), "H"),
                                          _dev_ptr(S, "complex128", (N, N), "S"), _stream_ptr(stream)))


def wpccc_couplings_noalloc(plan: Plan, j: int, z: float, H, S=None, stream=None):
    """As wpccc_couplings (one-centre plans), with the library's fixed per-device
    scratch array instead of the plan's workspace: allocates nothing."""
    N = wpccc_plan_path_info(plan, j)[0]
    _check(load_library().wpccc_couplings_noalloc(plan.handle, int(j), float(z),
                                                  _dev_ptr(H, "complex128", (N, N), "H"),
                                                  _dev_ptr(S, "complex128", (N, N), "S"), _stream_ptr(stream)))


def wpccc_step(plan: Plan, X, z: float, h: float, stream=None):
    """One RK4 step z -> z + h for all paths; X complex128 CUDA [n_traj, n_pad], in place."""
    _check(load_library().wpccc_step(plan.handle, _dev_ptr(X, "complex128", (plan.n_traj, plan.n_pad), "X"),
                                     float(z), float(h), _stream_ptr(stream)))


def wpccc_propagate(plan: Plan, zgrid, X, P=None, norm=None, stream=None):
    """Algorithm 1 over zgrid (host array) starting from X (in place)."""
    z = np.ascontiguousarray(zgrid, dtype=np.float64)
    shp = (plan.n_traj, plan.n_pad)
    _check(load_library().wpccc_propagate(
        plan.handle, z.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(z.size),
        _dev_ptr(X, "complex128", shp, "X"), _dev_ptr(P, "float64", shp, "P"),
        _dev_ptr(norm, "float64", (plan.n_traj,), "norm"), _stream_ptr(stream)))


def wpccc_adjoint(plan: Plan, zgrid, X0, gX, grad, X=None, stream=None):
    """Reverse-mode gradients (see include/wpccc.h): grad (float64 CUDA [n_traj, 3])
    <- dL/da, dL/dc, dL/db per path, given gX = dL/d conj(X) at the last point."""
    z = np.ascontiguousarray(zgrid, dtype=np.float64)
    shp = (plan.n_traj, plan.n_pad)
    _check(load_library().wpccc_adjoint(
        plan.handle, z.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(z.size),
        _dev_ptr(X0, "complex128", shp, "X0"), _dev_ptr(X, "complex128", shp, "X"),
        _dev_ptr(gX, "complex128", shp, "gX"), _dev_ptr(grad, "float64", (plan.n_traj, 3), "grad"),
        _stream_ptr(stream)))


def wpccc_plan_timing(plan: Plan, enable: bool):
    """Start (True) or stop (False) per-kernel HIP-event timing on the plan."""
    _check(load_library().wpccc_plan_timing(plan.handle, 1 if enable else 0))


def wpccc_plan_kernel_time(plan: Plan, kernel: str):
    """(total_ms, launches) of `kernel` since timing was enabled or last read."""
    ms, n = ctypes.c_double(), ctypes.c_longlong()
    _check(load_library().wpccc_plan_kernel_time(plan.handle, kernel.encode(), ctypes.byref(ms),
                                                 ctypes.byref(n)))
    return ms.value, n.value


def wpccc_measure_mfma(stream=None):
    """Sustained (FP64, FP32) 16x16x4 MFMA rates of the current device in TFLOP/s."""
    f64, f32 = ctypes.c_double(), ctypes.c_double()
    _check(load_library().wpccc_measure_mfma(ctypes.byref(f64), ctypes.byref(f32), _stream_ptr(stream)))
    return f64.value, f32.value


def wpccc_zgesv_batched(A, B, X, stream=None):
    """X[b] = A[b]^-1 B[b] on the GPU for complex128 CUDA tensors of shape
    [batch, n, n]: A[b] is read as stored column-major (pass the transpose of a
    row-major matrix, e.g. A.transpose(1, 2).contiguous()), B and X row-major."""
    if A.dim() != 3 or A.shape[1] != A.shape[2] or B.shape != A.shape or X.shape != A.shape:
        raise ValueError("A, B and X must be [batch, n, n] of one shape")
    batch, n = int(A.shape[0]), int(A.shape[1])
    shp = (batch, n, n)
    _check(load_library().wpccc_zgesv_batched(n, batch, _dev_ptr(A, "complex128", shp, "A"),
                                              _dev_ptr(B, "complex128", shp, "B"),
                                              _dev_ptr(X, "complex128", shp, "X"), _stream_ptr(stream)))


def wpccc_plan_groups(plan: Plan):
    """(n_groups, group of every path): paths sharing the basis pair and the speed."""
    n = ctypes.c_int()
    g = np.zeros(plan.n_traj, dtype=np.int32)
    _check(load_library().wpccc_plan_groups(plan.handle, ctypes.byref(n),
                                            g.ctypes.data_as(ctypes.POINTER(ctypes.c_int))))
    return n.value, g


def wpccc_observables(plan: Plan, P, chan, sigma=None, stream=None):
    """chan (float64 CUDA [n_traj, 6]) <- channel probabilities per path from P
    ([n_traj, n_pad]); sigma (float64 CUDA [n_groups, 6] or None) <- cross sections."""
    n_groups, _ = wpccc_plan_groups(plan)
    _check(load_library().wpccc_observables(
        plan.handle, _dev_ptr(P, "float64", (plan.n_traj, plan.n_pad), "P"),
        _dev_ptr(chan, "float64", (plan.n_traj, WPCCC_N_CHANNELS), "chan"),
        _dev_ptr(sigma, "float64", (n_groups, WPCCC_N_CHANNELS), "sigma"), _stream_ptr(stream)))
