"""Python binding of libexpwave.so (the C ABI in include/expwave.h).

Argument marshalling only: every step of the method runs in the native
library on the GPU. The functions below carry the C names and raise
`ExpwError` on a non-OK status. `Operator` is a thin convenience wrapper that
takes PyTorch tensors for device memory and the current HIP stream.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libexpwave.so")

EXPW_OK, EXPW_EINVAL, EXPW_ENOMEM, EXPW_EDEVICE, EXPW_ENONFINITE, EXPW_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
EXPW_F32, EXPW_F64 = 0, 1
EXPW_BC_ZERO, EXPW_BC_PERIODIC = 0, 1
EXPW_MAX_KRYLOV, EXPW_MAX_TAYLOR, EXPW_MAX_SOURCES = 64, 16, 64
EXPW_EXPM_DEVICE, EXPW_EXPM_HOST = 0, 1


class ExpwError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"expwave status {status}: {message}")
        self.status = status


class ExpwGrid(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("order", ctypes.c_int32),
                ("n", ctypes.c_int64 * 3), ("h", ctypes.c_double),
                ("dtype", ctypes.c_int32), ("bc", ctypes.c_int32),
                ("abc_cells", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("sigma_max", ctypes.c_double)]


_i32, _i64, _dbl, _vp, _sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p, ctypes.c_size_t
_pd = ctypes.POINTER(ctypes.c_double)
_pi64 = ctypes.POINTER(ctypes.c_int64)
_pi32 = ctypes.POINTER(ctypes.c_int32)
_pgrid = ctypes.POINTER(ExpwGrid)


class ExpwPmlGrid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("h", ctypes.c_double),
                ("dtype", ctypes.c_int32), ("abc_cells", ctypes.c_int32), ("beta0", ctypes.c_double)]


_ppml = ctypes.POINTER(ExpwPmlGrid)

# name -> (restype, argtypes); the list is the full C ABI of include/expwave.h
SIGNATURES = {
    "expw_version": (_i32, []),
    "expw_last_error": (ctypes.c_char_p, []),
    "expw_workspace_size": (_i32, [_pgrid, _i32, _i32, ctypes.POINTER(_sz)]),
    "expw_damping_profile": (_i32, [_i64, _dbl, _i32, _dbl, _i32, _pd]),
    "expw_spectrum_rectangle": (_i32, [_pgrid, _dbl, _pd, _pd]),
    "expw_ellipse": (_i32, [_dbl, _dbl, _pd, _pd, _pd]),
    "expw_faber_coefficients": (_i32, [_dbl, _dbl, _dbl, _dbl, _i32, _pd]),
    "expw_step_ellipse": (_i32, [_i32, _dbl, _dbl, _dbl, _pd, _pd, _pd]),
    "expw_faber_dense_coefficients": (_i32, [_dbl, _dbl, _dbl, _i32, _i32, _pd, _pd]),
    "expw_ricker_derivatives": (_i32, [_dbl, _dbl, _dbl, _i32, _pd]),
    "expw_faber_source_scalars": (_i32, [_dbl, _dbl, _dbl, _i32, _i32, _pd, _pd]),
    "expw_expm": (_i32, [_i32, _pd, _pd]),
    "expw_op_create": (_i32, [_pgrid, _vp, _i32, _i32, _vp, _sz, _vp, ctypes.POINTER(_vp)]),
    "expw_op_create_profiles": (_i32, [_pgrid, _vp, ctypes.POINTER(_pd), _i32, _i32, _vp, _sz, _vp,
                                       ctypes.POINTER(_vp)]),
    "expw_spectrum_rectangle_profiles": (_i32, [_pgrid, _dbl, ctypes.POINTER(_pd), _pd, _pd]),
    "expw_op_destroy": (_i32, [_vp]),
    "expw_set_stream": (_i32, [_vp, _vp]),
    "expw_get_spectrum": (_i32, [_vp, _pd, _pd]),
    "expw_get_ellipse": (_i32, [_vp, _pd, _pd, _pd]),
    "expw_set_ellipse": (_i32, [_vp, _dbl, _dbl, _dbl]),
    "expw_set_tuning": (_i32, [_vp, _i32]),
    "expw_set_pass_kernel": (_i32, [_vp, _i32]),
    "expw_autotune": (_i32, [_vp, _i32, _dbl, _vp, ctypes.c_char_p, ctypes.POINTER(_i32),
                             ctypes.POINTER(_i32), ctypes.POINTER(_dbl)]),
    "expw_apply": (_i32, [_vp, _vp, _vp]),
    "expw_apply_adjoint": (_i32, [_vp, _vp, _vp]),
    "expw_faber_adjoint_step": (_i32, [_vp, _vp, _vp, _dbl, _dbl, _i32, _vp, _vp]),
    "expw_krylov_adjoint_step": (_i32, [_vp, _vp, _vp, _dbl, _dbl, _i32, _vp, _vp]),
    "expw_inject_receivers": (_i32, [_vp, _vp, _dbl, _vp]),
    "expw_set_source_ricker": (_i32, [_vp, _i32, _pi64, _pd, _dbl, _dbl, _i32]),
    "expw_set_source_taylor": (_i32, [_vp, _i32, _pi64, _pd, _i32, _i64, _pd]),
    "expw_set_guard": (_i32, [_vp, _i32]),
    "expw_set_receivers": (_i32, [_vp, _i32, _vp]),
    "expw_step_faber": (_i32, [_vp, _vp, _dbl, _dbl, _i32, _i64, _vp]),
    "expw_step_faber_noalloc": (_i32, [_vp, _vp, _dbl, _dbl, _i32, _i64, _vp]),
    "expw_step_faber_dense": (_i32, [_vp, _vp, _dbl, _dbl, _i32, _i64, _vp, _vp]),
    "expw_faber_dense_output": (_i32, [_vp, _i32, _i64, _vp, _vp, _vp, _i64, _vp]),
    "expw_batch_table_bytes": (_i32, [_i32, _pgrid, ctypes.POINTER(_sz)]),
    "expw_batch_create": (_i32, [ctypes.POINTER(_vp), _i32, _pi32, _pd, ctypes.POINTER(_vp),
                                 ctypes.POINTER(_vp), _vp, _sz, _vp, ctypes.POINTER(_vp)]),
    "expw_batch_step_faber": (_i32, [_vp, _dbl, _i64, _i64]),
    "expw_batch_capture": (_i32, [_vp, _i64]),
    "expw_batch_destroy": (_i32, [_vp]),
    "expw_batch_set_persistent": (_i32, [_vp, _i32]),
    "expw_set_krylov_estimate": (_i32, [_vp, _i32]),
    "expw_krylov_estimate": (_i32, [_vp, ctypes.POINTER(_dbl)]),
    "expw_step_krylov": (_i32, [_vp, _vp, _dbl, _dbl, _i32, _i64, _vp]),
    "expw_step_rk4": (_i32, [_vp, _vp, _dbl, _dbl, _i64, _vp]),
    "expw_step_leapfrog": (_i32, [_vp, _vp, _dbl, _dbl, _i64, _vp]),
    "expw_sync_status": (_i32, [_vp]),
    "expw_krylov_info": (_i32, [_vp, _pi32, _pd]),
    "expw_set_krylov_expm": (_i32, [_vp, _i32]),
    "expw_set_krylov_persistent": (_i32, [_vp, _i32]),
    "expw_set_timing": (_i32, [_vp, _i32]),
    "expw_stream_bench": (_i32, [_i32, _i32, _vp, _vp, _vp, _sz, _i32, _vp, _pd]),
    "expw_get_timing": (_i32, [_vp, _pd, _pi64, _pd]),
    "expw_pml_check_grid": (_i32, [_ppml]),
    "expw_pml_spectrum_rectangle": (_i32, [_ppml, _dbl, _pd, _pd]),
    "expw_pml_surface_weights": (_i32, [_pd, _pd, _pd]),
    "expw_pml_workspace_size": (_i32, [_ppml, _i32, _i32, ctypes.POINTER(_sz)]),
    "expw_pml_create": (_i32, [_ppml, _vp, _i32, _i32, _vp, _sz, _vp, ctypes.POINTER(_vp)]),
    "expw_pml_destroy": (_i32, [_vp]),
    "expw_pml_get_ellipse": (_i32, [_vp, _pd, _pd, _pd]),
    "expw_pml_apply": (_i32, [_vp, _vp, _vp]),
    "expw_pml_set_source_ricker": (_i32, [_vp, _i32, _pi64, _pd, _dbl, _dbl, _i32]),
    "expw_pml_set_receivers": (_i32, [_vp, _i32, _vp]),
    "expw_pml_step_faber": (_i32, [_vp, _vp, _dbl, _dbl, _i32, _i64, _vp]),
    "expw_pml_step_rk4": (_i32, [_vp, _vp, _dbl, _dbl, _i64, _vp]),
    "expw_pml_step_krylov": (_i32, [_vp, _vp, _dbl, _dbl, _i32, _i64, _vp]),
    "expw_pml_set_path": (_i32, [_vp, _i32]),
    "expw_pml_path_for": (_i32, [_vp, _i32, _pi32]),
    "expw_pml_sync_status": (_i32, [_vp]),
}

KERNEL_CLASSES = ("faber", "krylov_matvec", "krylov_mgs", "krylov_aux", "rk4",
                  "leapfrog_v", "leapfrog_p", "gather", "krylov_arnoldi")

_lib = None


def load():
    """Load libexpwave.so (built in-tree); fails loudly when it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2401_16322_amd.build_native`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _check(status):
    if status != EXPW_OK:
        msg = load().expw_last_error()
        raise ExpwError(status, msg.decode() if msg else "")
    return status


def _dptr(arr):
    return arr.ctypes.data_as(_pd)


def make_grid(n, h, order=4, dtype=EXPW_F32, bc=EXPW_BC_ZERO, abc_cells=0, sigma_max=0.0):
    g = ExpwGrid()
    g.ndim = len(n)
    g.order = order
    nn = list(n) + [1] * (3 - len(n))
    for a in range(3):
        g.n[a] = int(nn[a])
    g.h = float(h)
    g.dtype = int(dtype)
    g.bc = int(bc)
    g.abc_cells = int(abc_cells)
    g.reserved = 0
    g.sigma_max = float(sigma_max)
    return g


# ---------------------------------------------------------------- host-only entry points

def expw_version():
    return load().expw_version()


def expw_last_error():
    return load().expw_last_error().decode()


def expw_workspace_size(grid, max_krylov_k, max_taylor_p):
    out = _sz(0)
    _check(load().expw_workspace_size(ctypes.byref(grid), max_krylov_k, max_taylor_p, ctypes.byref(out)))
    return out.value


def expw_damping_profile(n, h, cells, sigma_max, half):
    out = np.zeros(n)
    _check(load().expw_damping_profile(n, h, cells, sigma_max, int(half), _dptr(out)))
    return out


def expw_spectrum_rectangle(grid, c2_max):
    x_lo, B = _dbl(), _dbl()
    _check(load().expw_spectrum_rectangle(ctypes.byref(grid), c2_max, ctypes.byref(x_lo), ctypes.byref(B)))
    return x_lo.value, B.value


def _profile_ptrs(profiles):
    """(keep-alive arrays, C array of double*) for 2 * ndim 1D damping profiles."""
    arrs = [np.ascontiguousarray(p, dtype=np.float64) for p in profiles]
    ptrs = (_pd * len(arrs))(*[_dptr(a) for a in arrs])
    return arrs, ptrs


def expw_spectrum_rectangle_profiles(grid, c2_max, profiles):
    x_lo, B = _dbl(), _dbl()
    arrs, ptrs = _profile_ptrs(profiles)
    _check(load().expw_spectrum_rectangle_profiles(ctypes.byref(grid), c2_max, ptrs,
                                                   ctypes.byref(x_lo), ctypes.byref(B)))
    del arrs
    return x_lo.value, B.value


def expw_ellipse(x_lo, B):
    g, c0, c1 = _dbl(), _dbl(), _dbl()
    _check(load().expw_ellipse(x_lo, B, ctypes.byref(g), ctypes.byref(c0), ctypes.byref(c1)))
    return g.value, c0.value, c1.value


def expw_faber_coefficients(gamma, c0, c1, dt, m):
    out = np.zeros(m + 1)
    _check(load().expw_faber_coefficients(gamma, c0, c1, dt, m, _dptr(out)))
    return out


def expw_step_ellipse(dtype, gamma, c0, c1):
    g, a, b = _dbl(), _dbl(), _dbl()
    _check(load().expw_step_ellipse(int(dtype), gamma, c0, c1, ctypes.byref(g), ctypes.byref(a),
                                    ctypes.byref(b)))
    return g.value, a.value, b.value


def expw_faber_dense_coefficients(gamma, c0, c1, m, taus):
    taus = np.ascontiguousarray(taus, dtype=np.float64).ravel()
    out = np.zeros((taus.size, m + 1))
    _check(load().expw_faber_dense_coefficients(gamma, c0, c1, m, taus.size, _dptr(taus), _dptr(out)))
    return out


def expw_ricker_derivatives(t, f_peak, t_delay, p):
    out = np.zeros(p)
    _check(load().expw_ricker_derivatives(t, f_peak, t_delay, p, _dptr(out)))
    return out


def expw_faber_source_scalars(gamma, c0, c1, m, G):
    G = np.ascontiguousarray(G, dtype=np.float64)
    out = np.zeros(m)
    _check(load().expw_faber_source_scalars(gamma, c0, c1, m, G.size, _dptr(G), _dptr(out)))
    return out


def expw_expm(A):
    A = np.ascontiguousarray(A, dtype=np.float64)
    E = np.zeros_like(A)
    _check(load().expw_expm(A.shape[0], _dptr(A), _dptr(E)))
    return E


# ---------------------------------------------------------------- device entry points (raw)

def expw_op_create(grid, c2_ptr, max_krylov_k, max_taylor_p, ws_ptr, ws_bytes, stream):
    h = _vp()
    _check(load().expw_op_create(ctypes.byref(grid), c2_ptr, max_krylov_k, max_taylor_p, ws_ptr,
                                 ws_bytes, stream, ctypes.byref(h)))
    return h.value


def expw_op_create_profiles(grid, c2_ptr, profiles, max_krylov_k, max_taylor_p, ws_ptr, ws_bytes,
                            stream):
    h = _vp()
    arrs, ptrs = _profile_ptrs(profiles)
    _check(load().expw_op_create_profiles(ctypes.byref(grid), c2_ptr, ptrs, max_krylov_k,
                                          max_taylor_p, ws_ptr, ws_bytes, stream, ctypes.byref(h)))
    del arrs
    return h.value


def expw_op_destroy(op):
    _check(load().expw_op_destroy(op))


def expw_set_stream(op, stream):
    _check(load().expw_set_stream(op, stream))


def expw_get_spectrum(op):
    x_lo, B = _dbl(), _dbl()
    _check(load().expw_get_spectrum(op, ctypes.byref(x_lo), ctypes.byref(B)))
    return x_lo.value, B.value


def expw_get_ellipse(op):
    g, c0, c1 = _dbl(), _dbl(), _dbl()
    _check(load().expw_get_ellipse(op, ctypes.byref(g), ctypes.byref(c0), ctypes.byref(c1)))
    return g.value, c0.value, c1.value


def expw_set_ellipse(op, gamma, c0, c1):
    _check(load().expw_set_ellipse(op, gamma, c0, c1))


def expw_set_tuning(op, fuse):
    _check(load().expw_set_tuning(op, fuse))


EXPW_PASS_AUTO, EXPW_PASS_TILED, EXPW_PASS_STREAMED = 0, 1, 2


def expw_set_pass_kernel(op, kind):
    _check(load().expw_set_pass_kernel(op, int(kind)))


def expw_autotune(op, m, dt, scratch_ptr, cache_path=None):
    """(fuse, pass_kernel, ms per step) chosen by the library's autotuner."""
    fz, pk, ms = _i32(0), _i32(0), _dbl(0.0)
    path = None if cache_path is None else os.fsencode(cache_path)
    _check(load().expw_autotune(op, int(m), float(dt), scratch_ptr, path, ctypes.byref(fz),
                                ctypes.byref(pk), ctypes.byref(ms)))
    return fz.value, pk.value, ms.value


def expw_apply(op, x_ptr, y_ptr):
    _check(load().expw_apply(op, x_ptr, y_ptr))


def expw_apply_adjoint(op, x_ptr, y_ptr):
    _check(load().expw_apply_adjoint(op, x_ptr, y_ptr))


def expw_faber_adjoint_step(op, u_ptr, lam_ptr, t, dt, m, grad_ptr, terms_ptr):
    _check(load().expw_faber_adjoint_step(op, u_ptr, lam_ptr, t, dt, m, grad_ptr, terms_ptr))


def expw_krylov_adjoint_step(op, u_ptr, lam_ptr, t, dt, k, grad_ptr, basis_ptr):
    _check(load().expw_krylov_adjoint_step(op, u_ptr, lam_ptr, t, dt, k, grad_ptr, basis_ptr))


def expw_inject_receivers(op, values_ptr, scale, state_ptr):
    _check(load().expw_inject_receivers(op, values_ptr, scale, state_ptr))


def expw_set_source_ricker(op, nodes, amps, f_peak, t_delay, taylor_p):
    nodes = np.ascontiguousarray(nodes, dtype=np.int64)
    amps = np.ascontiguousarray(amps, dtype=np.float64)
    if nodes.size != amps.size:
        raise ValueError("nodes and amps differ in length")
    _check(load().expw_set_source_ricker(op, nodes.size, nodes.ctypes.data_as(_pi64), _dptr(amps),
                                         f_peak, t_delay, taylor_p))


def expw_set_source_taylor(op, nodes, amps, gder):
    """gder: (nsteps, taylor_p) array of g^(k)(t_n) for step n of each following call."""
    nodes = np.ascontiguousarray(nodes, dtype=np.int64)
    amps = np.ascontiguousarray(amps, dtype=np.float64)
    gder = np.ascontiguousarray(gder, dtype=np.float64)
    if nodes.size != amps.size:
        raise ValueError("nodes and amps differ in length")
    if gder.ndim != 2:
        raise ValueError("gder must be (nsteps, taylor_p)")
    _check(load().expw_set_source_taylor(op, nodes.size, nodes.ctypes.data_as(_pi64), _dptr(amps),
                                         gder.shape[1], gder.shape[0], _dptr(gder)))


def expw_set_receivers(op, n_rec, idx_ptr):
    _check(load().expw_set_receivers(op, n_rec, idx_ptr))


def expw_step_faber(op, state_ptr, t0, dt, m, nsteps, traces_ptr=None):
    _check(load().expw_step_faber(op, state_ptr, t0, dt, m, nsteps, traces_ptr))


def expw_step_faber_noalloc(op, state_ptr, t0, dt, m, nsteps, traces_ptr=None):
    _check(load().expw_step_faber_noalloc(op, state_ptr, t0, dt, m, nsteps, traces_ptr))


def expw_step_faber_dense(op, state_ptr, t0, dt, m, nsteps, traces_ptr, term_traces_ptr):
    _check(load().expw_step_faber_dense(op, state_ptr, t0, dt, m, nsteps, traces_ptr, term_traces_ptr))


def expw_faber_dense_output(op, m, n_samples, sample_step_ptr, coef_ptr, term_traces_ptr, nsteps,
                            out_ptr):
    _check(load().expw_faber_dense_output(op, m, n_samples, sample_step_ptr, coef_ptr,
                                          term_traces_ptr, nsteps, out_ptr))


def expw_batch_table_bytes(n_ops, grid):
    out = _sz(0)
    _check(load().expw_batch_table_bytes(n_ops, ctypes.byref(grid), ctypes.byref(out)))
    return out.value


def expw_batch_create(ops, m, dt, state_ptrs, trace_ptrs, table_ptr, table_bytes, stream):
    n = len(ops)
    P = _vp * n
    m_arr = (ctypes.c_int32 * n)(*[int(v) for v in m])
    dt_arr = (ctypes.c_double * n)(*[float(v) for v in dt])
    tr = P(*[p if p else None for p in trace_ptrs]) if trace_ptrs is not None else None
    h = _vp()
    _check(load().expw_batch_create(P(*ops), n, m_arr, dt_arr, P(*state_ptrs), tr, table_ptr,
                                    table_bytes, stream, ctypes.byref(h)))
    return h.value


def expw_batch_step_faber(batch, t0, nsteps, step0=0):
    _check(load().expw_batch_step_faber(batch, t0, nsteps, step0))


def expw_batch_capture(batch, nsteps):
    _check(load().expw_batch_capture(batch, nsteps))


def expw_batch_destroy(batch):
    _check(load().expw_batch_destroy(batch))


def expw_batch_set_persistent(batch, on):
    _check(load().expw_batch_set_persistent(batch, 1 if on else 0))


def expw_set_krylov_estimate(op, on):
    _check(load().expw_set_krylov_estimate(op, 1 if on else 0))


def expw_krylov_estimate(op):
    est = _dbl(0.0)
    _check(load().expw_krylov_estimate(op, ctypes.byref(est)))
    return est.value


def expw_step_krylov(op, state_ptr, t0, dt, k, nsteps, traces_ptr=None):
    _check(load().expw_step_krylov(op, state_ptr, t0, dt, k, nsteps, traces_ptr))


def expw_step_rk4(op, state_ptr, t0, dt, nsteps, traces_ptr=None):
    _check(load().expw_step_rk4(op, state_ptr, t0, dt, nsteps, traces_ptr))


def expw_step_leapfrog(op, state_ptr, t0, dt, nsteps, traces_ptr=None):
    _check(load().expw_step_leapfrog(op, state_ptr, t0, dt, nsteps, traces_ptr))


def expw_sync_status(op):
    _check(load().expw_sync_status(op))


def expw_krylov_info(op):
    k, b = _i32(), _dbl()
    _check(load().expw_krylov_info(op, ctypes.byref(k), ctypes.byref(b)))
    return k.value, b.value


def expw_set_krylov_expm(op, mode):
    _check(load().expw_set_krylov_expm(op, mode))


def expw_set_krylov_persistent(op, allow):
    _check(load().expw_set_krylov_persistent(op, int(bool(allow))))


def expw_stream_bench(kind, nontemporal, a_ptr, b_ptr, c_ptr, nbytes, reps, stream):
    ms = ctypes.c_double()
    _check(load().expw_stream_bench(int(kind), int(nontemporal), a_ptr, b_ptr, c_ptr, int(nbytes),
                                    int(reps), stream, ctypes.byref(ms)))
    return ms.value


def stream_ceiling(nbytes=1 << 30, reps=10):
    """HBM GB/s of the plain read, copy and triad streams over arrays of
    nbytes bytes (torch device memory), plain and non-temporal."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.ones_like(a)
    c = torch.empty_like(a)
    st = torch.cuda.current_stream().cuda_stream
    out = {}
    for kind, name, traffic in ((0, "read", 1), (1, "copy", 2), (2, "triad", 3)):
        for nt in (0, 1):
            ms = expw_stream_bench(kind, nt, a.data_ptr(), b.data_ptr(), c.data_ptr(), nbytes, reps, st)
            out[name + ("_nt" if nt else "")] = traffic * nbytes / (ms * 1e-3) / 1e9
    del a, b, c
    return out


def expw_set_timing(op, class_mask):
    _check(load().expw_set_timing(op, int(class_mask)))


def expw_get_timing(op):
    """{class: (ms, launches, algorithmic bytes)} since timing was enabled."""
    n = len(KERNEL_CLASSES)
    ms = (ctypes.c_double * n)()
    la = (ctypes.c_int64 * n)()
    by = (ctypes.c_double * n)()
    _check(load().expw_get_timing(op, ms, la, by))
    return {KERNEL_CLASSES[k]: (ms[k], la[k], by[k]) for k in range(n)}


# ---------------------------------------------------------------- torch convenience wrapper

class Operator:
    """The operator H on one grid, with device buffers held as torch tensors.

    c2: torch tensor on the GPU (float32 or float64) of numpy shape
    (nz, nx) or (nz, ny, nx). States are flat tensors of (ndim+1) * points
    values in the canonical layout [p | v_0 | ... | v_{d-1}].
    sigma_profiles: None (the quadratic layer of abc_cells and sigma_max) or
    2 * ndim 1D arrays: axis a at the integer points, then at the half points.
    """

    def __init__(self, n, h, c2, order=4, bc="zero", abc_cells=0, sigma_max=0.0,
                 max_krylov_k=0, max_taylor_p=8, sigma_profiles=None):
        import torch
        self._torch = torch
        if not c2.is_cuda:
            raise ValueError("c2 must be a GPU tensor")
        if c2.dtype not in (torch.float32, torch.float64):
            raise ValueError("c2 must be float32 or float64")
        self.dtype = c2.dtype
        self.dtype_code = EXPW_F32 if c2.dtype == torch.float32 else EXPW_F64
        self.device = c2.device
        self.n = tuple(int(v) for v in n)
        self.ndim = len(self.n)
        self.npts = int(np.prod(self.n))
        self.nstate = (self.ndim + 1) * self.npts
        self.grid = make_grid(self.n, h, order,
                              EXPW_F32 if c2.dtype == torch.float32 else EXPW_F64,
                              EXPW_BC_PERIODIC if bc == "periodic" else EXPW_BC_ZERO,
                              abc_cells, sigma_max)
        self.c2 = c2.contiguous()
        if self.c2.numel() != self.npts:
            raise ValueError("c2 has the wrong number of points")
        nbytes = expw_workspace_size(self.grid, max_krylov_k, max_taylor_p)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self._rec = None
        self.fuse = 0
        if sigma_profiles is None:
            self.op = expw_op_create(self.grid, self.c2.data_ptr(), max_krylov_k, max_taylor_p,
                                     self.workspace.data_ptr(), nbytes, self._stream())
        else:
            if len(sigma_profiles) != 2 * self.ndim or any(
                    len(sigma_profiles[2 * a + hf]) != self.n[a] for a in range(self.ndim) for hf in (0, 1)):
                raise ValueError("sigma_profiles: 2 * ndim arrays of n[a] values each")
            self.op = expw_op_create_profiles(self.grid, self.c2.data_ptr(), sigma_profiles,
                                              max_krylov_k, max_taylor_p, self.workspace.data_ptr(),
                                              nbytes, self._stream())

    def _stream(self):
        return self._torch.cuda.current_stream(self.device).cuda_stream

    def _sync_stream(self):
        expw_set_stream(self.op, self._stream())

    def _check_state(self, state):
        if state.dtype != self.dtype or not state.is_cuda or state.numel() != self.nstate \
                or not state.is_contiguous():
            raise ValueError("state must be a contiguous GPU tensor of the grid dtype and size")

    def _traces_ptr(self, traces, nsteps):
        if traces is None:
            return None
        if self._rec is None:
            raise ValueError("no receivers set")
        if traces.dtype != self.dtype or traces.numel() < nsteps * self._rec.numel() \
                or not traces.is_contiguous():
            raise ValueError("traces must hold nsteps * n_rec values of the grid dtype")
        return traces.data_ptr()

    @property
    def ellipse(self):
        return expw_get_ellipse(self.op)

    @ellipse.setter
    def ellipse(self, val):
        expw_set_ellipse(self.op, *val)

    @property
    def spectrum(self):
        return expw_get_spectrum(self.op)

    def set_tuning(self, fuse=0):
        expw_set_tuning(self.op, fuse)
        self.fuse = fuse

    def set_pass_kernel(self, kind=EXPW_PASS_AUTO):
        """Fused-pass kernel of 2D order-4 grids: auto, tiled or streamed."""
        expw_set_pass_kernel(self.op, kind)

    def autotune(self, m, dt, cache_path=None):
        """The library's autotuner (expw_autotune): times every depth and pass
        kernel this grid admits for Faber steps of degree m (or takes them
        from cache_path) and keeps the fastest. Returns (fuse, pass_kernel,
        ms per step)."""
        scratch = self._torch.zeros(self.nstate, dtype=self.dtype, device=self.device)
        self._sync_stream()
        fz, pk, ms = expw_autotune(self.op, m, dt, scratch.data_ptr(), cache_path)
        self.fuse = fz
        return fz, pk, ms

    def apply(self, x, out=None):
        self._check_state(x)
        y = self._torch.empty_like(x) if out is None else out
        self._sync_stream()
        expw_apply(self.op, x.data_ptr(), y.data_ptr())
        return y

    def apply_adjoint(self, x, out=None):
        """y = H^T x."""
        self._check_state(x)
        y = self._torch.empty_like(x) if out is None else out
        self._sync_stream()
        expw_apply_adjoint(self.op, x.data_ptr(), y.data_ptr())
        return y

    def faber_adjoint_step(self, u, lam, t, dt, m, grad, terms=None):
        """lam <- (Faber step from t)^T lam in place; grad (one value per
        point) += the c^2 gradient of <lam, step(u)>. terms: scratch of
        (m - 1) * nstate values (allocated when None)."""
        self._check_state(u)
        self._check_state(lam)
        if grad.dtype != self.dtype or grad.numel() != self.npts or not grad.is_contiguous():
            raise ValueError("grad must hold one value per grid point of the grid dtype")
        if m > 1:
            if terms is None:
                terms = self._torch.empty((m - 1) * self.nstate, dtype=self.dtype, device=u.device)
            if terms.dtype != self.dtype or terms.numel() < (m - 1) * self.nstate:
                raise ValueError("terms must hold (m - 1) * nstate values")
        self._sync_stream()
        expw_faber_adjoint_step(self.op, u.data_ptr(), lam.data_ptr(), t, dt, m, grad.data_ptr(),
                                terms.data_ptr() if m > 1 else None)
        return lam

    def set_krylov_estimate(self, on=True):
        """Form the a-posteriori error estimate of every later Krylov step."""
        expw_set_krylov_estimate(self.op, on)

    def krylov_estimate(self):
        """Largest error estimate over the steps of the last step_krylov call
        (dt beta h_{k+1,k} |e_k^T phi_1(dt H_k) e_1|)."""
        self._sync_stream()
        return expw_krylov_estimate(self.op)

    def krylov_adjoint_step(self, u, lam, t, dt, k, grad, basis=None):
        """lam <- the Krylov approximation (dimension k) of exp(dt H^T) lam in
        place; grad (one value per point) += the c^2 derivative of
        <lam, exp(dt H~) [u; e_p]> with both exponentials in their Krylov
        spaces (the forward one that of the step from u at t). basis: scratch
        of (k + 1) * nstate values (allocated when None)."""
        self._check_state(u)
        self._check_state(lam)
        if grad.dtype != self.dtype or grad.numel() != self.npts or not grad.is_contiguous():
            raise ValueError("grad must hold one value per grid point of the grid dtype")
        if basis is None:
            basis = self._torch.empty((k + 1) * self.nstate, dtype=self.dtype, device=u.device)
        if basis.dtype != self.dtype or basis.numel() < (k + 1) * self.nstate or not basis.is_contiguous():
            raise ValueError("basis must hold (k + 1) * nstate values")
        self._sync_stream()
        expw_krylov_adjoint_step(self.op, u.data_ptr(), lam.data_ptr(), t, dt, k, grad.data_ptr(),
                                 basis.data_ptr())
        return lam

    def inject_receivers(self, values, state, scale=1.0):
        """state pressure at the receivers += scale * values."""
        self._check_state(state)
        if self._rec is None:
            raise ValueError("no receivers set")
        if values.dtype != self.dtype or values.numel() < self._rec.numel() or not values.is_contiguous():
            raise ValueError("values must hold n_rec values of the grid dtype")
        self._sync_stream()
        expw_inject_receivers(self.op, values.data_ptr(), scale, state.data_ptr())

    def set_source_ricker(self, nodes, amps, f_peak, t_delay, taylor_p=8):
        self._sync_stream()
        expw_set_source_ricker(self.op, nodes, amps, f_peak, t_delay, taylor_p)

    def set_guard(self, on=True):
        """Check every state for NaN/Inf after each step; sync() then raises."""
        _check(load().expw_set_guard(self.op, int(bool(on))))

    def set_source_taylor(self, nodes, amps, gder):
        """A tabulated source: gder[n, k] = g^(k)(t_n) for step n of each following call."""
        self._sync_stream()
        expw_set_source_taylor(self.op, nodes, amps, gder)

    def set_receivers(self, nodes):
        torch = self._torch
        if nodes is None or len(nodes) == 0:
            self._rec = None
            self._sync_stream()
            expw_set_receivers(self.op, 0, None)
            return
        rec = torch.as_tensor(np.asarray(nodes, dtype=np.int64), device=self.device)
        self._rec = rec
        self._sync_stream()
        expw_set_receivers(self.op, rec.numel(), rec.data_ptr())

    def step_faber(self, state, t0, dt, m, nsteps=1, traces=None):
        self._check_state(state)
        self._sync_stream()
        expw_step_faber(self.op, state.data_ptr(), t0, dt, m, nsteps, self._traces_ptr(traces, nsteps))

    def step_faber_noalloc(self, state, t0, dt, m, nsteps=1, traces=None):
        """step_faber with the step's buffers in the library's static device
        scratch (no device allocation; see expw_step_faber_noalloc)."""
        self._check_state(state)
        self._sync_stream()
        expw_step_faber_noalloc(self.op, state.data_ptr(), t0, dt, m, nsteps,
                                self._traces_ptr(traces, nsteps))

    def step_faber_dense(self, state, t0, dt, m, nsteps, term_traces, traces=None):
        """Faber steps that record every term v_0..v_m at the receivers into
        term_traces (nsteps * (m + 1) * n_rec values of the grid dtype)."""
        self._check_state(state)
        if self._rec is None:
            raise ValueError("no receivers set")
        need = nsteps * (m + 1) * self._rec.numel()
        if term_traces.dtype != self.dtype or not term_traces.is_cuda \
                or term_traces.numel() < need or not term_traces.is_contiguous():
            raise ValueError("term_traces must hold nsteps * (m + 1) * n_rec values of the grid dtype")
        self._sync_stream()
        expw_step_faber_dense(self.op, state.data_ptr(), t0, dt, m, nsteps,
                              self._traces_ptr(traces, nsteps), term_traces.data_ptr())

    def dense_coefficients(self, m, taus):
        """Weights a_j(tau) (len(taus) x (m + 1)) of the ellipse the steps run with."""
        g, c0, c1 = expw_step_ellipse(self.dtype_code, *self.ellipse)
        return expw_faber_dense_coefficients(g, c0, c1, m, taus)

    def dense_output(self, m, term_traces, nsteps, sample_step, coef):
        """Receiver values at sample i: sum_j coef[i, j] * term j of step
        sample_step[i] (torch tensors on the GPU: int64 steps, float64 coef)."""
        torch = self._torch
        if self._rec is None:
            raise ValueError("no receivers set")
        sample_step = sample_step.to(device=term_traces.device, dtype=torch.int64).contiguous()
        coef = coef.to(device=term_traces.device, dtype=torch.float64).contiguous()
        ns = sample_step.numel()
        if coef.numel() != ns * (m + 1):
            raise ValueError("coef must hold n_samples * (m + 1) weights")
        if term_traces.dtype != self.dtype or term_traces.numel() < nsteps * (m + 1) * self._rec.numel():
            raise ValueError("term_traces too small")
        out = torch.empty(ns * self._rec.numel(), dtype=self.dtype, device=term_traces.device)
        self._sync_stream()
        expw_faber_dense_output(self.op, m, ns, sample_step.data_ptr(), coef.data_ptr(),
                                term_traces.data_ptr(), nsteps, out.data_ptr())
        return out.view(ns, self._rec.numel())

    def step_krylov(self, state, t0, dt, k, nsteps=1, traces=None):
        self._check_state(state)
        self._sync_stream()
        expw_step_krylov(self.op, state.data_ptr(), t0, dt, k, nsteps, self._traces_ptr(traces, nsteps))

    def step_rk4(self, state, t0, dt, nsteps=1, traces=None):
        self._check_state(state)
        self._sync_stream()
        expw_step_rk4(self.op, state.data_ptr(), t0, dt, nsteps, self._traces_ptr(traces, nsteps))

    def step_leapfrog(self, state, t0, dt, nsteps=1, traces=None):
        self._check_state(state)
        self._sync_stream()
        expw_step_leapfrog(self.op, state.data_ptr(), t0, dt, nsteps, self._traces_ptr(traces, nsteps))

    def sync(self):
        expw_sync_status(self.op)

    def krylov_info(self):
        return expw_krylov_info(self.op)

    def set_krylov_expm(self, mode):
        """"device" (default) or "host" evaluation of the small exponential."""
        expw_set_krylov_expm(self.op, EXPW_EXPM_HOST if mode == "host" else EXPW_EXPM_DEVICE)

    def set_krylov_persistent(self, allow=True):
        expw_set_krylov_persistent(self.op, allow)

    def set_timing(self, classes=None):
        """Time every launch of the given kernel classes (names of KERNEL_CLASSES;
        None = all, [] = off)."""
        self._sync_stream()
        if classes is None:
            mask = -1
        else:
            mask = 0
            for c in classes:
                mask |= 1 << KERNEL_CLASSES.index(c)
        expw_set_timing(self.op, mask)

    def timing(self):
        return expw_get_timing(self.op)

    def close(self):
        if getattr(self, "op", None):
            expw_op_destroy(self.op)
            self.op = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_pml_grid(nx, ny, h, dtype=EXPW_F32, abc_cells=0, beta0=0.0):
    g = ExpwPmlGrid()
    g.nx, g.ny, g.h, g.dtype, g.abc_cells, g.beta0 = int(nx), int(ny), float(h), int(dtype), int(abc_cells), float(beta0)
    return g


def expw_pml_spectrum_rectangle(grid, c2_max):
    x_lo, B = _dbl(), _dbl()
    _check(load().expw_pml_spectrum_rectangle(ctypes.byref(grid), c2_max, ctypes.byref(x_lo), ctypes.byref(B)))
    return x_lo.value, B.value


def expw_pml_surface_weights():
    d2, d1, dw = np.zeros((4, 9)), np.zeros((3, 8)), np.zeros((4, 8))
    _check(load().expw_pml_surface_weights(_dptr(d2), _dptr(d1), _dptr(dw)))
    return d2, d1, dw


def expw_pml_workspace_size(grid, max_taylor_p, max_krylov_k=0):
    out = _sz(0)
    _check(load().expw_pml_workspace_size(ctypes.byref(grid), max_krylov_k, max_taylor_p, ctypes.byref(out)))
    return out.value


class PMLOperator:
    """The paper's own operator (the 2D acoustic PML system with a free surface)
    on one grid. c2: GPU tensor (float32 or float64) of numpy shape (ny, nx),
    row 0 the free surface. States are flat tensors of 4 * nx * ny values
    [u | v | w_x | w_y]; only Faber steps run on this operator."""

    def __init__(self, nx, ny, h, c2, abc_cells=0, beta0=0.0, max_taylor_p=8, max_krylov_k=0):
        import torch
        self._torch = torch
        if not c2.is_cuda or c2.dtype not in (torch.float32, torch.float64):
            raise ValueError("c2 must be a float32 or float64 GPU tensor")
        self.dtype = c2.dtype
        self.device = c2.device
        self.nx, self.ny = int(nx), int(ny)
        self.npts = self.nx * self.ny
        self.nstate = 4 * self.npts
        self.grid = make_pml_grid(nx, ny, h, EXPW_F32 if c2.dtype == torch.float32 else EXPW_F64,
                                  abc_cells, beta0)
        self.c2 = c2.contiguous()
        if self.c2.numel() != self.npts:
            raise ValueError("c2 has the wrong number of points")
        nbytes = expw_pml_workspace_size(self.grid, max_taylor_p, max_krylov_k)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self._rec = None
        h_ = _vp()
        _check(load().expw_pml_create(ctypes.byref(self.grid), self.c2.data_ptr(), max_krylov_k, max_taylor_p,
                                      self.workspace.data_ptr(), nbytes,
                                      torch.cuda.current_stream(self.device).cuda_stream, ctypes.byref(h_)))
        self.op = h_.value

    def __del__(self):
        op = getattr(self, "op", None)
        if op:
            load().expw_pml_destroy(op)
            self.op = None

    def _check_state(self, state):
        if state.dtype != self.dtype or not state.is_cuda or state.numel() != self.nstate \
                or not state.is_contiguous():
            raise ValueError("state must be a contiguous GPU tensor of the grid dtype and size")

    @property
    def ellipse(self):
        g, c0, c1 = _dbl(), _dbl(), _dbl()
        _check(load().expw_pml_get_ellipse(self.op, ctypes.byref(g), ctypes.byref(c0), ctypes.byref(c1)))
        return g.value, c0.value, c1.value

    def apply(self, x, y):
        self._check_state(x)
        self._check_state(y)
        _check(load().expw_pml_apply(self.op, x.data_ptr(), y.data_ptr()))

    def set_source_ricker(self, nodes, amps, f_peak, t_delay, taylor_p):
        nodes = np.ascontiguousarray(nodes, dtype=np.int64)
        amps = np.ascontiguousarray(amps, dtype=np.float64)
        if nodes.size != amps.size:
            raise ValueError("nodes and amps differ in length")
        _check(load().expw_pml_set_source_ricker(self.op, nodes.size, nodes.ctypes.data_as(_pi64),
                                                 _dptr(amps), f_peak, t_delay, taylor_p))

    def set_receivers(self, nodes):
        t = self._torch.as_tensor(np.asarray(nodes, dtype=np.int64), device=self.device).contiguous()
        self._rec = t
        _check(load().expw_pml_set_receivers(self.op, t.numel(), t.data_ptr()))

    def step_faber(self, state, t0, dt, m, nsteps, traces=None):
        self._check_state(state)
        tp = None
        if traces is not None:
            if self._rec is None:
                raise ValueError("no receivers set")
            if traces.dtype != self.dtype or traces.numel() < nsteps * self._rec.numel() \
                    or not traces.is_contiguous():
                raise ValueError("traces must hold nsteps * n_rec values of the grid dtype")
            tp = traces.data_ptr()
        _check(load().expw_pml_step_faber(self.op, state.data_ptr(), t0, dt, m, nsteps, tp))

    def set_path(self, path):
        """0 automatic, 1 one thread per node, 2 LDS tiles, 3 two terms per pass,
        4 row-streamed passes."""
        _check(load().expw_pml_set_path(self.op, int(path)))

    def path_for(self, m):
        """The term kernel (1 to 4) a step of degree m takes."""
        out = _i32(0)
        _check(load().expw_pml_path_for(self.op, int(m), ctypes.byref(out)))
        return out.value

    def _traces(self, traces, nsteps):
        if traces is None:
            return None
        if self._rec is None:
            raise ValueError("no receivers set")
        if traces.dtype != self.dtype or traces.numel() < nsteps * self._rec.numel() \
                or not traces.is_contiguous():
            raise ValueError("traces must hold nsteps * n_rec values of the grid dtype")
        return traces.data_ptr()

    def step_krylov(self, state, t0, dt, k, nsteps, traces=None):
        self._check_state(state)
        _check(load().expw_pml_step_krylov(self.op, state.data_ptr(), t0, dt, k, nsteps,
                                           self._traces(traces, nsteps)))

    def step_rk4(self, state, t0, dt, nsteps, traces=None):
        self._check_state(state)
        _check(load().expw_pml_step_rk4(self.op, state.data_ptr(), t0, dt, nsteps, self._traces(traces, nsteps)))

    def sync(self):
        _check(load().expw_pml_sync_status(self.op))


class Batch:
    """Faber steps of several Operators (shots) in shared launches.

    ops: Operators of one dtype, ndim, order and bc; m, dt: per-shot degree
    and step; states: per-shot state tensors; traces: None or per-shot
    tensors (or None) of steps * n_rec values. The sources and receivers set
    on the operators now are the ones used.
    """

    def __init__(self, ops, m, dt, states, traces=None):
        import torch
        self._torch = torch
        if not (len(ops) == len(m) == len(dt) == len(states)):
            raise ValueError("ops, m, dt and states differ in length")
        for o, s in zip(ops, states):
            o._check_state(s)
        self.ops, self.states, self.traces = list(ops), list(states), traces
        nbytes = expw_batch_table_bytes(len(ops), ops[0].grid)
        self.table = torch.empty(nbytes, dtype=torch.uint8, device=ops[0].device)
        tptr = None
        if traces is not None:
            tptr = [t.data_ptr() if t is not None else None for t in traces]
        # the batch's own stream (default priority), ordered against the caller's
        self.stream = torch.cuda.Stream(device=ops[0].device)
        self.stream.wait_stream(torch.cuda.current_stream(ops[0].device))
        self.handle = expw_batch_create([o.op for o in ops], m, dt, [s.data_ptr() for s in states],
                                        tptr, self.table.data_ptr(), nbytes, self.stream.cuda_stream)

    def step(self, t0, nsteps=1, step0=0):
        """Steps step0 .. step0 + nsteps - 1: shot i's step n runs from
        t0 + n dt[i] and records its traces in row n."""
        cur = self._torch.cuda.current_stream(self.ops[0].device)
        self.stream.wait_stream(cur)
        expw_batch_step_faber(self.handle, t0, nsteps, step0)
        cur.wait_stream(self.stream)

    def set_persistent(self, on=True):
        """One cooperative launch per step (True) or one launch per pass."""
        expw_batch_set_persistent(self.handle, on)

    def capture(self, nsteps):
        """Capture nsteps steps into a HIP graph replayed by step() (0 drops it)."""
        self.stream.synchronize()
        expw_batch_capture(self.handle, nsteps)

    def close(self):
        if getattr(self, "handle", None):
            expw_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
