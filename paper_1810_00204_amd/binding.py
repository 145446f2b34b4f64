"""ctypes binding of libqvts.so (the C ABI in include/qvts.h).

Argument marshalling only: every step of the planning path runs in the HIP
kernels of the library.  PyTorch provides device memory and streams; tensors
are passed by ``data_ptr()``, streams by their ``hipStream_t`` handle.  There
is no fallback: if the library is missing, loading raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqvts.so")

QV_OK = 0
QV_ERR_INVALID_ARG = 1
QV_ERR_NOT_STOCHASTIC = 2
QV_ERR_BELIEF_INVALID = 3
QV_ERR_ZERO_LIKELIHOOD = 4
QV_ERR_WORKSPACE = 5
QV_ERR_HIP = 6
QV_ERR_UNSUPPORTED = 7

QV_MAX_ACTIONS = 9
QV_MAX_DEPTH = 6
QV_MAX_SAMPLES = 16
QV_PLAN_STORE_LEAVES = 1
QV_PLAN_TILED = 2
QV_PLAN_CHECK = 4
QV_MAX_BOUND_COLS = 1024
QV_PBVI_MAX_POINTS = 256
QV_BATCH_GRAPH = 1

# every function the header declares
EXPORTS = [
    "qv_status_string", "qv_last_hip_error",
    "qv_belief_update_workspace_bytes", "qv_belief_update", "qv_belief_update_noalloc",
    "qv_vi_workspace_bytes", "qv_value_iterate",
    "qv_fib_workspace_bytes", "qv_fib_iterate",
    "qv_check_workspace_bytes", "qv_model_check",
    "qv_blind_workspace_bytes", "qv_blind_iterate",
    "qv_search_workspace_bytes", "qv_search_layout_of", "qv_search_init", "qv_search_expand",
    "qv_search_result", "qv_search_update",
    "qv_pbvi_workspace_bytes", "qv_pbvi_layout_of", "qv_pbvi_init", "qv_pbvi_expand",
    "qv_pbvi_backup", "qv_pbvi_result",
    "qv_plan_workspace_bytes", "qv_plan_step", "qv_plan_layout",
    "qv_timing_enable", "qv_timing_read",
    "qv_filter_workspace_bytes", "qv_filter_nll_grad",
    "qv_batch_create", "qv_batch_destroy", "qv_batch_workspace_bytes", "qv_batch_set_shape",
    "qv_batch_get_shape", "qv_batch_plan", "qv_batch_autotune", "qv_batch_layout",
]


class qv_model(C.Structure):
    _fields_ = [("W", C.c_int32), ("H", C.c_int32),
                ("occ", C.c_void_p),
                ("A", C.c_int32),
                ("slip", C.c_float * 81),
                ("flip", C.c_float * 4),
                ("L", C.c_int32),
                ("lm_cell", C.c_void_p),
                ("lm_p", C.c_float),
                ("R", C.c_void_p),
                ("goal", C.c_int32),
                ("gamma", C.c_float)]


class qv_tree_layout(C.Structure):
    _fields_ = [("D", C.c_int32), ("n", C.c_int32), ("K", C.c_int32),
                ("A", C.c_int32), ("S", C.c_int32),
                ("tile_rows", C.c_int32), ("tiles", C.c_int32),
                ("level_slots", C.c_int64 * (QV_MAX_DEPTH + 1)),
                ("level_first", C.c_int64 * (QV_MAX_DEPTH + 2)),
                ("valid", C.c_size_t), ("z", C.c_size_t), ("count", C.c_size_t),
                ("pz", C.c_size_t), ("value", C.c_size_t), ("qvalue", C.c_size_t),
                ("reward", C.c_size_t),
                ("belief_offset", C.c_size_t * (QV_MAX_DEPTH + 1)),
                ("total_bytes", C.c_size_t)]


class qv_search_layout(C.Structure):
    _fields_ = [("n", C.c_int32), ("K", C.c_int32), ("A", C.c_int32), ("S", C.c_int32),
                ("max_nodes", C.c_int32)] + [(f, C.c_size_t) for f in (
                    "sig", "staytab", "lm_wall", "belief", "valid", "z", "count", "pz",
                    "weight", "parent", "depth", "U", "L", "H", "E", "expanded", "child_base",
                    "rb", "UQ", "LQ", "HQ", "EQ", "ctl", "log", "err", "total_bytes")]


class qv_pbvi_layout(C.Structure):
    _fields_ = [("A", C.c_int32), ("S", C.c_int32), ("ZC", C.c_int32),
                ("max_points", C.c_int32), ("ld", C.c_int32)] + [(f, C.c_size_t) for f in (
                    "sig", "staytab", "lm_wall", "points", "pred", "cand", "idx", "vals",
                    "dist", "dvalid", "dz", "dcount", "dpz", "src", "pick", "gamma0", "gamma1",
                    "ctl", "err", "total_bytes")]


class qv_kernel_time(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("launches", C.c_int64), ("total_ms", C.c_double)]


class QvError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {qv_status_string(status)} (status {status})")


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run `python -m paper_1810_00204_amd.build`")
        L = C.CDLL(LIB_PATH)
        mp = C.POINTER(qv_model)
        vp = C.c_void_p
        L.qv_status_string.argtypes = [C.c_int32]
        L.qv_status_string.restype = C.c_char_p
        L.qv_last_hip_error.argtypes = []
        L.qv_last_hip_error.restype = C.c_int32
        L.qv_belief_update_workspace_bytes.argtypes = [mp, C.c_int32]
        L.qv_belief_update_workspace_bytes.restype = C.c_size_t
        L.qv_belief_update.argtypes = [mp, C.c_int32, vp, vp, vp, vp, vp, C.c_int32, vp,
                                       C.c_size_t, vp]
        L.qv_belief_update.restype = C.c_int32
        L.qv_belief_update_noalloc.argtypes = [mp, C.c_int32, vp, vp, vp, vp, vp, C.c_int32, vp]
        L.qv_belief_update_noalloc.restype = C.c_int32
        L.qv_vi_workspace_bytes.argtypes = [mp, C.c_int32]
        L.qv_vi_workspace_bytes.restype = C.c_size_t
        L.qv_value_iterate.argtypes = [mp, C.c_float, C.c_int32, vp, C.POINTER(C.c_double),
                                       C.POINTER(C.c_int32), vp, C.c_size_t, vp]
        L.qv_value_iterate.restype = C.c_int32
        L.qv_check_workspace_bytes.argtypes = []
        L.qv_check_workspace_bytes.restype = C.c_size_t
        L.qv_model_check.argtypes = [mp, vp, vp, C.c_size_t, vp]
        L.qv_model_check.restype = C.c_int32
        L.qv_blind_workspace_bytes.argtypes = [mp, C.c_int32]
        L.qv_blind_workspace_bytes.restype = C.c_size_t
        L.qv_blind_iterate.argtypes = [mp, C.c_float, C.c_int32, vp, C.POINTER(C.c_double),
                                       C.POINTER(C.c_int32), vp, C.c_size_t, vp]
        L.qv_blind_iterate.restype = C.c_int32
        L.qv_search_workspace_bytes.argtypes = [mp, C.c_int32, C.c_int32]
        L.qv_search_workspace_bytes.restype = C.c_size_t
        L.qv_search_layout_of.argtypes = [mp, C.c_int32, C.c_int32, C.POINTER(qv_search_layout)]
        L.qv_search_layout_of.restype = C.c_int32
        L.qv_search_init.argtypes = [mp, vp, vp, C.c_int32, vp, C.c_int32, C.c_int32, vp,
                                     C.c_size_t, vp]
        L.qv_search_init.restype = C.c_int32
        L.qv_search_expand.argtypes = [mp, vp, vp, C.c_int32, C.c_int32, C.c_int32, C.c_uint64,
                                       C.c_uint32, C.c_int32, vp, C.c_size_t, vp]
        L.qv_search_expand.restype = C.c_int32
        L.qv_search_result.argtypes = [mp, C.c_int32, C.c_int32, vp, vp, vp, vp, C.c_size_t, vp]
        L.qv_search_result.restype = C.c_int32
        L.qv_search_update.argtypes = [mp, vp, vp, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                       C.c_int32, vp, C.c_size_t, vp]
        L.qv_search_update.restype = C.c_int32
        L.qv_pbvi_workspace_bytes.argtypes = [mp, C.c_int32, C.c_int32]
        L.qv_pbvi_workspace_bytes.restype = C.c_size_t
        L.qv_pbvi_layout_of.argtypes = [mp, C.c_int32, C.c_int32, C.POINTER(qv_pbvi_layout)]
        L.qv_pbvi_layout_of.restype = C.c_int32
        L.qv_pbvi_init.argtypes = [mp, vp, vp, C.c_int32, C.c_int32, vp, C.c_size_t, vp]
        L.qv_pbvi_init.restype = C.c_int32
        L.qv_pbvi_expand.argtypes = [mp, C.c_int32, C.c_int32, C.c_uint64, C.c_uint32,
                                     C.POINTER(C.c_int32), vp, C.c_size_t, vp]
        L.qv_pbvi_expand.restype = C.c_int32
        L.qv_pbvi_backup.argtypes = [mp, C.c_int32, C.c_int32, C.c_int32, vp, C.c_size_t, vp]
        L.qv_pbvi_backup.restype = C.c_int32
        L.qv_pbvi_result.argtypes = [mp, C.c_int32, C.c_int32, vp, C.c_int32,
                                     C.POINTER(C.c_int32), vp, C.c_size_t, vp]
        L.qv_pbvi_result.restype = C.c_int32
        L.qv_fib_workspace_bytes.argtypes = [mp, C.c_int32]
        L.qv_fib_workspace_bytes.restype = C.c_size_t
        L.qv_fib_iterate.argtypes = [mp, C.c_float, C.c_int32, vp, C.POINTER(C.c_double),
                                     C.POINTER(C.c_int32), vp, C.c_size_t, vp]
        L.qv_fib_iterate.restype = C.c_int32
        L.qv_plan_workspace_bytes.argtypes = [mp, C.c_int32, C.c_int32, C.c_int32]
        L.qv_plan_workspace_bytes.restype = C.c_size_t
        L.qv_plan_step.argtypes = [mp, vp, vp, C.c_int32, C.c_int32, C.c_uint64, C.c_uint32,
                                   C.c_int32, vp, vp, vp, C.c_size_t, vp]
        L.qv_plan_step.restype = C.c_int32
        L.qv_plan_layout.argtypes = [mp, C.c_int32, C.c_int32, C.c_int32,
                                     C.POINTER(qv_tree_layout)]
        L.qv_plan_layout.restype = C.c_int32
        L.qv_filter_workspace_bytes.argtypes = [mp, C.c_int32, C.c_int32, C.c_int32]
        L.qv_filter_workspace_bytes.restype = C.c_size_t
        L.qv_filter_nll_grad.argtypes = [mp, vp, vp, C.c_int32, C.c_int32, vp, C.c_int32, vp, vp,
                                         C.c_int32, vp, vp, vp, C.c_int32, vp, C.c_size_t, vp]
        L.qv_filter_nll_grad.restype = C.c_int32
        pp = C.POINTER(C.c_void_p)
        L.qv_batch_create.argtypes = [C.c_int32, mp, C.POINTER(C.c_int32), C.c_int32, C.c_int32,
                                      C.POINTER(C.c_void_p)]
        L.qv_batch_create.restype = C.c_int32
        L.qv_batch_destroy.argtypes = [vp]
        L.qv_batch_destroy.restype = C.c_int32
        L.qv_batch_workspace_bytes.argtypes = [vp]
        L.qv_batch_workspace_bytes.restype = C.c_size_t
        L.qv_batch_set_shape.argtypes = [vp, C.c_int32, C.c_int32]
        L.qv_batch_set_shape.restype = C.c_int32
        L.qv_batch_get_shape.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.qv_batch_get_shape.restype = C.c_int32
        L.qv_batch_plan.argtypes = [vp, pp, pp, C.c_uint64, vp, vp, vp, C.c_size_t, vp]
        L.qv_batch_plan.restype = C.c_int32
        L.qv_batch_autotune.argtypes = [vp, pp, pp, C.c_uint64, vp, vp, C.c_int32, vp,
                                        C.c_size_t, vp, C.POINTER(C.c_float)]
        L.qv_batch_autotune.restype = C.c_int32
        L.qv_batch_layout.argtypes = [vp, C.c_int32, C.POINTER(qv_tree_layout),
                                      C.POINTER(C.c_size_t)]
        L.qv_batch_layout.restype = C.c_int32
        L.qv_timing_enable.argtypes = [C.c_int32]
        L.qv_timing_enable.restype = C.c_int32
        L.qv_timing_read.argtypes = [C.POINTER(qv_kernel_time), C.c_int32, C.POINTER(C.c_int32)]
        L.qv_timing_read.restype = C.c_int32
        _lib = L
    return _lib


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    return int(t.data_ptr()) if hasattr(t, "data_ptr") else int(t)


def _stream(stream) -> Optional[int]:
    if stream is None:
        import torch
        return int(torch.cuda.current_stream().cuda_stream)
    return int(getattr(stream, "cuda_stream", stream))


# ---------------------------------------------------------------------------
# the C calls, one Python function each
# ---------------------------------------------------------------------------

def qv_status_string(status: int) -> str:
    return lib().qv_status_string(int(status)).decode()


def qv_last_hip_error() -> int:
    return int(lib().qv_last_hip_error())


def qv_belief_update_workspace_bytes(model, batch: int) -> int:
    return int(lib().qv_belief_update_workspace_bytes(C.byref(model.c), int(batch)))


def qv_belief_update(model, batch, b, a, z, b_out, p_out, check, ws, stream=None) -> int:
    return int(lib().qv_belief_update(C.byref(model.c), int(batch), _ptr(b), _ptr(a), _ptr(z),
                                      _ptr(b_out), _ptr(p_out), int(check), _ptr(ws),
                                      _nbytes(ws), _stream(stream)))


def qv_belief_update_noalloc(model, batch, b, a, z, b_out, p_out, check, stream=None) -> int:
    return int(lib().qv_belief_update_noalloc(C.byref(model.c), int(batch), _ptr(b), _ptr(a),
                                              _ptr(z), _ptr(b_out), _ptr(p_out), int(check),
                                              _stream(stream)))


def qv_vi_workspace_bytes(model, max_sweeps: int) -> int:
    return int(lib().qv_vi_workspace_bytes(C.byref(model.c), int(max_sweeps)))


def qv_value_iterate(model, tol, max_sweeps, Q, ws, stream=None):
    """Returns (status, residual, sweeps)."""
    res = C.c_double(0.0)
    sw = C.c_int32(0)
    st = lib().qv_value_iterate(C.byref(model.c), float(tol), int(max_sweeps), _ptr(Q),
                                C.byref(res), C.byref(sw), _ptr(ws), _nbytes(ws),
                                _stream(stream))
    return int(st), res.value, sw.value


def qv_check_workspace_bytes() -> int:
    return int(lib().qv_check_workspace_bytes())


def qv_model_check(model, b0, ws, stream=None) -> int:
    """Device validation of the model's arrays and (if given) the start belief."""
    return int(lib().qv_model_check(C.byref(model.c), _ptr(b0) if b0 is not None else None,
                                    _ptr(ws), _nbytes(ws), _stream(stream)))


def qv_blind_workspace_bytes(model, max_sweeps: int) -> int:
    return int(lib().qv_blind_workspace_bytes(C.byref(model.c), int(max_sweeps)))


def qv_blind_iterate(model, tol, max_sweeps, alpha, ws, stream=None):
    """Returns (status, residual, sweeps)."""
    res = C.c_double(0.0)
    sw = C.c_int32(0)
    st = lib().qv_blind_iterate(C.byref(model.c), float(tol), int(max_sweeps), _ptr(alpha),
                                C.byref(res), C.byref(sw), _ptr(ws), _nbytes(ws),
                                _stream(stream))
    return int(st), res.value, sw.value


def qv_search_workspace_bytes(model, n: int, max_nodes: int) -> int:
    return int(lib().qv_search_workspace_bytes(C.byref(model.c), int(n), int(max_nodes)))


def qv_search_layout_of(model, n: int, max_nodes: int):
    out = qv_search_layout()
    st = lib().qv_search_layout_of(C.byref(model.c), int(n), int(max_nodes), C.byref(out))
    return int(st), out


def qv_search_init(model, Ut, Lt, l_cols, b0, n, max_nodes, ws, stream=None) -> int:
    return int(lib().qv_search_init(C.byref(model.c), _ptr(Ut), _ptr(Lt), int(l_cols), _ptr(b0),
                                    int(n), int(max_nodes), _ptr(ws), _nbytes(ws),
                                    _stream(stream)))


def qv_search_expand(model, Ut, Lt, l_cols, n, max_nodes, seed, query_id, expansions, ws,
                     stream=None) -> int:
    return int(lib().qv_search_expand(C.byref(model.c), _ptr(Ut), _ptr(Lt), int(l_cols), int(n),
                                      int(max_nodes), C.c_uint64(int(seed) & (2 ** 64 - 1)),
                                      C.c_uint32(int(query_id) & (2 ** 32 - 1)),
                                      int(expansions), _ptr(ws), _nbytes(ws), _stream(stream)))


def qv_search_result(model, n, max_nodes, action_out, rootU_out, rootL_out, ws,
                     stream=None) -> int:
    return int(lib().qv_search_result(C.byref(model.c), int(n), int(max_nodes),
                                      _ptr(action_out), _ptr(rootU_out), _ptr(rootL_out),
                                      _ptr(ws), _nbytes(ws), _stream(stream)))


def qv_search_update(model, Ut, Lt, l_cols, n, max_nodes, a, z, ws, stream=None) -> int:
    return int(lib().qv_search_update(C.byref(model.c), _ptr(Ut), _ptr(Lt), int(l_cols), int(n),
                                      int(max_nodes), int(a), int(z), _ptr(ws), _nbytes(ws),
                                      _stream(stream)))


def qv_pbvi_workspace_bytes(model, max_points: int, init_cols: int) -> int:
    return int(lib().qv_pbvi_workspace_bytes(C.byref(model.c), int(max_points), int(init_cols)))


def qv_pbvi_layout_of(model, max_points: int, init_cols: int):
    out = qv_pbvi_layout()
    st = lib().qv_pbvi_layout_of(C.byref(model.c), int(max_points), int(init_cols),
                                 C.byref(out))
    return int(st), out


def qv_pbvi_init(model, b0, init, init_cols, max_points, ws, stream=None) -> int:
    return int(lib().qv_pbvi_init(C.byref(model.c), _ptr(b0), _ptr(init), int(init_cols),
                                  int(max_points), _ptr(ws), _nbytes(ws), _stream(stream)))


def qv_pbvi_expand(model, init_cols, max_points, seed, query_id, ws, stream=None):
    """-> (status, points added)."""
    added = C.c_int32(0)
    st = lib().qv_pbvi_expand(C.byref(model.c), int(init_cols), int(max_points),
                              C.c_uint64(int(seed) & (2 ** 64 - 1)),
                              C.c_uint32(int(query_id) & (2 ** 32 - 1)), C.byref(added),
                              _ptr(ws), _nbytes(ws), _stream(stream))
    return int(st), added.value


def qv_pbvi_backup(model, init_cols, max_points, sweeps, ws, stream=None) -> int:
    return int(lib().qv_pbvi_backup(C.byref(model.c), int(init_cols), int(max_points),
                                    int(sweeps), _ptr(ws), _nbytes(ws), _stream(stream)))


def qv_pbvi_result(model, init_cols, max_points, gamma_out, ld_out, ws, stream=None):
    """-> (status, number of points)."""
    npts = C.c_int32(0)
    st = lib().qv_pbvi_result(C.byref(model.c), int(init_cols), int(max_points),
                              _ptr(gamma_out), int(ld_out), C.byref(npts), _ptr(ws),
                              _nbytes(ws), _stream(stream))
    return int(st), npts.value


def qv_fib_workspace_bytes(model, max_sweeps: int) -> int:
    return int(lib().qv_fib_workspace_bytes(C.byref(model.c), int(max_sweeps)))


def qv_fib_iterate(model, tol, max_sweeps, alpha, ws, stream=None):
    """Returns (status, residual, sweeps)."""
    res = C.c_double(0.0)
    sw = C.c_int32(0)
    st = lib().qv_fib_iterate(C.byref(model.c), float(tol), int(max_sweeps), _ptr(alpha),
                              C.byref(res), C.byref(sw), _ptr(ws), _nbytes(ws),
                              _stream(stream))
    return int(st), res.value, sw.value


def qv_plan_workspace_bytes(model, D: int, n: int, flags: int = 0) -> int:
    return int(lib().qv_plan_workspace_bytes(C.byref(model.c), int(D), int(n), int(flags)))


def qv_plan_layout(model, D: int, n: int, flags: int = 0):
    out = qv_tree_layout()
    st = lib().qv_plan_layout(C.byref(model.c), int(D), int(n), int(flags), C.byref(out))
    return int(st), out


def qv_plan_step(model, Q, b0, D, n, seed, query_id, flags, action_out, rootQ_out, ws,
                 stream=None) -> int:
    return int(lib().qv_plan_step(C.byref(model.c), _ptr(Q), _ptr(b0), int(D), int(n),
                                  C.c_uint64(int(seed) & (2 ** 64 - 1)),
                                  C.c_uint32(int(query_id) & (2 ** 32 - 1)), int(flags),
                                  _ptr(action_out), _ptr(rootQ_out), _ptr(ws), _nbytes(ws),
                                  _stream(stream)))


def qv_filter_workspace_bytes(model, ntraj: int, T: int, ckpt_every: int) -> int:
    return int(lib().qv_filter_workspace_bytes(C.byref(model.c), int(ntraj), int(T),
                                               int(ckpt_every)))


def qv_filter_nll_grad(model, theta, phi, ntraj, T, b0, b0_per_traj, acts, obs, ckpt_every,
                       nll_out, g_slip, g_flip, check, ws, stream=None) -> int:
    return int(lib().qv_filter_nll_grad(C.byref(model.c), _ptr(theta), _ptr(phi), int(ntraj),
                                        int(T), _ptr(b0), int(b0_per_traj), _ptr(acts),
                                        _ptr(obs), int(ckpt_every), _ptr(nll_out), _ptr(g_slip),
                                        _ptr(g_flip), int(check), _ptr(ws), _nbytes(ws),
                                        _stream(stream)))


def _ptr_array(ts):
    arr = (C.c_void_p * max(len(ts), 1))()
    for i, t in enumerate(ts):
        arr[i] = _ptr(t)
    return arr


def qv_batch_create(models, depths, n: int, flags: int = 0):
    """Returns (status, handle); models: list of DeviceModel."""
    nq = len(models)
    cm = (qv_model * max(nq, 1))(*[m.c for m in models])
    dp = (C.c_int32 * max(nq, 1))(*[int(d) for d in depths])
    h = C.c_void_p()
    st = lib().qv_batch_create(int(nq), cm, dp, int(n), int(flags), C.byref(h))
    return int(st), h


def qv_batch_destroy(h) -> int:
    return int(lib().qv_batch_destroy(h))


def qv_batch_workspace_bytes(h) -> int:
    return int(lib().qv_batch_workspace_bytes(h))


def qv_batch_set_shape(h, tile_cells: int, chunk: int) -> int:
    return int(lib().qv_batch_set_shape(h, int(tile_cells), int(chunk)))


def qv_batch_get_shape(h):
    tc, ch = C.c_int32(0), C.c_int32(0)
    st = lib().qv_batch_get_shape(h, C.byref(tc), C.byref(ch))
    return int(st), int(tc.value), int(ch.value)


def qv_batch_plan(h, Qs, b0s, seed, actions, rootQ, ws, stream=None) -> int:
    return int(lib().qv_batch_plan(h, _ptr_array(Qs), _ptr_array(b0s),
                                   C.c_uint64(int(seed) & (2 ** 64 - 1)), _ptr(actions),
                                   _ptr(rootQ), _ptr(ws), _nbytes(ws), _stream(stream)))


def qv_batch_autotune(h, Qs, b0s, seed, actions, rootQ, reps, ws, stream=None):
    """Returns (status, best milliseconds per batch)."""
    ms = C.c_float(0.0)
    st = lib().qv_batch_autotune(h, _ptr_array(Qs), _ptr_array(b0s),
                                 C.c_uint64(int(seed) & (2 ** 64 - 1)), _ptr(actions),
                                 _ptr(rootQ), int(reps), _ptr(ws), _nbytes(ws), _stream(stream),
                                 C.byref(ms))
    return int(st), float(ms.value)


def qv_batch_layout(h, q: int):
    out = qv_tree_layout()
    off = C.c_size_t(0)
    st = lib().qv_batch_layout(h, int(q), C.byref(out), C.byref(off))
    return int(st), out, int(off.value)


def qv_timing_enable(on: bool) -> int:
    return int(lib().qv_timing_enable(1 if on else 0))


def qv_timing_read(max_entries: int = 64):
    """Returns (status, {kernel name: (launches, total_ms)})."""
    buf = (qv_kernel_time * max_entries)()
    n = C.c_int32(0)
    st = lib().qv_timing_read(buf, int(max_entries), C.byref(n))
    return int(st), {buf[i].name.decode(): (int(buf[i].launches), float(buf[i].total_ms))
                     for i in range(n.value)}


def _nbytes(t) -> int:
    if t is None:
        return 0
    return int(t.numel() * t.element_size())


# ---------------------------------------------------------------------------
# device-resident problem
# ---------------------------------------------------------------------------

class DeviceModel:
    """A problem's arrays on the device plus the qv_model struct that points
    at them (the tensors stay referenced for the struct's lifetime)."""

    def __init__(self, prob, device="cuda", slip=None, flip=None):
        import torch
        self.prob = prob
        self.occ = torch.as_tensor(np.ascontiguousarray(prob.occ, dtype=np.uint8)).to(device)
        lm = np.ascontiguousarray(prob.lm_cell, dtype=np.int32)
        self.lm_cell = torch.as_tensor(lm if lm.size else np.zeros(1, np.int32)).to(device)
        self.R = torch.as_tensor(np.ascontiguousarray(prob.R, dtype=np.float32)).to(device)
        sl = np.zeros(81, dtype=np.float32)
        src = np.asarray(prob.slip if slip is None else slip, dtype=np.float32).reshape(-1)
        sl[:src.size] = src
        fl = np.asarray(prob.flip if flip is None else flip, dtype=np.float32)
        self.c = qv_model(int(prob.W), int(prob.H), _ptr(self.occ), src.size // 9,
                          (C.c_float * 81)(*sl.tolist()), (C.c_float * 4)(*fl.tolist()),
                          int(lm.size), _ptr(self.lm_cell), float(prob.lm_p), _ptr(self.R),
                          int(prob.goal), float(prob.gamma))
        self.S = int(prob.W) * int(prob.H)
        self.A = src.size // 9


def check(status: int, what: str):
    if status != QV_OK:
        raise QvError(status, what)
