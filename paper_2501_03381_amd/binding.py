"""ctypes binding of libthoi.so: argument marshalling only, no arithmetic.

Mirrors ``include/thoi.h`` one to one (same function names, same struct layouts).  The
library is loaded from the package directory; if it is missing the first call raises
instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libthoi.so")

THOI_OK = 0
THOI_EINVAL = -1
THOI_EUNSUPPORTED = -2
THOI_EWORKSPACE = -3
THOI_EHIP = -4
THOI_EINVAL_DATA = -5

THOI_FP64, THOI_FP32, THOI_FP32_REFINE = 0, 1, 2
THOI_DTYPE_F64, THOI_DTYPE_F32 = 0, 1
THOI_SEL_RANGE, THOI_SEL_LIST, THOI_SEL_MASK = 0, 1, 2
THOI_NPLET_REFINED, THOI_NPLET_NOT_PD = 1, 2
THOI_WS_COPULIZE, THOI_WS_COV, THOI_WS_EVAL, THOI_WS_BACKWARD = 0, 1, 2, 3
THOI_OBJ_MEAN, THOI_OBJ_PAIRED_EFFECT = 0, 1
THOI_ENGINE_AUTO, THOI_ENGINE_FACTOR, THOI_ENGINE_PREFIX = 0, 1, 2
THOI_MAX_N_RANGE = 62
THOI_MAX_N = 128
THOI_MAX_K = 64
THOI_NOALLOC_SCRATCH_BYTES = 32 << 20

EXPORTS = [
    "thoi_copulize", "thoi_cov", "thoi_nplets_eval", "thoi_nplets_eval_backward", "thoi_reduce_init",
    "thoi_workspace_bytes", "thoi_ws_status_offset", "thoi_count", "thoi_unrank_host", "thoi_bias_offsets",
    "thoi_status_string", "thoi_version", "thoi_nplets_eval_multi", "thoi_multi_offsets",
    "thoi_multi_workspace_bytes", "thoi_objective", "thoi_objective_workspace_bytes", "thoi_eval_launch_shape",
    "thoi_nplets_eval_noalloc", "thoi_anneal", "thoi_greedy", "thoi_greedy_workspace_bytes",
]


class ThoiNplets(ctypes.Structure):
    _fields_ = [
        ("mode", ctypes.c_int32),
        ("kmin", ctypes.c_int32),
        ("kmax", ctypes.c_int32),
        ("g_begin", ctypes.c_int64),
        ("g_count", ctypes.c_int64),
        ("idx", ctypes.c_void_p),
        ("kmax_list", ctypes.c_int32),
        ("mask", ctypes.c_void_p),
        ("B", ctypes.c_int64),
    ]


class ThoiReduce(ctypes.Structure):
    _fields_ = [
        ("topk", ctypes.c_int32),
        ("hist_bins", ctypes.c_int32),
        ("hist_lo_hi", ctypes.c_void_p),
        ("top_val", ctypes.c_void_p),
        ("top_g", ctypes.c_void_p),
        ("hist", ctypes.c_void_p),
    ]


class ThoiEvalOpts(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int32),
        ("out_dtype", ctypes.c_int32),
        ("vif_tau", ctypes.c_double),
        ("bias_correct", ctypes.c_int32),
        ("T", ctypes.c_int32),
        ("write_entropy", ctypes.c_int32),
        ("reduce", ctypes.POINTER(ThoiReduce)),
        ("seg_tiles", ctypes.c_int32),
        ("grid_blocks", ctypes.c_int32),
        ("engine", ctypes.c_int32),
        ("class_seg_tiles", ctypes.c_int32 * 8),
        ("class_lanes", ctypes.c_int32 * 8),
    ]


class ThoiError(RuntimeError):
    def __init__(self, fn: str, status: int, msg: str):
        super().__init__(f"{fn}: {msg} (status {status})")
        self.status = status


_lib = None


def lib():
    """Load libthoi.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libthoi.so is not built ({LIB_PATH}); run `python -m paper_2501_03381_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    P, I32, I64, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    NP, OP = ctypes.POINTER(ThoiNplets), ctypes.POINTER(ThoiEvalOpts)
    L.thoi_copulize.argtypes = [P, I64, I64, I64, I32, P, P, SZ, P]
    L.thoi_cov.argtypes = [P, I32, I64, I64, I64, P, P, SZ, P]
    L.thoi_nplets_eval.argtypes = [P, I64, I32, NP, OP, P, P, P, SZ, P]
    L.thoi_nplets_eval_backward.argtypes = [P, I64, I32, NP, OP, P, P, P, SZ, P]
    L.thoi_nplets_eval_noalloc.argtypes = [P, I64, I32, NP, OP, P, P, P, P]
    L.thoi_reduce_init.argtypes = [ctypes.POINTER(ThoiReduce), I64, I32, P]
    L.thoi_workspace_bytes.argtypes = [I32, I64, I64, I32, NP, OP]
    L.thoi_workspace_bytes.restype = SZ
    L.thoi_ws_status_offset.argtypes = []
    L.thoi_ws_status_offset.restype = SZ
    L.thoi_count.argtypes = [I32, I32, I32]
    L.thoi_count.restype = I64
    L.thoi_unrank_host.argtypes = [I32, I32, I64, ctypes.POINTER(I32), ctypes.POINTER(I32)]
    L.thoi_bias_offsets.argtypes = [I32, I32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_double)]
    L.thoi_status_string.argtypes = [I32]
    L.thoi_status_string.restype = ctypes.c_char_p
    L.thoi_nplets_eval_multi.argtypes = [P, P, P, I64, I32, I32, OP, P, P, P, SZ, P]
    L.thoi_multi_offsets.argtypes = [P, I64, I32, I32, P]
    L.thoi_multi_workspace_bytes.argtypes = [P, I64, I32, I32, OP]
    L.thoi_multi_workspace_bytes.restype = SZ
    L.thoi_objective.argtypes = [P, I32, I64, I64, I32, P, ctypes.POINTER(ThoiReduce), P, SZ, P]
    L.thoi_objective_workspace_bytes.argtypes = [I64, I64, ctypes.POINTER(ThoiReduce)]
    L.thoi_objective_workspace_bytes.restype = SZ
    L.thoi_eval_launch_shape.argtypes = [I32, NP, OP, ctypes.POINTER(I32), ctypes.POINTER(I64)]
    D = ctypes.c_double
    L.thoi_anneal.argtypes = [P, I32, P, I32, I32, P, P, P, P, D, D, I32, I32, I32, I32, P, P, P, P, P, P]
    L.thoi_greedy.argtypes = [P, I64, I32, I32, I32, I32, I32, I32, I32, P, P, P, P, SZ, P]
    L.thoi_greedy_workspace_bytes.argtypes = [I64, I32, I32]
    L.thoi_greedy_workspace_bytes.restype = SZ
    L.thoi_version.argtypes = []
    L.thoi_version.restype = ctypes.c_char_p
    for fn in ("thoi_copulize", "thoi_cov", "thoi_nplets_eval", "thoi_nplets_eval_backward", "thoi_reduce_init",
               "thoi_unrank_host", "thoi_bias_offsets", "thoi_nplets_eval_multi", "thoi_multi_offsets",
               "thoi_objective", "thoi_eval_launch_shape", "thoi_nplets_eval_noalloc", "thoi_anneal", "thoi_greedy"):
        getattr(L, fn).restype = I32
    _lib = L
    return L


def check(fn: str, status: int) -> None:
    if status != THOI_OK:
        raise ThoiError(fn, status, lib().thoi_status_string(status).decode())


# ---------------------------------------------------------------------------- thin wrappers, same names
def thoi_copulize(X, D, T, N, z_dtype, Z, ws, ws_bytes, stream):
    check("thoi_copulize", lib().thoi_copulize(X, D, T, N, z_dtype, Z, ws, ws_bytes, stream))


def thoi_cov(Z, z_dtype, D, T, N, Sigma, ws, ws_bytes, stream):
    check("thoi_cov", lib().thoi_cov(Z, z_dtype, D, T, N, Sigma, ws, ws_bytes, stream))


def thoi_nplets_eval(Sigma, D, N, sel: ThoiNplets, opts: ThoiEvalOpts, out, flags, ws, ws_bytes, stream):
    check("thoi_nplets_eval", lib().thoi_nplets_eval(Sigma, D, N, ctypes.byref(sel), ctypes.byref(opts), out, flags,
                                                     ws, ws_bytes, stream))


def thoi_nplets_eval_noalloc(Sigma, D, N, sel: ThoiNplets, opts: ThoiEvalOpts, out, flags, status, stream):
    check("thoi_nplets_eval_noalloc", lib().thoi_nplets_eval_noalloc(Sigma, D, N, ctypes.byref(sel),
                                                                     ctypes.byref(opts), out, flags, status, stream))


def thoi_nplets_eval_backward(Sigma, D, N, sel: ThoiNplets, opts: ThoiEvalOpts, grad_out, grad_Sigma, ws, ws_bytes,
                              stream):
    check("thoi_nplets_eval_backward",
          lib().thoi_nplets_eval_backward(Sigma, D, N, ctypes.byref(sel), ctypes.byref(opts), grad_out, grad_Sigma,
                                          ws, ws_bytes, stream))


def thoi_reduce_init(red: ThoiReduce, D, kmax, stream):
    check("thoi_reduce_init", lib().thoi_reduce_init(ctypes.byref(red), D, kmax, stream))


def thoi_nplets_eval_multi(Sigma, N_d, T_d, D, kmin, kmax, opts: ThoiEvalOpts, out, flags, ws, ws_bytes, stream):
    check("thoi_nplets_eval_multi", lib().thoi_nplets_eval_multi(Sigma, N_d, T_d, D, kmin, kmax, ctypes.byref(opts),
                                                                 out, flags, ws, ws_bytes, stream))


def thoi_multi_offsets(N_d, kmin: int, kmax: int):
    """Host: exclusive prefix sums of per-dataset counts (length D + 1)."""
    import numpy as np
    Nd = np.ascontiguousarray(N_d, dtype=np.int32)
    off = np.zeros(len(Nd) + 1, dtype=np.int64)
    check("thoi_multi_offsets", lib().thoi_multi_offsets(Nd.ctypes.data_as(ctypes.c_void_p), len(Nd), kmin, kmax,
                                                         off.ctypes.data_as(ctypes.c_void_p)))
    return off


def thoi_multi_workspace_bytes(N_d, D, kmin, kmax, opts: ThoiEvalOpts) -> int:
    return int(lib().thoi_multi_workspace_bytes(N_d, D, kmin, kmax, ctypes.byref(opts)))


def thoi_objective(vals, val_dtype, D, B, kind, obj, red, ws, ws_bytes, stream):
    check("thoi_objective", lib().thoi_objective(vals, val_dtype, D, B, kind, obj,
                                                 ctypes.byref(red) if red is not None else None, ws, ws_bytes,
                                                 stream))


def thoi_anneal(Sigma, N, masks0, kappa, iters, move, a, b, accept, T0, alpha, maximize, across, k_min, k_max,
                cur_mask, cur_omega, best_mask, best_omega, accepted, stream):
    check("thoi_anneal", lib().thoi_anneal(Sigma, N, masks0, kappa, iters, move, a, b, accept, T0, alpha, maximize,
                                           across, k_min, k_max, cur_mask, cur_omega, best_mask, best_omega,
                                           accepted, stream))


def thoi_greedy(Sigma, D, N, k_first, steps, kappa, measure, kind, maximize, sols, vals, count, ws, ws_bytes,
                stream):
    check("thoi_greedy", lib().thoi_greedy(Sigma, D, N, k_first, steps, kappa, measure, kind, maximize, sols, vals,
                                           count, ws, ws_bytes, stream))


def thoi_greedy_workspace_bytes(D, N, kappa) -> int:
    return int(lib().thoi_greedy_workspace_bytes(D, N, kappa))


def thoi_objective_workspace_bytes(D, B, red=None) -> int:
    return int(lib().thoi_objective_workspace_bytes(D, B, ctypes.byref(red) if red is not None else None))


def thoi_eval_launch_shape(N, sel: ThoiNplets, opts: ThoiEvalOpts):
    """Host: (number of engine launches, largest work-items along x) of thoi_nplets_eval."""
    n, m = ctypes.c_int32(0), ctypes.c_int64(0)
    check("thoi_eval_launch_shape", lib().thoi_eval_launch_shape(N, ctypes.byref(sel), ctypes.byref(opts),
                                                                 ctypes.byref(n), ctypes.byref(m)))
    return n.value, m.value


def thoi_workspace_bytes(which, D, T, N, sel=None, opts=None) -> int:
    return int(lib().thoi_workspace_bytes(which, D, T, N, ctypes.byref(sel) if sel is not None else None,
                                          ctypes.byref(opts) if opts is not None else None))


def thoi_ws_status_offset() -> int:
    return int(lib().thoi_ws_status_offset())


def thoi_count(N: int, kmin: int, kmax: int) -> int:
    return int(lib().thoi_count(N, kmin, kmax))


def thoi_unrank_host(N: int, kmin: int, g: int):
    k = ctypes.c_int32(0)
    idx = (ctypes.c_int32 * THOI_MAX_K)()
    check("thoi_unrank_host", lib().thoi_unrank_host(N, kmin, g, ctypes.byref(k), idx))
    return tuple(idx[i] for i in range(k.value))


def thoi_bias_offsets(k: int, T: int):
    a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    check("thoi_bias_offsets", lib().thoi_bias_offsets(k, T, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return a.value, b.value, c.value


def thoi_status_string(s: int) -> str:
    return lib().thoi_status_string(s).decode()


def thoi_version() -> str:
    return lib().thoi_version().decode()
