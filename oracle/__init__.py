"""Plain FP64 CPU oracle for the THOI Gaussian-copula measures.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no code
with the HIP library ``paper_2501_03381_amd`` and never imports it.

The arithmetic lives in ``thoi_oracle.c`` (plain C, FP64, optional OpenMP over
n-plets); this module only compiles it with gcc, loads it with ctypes and
marshals NumPy arrays.  The top-K / histogram reducers are plain NumPy sorts over
oracle outputs.  See the header of ``thoi_oracle.c`` for the paper passages each
function follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "thoi_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

FLAG_NOT_PD = 2


def build(force: bool = False) -> str:
    """Compile ``thoi_oracle.c`` into ``liboracle.so`` with gcc (FP64, -O2, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", "-fopenmp",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    D, I, I64, P = ctypes.c_double, ctypes.c_int, ctypes.c_int64, ctypes.c_void_p
    lib.or_ndtri.argtypes, lib.or_ndtri.restype = [D], D
    lib.or_normal_score.argtypes, lib.or_normal_score.restype = [I64, I64], D
    lib.or_digamma.argtypes, lib.or_digamma.restype = [D], D
    lib.or_bias_eta.argtypes, lib.or_bias_eta.restype = [I, I64], D
    lib.or_copula.argtypes, lib.or_copula.restype = [P, I64, I64, P], I
    lib.or_covariance.argtypes, lib.or_covariance.restype = [P, I64, I64, P], None
    lib.or_lu_logdet.argtypes, lib.or_lu_logdet.restype = [P, I, ctypes.POINTER(I)], D
    lib.or_is_pd.argtypes, lib.or_is_pd.restype = [P, I], I
    lib.or_inverse.argtypes, lib.or_inverse.restype = [P, I, P], I
    lib.or_measures.argtypes, lib.or_measures.restype = [P, I, P, I, I, I64, P, P], I
    lib.or_eval_list.argtypes, lib.or_eval_list.restype = [P, I, P, I64, I, I, I64, P, P, P, I], I
    lib.or_enumerate.argtypes, lib.or_enumerate.restype = [I, I, I, P], I64
    lib.or_grad_list.argtypes, lib.or_grad_list.restype = [P, I, P, I64, I, P, P], I
    lib.or_max_threads.argtypes, lib.or_max_threads.restype = [I], I
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


# --------------------------------------------------------------------------- scalars
def ndtri(p: float) -> float:
    """Inverse standard-normal CDF (Newton on the C library's erfc)."""
    return _load().or_ndtri(float(p))


def normal_score(r: int, T: int) -> float:
    """Phi^{-1}(r / (T + 1)) for a 1-based rank r."""
    return _load().or_normal_score(int(r), int(T))


def digamma(x: float) -> float:
    return _load().or_digamma(float(x))


def bias_eta(n: int, T: int) -> float:
    """Bias corrector eta(n) of Eq. (bias_corrector), read with 1/2 on the digamma sum."""
    return _load().or_bias_eta(int(n), int(T))


def max_threads(nthreads: int = 0) -> int:
    return _load().or_max_threads(int(nthreads))


# --------------------------------------------------------------------------- copula / covariance
def copula(X: np.ndarray) -> np.ndarray:
    """Gaussian-copula transform of one dataset X [T][N] (sample-major), FP64."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    T, N = X.shape
    Z = np.empty_like(X)
    rc = _load().or_copula(_ptr(X), T, N, _ptr(Z))
    if rc != 0:
        raise ValueError("oracle copula: NaN in data or T < 2")
    return Z


def covariance(Z: np.ndarray) -> np.ndarray:
    """Mean-centred sample covariance with 1/(T-1) of Z [T][N]."""
    Z = np.ascontiguousarray(Z, dtype=np.float64)
    T, N = Z.shape
    S = np.empty((N, N), dtype=np.float64)
    _load().or_covariance(_ptr(Z), T, N, _ptr(S))
    return S


def gc_covariance(X: np.ndarray) -> np.ndarray:
    """Sigma_GC(X) of Eq. (gaussian_copula_covariance_estimator); X is [T][N]."""
    return covariance(copula(X))


# --------------------------------------------------------------------------- linear algebra
def lu_logdet(A: np.ndarray):
    """(sign, log|det A|) by LU with partial pivoting."""
    A = np.array(A, dtype=np.float64, order="C", copy=True)
    sign = ctypes.c_int(0)
    ld = _load().or_lu_logdet(_ptr(A), A.shape[0], ctypes.byref(sign))
    return sign.value, ld


def is_pd(A: np.ndarray) -> bool:
    A = np.ascontiguousarray(A, dtype=np.float64)
    return bool(_load().or_is_pd(_ptr(A), A.shape[0]))


def inverse(A: np.ndarray) -> np.ndarray:
    A = np.ascontiguousarray(A, dtype=np.float64)
    out = np.empty_like(A)
    if _load().or_inverse(_ptr(A), A.shape[0], _ptr(out)) != 0:
        raise ValueError("singular matrix")
    return out


# --------------------------------------------------------------------------- enumeration
def enumerate_nplets(N: int, kmin: int, kmax: int) -> np.ndarray:
    """All k-subsets for k = kmin..kmax, ascending order then lexicographic: [count][kmax], -1 padded."""
    lib = _load()
    n = lib.or_enumerate(N, kmin, kmax, None)
    out = np.empty((n, max(kmax, 1)), dtype=np.int32)
    lib.or_enumerate(N, kmin, kmax, _ptr(out))
    return out


def count_nplets(N: int, kmin: int, kmax: int) -> int:
    return int(_load().or_enumerate(N, kmin, kmax, None))


def pad_list(tuples, kmax: int | None = None) -> np.ndarray:
    """Pack a sequence of index tuples into a [B][kmax] int32 array padded with -1."""
    tuples = [tuple(sorted(int(v) for v in t)) for t in tuples]
    if kmax is None:
        kmax = max((len(t) for t in tuples), default=1)
    out = -np.ones((len(tuples), max(kmax, 1)), dtype=np.int32)
    for b, t in enumerate(tuples):
        out[b, : len(t)] = t
    return out


# --------------------------------------------------------------------------- measures
def measures(S: np.ndarray, idx, bias: bool = False, T: int = 0):
    """(TC, DTC, Omega, S-info), H(X^n), flag for one n-plet of covariance S."""
    S = np.ascontiguousarray(S, dtype=np.float64)
    t = np.ascontiguousarray(np.asarray(idx, dtype=np.int32))
    out = np.empty(4, dtype=np.float64)
    H = np.empty(1, dtype=np.float64)
    rc = _load().or_measures(_ptr(S), S.shape[0], _ptr(t), len(t), int(bias), int(T), _ptr(out), _ptr(H))
    if rc < 0:
        raise AssertionError("oracle: the two forms of Eq. (O-info) disagree")
    return out, float(H[0]), rc


def eval_list(S: np.ndarray, idx: np.ndarray, bias: bool = False, T: int = 0, nthreads: int = 0):
    """Measures of every row of idx [B][kmax] (-1 padded): returns out [4][B], H [B], flags [B]."""
    S = np.ascontiguousarray(S, dtype=np.float64)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    if idx.ndim == 1:
        idx = idx[None, :]
    B, kmax = idx.shape
    out = np.empty((4, B), dtype=np.float64)
    H = np.empty(B, dtype=np.float64)
    flags = np.zeros(B, dtype=np.uint8)
    rc = _load().or_eval_list(_ptr(S), S.shape[0], _ptr(idx), B, kmax, int(bias), int(T),
                              _ptr(out), _ptr(H), _ptr(flags), int(nthreads))
    if rc < 0:
        raise AssertionError("oracle: the two forms of Eq. (O-info) disagree")
    return out, H, flags


def eval_range(S: np.ndarray, kmin: int, kmax: int, bias: bool = False, T: int = 0, nthreads: int = 0):
    """Exhaustive evaluation of orders kmin..kmax in enumeration order."""
    idx = enumerate_nplets(S.shape[0], kmin, kmax)
    return eval_list(S, idx, bias=bias, T=T, nthreads=nthreads)


def grad_list(S: np.ndarray, idx: np.ndarray, w: np.ndarray) -> np.ndarray:
    """sum_b sum_m w[m][b] d measure_m(b) / d S, as an [N][N] matrix."""
    S = np.ascontiguousarray(S, dtype=np.float64)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    w = np.ascontiguousarray(w, dtype=np.float64)
    B, kmax = idx.shape
    G = np.zeros_like(S)
    if _load().or_grad_list(_ptr(S), S.shape[0], _ptr(idx), B, kmax, _ptr(w), _ptr(G)) != 0:
        raise ValueError("oracle gradient: a sub-matrix is not positive definite")
    return G


# --------------------------------------------------------------------------- reducers
def topk_per_order(omega: np.ndarray, orders: np.ndarray, g: np.ndarray, K: int):
    """Exact per-order top-K (largest) and bottom-K (smallest) Omega.

    Ties are broken by the lower global index g.  Returns {k: (top[(val, g)], bottom[(val, g)])}.
    NaN values are excluded.
    """
    res = {}
    for k in np.unique(orders):
        sel = (orders == k) & ~np.isnan(omega)
        v, gg = omega[sel], g[sel]
        top_i = np.lexsort((gg, -v))[:K]
        bot_i = np.lexsort((gg, v))[:K]
        res[int(k)] = ([(float(v[i]), int(gg[i])) for i in top_i], [(float(v[i]), int(gg[i])) for i in bot_i])
    return res


def histogram(values: np.ndarray, lo: float, hi: float, bins: int) -> np.ndarray:
    """Counts over [lo, hi] in `bins` equal bins plus [under, over]; a value equal to hi goes to the last bin."""
    v = values[~np.isnan(values)]
    out = np.zeros(bins + 2, dtype=np.int64)
    under = v < lo
    over = v > hi
    inside = v[~under & ~over]
    b = np.floor((inside - lo) / (hi - lo) * bins).astype(np.int64)
    b = np.minimum(b, bins - 1)
    np.add.at(out, b, 1)
    out[bins] = int(under.sum())
    out[bins + 1] = int(over.sum())
    return out


def objective(vals: np.ndarray, kind: str) -> np.ndarray:
    """One value per column of vals [D][B]: "mean" over the D rows, or "paired_effect" for D = 2P:
    x_p = vals[p] - vals[P + p], mean(x) / sd(x) with sd on P - 1 degrees of freedom (NaN when
    sd = 0).  NaN inputs give NaN."""
    v = np.asarray(vals, dtype=np.float64)
    if kind == "mean":
        return v.mean(axis=0)
    P = v.shape[0] // 2
    x = v[:P] - v[P:]
    m = x.mean(axis=0)
    sd = np.sqrt(((x - m) ** 2).sum(axis=0) / (P - 1))
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(sd > 0, m / sd, np.nan)
