"""Torch-facing calls of the MI355X THOI evaluator.

Torch provides device memory and the current HIP stream; every computation runs in the
hand-written kernels of ``libthoi.so`` through ``binding``.  All tensors must live on a
ROCm device (``cuda:N``); nothing here falls back to the CPU.

Typical use::

    Sigma = gc_covariance(X)                    # X: [T, N] or [D, T, N] float64 on cuda
    out, flags = nplets_measures(Sigma, orders=(3, N), precision="fp32_refine")
    tc, dtc, omega, s = out                     # each [D, B]
"""
from __future__ import annotations

import ctypes

import torch

from . import binding as B

_PREC = {"fp64": B.THOI_FP64, "fp32": B.THOI_FP32, "fp32_refine": B.THOI_FP32_REFINE}
_DT = {torch.float64: B.THOI_DTYPE_F64, torch.float32: B.THOI_DTYPE_F32}


def _ptr(t: torch.Tensor | None):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else None


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _require_device(t: torch.Tensor, name: str):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor (got {t.device})")


def _workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def device_status(ws: torch.Tensor) -> int:
    """The int32 status word a call left in its workspace (synchronises)."""
    off = B.thoi_ws_status_offset()
    return int(ws[off:off + 4].view(torch.int32).item())


def raise_on_device_status(ws: torch.Tensor, fn: str) -> None:
    st = device_status(ws)
    if st != B.THOI_OK:
        raise B.ThoiError(fn, st, B.thoi_status_string(st))


# ------------------------------------------------------------------------------------------------ copula / covariance
def copulize(X: torch.Tensor, z_dtype: torch.dtype = torch.float64, check: bool = True) -> torch.Tensor:
    """Gaussian-copula transform of X [T, N] or [D, T, N] (float64, sample-major)."""
    _require_device(X, "X")
    squeeze = X.dim() == 2
    Xd = (X[None] if squeeze else X).contiguous()
    if Xd.dtype != torch.float64:
        raise TypeError("X must be float64")
    D, T, N = Xd.shape
    Z = torch.empty((D, T, N), dtype=z_dtype, device=X.device)
    nb = B.thoi_workspace_bytes(B.THOI_WS_COPULIZE, D, T, N)
    ws = _workspace(nb, X.device)
    B.thoi_copulize(_ptr(Xd), D, T, N, _DT[z_dtype], _ptr(Z), _ptr(ws), ws.numel(), _stream(X.device))
    if check:
        raise_on_device_status(ws, "thoi_copulize")
    return Z[0] if squeeze else Z


def cov(Z: torch.Tensor) -> torch.Tensor:
    """Mean-centred covariance with 1/(T-1) of Z [T, N] or [D, T, N] -> float64 [N, N] or [D, N, N]."""
    _require_device(Z, "Z")
    squeeze = Z.dim() == 2
    Zd = (Z[None] if squeeze else Z).contiguous()
    D, T, N = Zd.shape
    S = torch.empty((D, N, N), dtype=torch.float64, device=Z.device)
    nb = B.thoi_workspace_bytes(B.THOI_WS_COV, D, T, N)
    ws = _workspace(nb, Z.device)
    B.thoi_cov(_ptr(Zd), _DT[Zd.dtype], D, T, N, _ptr(S), _ptr(ws), ws.numel(), _stream(Z.device))
    return S[0] if squeeze else S


def gc_covariance(X: torch.Tensor, z_dtype: torch.dtype = torch.float64) -> torch.Tensor:
    """Sigma_GC(X): copula transform followed by the covariance, both on the GPU."""
    return cov(copulize(X, z_dtype))


# ------------------------------------------------------------------------------------------------ selections
def range_selection(N: int, kmin: int, kmax: int, g_begin: int = 0, g_count: int | None = None) -> B.ThoiNplets:
    total = B.thoi_count(N, kmin, kmax)
    if g_count is None:
        g_count = total - g_begin
    return B.ThoiNplets(mode=B.THOI_SEL_RANGE, kmin=kmin, kmax=kmax, g_begin=g_begin, g_count=g_count,
                        idx=None, kmax_list=0, mask=None, B=0)


def list_selection(idx: torch.Tensor) -> B.ThoiNplets:
    _require_device(idx, "nplets")
    if idx.dtype != torch.int32 or idx.dim() != 2 or not idx.is_contiguous():
        raise TypeError("nplets must be a contiguous int32 [B, kmax] tensor padded with -1")
    return B.ThoiNplets(mode=B.THOI_SEL_LIST, kmin=0, kmax=0, g_begin=0, g_count=0, idx=_ptr(idx),
                        kmax_list=idx.shape[1], mask=None, B=idx.shape[0])


def mask_selection(mask: torch.Tensor) -> B.ThoiNplets:
    _require_device(mask, "masks")
    if mask.dtype != torch.int64 or mask.dim() != 1 or not mask.is_contiguous():
        raise TypeError("masks must be a contiguous int64 [B] tensor (bit j selects variable j)")
    return B.ThoiNplets(mode=B.THOI_SEL_MASK, kmin=0, kmax=0, g_begin=0, g_count=0, idx=None, kmax_list=0,
                        mask=_ptr(mask), B=mask.shape[0])


def _n_out(sel: B.ThoiNplets) -> int:
    return sel.g_count if sel.mode == B.THOI_SEL_RANGE else sel.B


_ENGINE = {"auto": B.THOI_ENGINE_AUTO, "factor": B.THOI_ENGINE_FACTOR, "prefix": B.THOI_ENGINE_PREFIX}


def make_opts(precision: str = "fp32_refine", out_dtype: torch.dtype = torch.float32, vif_tau: float = 1e3,
              bias_correct: bool = False, T: int = 0, write_entropy: bool = False, seg_tiles: int = 0,
              grid_blocks: int = 0, engine: str = "auto", class_seg_tiles=None, class_lanes=None) -> B.ThoiEvalOpts:
    """Evaluation options; engine: "auto", "factor" (one factorisation per n-plet) or "prefix"
    (prefix sharing for the whole orders of a RANGE selection).  class_seg_tiles / class_lanes:
    per register class of a RANGE selection, tiles per workgroup and n-plets per lane (0 = the
    library's choice; see tune.py)."""
    o = B.ThoiEvalOpts(precision=_PREC[precision], out_dtype=_DT[out_dtype], vif_tau=float(vif_tau),
                       bias_correct=int(bool(bias_correct)), T=int(T), write_entropy=int(bool(write_entropy)),
                       reduce=None, seg_tiles=int(seg_tiles), grid_blocks=int(grid_blocks),
                       engine=_ENGINE[engine])
    for c, v in enumerate(class_seg_tiles or ()):
        o.class_seg_tiles[c] = int(v)
    for c, v in enumerate(class_lanes or ()):
        o.class_lanes[c] = int(v)
    return o


def _untuned(opts: B.ThoiEvalOpts) -> bool:
    return opts.seg_tiles == 0 and not any(opts.class_seg_tiles) and not any(opts.class_lanes)


# ------------------------------------------------------------------------------------------------ evaluation
class Evaluator:
    """Reusable evaluation of one selection against D covariance matrices of N variables.

    Holds the output, flag and workspace buffers so that repeated calls allocate nothing.
    """

    def __init__(self, D: int, N: int, sel: B.ThoiNplets, opts: B.ThoiEvalOpts, device, out_dtype=torch.float32,
                 keep=(), tuned: bool = True):
        if tuned and sel.mode == B.THOI_SEL_RANGE and _untuned(opts):
            # per-class launch knobs from the autotuner's cache, when it holds this shape
            from . import tune
            knobs = tune.lookup_range(device, opts.precision, N, D)
            if knobs is not None:
                opts = B.ThoiEvalOpts.from_buffer_copy(opts)
                for c in range(8):
                    opts.class_seg_tiles[c], opts.class_lanes[c] = knobs[0][c], knobs[1][c]
        self.D, self.N, self.sel, self.opts = D, N, sel, opts
        self.keep = keep  # tensors the selection points to
        self.nout = _n_out(sel)
        planes = 5 if opts.write_entropy else 4
        self.out = torch.empty((planes, D, self.nout), dtype=out_dtype, device=device)
        self.flags = torch.empty((D, self.nout), dtype=torch.uint8, device=device)
        nb = B.thoi_workspace_bytes(B.THOI_WS_EVAL, D, 0, N, sel, opts)
        self.ws = _workspace(nb, device)
        self.device = device

    def __call__(self, Sigma: torch.Tensor, stream=None):
        S = Sigma if Sigma.dim() == 3 else Sigma[None]
        if S.dtype != torch.float64 or not S.is_contiguous() or tuple(S.shape) != (self.D, self.N, self.N):
            raise TypeError(f"Sigma must be contiguous float64 [{self.D}, {self.N}, {self.N}]")
        st = ctypes.c_void_p(stream) if stream is not None else _stream(self.device)
        B.thoi_nplets_eval(_ptr(S), self.D, self.N, self.sel, self.opts, _ptr(self.out), _ptr(self.flags),
                           _ptr(self.ws), self.ws.numel(), st)
        return self.out, self.flags

    def refine_count(self) -> int:
        """Number of n-plets the last FP32_REFINE call re-evaluated in FP64 (synchronises)."""
        return int(self.ws[4:8].view(torch.int32).item())

    def status(self) -> int:
        return device_status(self.ws)


def nplets_measures(Sigma: torch.Tensor, *, orders: tuple[int, int] | None = None,
                    g_range: tuple[int, int] | None = None, nplets: torch.Tensor | None = None,
                    masks: torch.Tensor | None = None, precision: str = "fp32_refine",
                    out_dtype: torch.dtype = torch.float32, vif_tau: float = 1e3, bias_correct: bool = False,
                    T: int = 0, write_entropy: bool = False, check: bool = True, engine: str = "auto"):
    """(TC, DTC, Omega, S[, H]) of every selected n-plet for every covariance matrix.

    Sigma: float64 [N, N] or [D, N, N] on the device.  Select with exactly one of
      orders=(kmin, kmax)           all n-plets of those orders (RANGE, optional g_range=(begin, count)),
      nplets=int32 [B, kmax] tensor ascending indices padded with -1 (LIST),
      masks=int64 [B] tensor        bit masks over N <= 64 variables (MASK).
    Returns (out [4 or 5, D, B], flags [D, B] uint8).
    """
    _require_device(Sigma, "Sigma")
    S = (Sigma[None] if Sigma.dim() == 2 else Sigma).contiguous()
    D, N, _ = S.shape
    keep = ()
    if (orders is not None) + (nplets is not None) + (masks is not None) != 1:
        raise ValueError("give exactly one of orders=, nplets=, masks=")
    if orders is not None:
        kmin, kmax = orders
        if g_range is None:
            sel = range_selection(N, kmin, kmax)
        else:
            sel = range_selection(N, kmin, kmax, g_range[0], g_range[1])
    elif nplets is not None:
        nplets = nplets.contiguous()
        sel, keep = list_selection(nplets), (nplets,)
    else:
        masks = masks.contiguous()
        sel, keep = mask_selection(masks), (masks,)
    opts = make_opts(precision, out_dtype, vif_tau, bias_correct, T, write_entropy, engine=engine)
    ev = Evaluator(D, N, sel, opts, S.device, out_dtype, keep)
    out, flags = ev(S)
    if check:
        raise_on_device_status(ev.ws, "thoi_nplets_eval")
    if Sigma.dim() == 2:
        return out[:, 0], flags[0]
    return out, flags


# ------------------------------------------------------------------------------------------------ uneven datasets
def pack_covariances(Sigmas) -> tuple[torch.Tensor, list[int]]:
    """Concatenate square float64 device matrices of different sizes (the multi-dataset layout)."""
    Ns = [int(S.shape[0]) for S in Sigmas]
    flat = torch.cat([S.contiguous().reshape(-1) for S in Sigmas]) if Sigmas else torch.empty(0, dtype=torch.float64)
    return flat, Ns


class MultiEvaluator:
    """All n-plets of orders kmin..kmax of D datasets of uneven size, one persistent launch per
    register class (thoi_nplets_eval_multi).  Output [P, total]; dataset d is the slice
    offsets[d]:offsets[d+1]."""

    def __init__(self, N_d, kmin: int, kmax: int, device, precision: str = "fp32_refine",
                 out_dtype: torch.dtype = torch.float32, T_d=None, bias_correct: bool = False,
                 write_entropy: bool = False, seg_tiles: int = 0, grid_blocks: int = 0, reduce_state=None):
        import numpy as np
        self.N_d = np.ascontiguousarray(N_d, dtype=np.int32)
        self.T_d = None if T_d is None else np.ascontiguousarray(T_d, dtype=np.int32)
        self.D, self.kmin, self.kmax = len(self.N_d), kmin, kmax
        self.offsets = B.thoi_multi_offsets(self.N_d, kmin, kmax)
        self.total = int(self.offsets[-1])
        if seg_tiles == 0 and grid_blocks == 0 and len(self.N_d) > 0:
            # launch knobs from the autotuner's cache, when it holds this shape
            from . import tune
            knobs = tune.lookup_multi(device, _PREC[precision], self.N_d, kmin, kmax)
            if knobs is not None:
                seg_tiles, grid_blocks = knobs
        self.opts = make_opts(precision, out_dtype, 1e3, bias_correct, 0, write_entropy, seg_tiles, grid_blocks)
        self.reduce_state = reduce_state
        if reduce_state is not None:
            self.opts.reduce = ctypes.pointer(reduce_state.struct)
        planes = 5 if write_entropy else 4
        self.out = None if reduce_state is not None else torch.empty((planes, self.total), dtype=out_dtype,
                                                                      device=device)
        self.flags = torch.empty(self.total, dtype=torch.uint8, device=device)
        nb = B.thoi_multi_workspace_bytes(self.N_d.ctypes.data_as(ctypes.c_void_p), self.D, kmin, kmax, self.opts)
        self.ws = _workspace(nb, device)
        self.device = device

    def __call__(self, Sigma_packed: torch.Tensor, stream=None):
        st = ctypes.c_void_p(stream) if stream is not None else _stream(self.device)
        Tp = self.T_d.ctypes.data_as(ctypes.c_void_p) if self.T_d is not None else None
        B.thoi_nplets_eval_multi(_ptr(Sigma_packed), self.N_d.ctypes.data_as(ctypes.c_void_p), Tp, self.D, self.kmin,
                                 self.kmax, self.opts, _ptr(self.out), _ptr(self.flags), _ptr(self.ws),
                                 self.ws.numel(), st)
        return self.out, self.flags

    def status(self) -> int:
        return device_status(self.ws)


def nplets_measures_multi(Sigmas, kmin: int, kmax: int, *, precision: str = "fp32_refine",
                          out_dtype: torch.dtype = torch.float32, T_d=None, bias_correct: bool = False,
                          write_entropy: bool = False, check: bool = True):
    """(out [P, total], flags [total], offsets [D+1]) for a list of float64 [N_d, N_d] device matrices."""
    flat, Ns = pack_covariances(Sigmas)
    ev = MultiEvaluator(Ns, kmin, kmax, flat.device, precision, out_dtype, T_d, bias_correct, write_entropy)
    out, flags = ev(flat)
    if check:
        raise_on_device_status(ev.ws, "thoi_nplets_eval_multi")
    return out, flags, ev.offsets


# ------------------------------------------------------------------------------------------------ streaming reduction
class ReduceState:
    """Per-(dataset, order) top-K / bottom-K Omega lists and Omega histograms, accumulated across
    calls of ``nplets_reduce`` (so an enumeration can be split into RANGE pieces).

    top_val, top_g: [D, kmax+1, 2, topk] (slot 0: largest Omega descending, slot 1: smallest
    ascending; g = -1 for unused slots).  hist: [D, kmax+1, bins+2] (bins, then under, over).
    """

    def __init__(self, D: int, kmax: int, topk: int, hist_bins: int, hist_range, device):
        import numpy as np
        self.D, self.kmax, self.topk, self.bins = D, kmax, topk, hist_bins
        K = max(topk, 1)
        self.top_val = torch.empty((D, kmax + 1, 2, K), dtype=torch.float64, device=device)
        self.top_g = torch.empty((D, kmax + 1, 2, K), dtype=torch.int64, device=device)
        self.hist = torch.empty((D, kmax + 1, max(hist_bins, 0) + 2), dtype=torch.int64, device=device)
        lohi = np.zeros((kmax + 1, 2), dtype=np.float64)
        if hist_bins > 0:
            r = np.asarray(hist_range, dtype=np.float64)
            lohi[:] = r if r.ndim == 2 else r[None, :]
        self.lohi = np.ascontiguousarray(lohi)
        self.struct = B.ThoiReduce(topk=topk, hist_bins=hist_bins,
                                   hist_lo_hi=self.lohi.ctypes.data_as(ctypes.c_void_p),
                                   top_val=_ptr(self.top_val), top_g=_ptr(self.top_g), hist=_ptr(self.hist))
        B.thoi_reduce_init(self.struct, D, kmax, _stream(device))

    def result(self):
        """Host copies: (top_val, top_g, hist) as NumPy arrays (synchronises)."""
        return self.top_val.cpu().numpy(), self.top_g.cpu().numpy(), self.hist.cpu().numpy()


def nplets_reduce(Sigma: torch.Tensor, *, orders=None, g_range=None, nplets=None, masks=None, topk: int = 100,
                  hist_bins: int = 256, hist_range=(-10.0, 10.0), precision: str = "fp32_refine",
                  vif_tau: float = 1e3, bias_correct: bool = False, T: int = 0, state: ReduceState | None = None,
                  flags: torch.Tensor | None = None, check: bool = True, engine: str = "auto") -> ReduceState:
    """Streaming reduction of Omega over the selected n-plets (no per-n-plet output).

    hist_range: (lo, hi) for every order, or an array [kmax+1, 2].  Pass `state` from an
    earlier call to accumulate (e.g. consecutive g_range pieces of one enumeration).
    """
    _require_device(Sigma, "Sigma")
    S = (Sigma[None] if Sigma.dim() == 2 else Sigma).contiguous()
    D, N, _ = S.shape
    sel, keep = _selection(N, orders, g_range, nplets, masks)
    if sel.mode == B.THOI_SEL_RANGE:
        kmax = sel.kmax
    elif sel.mode == B.THOI_SEL_LIST:
        kmax = min(sel.kmax_list, B.THOI_MAX_K)
    else:
        kmax = min(N, B.THOI_MAX_K)
    if state is None:
        state = ReduceState(D, kmax, topk, hist_bins, hist_range, S.device)
    if (state.D, state.kmax) != (D, kmax):
        raise ValueError("state does not match this selection")
    opts = make_opts(precision, torch.float32, vif_tau, bias_correct, T, False, engine=engine)
    opts.reduce = ctypes.pointer(state.struct)
    nb = B.thoi_workspace_bytes(B.THOI_WS_EVAL, D, 0, N, sel, opts)
    ws = _workspace(nb, S.device)
    B.thoi_nplets_eval(_ptr(S), D, N, sel, opts, None, _ptr(flags), _ptr(ws), ws.numel(), _stream(S.device))
    if check:
        raise_on_device_status(ws, "thoi_nplets_eval")
    del keep
    return state


# ------------------------------------------------------------------------------------------------ objectives over datasets
OBJECTIVES = {"mean": B.THOI_OBJ_MEAN, "paired_effect": B.THOI_OBJ_PAIRED_EFFECT}


def objective(vals: torch.Tensor, kind: str = "mean", *, write: bool = True, topk: int = 0, hist_bins: int = 0,
              hist_range=(-10.0, 10.0), state: ReduceState | None = None):
    """One value per n-plet from its values in D datasets (thoi_objective).

    vals: [D, B] float64 or float32 on the device (e.g. one plane of nplets_measures' output).
    kind: "mean" or "paired_effect" (datasets p and D/2 + p paired).
    Returns (obj [B] float64 or None, ReduceState or None); topk / hist_bins > 0 (or state=) streams
    the objective into a one-list reducer (kmax = 0) that merges across calls.
    """
    _require_device(vals, "vals")
    v = vals.contiguous()
    if v.dim() != 2 or v.dtype not in (torch.float64, torch.float32):
        raise TypeError("vals must be a [D, B] float64 or float32 tensor")
    D, Bn = v.shape
    dt = B.THOI_DTYPE_F64 if v.dtype == torch.float64 else B.THOI_DTYPE_F32
    obj = torch.empty(Bn, dtype=torch.float64, device=v.device) if write else None
    if state is None and (topk > 0 or hist_bins > 0):
        state = ReduceState(1, 0, topk, hist_bins, hist_range, v.device)
    red = state.struct if state is not None else None
    ws = _workspace(B.thoi_objective_workspace_bytes(D, Bn, red), v.device)
    B.thoi_objective(_ptr(v), dt, D, Bn, OBJECTIVES[kind], _ptr(obj), red, _ptr(ws), ws.numel(), _stream(v.device))
    return obj, state


# ------------------------------------------------------------------------------------------------ differentiation
def _selection(N, orders, g_range, nplets, masks):
    if (orders is not None) + (nplets is not None) + (masks is not None) != 1:
        raise ValueError("give exactly one of orders=, nplets=, masks=")
    if orders is not None:
        kmin, kmax = orders
        if g_range is None:
            return range_selection(N, kmin, kmax), ()
        return range_selection(N, kmin, kmax, g_range[0], g_range[1]), ()
    if nplets is not None:
        nplets = nplets.contiguous()
        return list_selection(nplets), (nplets,)
    masks = masks.contiguous()
    return mask_selection(masks), (masks,)


def measures_backward(Sigma: torch.Tensor, grad_out: torch.Tensor, *, orders=None, g_range=None, nplets=None,
                      masks=None, grad_Sigma: torch.Tensor | None = None) -> torch.Tensor:
    """grad_Sigma [D, N, N] (float32, accumulated) += sum_b sum_m grad_out[m, d, b] d measure_m / d Sigma_d.

    Entries of Sigma are treated as independent; the result is symmetric.
    """
    _require_device(Sigma, "Sigma")
    S = (Sigma[None] if Sigma.dim() == 2 else Sigma).contiguous()
    D, N, _ = S.shape
    sel, keep = _selection(N, orders, g_range, nplets, masks)
    g = grad_out.to(torch.float32)
    if g.dim() == 2:
        g = g[:, None]
    g = g.contiguous()
    if tuple(g.shape) != (4, D, _n_out(sel)):
        raise ValueError(f"grad_out must be [4, {D}, {_n_out(sel)}]")
    if grad_Sigma is None:
        grad_Sigma = torch.zeros((D, N, N), dtype=torch.float32, device=S.device)
    opts = make_opts("fp64", torch.float64)
    ws = _workspace(B.thoi_workspace_bytes(B.THOI_WS_BACKWARD, D, 0, N, sel, opts), S.device)
    B.thoi_nplets_eval_backward(_ptr(S), D, N, sel, opts, _ptr(g), _ptr(grad_Sigma), _ptr(ws), ws.numel(),
                                _stream(S.device))
    del keep
    return grad_Sigma


class NpletsMeasures(torch.autograd.Function):
    """(TC, DTC, Omega, S) of the selected n-plets as a differentiable function of Sigma.

    forward runs thoi_nplets_eval; backward runs the hand-written adjoint
    thoi_nplets_eval_backward (FP64 factorisation and inverse, FP32 quadratic part and accumulation).
    """

    @staticmethod
    def forward(ctx, Sigma, orders=None, g_range=None, nplets=None, masks=None, precision="fp32_refine",
                out_dtype=torch.float32):
        out, _ = nplets_measures(Sigma, orders=orders, g_range=g_range, nplets=nplets, masks=masks,
                                 precision=precision, out_dtype=out_dtype)
        ctx.save_for_backward(Sigma)
        ctx.sel = (orders, g_range, nplets, masks)
        return out[:4]

    @staticmethod
    def backward(ctx, grad_out):
        (Sigma,) = ctx.saved_tensors
        orders, g_range, nplets, masks = ctx.sel
        g = measures_backward(Sigma, grad_out, orders=orders, g_range=g_range, nplets=nplets, masks=masks)
        g = g.to(Sigma.dtype)
        if Sigma.dim() == 2:
            g = g[0]
        return g, None, None, None, None, None, None


def nplets_measures_autograd(Sigma, *, orders=None, g_range=None, nplets=None, masks=None,
                             precision="fp32_refine", out_dtype=torch.float32):
    return NpletsMeasures.apply(Sigma, orders, g_range, nplets, masks, precision, out_dtype)


# ------------------------------------------------------------------------------------------------ host helpers
count = B.thoi_count
unrank = B.thoi_unrank_host
bias_offsets = B.thoi_bias_offsets
