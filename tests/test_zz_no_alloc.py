"""GPU: thoi_nplets_eval_noalloc (library-owned workspace, nothing allocated per call) against
thoi_nplets_eval with a caller workspace, through the C ABI.

Both calls run the same kernels on the same inputs, so outputs, flags, reducer lists and
histograms must be bitwise equal; the device status word returned by the workspace-free call
must equal the one left in the caller's workspace.  The calls run back to back with shrinking
inputs so that each one starts from what the previous one left in the shared scratch array.
"""
import ctypes
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env(orc):
    import torch
    from paper_2501_03381_amd import api, binding, synth
    binding.lib()
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return torch, api, binding, synth, orc


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _both(torch, B, Sigma, D, N, sel, opts, nplanes, out_dtype, reduce_pair=None):
    """Run the evaluation with a caller workspace and without; returns both results as NumPy."""
    dev = Sigma.device
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    Bn = sel.g_count if sel.mode == B.THOI_SEL_RANGE else sel.B
    res = []
    for which in ("ws", "noalloc"):
        out = torch.full((nplanes, D, Bn), float("nan"), dtype=out_dtype, device=dev) if reduce_pair is None else None
        flags = torch.full((D, Bn), 255, dtype=torch.uint8, device=dev)
        o = opts
        red = None
        if reduce_pair is not None:
            red, keep = reduce_pair(which)
            o = B.ThoiEvalOpts(**{f: getattr(opts, f) for f, _ in B.ThoiEvalOpts._fields_})
            o.reduce = ctypes.pointer(red)
            B.thoi_reduce_init(red, D, sel.kmax, stream)
        if which == "ws":
            nb = B.thoi_workspace_bytes(B.THOI_WS_EVAL, D, 0, N, sel, o)
            ws = torch.empty(nb, dtype=torch.uint8, device=dev)
            B.thoi_nplets_eval(_p(Sigma), D, N, sel, o, _p(out), _p(flags), _p(ws), nb, stream)
            torch.cuda.synchronize()
            status = int(ws[:4].cpu().view(torch.int32)[0])
        else:
            st = torch.full((1,), 12345, dtype=torch.int32, device=dev)
            B.thoi_nplets_eval_noalloc(_p(Sigma), D, N, sel, o, _p(out), _p(flags), _p(st), stream)
            torch.cuda.synchronize()
            status = int(st.cpu()[0])
        r = {"flags": flags.cpu().numpy(), "status": status}
        if out is not None:
            r["out"] = out.cpu().numpy()
        if reduce_pair is not None:
            r["top_val"], r["top_g"], r["hist"] = (keep[0].cpu().numpy(), keep[1].cpu().numpy(),
                                                   keep[2].cpu().numpy())
        res.append(r)
    return res


def _assert_bitwise(a, b, what):
    for key in a:
        x, y = np.asarray(a[key]), np.asarray(b[key])
        if x.dtype.kind == "f":
            assert np.array_equal(x.view(np.uint8), y.view(np.uint8)), f"{what}: {key} differs"
        else:
            assert np.array_equal(x, y), f"{what}: {key} differs"


def test_noalloc_matches_workspace_call_on_shrinking_inputs(env):
    torch, api, B, synth, orc = env
    dev = torch.device("cuda:0")

    # 1. N = 20, all orders 3..20, FP32 with FP64 refinement; a near-duplicate column pair makes
    #    2^18 n-plets go through the refinement queue in the scratch array.
    X = synth.latent_20()
    rng = np.random.default_rng(11)
    X[:, 1] = X[:, 0] + 1e-4 * rng.standard_normal(X.shape[0])
    Sigma = api.gc_covariance(torch.from_numpy(X).to(dev))
    sel = B.ThoiNplets(mode=B.THOI_SEL_RANGE, kmin=3, kmax=20, g_begin=0, g_count=B.thoi_count(20, 3, 20))
    opts = B.ThoiEvalOpts(precision=B.THOI_FP32_REFINE, out_dtype=B.THOI_DTYPE_F32, vif_tau=1e3)
    assert B.thoi_workspace_bytes(B.THOI_WS_EVAL, 1, 0, 20, sel, opts) <= B.THOI_NOALLOC_SCRATCH_BYTES
    say("noalloc call 1: N=20 orders 3..20 fp32_refine, near-duplicate pair")
    a, b = _both(torch, B, Sigma, 1, 20, sel, opts, 4, torch.float32)
    _assert_bitwise(a, b, "N=20 fp32_refine")
    assert a["status"] == B.THOI_OK
    assert int(np.count_nonzero(a["flags"] & B.THOI_NPLET_REFINED)) >= 2 ** 18 - 20   # refinement ran

    # 2. smaller: N = 10, orders 3..10, plain FP64 with the entropy plane, against the oracle too
    X10 = synth.planted_10()
    S10 = api.gc_covariance(torch.from_numpy(X10).to(dev))
    sel10 = B.ThoiNplets(mode=B.THOI_SEL_RANGE, kmin=3, kmax=10, g_begin=0, g_count=968)
    opts10 = B.ThoiEvalOpts(precision=B.THOI_FP64, out_dtype=B.THOI_DTYPE_F64, vif_tau=1e3, write_entropy=1)
    say("noalloc call 2: N=10 orders 3..10 fp64 + entropy plane")
    a, b = _both(torch, B, S10, 1, 10, sel10, opts10, 5, torch.float64)
    _assert_bitwise(a, b, "N=10 fp64")
    assert a["status"] == B.THOI_OK
    ref, _, _ = orc.eval_range(S10.cpu().numpy(), 3, 10)
    assert np.nanmax(np.abs(b["out"][:4, 0] - ref)) < 1e-9

    # 3. smaller still: a LIST of 5 rows, 3 of them invalid -> status THOI_EINVAL_DATA in both
    idx = torch.tensor([[0, 1, 2, -1], [2, 1, 3, -1], [0, 10, -1, -1], [0, -1, 4, -1], [3, 4, 5, 6]],
                       dtype=torch.int32, device=dev)
    sel_l = B.ThoiNplets(mode=B.THOI_SEL_LIST, idx=ctypes.c_void_p(idx.data_ptr()), kmax_list=4, B=5)
    say("noalloc call 3: LIST of 5 rows with 3 invalid")
    a, b = _both(torch, B, S10, 1, 10, sel_l, opts10, 5, torch.float64)
    _assert_bitwise(a, b, "LIST with invalid rows")
    assert a["status"] == B.THOI_EINVAL_DATA
    assert np.all(b["flags"][0, 1:4] == B.THOI_NPLET_NOT_PD)


def test_noalloc_streaming_reduction(env):
    """Reduce mode keeps its segment counters in the scratch header: a second, smaller reduction
    must not see the first one's segments."""
    torch, api, B, synth, orc = env
    dev = torch.device("cuda:0")
    X = synth.latent_20(N=14, T=4000)
    Sigma = api.gc_covariance(torch.from_numpy(X).to(dev))
    for kmax, topk, bins in ((14, 20, 64), (9, 5, 16)):
        sel = B.ThoiNplets(mode=B.THOI_SEL_RANGE, kmin=3, kmax=kmax, g_begin=0, g_count=B.thoi_count(14, 3, kmax))
        opts = B.ThoiEvalOpts(precision=B.THOI_FP32_REFINE, out_dtype=B.THOI_DTYPE_F32, vif_tau=1e3)
        lohi = np.tile(np.array([-3.0, 3.0]), (kmax + 1, 1)).astype(np.float64)

        def pair(which, kmax=kmax, topk=topk, bins=bins, lohi=lohi):
            tv = torch.empty((1, kmax + 1, 2, topk), dtype=torch.float64, device=dev)
            tg = torch.empty((1, kmax + 1, 2, topk), dtype=torch.int64, device=dev)
            h = torch.empty((1, kmax + 1, bins + 2), dtype=torch.int64, device=dev)
            red = B.ThoiReduce(topk=topk, hist_bins=bins, hist_lo_hi=lohi.ctypes.data_as(ctypes.c_void_p),
                               top_val=_p(tv), top_g=_p(tg), hist=_p(h))
            pair.keep = (tv, tg, h, lohi)
            return red, pair.keep

        say(f"noalloc reduce: N=14 orders 3..{kmax}, top-{topk}, {bins} bins")
        a, b = _both(torch, B, Sigma, 1, 14, sel, opts, 4, torch.float32, reduce_pair=pair)
        _assert_bitwise(a, b, f"reduce orders 3..{kmax}")
        assert a["status"] == B.THOI_OK
        tot = b["hist"][0, 3:].sum(axis=1)
        assert [int(t) for t in tot] == [B.thoi_count(14, k, k) for k in range(3, kmax + 1)]
