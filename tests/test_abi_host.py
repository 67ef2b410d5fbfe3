"""Host-side checks of the C ABI (no GPU needed): exports, host helpers, argument errors."""
import ctypes
import itertools
import math
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "thoi.h")


@pytest.fixture(scope="module")
def B():
    from paper_2501_03381_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        from paper_2501_03381_amd import build
        build.build()
    binding.lib()
    return binding


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(thoi_[a-z_]+)\s*\(", text)))


def test_header_and_library_exports_match(B):
    declared = _declared()
    assert set(declared) == set(B.EXPORTS), declared
    L = B.lib()
    for name in declared:
        assert hasattr(L, name), name


def test_header_constants_match_binding(B):
    text = open(HEADER).read()
    for name in ("THOI_MAX_N_RANGE", "THOI_MAX_N", "THOI_MAX_K"):
        m = re.search(rf"#define {name} (\d+)", text)
        assert int(m.group(1)) == getattr(B, name)


def test_count_matches_eq_comb(B):
    for n in range(1, 63):
        assert B.thoi_count(n, 3, n) == (2 ** n - 1 - n - n * (n - 1) // 2 if n >= 3 else 0)
    assert B.thoi_count(20, 3, 20) == 1048365
    assert B.thoi_count(30, 3, 30) == 1073741358
    assert B.thoi_count(64, 0, 64) == -1          # 2^64 does not fit in int64
    assert B.thoi_count(62, 0, 62) == 2 ** 62


def test_unrank_host_brute_force(B):
    for N in (1, 4, 9, 12):
        for kmin in (0, 1, 3):
            if kmin > N:
                continue
            ref = [c for k in range(kmin, N + 1) for c in itertools.combinations(range(N), k)]
            for g, c in enumerate(ref):
                assert B.thoi_unrank_host(N, kmin, g) == c


def test_unrank_host_large_n_samples(B):
    rng = np.random.default_rng(3)
    for N in (30, 40, 62):
        total = B.thoi_count(N, 3, N)
        for g in rng.integers(0, total, 200):
            c = B.thoi_unrank_host(N, 3, int(g))
            k = len(c)
            # rank back: position of the order block plus the lexicographic rank
            off = sum(math.comb(N, j) for j in range(3, k))
            r, x = 0, 0
            for i, v in enumerate(c):
                for y in range(x, v):
                    r += math.comb(N - 1 - y, k - 1 - i)
                x = v + 1
            assert off + r == int(g)
            assert list(c) == sorted(set(c)) and all(0 <= v < N for v in c)


def test_bias_offsets_match_oracle(B, orc):
    """Offsets added to TC / DTC equal what the oracle's literal per-entropy correction adds."""
    from paper_2501_03381_amd import synth
    rng = np.random.default_rng(4)
    A = synth.random_spd(rng, 12, 20.0)
    for T in (50, 1000, 10001):
        for k in (1, 2, 3, 7, 12):
            o0, H0, _ = orc.measures(A, range(k))
            o1, H1, _ = orc.measures(A, range(k), bias=True, T=T)
            dtc, ddtc, eta = B.thoi_bias_offsets(k, T)
            assert abs((o1[0] - o0[0]) - dtc) < 1e-11
            assert abs((o1[1] - o0[1]) - ddtc) < 1e-11
            assert abs(eta - orc.bias_eta(k, T)) < 1e-11


def test_noalloc_scratch_limit_checked_before_launch(B):
    """The workspace-free evaluation states its fixed scratch size in the header and rejects a call
    that needs more before touching the device (no GPU needed: the check precedes every HIP call)."""
    text = open(HEADER).read()
    m = re.search(r"#define THOI_NOALLOC_SCRATCH_BYTES \(\(size_t\)(\d+) << (\d+)\)", text)
    assert m and int(m.group(1)) << int(m.group(2)) == B.THOI_NOALLOC_SCRATCH_BYTES
    L = B.lib()
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: the calls below fail their host checks
    sel = B.ThoiNplets(mode=B.THOI_SEL_RANGE, kmin=3, kmax=20, g_begin=0, g_count=1048365)
    opts = B.ThoiEvalOpts(precision=B.THOI_FP32_REFINE, out_dtype=B.THOI_DTYPE_F32, vif_tau=1e3)
    D = 8                             # refinement queue of 8 x 1,048,365 positions: 67 MB
    assert B.thoi_workspace_bytes(B.THOI_WS_EVAL, D, 0, 20, sel, opts) > B.THOI_NOALLOC_SCRATCH_BYTES
    assert L.thoi_nplets_eval_noalloc(fake, D, 20, ctypes.byref(sel), ctypes.byref(opts), fake, None, None,
                                      None) == B.THOI_EWORKSPACE
    # argument errors come first, exactly as for thoi_nplets_eval
    assert L.thoi_nplets_eval_noalloc(fake, 1, 20, ctypes.byref(sel), ctypes.byref(opts), None, None, None,
                                      None) == B.THOI_EINVAL
    assert L.thoi_nplets_eval_noalloc(fake, 1, 20, ctypes.byref(B.ThoiNplets(mode=7)), ctypes.byref(opts), fake,
                                      None, None, None) == B.THOI_EINVAL


def test_argument_errors_return_before_launch(B):
    L = B.lib()
    sel = B.ThoiNplets(mode=B.THOI_SEL_RANGE, kmin=3, kmax=20, g_begin=0, g_count=10)
    opts = B.ThoiEvalOpts(precision=B.THOI_FP32_REFINE, out_dtype=B.THOI_DTYPE_F32, vif_tau=1e3)
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: every call below fails validation first
    ev = lambda s, o, N=20, D=1, out=fake: L.thoi_nplets_eval(fake, D, N, ctypes.byref(s), ctypes.byref(o), out, None,
                                                             fake, 1 << 20, None)
    bad = B.ThoiNplets(mode=7)
    assert ev(bad, opts) == B.THOI_EINVAL
    assert ev(B.ThoiNplets(mode=B.THOI_SEL_RANGE, kmin=3, kmax=21, g_count=1), opts) == B.THOI_EINVAL     # kmax > N
    assert ev(B.ThoiNplets(mode=B.THOI_SEL_RANGE, kmin=3, kmax=20, g_begin=1048365, g_count=1), opts) == B.THOI_EINVAL
    assert ev(sel, opts, N=63) == B.THOI_EUNSUPPORTED          # RANGE limited to N <= 62
    assert ev(sel, opts, D=70000) == B.THOI_EUNSUPPORTED
    assert ev(sel, opts, out=None) == B.THOI_EINVAL
    assert ev(sel, B.ThoiEvalOpts(precision=9, out_dtype=1)) == B.THOI_EINVAL
    assert ev(sel, B.ThoiEvalOpts(precision=0, out_dtype=5)) == B.THOI_EINVAL
    assert ev(sel, B.ThoiEvalOpts(precision=0, out_dtype=0, bias_correct=1, T=10)) == B.THOI_EINVAL   # T < kmax + 2
    assert ev(B.ThoiNplets(mode=B.THOI_SEL_LIST, B=5, kmax_list=4, idx=None), opts) == B.THOI_EINVAL
    assert ev(B.ThoiNplets(mode=B.THOI_SEL_LIST, B=5, kmax_list=65, idx=fake), opts) == B.THOI_EUNSUPPORTED
    assert ev(B.ThoiNplets(mode=B.THOI_SEL_MASK, B=5, mask=fake), opts, N=65) == B.THOI_EUNSUPPORTED
    # workspace too small
    assert L.thoi_nplets_eval(fake, 1, 20, ctypes.byref(sel), ctypes.byref(opts), fake, None, fake, 16, None) == \
        B.THOI_EWORKSPACE
    assert L.thoi_copulize(fake, 1, 1, 4, 0, fake, fake, 1 << 20, None) == B.THOI_EINVAL        # T < 2
    assert L.thoi_copulize(fake, 1, 100, 4, 3, fake, fake, 1 << 20, None) == B.THOI_EINVAL      # dtype
    assert L.thoi_cov(fake, 0, 1, 100, 4, fake, fake, 0, None) == B.THOI_EWORKSPACE
    assert B.thoi_status_string(B.THOI_EINVAL_DATA).startswith("invalid data")
    assert "gfx950" in B.thoi_version()


def test_workspace_sizes(B):
    sel = B.ThoiNplets(mode=B.THOI_SEL_RANGE, kmin=3, kmax=20, g_begin=0, g_count=1048365)
    o64 = B.ThoiEvalOpts(precision=B.THOI_FP64, out_dtype=B.THOI_DTYPE_F64)
    o32r = B.ThoiEvalOpts(precision=B.THOI_FP32_REFINE, out_dtype=B.THOI_DTYPE_F32)
    assert B.thoi_workspace_bytes(B.THOI_WS_EVAL, 1, 0, 20, sel, o64) == 256
    assert B.thoi_workspace_bytes(B.THOI_WS_EVAL, 1, 0, 20, sel, o32r) >= 256 + 8 * 1048365
    assert B.thoi_workspace_bytes(B.THOI_WS_COPULIZE, 1, 1000, 10) == 256          # one chunk: no scratch
    assert B.thoi_workspace_bytes(B.THOI_WS_COPULIZE, 1, 10000, 20) > 10000 * 20 * 12
    assert B.thoi_ws_status_offset() == 0


def test_struct_layouts_match_header(B, tmp_path):
    """ctypes mirrors of the header's structs have the C sizes and field offsets (gcc, offsetof)."""
    import subprocess
    fields = {
        "thoi_nplets": ["mode", "kmin", "kmax", "g_begin", "g_count", "idx", "kmax_list", "mask", "B"],
        "thoi_reduce": ["topk", "hist_bins", "hist_lo_hi", "top_val", "top_g", "hist"],
        "thoi_eval_opts": ["precision", "out_dtype", "vif_tau", "bias_correct", "T", "write_entropy", "reduce",
                           "seg_tiles", "grid_blocks", "engine", "class_seg_tiles", "class_lanes"],
    }
    src = ["#include <stdio.h>", "#include <stddef.h>", '#include "thoi.h"', "int main(void) {"]
    for st, fs in fields.items():
        src.append(f'printf("{st} %zu\\n", sizeof({st}));')
        for f in fs:
            src.append(f'printf("{st}.{f} %zu\\n", offsetof({st}, {f}));')
    src.append("return 0; }")
    c = tmp_path / "layout.c"
    c.write_text("\n".join(src))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(c), "-o", str(exe)])
    got = dict(line.split() for line in subprocess.check_output([str(exe)], text=True).splitlines())
    mirror = {"thoi_nplets": B.ThoiNplets, "thoi_reduce": B.ThoiReduce, "thoi_eval_opts": B.ThoiEvalOpts}
    for st, cls in mirror.items():
        assert int(got[st]) == ctypes.sizeof(cls), st
        for f in fields[st]:
            assert int(got[f"{st}.{f}"]) == getattr(cls, f).offset, (st, f)


def test_multi_offsets_and_argument_errors(B):
    N_d = np.array([5, 12, 3, 30, 1], dtype=np.int32)
    off = B.thoi_multi_offsets(N_d, 3, 5)
    ref = np.concatenate([[0], np.cumsum([sum(math.comb(int(n), k) for k in range(3, 6) if k <= n) for n in N_d])])
    assert np.array_equal(off, ref)
    L = B.lib()
    fake = ctypes.c_void_p(0x1000)
    Np = N_d.ctypes.data_as(ctypes.c_void_p)
    opts = B.ThoiEvalOpts(precision=B.THOI_FP32_REFINE, out_dtype=B.THOI_DTYPE_F32)
    call = lambda N, D, kmin, kmax, o, T=None, out=fake: L.thoi_nplets_eval_multi(fake, N, T, D, kmin, kmax,
                                                                                   ctypes.byref(o), out, None, fake,
                                                                                   1 << 30, None)
    assert call(Np, 5, 3, 25, opts) == B.THOI_EUNSUPPORTED      # beyond the register classes
    assert call(Np, 5, 5, 3, opts) == B.THOI_EINVAL
    assert call(Np, 5, 3, 5, B.ThoiEvalOpts(precision=0, out_dtype=0, bias_correct=1)) == B.THOI_EINVAL  # no T_d
    bad = np.array([5, 63], dtype=np.int32)
    assert call(bad.ctypes.data_as(ctypes.c_void_p), 2, 3, 5, opts) == B.THOI_EUNSUPPORTED
    assert call(Np, 5, 3, 5, opts, out=None) == B.THOI_EINVAL
    assert call(Np, 5, 3, 5, B.ThoiEvalOpts(precision=1, out_dtype=1, seg_tiles=-1)) == B.THOI_EINVAL


def test_objective_argument_errors(B):
    L = B.lib()
    fake = ctypes.c_void_p(0x1000)
    red = B.ThoiReduce(topk=8, hist_bins=0, top_val=fake, top_g=fake)
    call = lambda D, Bn, kind, obj=fake, r=None, ws=1 << 20, dt=B.THOI_DTYPE_F64: L.thoi_objective(
        fake, dt, D, Bn, kind, obj, ctypes.byref(r) if r is not None else None, fake, ws, None)
    assert call(4, 10, 7) == B.THOI_EINVAL                               # unknown kind
    assert call(5, 10, B.THOI_OBJ_PAIRED_EFFECT) == B.THOI_EINVAL        # odd D
    assert call(2, 10, B.THOI_OBJ_PAIRED_EFFECT) == B.THOI_EINVAL        # one pair has no sd
    assert call(4, 10, B.THOI_OBJ_MEAN, obj=None) == B.THOI_EINVAL       # nothing to produce
    assert call(0, 10, B.THOI_OBJ_MEAN) == B.THOI_EINVAL
    assert call(4, 10, B.THOI_OBJ_MEAN, dt=4) == B.THOI_EINVAL
    assert call(70000, 10, B.THOI_OBJ_MEAN) == B.THOI_EUNSUPPORTED
    assert call(4, 10, B.THOI_OBJ_MEAN, r=B.ThoiReduce(topk=300, top_val=fake, top_g=fake)) == B.THOI_EUNSUPPORTED
    assert call(4, 100000, B.THOI_OBJ_MEAN, r=red, ws=16) == B.THOI_EWORKSPACE
    need = B.thoi_objective_workspace_bytes(4, 100000, red)
    assert need > B.thoi_objective_workspace_bytes(4, 100000, None) >= 256


def test_anneal_argument_errors(B):
    """thoi_anneal rejects bad shapes, bounds, schedules and missing arrays before any launch."""
    L = B.lib()
    f = ctypes.c_void_p(0x1000)

    def call(N=20, kappa=8, iters=5, move=f, a=f, b=f, u=f, T0=1.0, alpha=0.9, across=1, kmin=3, kmax=10, out=f):
        return L.thoi_anneal(f, N, f, kappa, iters, move, a, b, u, T0, alpha, 1, across, kmin, kmax, out, f, f, f, f,
                             None)
    assert call(N=1) == B.THOI_EINVAL
    assert call(N=129) == B.THOI_EINVAL
    assert call(kappa=0) == B.THOI_EINVAL
    assert call(iters=-1) == B.THOI_EINVAL
    assert call(kmin=0) == B.THOI_EINVAL
    assert call(kmin=11, kmax=10) == B.THOI_EINVAL
    assert call(kmax=20) == B.THOI_EINVAL                 # an order-N n-plet has no outsider to swap in
    assert call(N=100, kmax=65) == B.THOI_EUNSUPPORTED    # one wavefront factors orders up to 64
    assert call(T0=0.0) == B.THOI_EINVAL
    assert call(alpha=float("nan")) == B.THOI_EINVAL
    assert call(move=None) == B.THOI_EINVAL               # across orders needs the move draws
    assert call(u=None) == B.THOI_EINVAL
    assert call(out=None) == B.THOI_EINVAL
    assert call(kappa=1 << 21) == B.THOI_EUNSUPPORTED


def test_greedy_argument_errors(B):
    """thoi_greedy rejects bad shapes and sizes before any launch."""
    L = B.lib()
    f = ctypes.c_void_p(0x1000)
    need = B.thoi_greedy_workspace_bytes(1, 100, 16)
    assert need >= 100 * 16 * 24
    assert B.thoi_greedy_workspace_bytes(8, 100, 16) >= 100 * 16 * (16 + 8 * 8)

    def call(N=100, k0=3, steps=10, kappa=16, ws=need, out=f, D=1, measure=2, kind=B.THOI_OBJ_MEAN):
        return L.thoi_greedy(f, D, N, k0, steps, kappa, measure, kind, 1, out, f, f, f, ws, None)
    assert call(D=0) == B.THOI_EINVAL
    assert call(measure=4) == B.THOI_EINVAL
    assert call(kind=7) == B.THOI_EINVAL
    assert call(D=3, kind=B.THOI_OBJ_PAIRED_EFFECT) == B.THOI_EINVAL     # pairs need an even D >= 4
    assert call(D=70000) == B.THOI_EUNSUPPORTED
    assert call(D=4, ws=need) == B.THOI_EWORKSPACE                       # four datasets' measures
    assert call(N=1) == B.THOI_EINVAL
    assert call(N=129) == B.THOI_EINVAL
    assert call(k0=0) == B.THOI_EINVAL
    assert call(steps=-1) == B.THOI_EINVAL
    assert call(kappa=0) == B.THOI_EINVAL
    assert call(kappa=257) == B.THOI_EINVAL
    assert call(N=20, k0=15, steps=6) == B.THOI_EINVAL          # beyond order N
    assert call(k0=40, steps=25) == B.THOI_EUNSUPPORTED         # one wavefront factors orders up to 64
    assert call(kappa=64) == B.THOI_EUNSUPPORTED                # 6400 candidates: above the selection's sort
    assert call(out=None) == B.THOI_EINVAL
    assert call(ws=16) == B.THOI_EWORKSPACE
    assert call(steps=0, ws=0) == B.THOI_OK                     # nothing to do


def test_launch_plan_stays_below_dispatch_limit(B):
    """Every engine grid stays below 2^30 work-items along x (the dispatch limit is 2^32), also for
    enumerations whose one-workgroup-per-n-plet wave grid would exceed it: FP64 orders 19..30 at
    N=30 in output mode (1.08e8 n-plets above the FP64 register classes), full FP32 and FP64
    enumerations at N = 34..40, and a LIST of 2^33 rows."""
    lim = 1 << 30
    fake = ctypes.c_void_p(0x1000)
    cases = []
    for prec in (B.THOI_FP64, B.THOI_FP32, B.THOI_FP32_REFINE):
        cases.append((30, B.ThoiNplets(mode=B.THOI_SEL_RANGE, kmin=19, kmax=30, g_begin=0,
                                       g_count=B.thoi_count(30, 19, 30)), prec))
        for N in (34, 40):
            cases.append((N, B.ThoiNplets(mode=B.THOI_SEL_RANGE, kmin=3, kmax=N, g_begin=0,
                                          g_count=B.thoi_count(N, 3, N)), prec))
        cases.append((100, B.ThoiNplets(mode=B.THOI_SEL_LIST, B=1 << 33, kmax_list=40, idx=fake), prec))
    for N, sel, prec in cases:
        o = B.ThoiEvalOpts(precision=prec, out_dtype=B.THOI_DTYPE_F32)
        n, m = B.thoi_eval_launch_shape(N, sel, o)
        assert 1 <= n <= 7 and 0 < m < lim, (N, prec, n, m)
    # the N=20 workload keeps its usual shape: one launch per FP32 class, no large-order engine
    sel = B.ThoiNplets(mode=B.THOI_SEL_RANGE, kmin=3, kmax=20, g_begin=0, g_count=1048365)
    n, m = B.thoi_eval_launch_shape(20, sel, B.ThoiEvalOpts(precision=B.THOI_FP32_REFINE, out_dtype=1))
    # largest grid: orders 9..12, two n-plets per lane, 256 lanes per workgroup
    assert n == 4 and m == 256 * sum(-(-math.comb(20, k) // 512) for k in range(9, 13))
    assert B.lib().thoi_eval_launch_shape(20, ctypes.byref(B.ThoiNplets(mode=9)),
                                          ctypes.byref(B.ThoiEvalOpts(precision=0, out_dtype=0)),
                                          ctypes.byref(ctypes.c_int32()), ctypes.byref(ctypes.c_int64())) \
        == B.THOI_EINVAL


def test_tuner_keys_and_cache_lookup(tmp_path, monkeypatch):
    """The tuner's cache is keyed by (architecture, path, precision, register class, N bucket,
    dataset-count bucket); lookups assemble the per-class knobs of a shape (no GPU)."""
    import json
    from paper_2501_03381_amd import tune
    monkeypatch.setenv("THOI_TUNE_CACHE", str(tmp_path / "t.json"))
    assert tune.lookup_range("gfx950", "fp32_refine", 20, 1) is None
    assert [tune.n_bucket(n) for n in (5, 12, 13, 20, 30, 40, 62)] == \
        ["N<=12", "N<=12", "N<=16", "N<=24", "N<=32", "N<=48", "N<=62"]
    assert [tune.d_bucket(d) for d in (1, 2, 64, 65)] == ["D<=1", "D<=8", "D<=64", "D>64"]
    k1 = tune.range_key("gfx950", "fp32_refine", 1, 20, 1)
    assert k1 == "gfx950|range|fp32_refine|k9-12|N<=24|D<=1"
    assert tune.range_key("gfx950", "fp64", 1, 20, 1) == "gfx950|range|fp64|k7-10|N<=24|D<=1"
    json.dump({k1: {"seg_tiles": 3, "lanes": 1},
               tune.range_key("gfx950", "fp32_refine", 3, 20, 1): {"seg_tiles": 2, "lanes": 0},
               tune.multi_key("gfx950", "fp32", [10, 40, 22], 3, 5): {"seg_tiles": 4, "grid_blocks": 512}},
              open(tmp_path / "t.json", "w"))
    seg, lanes = tune.lookup_range("gfx950", "fp32_refine", 21, 1)     # same N bucket
    assert seg == [0, 3, 0, 2, 0, 0, 0, 0] and lanes == [0, 1, 0, 0, 0, 0, 0, 0]
    assert tune.lookup_range("gfx950", "fp32_refine", 30, 1) is None     # another N bucket
    assert tune.lookup_range("gfx942", "fp32_refine", 20, 1) is None     # another architecture
    assert tune.lookup_multi("gfx950", "fp32", [12, 33, 40], 3, 5) == (4, 512)
    assert tune.lookup_multi("gfx950", "fp32", [12, 33, 40], 3, 6) is None


def test_search_combinations_match_itertools():
    """The greedy's first-order rows: every k-subset in lexicographic order, as itertools gives."""
    import itertools
    from paper_2501_03381_amd.search import combinations
    for N, k in ((100, 3), (20, 1), (20, 5), (7, 7), (5, 0), (30, 4), (1, 1), (64, 2), (6, 3)):
        ref = list(itertools.combinations(range(N), k))
        got = combinations(N, k)
        assert got.dtype == np.int32 and got.shape == (len(ref), k), (N, k)
        assert [tuple(int(x) for x in r) for r in got] == ref, (N, k)
