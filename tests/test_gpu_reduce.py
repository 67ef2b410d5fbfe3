"""GPU parity of the streaming per-order top-K / bottom-K and histogram reduction of Omega.

Two kinds of check:
* exactness of the reduction: against a full-output run of the same kernels with FP64 output
  planes (the value each n-plet enters the reducer with is exactly the value written there), the
  lists are the exact selection (ties by the lower index) and every histogram bin equals the
  oracle module's binning of those values, with no slack;
* against the FP64 oracle: lists by the top-K acceptance rule and histograms bin by bin, a value
  being allowed on either side of an edge only when the oracle puts it within the tolerance of
  that edge (1e-9 for the FP64 path, 1e-3 for FP32 with refinement).
"""
import math
import sys

import numpy as np
import pytest

from _checks import check_hist, check_topk

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env(orc):
    import torch
    from paper_2501_03381_amd import api, binding, synth
    binding.lib()
    assert torch.cuda.is_available()
    return torch, api, binding, synth, orc


def dev(torch, x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def orders_of(idx):
    return (idx >= 0).sum(1)


def check_lists(top_val, top_g, omega, orders, K, tol):
    """Lists of every order against an exact sort of `omega` (ties by lower g)."""
    import oracle
    ref = oracle.topk_per_order(omega, orders, np.arange(len(omega)), K)
    for k, (top, bot) in ref.items():
        for l, lst in ((0, top), (1, bot)):
            n = len(lst)
            v = top_val[k, l, :n]
            g = top_g[k, l, :n]
            assert np.all(g >= 0), (k, l)
            assert np.all(top_g[k, l, n:] == -1)
            assert np.allclose(v, [x[0] for x in lst], atol=tol, rtol=0), (k, l)
            # every reported index carries the value reported for it
            assert np.allclose(omega[g], v, atol=tol, rtol=0), (k, l)
            assert np.all(orders[g] == k)
            if tol == 0.0:
                # exact values: the selection with ties by the lower index is unique
                assert np.array_equal(g, [x[1] for x in lst]), (k, l)


def test_reduce_range_matches_full_output(env):
    torch, api, B, synth, orc = env
    S = orc.gc_covariance(synth.latent_20(T=3000))
    Sd = dev(torch, S)
    idx = orc.enumerate_nplets(20, 3, 20)
    ords = orders_of(idx)
    say("full output fp32_refine N=20 (FP64 output planes)")
    out, _ = api.nplets_measures(Sd, orders=(3, 20), precision="fp32_refine", out_dtype=torch.float64)
    om = out[2].cpu().numpy()
    lohi = np.zeros((21, 2))
    lohi[:, 0], lohi[:, 1] = -2.0, 1.0
    say("reduce fp32_refine N=20 topk=100 bins=64")
    st = api.nplets_reduce(Sd, orders=(3, 20), topk=100, hist_bins=64, hist_range=lohi)
    tv, tg, h = st.result()
    check_lists(tv[0], tg[0], om, ords, 100, 0.0)
    for k in range(3, 21):
        ref = orc.histogram(om[ords == k], -2.0, 1.0, 64)
        assert np.array_equal(h[0, k], ref), k
        assert h[0, k].sum() == (ords == k).sum()
    assert np.all(h[0, :3] == 0)


def test_reduce_pieces_equal_single_launch(env):
    torch, api, B, synth, orc = env
    Sd = api.gc_covariance(dev(torch, synth.latent_20(T=2000)))
    total = B.thoi_count(20, 3, 20)
    say("reduce single launch")
    one = api.nplets_reduce(Sd, orders=(3, 20), topk=50, hist_bins=32, hist_range=(-3.0, 2.0)).result()
    cuts = [0, 1, 1000, 77777, 300000, 300001, 900000, total]
    st = None
    say("reduce in 7 uneven pieces")
    for a, b in zip(cuts[:-1], cuts[1:]):
        st = api.nplets_reduce(Sd, orders=(3, 20), g_range=(a, b - a), topk=50, hist_bins=32, hist_range=(-3.0, 2.0),
                               state=st)
    many = st.result()
    for x, y in zip(one, many):
        assert np.array_equal(x, y, equal_nan=True)


def test_reduce_against_oracle_fp64_and_fp32(env):
    torch, api, B, synth, orc = env
    X = synth.latent_20(T=3000)[:, :14]
    S = orc.gc_covariance(X)
    ref, _, _ = orc.eval_range(S, 3, 14)
    idx = orc.enumerate_nplets(14, 3, 14)
    ords = orders_of(idx)
    g_all = np.arange(len(idx))
    lo, hi, bins = -1.5, 1.0, 16
    for prec, tol in (("fp64", 1e-9), ("fp32_refine", 1e-3)):
        say(f"reduce {prec} N=14 vs oracle")
        st = api.nplets_reduce(dev(torch, S), orders=(3, 14), topk=30, hist_bins=bins, hist_range=(lo, hi),
                               precision=prec)
        tv, tg, h = st.result()
        near = 0
        for k in range(3, 15):
            sel = ords == k
            for l, largest in ((0, True), (1, False)):
                check_topk(tv[0, k, l], tg[0, k, l], g_all[sel], ref[2][sel], 30, tol, largest, f"{prec} k={k} l={l}")
            near += check_hist(h[0, k], ref[2][sel], lo, hi, bins, tol, f"{prec} k={k}")
        say(f"{prec}: {near} oracle values within {tol:g} of a bin edge")
        if prec == "fp64":
            assert near == 0          # no oracle value this close to an edge: every bin is exact


def test_reduce_list_mixed_orders_and_wave_engine(env):
    torch, api, B, synth, orc = env
    X, idx = synth.latent_100(B=5000)
    S = orc.gc_covariance(X)
    idx = idx[:, :20]
    Sd, Id = dev(torch, S), dev(torch, idx)
    ords = orders_of(idx)
    for prec in ("fp64", "fp32_refine"):          # fp64: orders 19, 20 use the wave engine
        say(f"reduce LIST {prec} N=100")
        out, _ = api.nplets_measures(Sd, nplets=Id, precision=prec, out_dtype=torch.float64)
        om = out[2].cpu().numpy()
        st = api.nplets_reduce(Sd, nplets=Id, topk=20, hist_bins=40, hist_range=(-4.0, 4.0), precision=prec)
        tv, tg, h = st.result()
        check_lists(tv[0], tg[0], om, ords, 20, 0.0)
        for k in range(8, 21):
            assert np.array_equal(h[0, k], orc.histogram(om[ords == k], -4.0, 4.0, 40)), k


def test_reduce_range_pair_and_wave_engines(env):
    """Orders 19..32 of a FP64 reduction run two n-plets per wavefront, orders 33..36 one per
    wavefront; both feed the reducer exactly what the full-output run writes."""
    torch, api, B, synth, orc = env
    N, kmin = 36, 30
    Sd = dev(torch, orc.gc_covariance(synth.ar1_30(N=N, T=3000)))
    total = B.thoi_count(N, kmin, N)
    ords = np.concatenate([np.full(math.comb(N, k), k) for k in range(kmin, N + 1)])
    assert len(ords) == total
    say(f"full output fp64 N={N} orders {kmin}..{N}")
    out, _ = api.nplets_measures(Sd, orders=(kmin, N), precision="fp64", out_dtype=torch.float64)
    om = out[2].cpu().numpy()
    say(f"reduce fp64 N={N} orders {kmin}..{N} topk=30 bins=24")
    st = api.nplets_reduce(Sd, orders=(kmin, N), topk=30, hist_bins=24, hist_range=(-40.0, 5.0), precision="fp64")
    tv, tg, h = st.result()
    check_lists(tv[0], tg[0], om, ords, 30, 0.0)
    for k in range(kmin, N + 1):
        assert np.array_equal(h[0, k], orc.histogram(om[ords == k], -40.0, 5.0, 24)), k


def test_reduce_refined_values_enter(env):
    torch, api, B, synth, orc = env
    rng = np.random.default_rng(8)
    X = synth.latent_20(T=4000)
    X[:, 1] = X[:, 0] + 1e-4 * rng.standard_normal(4000)
    S = orc.gc_covariance(X)
    Sd = dev(torch, S)
    idx = orc.enumerate_nplets(20, 3, 6)
    ref, _, _ = orc.eval_list(S, idx)
    say("reduce with FP64-refined n-plets")
    out, flags = api.nplets_measures(Sd, orders=(3, 6), precision="fp32_refine", out_dtype=torch.float64)
    assert ((flags.cpu().numpy() & B.THOI_NPLET_REFINED) != 0).sum() > 0
    om = out[2].cpu().numpy()
    st = api.nplets_reduce(Sd, orders=(3, 6), topk=40, hist_bins=20, hist_range=(-3.0, 3.0))
    tv, tg, h = st.result()
    ords = orders_of(idx)
    g_all = np.arange(len(idx))
    check_lists(tv[0], tg[0], om, ords, 40, 0.0)
    for k in range(3, 7):
        sel = ords == k
        assert np.array_equal(h[0, k], orc.histogram(om[sel], -3.0, 3.0, 20)), k
        for l, largest in ((0, True), (1, False)):
            check_topk(tv[0, k, l], tg[0, k, l], g_all[sel], ref[2][sel], 40, 1e-3, largest, f"k={k} l={l}")
        check_hist(h[0, k], ref[2][sel], -3.0, 3.0, 20, 1e-3, f"k={k}")


def test_reduce_list_sizes_exact(env):
    """K = 1, one wavefront's worth (64), one past it and the maximum (256): the per-wavefront
    lists are merged in blocks of 64 outputs, and the admission bounds shared between workgroups
    drop values early; the selection must stay exact on the FP32 and FP64 paths."""
    torch, api, B, synth, orc = env
    S = orc.gc_covariance(synth.latent_20(T=3000))
    Sd = dev(torch, S)
    idx = orc.enumerate_nplets(20, 3, 20)
    ords = orders_of(idx)
    for prec in ("fp32_refine", "fp64"):
        out, _ = api.nplets_measures(Sd, orders=(3, 20), precision=prec, out_dtype=torch.float64)
        om = out[2].cpu().numpy()
        for K in (1, 64, 65, 256):
            say(f"reduce {prec} N=20 orders 3..20 topk={K}")
            tv, tg, _ = api.nplets_reduce(Sd, orders=(3, 20), topk=K, precision=prec).result()
            check_lists(tv[0], tg[0], om, ords, K, 0.0)


def test_reduce_many_datasets(env):
    torch, api, B, synth, orc = env
    Xs = synth.replicas_20(3, T=2000)
    Sd = api.gc_covariance(dev(torch, Xs))
    idx = orc.enumerate_nplets(20, 3, 20)
    ords = orders_of(idx)
    say("reduce D=3 N=20")
    out, _ = api.nplets_measures(Sd, orders=(3, 20), precision="fp32_refine", out_dtype=torch.float64)
    st = api.nplets_reduce(Sd, orders=(3, 20), topk=10, hist_bins=8, hist_range=(-5.0, 5.0))
    tv, tg, h = st.result()
    for d in range(3):
        om = out[2, d].cpu().numpy()
        check_lists(tv[d], tg[d], om, ords, 10, 0.0)
        for k in range(3, 21):
            assert np.array_equal(h[d, k], orc.histogram(om[ords == k], -5.0, 5.0, 8)), (d, k)
