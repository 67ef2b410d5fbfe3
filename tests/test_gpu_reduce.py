"""GPU parity of the streaming per-order top-K / bottom-K and histogram reduction of Omega.

Exactness is checked against a full-output run of the same kernels (same arithmetic): the
lists are an exact selection of those values and the histogram counts them; values are
checked against the FP64 oracle at the FP32 tolerance.
"""
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


def test_reduce_range_matches_full_output(env):
    torch, api, B, synth, orc = env
    S = orc.gc_covariance(synth.latent_20(T=3000))
    Sd = dev(torch, S)
    idx = orc.enumerate_nplets(20, 3, 20)
    ords = orders_of(idx)
    say("full output fp32_refine N=20")
    out, _ = api.nplets_measures(Sd, orders=(3, 20), precision="fp32_refine")
    om = out[2].cpu().numpy().astype(np.float64)
    lohi = np.zeros((21, 2))
    lohi[:, 0], lohi[:, 1] = -2.0, 1.0
    say("reduce fp32_refine N=20 topk=100 bins=64")
    st = api.nplets_reduce(Sd, orders=(3, 20), topk=100, hist_bins=64, hist_range=lohi)
    tv, tg, h = st.result()
    check_lists(tv[0], tg[0], om, ords, 100, 1e-6)
    for k in range(3, 21):
        ref = orc.histogram(om[ords == k], -2.0, 1.0, 64)
        assert h[0, k].sum() == ref.sum() == (ords == k).sum()
        assert np.abs(h[0, k] - ref).sum() <= 2, k
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
    for prec, tol in (("fp64", 1e-9), ("fp32_refine", 1e-3)):
        say(f"reduce {prec} N=14 vs oracle")
        st = api.nplets_reduce(dev(torch, S), orders=(3, 14), topk=30, hist_bins=16, hist_range=(-1.5, 1.0),
                               precision=prec)
        tv, tg, h = st.result()
        check_lists(tv[0], tg[0], ref[2], ords, 30, tol)
        for k in range(3, 15):
            assert h[0, k].sum() == (ords == k).sum()


def test_reduce_list_mixed_orders_and_wave_engine(env):
    torch, api, B, synth, orc = env
    X, idx = synth.latent_100(B=5000)
    S = orc.gc_covariance(X)
    idx = idx[:, :20]
    Sd, Id = dev(torch, S), dev(torch, idx)
    for prec in ("fp64", "fp32_refine"):          # fp64: orders 19, 20 use the wave engine
        say(f"reduce LIST {prec} N=100")
        out, _ = api.nplets_measures(Sd, nplets=Id, precision=prec, out_dtype=torch.float64)
        om = out[2].cpu().numpy()
        st = api.nplets_reduce(Sd, nplets=Id, topk=20, hist_bins=40, hist_range=(-4.0, 4.0), precision=prec)
        tv, tg, h = st.result()
        check_lists(tv[0], tg[0], om, orders_of(idx), 20, 1e-9)
        ords = orders_of(idx)
        for k in range(8, 21):
            assert h[0, k].sum() == (ords == k).sum()


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
    out, flags = api.nplets_measures(Sd, orders=(3, 6), precision="fp32_refine")
    assert ((flags.cpu().numpy() & B.THOI_NPLET_REFINED) != 0).sum() > 0
    st = api.nplets_reduce(Sd, orders=(3, 6), topk=40, hist_bins=20, hist_range=(-3.0, 3.0))
    tv, tg, h = st.result()
    check_lists(tv[0], tg[0], ref[2], orders_of(idx), 40, 1e-3)
    ords = orders_of(idx)
    for k in range(3, 7):
        assert h[0, k].sum() == (ords == k).sum()


def test_reduce_many_datasets(env):
    torch, api, B, synth, orc = env
    Xs = synth.replicas_20(3, T=2000)
    Sd = api.gc_covariance(dev(torch, Xs))
    idx = orc.enumerate_nplets(20, 3, 20)
    ords = orders_of(idx)
    say("reduce D=3 N=20")
    out, _ = api.nplets_measures(Sd, orders=(3, 20), precision="fp32_refine")
    st = api.nplets_reduce(Sd, orders=(3, 20), topk=10, hist_bins=8, hist_range=(-5.0, 5.0))
    tv, tg, h = st.result()
    for d in range(3):
        check_lists(tv[d], tg[d], out[2, d].cpu().numpy().astype(np.float64), ords, 10, 1e-6)
