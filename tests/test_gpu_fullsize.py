"""Parity at the full sizes of the method's configurations, in the launch configurations bench.py
times: checked on outputs the oracle can compute one by one, or by properties that hold at any
size.

* N=30, T=1200 AR(1) mixture: all 1,073,741,358 n-plets of orders 3..30 in reduce mode.  Histogram
  totals equal C(30, k) exactly; every reported top-100 / bottom-100 n-plet's Omega equals the
  oracle's; in a seeded sample of 10^5 n-plets nothing beats the reported extremes, and every
  sampled n-plet clearly beyond the K-th reported value is in the reported list.
* 1024 uneven datasets (N ~ U{10..40}, T ~ U{500..5000}), orders 3..5, one multi-dataset call:
  every dataset with N <= 20 against the oracle exhaustively, the others on seeded samples.
* N=100, T=2000: 10^5 n-plets of order 8..20, forward and the adjoint of sum(Omega) against the
  oracle's explicit-inverse gradient of the same sum.
"""
import math
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


def test_ar1_30_exhaustive_reduce(env):
    torch, api, B, synth, orc = env
    N, kmin, kmax, K = 30, 3, 30, 100
    X = synth.ar1_30()
    S = orc.gc_covariance(X)
    Sd = torch.from_numpy(S).cuda()
    lohi = np.zeros((kmax + 1, 2))
    lohi[:, 0], lohi[:, 1] = -40.0, 10.0
    say("ar1_30: all 1,073,741,358 n-plets, fp32_refine, top-100 / bottom-100 + 256 bins")
    st = api.nplets_reduce(Sd, orders=(kmin, kmax), topk=K, hist_bins=256, hist_range=lohi, precision="fp32_refine")
    tv, tg, h = st.result()
    for k in range(kmin, kmax + 1):
        assert int(h[0, k].sum()) == math.comb(N, k), k
    assert int(h[0].sum()) == B.thoi_count(N, kmin, kmax)
    # every reported n-plet, recomputed by the oracle
    rows, vals, where = [], [], []
    for k in range(kmin, kmax + 1):
        for l in range(2):
            n = min(K, math.comb(N, k))
            g = tg[0, k, l, :n]
            assert np.all(g >= 0) and np.all(tg[0, k, l, n:] == -1), (k, l)
            for j, gg in enumerate(g):
                rows.append(B.thoi_unrank_host(N, kmin, int(gg)))
                vals.append(tv[0, k, l, j])
                where.append((k, l, j))
    say(f"oracle on the {len(rows)} reported n-plets")
    ref, _, _ = orc.eval_list(S, orc.pad_list(rows, kmax))
    assert np.abs(ref[2] - np.array(vals)).max() < 1e-3
    for (k, l, j), r in zip(where, rows):
        assert len(r) == k
    # a seeded sample of 10^5 n-plets against the lists (membership by global rank)
    rng = np.random.default_rng(30)
    ks = rng.integers(kmin, kmax + 1, 100000)
    samp = [tuple(sorted(rng.choice(N, int(k), replace=False))) for k in ks]
    say("oracle on a seeded sample of 10^5 n-plets")
    sv, _, _ = orc.eval_list(S, orc.pad_list(samp, kmax))
    def rank(c):
        k = len(c)
        g = sum(math.comb(N, j) for j in range(kmin, k))
        x = 0
        for i, v in enumerate(c):
            for y in range(x, v):
                g += math.comb(N - 1 - y, k - 1 - i)
            x = v + 1
        return g

    for k in range(kmin, kmax + 1):
        sel = np.nonzero(ks == k)[0]
        if len(sel) == 0:
            continue
        n = min(K, math.comb(N, k))
        top, bot = set(tg[0, k, 0, :n].tolist()), set(tg[0, k, 1, :n].tolist())
        v = sv[2][sel]
        assert v.max() <= tv[0, k, 0, 0] + 1e-3 and v.min() >= tv[0, k, 1, 0] - 1e-3, k
        # a sampled n-plet clearly above the K-th largest (below the K-th smallest) is in the list
        for i in sel[v > tv[0, k, 0, n - 1] + 1e-3]:
            assert rank(samp[i]) in top, (k, samp[i])
        for i in sel[v < tv[0, k, 1, n - 1] - 1e-3]:
            assert rank(samp[i]) in bot, (k, samp[i])


def test_uneven_1024_datasets(env):
    torch, api, B, synth, orc = env
    Xs = synth.uneven_many(D=1024, seed=3)
    say("uneven: copula + covariance of 1024 datasets on the GPU")
    Sig = [api.gc_covariance(torch.from_numpy(X).cuda()) for X in Xs]
    say("uneven: all n-plets of orders 3..5 of 1024 datasets, one multi-dataset call, fp32_refine")
    out, flags, off = api.nplets_measures_multi(Sig, 3, 5, precision="fp32_refine")
    out = out.cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(31)
    checked = 0
    for d, X in enumerate(Xs):
        N = X.shape[1]
        So = orc.gc_covariance(X)
        idx = orc.enumerate_nplets(N, 3, 5)
        assert off[d + 1] - off[d] == len(idx)
        pick = np.arange(len(idx)) if N <= 20 else np.unique(rng.integers(0, len(idx), 300))
        ref, _, _ = orc.eval_list(So, idx[pick])
        got = out[:, off[d]:off[d + 1]][:, pick]
        assert np.abs(got - ref).max() < 1e-3, d
        checked += len(pick)
    say(f"uneven: {checked} n-plets checked against the oracle")
    assert off[-1] > 1.5e8


def test_latent100_forward_and_adjoint(env):
    torch, api, B, synth, orc = env
    X, idx = synth.latent_100()
    S = orc.gc_covariance(X)
    Sd = torch.from_numpy(S).cuda()
    rows = torch.from_numpy(idx).cuda()
    say("latent_100: 10^5 n-plets of order 8..20, forward fp32_refine")
    out, _ = api.nplets_measures(Sd, nplets=rows, precision="fp32_refine")
    ref, _, _ = orc.eval_list(S, idx)
    assert np.abs(out.cpu().numpy().astype(np.float64) - ref).max() < 1e-3
    say("latent_100: adjoint of sum(Omega) over the 10^5 n-plets")
    w = torch.zeros((4, idx.shape[0]), dtype=torch.float32, device=Sd.device)
    w[2] = 1.0
    G = api.measures_backward(Sd, w, nplets=rows)[0].double().cpu().numpy()
    wo = np.zeros((4, idx.shape[0]))
    wo[2] = 1.0
    Go = orc.grad_list(S, idx, wo)
    assert np.linalg.norm(G - Go) <= 1e-3 * np.linalg.norm(Go)
