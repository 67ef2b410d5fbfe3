"""GPU parity of the multi-dataset path (datasets of uneven N and T in one persistent launch per
register class) against the FP64 oracle, dataset by dataset."""
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


def uneven(synth, D, n_lo, n_hi, t_lo, t_hi, seed):
    return synth.uneven_many(D=D, seed=seed, n_lo=n_lo, n_hi=n_hi, t_lo=t_lo, t_hi=t_hi)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-9), ("fp32_refine", 1e-3), ("fp32", 1e-3)])
def test_multi_uneven_against_oracle(env, prec, tol):
    torch, api, B, synth, orc = env
    Xs = uneven(synth, 40, 6, 30, 500, 3000, 11)
    Sig = [orc.gc_covariance(X) for X in Xs]
    say(f"multi {prec} D=40 N 6..30 orders 3..5")
    odt = torch.float64 if prec == "fp64" else torch.float32
    out, flags, off = api.nplets_measures_multi([dev(torch, S) for S in Sig], 3, 5, precision=prec, out_dtype=odt)
    out = out.cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(12)
    for d, S in enumerate(Sig):
        N = S.shape[0]
        idx = orc.enumerate_nplets(N, 3, 5)
        assert off[d + 1] - off[d] == len(idx)
        pick = np.arange(len(idx)) if len(idx) <= 3000 else np.unique(rng.integers(0, len(idx), 3000))
        ref, _, _ = orc.eval_list(S, idx[pick])
        got = out[:, off[d]:off[d + 1]][:, pick]
        assert np.abs(got - ref).max() <= tol, (d, N)


def test_multi_two_chunks_bias_and_entropy(env):
    torch, api, B, synth, orc = env
    Xs = uneven(synth, 300, 4, 12, 200, 900, 13)       # more than one chunk of 256 datasets
    Sig = [orc.gc_covariance(X) for X in Xs]
    T_d = np.array([X.shape[0] for X in Xs], dtype=np.int32)
    say("multi fp64 D=300 orders 1..8 with bias correction and entropy plane")
    out, flags, off = api.nplets_measures_multi([dev(torch, S) for S in Sig], 1, 8, precision="fp64",
                                                out_dtype=torch.float64, T_d=T_d, bias_correct=True,
                                                write_entropy=True)
    out = out.cpu().numpy()
    for d, S in enumerate(Sig):
        N = S.shape[0]
        idx = orc.enumerate_nplets(N, 1, min(8, N))
        ref, Href, _ = orc.eval_list(S, idx, bias=True, T=int(T_d[d]))
        got = out[:, off[d]:off[d + 1]]
        assert np.abs(got[:4] - ref).max() <= 1e-9, d
        assert np.abs(got[4] - Href).max() <= 1e-9, d


def test_multi_refinement_and_reduce(env):
    torch, api, B, synth, orc = env
    Xs = uneven(synth, 12, 10, 24, 800, 2000, 14)
    rng = np.random.default_rng(15)
    for X in Xs[:4]:
        X[:, 1] = X[:, 0] + 1e-4 * rng.standard_normal(X.shape[0])      # ill-conditioned pairs
    Sig = [orc.gc_covariance(X) for X in Xs]
    Sd = [dev(torch, S) for S in Sig]
    say("multi fp32_refine with near-duplicate columns")
    out, flags, off = api.nplets_measures_multi(Sd, 3, 6, precision="fp32_refine")
    out, flags = out.cpu().numpy().astype(np.float64), flags.cpu().numpy()
    assert ((flags & B.THOI_NPLET_REFINED) != 0).sum() > 0
    for d, S in enumerate(Sig):
        idx = orc.enumerate_nplets(S.shape[0], 3, 6)
        ref, _, _ = orc.eval_list(S, idx)
        assert np.abs(out[:, off[d]:off[d + 1]] - ref).max() <= 1e-3, d
    say("multi reduce top-10 / 16 bins")
    flat, Ns = api.pack_covariances(Sd)
    st = api.ReduceState(len(Sd), 6, 10, 16, (-3.0, 3.0), flat.device)
    ev = api.MultiEvaluator(Ns, 3, 6, flat.device, "fp32_refine", reduce_state=st)
    ev(flat)
    assert ev.status() == 0
    tv, tg, h = st.result()
    import oracle
    for d in range(len(Sd)):
        om = out[2, off[d]:off[d + 1]]
        ords = (orc.enumerate_nplets(Ns[d], 3, 6) >= 0).sum(1)
        ref = oracle.topk_per_order(om, ords, np.arange(len(om)), 10)
        for k, (top, bot) in ref.items():
            assert np.allclose(tv[d, k, 0, :len(top)], [x[0] for x in top], atol=1e-6)
            assert np.allclose(tv[d, k, 1, :len(bot)], [x[0] for x in bot], atol=1e-6)
            assert np.allclose(om[tg[d, k, 0, :len(top)]], tv[d, k, 0, :len(top)], atol=1e-6)
            assert h[d, k].sum() == (ords == k).sum()


def test_tuning_knobs_do_not_change_results(env, tmp_path, monkeypatch):
    torch, api, B, synth, orc = env
    from paper_2501_03381_amd import tune
    monkeypatch.setenv("THOI_TUNE_CACHE", str(tmp_path / "tune.json"))
    Sd = api.gc_covariance(dev(torch, synth.latent_20(T=2000)))
    sel = api.range_selection(20, 3, 20)
    for prec, odt in (("fp32_refine", torch.float32), ("fp64", torch.float64)):
        say(f"seg_tiles library choice / 1 / 2 / 3 / 8 give identical RANGE results, {prec}")
        outs = []
        for st in (0, 1, 2, 3, 8):
            ev = api.Evaluator(1, 20, sel, api.make_opts(prec, odt, seg_tiles=st), Sd.device, odt)
            o, f = ev(Sd)
            outs.append((o.clone(), f.clone()))
        for o, f in outs[1:]:
            assert torch.equal(o, outs[0][0]) and torch.equal(f, outs[0][1])
        say(f"per-class tiles per workgroup and n-plets per lane give identical RANGE results, {prec}")
        for cs, cl in (([3, 1, 2, 5, 1, 0, 0, 0], [1, 1, 1, 0, 0, 0, 0, 0]), ([1, 4, 1, 1, 2, 0, 0, 0], [1, 0, 1, 0, 0, 0, 0, 0])):
            ev = api.Evaluator(1, 20, sel, api.make_opts(prec, odt, class_seg_tiles=cs, class_lanes=cl), Sd.device, odt)
            o, f = ev(Sd)
            assert torch.equal(o, outs[0][0]) and torch.equal(f, outs[0][1]), (cs, cl)
    say("tune_range, then an Evaluator built without knobs takes them from the cache")
    r = tune.tune_range(Sd, 3, 20, seg_candidates=(1, 2))
    assert all(v in (0, 1, 2) for v in r["class_seg_tiles"]) and all(v in (0, 1) for v in r["class_lanes"])
    assert len(r["classes"]) == 4 and all(e["ms"] > 0 for e in r["classes"].values())
    ev = api.Evaluator(1, 20, sel, api.make_opts("fp32_refine", torch.float32), Sd.device, torch.float32)
    assert list(ev.opts.class_seg_tiles) == r["class_seg_tiles"] and list(ev.opts.class_lanes) == r["class_lanes"]
    o, f = ev(Sd)
    ref = api.Evaluator(1, 20, sel, api.make_opts("fp32_refine", torch.float32), Sd.device, torch.float32,
                        tuned=False)(Sd)
    assert torch.equal(o, ref[0]) and torch.equal(f, ref[1])
    Xs = uneven(synth, 20, 8, 20, 500, 1000, 16)
    Sig = [dev(torch, orc.gc_covariance(X)) for X in Xs]
    flat, Ns = api.pack_covariances(Sig)
    say("multi grid/segment knobs give identical results")
    res = []
    for st, gb in ((1, 0), (4, 64), (2, 7)):
        ev = api.MultiEvaluator(Ns, 3, 6, flat.device, "fp32_refine", seg_tiles=st, grid_blocks=gb)
        o, f = ev(flat)
        res.append(o.clone())
    assert all(torch.equal(res[0], r_) for r_ in res[1:])
    say("tune_multi, then a MultiEvaluator built without knobs takes them from the cache")
    t = tune.tune_multi(flat, Ns, 3, 6, seg_candidates=(1, 4), grid_candidates=(0, 256))
    assert t["seg_tiles"] in (1, 4) and t["grid_blocks"] in (0, 256)
    ev = api.MultiEvaluator(Ns, 3, 6, flat.device, "fp32_refine")
    assert (ev.opts.seg_tiles, ev.opts.grid_blocks) == (t["seg_tiles"], t["grid_blocks"])
    o, f = ev(flat)
    assert torch.equal(o, res[0])
