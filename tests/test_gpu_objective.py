"""GPU parity of the objectives over datasets (thoi_objective) and of the multi-dataset greedy
search against the oracle."""
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
    from paper_2501_03381_amd import api, binding, search, synth
    binding.lib()
    assert torch.cuda.is_available()
    return torch, api, search, synth, orc


@pytest.mark.parametrize("kind,D,Bn,dtype", [("mean", 5, 3001, "f64"), ("paired_effect", 8, 70001, "f64"),
                                             ("paired_effect", 6, 257, "f32"), ("mean", 1, 1, "f64")])
def test_objective_values_and_reducer(env, kind, D, Bn, dtype):
    torch, api, search, synth, orc = env
    rng = np.random.default_rng(D * 1000 + Bn)
    v = rng.standard_normal((D, Bn))
    v[:, ::97] = np.round(v[:, ::97], 1)            # exact ties among objectives
    if Bn > 10:
        v[1, 5] = np.nan
        v[:, 7] = v[0, 7]                           # paired differences all 0 -> sd 0 -> NaN
    if dtype == "f32":
        v = v.astype(np.float32).astype(np.float64)
    t = torch.from_numpy(v).cuda()
    t = t.float() if dtype == "f32" else t
    say(f"objective {kind} D={D} B={Bn} {dtype} with top-16 and 32 bins")
    obj, st = api.objective(t, kind, topk=16, hist_bins=32, hist_range=(-3.0, 3.0))
    ref = orc.objective(v, kind)
    got = obj.cpu().numpy()
    assert np.array_equal(np.isnan(got), np.isnan(ref))
    assert np.nanmax(np.abs(got - ref)) <= 1e-12 * max(1.0, np.nanmax(np.abs(ref)))
    tv, tg, h = st.result()
    top = orc.topk_per_order(ref, np.zeros(Bn, dtype=np.int64), np.arange(Bn), 16)[0]
    assert [g for _, g in top[0]] == list(tg[0, 0, 0, : len(top[0])])
    assert [g for _, g in top[1]] == list(tg[0, 0, 1, : len(top[1])])
    assert np.array_equal(h[0, 0], orc.histogram(ref[~np.isnan(ref)], -3.0, 3.0, 32))


def test_objective_reducer_merges_across_calls(env):
    torch, api, search, synth, orc = env
    rng = np.random.default_rng(3)
    v = rng.standard_normal((4, 5000))
    say("objective reducer: two halves merged equal one call")
    _, whole = api.objective(torch.from_numpy(v).cuda(), "mean", write=False, topk=10)
    st = api.ReduceState(1, 0, 10, 0, (0.0, 1.0), torch.device("cuda"))
    api.objective(torch.from_numpy(np.ascontiguousarray(v[:, :2500])).cuda(), "mean", write=False, state=st)
    tv_a, tg_a, _ = st.result()
    ref = orc.objective(v, "mean")
    top = orc.topk_per_order(ref, np.zeros(5000, dtype=np.int64), np.arange(5000), 10)[0]
    tv, tg, _ = whole.result()
    assert [g for _, g in top[0]] == list(tg[0, 0, 0])
    first = orc.topk_per_order(ref[:2500], np.zeros(2500, dtype=np.int64), np.arange(2500), 10)[0]
    assert [g for _, g in first[0]] == list(tg_a[0, 0, 0])


@pytest.mark.parametrize("kind,maximize", [("paired_effect", False), ("mean", True)])
def test_greedy_multi_matches_oracle(env, kind, maximize):
    torch, api, search, synth, orc = env
    from oracle import search as osearch
    X = synth.condition_pairs(6)
    Sig = np.stack([orc.gc_covariance(x) for x in X])
    say(f"greedy over 12 datasets, objective {kind}, orders 3..7, fp64")
    got = search.greedy_multi(torch.from_numpy(Sig).cuda(), 3, 7, kappa=6, kind=kind, maximize=maximize)
    ref = osearch.greedy_multi(Sig, 3, 7, kappa=6, kind=kind, maximize=maximize)
    for k in range(3, 8):
        assert [tuple(int(x) for x in r) for r in got[k][0]] == list(ref[k][0]), k
        assert np.abs(got[k][1] - ref[k][1]).max() < 1e-9, k
    if kind == "paired_effect":
        assert tuple(got[3][0][0]) == (2, 5, 9)


@pytest.mark.parametrize("kind,measure", [("mean", "omega"), ("paired_effect", "omega"), ("mean", "s")])
def test_greedy_multi_device_matches_host_loop(env, kind, measure):
    """The device greedy over datasets (objective formed in its selection kernel) against the
    host-driven loop (evaluator call + objective reduction per order): the same solutions and
    objectives within 1e-9 at every order, both directions."""
    torch, api, search, synth, orc = env
    X = synth.condition_pairs(8)
    Sig = torch.from_numpy(np.stack([orc.gc_covariance(x) for x in X])).cuda()
    for maximize in (True, False):
        say(f"greedy over 16 datasets, {kind} of {measure}, orders 3..9, device vs host loop, maximize={maximize}")
        got = search.greedy_multi(Sig, 3, 9, kappa=8, measure=measure, kind=kind, maximize=maximize, on_device=True)
        ref = search.greedy_multi(Sig, 3, 9, kappa=8, measure=measure, kind=kind, maximize=maximize, on_device=False)
        for k in range(3, 10):
            assert np.array_equal(got[k][0], ref[k][0]), k
            assert np.abs(got[k][1] - ref[k][1]).max() < 1e-9, k

