"""GPU parity of the n-plet searches (greedy growth, gradient-ranked swap refinement) against the
oracle's plain versions, plus closed forms on the concatenated PGM."""
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
    from oracle import search as osearch
    from paper_2501_03381_amd import binding, search, synth
    binding.lib()
    assert torch.cuda.is_available()
    return torch, search, osearch, synth, orc


def dev(torch, x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def omega_r_block(k, c):
    n = k - 1
    return 0.5 * (n * math.log(1 + c * c) - math.log(1 + n * c * c))


@pytest.mark.parametrize("maximize", [True, False])
def test_greedy_matches_oracle_latent20(env, maximize):
    torch, search, osearch, synth, orc = env
    S = orc.gc_covariance(synth.latent_20())
    say(f"greedy latent_20 orders 3..12 kappa 8 maximize={maximize} fp64")
    got = search.greedy(dev(torch, S), 3, 12, kappa=8, maximize=maximize, precision="fp64")
    ref = osearch.greedy(S, 3, 12, kappa=8, maximize=maximize)
    for k in range(3, 13):
        gs, gv = got[k]
        rs, rv = ref[k]
        assert [tuple(int(x) for x in r) for r in gs] == list(rs), k
        assert np.abs(gv - rv).max() < 1e-9, k
    say("greedy latent_20 fp32_refine")
    got32 = search.greedy(dev(torch, S), 3, 12, kappa=8, maximize=maximize, precision="fp32_refine")
    for k in range(3, 13):
        assert abs(got32[k][1][0] - ref[k][1][0]) < 1e-3, k
        # every reported value is the n-plet's own Omega
        out, _, _ = orc.eval_list(S, orc.pad_list([tuple(r) for r in got32[k][0]]))
        assert np.abs(out[2] - got32[k][1]).max() < 1e-3, k


def test_greedy_pgm_closed_forms(env):
    torch, search, osearch, synth, orc = env
    S = synth.concatenated_100()
    say("greedy concatenated PGM N=100 orders 3..20 maximize")
    out = search.greedy(dev(torch, S), 3, 20, kappa=4, maximize=True, precision="fp64")
    for k in range(3, 21):
        sols, vals = out[k]
        assert abs(vals[0] - omega_r_block(k, 1.0)) < 1e-9, k
        assert 39 in sols[0] and all(20 <= v <= 39 for v in sols[0]), k
        out_o, _, _ = orc.eval_list(S, orc.pad_list([tuple(r) for r in sols]))
        assert np.abs(out_o[2] - vals).max() < 1e-9, k         # ties may pick other members: check validity
    assert tuple(out[20][0][0]) == tuple(range(20, 40))


def test_greedy_device_matches_host_loop(env):
    """The device greedy (two launches per order, two-word masks above 64 variables) against the
    host-driven loop over the batched reducer: the same solutions in the same order and values
    within 1e-9, on the 100-variable latent model and on latent_20, both directions."""
    torch, search, osearch, synth, orc = env
    cases = [(orc.gc_covariance(synth.latent_100()[0]), 3, 14, 12), (orc.gc_covariance(synth.latent_20()), 2, 16, 32)]
    for S, k0, k1, kappa in cases:
        for maximize in (True, False):
            say(f"greedy N={S.shape[0]} orders {k0}..{k1} kappa {kappa} maximize={maximize}: device vs host loop")
            got = search.greedy(dev(torch, S), k0, k1, kappa=kappa, maximize=maximize, on_device=True)
            ref = search.greedy(dev(torch, S), k0, k1, kappa=kappa, maximize=maximize, on_device=False)
            for k in range(k0, k1 + 1):
                assert np.array_equal(got[k][0], ref[k][0]), k
                assert np.abs(got[k][1] - ref[k][1]).max() < 1e-9, k


def test_greedy_device_selection_paths(env):
    """Each path of the device selection against the host-driven loop on latent_20: the whole
    bitonic sort (kappa N <= 128, and kappa > 128), and the chunk sort with pairwise best-half
    merges (kappa <= 128; 2560 slots, sorted as 4096 entries in 32 chunks)."""
    torch, search, osearch, synth, orc = env
    S = orc.gc_covariance(synth.latent_20())
    for k0, k1, kappa in ((2, 6, 4), (2, 5, 160), (2, 6, 128)):
        for maximize in (True, False):
            say(f"greedy selection N=20 orders {k0}..{k1} kappa {kappa} maximize={maximize}: device vs host loop")
            got = search.greedy(dev(torch, S), k0, k1, kappa=kappa, maximize=maximize, on_device=True)
            ref = search.greedy(dev(torch, S), k0, k1, kappa=kappa, maximize=maximize, on_device=False)
            for k in range(k0, k1 + 1):
                assert np.array_equal(got[k][0], ref[k][0]), (kappa, k)
                assert np.abs(got[k][1] - ref[k][1]).max() < 1e-9, (kappa, k)


def _gpu_gradients(torch, S, sols):
    from paper_2501_03381_amd import api
    kappa, N = len(sols), S.shape[0]
    Sd = dev(torch, S)
    Srep = Sd[None].expand(kappa, N, N).contiguous()
    w = torch.zeros((4, kappa, kappa), dtype=torch.float32, device=Sd.device)
    w[2, torch.arange(kappa), torch.arange(kappa)] = 1.0
    rows = dev(torch, np.array(sols, dtype=np.int32))
    return api.measures_backward(Srep, w, nplets=rows).double().cpu().numpy()


def test_swap_scores_match_oracle(env):
    torch, search, osearch, synth, orc = env
    S = orc.gc_covariance(synth.latent_20())
    sols = [(0, 3, 5, 9, 12), (1, 2, 4, 8, 13, 17, 19), (3, 6, 7, 10)]
    say("swap sensitivity map from the adjoint vs oracle gradient")
    Gall = _gpu_gradients(torch, S, sols[1:2] * 3)        # three datasets, one solution each
    assert np.abs(Gall[0] - Gall[2]).max() == 0.0
    for sol in sols:
        Gd = _gpu_gradients(torch, S, [sol])[0]
        sc = search.swap_scores(S, np.array(sol), Gd)
        w = np.zeros((4, 1))
        w[2, 0] = 1.0
        Go = orc.grad_list(S, orc.pad_list([sol]), w)
        for a, u in enumerate(sol):
            for v in range(20):
                if v in sol:
                    assert np.isnan(sc[a, v])
                    continue
                ref = osearch.predicted_swap_change(S, sol, Go, u, v)
                assert abs(sc[a, v] - ref) < 1e-5 * max(1.0, abs(ref)), (sol, u, v)


def test_swap_refine_matches_oracle(env):
    torch, search, osearch, synth, orc = env
    S = orc.gc_covariance(synth.latent_20())
    starts = [(0, 1, 2, 10, 11, 12), (3, 4, 6, 7, 15, 16), (2, 5, 8, 13, 18, 19)]
    for maximize in (True, False):
        say(f"swap refine latent_20 (every swap evaluated) maximize={maximize}")
        sols, vals, its = search.swap_refine(dev(torch, S), np.array(starts), maximize=maximize, top_m=None)
        for r, st in enumerate(starts):
            sol, val, it = osearch.swap_refine(S, st, maximize=maximize, top_m=None)
            assert tuple(int(x) for x in sols[r]) == sol and its[r] == it
            assert abs(vals[r] - val) < 1e-9


def test_swap_refine_pgm_and_ranked(env):
    torch, search, osearch, synth, orc = env
    S = synth.concatenated_100()
    start = np.array([sorted([v for v in range(20, 40) if v != 25] + [85])])
    say("swap refine repairs the strong R system")
    sols, vals, its = search.swap_refine(dev(torch, S), start, maximize=True, top_m=None)
    assert tuple(sols[0]) == tuple(range(20, 40)) and its[0] == 1
    assert abs(vals[0] - 5.0870320785) < 1e-9
    say("gradient-ranked swap refine (top 8) on correlated data")
    Sl = orc.gc_covariance(synth.latent_20())
    st = np.array([(0, 2, 5, 7, 9), (1, 4, 6, 11, 14)])
    v0 = orc.eval_list(Sl, orc.pad_list([tuple(r) for r in st]))[0][2]
    sols, vals, its = search.swap_refine(dev(torch, Sl), st, maximize=False, top_m=8)
    assert np.all(vals <= v0 + 1e-12)
    check = orc.eval_list(Sl, orc.pad_list([tuple(r) for r in sols]))[0][2]
    assert np.abs(check - vals).max() < 1e-9


@pytest.mark.parametrize("mode", ["within", "across"])
def test_anneal_matches_oracle(env, mode):
    torch, search, osearch, synth, orc = env
    S = orc.gc_covariance(synth.latent_20())
    m0 = synth.sa_initial(21, 48, 20, 3, 10)           # mixed orders in every batch
    dr = synth.sa_draws(22, 60, 48)
    for maximize in (True, False):
        say(f"anneal latent_20 kappa 48 x 60 iterations mode={mode} maximize={maximize} fp64")
        best, vb, cur, vc, acc = search.anneal(dev(torch, S), m0, dr, T0=0.05, alpha=0.95, maximize=maximize,
                                               mode=mode)
        rb, rvb, rc, rvc, racc = osearch.anneal(S, m0, dr, T0=0.05, alpha=0.95, maximize=maximize, mode=mode)
        assert [tuple(np.nonzero(m)[0]) for m in best] == list(rb)
        assert [tuple(np.nonzero(m)[0]) for m in cur] == list(rc)
        assert list(acc) == list(racc)
        assert np.abs(vb - np.array(rvb)).max() < 1e-9 and np.abs(vc - np.array(rvc)).max() < 1e-9


def test_anneal_device_matches_host_loop_wide(env):
    """The device annealer (one launch per iteration, two-word masks above 64 variables) against
    the host-driven loop over the batched evaluator, on the 100-variable latent model (sampled
    data: no two n-plets share an Omega exactly, so both loops take the same decisions): the same
    states, best states and acceptance counts, values within 1e-9, in both modes."""
    torch, search, osearch, synth, orc = env
    S = orc.gc_covariance(synth.latent_100()[0])
    m0 = synth.sa_initial(41, 24, 100, 18, 22)
    dr = synth.sa_draws(42, 40, 24)
    for mode in ("within", "across"):
        for maximize in (True, False):
            say(f"anneal N=100 kappa 24 x 40 mode={mode} maximize={maximize}: device vs host loop")
            kw = dict(T0=0.2, alpha=0.97, maximize=maximize, mode=mode, k_min=16, k_max=24)
            got = search.anneal(dev(torch, S), m0, dr, on_device=True, **kw)
            ref = search.anneal(dev(torch, S), m0, dr, on_device=False, **kw)
            for x, y in ((got[0], ref[0]), (got[2], ref[2])):
                assert np.array_equal(x, y)
            assert np.array_equal(got[4], ref[4])
            assert np.abs(got[1] - ref[1]).max() < 1e-9 and np.abs(got[3] - ref[3]).max() < 1e-9
            assert got[4].sum() > 0


def test_search_device_loops_above_order_32(env):
    """Orders above 32 take the one-wavefront-per-n-plet kernels of the device greedy and
    annealer: both equal the host-driven loops on the 100-variable latent model."""
    torch, search, osearch, synth, orc = env
    S = orc.gc_covariance(synth.latent_100()[0])
    say("greedy N=100 orders 3..36 kappa 4: device vs host loop")
    got = search.greedy(dev(torch, S), 3, 36, kappa=4, maximize=False, on_device=True)
    ref = search.greedy(dev(torch, S), 3, 36, kappa=4, maximize=False, on_device=False)
    for k in range(3, 37):
        assert np.array_equal(got[k][0], ref[k][0]), k
        assert np.abs(got[k][1] - ref[k][1]).max() < 1e-9, k
    m0 = synth.sa_initial(51, 12, 100, 33, 38)
    dr = synth.sa_draws(52, 12, 12)
    say("anneal N=100 kappa 12 x 12 across orders 30..40: device vs host loop")
    kw = dict(T0=0.2, alpha=0.97, maximize=True, mode="across", k_min=30, k_max=40)
    got = search.anneal(dev(torch, S), m0, dr, on_device=True, **kw)
    ref = search.anneal(dev(torch, S), m0, dr, on_device=False, **kw)
    assert np.array_equal(got[0], ref[0]) and np.array_equal(got[2], ref[2])
    assert np.array_equal(got[4], ref[4])
    assert np.abs(got[1] - ref[1]).max() < 1e-9 and np.abs(got[3] - ref[3]).max() < 1e-9


def test_anneal_pgm_blocks(env):
    torch, search, osearch, synth, orc = env
    S = synth.block_diag(synth.r_system(5, 1.0), synth.s_system(5, 1.0), np.eye(6))
    m0 = synth.sa_initial(11, 32, 18, 3, 8)
    dr = synth.sa_draws(12, 300, 32)
    say("anneal small PGM across orders, maximise and minimise")
    best, vb, _, _, _ = search.anneal(dev(torch, S), m0, dr, T0=0.5, alpha=0.98, maximize=True, mode="across")
    i = int(np.argmax(vb))
    assert abs(vb[i] - omega_r_block(6, 1.0)) < 1e-9 and best[i][:6].all()
    best, vb, _, _, _ = search.anneal(dev(torch, S), m0, dr, T0=0.5, alpha=0.98, maximize=False, mode="across")
    i = int(np.argmin(vb))
    assert abs(vb[i] + omega_r_block(6, 1.0)) < 1e-9 and best[i][6:12].all()
