"""Pins of the oracle's searches (CPU): greedy growth on the 100-variable concatenated PGM
(Supplementary, PGMs and the concatenated system) against closed forms, and the first-order swap
prediction against exact changes."""
import math

import numpy as np
import pytest

from paper_2501_03381_amd import synth


def omega_r_block(k, c):
    """Omega of Y plus k-1 of the X's of an R-system: an R-system itself, -Omega_S(n=k-1, c)."""
    n = k - 1
    return 0.5 * (n * math.log(1 + c * c) - math.log(1 + n * c * c))


def omega_s_sub(k, n, c):
    """Omega of Y plus m = k-1 of the n X's of an S-system: the other n-m inputs are extra noise on
    Y, so (Omega being scale invariant) it is an S-system of m inputs with c' = c / sqrt((n-m)c^2 + 1)."""
    m = k - 1
    cp = c / math.sqrt((n - m) * c * c + 1)
    return 0.5 * (math.log(1 + m * cp * cp) - m * math.log(1 + cp * cp))


@pytest.fixture(scope="module")
def osearch(orc):
    from oracle import search
    return search


def test_greedy_max_finds_the_strong_r_system(osearch):
    S = synth.concatenated_100()
    out = osearch.greedy(S, 3, 20, kappa=2, maximize=True)
    for k in range(3, 21):
        sols, vals = out[k]
        assert abs(vals[0] - omega_r_block(k, 1.0)) < 1e-9, k
        assert 39 in sols[0] and all(20 <= v <= 39 for v in sols[0]), (k, sols[0])
    assert tuple(out[20][0][0]) == tuple(range(20, 40))
    assert abs(out[20][1][0] - 5.0870320785) < 1e-9          # closed form, strong R (n=19, c=1)


def test_greedy_min_finds_the_strong_s_system(osearch):
    S = synth.concatenated_100()
    out = osearch.greedy(S, 3, 20, kappa=2, maximize=False)
    for k in range(3, 21):
        sols, vals = out[k]
        assert abs(vals[0] - omega_s_sub(k, 19, 1.0)) < 1e-9, k
        assert 79 in sols[0] and all(60 <= v <= 79 for v in sols[0]), (k, sols[0])
    assert tuple(out[20][0][0]) == tuple(range(60, 80))
    assert abs(out[20][1][0] + 5.0870320785) < 1e-9          # closed form, strong S (n=19, c=1)


def test_greedy_keeps_distinct_solutions_in_order(osearch, orc):
    rng = np.random.default_rng(5)
    S = synth.random_spd(rng, 12, 30.0)
    out = osearch.greedy(S, 2, 6, kappa=5, maximize=True)
    idx_all = orc.enumerate_nplets(12, 2, 2)
    om2, _, _ = orc.eval_list(S, idx_all)
    assert np.allclose(out[2][1], np.sort(om2[2])[::-1][:5])      # exhaustive first order
    for k, (sols, vals) in out.items():
        assert len(set(sols)) == len(sols)
        assert np.all(np.diff(vals) <= 0)


def test_swap_prediction_is_first_order(osearch, orc):
    """Replacing u by a variable v whose covariances differ from u's by delta: the predicted
    change of Omega has error O(delta^2)."""
    rng = np.random.default_rng(6)
    A = synth.random_spd(rng, 8, 20.0)
    u, sol = 3, (1, 3, 4, 6)
    a = rng.standard_normal(8)
    errs = []
    for delta in (1e-3, 1e-4):
        S = np.zeros((9, 9))
        S[:8, :8] = A
        S[8, :8] = S[:8, 8] = A[u] + delta * a
        S[8, 8] = A[u, u] + delta * abs(a[u]) + delta      # keep Sigma positive definite
        S[8, u] = S[u, 8] = A[u, u] + delta * a[u]
        w = np.zeros((4, 1))
        w[2, 0] = 1.0
        G = orc.grad_list(S, orc.pad_list([sol]), w)
        pred = osearch.predicted_swap_change(S, sol, G, u, 8)
        new = tuple(sorted([x for x in sol if x != u] + [8]))
        out, _, _ = orc.eval_list(S, orc.pad_list([sol, new]))
        errs.append(abs(pred - (out[2][1] - out[2][0])))
    assert errs[1] < errs[0] / 30                            # quadratic in delta
    assert errs[0] < 1e-4


def test_swap_refine_repairs_a_perturbed_r_system(osearch):
    """Every swap evaluated: one swap restores the strong R system (closed form)."""
    S = synth.concatenated_100()
    start = tuple(sorted([v for v in range(20, 40) if v != 25] + [85]))
    sol, val, it = osearch.swap_refine(S, start, maximize=True, top_m=None)
    assert sol == tuple(range(20, 40)) and it == 1
    assert abs(val - 5.0870320785) < 1e-9


def test_swap_refine_ranked_is_monotone_and_locally_optimal(osearch, orc):
    """Gradient-ranked swaps on correlated data: the objective never gets worse, and at the end
    none of the ranked swaps improves it."""
    rng = np.random.default_rng(8)
    S = synth.random_spd(rng, 14, 50.0)
    start = (0, 2, 5, 7, 9)
    v0 = osearch._omega(S, [start])[0]
    sol, val, it = osearch.swap_refine(S, start, maximize=False, top_m=8)
    assert val <= v0 and len(set(sol)) == 5
    assert abs(osearch._omega(S, [sol])[0] - val) < 1e-12
    # stopping point: none of the 8 best-ranked swaps of the final solution lowers Omega
    w = np.zeros((4, 1))
    w[2, 0] = 1.0
    G = orc.grad_list(S, orc.pad_list([sol]), w)
    ranked = sorted((osearch.predicted_swap_change(S, sol, G, u, v), u, v)
                    for u in sol for v in range(14) if v not in sol)[:8]
    nb = [tuple(sorted([x for x in sol if x != u] + [v])) for _, u, v in ranked]
    assert np.nanmin(osearch._omega(S, nb)) >= val - 1e-7


# ------------------------------------------------------------------------------------------------ annealing
def small_pgm():
    """R-system (5 inputs, c=1) | S-system (5 inputs, c=1) | 6 independent: N = 18."""
    return synth.block_diag(synth.r_system(5, 1.0), synth.s_system(5, 1.0), np.eye(6))


def test_anneal_across_orders_finds_the_blocks(osearch):
    S = small_pgm()
    m0 = synth.sa_initial(11, 32, 18, 3, 8)
    dr = synth.sa_draws(12, 300, 32)
    best, vb, _, _, _ = osearch.anneal(S, m0, dr, T0=0.5, alpha=0.98, maximize=True, mode="across")
    i = int(np.argmax(vb))
    assert abs(vb[i] - omega_r_block(6, 1.0)) < 1e-9 and set(range(6)) <= set(best[i])
    best, vb, _, _, _ = osearch.anneal(S, m0, dr, T0=0.5, alpha=0.98, maximize=False, mode="across")
    i = int(np.argmin(vb))
    assert abs(vb[i] + omega_r_block(6, 1.0)) < 1e-9 and set(range(6, 12)) <= set(best[i])


def test_anneal_temperature_limits(osearch):
    S = synth.random_spd(np.random.default_rng(13), 12, 20.0)
    m0 = synth.sa_initial(14, 16, 12, 3, 6)
    dr = synth.sa_draws(15, 40, 16)
    # infinite temperature: every (positive-definite) proposal is taken
    _, _, _, _, acc = osearch.anneal(S, m0, dr, T0=1e300, alpha=1.0, mode="across")
    assert all(a == 40 for a in acc)
    # zero temperature: only non-worsening moves, so the final energy is the best one and no worse
    # than the start
    e0 = osearch._omega(S, [tuple(np.nonzero(m)[0]) for m in m0])
    best, vb, cur, vc, _ = osearch.anneal(S, m0, dr, T0=1e-300, alpha=1.0, maximize=True, mode="within")
    assert np.all(np.array(vc) >= e0 - 1e-15) and np.allclose(vc, vb, rtol=0, atol=0)
    assert [len(c) for c in cur] == [int(m.sum()) for m in m0]          # within: orders kept


# ------------------------------------------------------------------------------------------------ objectives over datasets
def test_objective_definitions(orc):
    v = np.array([[1.0, 5.0, 2.0], [2.0, 5.0, np.nan], [3.0, 5.0, 1.0],
                  [0.0, 1.0, 0.0], [0.0, 1.0, 0.0], [0.0, 1.0, 0.0]])
    assert np.allclose(orc.objective(v[:3], "mean")[:2], [2.0, 5.0]) and np.isnan(orc.objective(v[:3], "mean")[2])
    eff = orc.objective(v, "paired_effect")        # P = 3: x = (1, 2, 3) -> 2 / 1; x = (4, 4, 4) -> sd 0
    assert abs(eff[0] - 2.0) < 1e-15 and np.isnan(eff[1]) and np.isnan(eff[2])
    # a t statistic written out: x = (1, 4, 6, 9), mean 5, sd sqrt(34/3)
    w = np.array([[1.0], [4.0], [6.0], [9.0], [0.0], [0.0], [0.0], [0.0]])
    assert abs(orc.objective(w, "paired_effect")[0] - 5.0 / math.sqrt(34.0 / 3.0)) < 1e-14


def test_greedy_multi_finds_the_planted_condition_effect(osearch, orc):
    X = synth.condition_pairs(6)
    Sig = np.stack([orc.gc_covariance(x) for x in X])
    out = osearch.greedy_multi(Sig, 3, 5, kappa=4, kind="paired_effect", maximize=False)
    assert out[3][0][0] == (2, 5, 9) and out[3][1][0] < -3.0
    # one dataset and the mean: the same search as the single-dataset greedy
    one = osearch.greedy_multi(Sig[:1], 3, 6, kappa=5, kind="mean", maximize=True)
    ref = osearch.greedy(Sig[0], 3, 6, kappa=5, maximize=True)
    for k in range(3, 7):
        assert list(one[k][0]) == list(ref[k][0]) and np.allclose(one[k][1], ref[k][1], rtol=0, atol=1e-15)
