"""The test-side checks (tests/_checks.py) against brute force, so that the GPU parity tests built
on them can be trusted: the index map against itertools order, the top-K rule and the
histogram rule against planted lists and counts."""
import itertools
import math

import numpy as np
import pytest

from _checks import check_hist, check_topk, lex_rank, lex_unrank


@pytest.mark.parametrize("N,kmin,kmax", [(9, 0, 9), (12, 3, 7), (20, 18, 20)])
def test_lex_rank_unrank_is_itertools_order(N, kmin, kmax):
    g = 0
    for k in range(kmin, kmax + 1):
        for c in itertools.combinations(range(N), k):
            assert lex_rank(c, N, kmin) == g
            assert lex_unrank(g, N, kmin) == c
            g += 1
    assert g == sum(math.comb(N, k) for k in range(kmin, kmax + 1))
    if kmax == N:
        with pytest.raises(ValueError):
            lex_unrank(g, N, kmin)


def test_lex_rank_wide():
    # deep inside an order of a wide system: unrank inverts rank on random tuples
    rng = np.random.default_rng(0)
    for N, k in ((62, 30), (100, 20), (40, 3)):
        for _ in range(200):
            c = tuple(sorted(rng.choice(N, k, replace=False).tolist()))
            assert lex_unrank(lex_rank(c, N, 1), N, 1) == c


def _list(v, g, K, largest):
    order = np.lexsort((g, -v if largest else v))[:K]
    out_v = np.full(K + 3, np.nan)
    out_g = -np.ones(K + 3, dtype=np.int64)
    out_v[:len(order)] = v[order]
    out_g[:len(order)] = g[order]
    return out_v, out_g


def test_check_topk_accepts_exact_and_rejects_mistakes():
    rng = np.random.default_rng(1)
    v = rng.standard_normal(500)
    g = np.arange(1000, 1500)
    for largest in (True, False):
        lv, lg = _list(v, g, 20, largest)
        check_topk(lv, lg, g, v, 20, 1e-9, largest)
        # values within tolerance of the K-th may be exchanged: put the 21st 1e-4 from the
        # 20th, then a list holding the 21st instead of the 20th passes at tol 1e-3
        rank = np.argsort(-v if largest else v, kind="stable")
        w = v.copy()
        w[rank[20]] = v[rank[19]] + (-1e-4 if largest else 1e-4)
        alt = w.copy()
        alt[rank[19]], alt[rank[20]] = w[rank[20]], w[rank[19]]
        lv2, lg2 = _list(alt, g, 20, largest)
        lv2[:20] = w[[int(x) - 1000 for x in lg2[:20]]]
        check_topk(lv2, lg2, g, w, 20, 1e-3, largest)
        with pytest.raises(AssertionError):
            check_topk(lv2, lg2, g, w, 20, 1e-6, largest)
        # a dropped member, a wrong value, a wrong order: each caught
        bad = lg.copy()
        bad[3] = g[np.argsort(v)[250]]
        with pytest.raises(AssertionError):
            check_topk(lv, bad, g, v, 20, 1e-9, largest)
        badv = lv.copy()
        badv[5] += 0.01
        with pytest.raises(AssertionError):
            check_topk(badv, lg, g, v, 20, 1e-3, largest)
        swp = lv.copy(), lg.copy()
        swp[0][[0, 1]] = swp[0][[1, 0]]
        swp[1][[0, 1]] = swp[1][[1, 0]]
        with pytest.raises(AssertionError):
            check_topk(swp[0], swp[1], g, v, 20, 1e-9, largest)
    # fewer n-plets than K
    lv, lg = _list(v[:7], g[:7], 20, True)
    check_topk(lv, lg, g[:7], v[:7], 20, 1e-9, True)


def test_check_hist_exact_and_near_edges():
    rng = np.random.default_rng(2)
    v = rng.uniform(-1.2, 1.3, 4000)
    v[:3] = [-1.0, 1.0, 0.0]                      # on lo, on hi, on an inner edge
    lo, hi, bins = -1.0, 1.0, 16
    ref = np.zeros(bins + 2, dtype=np.int64)
    inside = (v >= lo) & (v <= hi)
    b = np.minimum(np.floor((v[inside] - lo) / (hi - lo) * bins).astype(int), bins - 1)
    np.add.at(ref, b, 1)
    ref[bins], ref[bins + 1] = (v < lo).sum(), (v > hi).sum()
    assert check_hist(ref, v, lo, hi, bins, 0.0) == 0
    # moving a value across an edge is allowed only when it lies within tol of that edge
    moved = ref.copy()
    moved[8] -= 1
    moved[7] += 1                                  # the value 0.0 sits on the edge of bins 7 | 8
    check_hist(moved, v, lo, hi, bins, 1e-9)
    with pytest.raises(AssertionError):
        check_hist(moved, v, lo, hi, bins, 0.0)
    far = ref.copy()
    far[2] -= 1
    far[9] += 1
    with pytest.raises(AssertionError):
        check_hist(far, v, lo, hi, bins, 1e-3)
    with pytest.raises(AssertionError):
        check_hist(ref[:-1].tolist() + [ref[-1] + 1], v, lo, hi, bins, 1e-3)
