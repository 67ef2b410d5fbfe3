"""Test-side helpers shared by the GPU parity tests.  Nothing here calls the HIP library: the
n-plet index map is written out from the binomial definition of lexicographic rank, and the
reducer checks compare against values the FP64 oracle computed.

* ``lex_rank`` / ``lex_unrank``: global index g of an n-plet in the enumeration the library uses
  (orders kmin.. ascending; inside an order the k-subsets of {0..N-1} in lexicographic order,
  the order of ``itertools.combinations``; Supplementary, Eq. comb counts them).
* ``check_topk``: the acceptance rule for a top-K / bottom-K list when several lists are correct
  (values within tolerance of the K-th one may be exchanged): every reported (g, value) matches
  the reference value of g, the K-th reported value matches the reference K-th value, every
  reference n-plet clearly beyond the K-th value is reported, the list is sorted with ties by the
  lower g.
* ``check_hist``: a histogram against the reference values binned with the same rule; a value
  within ``tol`` of a bin edge may fall on either side, every other value must be in its bin.
"""
from __future__ import annotations

import math

import numpy as np


def lex_rank(c, N: int, kmin: int) -> int:
    """Global index of the sorted tuple c (orders kmin..len(c)-1 come first)."""
    k = len(c)
    g = sum(math.comb(N, j) for j in range(kmin, k))
    x = 0
    for i, v in enumerate(c):
        for y in range(x, v):
            g += math.comb(N - 1 - y, k - 1 - i)
        x = v + 1
    return g


def lex_unrank(g: int, N: int, kmin: int) -> tuple:
    """Inverse of lex_rank: the n-plet at global index g."""
    k = kmin
    while g >= math.comb(N, k):
        g -= math.comb(N, k)
        k += 1
        if k > N:
            raise ValueError("index beyond the enumeration")
    out, x = [], 0
    for i in range(k):
        m = k - 1 - i
        while g >= math.comb(N - 1 - x, m):
            g -= math.comb(N - 1 - x, m)
            x += 1
        out.append(x)
        x += 1
    return tuple(out)


def check_topk(vals, gs, ref_g, ref_v, K: int, tol: float, largest: bool, what: str = ""):
    """vals/gs: the reported list of one order (length >= min(K, count), unused slots g = -1);
    ref_g/ref_v: every n-plet of that order (global index, reference value)."""
    ref_g = np.asarray(ref_g, dtype=np.int64)
    ref_v = np.asarray(ref_v, dtype=np.float64)
    ok = ~np.isnan(ref_v)
    ref_g, ref_v = ref_g[ok], ref_v[ok]
    n = min(K, len(ref_g))
    vals = np.asarray(vals, dtype=np.float64)
    gs = np.asarray(gs, dtype=np.int64)
    assert np.all(gs[:n] >= 0) and np.all(gs[n:] == -1), f"{what}: {n} slots expected"
    v, g = vals[:n], gs[:n]
    assert len(set(g.tolist())) == n, f"{what}: repeated n-plet"
    # sorted, ties by the lower g
    sgn = -1.0 if largest else 1.0
    order = np.lexsort((g, sgn * v))
    assert np.array_equal(order, np.arange(n)), f"{what}: list not in (value, g) order"
    # (i) every reported value is the reference value of its n-plet
    pos = {int(x): i for i, x in enumerate(ref_g.tolist())}
    assert all(int(x) in pos for x in g), f"{what}: reported n-plet outside the order"
    rv = ref_v[[pos[int(x)] for x in g]]
    err = np.abs(rv - v)
    assert err.max() <= tol, f"{what}: reported value off by {err.max():.3e}"
    # (ii) the K-th value
    srt = np.sort(ref_v)[::-1] if largest else np.sort(ref_v)
    kth = srt[n - 1]
    assert abs(v[n - 1] - kth) <= tol, f"{what}: K-th value {v[n - 1]} vs {kth}"
    # (iii) membership: whatever is clearly beyond the K-th value is reported, and nothing
    # clearly short of it is
    beyond = ref_g[ref_v > kth + tol] if largest else ref_g[ref_v < kth - tol]
    missing = set(beyond.tolist()) - set(g.tolist())
    assert not missing, f"{what}: {len(missing)} n-plets beyond the K-th value not reported"
    short = rv < kth - tol if largest else rv > kth + tol
    assert not short.any(), f"{what}: reported n-plet clearly short of the K-th value"
    return float(err.max())


def _bin(v, lo, hi, bins):
    b = np.floor((v - lo) / (hi - lo) * bins).astype(np.int64)
    return np.minimum(b, bins - 1)


def check_hist(h, ref_v, lo: float, hi: float, bins: int, tol: float, what: str = ""):
    """h: [bins + 2] counts (bins, under, over); ref_v: reference values (NaN not counted).
    Returns the number of reference values within tol of an edge."""
    h = np.asarray(h, dtype=np.int64)
    v = np.asarray(ref_v, dtype=np.float64)
    v = v[~np.isnan(v)]
    assert int(h.sum()) == len(v), f"{what}: total {h.sum()} vs {len(v)}"

    def slot(x):
        out = np.where(x < lo, bins, np.where(x > hi, bins + 1, 0))
        inside = (x >= lo) & (x <= hi)
        out[inside] = _bin(x[inside], lo, hi, bins)
        return out

    a, b = slot(v - tol), slot(v + tol)
    certain = a == b
    lower = np.zeros(bins + 2, dtype=np.int64)
    np.add.at(lower, a[certain], 1)
    upper = lower.copy()
    unc = ~certain
    for s0, s1 in zip(a[unc], b[unc]):
        # every slot the value could reach (under/overflow sit outside [lo, hi])
        reach = {int(s0), int(s1)}
        if s0 < bins and s1 < bins:
            reach.update(range(int(s0), int(s1) + 1))
        for s in reach:
            upper[s] += 1
    bad = np.nonzero((h < lower) | (h > upper))[0]
    assert bad.size == 0, f"{what}: bins {bad.tolist()} outside [certain, certain + near-edge] " \
                          f"(got {h[bad].tolist()}, bounds {lower[bad].tolist()}..{upper[bad].tolist()})"
    return int(unc.sum())


def fd_nplet_grad(orc, S, row, w, h: float = 1e-6):
    """Central finite differences (FP64) of sum_m w[m] * measure_m of one n-plet with respect to
    the covariance entries, from the oracle's literal measures (one LU per determinant).  The
    symmetric pair (i, j), (j, i) is perturbed together by +-h, so the difference quotient is
    G_ij (i == j) or 2 G_ij (i != j) for the gradient G with entries treated as independent;
    returns G on the n-plet's k x k block."""
    r = np.asarray(row)
    r = r[r >= 0]
    k = len(r)
    sub = np.ascontiguousarray(np.asarray(S)[np.ix_(r, r)], dtype=np.float64)
    loc = np.arange(k, dtype=np.int32)[None, :]
    w = np.asarray(w, dtype=np.float64).reshape(4)

    def f(M):
        o, _, _ = orc.eval_list(M, loc)
        return float(o[:, 0] @ w)

    G = np.zeros((k, k))
    for i in range(k):
        for j in range(i, k):
            P, M = sub.copy(), sub.copy()
            P[i, j] += h
            M[i, j] -= h
            if i != j:
                P[j, i] += h
                M[j, i] -= h
            d = (f(P) - f(M)) / (2.0 * h)
            G[i, j] = G[j, i] = d if i == j else 0.5 * d
    return r, G
