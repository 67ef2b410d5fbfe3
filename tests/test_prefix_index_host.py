"""Host check of the prefix engine's index arithmetic (no GPU).  Replaying, with Python integers,
how a workgroup and lane find their work must produce every n-plet of the order exactly once, at
its own lexicographic rank (itertools.combinations order).  The steps replayed are:
- an order's prefixes (k - S variables, S = 3 tail variables from order 4 on, else 2) are grouped
  by their last variable q;
- each q gets units of 64 prefixes x L consecutive tails, four units per 256-thread workgroup;
- a lane's prefix is unranked among the (k-S-1)-subsets of {0..q-1}, its first tail among the
  S-subsets of {q+1..N-1};
- the position of the prefix's first n-plet is a hockey-stick sum of binomials, and the lane steps
  through the following tails by the lexicographic successor."""
import itertools
import math

import pytest

THREADS = 256


def tail_of(k):
    return 3 if k >= 4 else 2


def tails(N, k, D=1):
    """Tails per lane: a power of two up to 16, about C(N, k) D / 2^18."""
    want = math.comb(N, k) * D / 262144.0
    L = 1
    while L < 16 and 2 * L <= want:
        L *= 2
    return L


def units(N, k, q, L):
    S = tail_of(k)
    M = k - S
    npref = math.comb(q, M - 1)
    ntail = math.comb(N - 1 - q, S)
    nchunk = (ntail + L - 1) // L
    return npref, ntail, nchunk, (npref + 63) // 64 * nchunk


def blocks(N, k, L):
    S = tail_of(k)
    return sum((units(N, k, q, L)[3] + 3) // 4 for q in range(k - S - 1, N - S))


def unrank(r, n, j):
    """r-th j-subset of {0..n-1} in lexicographic order."""
    out, x = [], 0
    for i in range(j):
        m = j - 1 - i
        while x < n:
            b = math.comb(n - 1 - x, m)
            if r < b:
                break
            r -= b
            x += 1
        out.append(x)
        x += 1
    return out


def lane_nplets(N, k, blk, thread, L):
    S = tail_of(k)
    M = k - S
    lb, q = blk, k - S - 1
    while q <= N - 1 - S:
        npref, ntail, nchunk, nunits = units(N, k, q, L)
        nb = (nunits + 3) // 4
        if lb < nb:
            break
        lb -= nb
        q += 1
    unit = lb * 4 + thread // 64
    if unit >= nunits:
        return []
    pb, ch = divmod(unit, nchunk)
    r = pb * 64 + thread % 64
    if r >= npref:
        return []
    c = unrank(r, q, M - 1) + [q]
    pos, prev = 0, -1
    for i in range(M):
        pos += math.comb(N - prev - 1, k - i) - math.comb(N - c[i], k - i)
        prev = c[i]
    t0 = ch * L
    tail = [q + 1 + x for x in unrank(t0, N - 1 - q, S)]
    out = []
    for it in range(L):
        tr = t0 + it
        if tr >= ntail:
            break
        out.append((pos + tr, tuple(c + tail)))
        piv = max(i for i in range(S) if tail[i] < N - S + i) if tr + 1 < ntail else 0
        tail[piv] += 1
        for i in range(piv + 1, S):
            tail[i] = tail[i - 1] + 1
    return out


def test_tails_per_lane():
    assert tails(20, 10) == 1 and tails(20, 10, 64) == 32 // 2 and tails(30, 15) == 16 and tails(30, 5) == 1


@pytest.mark.parametrize("N,k,L", [(6, 3, 1), (9, 4, 2), (10, 5, 8), (12, 4, 16), (13, 7, 4), (14, 14, 16), (16, 9, 8),
                                   (20, 3, 1), (20, 10, 1), (20, 10, 16)])
def test_prefix_lanes_cover_every_nplet_once_at_its_rank(N, k, L):
    want = list(itertools.combinations(range(N), k))
    got = {}
    for blk in range(blocks(N, k, L)):
        for th in range(THREADS):
            for pos, t in lane_nplets(N, k, blk, th, L):
                assert pos not in got, (N, k, pos)
                got[pos] = t
    assert len(got) == len(want)
    assert all(got[i] == want[i] for i in range(len(want)))


def test_prefix_wave_lanes_walk_the_same_tails():
    """All active lanes of a wavefront have the same last prefix variable and the same tails, so
    the levels re-bordered after each step are the same for the whole wavefront."""
    N, k, L = 18, 8, 8
    S = tail_of(k)
    for blk in range(blocks(N, k, L)):
        for w in range(4):
            seqs = {tuple(t[k - S - 1:] for _, t in lane_nplets(N, k, blk, 64 * w + ln, L))
                    for ln in range(64) if lane_nplets(N, k, blk, 64 * w + ln, L)}
            assert len(seqs) <= 1
