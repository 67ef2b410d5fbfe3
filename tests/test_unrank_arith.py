"""Host check of the arithmetic the device unranking uses for N <= 33 (not gpu).

The lane engine unranks a lexicographic rank in one pass over x = 0..N-1, carrying
b = C(N-1-x, m) in IEEE double and updating it by C(n-1, m) = C(n, m)(n-m)/n after a skip and
C(n-1, m-1) = C(n, m) m/n after a take, each quotient taken as round-to-nearest of
(b * f) * fl(1/n).  The same double operations, in the same order, are replayed here on the host
(Python floats are IEEE doubles) and compared with itertools.combinations order: exhaustively
for N <= 16 and on sampled ranks, including the first and last of every order, up to N = 33.
"""
import itertools
import math
import random


def unrank_pass(r, N, K):
    rr = float(r)
    b = float(math.comb(N - 1, K - 1))
    m = K - 1
    mask = 0
    for x in range(N):
        n = N - 1 - x
        inv = 1.0 / n if n > 0 else 0.0
        take = rr < b
        bt = float(round(b * float(m) * inv))
        bs = float(round(b * float(n - m) * inv))
        if take:
            mask |= 1 << x
            m -= 1
            b = bt
        else:
            rr = rr - b
            b = bs
    out = []
    while mask:
        out.append((mask & -mask).bit_length() - 1)
        mask &= mask - 1
    return out


def walk(r, N, K):
    out, x = [], 0
    for i in range(K):
        while math.comb(N - 1 - x, K - 1 - i) <= r:
            r -= math.comb(N - 1 - x, K - 1 - i)
            x += 1
        out.append(x)
        x += 1
    return out


def test_exhaustive_small():
    for N in (1, 2, 5, 9, 16):
        for K in range(1, N + 1):
            for r, comb in enumerate(itertools.combinations(range(N), K)):
                assert unrank_pass(r, N, K) == list(comb), (N, K, r)


def test_sampled_up_to_33():
    rng = random.Random(33)
    for N in (20, 25, 30, 33):
        for K in range(1, N + 1):
            tot = math.comb(N, K)
            for r in [0, tot - 1] + [rng.randrange(tot) for _ in range(40)]:
                assert unrank_pass(r, N, K) == walk(r, N, K), (N, K, r)
