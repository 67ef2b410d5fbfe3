"""Plain reference versions of the n-plet searches, on the FP64 oracle.

TEST INFRASTRUCTURE ONLY (see the package header): written independently of
``paper_2501_03381_amd.search`` and sharing no code with it.

greedy (Methods, "Heuristics", "Greedy Algorithm"): the kappa best n-plets of the first order by
exhaustive evaluation; then, order after order, every kept n-plet is extended by each variable it
lacks, the distinct extensions are evaluated and the kappa best kept.  Ties go to the
lexicographically smaller n-plet; n-plets that are not positive definite never win.

swap_refine: best-improvement local search over single-variable swaps.  Candidate swaps are
ranked by the first-order change of Omega, computed from the oracle's explicit-inverse gradient
(a change Delta of Sigma_S moves Omega by sum_ab G_ab Delta_ab); the top_m ranked swaps (all when
top_m is None) are evaluated exactly and the best improvement above tol is taken.
"""
from __future__ import annotations

import numpy as np

from . import enumerate_nplets, eval_list, grad_list, pad_list


def _omega(S, tuples):
    out, _, _ = eval_list(S, pad_list(tuples, max(len(t) for t in tuples)))
    return out[2]


def _select(tuples, om, kappa, maximize):
    keyed = []
    for t, v in zip(tuples, om):
        if np.isnan(v):
            continue
        keyed.append(((-v if maximize else v), t))
    keyed.sort()                         # by objective, then lexicographic tuple
    best = keyed[:kappa]
    return [t for _, t in best], np.array([(-s if maximize else s) for s, _ in best])


def greedy(S, k_first, k_last, kappa=16, maximize=True):
    N = S.shape[0]
    first = [tuple(int(x) for x in row if x >= 0) for row in enumerate_nplets(N, k_first, k_first)]
    sols, vals = _select(first, _omega(S, first), kappa, maximize)
    out = {k_first: (sols, vals)}
    for k in range(k_first + 1, k_last + 1):
        cand = set()
        for s in sols:
            for v in range(N):
                if v not in s:
                    cand.add(tuple(sorted(s + (v,))))
        cand = sorted(cand)
        sols, vals = _select(cand, _omega(S, cand), kappa, maximize)
        out[k] = (sols, vals)
    return out


def predicted_swap_change(S, sol, G, u, v):
    """First-order change of Omega when variable u of sol is replaced by v."""
    d = 0.0
    for j in sol:
        if j == u:
            continue
        d += 2.0 * G[u, j] * (S[v, j] - S[u, j])
    d += G[u, u] * (S[v, v] - S[u, u])
    return d


def swap_refine(S, sol, maximize=True, top_m=None, max_iter=50, tol=1e-7):
    N = S.shape[0]
    cur = tuple(sol)
    val = _omega(S, [cur])[0]
    sign = 1.0 if maximize else -1.0
    it = 0
    while it < max_iter:
        w = np.zeros((4, 1))
        w[2, 0] = 1.0
        G = grad_list(S, pad_list([cur]), w)
        ranked = []
        for u in cur:
            for v in range(N):
                if v in cur:
                    continue
                ranked.append((-sign * predicted_swap_change(S, cur, G, u, v), u, v))
        ranked.sort()
        if top_m is not None:
            ranked = ranked[:top_m]
        cands = [tuple(sorted([x for x in cur if x != u] + [v])) for _, u, v in ranked]
        om = _omega(S, cands)
        best = None
        for c, o in zip(cands, om):
            if np.isnan(o):
                continue
            gain = sign * (o - val)
            if gain > tol and (best is None or gain > best[0] or (gain == best[0] and c < best[1])):
                best = (gain, c, o)
        if best is None:
            break
        cur, val = best[1], best[2]
        it += 1
    return cur, val, it
