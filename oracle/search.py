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


def anneal(S, masks0, draws, T0=1.0, alpha=0.99, maximize=True, mode="within", k_min=3, k_max=None):
    """Batched simulated annealing over masked n-plets (Methods, "Simulated Annealing Algorithm").

    Every chain proposes one neighbour per iteration: within an order a swap (a member out, an
    outsider in); across orders an addition when draws['move'] < 1/3, a removal when it is in
    [1/3, 2/3), else a swap, a swap also replacing a move that would leave [k_min, k_max].  The
    member and the outsider are the floor(u * count)-th in ascending order, u from draws['a'] and
    draws['b'].  Energy E = Omega (maximising) or -Omega; a proposal with dE > 0 is taken, otherwise
    with probability exp(dE / Temp) (the Metropolis rule; the printed rule's sign is garbled),
    decided by draws['accept'] < exp(dE / Temp).  Temp = T0 * alpha^t.  Non-positive-definite
    proposals are rejected.
    """
    kappa, N = masks0.shape
    k_max = N - 1 if k_max is None else k_max          # a swap always has an outsider to take in
    assert k_max <= N - 1 and all(k_min <= m.sum() <= k_max for m in masks0)
    sign = 1.0 if maximize else -1.0
    cur = [tuple(int(v) for v in np.nonzero(m)[0]) for m in masks0]
    E = [sign * o for o in _omega(S, cur)]
    best, Ebest = list(cur), list(E)
    accepted = [0] * kappa
    temp = T0
    for t in range(draws["accept"].shape[0]):
        props = []
        for j in range(kappa):
            inside = list(cur[j])
            outside = [v for v in range(N) if v not in cur[j]]
            k = len(inside)
            m = draws["move"][t, j]
            if mode == "across" and m < 1.0 / 3.0 and k < k_max:
                new = inside + [outside[int(draws["b"][t, j] * len(outside))]]
            elif mode == "across" and 1.0 / 3.0 <= m < 2.0 / 3.0 and k > k_min:
                drop = inside[int(draws["a"][t, j] * k)]
                new = [v for v in inside if v != drop]
            else:
                drop = inside[int(draws["a"][t, j] * k)]
                new = [v for v in inside if v != drop] + [outside[int(draws["b"][t, j] * len(outside))]]
            props.append(tuple(sorted(new)))
        Ep = [sign * o for o in _omega(S, props)]
        for j in range(kappa):
            if np.isnan(Ep[j]):
                continue
            dE = Ep[j] - E[j]
            if dE > 0 or draws["accept"][t, j] < np.exp(dE / temp):
                cur[j], E[j] = props[j], Ep[j]
                accepted[j] += 1
            if E[j] > Ebest[j]:
                best[j], Ebest[j] = cur[j], E[j]
        temp *= alpha
    return best, [sign * e for e in Ebest], cur, [sign * e for e in E], accepted


def greedy_multi(Sigmas, k_first, k_last, kappa=16, measure="omega", kind="mean", maximize=True):
    """Greedy growth on an objective over datasets: each candidate's measure in every covariance
    matrix, combined by oracle.objective, the kappa best kept (ties: lexicographic)."""
    from . import objective
    m = {"tc": 0, "dtc": 1, "omega": 2, "s": 3}[measure]
    D, N, _ = Sigmas.shape

    def score(tuples):
        idx = pad_list(tuples, max(len(t) for t in tuples))
        vals = np.stack([eval_list(Sigmas[d], idx)[0][m] for d in range(D)])
        return objective(vals, kind)

    first = [tuple(int(x) for x in row if x >= 0) for row in enumerate_nplets(N, k_first, k_first)]
    sols, vals = _select(first, score(first), kappa, maximize)
    out = {k_first: (sols, vals)}
    for k in range(k_first + 1, k_last + 1):
        cand = sorted({tuple(sorted(s + (v,))) for s in sols for v in range(N) if v not in s})
        sols, vals = _select(cand, score(cand), kappa, maximize)
        out[k] = (sols, vals)
    return out
