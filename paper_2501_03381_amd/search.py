"""Proposal-driven search for n-plets of extreme O-information on the GPU evaluator.

Greedy growth (Methods, "Heuristics", "Greedy Algorithm"): start from the kappa best n-plets of an
exhaustive pass over the first order, then at every step extend each current solution by every
variable it does not contain, evaluate all the candidates of the next order in one batched call
and keep the kappa best.  Candidates reached from two parents are one candidate (the kept
solutions are distinct n-plets).  Ties are broken by the lexicographically smaller n-plet.

Swap refinement (an extension the paper points to as future work, Discussion): for a solution S
of order k, the adjoint kernel gives G = dOmega/dSigma_S; swapping u in S for v outside changes
Sigma_S in row and column u only, so to first order

    dOmega(u -> v) ~= 2 sum_{j in S, j != u} G_uj (Sigma_vj - Sigma_uj) + G_uu (Sigma_vv - Sigma_uu).

The swaps are ranked by this prediction, the best `top_m` are evaluated exactly in one batched
call, and the best exact improvement is taken; the search stops when no evaluated swap improves
the objective by more than `tol`.

Index bookkeeping (candidate rows, de-duplication) is host NumPy; every measure and every
gradient comes from the HIP kernels (LIST selection, streaming top-K reduction, adjoint).
"""
from __future__ import annotations

import numpy as np
import torch

from . import api, binding as B


def _rows_to_device(rows: np.ndarray, device) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(rows, dtype=np.int32)).to(device)


def _best_rows(Sigma: torch.Tensor, rows: np.ndarray, kappa: int, maximize: bool, precision: str):
    """The kappa best rows of a [B][k] candidate list by Omega (device reducer; ties: lower row)."""
    k = rows.shape[1]
    st = api.nplets_reduce(Sigma, nplets=_rows_to_device(rows, Sigma.device), topk=kappa, hist_bins=0,
                           precision=precision)
    tv, tg, _ = st.result()
    slot = 0 if maximize else 1
    g = tg[0, k, slot]
    keep = g >= 0
    return rows[g[keep]], tv[0, k, slot][keep]


def expand(solutions: np.ndarray, N: int) -> np.ndarray:
    """Every solution extended by each variable it lacks, sorted within rows, duplicates removed,
    rows in lexicographic order."""
    kappa, t = solutions.shape
    mask = np.zeros((kappa, N), dtype=bool)
    mask[np.arange(kappa)[:, None], solutions] = True
    par, var = np.nonzero(~mask)
    rows = np.concatenate([solutions[par], var[:, None]], axis=1)
    rows.sort(axis=1)
    return np.unique(rows, axis=0).astype(np.int32)


def greedy(Sigma: torch.Tensor, k_first: int, k_last: int, kappa: int = 16, maximize: bool = True,
           precision: str = "fp64"):
    """Greedy growth from order k_first to k_last.

    Returns {k: (solutions [<=kappa][k] int32, Omega [<=kappa])}, best first at every order.
    """
    S = Sigma[0] if Sigma.dim() == 3 else Sigma
    N = S.shape[0]
    if not (1 <= k_first <= k_last <= N):
        raise ValueError("need 1 <= k_first <= k_last <= N")
    if not (1 <= kappa <= 256):
        raise ValueError("kappa must be in 1..256 (the reducer's list length)")
    if N <= B.THOI_MAX_N_RANGE:
        # exhaustive first order, unranked on the device
        st = api.nplets_reduce(S, orders=(k_first, k_first), topk=kappa, hist_bins=0, precision=precision)
        tv, tg, _ = st.result()
        slot = 0 if maximize else 1
        g = tg[0, k_first, slot]
        g = g[g >= 0]
        sols = np.array([api.unrank(N, k_first, int(x)) for x in g], dtype=np.int32).reshape(len(g), k_first)
        out = {k_first: (sols, tv[0, k_first, slot][: len(g)])}
    else:
        # wider systems: the first order as an explicit list (lexicographic rows)
        import itertools
        rows = np.array(list(itertools.combinations(range(N), k_first)), dtype=np.int32).reshape(-1, k_first)
        sols, vals = _best_rows(S, rows, kappa, maximize, precision)
        out = {k_first: (sols, vals)}
    for k in range(k_first + 1, k_last + 1):
        cand = expand(sols, N)
        sols, vals = _best_rows(S, cand, kappa, maximize, precision)
        out[k] = (sols, vals)
    return out


def _omega_rows(S: torch.Tensor, rows: np.ndarray, precision: str) -> np.ndarray:
    odt = torch.float64 if precision == "fp64" else torch.float32
    out, _ = api.nplets_measures(S, nplets=_rows_to_device(rows, S.device), precision=precision, out_dtype=odt)
    return out[2].double().cpu().numpy().reshape(-1)          # S is [N, N]: out is [planes, B]


def swap_scores(Sigma_h: np.ndarray, sol: np.ndarray, G: np.ndarray) -> np.ndarray:
    """First-order change of Omega for every swap u -> v (u in sol, v outside): [k][N], with
    NaN where v is already in sol.  G is dOmega/dSigma (entries treated as independent)."""
    k = len(sol)
    N = Sigma_h.shape[0]
    Gs = G[np.ix_(sol, sol)]
    Ss = Sigma_h[np.ix_(sol, sol)]
    # 2 sum_{j != u} G_uj (Sigma_vj - Sigma_uj) + G_uu (Sigma_vv - Sigma_uu)
    Sv = Sigma_h[:, sol]                         # [N][k]: Sigma_vj
    off = Gs.copy()
    np.fill_diagonal(off, 0.0)
    term = 2.0 * (off @ Sv.T - (off * Ss).sum(1)[:, None])          # [k][N]
    term += np.diag(Gs)[:, None] * (np.diag(Sigma_h)[None, :] - np.diag(Ss)[:, None])
    term[:, sol] = np.nan
    return term


def swap_refine(Sigma: torch.Tensor, solutions: np.ndarray, maximize: bool = True, top_m: int | None = None,
                max_iter: int = 50, tol: float = 1e-7, precision: str = "fp64"):
    """Refine each row of `solutions` (all of one order k) by single-variable swaps ranked with the
    adjoint.  top_m=None evaluates every swap.  Returns (solutions, Omega, iterations per row)."""
    S = Sigma[0] if Sigma.dim() == 3 else Sigma
    N = S.shape[0]
    Sh = S.double().cpu().numpy()
    sols = np.array(solutions, dtype=np.int32, copy=True)
    kappa, k = sols.shape
    vals = _omega_rows(S, sols, precision)
    active = np.ones(kappa, dtype=bool)
    iters = np.zeros(kappa, dtype=np.int64)
    sign = 1.0 if maximize else -1.0
    Srep = S[None].expand(kappa, N, N).contiguous()
    for _ in range(max_iter):
        if not active.any():
            break
        # per-solution gradients in one adjoint call: dataset d carries solution d only
        w = torch.zeros((4, kappa, kappa), dtype=torch.float32, device=S.device)
        w[2, torch.arange(kappa), torch.arange(kappa)] = 1.0
        G = api.measures_backward(Srep, w, nplets=_rows_to_device(sols, S.device)).double().cpu().numpy()
        cand_rows, owner = [], []
        for r in np.nonzero(active)[0]:
            sc = sign * swap_scores(Sh, sols[r], G[r])
            us, vs = np.nonzero(~np.isnan(sc))
            order = np.lexsort((vs, us, -sc[us, vs]))          # best prediction first, then (u, v)
            if top_m is not None:
                order = order[:top_m]
            for i in order:
                row = sols[r].copy()
                row[us[i]] = vs[i]
                row.sort()
                cand_rows.append(row)
                owner.append(r)
        cand = np.array(cand_rows, dtype=np.int32).reshape(len(cand_rows), k)
        owner = np.array(owner)
        om = _omega_rows(S, cand, precision)
        for r in np.nonzero(active)[0]:
            sel = np.nonzero(owner == r)[0]
            gain = sign * (om[sel] - vals[r])
            gain = np.where(np.isnan(gain), -np.inf, gain)
            best_gain = gain.max() if len(sel) else -np.inf
            if not best_gain > tol:
                active[r] = False
                continue
            ties = sel[gain == best_gain]
            pick = ties[np.lexsort(cand[ties].T[::-1])[0]]           # lexicographically smallest n-plet
            sols[r] = cand[pick]
            vals[r] = om[pick]
            iters[r] += 1
    return sols, vals, iters
