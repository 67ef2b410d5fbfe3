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


def combinations(N: int, k: int) -> np.ndarray:
    """Every k-subset of range(N) as sorted int32 rows [C(N, k)][k], in lexicographic order
    (built level by level: each row is extended by every value above its last one)."""
    rows = np.zeros((1, 0), dtype=np.int32)
    for level in range(k):
        last = rows[:, -1] if level > 0 else np.full(len(rows), -1, dtype=np.int64)
        # values last+1 .. N-(k-level) keep room for the remaining levels
        hi = N - (k - level)
        cnt = np.maximum(hi - last, 0)
        rep = np.repeat(np.arange(len(rows)), cnt)
        start = np.repeat(np.cumsum(cnt) - cnt, cnt)
        val = np.repeat(last + 1, cnt) + (np.arange(len(rep)) - start)
        rows = np.concatenate([rows[rep], val[:, None].astype(np.int32)], axis=1)
    return rows.astype(np.int32)


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


def _to_masks(rows: np.ndarray, N: int) -> torch.Tensor:
    """[n][k] index rows -> [n][2] int64 (two 64-bit mask words per row)."""
    words = np.zeros((len(rows), 2), dtype=np.uint64)
    for r, row in enumerate(rows):
        for v in row:
            words[r, int(v) // 64] |= np.uint64(1) << np.uint64(int(v) % 64)
    return torch.from_numpy(words.view(np.int64).copy())


def _from_masks(words: np.ndarray, N: int) -> np.ndarray:
    i = np.arange(N)
    bits = (words.view(np.uint64)[:, i // 64] >> (i % 64).astype(np.uint64)[None, :]) & np.uint64(1)
    return np.array([np.nonzero(b)[0] for b in bits], dtype=np.int32)


def _greedy_device(S: torch.Tensor, sols: np.ndarray, vals: np.ndarray, k_first: int, k_last: int, kappa: int,
                   maximize: bool, measure: int = 2, kind: int = B.THOI_OBJ_MEAN):
    """Orders k_first+1..k_last on the device (thoi_greedy) from the first order's solutions.
    S: [N, N] or [D, N, N]; the objective is `measure` combined over the D datasets by `kind`."""
    Sd = (S[None] if S.dim() == 2 else S).to(torch.float64).contiguous()
    D, N = Sd.shape[0], Sd.shape[1]
    dev = S.device
    steps = k_last - k_first
    sm = torch.zeros((steps + 1, kappa, 2), dtype=torch.int64, device=dev)
    sv = torch.zeros((steps + 1, kappa), dtype=torch.float64, device=dev)
    cnt = torch.zeros(steps + 1, dtype=torch.int32, device=dev)
    n0 = len(sols)
    sm[0, :n0] = _to_masks(sols, N).to(dev)
    sv[0, :n0] = torch.from_numpy(np.asarray(vals, dtype=np.float64)).to(dev)
    cnt[0] = n0
    ws = api._workspace(B.thoi_greedy_workspace_bytes(D, N, kappa), dev)
    B.thoi_greedy(api._ptr(Sd), D, N, k_first, steps, kappa, measure, kind, 1 if maximize else 0, api._ptr(sm),
                  api._ptr(sv), api._ptr(cnt), api._ptr(ws), ws.numel(), api._stream(dev))
    sm, sv, cnt = sm.cpu().numpy(), sv.cpu().numpy(), cnt.cpu().numpy()
    out = {}
    for s in range(steps + 1):
        n = int(cnt[s])
        out[k_first + s] = (_from_masks(sm[s, :n], N).reshape(n, k_first + s), sv[s, :n])
    return out


def greedy(Sigma: torch.Tensor, k_first: int, k_last: int, kappa: int = 16, maximize: bool = True,
           precision: str = "fp64", on_device: bool | None = None):
    """Greedy growth from order k_first to k_last.

    Returns {k: (solutions [<=kappa][k] int32, Omega [<=kappa])}, best first at every order.
    on_device (default: with precision "fp64", N <= 128, k_last <= 64 and kappa * N <= 4096): the
    orders after the first run on the device in one call (thoi_greedy: two launches per order, no
    host round trip); otherwise every order is one batched reducer call decided on the host.
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
        rows = combinations(N, k_first)
        sols, vals = _best_rows(S, rows, kappa, maximize, precision)
        out = {k_first: (sols, vals)}
    if on_device is None:
        on_device = precision == "fp64" and N <= 128 and k_last <= 64 and kappa * N <= 4096
    if on_device and k_last > k_first and len(sols) > 0:
        return _greedy_device(S, sols, out[k_first][1], k_first, k_last, kappa, maximize)
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


# ------------------------------------------------------------------------------------------------ annealing
def _propose(cur: np.ndarray, move: np.ndarray, a: np.ndarray, b: np.ndarray, mode: str, k_min: int,
             k_max: int) -> np.ndarray:
    """One neighbour per chain.  Within an order: swap a member for an outsider.  Across orders:
    add (move < 1/3), remove (move in [1/3, 2/3)) or swap, a swap also replacing a move that would
    leave [k_min, k_max].  The member / outsider is the floor(u * count)-th in ascending order."""
    kappa, N = cur.shape
    k = cur.sum(1)
    if mode == "across":
        add = (move < 1.0 / 3.0) & (k < k_max)
        rem = (move >= 1.0 / 3.0) & (move < 2.0 / 3.0) & (k > k_min)
    else:
        add = rem = np.zeros(kappa, dtype=bool)
    swap = ~(add | rem)
    rows = np.arange(kappa)
    # the (p+1)-th member / outsider of each row, by running counts
    pa = (a * k).astype(np.int64)
    drop = np.argmax(cur & (np.cumsum(cur, 1) == (pa + 1)[:, None]), axis=1)
    out = ~cur
    pb = (b * (N - k)).astype(np.int64)
    take = np.argmax(out & (np.cumsum(out, 1) == (pb + 1)[:, None]), axis=1)
    prop = cur.copy()
    d = swap | rem
    prop[rows[d], drop[d]] = False
    t = swap | add
    prop[rows[t], take[t]] = True
    return prop


def _omega_masks(S: torch.Tensor, masks: np.ndarray, precision: str) -> np.ndarray:
    N = masks.shape[1]
    odt = torch.float64 if precision == "fp64" else torch.float32
    if N <= 64:
        bits = (masks.astype(np.uint64) << np.arange(N, dtype=np.uint64)[None, :]).sum(1, dtype=np.uint64)
        mt = torch.from_numpy(bits.view(np.int64)).to(S.device)
        out, _ = api.nplets_measures(S, masks=mt, precision=precision, out_dtype=odt)
    else:
        k = int(masks.sum(1).max())
        rows = -np.ones((len(masks), k), dtype=np.int32)
        for j, m in enumerate(masks):
            nz = np.nonzero(m)[0]
            rows[j, : len(nz)] = nz
        out, _ = api.nplets_measures(S, nplets=_rows_to_device(rows, S.device), precision=precision, out_dtype=odt)
    return out[2].double().cpu().numpy().reshape(-1)


def anneal(Sigma: torch.Tensor, masks0: np.ndarray, draws: dict, T0: float = 1.0, alpha: float = 0.99,
           maximize: bool = True, mode: str = "within", k_min: int = 3, k_max: int | None = None,
           precision: str = "fp64", on_device: bool | None = None):
    """Batched simulated annealing (Methods, "Heuristics", "Simulated Annealing Algorithm").

    kappa chains start from masks0 [kappa][N] (orders may differ: one call evaluates the mixed
    orders together, MASK selection for N <= 64, else LIST).  Per iteration every chain proposes a
    neighbour; with energy E = Omega (maximise) or -Omega (minimise) and dE = E_new - E_cur, the
    proposal is taken if dE > 0, else with probability exp(dE / Temp) (the printed rule has the
    sign garbled; this is the standard Metropolis reading), decided by draws['accept'].  Temp
    starts at T0 and is multiplied by alpha each iteration.  Proposals that are not positive
    definite are rejected.  Returns (best masks, best Omega, final masks, final Omega, accepted
    count per chain).

    on_device (default: with precision "fp64", N <= 128 and orders <= 64): the whole run goes to
    the device in one call (thoi_anneal: one kernel launch per iteration, no host round trip);
    otherwise every iteration evaluates its proposals with one batched evaluator call and decides
    on the host.
    """
    if mode not in ("within", "across"):
        raise ValueError("mode is 'within' or 'across'")
    S = Sigma[0] if Sigma.dim() == 3 else Sigma
    cur = np.array(masks0, dtype=bool, copy=True)
    kappa, N = cur.shape
    k_max = N - 1 if k_max is None else k_max          # a swap always has an outsider to take in
    ks = cur.sum(1)
    if k_max > N - 1 or k_min < 1 or ks.min() < k_min or ks.max() > k_max:
        raise ValueError("need 1 <= k_min <= every initial order <= k_max <= N - 1")
    sign = 1.0 if maximize else -1.0
    if on_device is None:
        on_device = (precision == "fp64" and N <= 128 and ks.max() <= 64 and (mode == "within" or k_max <= 64)
                     and T0 > 0 and alpha > 0)
    if on_device:
        # within an order no chain changes its order: the bounds are the initial orders (the
        # device picks its factorisation by the largest order a chain can reach)
        kx = int(ks.max()) if mode == "within" else k_max
        kn = int(ks.min()) if mode == "within" else k_min
        return _anneal_device(S, cur, draws, T0, alpha, maximize, mode, kn, kx)
    om = _omega_masks(S, cur, precision)
    E = sign * om
    best, Ebest = cur.copy(), E.copy()
    accepted = np.zeros(kappa, dtype=np.int64)
    temp = T0
    iters = draws["accept"].shape[0]
    for t in range(iters):
        prop = _propose(cur, draws["move"][t], draws["a"][t], draws["b"][t], mode, k_min, k_max)
        Ep = sign * _omega_masks(S, prop, precision)
        dE = Ep - E
        with np.errstate(over="ignore", invalid="ignore"):
            take = (dE > 0) | (draws["accept"][t] < np.exp(dE / temp))
        take &= ~np.isnan(Ep)
        cur[take], E[take] = prop[take], Ep[take]
        accepted += take
        better = E > Ebest
        best[better], Ebest[better] = cur[better], E[better]
        temp *= alpha
    return best, sign * Ebest, cur, sign * E, accepted


def _anneal_device(S: torch.Tensor, cur: np.ndarray, draws: dict, T0: float, alpha: float, maximize: bool,
                   mode: str, k_min: int, k_max: int):
    kappa, N = cur.shape
    dev = S.device
    Sd = S.to(torch.float64).contiguous()
    words = np.zeros((kappa, 2), dtype=np.uint64)
    for h in range(2):
        part = cur[:, 64 * h: 64 * (h + 1)]
        words[:, h] = (part.astype(np.uint64) << np.arange(part.shape[1], dtype=np.uint64)[None, :]).sum(
            1, dtype=np.uint64)
    m0 = torch.from_numpy(words.view(np.int64).copy()).to(dev)
    iters = int(draws["accept"].shape[0])

    def rows(name):
        x = np.ascontiguousarray(np.asarray(draws[name], dtype=np.float64)[:iters].reshape(iters, kappa))
        return torch.from_numpy(x).to(dev)
    across = mode == "across"
    dm = rows("move") if across else None
    da, db, du = rows("a"), rows("b"), rows("accept")
    cm = torch.empty((kappa, 2), dtype=torch.int64, device=dev)
    bm = torch.empty_like(cm)
    co = torch.empty(kappa, dtype=torch.float64, device=dev)
    bo = torch.empty_like(co)
    acc = torch.empty(kappa, dtype=torch.int64, device=dev)
    B.thoi_anneal(api._ptr(Sd), N, api._ptr(m0), kappa, iters, api._ptr(dm), api._ptr(da), api._ptr(db),
                  api._ptr(du), float(T0), float(alpha), 1 if maximize else 0, 1 if across else 0, k_min, k_max,
                  api._ptr(cm), api._ptr(co), api._ptr(bm), api._ptr(bo), api._ptr(acc), api._stream(dev))

    def unpack(t):
        v = t.cpu().numpy().view(np.uint64)
        i = np.arange(N)
        return ((v[:, i // 64] >> (i % 64).astype(np.uint64)[None, :]) & np.uint64(1)).astype(bool)
    return unpack(bm), bo.cpu().numpy(), unpack(cm), co.cpu().numpy(), acc.cpu().numpy()


# ------------------------------------------------------------------------------------------------ across datasets
MEASURES = {"tc": 0, "dtc": 1, "omega": 2, "s": 3}


def _best_rows_multi(Sigmas: torch.Tensor, rows: np.ndarray, kappa: int, measure: str, kind: str, maximize: bool,
                     precision: str):
    odt = torch.float64 if precision == "fp64" else torch.float32
    out, _ = api.nplets_measures(Sigmas, nplets=_rows_to_device(rows, Sigmas.device), precision=precision,
                                 out_dtype=odt)
    _, st = api.objective(out[MEASURES[measure]], kind, write=False, topk=kappa)
    tv, tg, _ = st.result()
    slot = 0 if maximize else 1
    g = tg[0, 0, slot]
    keep = g >= 0
    return rows[g[keep]], tv[0, 0, slot][keep]


def greedy_multi(Sigmas: torch.Tensor, k_first: int, k_last: int, kappa: int = 16, measure: str = "omega",
                 kind: str = "mean", maximize: bool = True, precision: str = "fp64", on_device: bool | None = None):
    """Greedy growth (as `greedy`) on an objective over D datasets: every candidate is evaluated in
    all D covariance matrices in one call (the paper's B x D pairing), `kind` ("mean" or
    "paired_effect") turns its D values of `measure` into one number on the device, and the kappa
    best are kept.  Sigmas: [D, N, N] float64.  Returns {k: (solutions, objective)}.  on_device
    (default: with precision "fp64", N <= 128, k_last <= 64 and kappa * N <= 4096): the orders
    after the first run on the device in one call (thoi_greedy); otherwise each order is one
    evaluator call plus one objective reduction, decided on the host."""
    D, N, _ = Sigmas.shape
    rows = combinations(N, k_first)
    sols, vals = _best_rows_multi(Sigmas, rows, kappa, measure, kind, maximize, precision)
    out = {k_first: (sols, vals)}
    if on_device is None:
        on_device = precision == "fp64" and N <= 128 and k_last <= 64 and kappa * N <= 4096
    if on_device and k_last > k_first and len(sols) > 0:
        kd = B.THOI_OBJ_MEAN if kind == "mean" else B.THOI_OBJ_PAIRED_EFFECT
        return _greedy_device(Sigmas, sols, vals, k_first, k_last, kappa, maximize, MEASURES[measure], kd)
    for k in range(k_first + 1, k_last + 1):
        sols, vals = _best_rows_multi(Sigmas, expand(sols, N), kappa, measure, kind, maximize, precision)
        out[k] = (sols, vals)
    return out
