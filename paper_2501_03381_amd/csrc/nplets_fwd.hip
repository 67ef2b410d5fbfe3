// Forward evaluation of (TC, DTC, Omega, S) over batches of n-plets on gfx950.
//
// Work decomposition (replacing the expand-and-index batching of Methods, "Batched
// sub-covariance matrices", and the identity padding of "padded batches"):
//  - every workgroup handles one dataset d (grid.y) and a segment of tiles of n-plets of ONE
//    order k, so the order is uniform in the workgroup and the per-order code is fully unrolled;
//  - the dataset's correlation matrix is staged once per workgroup in LDS; an n-plet's
//    sub-matrix is gathered from there into registers and never exists in HBM;
//  - RANGE mode unranks each n-plet from its global index in the lane (no index tensors);
//  - orders are grouped into a few kernel classes by register footprint; each class is one
//    launch covering all of its orders (per-order segments are mapped from blockIdx);
//  - orders above the register classes use one wavefront per n-plet with the matrix in LDS.
// FP32_REFINE: the FP32 lane engine flags n-plets whose max VIF exceeds tau (or that failed);
// a follow-up FP64 kernel re-evaluates exactly those and overwrites their results.
// Results go either to the output planes or to the streaming reducer (reduce_common.hpp).
#include "nplets_fwd_common.hpp"
#include "nplets_prefix.hpp"
#include "nplets_wave2.hpp"

namespace thoi {

namespace {

template <typename F, int KLO, int KHI, int MODE, bool RED, int S = lane_per_thread<F>(KHI, MODE)>
__global__ __launch_bounds__(kTile) void k_eval_lane(EvalArgs a, PieceTable tab, RedArgs red)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double sbias[3];
    const int N = a.N;
    const int d = blockIdx.y;
    const int64_t blk = blockIdx.x;
    const int64_t per_blk = (int64_t)kTile * S * a.seg_tiles;
    // which order / piece does this workgroup belong to (uniform in the workgroup)
    int k = -1;
    int64_t first = 0, pos0 = 0, cnt = 0, blk0 = 0;
    if constexpr (MODE == THOI_SEL_RANGE) {
        for (int p = 0; p < tab.n; ++p) {
            const int64_t nb = (tab.p[p].cnt + per_blk - 1) / per_blk;
            if (blk >= tab.p[p].blk0 && blk < tab.p[p].blk0 + nb) {
                k = tab.p[p].k; first = tab.p[p].first; pos0 = tab.p[p].pos0; cnt = tab.p[p].cnt; blk0 = tab.p[p].blk0;
            }
        }
    } else {
        for (int kk = KLO; kk <= KHI; ++kk) {
            const int64_t c = a.lcnt[kk];
            const int64_t nb = (c + per_blk - 1) / per_blk;
            const int64_t b0 = a.lblk0[kk];
            if (c > 0 && blk >= b0 && blk < b0 + nb) { k = kk; first = a.lbase[kk]; cnt = c; blk0 = b0; }
        }
    }
    if (k < 0) return;

    const int kb = (MODE == THOI_SEL_RANGE) ? KHI : 0;
    F* sR = reinterpret_cast<F*>(smem);
    const size_t off = ((size_t)N * N * sizeof(F) + 15) / 16 * 16;
    double* sIsd = reinterpret_cast<double*>(smem + off);
    double* sLogd = sIsd + N;
    uint64_t* sBin = reinterpret_cast<uint64_t*>(sLogd + N);
    RedLds Rl = red_view(smem + lane_stage_bytes(N, kb, sizeof(F)), red.topk, red.bins);
    if (threadIdx.x == 0) bias_for(a.bias, k, sbias[0], sbias[1], sbias[2]);
    stage_corr<F>(a.Sigma + (int64_t)d * N * N, N, sR, sIsd, sLogd, MODE == THOI_SEL_RANGE ? sBin : nullptr, kb);
    constexpr bool reduce = RED;
    if constexpr (RED) red_begin(Rl, red, d, k);

    LaneCtx cx;
    cx.d = d;
    cx.first = first;
    cx.pos0 = pos0;
    cx.N = N;
    cx.kb = kb;
    cx.reduce = reduce;
    cx.dtc = sbias[0];
    cx.ddtc = sbias[1];
    cx.eta = sbias[2];
    const int64_t base = (blk - blk0) * per_blk;
    for (int t = 0; t < a.seg_tiles; ++t) {
        const int64_t tb = base + (int64_t)t * kTile * S;
        if (tb >= cnt) break;                         // uniform: same for the whole workgroup
        cx.local = tb + (int64_t)S * threadIdx.x;
        double omega[S] = {};
        int64_t gidx[S] = {};
        bool valid[S] = {};
        if (cx.local < cnt) dispatch_k<F, KLO, KHI, MODE, S>(k, a, cx, sR, sLogd, sBin, cnt, omega, gidx, valid);
        if constexpr (RED) {
#pragma unroll
            for (int j = 0; j < S; ++j) red_push(Rl, red, k, valid[j], omega[j], gidx[j]);
        }
    }
    if constexpr (RED) red_end(Rl, red, a.hdr, d, k);
}

template <int MODE, bool RED>
__global__ __launch_bounds__(64) void k_eval_wave(EvalArgs a, PieceTable tab, RedArgs red, int klo, int kmax)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double sbias[3];
    const int N = a.N;
    const int d = blockIdx.y;
    const int64_t blk = blockIdx.x;
    const int wt = a.wave_tile_hi;
    int k = -1;
    int64_t first = 0, pos0 = 0, cnt = 0, blk0 = 0;
    if constexpr (MODE == THOI_SEL_RANGE) {
        for (int p = 0; p < tab.n; ++p) {
            if (tab.p[p].k < klo || tab.p[p].k > kmax) continue;   // another launch's orders
            const int64_t nb = (tab.p[p].cnt + wt - 1) / wt;
            if (blk >= tab.p[p].blk0 && blk < tab.p[p].blk0 + nb) {
                k = tab.p[p].k; first = tab.p[p].first; pos0 = tab.p[p].pos0; cnt = tab.p[p].cnt; blk0 = tab.p[p].blk0;
            }
        }
    } else {
        for (int kk = klo; kk <= kmax; ++kk) {
            const int64_t c = a.lcnt[kk];
            const int64_t nb = (c + wt - 1) / wt;
            const int64_t b0 = a.lblk0[kk];
            if (c > 0 && blk >= b0 && blk < b0 + nb) { k = kk; first = a.lbase[kk]; cnt = c; blk0 = b0; }
        }
    }
    if (k < 0) return;
    const int ks = kmax + 1;
    double* sR = reinterpret_cast<double*>(smem);
    double* sIsd = sR + N * N;
    double* sLogd = sIsd + N;
    uint64_t* sBin = reinterpret_cast<uint64_t*>(sLogd + N);
    double* sM = reinterpret_cast<double*>(sBin + (MODE == THOI_SEL_RANGE ? N * 64 : 0));
    double* sInv = sM + 64 * ks;
    int* cidx = reinterpret_cast<int*>(sInv + 64);
    double* res_v = reinterpret_cast<double*>(cidx + 64);
    int64_t* res_g = reinterpret_cast<int64_t*>(res_v + 64);
    int* res_ok = reinterpret_cast<int*>(res_g + 64);
    RedLds S = red_view(smem + wave_stage_bytes(N, kmax, MODE == THOI_SEL_RANGE), red.topk, red.bins);
    if (threadIdx.x == 0) bias_for(a.bias, k, sbias[0], sbias[1], sbias[2]);
    if constexpr (MODE == THOI_SEL_RANGE) stage_binomials(N, 64, sBin);
    stage_corr<double>(a.Sigma + (int64_t)d * N * N, N, sR, sIsd, sLogd);
    constexpr bool reduce = RED;
    if constexpr (RED) red_begin(S, red, d, k);

    const int lane = threadIdx.x;
    const int64_t l0 = (blk - blk0) * wt;
    const int64_t l1 = l0 + wt < cnt ? l0 + wt : cnt;
    for (int64_t c0 = l0; c0 < l1; c0 += 64) {
        const int64_t c1 = c0 + 64 < l1 ? c0 + 64 : l1;
        for (int64_t l = c0; l < c1; ++l) {
            int64_t pos, gidx;
            if constexpr (MODE == THOI_SEL_RANGE) {
                if (lane == 0) unrank_lex_rt((uint64_t)(first + l), N, k, sBin, 64, cidx);
                pos = pos0 + l;
                gidx = a.g_begin + pos;
            } else if constexpr (MODE == THOI_SEL_LIST) {
                pos = a.perm[first + l];
                gidx = pos;
                if (lane < k) cidx[lane] = a.idx[pos * a.kmax_list + lane];
            } else {
                pos = a.perm[first + l];
                gidx = pos;
                if (lane == 0) {
                    uint64_t m = a.mask[pos];
                    for (int i = 0; i < k; ++i) { cidx[i] = __builtin_ctzll(m); m &= m - 1; }
                }
            }
            __syncthreads();
            const FactorOut<double> f = wave_factor(sR, N, cidx, k, sM, ks, sInv);
            double sumlogd = 0.0;
            if (a.write_H) sumlogd = wave_sum(lane < k ? sLogd[cidx[lane]] : 0.0);
            if (lane == 0) {
                // the wave engine is already FP64: never queue a refinement
                EvalArgs b = a;
                if (b.precision == THOI_FP32_REFINE) b.precision = THOI_FP64;
                double om = 0.0;
                const bool ok = store_result<double>(b, reduce, d, pos, k, f, sumlogd, sbias[0], sbias[1], sbias[2],
                                                     true, om);
                res_v[l - c0] = om;
                res_g[l - c0] = gidx;
                res_ok[l - c0] = ok;
            }
            __syncthreads();
        }
        if constexpr (RED) {
            const int i = lane;
            const bool have = c0 + i < c1;
            red_push(S, red, k, have && res_ok[i], have ? res_v[i] : 0.0, have ? res_g[i] : 0);
        }
    }
    if constexpr (RED) red_end(S, red, a.hdr, d, k);
}

// ------------------------------------------------------------------------------------------------
// Host side
// ------------------------------------------------------------------------------------------------
// Launch plan of a call: workgroups per class and per wave launch; exact for RANGE, an upper
// bound for LIST / MASK.
struct Plan {
    int ncls;
    PieceTable tabs[8];
    int64_t nblk[8];
    PieceTable wtab;     // RANGE pieces above the lane classes (pair and wave engines)
    int64_t wblk;        // pair-engine workgroups (orders up to kW2Max)
    int64_t wblk_hi;     // wave-engine workgroups (orders above kW2Max)
    int wkmax;
    int seg_tiles, wave_tile, wave_tile_hi;
    int cls_seg[8];      // per class: tiles per workgroup (RANGE: tunable per class; else seg_tiles)
    int cls_S[8];        // per class: n-plets per lane
    int64_t seg_cap;
    bool serial;     // every launch on the caller's stream (no side streams)
    int npcls;       // prefix engine: classes, their order tables and workgroups
    PfxTable ptabs[4];
    int64_t pnblk[4];
};

// Grids are kept well below the dispatch limit of 2^32 work-items along x: a class grid by
// growing the tiles per workgroup, the wave grid by growing the n-plets per workgroup (both
// engines loop over their share, so any tile count is valid).
constexpr int64_t kMaxGridItems = int64_t(1) << 30;

// Prefix engine for order k of this precision: the class index, or -1.
int pfx_class_of(bool f64, int k)
{
    const PfxClass* cls = f64 ? kPfxF64Classes : kPfxF32Classes;
    const int n = f64 ? (int)(sizeof(kPfxF64Classes) / sizeof(PfxClass)) : (int)(sizeof(kPfxF32Classes) / sizeof(PfxClass));
    for (int c = 0; c < n; ++c)
        if (k >= cls[c].lo && k <= cls[c].hi) return c;
    return -1;
}

// Whether a whole order k of a RANGE call goes to the prefix engine.  The library's choice
// (THOI_ENGINE_AUTO) follows measurements of both engines on the N = 30 reduction (streaming
// top-100 and 256 bins): orders 7..8 FP64 1.31 ms against 1.55 ms, FP32 + refinement 1.28 against
// 1.49; orders 9..12 FP64 9.4 against 14.4 ms, FP32 + refinement 5.6 against 6.9; orders 13..16
// FP32 + refinement 33.5 against 28.6 ms (the factorisation engine wins).  In FP32 the gain on
// orders 7..12 alone does not carry over to a whole enumeration, where the factorisation classes
// of those orders overlap the longer ones (all orders 3..30: 67.7 ms with the prefix engine for
// 7..12, 67.2 ms without), so FP32 keeps the factorisation engine.  Orders up to 6 have too few
// prefixes per workgroup (3..6: 1.4 against 0.8 ms), at N = 20 every order has too few tails per
// prefix, and in output mode each lane's outputs are consecutive but the lanes' are far apart, so
// the stores do not coalesce.
bool use_prefix(int engine, bool reduce, bool f64, int N, int k, int64_t D)
{
    if (engine == THOI_ENGINE_PREFIX) return true;
    if (engine != THOI_ENGINE_AUTO) return false;
    return f64 && reduce && k >= 7 && k <= 12 && pfx_tails(N, k, D) >= 4;
}

template <typename F>
Plan make_plan(int N, int64_t D, const thoi_nplets* sel, bool reduce, const thoi_eval_opts* o)
{
    const int precision = o->precision, seg_tiles_hint = o->seg_tiles, engine = o->engine;
    Plan P{};
    const bool f64 = sizeof(F) == 8;
    P.npcls = f64 ? (int)(sizeof(kPfxF64Classes) / sizeof(PfxClass)) : (int)(sizeof(kPfxF32Classes) / sizeof(PfxClass));
    // an order goes to the prefix engine when the call covers it completely
    auto prefix_order = [&](int k, int64_t lo, int64_t hi, int64_t g, int64_t ck) {
        return sel->mode == THOI_SEL_RANGE && use_prefix(engine, reduce, f64, N, k, D) && pfx_class_of(f64, k) >= 0 &&
               lo == g && hi == g + ck;
    };
    const KClass* cls = classes_for<F>(P.ncls);
    const int lane_max = lane_max_for(precision);
    const int64_t Bn = sel_B(sel);
    // reduce mode: a workgroup walks a segment of tiles so that one launch has a few thousand
    // workgroups and the number of segments to merge stays bounded
    // FP64 ranges: two tiles per workgroup amortise the staging of the correlation matrix
    // (measured faster for FP64; for FP32 the concurrent class launches fill the GPU better with
    // one tile per workgroup)
    P.seg_tiles = (sizeof(F) == 8 && sel->mode == THOI_SEL_RANGE) ? 2 : 1;
    if (reduce) {
        const int64_t tiles = (Bn + kTile - 1) / kTile;
        P.seg_tiles = (int)((tiles + 16383) / 16384);
        if (P.seg_tiles < 1) P.seg_tiles = 1;
    }
    if (seg_tiles_hint > 0) P.seg_tiles = seg_tiles_hint;
    // largest share of one class (or of the pair / wave engine): n-plets per launch bound the grids
    int64_t cls_cnt[8] = {0}, pair_cnt = 0, wave_cnt = 0;
    if (sel->mode == THOI_SEL_RANGE) {
        int64_t g = 0;
        const int64_t gb = sel->g_begin, ge = sel->g_begin + sel->g_count;
        for (int k = sel->kmin; k <= sel->kmax; ++k) {
            const int64_t ck = (int64_t)binom_u64(N, k);
            const int64_t lo = gb > g ? gb : g, hi = ge < g + ck ? ge : g + ck;
            if (hi > lo && !prefix_order(k, lo, hi, g, ck)) {
                if (k <= lane_max) cls_cnt[class_of<F>(k)] += hi - lo;
                else if (k <= kW2Max) pair_cnt += hi - lo;
                else wave_cnt += hi - lo;
            }
            g += ck;
        }
    } else {
        for (int c = 0; c < P.ncls; ++c) cls_cnt[c] = Bn;
        if (sel_kmax(sel, N) > lane_max) pair_cnt = Bn;
        if (sel_kmax(sel, N) > kW2Max) wave_cnt = Bn;
    }
    const bool range = sel->mode == THOI_SEL_RANGE;
    for (int c = 0; c < P.ncls; ++c) {
        P.cls_S[c] = range ? lane_per_thread<F>(cls[c].hi, THOI_SEL_RANGE) : 1;
        if (range && o->class_lanes[c] == 1) P.cls_S[c] = 1;
        // threads of class c: about cls_cnt / S plus one tile per piece; the grid stays below
        // kMaxGridItems by walking more tiles per workgroup
        const int64_t threads = cls_cnt[c] / P.cls_S[c] + (int64_t)kTile * (kMaxPieces + 1);
        const int64_t need = (threads + kMaxGridItems - 1) / kMaxGridItems;
        if (range) {
            P.cls_seg[c] = o->class_seg_tiles[c] > 0 ? o->class_seg_tiles[c] : P.seg_tiles;
            if (need > P.cls_seg[c]) P.cls_seg[c] = (int)need;
        } else if (need > P.seg_tiles) {
            P.seg_tiles = (int)need;
        }
    }
    if (!range)
        for (int c = 0; c < P.ncls; ++c) P.cls_seg[c] = P.seg_tiles;
    // pair engine: about 16384 workgroups in output mode and 8192 in reduce mode over all D
    // datasets (each reducing workgroup leaves one segment of top-K lists to merge), at least one
    // chunk of kPairThreads n-plets per reducing workgroup; a multiple of kPairHalves n-plets per
    // workgroup
    {
        int64_t groups = (reduce ? 8192 : 16384) / (D > 0 ? D : 1);
        groups = groups < 64 ? 64 : groups;
        const int64_t unit = reduce ? kPairThreads : kPairHalves;
        int64_t t = (pair_cnt + groups - 1) / groups;
        t = (t + unit - 1) / unit * unit;
        t = t < unit ? unit : t;
        const int64_t lim = kMaxGridItems / kPairThreads - kMaxPieces - 1;
        if ((pair_cnt + t - 1) / t > lim) t = (pair_cnt + lim - 1) / lim;
        P.wave_tile = (int)t;
    }
    // wave engine: one n-plet per workgroup in output mode (few, long factorisations), 64 in
    // reduce mode; more when the grid would exceed its bound
    P.wave_tile_hi = reduce ? kWaveTileRed : kWaveTileOut;
    {
        const int64_t groups = (wave_cnt + P.wave_tile_hi - 1) / P.wave_tile_hi + kMaxPieces + 1;
        if (groups * 64 > kMaxGridItems) {
            const int64_t t = (wave_cnt + kMaxGridItems / 64 - kMaxPieces - 2) / (kMaxGridItems / 64 - kMaxPieces - 1);
            P.wave_tile_hi = (int)(t > P.wave_tile_hi ? t : P.wave_tile_hi);
        }
    }
    const int64_t per_blk = (int64_t)kTile * P.seg_tiles;     // one n-plet per lane (index lists)
    if (sel->mode == THOI_SEL_RANGE) {
        int64_t g = 0;
        const int64_t gb = sel->g_begin, ge = sel->g_begin + sel->g_count;
        for (int k = sel->kmin; k <= sel->kmax; ++k) {
            const int64_t ck = (int64_t)binom_u64(N, k);
            const int64_t lo = gb > g ? gb : g, hi = ge < g + ck ? ge : g + ck;
            if (hi > lo && prefix_order(k, lo, hi, g, ck)) {
                const int c = pfx_class_of(f64, k);
                PfxPiece pp{};
                pp.k = k;
                pp.pos0 = lo - gb;
                pp.L = pfx_tails(N, k, D);
                pp.nblk = pfx_blocks(N, k, pp.L);
                pp.nphys = pp.nblk < kPfxMaxGroups ? pp.nblk : kPfxMaxGroups;
                pp.blk0 = P.pnblk[c];
                P.pnblk[c] += pp.nphys;
                P.ptabs[c].p[P.ptabs[c].n++] = pp;
            } else if (hi > lo) {
                Piece p{};
                p.k = k;
                p.first = lo - g;
                p.pos0 = lo - gb;
                p.cnt = hi - lo;
                if (k <= lane_max) {
                    const int c = class_of<F>(k);
                    const int64_t pb = (int64_t)kTile * P.cls_seg[c] * P.cls_S[c];
                    p.blk0 = P.nblk[c];
                    P.nblk[c] += (p.cnt + pb - 1) / pb;
                    P.tabs[c].p[P.tabs[c].n++] = p;
                } else if (k <= kW2Max) {
                    p.blk0 = P.wblk;
                    P.wblk += (p.cnt + P.wave_tile - 1) / P.wave_tile;
                    P.wtab.p[P.wtab.n++] = p;
                    P.wkmax = k > P.wkmax ? k : P.wkmax;
                } else {
                    p.blk0 = P.wblk_hi;
                    P.wblk_hi += (p.cnt + P.wave_tile_hi - 1) / P.wave_tile_hi;
                    P.wtab.p[P.wtab.n++] = p;
                    P.wkmax = k > P.wkmax ? k : P.wkmax;
                }
            }
            g += ck;
        }
    } else {
        for (int c = 0; c < P.ncls; ++c) P.nblk[c] = (Bn + per_blk - 1) / per_blk + (cls[c].hi - cls[c].lo + 1);
        const int kcap = sel_kmax(sel, N);
        if (kcap > lane_max) {
            P.wblk = (Bn + P.wave_tile - 1) / P.wave_tile + ((kcap < kW2Max ? kcap : kW2Max) - lane_max);
            P.wkmax = kcap;
        }
        if (kcap > kW2Max) P.wblk_hi = (Bn + P.wave_tile_hi - 1) / P.wave_tile_hi + (kcap - kW2Max);
    }
    P.seg_cap = P.wblk + P.wblk_hi;
    for (int c = 0; c < P.ncls; ++c) P.seg_cap += P.nblk[c];
    for (int c = 0; c < P.npcls; ++c) P.seg_cap += P.pnblk[c];
    return P;
}

struct EvalWs {
    size_t refine_off, korder_off, cnt_off, base_off, blk0_off, cursor_off, perm_off;
    size_t seg_key_off, seg_g_off, seg_hdr_off, late_off, bound_off, clear_end, total;
    uint32_t refine_cap, seg_cap, late_cap;
};

EvalWs eval_layout(int64_t D, int32_t N, const thoi_nplets* sel, const thoi_eval_opts* opts)
{
    EvalWs w{};
    const int64_t B = sel_B(sel);
    const bool reduce = opts->reduce != nullptr;
    size_t off = kWsHeader;
    if (reduce && opts->reduce->topk > 0) {
        // admission bounds [D][kmax+1][2], cleared with the header
        w.bound_off = off;
        off = align_up(off + (size_t)D * (sel_kmax(sel, N) + 1) * 2 * 8, 256);
    }
    w.clear_end = off;
    if (opts->precision == THOI_FP32_REFINE) {
        const int64_t want = D * B;
        const int64_t cap = want < (int64_t(1) << 24) ? want : (int64_t(1) << 24);
        w.refine_cap = (uint32_t)(cap > 0 ? cap : 1);
        w.refine_off = off;
        off = align_up(off + (size_t)w.refine_cap * 8, 256);
    }
    if (sel->mode != THOI_SEL_RANGE) {
        w.korder_off = off; off = align_up(off + (size_t)B, 256);
        w.cnt_off = off; off = align_up(off + kListOrders * 8, 256);
        w.base_off = off; off = align_up(off + kListOrders * 8, 256);
        w.blk0_off = off; off = align_up(off + kListOrders * 8, 256);
        w.cursor_off = off; off = align_up(off + kListOrders * 8, 256);
        w.perm_off = off; off = align_up(off + (size_t)B * 8, 256);
    }
    if (reduce && opts->reduce->topk > 0) {
        const int K = opts->reduce->topk;
        const Plan P = opts->precision == THOI_FP64 ? make_plan<double>(N, D, sel, true, opts)
                                                    : make_plan<float>(N, D, sel, true, opts);
        const int64_t segs = P.seg_cap * D;
        w.seg_cap = (uint32_t)(segs > 0 ? segs : 1);
        w.seg_key_off = off; off = align_up(off + (size_t)w.seg_cap * 2 * K * 8, 256);
        w.seg_g_off = off; off = align_up(off + (size_t)w.seg_cap * 2 * K * 8, 256);
        w.seg_hdr_off = off; off = align_up(off + (size_t)w.seg_cap * sizeof(SegHdr), 256);
        w.late_cap = w.refine_cap;
        if (w.late_cap) { w.late_off = off; off = align_up(off + (size_t)w.late_cap * sizeof(LateEntry), 256); }
    }
    w.total = off;
    return w;
}

typedef void (*LaneKernel)(EvalArgs, PieceTable, RedArgs);

// Class kernel with S n-plets per lane: S = 1 is instantiated as a tuning alternative where the
// default is 2 (RANGE mode, classes with register room).
template <typename F, int KLO, int KHI, int MODE, bool RED>
LaneKernel lane_kernel_s(int S)
{
    constexpr int Sd = lane_per_thread<F>(KHI, MODE);
    if constexpr (Sd > 1) {
        if (S == 1) return k_eval_lane<F, KLO, KHI, MODE, RED, 1>;
    }
    return k_eval_lane<F, KLO, KHI, MODE, RED, Sd>;
}

template <typename F, int MODE, bool RED>
LaneKernel lane_kernel_r(int cls, int S)
{
    if constexpr (sizeof(F) == 4) {
        switch (cls) {
            case 0: return lane_kernel_s<F, 0, 8, MODE, RED>(S);
            case 1: return lane_kernel_s<F, 9, 12, MODE, RED>(S);
            case 2: return lane_kernel_s<F, 13, 16, MODE, RED>(S);
            case 3: return lane_kernel_s<F, 17, 20, MODE, RED>(S);
            default: return lane_kernel_s<F, 21, 24, MODE, RED>(S);
        }
    } else {
        switch (cls) {
            case 0: return lane_kernel_s<F, 0, 6, MODE, RED>(S);
            case 1: return lane_kernel_s<F, 7, 10, MODE, RED>(S);
            case 2: return lane_kernel_s<F, 11, 14, MODE, RED>(S);
            default: return lane_kernel_s<F, 15, 18, MODE, RED>(S);
        }
    }
}

template <typename F, int MODE>
LaneKernel lane_kernel(int cls, bool reduce, int S)
{
    return reduce ? lane_kernel_r<F, MODE, true>(cls, S) : lane_kernel_r<F, MODE, false>(cls, S);
}

typedef void (*WaveKernel)(EvalArgs, PieceTable, RedArgs, int, int);

template <int MODE>
WaveKernel wave_kernel(bool reduce)
{
    return reduce ? k_eval_wave<MODE, true> : k_eval_wave<MODE, false>;
}


template <typename F, int MODE>
void launch_engines(EvalArgs& a, const Plan& P, const RedArgs& red, hipStream_t s)
{
    int ncls = 0;
    const KClass* cls = classes_for<F>(ncls);
    const bool reduce = red.active != 0;
    const int N = a.N;
    // the class launches are independent: fan them out over side streams
    int nl = (P.wblk ? 1 : 0) + (P.wblk_hi ? 1 : 0);
    for (int c = 0; c < ncls; ++c) nl += P.nblk[c] != 0;
    for (int c = 0; c < P.npcls; ++c) nl += P.pnblk[c] != 0;
    FanScope fan(s, P.serial ? 1 : nl);
    int b = 0;
    if constexpr (MODE == THOI_SEL_RANGE) {
        for (int c = P.npcls - 1; c >= 0; --c) {      // the longest lanes first
            if (P.pnblk[c] == 0) continue;
            pfx_launch(sizeof(F) == 8, c, reduce, a, P.ptabs[c], red, P.pnblk[c], a.D, fan.stream(b++));
        }
    }
    const int* order = sizeof(F) == 4 ? kF32LaunchOrder : kF64LaunchOrder;
    for (int oc = 0; oc < ncls; ++oc) {
        const int c = order[oc];
        if (P.nblk[c] == 0) continue;
        const int kb = MODE == THOI_SEL_RANGE ? cls[c].hi : 0;
        const size_t lds = lane_stage_bytes(N, kb, sizeof(F)) + red_lds(red);
        const LaneKernel kern = lane_kernel<F, MODE>(c, reduce, P.cls_S[c]);
        EvalArgs ac = a;
        ac.seg_tiles = P.cls_seg[c];
        hipLaunchKernelGGL(kern, dim3((unsigned)P.nblk[c], (unsigned)a.D), dim3(kTile), lds, fan.stream(b++), ac,
                           P.tabs[c], red);
    }
    // orders above the lane engine: up to kW2Max two n-plets per wavefront (rows in registers),
    // above that one per wavefront; each launch takes only its orders of the shared piece table
    if (P.wblk)
        pair_launch(MODE, reduce, a, P.wtab, red, lane_max_for(a.precision) + 1, P.wkmax < kW2Max ? P.wkmax : kW2Max,
                    P.wblk, fan.stream(b++));
    if (P.wblk_hi) {
        const size_t lds = wave_stage_bytes(N, P.wkmax, MODE == THOI_SEL_RANGE) + red_lds(red);
        const WaveKernel wk = wave_kernel<MODE>(reduce);
        hipLaunchKernelGGL(wk, dim3((unsigned)P.wblk_hi, (unsigned)a.D), dim3(64), lds, fan.stream(b++), a, P.wtab,
                           red, kW2Max + 1, P.wkmax);
    }
}

template <typename F, int MODE>
void launch_list(EvalArgs& a, const Plan& P, const RedArgs& red, const EvalWs& w, char* base, int64_t Bn,
                 hipStream_t s)
{
    const int lane_max = lane_max_for(a.precision);
    uint8_t* korder = reinterpret_cast<uint8_t*>(base + w.korder_off);
    unsigned long long* cnt = reinterpret_cast<unsigned long long*>(base + w.cnt_off);
    int64_t* lbase = reinterpret_cast<int64_t*>(base + w.base_off);
    int64_t* lblk0 = reinterpret_cast<int64_t*>(base + w.blk0_off);
    unsigned long long* cursor = reinterpret_cast<unsigned long long*>(base + w.cursor_off);
    int64_t* perm = reinterpret_cast<int64_t*>(base + w.perm_off);
    a.perm = perm;
    a.lcnt = reinterpret_cast<const int64_t*>(cnt);
    a.lbase = lbase;
    a.lblk0 = lblk0;

    hipLaunchKernelGGL(k_ws_clear, dim3(1), dim3(256), 0, s, reinterpret_cast<uint32_t*>(cnt), (int64_t)kListOrders * 2);
    const unsigned nb = (unsigned)((Bn + 255) / 256);
    hipLaunchKernelGGL(k_list_classify<MODE>, dim3(nb), dim3(256), 0, s, a, red.active, Bn, korder, cnt);
    ClassMap cm{};
    for (int k = 0; k < kListOrders; ++k) {
        cm.wave[k] = (int8_t)(k > kW2Max ? 2 : (k > lane_max ? 1 : 0));
        cm.cls[k] = (int8_t)class_of<F>(k <= lane_max ? k : lane_max);
    }
    hipLaunchKernelGGL(k_list_scan, dim3(1), dim3(64), 0, s, cnt, lbase, lblk0, cursor, cm,
                       (int64_t)kTile * P.seg_tiles, (int64_t)P.wave_tile, (int64_t)P.wave_tile_hi);
    hipLaunchKernelGGL(k_list_scatter, dim3(nb), dim3(256), 0, s, Bn, korder, lbase, cursor, perm);
    launch_engines<F, MODE>(a, P, red, s);
}

template <typename F>
void launch_forward(EvalArgs& a, const thoi_nplets* sel, const Plan& P, const RedArgs& red, const EvalWs& w,
                    char* base, hipStream_t s)
{
    const int64_t Bn = sel_B(sel);
    if (sel->mode == THOI_SEL_RANGE) launch_engines<F, THOI_SEL_RANGE>(a, P, red, s);
    else if (sel->mode == THOI_SEL_LIST) launch_list<F, THOI_SEL_LIST>(a, P, red, w, base, Bn, s);
    else launch_list<F, THOI_SEL_MASK>(a, P, red, w, base, Bn, s);
}

}  // namespace

size_t eval_ws_bytes(int64_t D, int32_t N, const thoi_nplets* sel, const thoi_eval_opts* opts)
{
    return eval_layout(D, N, sel, opts).total;
}

// Largest LDS footprint any kernel of this call needs (the host rejects calls above the limit).
size_t eval_lds_bytes(int32_t N, const thoi_nplets* sel, const thoi_eval_opts* opts)
{
    const bool range = sel->mode == THOI_SEL_RANGE;
    const bool reduce = opts->reduce != nullptr;
    const int kmax = sel_kmax(sel, N);
    const int fsize = opts->precision == THOI_FP64 ? 8 : 4;
    const int lane_max = lane_max_for(opts->precision);
    size_t need = lane_stage_bytes(N, range ? kF32LaneMax : 0, fsize) + red_lds(opts->reduce);
    if (kmax > lane_max) {
        size_t w = pair_lds_bytes(N, red_lds(opts->reduce));
        if (kmax > kW2Max) {
            const size_t w2 = wave_stage_bytes(N, kmax, range) + red_lds(opts->reduce);
            w = w > w2 ? w : w2;
        }
        need = need > w ? need : w;
    }
    return need;
}

thoi_status launch_eval(const double* Sigma, int64_t D, int32_t N, const thoi_nplets* sel, const thoi_eval_opts* opts,
                        void* out, uint8_t* flags, void* ws, size_t ws_bytes, hipStream_t s, bool serial)
{
    const EvalWs w = eval_layout(D, N, sel, opts);
    if (ws == nullptr || ws_bytes < w.total) return THOI_EWORKSPACE;
    char* base = static_cast<char*>(ws);
    const bool reduce = opts->reduce != nullptr;
    EvalArgs a{};
    a.Sigma = Sigma;
    a.N = N;
    a.D = (int32_t)D;
    a.B = sel_B(sel);
    a.g_begin = sel->mode == THOI_SEL_RANGE ? sel->g_begin : 0;
    a.out = out;
    a.out_f32 = opts->out_dtype == THOI_DTYPE_F32;
    a.write_H = (opts->write_entropy && !reduce) ? 1 : 0;
    a.flags = flags;
    a.precision = opts->precision;
    a.vif_tau = (float)(opts->vif_tau > 0 ? opts->vif_tau : 1e3);
    a.hdr = reinterpret_cast<WsHeader*>(base);
    a.refine_list = opts->precision == THOI_FP32_REFINE ? reinterpret_cast<int64_t*>(base + w.refine_off) : nullptr;
    a.refine_cap = w.refine_cap;
    a.bias.on = opts->bias_correct ? 1 : 0;
    a.bias.T = opts->T;
    if (opts->bias_correct) bias_psi_seeds(opts->T, &a.bias.psi1, &a.bias.psi2);
    a.idx = sel->idx;
    a.kmax_list = sel->kmax_list;
    a.mask = sel->mask;

    RedArgs red{};
    const int kmax = sel_kmax(sel, N);
    if (reduce) {
        const thoi_reduce* r = opts->reduce;
        red.active = 1;
        red.topk = r->topk;
        red.bins = r->hist_bins;
        red.kmax = kmax;
        red.top_val = r->top_val;
        red.top_g = r->top_g;
        red.hist = reinterpret_cast<unsigned long long*>(r->hist);
        red.seg_key = reinterpret_cast<uint64_t*>(base + w.seg_key_off);
        red.seg_g = reinterpret_cast<int64_t*>(base + w.seg_g_off);
        red.seg_hdr = reinterpret_cast<SegHdr*>(base + w.seg_hdr_off);
        red.seg_next = &a.hdr->seg_next;
        red.seg_cap = w.seg_cap;
        red.late = w.late_cap ? reinterpret_cast<LateEntry*>(base + w.late_off) : nullptr;
        red.late_next = &a.hdr->late_next;
        red.late_cap = w.late_cap;
        red.bound = r->topk > 0 ? reinterpret_cast<unsigned long long*>(base + w.bound_off) : nullptr;
        for (int k = 0; k <= kmax; ++k) {
            red.lo[k] = r->hist_bins ? r->hist_lo_hi[2 * k] : 0.0;
            red.hi[k] = r->hist_bins ? r->hist_lo_hi[2 * k + 1] : 1.0;
        }
    }

    ws_clear(base, w.clear_end, s);
    if (D == 0 || a.B == 0) return hip_status(hipGetLastError());

    if (opts->precision == THOI_FP64) {
        Plan P = make_plan<double>(N, D, sel, reduce, opts);
        P.serial = serial;
        a.seg_tiles = P.seg_tiles;
        a.wave_tile = P.wave_tile;
        a.wave_tile_hi = P.wave_tile_hi;
        launch_forward<double>(a, sel, P, red, w, base, s);
    } else {
        Plan P = make_plan<float>(N, D, sel, reduce, opts);
        P.serial = serial;
        a.seg_tiles = P.seg_tiles;
        a.wave_tile = P.wave_tile;
        a.wave_tile_hi = P.wave_tile_hi;
        launch_forward<float>(a, sel, P, red, w, base, s);
    }

    if (opts->precision == THOI_FP32_REFINE) {
        RangeOrders ro{};
        if (sel->mode == THOI_SEL_RANGE) {
            ro.kmin = sel->kmin;
            ro.kmax = sel->kmax;
            ro.g_begin = sel->g_begin;
            int64_t g = 0;
            for (int k = sel->kmin; k <= sel->kmax + 1 && k <= THOI_MAX_K + 1; ++k) {
                ro.ostart[k] = g;
                if (k <= sel->kmax) g += (int64_t)binom_u64(N, k);
            }
        }
        // every queued n-plet comes from an FP32 lane class (order <= 24)
        refine_launch(sel->mode, a, ro, red, s);
    }
    if (reduce && red.topk > 0)
        hipLaunchKernelGGL(k_red_final, dim3((unsigned)(kmax + 1), (unsigned)D), dim3(256), 0, s, red, a.hdr);
    return hip_status(hipGetLastError());
}

void eval_launch_shape(int32_t N, const thoi_nplets* sel, const thoi_eval_opts* opts, int32_t* n_launches,
                       int64_t* max_items_x)
{
    const bool reduce = opts->reduce != nullptr;
    const Plan P = opts->precision == THOI_FP64 ? make_plan<double>(N, 1, sel, reduce, opts)
                                                : make_plan<float>(N, 1, sel, reduce, opts);
    int n = 0;
    int64_t mx = 0;
    for (int c = 0; c < P.ncls; ++c) {
        if (P.nblk[c] == 0) continue;
        ++n;
        mx = P.nblk[c] * kTile > mx ? P.nblk[c] * kTile : mx;
    }
    if (P.wblk) {
        ++n;
        mx = P.wblk * kPairThreads > mx ? P.wblk * kPairThreads : mx;
    }
    if (P.wblk_hi) {
        ++n;
        mx = P.wblk_hi * 64 > mx ? P.wblk_hi * 64 : mx;
    }
    for (int c = 0; c < P.npcls; ++c) {
        if (P.pnblk[c] == 0) continue;
        ++n;
        mx = P.pnblk[c] * kPfxThreads > mx ? P.pnblk[c] * kPfxThreads : mx;
    }
    *n_launches = n;
    *max_items_x = mx;
}

thoi_status launch_reduce_init(const thoi_reduce* red, int64_t D, int32_t kmax, hipStream_t s)
{
    const int64_t ntop = red->topk > 0 ? D * (kmax + 1) * 2 * red->topk : 0;
    const int64_t nhist = red->hist_bins > 0 ? D * (kmax + 1) * (red->hist_bins + 2) : 0;
    if (ntop + nhist == 0) return THOI_OK;
    hipLaunchKernelGGL(k_red_init, dim3(256), dim3(256), 0, s, red->top_val, red->top_g, ntop,
                       reinterpret_cast<unsigned long long*>(red->hist), nhist);
    return hip_status(hipGetLastError());
}

}  // namespace thoi
