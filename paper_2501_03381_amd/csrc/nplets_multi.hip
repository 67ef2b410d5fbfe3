// Many datasets of uneven size (N_d variables, T_d samples) in one call on gfx950.
//
// The paper batches D datasets of identical size (Methods, "Parallel and batched computation of
// HOI"); here every dataset keeps its own N_d, so the work is a ragged set of (dataset, order)
// blocks.  A one-workgroup planning kernel turns the per-dataset sizes into a work table in the
// workspace: per register class, the (dataset, order) entries in dataset-major order, each split
// into work units of kTile * seg_tiles n-plets, with their output offsets and the digamma seeds
// of the dataset's bias correction.  Each class then runs ONE persistent launch whose workgroups
// stride over the class's units, binary-search the unit's entry, restage the dataset's
// correlation matrix only when the dataset changes, and evaluate with the same register engine
// as the single-dataset path.  Datasets are processed in chunks of kChunkD.
#include "nplets_fwd_common.hpp"

namespace thoi {
namespace {

constexpr int kChunkD = 256;
constexpr int kMaxClasses = 8;

struct MultiChunk {
    int32_t n;                  // datasets in the chunk
    int32_t kmin, kmax;
    int32_t nmax;               // largest N_d of the chunk
    int32_t bias;
    int32_t ncls;
    int32_t cls_lo[kMaxClasses], cls_hi[kMaxClasses];
    int64_t per_unit;           // n-plets per work unit
    int64_t sig_base;           // element offset of the chunk's first matrix
    int64_t out_base;           // output position of the chunk's first n-plet
    uint8_t N[kChunkD];
    int32_t T[kChunkD];
};

struct MultiUnit {
    int32_t d, k;               // chunk-local dataset, order
    int64_t unit0;              // first unit of the entry inside its class
    int64_t cnt;                // n-plets = C(N_d, k)
    int64_t pos0;               // absolute output position of the entry's first n-plet
    int64_t gbase;              // index inside dataset d of the entry's first n-plet
};

struct MultiPlan {
    int64_t sig_off[kChunkD];          // absolute element offset of matrix d
    int64_t out_off[kChunkD + 1];      // absolute output offset of dataset d
    int64_t ostart[kChunkD][THOI_MAX_K + 2];   // index inside dataset d of the first n-plet of order k
    double psi1[kChunkD], psi2[kChunkD];
    int32_t cls_first[kMaxClasses], cls_count[kMaxClasses];
    int64_t cls_units[kMaxClasses];
    MultiUnit units[kChunkD * (THOI_MAX_K + 1)];
};

// psi at the integer or half-integer twice_x / 2 from the exact finite sums (Kahan-compensated).
__device__ double psi_exact_sum(int twice_x)
{
    const double gamma = 0.57721566490153286061;
    double s = 0.0, comp = 0.0;
    if (twice_x % 2 == 0) {
        for (int i = twice_x / 2 - 1; i >= 1; --i) {
            const double y = 1.0 / i - comp, t = s + y;
            comp = (t - s) - y;
            s = t;
        }
        return -gamma + s;
    }
    for (int i = (twice_x - 1) / 2; i >= 1; --i) {
        const double y = 2.0 / (2.0 * i - 1.0) - comp, t = s + y;
        comp = (t - s) - y;
        s = t;
    }
    return -gamma - 2.0 * 0.69314718055994530942 + s;
}

// One workgroup of 256: the work table of one chunk.
__global__ __launch_bounds__(256) void k_multi_plan(MultiChunk ch, MultiPlan* __restrict__ plan)
{
    __shared__ uint64_t bin[THOI_MAX_N_RANGE + 1][THOI_MAX_K + 2];
    // Pascal's triangle, rows 0..nmax, by wave 0 (lane m holds column m)
    if (threadIdx.x < 64) {
        const int m = threadIdx.x;
        uint64_t v = (m == 0) ? 1ull : 0ull;
        for (int n = 0; n <= ch.nmax; ++n) {
            if (n > 0) {
                const uint32_t lo = __shfl_up((uint32_t)v, 1, 64);
                const uint32_t hi = __shfl_up((uint32_t)(v >> 32), 1, 64);
                if (m > 0) v += ((uint64_t)hi << 32) | lo;
            }
            bin[n][m] = v;
            if (m == 63) bin[n][64] = (n >= 64) ? 1ull : 0ull;
        }
    }
    __syncthreads();
    const int d = threadIdx.x;
    if (d < ch.n) {
        const int Nd = ch.N[d];
        int64_t s = 0;
        for (int k = ch.kmin; k <= ch.kmax + 1; ++k) {
            plan->ostart[d][k] = s;
            if (k <= ch.kmax && k <= Nd) s += (int64_t)bin[Nd][k];
        }
        if (ch.bias) {
            plan->psi1[d] = psi_exact_sum(ch.T[d] - 1);
            plan->psi2[d] = psi_exact_sum(ch.T[d] - 2);
        } else {
            plan->psi1[d] = plan->psi2[d] = 0.0;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t so = ch.sig_base, oo = ch.out_base;
        for (int e = 0; e < ch.n; ++e) {
            plan->sig_off[e] = so;
            plan->out_off[e] = oo;
            so += (int64_t)ch.N[e] * ch.N[e];
            oo += plan->ostart[e][ch.kmax + 1];
        }
        plan->out_off[ch.n] = oo;
        int ne = 0;
        for (int c = 0; c < ch.ncls; ++c) {
            plan->cls_first[c] = ne;
            int64_t units = 0;
            for (int e = 0; e < ch.n; ++e) {
                const int Nd = ch.N[e];
                for (int k = ch.cls_lo[c]; k <= ch.cls_hi[c]; ++k) {
                    if (k < ch.kmin || k > ch.kmax || k > Nd) continue;
                    MultiUnit u;
                    u.d = e;
                    u.k = k;
                    u.unit0 = units;
                    u.cnt = (int64_t)bin[Nd][k];
                    u.gbase = plan->ostart[e][k];
                    u.pos0 = plan->out_off[e] + u.gbase;
                    units += (u.cnt + ch.per_unit - 1) / ch.per_unit;
                    plan->units[ne++] = u;
                }
            }
            plan->cls_count[c] = ne - plan->cls_first[c];
            plan->cls_units[c] = units;
        }
    }
}

__device__ __forceinline__ int find_unit(const MultiPlan* plan, int first, int count, int64_t u)
{
    int lo = first, hi = first + count - 1;   // last entry with unit0 <= u
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (plan->units[mid].unit0 <= u) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Persistent launch of one register class.  grid (G), block kTile.
// LDS: sR [nmax^2] F | sIsd [nmax] | sLogd [nmax] | sBin [nmax * KHI] | (reduce) RedLds
template <typename F, int KLO, int KHI, bool RED>
__global__ __launch_bounds__(kTile) void k_eval_multi(EvalArgs a, const MultiPlan* __restrict__ plan, MultiChunk ch,
                                                      int cls, RedArgs red)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double sbias[3];
    const int nmax = ch.nmax;
    F* sR = reinterpret_cast<F*>(smem);
    const size_t off = ((size_t)nmax * nmax * sizeof(F) + 15) / 16 * 16;
    double* sIsd = reinterpret_cast<double*>(smem + off);
    double* sLogd = sIsd + nmax;
    uint64_t* sBin = reinterpret_cast<uint64_t*>(sLogd + nmax);
    RedLds& S = *reinterpret_cast<RedLds*>(smem + lane_stage_bytes(nmax, KHI, sizeof(F)));
    stage_binomials(nmax, KHI, sBin);   // C(n, m) does not depend on the dataset
    __syncthreads();

    const int first = plan->cls_first[cls], count = plan->cls_count[cls];
    const int64_t total = plan->cls_units[cls];
    int staged = -1;
    for (int64_t u = blockIdx.x; u < total; u += gridDim.x) {
        const MultiUnit U = plan->units[find_unit(plan, first, count, u)];
        const int Nd = ch.N[U.d];
        if (U.d != staged) {
            stage_corr<F>(a.Sigma + plan->sig_off[U.d], Nd, sR, sIsd, sLogd);
            staged = U.d;
        }
        if (threadIdx.x == 0) {
            BiasParams bp;
            bp.on = ch.bias;
            bp.T = ch.T[U.d];
            bp.psi1 = plan->psi1[U.d];
            bp.psi2 = plan->psi2[U.d];
            bias_for(bp, U.k, sbias[0], sbias[1], sbias[2]);
        }
        if constexpr (RED) red_begin(S, red.topk, red.bins);   // contains a barrier
        else __syncthreads();
        LaneCtx cx;
        cx.d = 0;
        cx.first = 0;
        cx.pos0 = U.pos0;
        cx.gbase = U.gbase;
        cx.N = Nd;
        cx.kb = KHI;
        cx.reduce = RED;
        cx.dtc = sbias[0];
        cx.ddtc = sbias[1];
        cx.eta = sbias[2];
        const int64_t base = (u - U.unit0) * ch.per_unit;
        for (int64_t tb = base; tb < base + ch.per_unit && tb < U.cnt; tb += kTile) {
            cx.local = tb + threadIdx.x;
            double omega[1] = {0.0};
            int64_t gidx[1] = {0};
            bool valid[1] = {false};
            if (cx.local < U.cnt) dispatch_k<F, KLO, KHI, kSelMulti, 1>(U.k, a, cx, sR, sLogd, sBin, U.cnt, omega, gidx, valid);
            if constexpr (RED) red_push(S, red, U.k, valid[0], omega[0], gidx[0]);
        }
        if constexpr (RED) red_end(S, red, a.hdr, U.d, U.k);
        __syncthreads();
    }
}

// FP64 re-evaluation of the queued n-plets of a chunk.  grid (G), block 64.
// LDS: sR [nmax^2] f64 | sIsd [nmax] | sLogd [nmax] | sBin [nmax*64] | sM [64*ks] | sInv [64] | cidx [64]
__global__ __launch_bounds__(64) void k_refine_multi(EvalArgs a, const MultiPlan* __restrict__ plan, MultiChunk ch,
                                                     RedArgs red)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int nmax = ch.nmax;
    const int ks = ch.kmax + 1;
    double* sR = reinterpret_cast<double*>(smem);
    double* sIsd = sR + nmax * nmax;
    double* sLogd = sIsd + nmax;
    uint64_t* sBin = reinterpret_cast<uint64_t*>(sLogd + nmax);
    double* sM = reinterpret_cast<double*>(sBin + nmax * 64);
    double* sInv = sM + 64 * ks;
    int* cidx = reinterpret_cast<int*>(sInv + 64);
    __shared__ int sk, sd;
    __shared__ int64_t sg;
    // the queue is complete (the class kernels ran before this one); a workgroup without a
    // queued n-plet leaves before staging anything
    const uint32_t n = min(a.hdr->refine_count, a.refine_cap);
    if (blockIdx.x >= n) return;
    stage_binomials(nmax, 64, sBin);
    __syncthreads();
    const int lane = threadIdx.x;
    const bool reduce = red.active != 0;
    int staged = -1;
    for (uint32_t q = blockIdx.x; q < n; q += gridDim.x) {
        const int64_t o = a.refine_list[q];
        if (lane == 0) {
            int lo = 0, hi = ch.n - 1;     // dataset: last out_off <= o
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (plan->out_off[mid] <= o) lo = mid; else hi = mid - 1;
            }
            const int d = lo;
            const int64_t local = o - plan->out_off[d];
            int k = ch.kmin;
            while (k < ch.kmax && local >= plan->ostart[d][k + 1]) ++k;
            unrank_lex_rt((uint64_t)(local - plan->ostart[d][k]), ch.N[d], k, sBin, 64, cidx);
            sk = k;
            sd = d;
            sg = local;
        }
        __syncthreads();
        const int k = sk, d = sd;
        if (d != staged) {
            stage_corr<double>(a.Sigma + plan->sig_off[d], ch.N[d], sR, sIsd, sLogd);
            staged = d;
        }
        const FactorOut<double> f = wave_factor(sR, ch.N[d], cidx, k, sM, ks, sInv);
        double sumlogd = 0.0;
        if (a.write_H) sumlogd = wave_sum(lane < k ? sLogd[cidx[lane]] : 0.0);
        if (lane == 0) {
            EvalArgs b = a;
            b.precision = THOI_FP64;
            b.flags = nullptr;
            BiasParams bp;
            bp.on = ch.bias;
            bp.T = ch.T[d];
            bp.psi1 = plan->psi1[d];
            bp.psi2 = plan->psi2[d];
            double dtc, ddtc, eta, om = 0.0;
            bias_for(bp, k, dtc, ddtc, eta);
            const bool ok = store_result<double>(b, reduce, 0, o, k, f, sumlogd, dtc, ddtc, eta, true, om);
            if (a.flags) a.flags[o] = (uint8_t)(THOI_NPLET_REFINED | (ok ? 0 : THOI_NPLET_NOT_PD));
            if (reduce && ok) red_late(red, a.hdr, d, k, sg, om);
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------------------------------------
// Host side
// ------------------------------------------------------------------------------------------------
typedef void (*MultiKernel)(EvalArgs, const MultiPlan*, MultiChunk, int, RedArgs);

template <typename F, bool RED>
MultiKernel multi_kernel_r(int cls)
{
    if constexpr (sizeof(F) == 4) {
        switch (cls) {
            case 0: return k_eval_multi<F, 0, 8, RED>;
            case 1: return k_eval_multi<F, 9, 12, RED>;
            case 2: return k_eval_multi<F, 13, 16, RED>;
            case 3: return k_eval_multi<F, 17, 20, RED>;
            default: return k_eval_multi<F, 21, 24, RED>;
        }
    } else {
        switch (cls) {
            case 0: return k_eval_multi<F, 0, 6, RED>;
            case 1: return k_eval_multi<F, 7, 10, RED>;
            case 2: return k_eval_multi<F, 11, 14, RED>;
            default: return k_eval_multi<F, 15, 18, RED>;
        }
    }
}

int64_t chunk_units(const int32_t* N_d, int64_t d0, int64_t n, int kmin, int kmax, int64_t per_unit)
{
    int64_t u = 0;
    for (int64_t e = d0; e < d0 + n; ++e)
        for (int k = kmin; k <= kmax && k <= N_d[e]; ++k) u += ((int64_t)binom_u64(N_d[e], k) + per_unit - 1) / per_unit;
    return u;
}

int64_t chunk_count(const int32_t* N_d, int64_t d0, int64_t n, int kmin, int kmax)
{
    int64_t s = 0;
    for (int64_t e = d0; e < d0 + n; ++e)
        for (int k = kmin; k <= kmax && k <= N_d[e]; ++k) s += (int64_t)binom_u64(N_d[e], k);
    return s;
}

int default_seg_tiles(const thoi_eval_opts* o) { return o->seg_tiles > 0 ? o->seg_tiles : (o->reduce ? 8 : 2); }

struct MultiWs {
    size_t plan_off, refine_off, seg_key_off, seg_g_off, seg_hdr_off, late_off, total;
    uint32_t refine_cap, seg_cap, late_cap;
};

MultiWs multi_layout(const int32_t* N_d, int64_t D, int kmin, int kmax, const thoi_eval_opts* o)
{
    MultiWs w{};
    size_t off = kWsHeader;
    w.plan_off = off;
    off = align_up(off + sizeof(MultiPlan), 256);
    const int64_t per_unit = (int64_t)kTile * default_seg_tiles(o);
    int64_t max_cnt = 0, max_units = 0;
    for (int64_t d0 = 0; d0 < D; d0 += kChunkD) {
        const int64_t n = D - d0 < kChunkD ? D - d0 : kChunkD;
        const int64_t c = chunk_count(N_d, d0, n, kmin, kmax);
        const int64_t u = chunk_units(N_d, d0, n, kmin, kmax, per_unit);
        max_cnt = c > max_cnt ? c : max_cnt;
        max_units = u > max_units ? u : max_units;
    }
    if (o->precision == THOI_FP32_REFINE) {
        const int64_t cap = max_cnt < (int64_t(1) << 24) ? max_cnt : (int64_t(1) << 24);
        w.refine_cap = (uint32_t)(cap > 0 ? cap : 1);
        w.refine_off = off;
        off = align_up(off + (size_t)w.refine_cap * 8, 256);
    }
    if (o->reduce && o->reduce->topk > 0) {
        const int K = o->reduce->topk;
        w.seg_cap = (uint32_t)(max_units > 0 ? max_units : 1);
        w.seg_key_off = off; off = align_up(off + (size_t)w.seg_cap * 2 * K * 8, 256);
        w.seg_g_off = off; off = align_up(off + (size_t)w.seg_cap * 2 * K * 8, 256);
        w.seg_hdr_off = off; off = align_up(off + (size_t)w.seg_cap * sizeof(SegHdr), 256);
        w.late_cap = w.refine_cap;
        if (w.late_cap) { w.late_off = off; off = align_up(off + (size_t)w.late_cap * sizeof(LateEntry), 256); }
    }
    w.total = off;
    return w;
}

template <typename F>
void launch_multi_chunk(EvalArgs& a, const MultiChunk& ch, const MultiPlan* plan, const RedArgs& red, int grid_blocks,
                        const int64_t* cls_units_host, hipStream_t s)
{
    const bool reduce = red.active != 0;
    int ncls = 0;
    const KClass* cls = classes_for<F>(ncls);
    int nl = 0;
    for (int c = 0; c < ncls; ++c) nl += cls_units_host[c] != 0;
    FanScope fan(s, nl);       // the class launches are independent
    int b = 0;
    for (int c = 0; c < ncls; ++c) {
        if (cls_units_host[c] == 0) continue;
        const int64_t G = grid_blocks > 0 ? grid_blocks : (cls_units_host[c] < 2048 ? cls_units_host[c] : 2048);
        const size_t lds = lane_stage_bytes(ch.nmax, cls[c].hi, sizeof(F)) + red_lds(reduce);
        const MultiKernel kern = reduce ? multi_kernel_r<F, true>(c) : multi_kernel_r<F, false>(c);
        hipLaunchKernelGGL(kern, dim3((unsigned)G), dim3(kTile), lds, fan.stream(b++), a, plan, ch, c, red);
    }
}

}  // namespace

size_t multi_ws_bytes(const int32_t* N_d, int64_t D, int32_t kmin, int32_t kmax, const thoi_eval_opts* opts)
{
    return multi_layout(N_d, D, kmin, kmax, opts).total;
}

size_t multi_lds_bytes(int32_t nmax, int32_t kmax, const thoi_eval_opts* opts)
{
    const int fsize = opts->precision == THOI_FP64 ? 8 : 4;
    size_t need = lane_stage_bytes(nmax, kF32LaneMax, fsize) + red_lds(opts->reduce != nullptr);
    if (opts->precision == THOI_FP32_REFINE) {
        const size_t r = (size_t)nmax * nmax * 8 + (size_t)nmax * 16 + (size_t)nmax * 64 * 8 +
                         (size_t)64 * (kmax + 1) * 8 + 64 * 8 + 64 * 4;
        need = need > r ? need : r;
    }
    return need;
}

int multi_lane_max(int32_t precision) { return lane_max_for(precision); }

thoi_status launch_multi(const double* Sigma, const int32_t* N_d, const int32_t* T_d, int64_t D, int32_t kmin,
                         int32_t kmax, const thoi_eval_opts* opts, void* out, uint8_t* flags, void* ws,
                         size_t ws_bytes, hipStream_t s)
{
    const MultiWs w = multi_layout(N_d, D, kmin, kmax, opts);
    if (ws == nullptr || ws_bytes < w.total) return THOI_EWORKSPACE;
    char* base = static_cast<char*>(ws);
    const bool reduce = opts->reduce != nullptr;
    const int seg_tiles = default_seg_tiles(opts);
    int64_t total = 0;
    for (int64_t d0 = 0; d0 < D; d0 += kChunkD) {
        const int64_t n = D - d0 < kChunkD ? D - d0 : kChunkD;
        total += chunk_count(N_d, d0, n, kmin, kmax);
    }
    EvalArgs a{};
    a.Sigma = Sigma;
    a.D = 1;
    a.B = total;
    a.out = out;
    a.out_f32 = opts->out_dtype == THOI_DTYPE_F32;
    a.write_H = (opts->write_entropy && !reduce) ? 1 : 0;
    a.flags = flags;
    a.precision = opts->precision;
    a.vif_tau = (float)(opts->vif_tau > 0 ? opts->vif_tau : 1e3);
    a.hdr = reinterpret_cast<WsHeader*>(base);
    a.refine_list = opts->precision == THOI_FP32_REFINE ? reinterpret_cast<int64_t*>(base + w.refine_off) : nullptr;
    a.refine_cap = w.refine_cap;
    a.seg_tiles = seg_tiles;
    MultiPlan* plan = reinterpret_cast<MultiPlan*>(base + w.plan_off);

    int ncls = 0;
    const KClass* cls = opts->precision == THOI_FP64 ? classes_for<double>(ncls) : classes_for<float>(ncls);
    int64_t sig_base = 0, out_base = 0;
    for (int64_t d0 = 0; d0 < D; d0 += kChunkD) {
        const int64_t n = D - d0 < kChunkD ? D - d0 : kChunkD;
        MultiChunk ch{};
        ch.n = (int32_t)n;
        ch.kmin = kmin;
        ch.kmax = kmax;
        ch.bias = opts->bias_correct ? 1 : 0;
        ch.ncls = ncls;
        for (int c = 0; c < ncls; ++c) { ch.cls_lo[c] = cls[c].lo; ch.cls_hi[c] = cls[c].hi; }
        ch.per_unit = (int64_t)kTile * seg_tiles;
        ch.sig_base = sig_base;
        ch.out_base = out_base;
        int64_t cls_units[kMaxClasses] = {0};
        for (int64_t e = 0; e < n; ++e) {
            const int Nd = N_d[d0 + e];
            ch.N[e] = (uint8_t)Nd;
            ch.T[e] = T_d ? T_d[d0 + e] : 0;
            ch.nmax = Nd > ch.nmax ? Nd : ch.nmax;
            sig_base += (int64_t)Nd * Nd;
            for (int k = kmin; k <= kmax && k <= Nd; ++k) {
                int c = 0;
                while (c < ncls - 1 && k > cls[c].hi) ++c;
                cls_units[c] += ((int64_t)binom_u64(Nd, k) + ch.per_unit - 1) / ch.per_unit;
                out_base += (int64_t)binom_u64(Nd, k);
            }
        }
        RedArgs red{};
        if (reduce) {
            const thoi_reduce* r = opts->reduce;
            const int64_t stride_top = (int64_t)(kmax + 1) * 2 * r->topk;
            const int64_t stride_h = (int64_t)(kmax + 1) * (r->hist_bins + 2);
            red.active = 1;
            red.topk = r->topk;
            red.bins = r->hist_bins;
            red.kmax = kmax;
            red.top_val = r->topk ? r->top_val + d0 * stride_top : nullptr;
            red.top_g = r->topk ? r->top_g + d0 * stride_top : nullptr;
            red.hist = r->hist_bins ? reinterpret_cast<unsigned long long*>(r->hist) + d0 * stride_h : nullptr;
            red.seg_key = reinterpret_cast<uint64_t*>(base + w.seg_key_off);
            red.seg_g = reinterpret_cast<int64_t*>(base + w.seg_g_off);
            red.seg_hdr = reinterpret_cast<SegHdr*>(base + w.seg_hdr_off);
            red.seg_next = &a.hdr->seg_next;
            red.seg_cap = w.seg_cap;
            red.late = w.late_cap ? reinterpret_cast<LateEntry*>(base + w.late_off) : nullptr;
            red.late_next = &a.hdr->late_next;
            red.late_cap = w.late_cap;
            for (int k = 0; k <= kmax; ++k) {
                red.lo[k] = r->hist_bins ? r->hist_lo_hi[2 * k] : 0.0;
                red.hi[k] = r->hist_bins ? r->hist_lo_hi[2 * k + 1] : 1.0;
            }
        }
        // a chunk owns the header: the status word keeps the first error of the call
        hipLaunchKernelGGL(k_ws_clear, dim3(1), dim3(64), 0, s, reinterpret_cast<uint32_t*>(base) + 1,
                           (int64_t)(kWsHeader / 4 - 1));
        if (d0 == 0) hipLaunchKernelGGL(k_ws_clear, dim3(1), dim3(64), 0, s, reinterpret_cast<uint32_t*>(base), (int64_t)1);
        hipLaunchKernelGGL(k_multi_plan, dim3(1), dim3(256), 0, s, ch, plan);
        if (opts->precision == THOI_FP64) launch_multi_chunk<double>(a, ch, plan, red, opts->grid_blocks, cls_units, s);
        else launch_multi_chunk<float>(a, ch, plan, red, opts->grid_blocks, cls_units, s);
        if (opts->precision == THOI_FP32_REFINE) {
            const size_t lds = (size_t)ch.nmax * ch.nmax * 8 + (size_t)ch.nmax * 16 + (size_t)ch.nmax * 64 * 8 +
                               (size_t)64 * (kmax + 1) * 8 + 64 * 8 + 64 * 4;
            hipLaunchKernelGGL(k_refine_multi, dim3(512), dim3(64), lds, s, a, plan, ch, red);
        }
        if (reduce && red.topk > 0)
            hipLaunchKernelGGL(k_red_final, dim3((unsigned)(kmax + 1), (unsigned)n), dim3(256), 0, s, red, a.hdr);
    }
    return hip_status(hipGetLastError());
}

}  // namespace thoi
