// Many datasets of uneven size (N_d variables, T_d samples) in one call on gfx950.
//
// The paper batches D datasets of identical size (Methods, "Parallel and batched computation of
// HOI"); here every dataset keeps its own N_d, so the work is a ragged set of (dataset, order)
// blocks.  The launch sequence is fixed, whatever D:
//   1. the per-dataset sizes travel in kernel arguments, 512 datasets per upload launch, into
//      tables in the workspace;
//   2. one planning kernel (one workgroup, block-wide prefix sums over the datasets) derives each
//      dataset's matrix offset, output offset, bias seeds and, per register class, its first
//      work unit (a unit is kTile * S * seg_tiles n-plets of one (dataset, order));
//   3. ONE persistent launch per register class covers every dataset: workgroup b walks the
//      contiguous unit range [b U / G, (b + 1) U / G), so consecutive units share their dataset
//      and the correlation matrix is restaged only when the dataset changes;
//   4. FP64 refinement of the queued n-plets, and the final merge of the streaming reduction.
#include "nplets_fwd_common.hpp"

namespace thoi {
static_assert(kTile <= 64 * kRedWaves, "the reducer keeps lists for at most kRedWaves wavefronts");
namespace {

constexpr int kMaxClasses = 8;

// n-plets per lane of a class (consecutive, one unranking then successors): several in the class
// of the smallest orders, whose factorisation is a few dozen instructions and where the
// unranking would otherwise dominate (FP32 six: at orders 3..5 over 1024 datasets four, six,
// seven and eight per lane measured 1.89, 1.67, 2.0 and 2.11 ms); elsewhere as in the
// single-dataset engine.
template <typename F>
__host__ __device__ constexpr int multi_per_lane(int khi)
{
    return khi <= (sizeof(F) == 4 ? 8 : 6) ? (sizeof(F) == 4 ? 6 : 8) : lane_per_thread<F>(khi, THOI_SEL_RANGE);
}
constexpr int kUpload = 512;          // datasets per upload launch
constexpr int kPlanThreads = 1024;

// Per-dataset tables in the workspace (structure of arrays).
struct MultiTabs {
    int32_t* N;                      // [D]
    int32_t* T;                      // [D]
    int64_t* sig_off;                // [D]   element offset of matrix d
    int64_t* out_off;                // [D+1] output position of dataset d's first n-plet
    double* psi1;                    // [D]   digamma seeds of the bias correction
    double* psi2;
    int64_t* unit_off;               // [kMaxClasses][D+1] first unit of dataset d in class c
};

struct MultiArgs {
    MultiTabs t;
    int64_t D;
    int32_t kmin, kmax, bias, ncls;
    int32_t cls_lo[kMaxClasses], cls_hi[kMaxClasses];
    int32_t S[kMaxClasses];          // n-plets per lane of each class
    int64_t per_unit[kMaxClasses];   // n-plets per unit of each class
};

struct UploadArgs {
    int64_t d0;
    int32_t n;
    uint8_t N[kUpload];
    int32_t T[kUpload];
};

__global__ __launch_bounds__(256) void k_multi_upload(UploadArgs u, int32_t* __restrict__ N, int32_t* __restrict__ T)
{
    for (int i = threadIdx.x; i < u.n; i += blockDim.x) {
        N[u.d0 + i] = u.N[i];
        T[u.d0 + i] = u.T[i];
    }
}

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

// Exclusive prefix sum of v over the workgroup (blockDim.x = kPlanThreads); returns the
// workgroup total in *tot.  sc: LDS scratch of kPlanThreads / 64 entries.
__device__ __forceinline__ int64_t block_exscan(int64_t v, int64_t* sc, int64_t* tot)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int64_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) sc[w] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t s = 0;
        for (int i = 0; i < kPlanThreads / 64; ++i) { const int64_t t = sc[i]; sc[i] = s; s += t; }
        sc[kPlanThreads / 64] = s;
    }
    __syncthreads();
    const int64_t r = x - v + sc[w];
    *tot = sc[kPlanThreads / 64];
    __syncthreads();
    return r;
}

// One workgroup of kPlanThreads: every table of MultiTabs from N and T, datasets in tiles of
// kPlanThreads with the running offsets carried from tile to tile.
__global__ __launch_bounds__(kPlanThreads) void k_multi_plan(MultiArgs m)
{
    __shared__ int64_t sc[kPlanThreads / 64 + 1];
    int64_t sig = 0, out = 0, unit[kMaxClasses] = {};
    for (int64_t d0 = 0; d0 < m.D; d0 += kPlanThreads) {
        const int64_t d = d0 + threadIdx.x;
        const bool in = d < m.D;
        const int Nd = in ? m.t.N[d] : 0;
        int64_t cnt = 0, u[kMaxClasses] = {};
        for (int k = m.kmin; k <= m.kmax && k <= Nd; ++k) {
            const int64_t c = (int64_t)kPascal.v[Nd][k];
            cnt += c;
            int cl = 0;
            while (cl < m.ncls - 1 && k > m.cls_hi[cl]) ++cl;
            u[cl] += (c + m.per_unit[cl] - 1) / m.per_unit[cl];
        }
        int64_t tot;
        const int64_t es = block_exscan(in ? (int64_t)Nd * Nd : 0, sc, &tot);
        if (in) m.t.sig_off[d] = sig + es;
        sig += tot;
        const int64_t eo = block_exscan(cnt, sc, &tot);
        if (in) m.t.out_off[d] = out + eo;
        out += tot;
        for (int cl = 0; cl < m.ncls; ++cl) {
            const int64_t eu = block_exscan(u[cl], sc, &tot);
            if (in) m.t.unit_off[cl * (m.D + 1) + d] = unit[cl] + eu;
            unit[cl] += tot;
        }
        if (in) {
            if (m.bias) {
                m.t.psi1[d] = psi_exact_sum(m.t.T[d] - 1);
                m.t.psi2[d] = psi_exact_sum(m.t.T[d] - 2);
            } else {
                m.t.psi1[d] = m.t.psi2[d] = 0.0;
            }
        }
    }
    if (threadIdx.x == 0) {
        m.t.out_off[m.D] = out;
        for (int cl = 0; cl < m.ncls; ++cl) m.t.unit_off[cl * (m.D + 1) + m.D] = unit[cl];
    }
}

// Index inside dataset d (N_d variables) of the first n-plet of order k (orders from kmin).
__device__ __forceinline__ int64_t multi_ostart(int Nd, int kmin, int k)
{
    int64_t s = 0;
    for (int j = kmin; j < k && j <= Nd; ++j) s += (int64_t)kPascal.v[Nd][j];
    return s;
}

// Persistent launch of one register class.  grid (G), block kTile; U units in the class.
// LDS: sR [nmax^2] F | sIsd [nmax] | sLogd [nmax] | sBin [nmax * KHI] | (reduce) RedLds
template <typename F, int KLO, int KHI, bool RED>
__global__ __launch_bounds__(kTile) void k_eval_multi(EvalArgs a, MultiArgs m, int cls, int64_t U, int nmax,
                                                      RedArgs red)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double sbias[3];
    constexpr int S = multi_per_lane<F>(KHI);
    F* sR = reinterpret_cast<F*>(smem);
    const size_t off = ((size_t)nmax * nmax * sizeof(F) + 15) / 16 * 16;
    double* sIsd = reinterpret_cast<double*>(smem + off);
    double* sLogd = sIsd + nmax;
    uint64_t* sBin = reinterpret_cast<uint64_t*>(sLogd + nmax);
    RedLds Rl = red_view(smem + lane_stage_bytes(nmax, KHI, sizeof(F)), red.topk, red.bins);
    const int64_t G = gridDim.x;
    const int64_t u0 = (int64_t)blockIdx.x * U / G, u1 = ((int64_t)blockIdx.x + 1) * U / G;
    if (u0 >= u1) return;                                  // uniform
    stage_binomials(nmax, KHI, sBin);                      // C(n, m) does not depend on the dataset
    const int64_t* uo = m.t.unit_off + (int64_t)cls * (m.D + 1);
    const int64_t per_unit = m.per_unit[cls];
    const int klo = KLO > m.kmin ? KLO : m.kmin, khi = KHI < m.kmax ? KHI : m.kmax;
    // dataset of unit u0: the last d with uo[d] <= u0 (datasets without units repeat the offset)
    int64_t lo = 0, hi = m.D - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (uo[mid] <= u0) lo = mid; else hi = mid - 1;
    }
    int64_t d = lo;
    int64_t u = u0;
    int staged = -1, kred = -1;
    while (u < u1) {                                        // uniform: every value below is
        const int Nd = m.t.N[d];
        const int64_t du0 = uo[d], du1 = uo[d + 1];
        if (u >= du1) { ++d; continue; }                    // dataset exhausted (or empty)
        // order and unit inside the dataset
        int k = klo;
        int64_t rel = u - du0, cnt = 0, nu = 0;
        for (; k <= khi && k <= Nd; ++k) {
            cnt = (int64_t)kPascal.v[Nd][k];
            nu = (cnt + per_unit - 1) / per_unit;
            if (rel < nu) break;
            rel -= nu;
        }
        if (staged != (int)d || kred != k) {
            if constexpr (RED) {
                if (kred >= 0) red_end(Rl, red, a.hdr, staged, kred);
            }
            __syncthreads();
            if (staged != (int)d) stage_corr<F>(a.Sigma + m.t.sig_off[d], Nd, sR, sIsd, sLogd);
            if (threadIdx.x == 0) {
                BiasParams bp;
                bp.on = m.bias;
                bp.T = m.t.T[d];
                bp.psi1 = m.t.psi1[d];
                bp.psi2 = m.t.psi2[d];
                bias_for(bp, k, sbias[0], sbias[1], sbias[2]);
            }
            if constexpr (RED) red_begin(Rl, red, (int)d, k);   // contains a barrier
            else __syncthreads();
            staged = (int)d;
            kred = k;
        }
        const int64_t gbase = multi_ostart(Nd, m.kmin, k);
        LaneCtx cx;
        cx.d = 0;
        cx.first = 0;
        cx.pos0 = m.t.out_off[d] + gbase;
        cx.gbase = gbase;
        cx.N = Nd;
        cx.kb = KHI;
        cx.reduce = RED;
        cx.dtc = sbias[0];
        cx.ddtc = sbias[1];
        cx.eta = sbias[2];
        // this and the following units of the same (dataset, order) inside the range
        const int64_t run = nu - rel < u1 - u ? nu - rel : u1 - u;
        const int64_t b0 = rel * per_unit, b1 = (rel + run) * per_unit < cnt ? (rel + run) * per_unit : cnt;
        for (int64_t tb = b0; tb < b1; tb += (int64_t)kTile * S) {
            cx.local = tb + (int64_t)S * threadIdx.x;
            double omega[S] = {};
            int64_t gidx[S] = {};
            bool valid[S] = {};
            if (cx.local < b1) dispatch_k<F, KLO, KHI, kSelMulti, S>(k, a, cx, sR, sLogd, sBin, b1, omega, gidx, valid);
            if constexpr (RED) {
#pragma unroll
                for (int j = 0; j < S; ++j) red_push(Rl, red, k, valid[j], omega[j], gidx[j]);
            }
        }
        u += run;
    }
    if constexpr (RED) {
        if (kred >= 0) red_end(Rl, red, a.hdr, staged, kred);
    }
}

// FP64 re-evaluation of the queued n-plets.  grid (G), block 64.
// LDS: sR [nmax^2] f64 | sIsd [nmax] | sLogd [nmax] | sBin [nmax*64] | sM [64*ks] | sInv [64] | cidx [64]
__global__ __launch_bounds__(64) void k_refine_multi(EvalArgs a, MultiArgs m, int nmax, RedArgs red)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int ks = m.kmax + 1;
    double* sR = reinterpret_cast<double*>(smem);
    double* sIsd = sR + nmax * nmax;
    double* sLogd = sIsd + nmax;
    uint64_t* sBin = reinterpret_cast<uint64_t*>(sLogd + nmax);
    double* sM = reinterpret_cast<double*>(sBin + nmax * 64);
    double* sInv = sM + 64 * ks;
    int* cidx = reinterpret_cast<int*>(sInv + 64);
    __shared__ int sk;
    __shared__ int64_t sd, sg;
    // the queue is complete (the class kernels ran before this one); a workgroup without a
    // queued n-plet leaves before staging anything
    const uint32_t n = min(a.hdr->refine_count, a.refine_cap);
    if (blockIdx.x >= n) return;
    stage_binomials(nmax, 64, sBin);
    __syncthreads();
    const int lane = threadIdx.x;
    const bool reduce = red.active != 0;
    int64_t staged = -1;
    for (uint32_t q = blockIdx.x; q < n; q += gridDim.x) {
        const int64_t o = a.refine_list[q];
        if (lane == 0) {
            int64_t lo = 0, hi = m.D - 1;     // dataset: the last out_off <= o
            while (lo < hi) {
                const int64_t mid = (lo + hi + 1) >> 1;
                if (m.t.out_off[mid] <= o) lo = mid; else hi = mid - 1;
            }
            const int Nd = m.t.N[lo];
            const int64_t local = o - m.t.out_off[lo];
            int k = m.kmin;
            int64_t st = 0;
            while (k < m.kmax && k < Nd && local >= st + (int64_t)kPascal.v[Nd][k]) { st += (int64_t)kPascal.v[Nd][k]; ++k; }
            unrank_lex_rt((uint64_t)(local - st), Nd, k, sBin, 64, cidx);
            sk = k;
            sd = lo;
            sg = local;
        }
        __syncthreads();
        const int k = sk;
        const int64_t d = sd;
        const int Nd = m.t.N[d];
        if (d != staged) {
            stage_corr<double>(a.Sigma + m.t.sig_off[d], Nd, sR, sIsd, sLogd);
            staged = d;
        }
        const FactorOut<double> f = wave_factor(sR, Nd, cidx, k, sM, ks, sInv);
        double sumlogd = 0.0;
        if (a.write_H) sumlogd = wave_sum(lane < k ? sLogd[cidx[lane]] : 0.0);
        if (lane == 0) {
            EvalArgs b = a;
            b.precision = THOI_FP64;
            b.flags = nullptr;
            BiasParams bp;
            bp.on = m.bias;
            bp.T = m.t.T[d];
            bp.psi1 = m.t.psi1[d];
            bp.psi2 = m.t.psi2[d];
            double dtc, ddtc, eta, om = 0.0;
            bias_for(bp, k, dtc, ddtc, eta);
            const bool ok = store_result<double>(b, reduce, 0, o, k, f, sumlogd, dtc, ddtc, eta, true, om);
            if (a.flags) a.flags[o] = (uint8_t)(THOI_NPLET_REFINED | (ok ? 0 : THOI_NPLET_NOT_PD));
            if (reduce && ok) red_late(red, a.hdr, (int)d, k, sg, om);
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------------------------------------
// Host side
// ------------------------------------------------------------------------------------------------
typedef void (*MultiKernel)(EvalArgs, MultiArgs, int, int64_t, int, RedArgs);

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

int default_seg_tiles(const thoi_eval_opts* o) { return o->seg_tiles > 0 ? o->seg_tiles : (o->reduce ? 8 : 2); }

// Classes, n-plets per lane and per unit of a precision.
struct MultiShape {
    int ncls;
    KClass cls[kMaxClasses];
    int S[kMaxClasses];
    int64_t per_unit[kMaxClasses];
};

MultiShape multi_shape(const thoi_eval_opts* o)
{
    MultiShape sh{};
    const bool f64 = o->precision == THOI_FP64;
    const KClass* c = f64 ? classes_for<double>(sh.ncls) : classes_for<float>(sh.ncls);
    for (int i = 0; i < sh.ncls; ++i) {
        sh.cls[i] = c[i];
        sh.S[i] = f64 ? multi_per_lane<double>(c[i].hi) : multi_per_lane<float>(c[i].hi);
        sh.per_unit[i] = (int64_t)kTile * sh.S[i] * default_seg_tiles(o);
    }
    return sh;
}

int class_of_order(const MultiShape& sh, int k)
{
    int c = 0;
    while (c < sh.ncls - 1 && k > sh.cls[c].hi) ++c;
    return c;
}

struct MultiWs {
    size_t N_off, T_off, sig_off, out_off, psi1_off, psi2_off, unit_off;
    size_t refine_off, seg_key_off, seg_g_off, seg_hdr_off, late_off, bound_off, clear_end, total;
    uint32_t refine_cap, seg_cap, late_cap;
};

// Work units and (dataset, order) entries of every class (host replay of the plan's counts).
void multi_counts(const int32_t* N_d, int64_t D, int kmin, int kmax, const MultiShape& sh, int64_t* units,
                  int64_t* entries, int64_t* total)
{
    for (int c = 0; c < kMaxClasses; ++c) units[c] = entries[c] = 0;
    *total = 0;
    for (int64_t d = 0; d < D; ++d)
        for (int k = kmin; k <= kmax && k <= N_d[d]; ++k) {
            const int c = class_of_order(sh, k);
            const int64_t n = (int64_t)binom_u64(N_d[d], k);
            units[c] += (n + sh.per_unit[c] - 1) / sh.per_unit[c];
            entries[c] += 1;
            *total += n;
        }
}

int64_t class_grid(int64_t units, int grid_blocks)
{
    const int64_t G = grid_blocks > 0 ? grid_blocks : 2048;
    return units < G ? units : G;
}

MultiWs multi_layout(const int32_t* N_d, int64_t D, int kmin, int kmax, const thoi_eval_opts* o)
{
    MultiWs w{};
    const MultiShape sh = multi_shape(o);
    int64_t units[kMaxClasses], entries[kMaxClasses], total = 0;
    multi_counts(N_d, D, kmin, kmax, sh, units, entries, &total);
    size_t off = kWsHeader;
    if (o->reduce && o->reduce->topk > 0) {
        // admission bounds [D][kmax+1][2], cleared with the header
        w.bound_off = off;
        off = align_up(off + (size_t)D * (kmax + 1) * 2 * 8, 256);
    }
    w.clear_end = off;
    w.N_off = off; off = align_up(off + (size_t)D * 4, 256);
    w.T_off = off; off = align_up(off + (size_t)D * 4, 256);
    w.sig_off = off; off = align_up(off + (size_t)D * 8, 256);
    w.out_off = off; off = align_up(off + (size_t)(D + 1) * 8, 256);
    w.psi1_off = off; off = align_up(off + (size_t)D * 8, 256);
    w.psi2_off = off; off = align_up(off + (size_t)D * 8, 256);
    w.unit_off = off; off = align_up(off + (size_t)kMaxClasses * (D + 1) * 8, 256);
    if (o->precision == THOI_FP32_REFINE) {
        const int64_t cap = total < (int64_t(1) << 24) ? total : (int64_t(1) << 24);
        w.refine_cap = (uint32_t)(cap > 0 ? cap : 1);
        w.refine_off = off;
        off = align_up(off + (size_t)w.refine_cap * 8, 256);
    }
    if (o->reduce && o->reduce->topk > 0) {
        const int K = o->reduce->topk;
        // a workgroup writes one segment per (dataset, order) it touches: at most the class's
        // entries plus one split entry per workgroup
        int64_t segs = 0;
        for (int c = 0; c < sh.ncls; ++c) segs += entries[c] + class_grid(units[c], o->grid_blocks);
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

size_t refine_multi_lds(int nmax, int kmax)
{
    return (size_t)nmax * nmax * 8 + (size_t)nmax * 16 + (size_t)nmax * 64 * 8 + (size_t)64 * (kmax + 1) * 8 + 64 * 8 +
           64 * 4;
}

}  // namespace

size_t multi_ws_bytes(const int32_t* N_d, int64_t D, int32_t kmin, int32_t kmax, const thoi_eval_opts* opts)
{
    return multi_layout(N_d, D, kmin, kmax, opts).total;
}

size_t multi_lds_bytes(int32_t nmax, int32_t kmax, const thoi_eval_opts* opts)
{
    const int fsize = opts->precision == THOI_FP64 ? 8 : 4;
    size_t need = lane_stage_bytes(nmax, kF32LaneMax, fsize) + red_lds(opts->reduce);
    if (opts->precision == THOI_FP32_REFINE) {
        const size_t r = refine_multi_lds(nmax, kmax);
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
    const MultiShape sh = multi_shape(opts);
    int64_t units[kMaxClasses], entries[kMaxClasses], total = 0;
    multi_counts(N_d, D, kmin, kmax, sh, units, entries, &total);
    int nmax = 0;
    for (int64_t d = 0; d < D; ++d) nmax = N_d[d] > nmax ? N_d[d] : nmax;

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
    a.seg_tiles = default_seg_tiles(opts);

    MultiArgs m{};
    m.t.N = reinterpret_cast<int32_t*>(base + w.N_off);
    m.t.T = reinterpret_cast<int32_t*>(base + w.T_off);
    m.t.sig_off = reinterpret_cast<int64_t*>(base + w.sig_off);
    m.t.out_off = reinterpret_cast<int64_t*>(base + w.out_off);
    m.t.psi1 = reinterpret_cast<double*>(base + w.psi1_off);
    m.t.psi2 = reinterpret_cast<double*>(base + w.psi2_off);
    m.t.unit_off = reinterpret_cast<int64_t*>(base + w.unit_off);
    m.D = D;
    m.kmin = kmin;
    m.kmax = kmax;
    m.bias = opts->bias_correct ? 1 : 0;
    m.ncls = sh.ncls;
    for (int c = 0; c < sh.ncls; ++c) {
        m.cls_lo[c] = sh.cls[c].lo;
        m.cls_hi[c] = sh.cls[c].hi;
        m.S[c] = sh.S[c];
        m.per_unit[c] = sh.per_unit[c];
    }

    RedArgs red{};
    if (reduce) {
        const thoi_reduce* r = opts->reduce;
        red.active = 1;
        red.topk = r->topk;
        red.bins = r->hist_bins;
        red.kmax = kmax;
        red.top_val = r->topk ? r->top_val : nullptr;
        red.top_g = r->topk ? r->top_g : nullptr;
        red.hist = r->hist_bins ? reinterpret_cast<unsigned long long*>(r->hist) : nullptr;
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
    for (int64_t d0 = 0; d0 < D; d0 += kUpload) {
        UploadArgs u{};
        u.d0 = d0;
        u.n = (int32_t)(D - d0 < kUpload ? D - d0 : kUpload);
        for (int i = 0; i < u.n; ++i) {
            u.N[i] = (uint8_t)N_d[d0 + i];
            u.T[i] = T_d ? T_d[d0 + i] : 0;
        }
        hipLaunchKernelGGL(k_multi_upload, dim3(1), dim3(256), 0, s, u, m.t.N, m.t.T);
    }
    hipLaunchKernelGGL(k_multi_plan, dim3(1), dim3(kPlanThreads), 0, s, m);
    {
        int nl = 0;
        for (int c = 0; c < sh.ncls; ++c) nl += units[c] != 0;
        FanScope fan(s, nl);       // the class launches are independent
        int b = 0;
        for (int c = 0; c < sh.ncls; ++c) {
            if (units[c] == 0) continue;
            const int64_t G = class_grid(units[c], opts->grid_blocks);
            const size_t lds = lane_stage_bytes(nmax, sh.cls[c].hi, opts->precision == THOI_FP64 ? 8 : 4) + red_lds(red);
            MultiKernel kern;
            if (opts->precision == THOI_FP64) kern = reduce ? multi_kernel_r<double, true>(c) : multi_kernel_r<double, false>(c);
            else kern = reduce ? multi_kernel_r<float, true>(c) : multi_kernel_r<float, false>(c);
            hipLaunchKernelGGL(kern, dim3((unsigned)G), dim3(kTile), lds, fan.stream(b++), a, m, c, units[c], nmax, red);
        }
    }
    if (opts->precision == THOI_FP32_REFINE)
        hipLaunchKernelGGL(k_refine_multi, dim3(512), dim3(64), refine_multi_lds(nmax, kmax), s, a, m, nmax, red);
    if (reduce && red.topk > 0)
        hipLaunchKernelGGL(k_red_final, dim3((unsigned)(kmax + 1), (unsigned)D), dim3(256), 0, s, red, a.hdr);
    return hip_status(hipGetLastError());
}

}  // namespace thoi
