// Forward evaluation of (TC, DTC, Omega, S) over batches of n-plets on gfx950.
//
// Work decomposition (replacing the expand-and-index batching of Methods, "Batched
// sub-covariance matrices", and the identity padding of "padded batches"):
//  - every workgroup handles one dataset d (grid.y) and one tile of n-plets of ONE order k, so
//    the order is uniform in the workgroup and the per-order code is fully unrolled;
//  - the dataset's correlation matrix is staged once per workgroup in LDS; an n-plet's
//    sub-matrix is gathered from there into registers and never exists in HBM;
//  - RANGE mode unranks each n-plet from its global index in the lane (no index tensors);
//  - orders are grouped into a few kernel classes by register footprint; each class is one
//    launch covering all of its orders (per-order tiles are mapped from blockIdx);
//  - orders above the register classes use one wavefront per n-plet with the matrix in LDS.
// FP32_REFINE: the FP32 lane engine flags n-plets whose max VIF exceeds tau (or that failed);
// a follow-up FP64 kernel re-evaluates exactly those and overwrites their results.
#include "nplets_common.hpp"

namespace thoi {

namespace {

constexpr int kTile = 256;          // n-plets (= threads) per lane-engine workgroup
constexpr int kMaxPieces = 24;      // orders per launch class
constexpr int kWaveTile = 8;        // n-plets per wave-engine workgroup
constexpr int kListOrders = THOI_MAX_K + 2;   // k = 0..64 and one "invalid" bucket

// Kernel classes: [lo, hi] of orders evaluated by one launch of the lane engine.
struct KClass { int lo, hi; };
constexpr KClass kF32Classes[] = {{0, 8}, {9, 12}, {13, 16}, {17, 20}, {21, 24}};
constexpr KClass kF64Classes[] = {{0, 6}, {7, 10}, {11, 14}, {15, 18}};
constexpr int kF32LaneMax = 24;
constexpr int kF64LaneMax = 18;

struct Piece {
    int32_t k;
    int32_t pad;
    int64_t first;   // RANGE: first lexicographic rank inside C(N, k); LIST/MASK: first slot of perm
    int64_t pos0;    // RANGE: output position of `first`
    int64_t cnt;     // n-plets in the piece
    int64_t tile0;   // first tile of the piece inside its launch
};
struct PieceTable {
    int32_t n;
    int32_t pad;
    Piece p[kMaxPieces];
};
struct BiasTable {   // per order k - lo of the class (or k for the wave engine, up to 64)
    double dtc[THOI_MAX_K + 1], ddtc[THOI_MAX_K + 1], eta[THOI_MAX_K + 1];
};

struct EvalArgs {
    const double* Sigma;
    int32_t N, D;
    int64_t B;               // output positions per dataset
    void* out;
    int32_t out_f32, write_H;
    uint8_t* flags;
    int32_t precision;
    float vif_tau;
    WsHeader* hdr;
    int64_t* refine_list;
    uint32_t refine_cap;
    int32_t bias;
    // LIST / MASK
    const int32_t* idx;
    int32_t kmax_list;
    const uint64_t* mask;
    const int64_t* perm;     // [B] positions sorted by order
    const int64_t* lcnt;     // [kListOrders] per-order counts
    const int64_t* lbase;    // [kListOrders] first slot in perm
    const int64_t* ltile0;   // [kListOrders] first tile of the order inside its class
};

// ------------------------------------------------------------------------------------------------
// Result handling shared by the engines
// ------------------------------------------------------------------------------------------------
template <typename F>
__device__ __forceinline__ void store_result(const EvalArgs& a, int d, int64_t pos, int k, const FactorOut<F>& f,
                                             double sumlogd, double dtc, double ddtc, double eta,
                                             bool refine_path)
{
    const int64_t o = (int64_t)d * a.B + pos;
    uint8_t flag = 0;
    F TC, DTC;
    const bool finite = isfinite(f.ld) && isfinite(f.sa);
    bool bad = !f.ok || !finite;
    if (!refine_path && a.precision == THOI_FP32_REFINE) {
        const bool need = bad || !(f.vmax <= (F)a.vif_tau);
        // wave-aggregated append to the refine list
        const uint64_t ballot = __ballot(need);
        if (ballot) {
            const int lane = threadIdx.x & 63;
            const int leader = __ffsll((unsigned long long)ballot) - 1;
            uint32_t base = 0;
            if (lane == leader) base = atomicAdd(&a.hdr->refine_count, (uint32_t)__popcll(ballot));
            base = __shfl(base, leader, 64);
            if (need) {
                const uint32_t slot = base + (uint32_t)__popcll(ballot & __lanemask_lt());
                if (slot < a.refine_cap) a.refine_list[slot] = o;
                else raise_status(a.hdr, THOI_EWORKSPACE);
                flag = THOI_NPLET_REFINED;
            }
        }
        bad = false;  // leave the FP32 values; the FP64 pass overwrites them
    }
    if (bad) {
        TC = DTC = (F)__builtin_nan("");
        flag |= THOI_NPLET_NOT_PD;
    } else {
        TC = F(-0.5) * f.ld + (F)dtc;
        DTC = F(0.5) * (f.ld + f.sa) + (F)ddtc;
    }
    const F OM = TC - DTC, SI = TC + DTC;
    const int64_t plane = (int64_t)a.D * a.B;
    if (a.out_f32) {
        float* op = static_cast<float*>(a.out);
        op[o] = (float)TC; op[plane + o] = (float)DTC; op[2 * plane + o] = (float)OM; op[3 * plane + o] = (float)SI;
        if (a.write_H) op[4 * plane + o] = bad ? __builtin_nanf("") : (float)(0.5 * (k * kLog2PiE + (double)f.ld + sumlogd) - eta);
    } else {
        double* op = static_cast<double*>(a.out);
        op[o] = (double)TC; op[plane + o] = (double)DTC; op[2 * plane + o] = (double)OM; op[3 * plane + o] = (double)SI;
        if (a.write_H) op[4 * plane + o] = bad ? __builtin_nan("") : 0.5 * (k * kLog2PiE + (double)f.ld + sumlogd) - eta;
    }
    if (a.flags) a.flags[o] = flag;
}

// ------------------------------------------------------------------------------------------------
// Lane engine kernels
// ------------------------------------------------------------------------------------------------
struct LaneCtx {
    int d;
    int64_t local;       // index of the n-plet inside its piece
    int64_t first, pos0;
    int N;
    int kb;
};

template <typename F, int K, int MODE>
__device__ __forceinline__ void lane_task(const EvalArgs& a, const LaneCtx& cx, const F* sR, const double* sLogd,
                                          const uint64_t* sBin, const BiasTable& bt, int klo)
{
    int c[K > 0 ? K : 1];
    int64_t pos;
    if constexpr (MODE == THOI_SEL_RANGE) {
        unrank_lex<K>((uint64_t)(cx.first + cx.local), cx.N, sBin, cx.kb, c);
        pos = cx.pos0 + cx.local;
    } else if constexpr (MODE == THOI_SEL_LIST) {
        pos = a.perm[cx.first + cx.local];
        const int32_t* row = a.idx + pos * a.kmax_list;
#pragma unroll
        for (int i = 0; i < K; ++i) c[i] = row[i];
    } else {
        pos = a.perm[cx.first + cx.local];
        uint64_t m = a.mask[pos];
#pragma unroll
        for (int i = 0; i < K; ++i) { c[i] = __builtin_ctzll(m); m &= m - 1; }
    }
    const FactorOut<F> f = lane_factor<F, K>(c, sR, cx.N);
    double sumlogd = 0.0;
    if (a.write_H) {
#pragma unroll
        for (int i = 0; i < K; ++i) sumlogd += sLogd[c[i]];
    }
    const int e = K - klo;
    store_result<F>(a, cx.d, pos, K, f, sumlogd, bt.dtc[e], bt.ddtc[e], bt.eta[e], false);
}

template <typename F, int K, int KHI, int MODE>
__device__ __forceinline__ void dispatch_k(int k, const EvalArgs& a, const LaneCtx& cx, const F* sR,
                                           const double* sLogd, const uint64_t* sBin, const BiasTable& bt, int klo)
{
    if (k == K) {
        lane_task<F, K, MODE>(a, cx, sR, sLogd, sBin, bt, klo);
        return;
    }
    if constexpr (K < KHI) dispatch_k<F, K + 1, KHI, MODE>(k, a, cx, sR, sLogd, sBin, bt, klo);
}

// LDS: sR [N*N] F | sIsd [N] f64 | sLogd [N] f64 | sBin [N*kb] u64
__host__ __device__ inline size_t lane_lds_bytes(int N, int kb, int fsize)
{
    size_t off = (size_t)N * N * fsize;
    off = (off + 7) / 8 * 8;
    off += (size_t)N * 8 * 2;
    off += (size_t)N * kb * 8;
    return off;
}

template <typename F, int KLO, int KHI, int MODE>
__global__ __launch_bounds__(kTile) void k_eval_lane(EvalArgs a, PieceTable tab, BiasTable bt)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int N = a.N;
    const int d = blockIdx.y;
    const int64_t tile = blockIdx.x;
    // which order / piece does this tile belong to (uniform in the workgroup)
    int k = -1;
    int64_t first = 0, pos0 = 0, cnt = 0, tile0 = 0;
    if constexpr (MODE == THOI_SEL_RANGE) {
        for (int p = 0; p < tab.n; ++p) {
            const int64_t nt = (tab.p[p].cnt + kTile - 1) / kTile;
            if (tile >= tab.p[p].tile0 && tile < tab.p[p].tile0 + nt) {
                k = tab.p[p].k; first = tab.p[p].first; pos0 = tab.p[p].pos0; cnt = tab.p[p].cnt; tile0 = tab.p[p].tile0;
            }
        }
    } else {
        for (int kk = KLO; kk <= KHI; ++kk) {
            const int64_t c = a.lcnt[kk];
            const int64_t nt = (c + kTile - 1) / kTile;
            const int64_t t0 = a.ltile0[kk];
            if (c > 0 && tile >= t0 && tile < t0 + nt) { k = kk; first = a.lbase[kk]; cnt = c; tile0 = t0; }
        }
    }
    if (k < 0) return;

    const int kb = (MODE == THOI_SEL_RANGE) ? KHI : 0;
    F* sR = reinterpret_cast<F*>(smem);
    size_t off = ((size_t)N * N * sizeof(F) + 7) / 8 * 8;
    double* sIsd = reinterpret_cast<double*>(smem + off);
    double* sLogd = sIsd + N;
    uint64_t* sBin = reinterpret_cast<uint64_t*>(sLogd + N);
    if constexpr (MODE == THOI_SEL_RANGE) stage_binomials(N, kb, sBin);
    stage_corr<F>(a.Sigma + (int64_t)d * N * N, N, sR, sIsd, sLogd);

    LaneCtx cx;
    cx.d = d;
    cx.local = (tile - tile0) * kTile + threadIdx.x;
    cx.first = first;
    cx.pos0 = pos0;
    cx.N = N;
    cx.kb = kb;
    const bool active = cx.local < cnt;
    if (active) dispatch_k<F, KLO, KHI, MODE>(k, a, cx, sR, sLogd, sBin, bt, KLO);
}

// ------------------------------------------------------------------------------------------------
// Wave engine kernel: orders above the register classes (one wavefront per n-plet, FP64).
// grid (tiles, D), block 64.  For RANGE a PieceTable of the orders; for LIST/MASK the device
// per-order table restricted to [klo, 64].
// LDS: sR [N*N] f64 | sIsd [N] | sLogd [N] | sBin [N*64] | sM [64*ks] | sInv [64] | cidx [64] int
// ------------------------------------------------------------------------------------------------
__host__ __device__ inline size_t wave_lds_bytes(int N, int kmax, bool with_bin)
{
    const int ks = kmax + 1;
    size_t off = (size_t)N * N * 8 + (size_t)N * 16 + (with_bin ? (size_t)N * 64 * 8 : 0);
    off += (size_t)64 * ks * 8 + 64 * 8 + 64 * 4;
    return off;
}

template <int MODE>
__global__ __launch_bounds__(64) void k_eval_wave(EvalArgs a, PieceTable tab, BiasTable bt, int klo, int kmax)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int N = a.N;
    const int d = blockIdx.y;
    const int64_t tile = blockIdx.x;
    int k = -1;
    int64_t first = 0, pos0 = 0, cnt = 0, tile0 = 0;
    if constexpr (MODE == THOI_SEL_RANGE) {
        for (int p = 0; p < tab.n; ++p) {
            const int64_t nt = (tab.p[p].cnt + kWaveTile - 1) / kWaveTile;
            if (tile >= tab.p[p].tile0 && tile < tab.p[p].tile0 + nt) {
                k = tab.p[p].k; first = tab.p[p].first; pos0 = tab.p[p].pos0; cnt = tab.p[p].cnt; tile0 = tab.p[p].tile0;
            }
        }
    } else {
        for (int kk = klo; kk <= kmax; ++kk) {
            const int64_t c = a.lcnt[kk];
            const int64_t nt = (c + kWaveTile - 1) / kWaveTile;
            const int64_t t0 = a.ltile0[kk];
            if (c > 0 && tile >= t0 && tile < t0 + nt) { k = kk; first = a.lbase[kk]; cnt = c; tile0 = t0; }
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
    if constexpr (MODE == THOI_SEL_RANGE) stage_binomials(N, 64, sBin);
    stage_corr<double>(a.Sigma + (int64_t)d * N * N, N, sR, sIsd, sLogd);

    const int lane = threadIdx.x;
    const int64_t l0 = (tile - tile0) * kWaveTile;
    const int64_t l1 = l0 + kWaveTile < cnt ? l0 + kWaveTile : cnt;
    for (int64_t l = l0; l < l1; ++l) {
        int64_t pos;
        if constexpr (MODE == THOI_SEL_RANGE) {
            if (lane == 0) unrank_lex_rt((uint64_t)(first + l), N, k, sBin, 64, cidx);
            pos = pos0 + l;
        } else if constexpr (MODE == THOI_SEL_LIST) {
            pos = a.perm[first + l];
            if (lane < k) cidx[lane] = a.idx[pos * a.kmax_list + lane];
        } else {
            pos = a.perm[first + l];
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
            store_result<double>(b, d, pos, k, f, sumlogd, bt.dtc[k], bt.ddtc[k], bt.eta[k], true);
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------------------------------------
// Refinement: FP64 re-evaluation of the n-plets queued by the FP32 lane engine.
// grid (G), block 64, grid-stride over the queue.  RANGE n-plets are unranked from the global
// index; `ostart[k]` is the global index of the first n-plet of order k.
// ------------------------------------------------------------------------------------------------
struct RangeOrders {
    int32_t kmin, kmax;
    int64_t g_begin;
    int64_t ostart[THOI_MAX_K + 2];
};

template <int MODE>
__global__ __launch_bounds__(64) void k_refine(EvalArgs a, RangeOrders ro, BiasTable bt, int kmax)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int N = a.N;
    const int ks = kmax + 1;
    double* sR = reinterpret_cast<double*>(smem);
    double* sIsd = sR + N * N;
    double* sLogd = sIsd + N;
    uint64_t* sBin = reinterpret_cast<uint64_t*>(sLogd + N);
    double* sM = reinterpret_cast<double*>(sBin + (MODE == THOI_SEL_RANGE ? N * 64 : 0));
    double* sInv = sM + 64 * ks;
    int* cidx = reinterpret_cast<int*>(sInv + 64);
    __shared__ int sk;
    if constexpr (MODE == THOI_SEL_RANGE) stage_binomials(N, 64, sBin);
    __syncthreads();
    const uint32_t n = min(a.hdr->refine_count, a.refine_cap);
    const int lane = threadIdx.x;
    int staged = -1;
    for (uint32_t q = blockIdx.x; q < n; q += gridDim.x) {
        const int64_t o = a.refine_list[q];
        const int d = (int)(o / a.B);
        const int64_t pos = o - (int64_t)d * a.B;
        if (d != staged) {
            stage_corr<double>(a.Sigma + (int64_t)d * N * N, N, sR, sIsd, sLogd);
            staged = d;
        }
        if (lane == 0) {
            int k = 0;
            if constexpr (MODE == THOI_SEL_RANGE) {
                const int64_t g = ro.g_begin + pos;
                k = ro.kmin;
                while (k < ro.kmax && g >= ro.ostart[k + 1]) ++k;
                unrank_lex_rt((uint64_t)(g - ro.ostart[k]), N, k, sBin, 64, cidx);
            } else if constexpr (MODE == THOI_SEL_LIST) {
                const int32_t* row = a.idx + pos * a.kmax_list;
                while (k < a.kmax_list && row[k] >= 0) { cidx[k] = row[k]; ++k; }
            } else {
                uint64_t m = a.mask[pos];
                while (m) { cidx[k++] = __builtin_ctzll(m); m &= m - 1; }
            }
            sk = k;
        }
        __syncthreads();
        const int k = sk;
        const FactorOut<double> f = wave_factor(sR, N, cidx, k, sM, ks, sInv);
        double sumlogd = 0.0;
        if (a.write_H) sumlogd = wave_sum(lane < k ? sLogd[cidx[lane]] : 0.0);
        if (lane == 0) {
            EvalArgs b = a;
            b.precision = THOI_FP64;
            b.flags = nullptr;
            store_result<double>(b, d, pos, k, f, sumlogd, bt.dtc[k], bt.ddtc[k], bt.eta[k], true);
            if (a.flags) a.flags[o] = (uint8_t)(THOI_NPLET_REFINED | ((!f.ok || !isfinite(f.ld) || !isfinite(f.sa)) ? THOI_NPLET_NOT_PD : 0));
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------------------------------------
// LIST / MASK: order bucketing on the device.
// ------------------------------------------------------------------------------------------------
__global__ void k_ws_clear(uint32_t* p, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = 0;
}

// grid ceil(B/256): order of every row (THOI_MAX_K + 1 = invalid) and per-order counts.
template <int MODE>
__global__ __launch_bounds__(256) void k_list_classify(EvalArgs a, int64_t Bn, uint8_t* __restrict__ korder,
                                                       unsigned long long* __restrict__ cnt)
{
    __shared__ unsigned int h[kListOrders];
    for (int i = threadIdx.x; i < kListOrders; i += blockDim.x) h[i] = 0;
    __syncthreads();
    const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (b < Bn) {
        int k = 0;
        bool ok = true;
        if constexpr (MODE == THOI_SEL_LIST) {
            const int32_t* row = a.idx + b * a.kmax_list;
            int prev = -1;
            for (int j = 0; j < a.kmax_list; ++j) {
                const int v = row[j];
                if (v < 0) {
                    if (v != -1) ok = false;
                    for (int jj = j + 1; jj < a.kmax_list; ++jj) ok = ok && (row[jj] == -1);
                    break;
                }
                ok = ok && v > prev && v < a.N;
                prev = v;
                ++k;
            }
            ok = ok && k <= THOI_MAX_K;
        } else {
            const uint64_t m = a.mask[b];
            k = __popcll(m);
            ok = (a.N >= 64) || ((m >> a.N) == 0);
        }
        if (!ok) {
            k = THOI_MAX_K + 1;
            raise_status(a.hdr, THOI_EINVAL_DATA);
            const int64_t plane = (int64_t)a.D * a.B;
            for (int d = 0; d < a.D; ++d) {
                const int64_t o = (int64_t)d * a.B + b;
                if (a.out) {
                    for (int m = 0; m < 4 + a.write_H; ++m) {
                        if (a.out_f32) static_cast<float*>(a.out)[m * plane + o] = __builtin_nanf("");
                        else static_cast<double*>(a.out)[m * plane + o] = __builtin_nan("");
                    }
                }
                if (a.flags) a.flags[o] = THOI_NPLET_NOT_PD;
            }
        }
        korder[b] = (uint8_t)k;
        atomicAdd(&h[k], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kListOrders; i += blockDim.x)
        if (h[i]) atomicAdd(&cnt[i], (unsigned long long)h[i]);
}

struct ClassMap { int8_t cls[kListOrders]; int8_t wave[kListOrders]; };

// 1 workgroup: per-order base in perm, and first tile of each order inside its launch class.
__global__ void k_list_scan(const unsigned long long* __restrict__ cnt, int64_t* __restrict__ base,
                            int64_t* __restrict__ tile0, unsigned long long* __restrict__ cursor, ClassMap cm)
{
    if (threadIdx.x != 0) return;
    int64_t b = 0;
    int64_t ct[16] = {0};
    int64_t wt = 0;
    for (int k = 0; k < kListOrders; ++k) {
        base[k] = b;
        cursor[k] = 0;
        const int64_t c = (int64_t)cnt[k];
        b += c;
        if (k > THOI_MAX_K) { tile0[k] = 0; continue; }
        if (cm.wave[k]) {
            tile0[k] = wt;
            wt += (c + kWaveTile - 1) / kWaveTile;
        } else {
            const int cl = cm.cls[k];
            tile0[k] = ct[cl];
            ct[cl] += (c + kTile - 1) / kTile;
        }
    }
}

// grid ceil(B/256): perm[base[k] + slot] = b for every valid row.
__global__ __launch_bounds__(256) void k_list_scatter(int64_t Bn, const uint8_t* __restrict__ korder,
                                                      const int64_t* __restrict__ base,
                                                      unsigned long long* __restrict__ cursor, int64_t* __restrict__ perm)
{
    __shared__ unsigned int h[kListOrders];
    __shared__ unsigned long long start[kListOrders];
    for (int i = threadIdx.x; i < kListOrders; i += blockDim.x) h[i] = 0;
    __syncthreads();
    const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int k = -1;
    unsigned int mine = 0;
    if (b < Bn) {
        k = korder[b];
        if (k <= THOI_MAX_K) mine = atomicAdd(&h[k], 1u);
        else k = -1;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kListOrders; i += blockDim.x)
        start[i] = h[i] ? atomicAdd(&cursor[i], (unsigned long long)h[i]) : 0ull;
    __syncthreads();
    if (k >= 0) perm[base[k] + (int64_t)start[k] + mine] = b;
}

// ------------------------------------------------------------------------------------------------
// Host side
// ------------------------------------------------------------------------------------------------
struct EvalWs {
    size_t refine_off, korder_off, cnt_off, base_off, tile0_off, cursor_off, perm_off, total;
    uint32_t refine_cap;
};

int64_t sel_B(const thoi_nplets* sel) { return sel->mode == THOI_SEL_RANGE ? sel->g_count : sel->B; }

EvalWs eval_layout(int64_t D, const thoi_nplets* sel, const thoi_eval_opts* opts)
{
    EvalWs w{};
    const int64_t B = sel_B(sel);
    size_t off = kWsHeader;
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
        w.tile0_off = off; off = align_up(off + kListOrders * 8, 256);
        w.cursor_off = off; off = align_up(off + kListOrders * 8, 256);
        w.perm_off = off; off = align_up(off + (size_t)B * 8, 256);
    }
    w.total = off;
    return w;
}

template <typename F>
const KClass* classes_for(int& n)
{
    if constexpr (sizeof(F) == 4) { n = (int)(sizeof(kF32Classes) / sizeof(KClass)); return kF32Classes; }
    n = (int)(sizeof(kF64Classes) / sizeof(KClass));
    return kF64Classes;
}

typedef void (*LaneKernel)(EvalArgs, PieceTable, BiasTable);

template <typename F, int MODE>
LaneKernel lane_kernel(int cls)
{
    if constexpr (sizeof(F) == 4) {
        switch (cls) {
            case 0: return k_eval_lane<F, 0, 8, MODE>;
            case 1: return k_eval_lane<F, 9, 12, MODE>;
            case 2: return k_eval_lane<F, 13, 16, MODE>;
            case 3: return k_eval_lane<F, 17, 20, MODE>;
            default: return k_eval_lane<F, 21, 24, MODE>;
        }
    } else {
        switch (cls) {
            case 0: return k_eval_lane<F, 0, 6, MODE>;
            case 1: return k_eval_lane<F, 7, 10, MODE>;
            case 2: return k_eval_lane<F, 11, 14, MODE>;
            default: return k_eval_lane<F, 15, 18, MODE>;
        }
    }
}

// Bias offsets for orders lo..hi at entries [k - lo].
BiasTable make_bias(const thoi_eval_opts* o, int lo, int hi)
{
    BiasTable bt{};
    for (int k = lo; k <= hi && k - lo <= THOI_MAX_K; ++k) {
        double a = 0, b = 0, c = 0;
        if (o->bias_correct && k + 2 <= o->T) bias_offsets(k, o->T, &a, &b, &c);
        bt.dtc[k - lo] = a;
        bt.ddtc[k - lo] = b;
        bt.eta[k - lo] = c;
    }
    return bt;
}

template <typename F>
int lane_max_for() { return sizeof(F) == 4 ? kF32LaneMax : kF64LaneMax; }

template <typename F>
int class_of(int k)
{
    int n = 0;
    const KClass* cls = classes_for<F>(n);
    int c = 0;
    while (c < n - 1 && k > cls[c].hi) ++c;
    return c;
}

// RANGE: split [g_begin, g_begin + g_count) into per-order pieces and launch each class once.
template <typename F>
void launch_range(const EvalArgs& a, const thoi_nplets* sel, const thoi_eval_opts* opts, hipStream_t s)
{
    int ncls = 0;
    const KClass* cls = classes_for<F>(ncls);
    const int lane_max = lane_max_for<F>();
    const int N = a.N;
    int64_t g = 0;
    for (int k = 0; k < sel->kmin; ++k) (void)k;
    const int64_t gb = sel->g_begin, ge = sel->g_begin + sel->g_count;
    PieceTable tabs[8] = {};
    PieceTable wtab{};
    int64_t ntiles[8] = {0}, wtiles = 0;
    int wkmax = 0;
    for (int k = sel->kmin; k <= sel->kmax; ++k) {
        const int64_t ck = (int64_t)binom_u64(N, k);
        const int64_t lo = gb > g ? gb : g, hi = ge < g + ck ? ge : g + ck;
        if (hi > lo) {
            Piece p{};
            p.k = k;
            p.first = lo - g;
            p.pos0 = lo - gb;
            p.cnt = hi - lo;
            if (k <= lane_max) {
                const int c = class_of<F>(k);
                p.tile0 = ntiles[c];
                ntiles[c] += (p.cnt + kTile - 1) / kTile;
                tabs[c].p[tabs[c].n++] = p;
            } else {
                p.tile0 = wtiles;
                wtiles += (p.cnt + kWaveTile - 1) / kWaveTile;
                wtab.p[wtab.n++] = p;
                wkmax = k > wkmax ? k : wkmax;
            }
        }
        g += ck;
    }
    for (int c = 0; c < ncls; ++c) {
        if (tabs[c].n == 0) continue;
        const BiasTable bt = make_bias(opts, cls[c].lo, cls[c].hi);
        const size_t lds = lane_lds_bytes(N, cls[c].hi, sizeof(F));
        dim3 grid((unsigned)ntiles[c], (unsigned)a.D);
        const LaneKernel kern = lane_kernel<F, THOI_SEL_RANGE>(c);
        hipLaunchKernelGGL(kern, grid, dim3(kTile), lds, s, a, tabs[c], bt);
    }
    if (wtab.n) {
        const BiasTable bt = make_bias(opts, 0, THOI_MAX_K);
        dim3 grid((unsigned)wtiles, (unsigned)a.D);
        hipLaunchKernelGGL(k_eval_wave<THOI_SEL_RANGE>, grid, dim3(64), wave_lds_bytes(N, wkmax, true), s, a, wtab, bt, 0, wkmax);
    }
}

// LIST / MASK: bucket rows by order on the device, then launch every class with an upper-bound grid.
template <typename F, int MODE>
void launch_list(EvalArgs& a, const thoi_eval_opts* opts, const EvalWs& w, char* base, int64_t Bn, hipStream_t s)
{
    int ncls = 0;
    const KClass* cls = classes_for<F>(ncls);
    const int lane_max = lane_max_for<F>();
    uint8_t* korder = reinterpret_cast<uint8_t*>(base + w.korder_off);
    unsigned long long* cnt = reinterpret_cast<unsigned long long*>(base + w.cnt_off);
    int64_t* lbase = reinterpret_cast<int64_t*>(base + w.base_off);
    int64_t* ltile0 = reinterpret_cast<int64_t*>(base + w.tile0_off);
    unsigned long long* cursor = reinterpret_cast<unsigned long long*>(base + w.cursor_off);
    int64_t* perm = reinterpret_cast<int64_t*>(base + w.perm_off);
    a.perm = perm;
    a.lcnt = reinterpret_cast<const int64_t*>(cnt);
    a.lbase = lbase;
    a.ltile0 = ltile0;

    hipLaunchKernelGGL(k_ws_clear, dim3(1), dim3(256), 0, s, reinterpret_cast<uint32_t*>(cnt), (int64_t)kListOrders * 2);
    const unsigned nb = (unsigned)((Bn + 255) / 256);
    if (Bn > 0) hipLaunchKernelGGL(k_list_classify<MODE>, dim3(nb), dim3(256), 0, s, a, Bn, korder, cnt);
    ClassMap cm{};
    for (int k = 0; k < kListOrders; ++k) {
        cm.wave[k] = (k > lane_max) ? 1 : 0;
        cm.cls[k] = (int8_t)class_of<F>(k <= lane_max ? k : lane_max);
    }
    hipLaunchKernelGGL(k_list_scan, dim3(1), dim3(64), 0, s, cnt, lbase, ltile0, cursor, cm);
    if (Bn == 0) return;
    hipLaunchKernelGGL(k_list_scatter, dim3(nb), dim3(256), 0, s, Bn, korder, lbase, cursor, perm);

    const int N = a.N;
    PieceTable none{};
    for (int c = 0; c < ncls; ++c) {
        const BiasTable bt = make_bias(opts, cls[c].lo, cls[c].hi);
        const size_t lds = lane_lds_bytes(N, 0, sizeof(F));
        const int64_t grid_x = (Bn + kTile - 1) / kTile + (cls[c].hi - cls[c].lo + 1);
        const LaneKernel kern = lane_kernel<F, MODE>(c);
        hipLaunchKernelGGL(kern, dim3((unsigned)grid_x, (unsigned)a.D), dim3(kTile), lds, s, a, none, bt);
    }
    const int kcap = MODE == THOI_SEL_LIST ? a.kmax_list : (N < 64 ? N : 64);
    if (kcap > lane_max) {
        const BiasTable bt = make_bias(opts, 0, THOI_MAX_K);
        const int64_t grid_x = (Bn + kWaveTile - 1) / kWaveTile + (kcap - lane_max);
        hipLaunchKernelGGL(k_eval_wave<MODE>, dim3((unsigned)grid_x, (unsigned)a.D), dim3(64),
                           wave_lds_bytes(N, kcap, false), s, a, none, bt, lane_max + 1, kcap);
    }
}

template <typename F>
void launch_forward(EvalArgs& a, const thoi_nplets* sel, const thoi_eval_opts* opts, const EvalWs& w, char* base,
                    hipStream_t s)
{
    const int64_t Bn = sel_B(sel);
    if (sel->mode == THOI_SEL_RANGE) launch_range<F>(a, sel, opts, s);
    else if (sel->mode == THOI_SEL_LIST) launch_list<F, THOI_SEL_LIST>(a, opts, w, base, Bn, s);
    else launch_list<F, THOI_SEL_MASK>(a, opts, w, base, Bn, s);
}

}  // namespace

size_t eval_ws_bytes(int64_t D, int32_t N, const thoi_nplets* sel, const thoi_eval_opts* opts)
{
    (void)N;
    return eval_layout(D, sel, opts).total;
}

// Largest LDS footprint any kernel of this call needs (the host rejects calls above the limit).
size_t eval_lds_bytes(int32_t N, const thoi_nplets* sel, const thoi_eval_opts* opts)
{
    const bool range = sel->mode == THOI_SEL_RANGE;
    const int kmax = range ? sel->kmax : (sel->mode == THOI_SEL_LIST ? sel->kmax_list : (N < 64 ? N : 64));
    const int fsize = opts->precision == THOI_FP64 ? 8 : 4;
    const int lane_max = opts->precision == THOI_FP64 ? kF64LaneMax : kF32LaneMax;
    size_t need = lane_lds_bytes(N, range ? kF32LaneMax : 0, fsize);   // kb <= largest class bound
    if (kmax > lane_max || opts->precision == THOI_FP32_REFINE) {
        const size_t w = wave_lds_bytes(N, kmax < 64 ? kmax : 64, range);
        need = need > w ? need : w;
    }
    return need;
}

thoi_status launch_eval(const double* Sigma, int64_t D, int32_t N, const thoi_nplets* sel, const thoi_eval_opts* opts,
                        void* out, uint8_t* flags, void* ws, size_t ws_bytes, hipStream_t s)
{
    const EvalWs w = eval_layout(D, sel, opts);
    if (ws == nullptr || ws_bytes < w.total) return THOI_EWORKSPACE;
    char* base = static_cast<char*>(ws);
    EvalArgs a{};
    a.Sigma = Sigma;
    a.N = N;
    a.D = (int32_t)D;
    a.B = sel_B(sel);
    a.out = out;
    a.out_f32 = opts->out_dtype == THOI_DTYPE_F32;
    a.write_H = opts->write_entropy ? 1 : 0;
    a.flags = flags;
    a.precision = opts->precision;
    a.vif_tau = (float)(opts->vif_tau > 0 ? opts->vif_tau : 1e3);
    a.hdr = reinterpret_cast<WsHeader*>(base);
    a.refine_list = opts->precision == THOI_FP32_REFINE ? reinterpret_cast<int64_t*>(base + w.refine_off) : nullptr;
    a.refine_cap = w.refine_cap;
    a.bias = opts->bias_correct;
    a.idx = sel->idx;
    a.kmax_list = sel->kmax_list;
    a.mask = sel->mask;

    hipLaunchKernelGGL(k_ws_clear, dim3(1), dim3(64), 0, s, reinterpret_cast<uint32_t*>(base), (int64_t)(kWsHeader / 4));
    if (D == 0 || a.B == 0) return hip_status(hipGetLastError());

    if (opts->precision == THOI_FP64) launch_forward<double>(a, sel, opts, w, base, s);
    else launch_forward<float>(a, sel, opts, w, base, s);

    if (opts->precision == THOI_FP32_REFINE) {
        RangeOrders ro{};
        int kmax = THOI_MAX_K;
        if (sel->mode == THOI_SEL_RANGE) {
            ro.kmin = sel->kmin;
            ro.kmax = sel->kmax;
            ro.g_begin = sel->g_begin;
            int64_t g = 0;
            for (int k = sel->kmin; k <= sel->kmax + 1 && k <= THOI_MAX_K + 1; ++k) {
                ro.ostart[k] = g;
                if (k <= sel->kmax) g += (int64_t)binom_u64(N, k);
            }
            kmax = sel->kmax;
        } else if (sel->mode == THOI_SEL_LIST) {
            kmax = sel->kmax_list < THOI_MAX_K ? sel->kmax_list : THOI_MAX_K;
        } else {
            kmax = N < THOI_MAX_K ? N : THOI_MAX_K;
        }
        const BiasTable bt = make_bias(opts, 0, THOI_MAX_K);
        const size_t lds = wave_lds_bytes(N, kmax, sel->mode == THOI_SEL_RANGE);
        const unsigned G = 1024;
        if (sel->mode == THOI_SEL_RANGE)
            hipLaunchKernelGGL(k_refine<THOI_SEL_RANGE>, dim3(G), dim3(64), lds, s, a, ro, bt, kmax);
        else if (sel->mode == THOI_SEL_LIST)
            hipLaunchKernelGGL(k_refine<THOI_SEL_LIST>, dim3(G), dim3(64), lds, s, a, ro, bt, kmax);
        else
            hipLaunchKernelGGL(k_refine<THOI_SEL_MASK>, dim3(G), dim3(64), lds, s, a, ro, bt, kmax);
    }
    return hip_status(hipGetLastError());
}

}  // namespace thoi
