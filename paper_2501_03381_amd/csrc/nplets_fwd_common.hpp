// Definitions shared by the forward translation units (single-selection and multi-dataset).
// Everything here has internal linkage: each translation unit gets its own copy.
#pragma once

#include "nplets_common.hpp"
#include "reduce_common.hpp"

namespace thoi {

// Argument structures of the forward kernels: defined outside the anonymous namespace (the same
// definition in every translation unit) so that launchers in one unit can take them from another.
inline constexpr int kMaxPieces = 24;      // orders per launch class

struct Piece {
    int32_t k;
    int32_t pad;
    int64_t first;   // RANGE: first lexicographic rank inside C(N, k)
    int64_t pos0;    // RANGE: output position of `first`
    int64_t cnt;     // n-plets in the piece
    int64_t blk0;    // first workgroup of the piece inside its launch
};
struct PieceTable {
    int32_t n;
    int32_t pad;
    Piece p[kMaxPieces];
};

// Bias offsets of Eq. (bias_corrector) are rebuilt on the device from two digamma seeds:
// psi_j = psi((T-j)/2), psi_j = psi_{j-2} - 2/(T-j).
struct BiasParams {
    int32_t on, T;
    double psi1, psi2;
};

// RANGE refinement: the orders of the call and the global index of the first n-plet of each.
struct RangeOrders {
    int32_t kmin, kmax;
    int64_t g_begin;
    int64_t ostart[THOI_MAX_K + 2];
};

struct EvalArgs {
    const double* Sigma;
    int32_t N, D;
    int64_t B;               // output positions per dataset
    int64_t g_begin;         // RANGE: global index of position 0
    void* out;
    int32_t out_f32, write_H;
    uint8_t* flags;
    int32_t precision;
    float vif_tau;
    WsHeader* hdr;
    int64_t* refine_list;
    uint32_t refine_cap;
    int32_t seg_tiles;       // lane engine: tiles of kTile n-plets per workgroup
    int32_t wave_tile;       // pair engine (orders up to 32 above the lane classes): n-plets per workgroup
    int32_t wave_tile_hi;    // wave engine (orders above 32): n-plets per workgroup
    BiasParams bias;
    // LIST / MASK
    const int32_t* idx;
    int32_t kmax_list;
    const uint64_t* mask;
    const int64_t* perm;     // [B] positions sorted by order
    const int64_t* lcnt;     // [kListOrders] per-order counts
    const int64_t* lbase;    // [kListOrders] first slot in perm
    const int64_t* lblk0;    // [kListOrders] first workgroup of the order inside its launch
};

namespace {


constexpr int kTile = 256;          // n-plets (= threads) per lane-engine tile
constexpr int kWaveTileOut = 1;     // n-plets per wave-engine workgroup (output mode): spread the few, long factorisations over CUs
constexpr int kWaveTileRed = 64;    // n-plets per wave-engine workgroup (reduce mode)
constexpr int kListOrders = THOI_MAX_K + 2;   // k = 0..64 and one "invalid" bucket

// Kernel classes: [lo, hi] of orders evaluated by one launch of the lane engine.
struct KClass { int lo, hi; };
constexpr KClass kF32Classes[] = {{0, 8}, {9, 12}, {13, 16}, {17, 20}, {21, 24}};
constexpr KClass kF64Classes[] = {{0, 6}, {7, 10}, {11, 14}, {15, 18}};
// Launch order of the classes of one evaluation.  The concurrent class grids start dispatching in
// launch order, each once the previous one has placed its workgroups.  A class whose grid fits in
// one round of waves but whose lanes run longest (FP32 orders 13..16 at N = 20) goes first, and
// the largest grid fills the GPU around it.  FP64 keeps ascending order: its long classes need
// several rounds at one wave per SIMD and, launched first, hold every SIMD.
constexpr int kF32LaunchOrder[] = {2, 1, 3, 0, 4};
constexpr int kF64LaunchOrder[] = {0, 1, 2, 3};
static_assert(sizeof(kF32LaunchOrder) / sizeof(int) == sizeof(kF32Classes) / sizeof(KClass), "one entry per class");
static_assert(sizeof(kF64LaunchOrder) / sizeof(int) == sizeof(kF64Classes) / sizeof(KClass), "one entry per class");
constexpr int kF32LaneMax = 24;
constexpr int kF64LaneMax = 18;

__device__ __forceinline__ void bias_for(const BiasParams& bp, int k, double& dtc, double& ddtc, double& eta)
{
    dtc = ddtc = eta = 0.0;
    if (!bp.on || k <= 0) return;
    double pm2 = bp.psi1, pm1 = bp.psi2;   // psi_{j-2}, psi_{j-1} as j advances
    double P = 0.0, Pkm1 = 0.0, psik = bp.psi1;
    for (int j = 1; j <= k; ++j) {
        double pj;
        if (j == 1) pj = bp.psi1;
        else if (j == 2) pj = bp.psi2;
        else { pj = pm2 - 2.0 / (double)(bp.T - j); pm2 = pm1; pm1 = pj; }
        if (j == k) { Pkm1 = P; psik = pj; }
        P += pj;
    }
    dtc = 0.5 * (P - k * bp.psi1);
    ddtc = 0.5 * ((k - 1) * psik - Pkm1);
    eta = 0.5 * (k * log(2.0 / (double)(bp.T - 1)) + P);
}

// ------------------------------------------------------------------------------------------------
// Result handling shared by the engines.  Returns whether the value may enter the reducer.
// ------------------------------------------------------------------------------------------------
template <typename F>
__device__ __forceinline__ bool store_result(const EvalArgs& a, bool reduce, int d, int64_t pos, int k,
                                             const FactorOut<F>& f, double sumlogd, double dtc, double ddtc,
                                             double eta, bool fp64_pass, double& omega)
{
    const int64_t o = (int64_t)d * a.B + pos;
    uint8_t flag = 0;
    F TC, DTC;
    const bool finite = isfinite(f.ld) && isfinite(f.sa);
    bool bad = !f.ok || !finite;
    bool queued = false;
    if (!fp64_pass && a.precision == THOI_FP32_REFINE) {
        const bool need = bad || !(f.vmax <= (F)a.vif_tau);
        // wave-aggregated append to the refine queue
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
                queued = true;
            }
        }
        bad = false;  // the FP32 values stay until the FP64 pass overwrites them
    }
    if (bad) {
        TC = DTC = (F)__builtin_nan("");
        flag |= THOI_NPLET_NOT_PD;
    } else {
        TC = F(-0.5) * f.ld + (F)dtc;
        DTC = F(0.5) * (f.ld + f.sa) + (F)ddtc;
    }
    const F OM = TC - DTC, SI = TC + DTC;
    omega = (double)OM;
    if (!reduce) {
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
    }
    if (a.flags) a.flags[o] = flag;
    return !bad && !queued;
}

// ------------------------------------------------------------------------------------------------
// Lane engine
// ------------------------------------------------------------------------------------------------
// internal selection mode: every n-plet of orders kmin..kmax of each of several datasets
constexpr int kSelMulti = 3;

struct LaneCtx {
    int d;
    int64_t local;       // index of the n-plet inside its piece
    int64_t first, pos0;
    int64_t gbase;       // multi-dataset: index inside the dataset of the piece's first n-plet
    int N;
    int kb;
    bool reduce;
    double dtc, ddtc, eta;
};

// Next combination of the same order in lexicographic order (the caller knows it exists):
// the last index that can still grow grows by one and the indices after it follow it.
template <int K>
__device__ __forceinline__ void next_lex(int (&c)[K > 0 ? K : 1], int N)
{
    if constexpr (K > 0) {
        int piv = 0;
#pragma unroll
        for (int i = 0; i < K; ++i) piv = c[i] < N - K + i ? i : piv;
        c[0] += piv == 0 ? 1 : 0;
#pragma unroll
        for (int i = 1; i < K; ++i) c[i] = i == piv ? c[i] + 1 : (i > piv ? c[i - 1] + 1 : c[i]);
    }
}

// Factor one n-plet of order K and store (or hand back) its measures.
template <typename F, int K>
__device__ __forceinline__ bool lane_eval(const EvalArgs& a, const LaneCtx& cx, const F* sR, const double* sLogd,
                                          const int (&c)[K > 0 ? K : 1], int64_t pos, double& omega)
{
    const FactorOut<F> f = lane_factor<F, K>(c, sR, cx.N);
    double sumlogd = 0.0;
    if (a.write_H) {
#pragma unroll
        for (int i = 0; i < K; ++i) sumlogd += sLogd[c[i]];
    }
    return store_result<F>(a, cx.reduce, cx.d, pos, K, f, sumlogd, cx.dtc, cx.ddtc, cx.eta, false, omega);
}

// S consecutive n-plets of one lane, starting at cx.local inside the piece (cnt n-plets).  In
// lexicographic modes the first is unranked and the others follow by next_lex, so the unranking
// is paid once per S n-plets.
template <typename F, int K, int MODE, int S>
__device__ __forceinline__ void lane_task(const EvalArgs& a, const LaneCtx& cx, const F* sR, const double* sLogd,
                                          const uint64_t* sBin, int64_t cnt, double (&omega)[S],
                                          int64_t (&gidx)[S], bool (&valid)[S])
{
    int c[K > 0 ? K : 1];
    if constexpr (MODE == THOI_SEL_RANGE || MODE == kSelMulti) {
        unrank_lex<K>((uint64_t)(cx.first + cx.local), cx.N, sBin, cx.kb, c);
#pragma unroll
        for (int j = 0; j < S; ++j) {
            if (j > 0) {
                if (cx.local + j >= cnt) break;
                next_lex<K>(c, cx.N);
            }
            const int64_t pos = cx.pos0 + cx.local + j;
            gidx[j] = MODE == THOI_SEL_RANGE ? a.g_begin + pos : cx.gbase + cx.local + j;
            valid[j] = lane_eval<F, K>(a, cx, sR, sLogd, c, pos, omega[j]);
        }
    } else {
        static_assert(S == 1, "index lists are evaluated one n-plet per lane");
        const int64_t pos = a.perm[cx.first + cx.local];
        gidx[0] = pos;
        if constexpr (MODE == THOI_SEL_LIST) {
            const int32_t* row = a.idx + pos * a.kmax_list;
#pragma unroll
            for (int i = 0; i < K; ++i) c[i] = row[i];
        } else {
            uint64_t m = a.mask[pos];
#pragma unroll
            for (int i = 0; i < K; ++i) { c[i] = __builtin_ctzll(m); m &= m - 1; }
        }
        valid[0] = lane_eval<F, K>(a, cx, sR, sLogd, c, pos, omega[0]);
    }
}

template <typename F, int K, int KHI, int MODE, int S>
__device__ __forceinline__ void dispatch_k(int k, const EvalArgs& a, const LaneCtx& cx, const F* sR,
                                           const double* sLogd, const uint64_t* sBin, int64_t cnt,
                                           double (&omega)[S], int64_t (&gidx)[S], bool (&valid)[S])
{
    if (k == K) lane_task<F, K, MODE, S>(a, cx, sR, sLogd, sBin, cnt, omega, gidx, valid);
    else if constexpr (K < KHI) dispatch_k<F, K + 1, KHI, MODE, S>(k, a, cx, sR, sLogd, sBin, cnt, omega, gidx, valid);
}

// n-plets per lane in the lane engine: two in RANGE mode where the class leaves register room
// for the index set carried from one to the next, else one.
template <typename F>
__host__ __device__ constexpr int lane_per_thread(int khi, int mode)
{
    return mode == THOI_SEL_RANGE && khi <= (sizeof(F) == 4 ? 16 : 10) ? 2 : 1;
}

// LDS: sR [N*N] F | sIsd [N] f64 | sLogd [N] f64 | sBin [N*kb] u64 | (reduce) RedLds
__host__ __device__ inline size_t lane_stage_bytes(int N, int kb, int fsize)
{
    size_t off = (size_t)N * N * fsize;
    off = (off + 15) / 16 * 16;
    off += (size_t)N * 8 * 2;
    off += (size_t)N * kb * 8;
    return (off + 15) / 16 * 16;
}


// ------------------------------------------------------------------------------------------------
// Wave engine kernel: orders above the register classes (one wavefront per n-plet, FP64).
// grid (workgroups, D), block 64.
// LDS: sR [N*N] f64 | sIsd [N] | sLogd [N] | sBin [N*64] (RANGE) | sM [64*ks] | sInv [64] |
//      cidx [64] int | res_v [64] | res_g [64] | res_ok [64] | (reduce) RedLds
// ------------------------------------------------------------------------------------------------
__host__ __device__ inline size_t wave_stage_bytes(int N, int kmax, bool with_bin)
{
    const int ks = kmax + 1;
    size_t off = (size_t)N * N * 8 + (size_t)N * 16 + (with_bin ? (size_t)N * 64 * 8 : 0);
    off += (size_t)64 * ks * 8 + 64 * 8 + 64 * 4;
    off += 64 * 8 + 64 * 8 + 64 * 4;
    return (off + 15) / 16 * 16;
}


// ------------------------------------------------------------------------------------------------
// Final merge of the streaming reduction: one workgroup per (order k, dataset d).
// ------------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_red_final(RedArgs red, WsHeader* hdr)
{
    __shared__ RedFinal S;
    const int k = blockIdx.x, d = blockIdx.y;
    const int K = red.topk;
    if (K <= 0) return;
    double* tv = red.top_val + ((int64_t)d * (red.kmax + 1) + k) * 2 * K;
    int64_t* tg = red.top_g + ((int64_t)d * (red.kmax + 1) + k) * 2 * K;
    for (int i = threadIdx.x; i < 2 * K; i += blockDim.x) {
        const int l = i / K, j = i % K;
        const bool has = tg[i] >= 0;
        S.key[l][0][j] = has ? red_list_key(l, tv[i]) : kKeyEmpty;
        S.g[l][0][j] = has ? tg[i] : kGEmpty;
    }
    if (threadIdx.x == 0) { S.cur[0] = S.cur[1] = 0; }
    __syncthreads();
    // Segments in batches of one per thread: each thread tests its segment's two list heads
    // against the current K-th entries, the candidates are compacted, and only those are merged
    // (tested again against the threshold as it tightens).  After the first batches almost no
    // segment beats the running lists, so a batch costs one round of parallel loads.
    __shared__ uint32_t cand[2][256];
    __shared__ int ncand[2];
    const uint32_t nseg = min(hdr->seg_next, red.seg_cap);
    for (uint32_t s0 = 0; s0 < nseg; s0 += blockDim.x) {
        if (threadIdx.x < 2) ncand[threadIdx.x] = 0;
        __syncthreads();
        const uint32_t s = s0 + threadIdx.x;
        if (s < nseg) {
            const SegHdr h = red.seg_hdr[s];
            if (h.d == d && h.k == k) {
                for (int l = 0; l < 2; ++l) {
                    const int64_t e = ((int64_t)s * 2 + l) * K;
                    const int c = S.cur[l];
                    if (red_less(red.seg_key[e], red.seg_g[e], S.key[l][c][K - 1], S.g[l][c][K - 1]))
                        cand[l][atomicAdd(&ncand[l], 1)] = s;
                }
            }
        }
        __syncthreads();
        for (int l = 0; l < 2; ++l) {
            const int nc = ncand[l];
            for (int j = 0; j < nc; ++j) {
                const int64_t e = ((int64_t)cand[l][j] * 2 + l) * K;
                const uint64_t* bk = red.seg_key + e;
                const int64_t* bg = red.seg_g + e;
                const int c = S.cur[l];
                if (!red_less(bk[0], bg[0], S.key[l][c][K - 1], S.g[l][c][K - 1])) continue;   // uniform
                red_final_merge(S, l, K, bk, bg, K);
            }
        }
        __syncthreads();                         // every thread has read ncand before the reset
    }
    const uint32_t nlate = min(hdr->late_next, red.late_cap);
    for (uint32_t b0 = 0; b0 < nlate; b0 += blockDim.x) {
        const uint32_t i = b0 + threadIdx.x;
        bool mine = false;
        double v = 0.0;
        int64_t g = 0;
        if (i < nlate) {
            const LateEntry e = red.late[i];
            mine = e.d == d && e.k == k;
            v = e.v;
            g = e.g;
        }
        red_final_offer(S, 0, K, mine, red_list_key(0, v), g);
        red_final_offer(S, 1, K, mine, red_list_key(1, v), g);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 2 * K; i += blockDim.x) {
        const int l = i / K, j = i % K;
        const uint64_t key = S.key[l][S.cur[l]][j];
        const bool has = key != kKeyEmpty;
        tv[i] = has ? red_list_val(l, key) : __builtin_nan("");
        tg[i] = has ? S.g[l][S.cur[l]][j] : -1;
    }
}

__global__ void k_red_init(double* top_val, int64_t* top_g, int64_t ntop, unsigned long long* hist, int64_t nhist)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < ntop; i += stride) {
        top_val[i] = __builtin_nan("");
        top_g[i] = -1;
    }
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nhist; i += stride) hist[i] = 0;
}

// ------------------------------------------------------------------------------------------------
// LIST / MASK: order bucketing on the device.
// ------------------------------------------------------------------------------------------------
__global__ void k_ws_clear(uint32_t* p, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = 0;
}

// Zero the first `bytes` of a workspace: the header and the admission bounds that follow it.
inline void ws_clear(void* base, size_t bytes, hipStream_t s)
{
    const int64_t n = (int64_t)(bytes / 4);
    int64_t g = (n + 1023) / 1024;
    g = g < 1 ? 1 : (g > 1024 ? 1024 : g);
    hipLaunchKernelGGL(k_ws_clear, dim3((unsigned)g), dim3(256), 0, s, reinterpret_cast<uint32_t*>(base), n);
}


// grid ceil(B/256): order of every row (THOI_MAX_K + 1 = invalid) and per-order counts.
template <int MODE>
__global__ __launch_bounds__(256) void k_list_classify(EvalArgs a, int reduce, int64_t Bn, uint8_t* __restrict__ korder,
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
            // the row's entries are read eight at a time, all loads of a batch in flight together:
            // strictly ascending ids in [0, N), then only -1 padding
            const int32_t* row = a.idx + b * a.kmax_list;
            int prev = -1;
            bool ended = false;
            for (int j0 = 0; j0 < a.kmax_list; j0 += 8) {
                int v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) v[u] = j0 + u < a.kmax_list ? row[j0 + u] : -1;
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    if (ended || v[u] < 0) {
                        ok = ok && v[u] == -1;
                        ended = true;
                    } else {
                        ok = ok && v[u] > prev && v[u] < a.N;
                        prev = v[u];
                        ++k;
                    }
                }
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
                if (!reduce && a.out) {
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

// per order: lane-engine class, and 0 (lane engine), 1 (pair engine) or 2 (wave engine)
struct ClassMap { int8_t cls[kListOrders]; int8_t wave[kListOrders]; };

// 1 workgroup: per-order base in perm, and first workgroup of each order inside its launch.
__global__ void k_list_scan(const unsigned long long* __restrict__ cnt, int64_t* __restrict__ base,
                            int64_t* __restrict__ blk0, unsigned long long* __restrict__ cursor, ClassMap cm,
                            int64_t per_lane_blk, int64_t per_pair_blk, int64_t per_wave_blk)
{
    // One thread per order loads its count and class, and divides the count into workgroups (a
    // 64-bit division is a long instruction sequence); one thread then scans in LDS only (byte reads
    // of the class map from the kernel arguments, or global stores, in that serial loop made every
    // iteration wait for memory); all threads write the results.
    __shared__ int64_t c[kListOrders], nb[kListOrders], sb[kListOrders], sk[kListOrders];
    __shared__ int64_t ct[16];
    __shared__ int8_t wv[kListOrders], cl[kListOrders];
    for (int k = threadIdx.x; k < kListOrders; k += blockDim.x) {
        const int64_t ck = (int64_t)cnt[k];
        const int w = cm.wave[k];
        c[k] = ck;
        wv[k] = (int8_t)w;
        cl[k] = cm.cls[k];
        const int64_t per = w == 2 ? per_wave_blk : (w == 1 ? per_pair_blk : per_lane_blk);
        nb[k] = k > THOI_MAX_K ? 0 : (ck + per - 1) / per;
        cursor[k] = 0;
    }
    for (int k = threadIdx.x; k < 16; k += blockDim.x) ct[k] = 0;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t b = 0;
        int64_t wp = 0, ww = 0;
        for (int k = 0; k < kListOrders; ++k) {
            sb[k] = b;
            b += c[k];
            if (k > THOI_MAX_K) { sk[k] = 0; continue; }
            if (wv[k] == 1) {
                sk[k] = wp;
                wp += nb[k];
            } else if (wv[k] == 2) {
                sk[k] = ww;
                ww += nb[k];
            } else {
                sk[k] = ct[cl[k]];
                ct[cl[k]] += nb[k];
            }
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < kListOrders; k += blockDim.x) {
        base[k] = sb[k];
        blk0[k] = sk[k];
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

int64_t sel_B(const thoi_nplets* sel) { return sel->mode == THOI_SEL_RANGE ? sel->g_count : sel->B; }

int sel_kmax(const thoi_nplets* sel, int N)
{
    if (sel->mode == THOI_SEL_RANGE) return sel->kmax;
    if (sel->mode == THOI_SEL_LIST) return sel->kmax_list < THOI_MAX_K ? sel->kmax_list : THOI_MAX_K;
    return N < THOI_MAX_K ? N : THOI_MAX_K;
}

template <typename F>
const KClass* classes_for(int& n)
{
    if constexpr (sizeof(F) == 4) { n = (int)(sizeof(kF32Classes) / sizeof(KClass)); return kF32Classes; }
    n = (int)(sizeof(kF64Classes) / sizeof(KClass));
    return kF64Classes;
}

int lane_max_for(int precision) { return precision == THOI_FP64 ? kF64LaneMax : kF32LaneMax; }

template <typename F>
int class_of(int k)
{
    int n = 0;
    const KClass* cls = classes_for<F>(n);
    int c = 0;
    while (c < n - 1 && k > cls[c].hi) ++c;
    return c;
}


size_t red_lds(const RedArgs& r) { return r.active ? red_lds_bytes(r.topk, r.bins) : 0; }
size_t red_lds(const thoi_reduce* r) { return r ? red_lds_bytes(r->topk, r->hist_bins) : 0; }

}  // namespace
}  // namespace thoi
