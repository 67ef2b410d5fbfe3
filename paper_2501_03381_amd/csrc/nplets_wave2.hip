// Pair engine: FP64 evaluation of n-plets whose order is above the register classes (up to 32),
// two n-plets per wavefront.
//
// Each half-wave (32 lanes) factors one n-plet; lane i keeps row i of the sub-matrix in registers
// (32 doubles, indexed by compile-time constants only: every loop below is unrolled to order 32
// and guarded by the runtime order, which is the same for the whole wavefront).  Right-looking
// Cholesky: at step j the lanes i >= j publish a_ij in LDS, every lane reads the pivot and the
// column, scales its entry and updates its row.  W = L^-1 by forward substitution, one row per
// step: lane t publishes row t of W in LDS, the later rows accumulate L_it W_t, and every lane j
// adds W_tj^2 to the squared norm of column j, which is a_j = (R_S^-1)_jj.  log det and
// sum log a_j are half-wave sums, max a_j a half-wave maximum.  The measures follow as in the
// lane engine (TC = -ld/2, DTC = (ld + sum log a_j)/2, Omega, S; Methods, entropy terms of the
// Gaussian copula).  Only the lanes of one wavefront exchange data through LDS, so a wavefront
// needs no workgroup barrier: LDS operations of one wavefront complete in issue order, and a
// wavefront-scope fence keeps the compiler from reordering them.
#include "nplets_wave2.hpp"
#include "pair_factor.hpp"

namespace thoi {
static_assert(kPairThreads <= 64 * kRedWaves, "the reducer keeps lists for at most kRedWaves wavefronts");
namespace {

// Lexicographic unranking of rank r among the k-subsets of {0..N-1} (one lane), binomials from the
// compile-time table.
__device__ __forceinline__ void pair_unrank(uint64_t r, int N, int k, int* __restrict__ c)
{
    int x = 0;
    for (int i = 0; i < k; ++i) {
        const int m = k - 1 - i;
        while (x < N) {
            const uint64_t b = kPascal.v[N - 1 - x][m];
            if (r < b) break;
            r -= b;
            ++x;
        }
        c[i] = x++;
    }
}

// LDS: sR [N*N] f64 | sIsd [N] | sLogd [N] | col [8 halves][2][32] f64 | wrow [8][2][32] f64 |
//      cidx [8][32] int | (reduce) res_v [256] f64 | res_g [256] i64 | res_ok [256] int | RedLds
__host__ __device__ inline size_t w2_stage_bytes(int N, bool reduce)
{
    size_t off = (size_t)N * N * 8 + (size_t)N * 16;
    off += 2 * kPairHalves * 2 * (size_t)kW2Max * 8 + kPairHalves * (size_t)kW2Max * 4;
    if (reduce) off += (size_t)kPairThreads * (8 + 8 + 4);
    return (off + 15) / 16 * 16;
}

// grid (workgroups, D), block kPairThreads.  A workgroup takes a.wave_tile n-plets of one order k
// in chunks of up to kPairThreads; in a chunk each half-wave evaluates a run of consecutive
// n-plets (lexicographic successors in RANGE mode, so only the first of a run is unranked).  In
// reduce mode the chunk's results go to the workgroup's reducer together.
template <int MODE, bool RED>
__global__ __launch_bounds__(kPairThreads, 4) void k_eval_pair(EvalArgs a, PieceTable tab, RedArgs red, int klo, int kmax)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double sbias[3];
    const int N = a.N;
    const int d = blockIdx.y;
    const int64_t blk = blockIdx.x;
    const int wt = a.wave_tile;
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
    double* sR = reinterpret_cast<double*>(smem);
    double* sIsd = sR + N * N;
    double* sLogd = sIsd + N;
    double* scol = sLogd + N;
    double* swrow = scol + kPairHalves * 2 * kW2Max;
    int* scidx = reinterpret_cast<int*>(swrow + kPairHalves * 2 * kW2Max);
    double* res_v = reinterpret_cast<double*>(scidx + kPairHalves * kW2Max);
    int64_t* res_g = reinterpret_cast<int64_t*>(res_v + kPairThreads);
    int* res_ok = reinterpret_cast<int*>(res_g + kPairThreads);
    RedLds S = red_view(smem + w2_stage_bytes(N, RED), red.topk, red.bins);
    if (threadIdx.x == 0) bias_for(a.bias, k, sbias[0], sbias[1], sbias[2]);
    stage_corr<double>(a.Sigma + (int64_t)d * N * N, N, sR, sIsd, sLogd);
    if constexpr (RED) red_begin(S, red, d, k);
    __syncthreads();

    const int q = threadIdx.x >> 5, i = threadIdx.x & 31, h = q & 1;
    int* ch = scidx + q * kW2Max;
    double* col = scol + q * 2 * kW2Max;
    double* wrow = swrow + q * 2 * kW2Max;
    const int64_t l0 = (blk - blk0) * wt;
    const int64_t l1 = l0 + wt < cnt ? l0 + wt : cnt;
    for (int64_t c0 = l0; c0 < l1; c0 += kPairThreads) {
        const int64_t c1 = c0 + kPairThreads < l1 ? c0 + kPairThreads : l1;
        const int run = (int)((c1 - c0 + kPairHalves - 1) / kPairHalves);
        const int64_t r0 = c0 + (int64_t)q * run;
        const int64_t r1 = r0 + run < c1 ? r0 + run : c1;
        // the wavefront's two halves step together; an exhausted half factors a dummy
        const int64_t o_r0 = c0 + (int64_t)(q ^ 1) * run;
        const int64_t o_r1 = o_r0 + run < c1 ? o_r0 + run : c1;
        const int n_me = (int)(r1 > r0 ? r1 - r0 : 0), n_other = (int)(o_r1 > o_r0 ? o_r1 - o_r0 : 0);
        const int steps = n_me > n_other ? n_me : n_other;
        int ci = i;                              // lane i's variable (RANGE: kept across the run)
        if constexpr (MODE == THOI_SEL_RANGE) {
            if (r0 < r1) {
                if (i == 0) pair_unrank((uint64_t)(first + r0), N, k, ch);
                wave_sync();
                ci = i < k ? ch[i] : i;
            }
        }
        for (int it = 0; it < steps; ++it) {
            const int64_t my = r0 + it;
            const bool act = my < r1;
            int64_t pos = 0, gidx = 0;
            if (act) {
                if constexpr (MODE == THOI_SEL_RANGE) {
                    pos = pos0 + my;
                    gidx = a.g_begin + pos;
                    if (it > 0) {
                        // lexicographic successor: the last position that can grow grows, the later
                        // ones follow it
                        const bool can = i < k && ci < N - k + i;
                        const uint32_t bits = (uint32_t)(__ballot(can) >> (32 * h));
                        const int p = 31 - __builtin_clz(bits | 1u);
                        const int cp = __shfl(ci, p, 32);
                        if (i >= p && i < k) ci = cp + 1 + (i - p);
                    }
                } else if constexpr (MODE == THOI_SEL_LIST) {
                    pos = a.perm[first + my];
                    gidx = pos;
                    if (i < k) ci = a.idx[pos * a.kmax_list + i];
                } else {
                    pos = a.perm[first + my];
                    gidx = pos;
                    uint64_t m = a.mask[pos];
                    // lane i takes the (i+1)-th set bit
                    for (int t = 0; t < i && m; ++t) m &= m - 1;
                    if (i < k) ci = __builtin_ctzll(m);
                }
            } else {
                ci = i;                          // variables 0..k-1; the result is discarded
            }
            if (i < k) ch[i] = ci;
            wave_sync();
            const FactorOut<double> f = pair_factor<false>(sR, N, ch, k, k, col, wrow);
            double sumlogd = 0.0;
            if (a.write_H) sumlogd = half_sum(i < k ? sLogd[ci] : 0.0);
            if (i == 0 && act) {
                double om = 0.0;
                // FP64 already: never queued for refinement
                EvalArgs b = a;
                if (b.precision == THOI_FP32_REFINE) b.precision = THOI_FP64;
                const bool ok = store_result<double>(b, RED, d, pos, k, f, sumlogd, sbias[0], sbias[1], sbias[2], true, om);
                if constexpr (RED) {
                    const int slot = (int)(my - c0);
                    res_v[slot] = om;
                    res_g[slot] = gidx;
                    res_ok[slot] = ok;
                }
            }
            wave_sync();
        }
        if constexpr (RED) {
            __syncthreads();
            const int t = threadIdx.x;
            const bool have = c0 + t < c1;
            red_push(S, red, k, have && res_ok[t], have ? res_v[t] : 0.0, have ? res_g[t] : 0);
            __syncthreads();
        }
    }
    if constexpr (RED) red_end(S, red, a.hdr, d, k);
}

// ------------------------------------------------------------------------------------------------
// Refinement: FP64 re-evaluation of the n-plets queued by the FP32 lane engine.
// ------------------------------------------------------------------------------------------------
constexpr int kRefineThreads = 256;
// Largest order refined one per lane (a register triangle of order 18 would spill); orders above
// go to the pair factoriser.  Lanes factor at order 8 (orders up to 8), 14 (9..14) or 16 (15, 16).
constexpr int kRefineLaneMax = 16;
constexpr int kRefineStageMaxN = 64;   // largest N whose correlation matrix is staged in LDS

// Order of queued n-plet `pos` and, in RANGE mode, its rank inside that order.
template <int MODE>
__device__ __forceinline__ int queued_order(const EvalArgs& a, const RangeOrders& ro, int64_t pos, uint64_t& rank)
{
    int k = 0;
    rank = 0;
    if constexpr (MODE == THOI_SEL_RANGE) {
        const int64_t g = ro.g_begin + pos;
        k = ro.kmin;
        while (k < ro.kmax && g >= ro.ostart[k + 1]) ++k;
        rank = (uint64_t)(g - ro.ostart[k]);
    } else if constexpr (MODE == THOI_SEL_LIST) {
        const int32_t* row = a.idx + pos * a.kmax_list;
        while (k < a.kmax_list && row[k] >= 0) ++k;
    } else {
        k = __builtin_popcountll(a.mask[pos]);
    }
    return k;
}

// Store the FP64 result of queued entry o (dataset d, position pos) over its FP32 one.
__device__ __forceinline__ void refine_store(const EvalArgs& a, const RangeOrders& ro, const RedArgs& red, int mode,
                                             int64_t o, int d, int64_t pos, int k, const FactorOut<double>& f,
                                             double sumlogd)
{
    EvalArgs b = a;
    b.precision = THOI_FP64;
    b.flags = nullptr;
    const bool reduce = red.active != 0;
    double dtc, ddtc, eta, om = 0.0;
    bias_for(a.bias, k, dtc, ddtc, eta);
    const bool ok = store_result<double>(b, reduce, d, pos, k, f, sumlogd, dtc, ddtc, eta, true, om);
    if (a.flags) a.flags[o] = (uint8_t)(THOI_NPLET_REFINED | (ok ? 0 : THOI_NPLET_NOT_PD));
    if (reduce && ok) red_late(red, a.hdr, d, k, mode == THOI_SEL_RANGE ? ro.g_begin + pos : pos, om);
}

// One lane, runtime order k <= KP: the n-plet's entries are gathered from Sigma of its own
// dataset, scaled to correlations, and factored in registers as the order-KP matrix
// diag(R_S, I).  The identity block adds pivots 1 and inverse-diagonal entries 1, so log det,
// sum log a_j and max a_j (>= 1 for a correlation matrix) are those of R_S, and the operations on
// R_S's own entries are the same as at order k.  One code body per KP serves every order (code
// per order would not fit the instruction cache when the wavefronts of a CU refine different
// orders).
template <int MODE, int KP, bool STAGED>
__device__ __forceinline__ void refine_lane(const EvalArgs& a, const RangeOrders& ro, const RedArgs& red, int64_t o,
                                            int d, int64_t pos, int k, uint64_t rank, const uint64_t* sBin,
                                            const double* sR, const double* sLogd)
{
    const int N = a.N;
    uint64_t mask = 0;
    int c[KP];
    if constexpr (MODE == THOI_SEL_RANGE) {
        // lexicographic unranking into a bit mask: take x while the rank is below C(N-1-x, m)
        int m = k - 1;
        for (int x = 0; x < N && m >= 0; ++x) {
            const uint64_t b = sBin[(N - 1 - x) * kW2Max + m];
            if (rank < b) { mask |= 1ull << x; --m; }
            else rank -= b;
        }
    } else if constexpr (MODE == THOI_SEL_MASK) {
        mask = a.mask[pos];
    }
    if constexpr (MODE == THOI_SEL_LIST) {
        const int32_t* row = a.idx + pos * a.kmax_list;
#pragma unroll
        for (int i = 0; i < KP; ++i) c[i] = i < k ? row[i] : 0;
    } else {
#pragma unroll
        for (int i = 0; i < KP; ++i) {
            c[i] = i < k ? __builtin_ctzll(mask) : 0;
            mask &= mask - 1;
        }
    }
    double sumlogd = 0.0;
    FactorOut<double> f;
    if constexpr (STAGED) {
        // the dataset's correlation matrix and log variances are staged in LDS
        if (a.write_H) {
#pragma unroll
            for (int i = 0; i < KP; ++i)
                if (i < k) sumlogd += sLogd[c[i]];
        }
        f = lane_factor_by<double, KP>([&](int i, int j) { return i < k ? sR[c[i] * N + c[j]] : 0.0; });
    } else {
        const double* Sg = a.Sigma + (int64_t)d * N * N;
        double sd[KP];
#pragma unroll
        for (int i = 0; i < KP; ++i) {
            sd[i] = 1.0;
            if (i < k) {
                const double di = Sg[(int64_t)c[i] * N + c[i]];
                sd[i] = di > 0.0 ? 1.0 / sqrt(di) : __builtin_nan("");
                if (a.write_H) sumlogd += log(di);
            }
        }
        f = lane_factor_by<double, KP>(
            [&](int i, int j) { return i < k ? Sg[(int64_t)c[i] * N + c[j]] * sd[i] * sd[j] : 0.0; });
    }
    refine_store(a, ro, red, MODE, o, d, pos, k, f, sumlogd);
}

// grid (G), block kRefineThreads.  Round j gives thread t of workgroup b the queue entry
// j G T + t G + b (T threads per workgroup): consecutive entries (appended together, usually of
// one order) go to different workgroups.  The workgroup sorts its entries in LDS by the padded
// order that factors them, so that each wavefront mostly runs one code body; entries of order
// above kRefineLaneMax are then dealt round-robin to the wavefronts, two per wavefront at a time.
// The queue is complete (the class kernels ran before this one).
template <int MODE>
__global__ __launch_bounds__(kRefineThreads) void k_refine(EvalArgs a, RangeOrders ro, RedArgs red)
{
    constexpr int kWaves = kRefineThreads / 64;
    __shared__ uint64_t sBin[64 * kW2Max];   // C(n, m), n < N, m < 32 (RANGE)
    __shared__ int64_t sOst[THOI_MAX_K + 2];
    __shared__ double scol[kPairHalves * 2 * kW2Max];
    __shared__ double swrow[kPairHalves * 2 * kW2Max];
    __shared__ int scidx[kPairHalves * kW2Max];
    __shared__ int64_t eo[kRefineThreads];    // sorted entries: queue value, rank, order
    __shared__ uint64_t erank[kRefineThreads];
    __shared__ int ek[kRefineThreads];
    __shared__ int ccount[4], cbase[4];
    __shared__ int dmin, dmax;
    extern __shared__ __align__(16) unsigned char smem[];   // correlation matrix [N*N] | 1/sd [N] | log var [N]
    double* sR = reinterpret_cast<double*>(smem);
    double* sIsd = sR + a.N * a.N;
    double* sLogd = sIsd + a.N;
    const int N = a.N;
    const int64_t n = (int64_t)min(a.hdr->refine_count, a.refine_cap);
    const int64_t G = gridDim.x;
    if ((int64_t)blockIdx.x >= n) return;     // uniform in the workgroup: no entry
    if constexpr (MODE == THOI_SEL_RANGE) {
        stage_binomials(N, kW2Max, sBin);
        for (int t = threadIdx.x; t <= ro.kmax + 1 && t < THOI_MAX_K + 2; t += blockDim.x) sOst[t] = ro.ostart[t];
    }
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int h = lane >> 5, i = lane & 31;
    int* ch = scidx + (2 * w + h) * kW2Max;
    double* col = scol + (2 * w + h) * 2 * kW2Max;
    double* wrow = swrow + (2 * w + h) * 2 * kW2Max;
    for (int64_t j0 = 0; j0 < n; j0 += G * kRefineThreads) {
        if (threadIdx.x < 4) ccount[threadIdx.x] = 0;
        if (threadIdx.x == 0) { dmin = INT32_MAX; dmax = -1; }
        __syncthreads();
        // load, classify (0: padded 8, 1: 14, 2: kRefineLaneMax, 3: pair), count
        const int64_t q = j0 + (int64_t)threadIdx.x * G + blockIdx.x;
        int64_t o = -1;
        int k = 0, cls = 0;
        uint64_t rank = 0;
        if (q < n) {
            o = a.refine_list[q];
            const int d = (int)(o / a.B);
            const int64_t pos = o - (int64_t)d * a.B;
            if constexpr (MODE == THOI_SEL_RANGE) {
                const int64_t g = ro.g_begin + pos;
                k = ro.kmin;
                while (k < ro.kmax && g >= sOst[k + 1]) ++k;
                rank = (uint64_t)(g - sOst[k]);
            } else {
                k = queued_order<MODE>(a, ro, pos, rank);
            }
            cls = k <= 8 ? 0 : (k <= 14 ? 1 : (k <= kRefineLaneMax ? 2 : 3));
            atomicMin(&dmin, d);
            atomicMax(&dmax, d);
        }
        const int slot = q < n ? atomicAdd(&ccount[cls], 1) : -1;
        __syncthreads();
        // entries of one dataset (always so for a single dataset) and N <= 64: gather from LDS
        const bool staged = N <= kRefineStageMaxN && dmin == dmax;
        if (staged) stage_corr<double>(a.Sigma + (int64_t)dmin * N * N, N, sR, sIsd, sLogd);
        if (threadIdx.x == 0) {
            cbase[0] = 0;
            cbase[1] = ccount[0];
            cbase[2] = cbase[1] + ccount[1];
            cbase[3] = cbase[2] + ccount[2];
        }
        __syncthreads();
        if (slot >= 0) {
            const int e = cbase[cls] + slot;
            eo[e] = o;
            erank[e] = rank;
            ek[e] = k;
        }
        __syncthreads();
        const int nlane = cbase[3], npair = ccount[3];
        // lane path: sorted entry threadIdx.x
        if ((int)threadIdx.x < nlane) {
            const int64_t oo = eo[threadIdx.x];
            const int d = (int)(oo / a.B);
            const int64_t pos = oo - (int64_t)d * a.B;
            const int kk = ek[threadIdx.x];
            const uint64_t rk = erank[threadIdx.x];
            if (!staged) refine_lane<MODE, kRefineLaneMax, false>(a, ro, red, oo, d, pos, kk, rk, sBin, sR, sLogd);
            else if (kk <= 8) refine_lane<MODE, 8, true>(a, ro, red, oo, d, pos, kk, rk, sBin, sR, sLogd);
            else if (kk <= 14) refine_lane<MODE, 14, true>(a, ro, red, oo, d, pos, kk, rk, sBin, sR, sLogd);
            else refine_lane<MODE, kRefineLaneMax, true>(a, ro, red, oo, d, pos, kk, rk, sBin, sR, sLogd);
        }
        // pair path: wavefront w takes pairs w, w + kWaves, ... of the sorted high-order entries
        for (int p0 = 2 * w; p0 < npair; p0 += 2 * kWaves) {
            const int e = p0 + h;
            const bool hact = e < npair;
            int64_t ho = 0, hpos = 0;
            int hd = 0, kh = 0;
            uint64_t hrank = 0;
            if (hact) {
                ho = eo[nlane + e];
                hd = (int)(ho / a.B);
                hpos = ho - (int64_t)hd * a.B;
                kh = ek[nlane + e];
                hrank = erank[nlane + e];
                if constexpr (MODE == THOI_SEL_RANGE) {
                    if (i == 0) unrank_lex_rt(hrank, N, kh, sBin, kW2Max, ch);
                } else if constexpr (MODE == THOI_SEL_LIST) {
                    if (i < kh) ch[i] = a.idx[hpos * a.kmax_list + i];
                } else {
                    uint64_t m = a.mask[hpos];
                    for (int t = 0; t < i && m; ++t) m &= m - 1;
                    if (i < kh) ch[i] = __builtin_ctzll(m);
                }
            }
            wave_sync();
            // every shuffle runs with the whole wavefront active (an inactive source lane reads 0)
            const int k0 = __shfl(kh, 0), k1 = __shfl(kh, 32);
            const double* Sg = a.Sigma + (int64_t)hd * N * N;
            double sumlogd = 0.0;
            FactorOut<double> f;
            if (staged) {
                f = pair_factor<false>(sR, N, ch, k0 > k1 ? k0 : k1, kh, col, wrow);
                if (a.write_H) sumlogd = half_sum(i < kh ? sLogd[ch[i]] : 0.0);
            } else {
                f = pair_factor<true>(Sg, N, ch, k0 > k1 ? k0 : k1, kh, col, wrow);
                if (a.write_H) sumlogd = half_sum(i < kh ? log(Sg[(int64_t)ch[i] * N + ch[i]]) : 0.0);
            }
            if (i == 0 && hact) refine_store(a, ro, red, MODE, ho, hd, hpos, kh, f, sumlogd);
            wave_sync();
        }
        __syncthreads();                         // the sorted arrays are rewritten next round
    }
}

}  // namespace

void refine_launch(int mode, const EvalArgs& a, const RangeOrders& ro, const RedArgs& red, hipStream_t s)
{
    // one workgroup per CU at most (the kernel runs one wave per SIMD); larger queues take more
    // rounds inside the kernel, and an empty queue dispatches a single round of workgroups
    const int64_t need = ((int64_t)a.refine_cap + kRefineThreads - 1) / kRefineThreads;
    const unsigned G = (unsigned)(need < 256 ? (need > 0 ? need : 1) : 256);
    const size_t lds = a.N <= kRefineStageMaxN ? ((size_t)a.N * a.N + 2 * (size_t)a.N) * sizeof(double) : 0;
    if (mode == THOI_SEL_RANGE) hipLaunchKernelGGL(k_refine<THOI_SEL_RANGE>, dim3(G), dim3(kRefineThreads), lds, s, a, ro, red);
    else if (mode == THOI_SEL_LIST) hipLaunchKernelGGL(k_refine<THOI_SEL_LIST>, dim3(G), dim3(kRefineThreads), lds, s, a, ro, red);
    else hipLaunchKernelGGL(k_refine<THOI_SEL_MASK>, dim3(G), dim3(kRefineThreads), lds, s, a, ro, red);
}

size_t pair_lds_bytes(int N, size_t red_bytes)
{
    return w2_stage_bytes(N, red_bytes > 0) + red_bytes;
}

void pair_launch(int mode, bool reduce, const EvalArgs& a, const PieceTable& t, const RedArgs& red, int klo, int kmax,
                 int64_t nblk, hipStream_t s)
{
    const size_t lds = pair_lds_bytes(a.N, red_lds(red));
    const dim3 grid((unsigned)nblk, (unsigned)a.D);
    if (mode == THOI_SEL_RANGE) {
        if (reduce) hipLaunchKernelGGL((k_eval_pair<THOI_SEL_RANGE, true>), grid, dim3(kPairThreads), lds, s, a, t, red, klo, kmax);
        else hipLaunchKernelGGL((k_eval_pair<THOI_SEL_RANGE, false>), grid, dim3(kPairThreads), lds, s, a, t, red, klo, kmax);
    } else if (mode == THOI_SEL_LIST) {
        if (reduce) hipLaunchKernelGGL((k_eval_pair<THOI_SEL_LIST, true>), grid, dim3(kPairThreads), lds, s, a, t, red, klo, kmax);
        else hipLaunchKernelGGL((k_eval_pair<THOI_SEL_LIST, false>), grid, dim3(kPairThreads), lds, s, a, t, red, klo, kmax);
    } else {
        if (reduce) hipLaunchKernelGGL((k_eval_pair<THOI_SEL_MASK, true>), grid, dim3(kPairThreads), lds, s, a, t, red, klo, kmax);
        else hipLaunchKernelGGL((k_eval_pair<THOI_SEL_MASK, false>), grid, dim3(kPairThreads), lds, s, a, t, red, klo, kmax);
    }
}

}  // namespace thoi
