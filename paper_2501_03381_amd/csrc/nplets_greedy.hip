// Greedy growth run on the device (Methods, "Heuristics", "Greedy Algorithm"): from the kappa
// best n-plets of one order, every solution is extended by every variable it lacks, all
// candidates of the next order are evaluated, and the kappa best are kept; the orders follow one
// another with no host round trip (two launches per order).  The objective is one measure (TC,
// DTC, O-information or S-information) in one dataset, or its mean or paired effect size over D
// datasets (Discussion: functions of the measures optimised across datasets).
//
// Candidate (p, v) is solution p extended by variable v.  A candidate reached from several parents
// is evaluated once, from the first of them (the lowest p whose solution is a subset of it).  One
// 64-lane workgroup per candidate and dataset factors its correlation block (FP64), taking the
// sums of the logs in variable order, so candidates that differ only by which independent
// variable they hold get bit-identical values.  One workgroup then forms each candidate's
// objective, sorts the candidates of the order by it and, among equal values, by the n-plet in
// lexicographic order (the smaller first), and keeps the first kappa.
#include "thoi_internal.hpp"
#include "nplets_common.hpp"
#include "objective_common.hpp"
#include "pair_factor.hpp"

namespace thoi {
namespace {

constexpr int kSelThreads = 1024;
constexpr int kSelMax = 4096;           // candidates of one order that the selection sorts in LDS

struct Mask {
    uint64_t w[2];
};

__device__ __forceinline__ int popc(const Mask& m) { return __popcll(m.w[0]) + __popcll(m.w[1]); }

__device__ __forceinline__ bool has(const Mask& m, int v) { return (m.w[v >> 6] >> (v & 63)) & 1ull; }

__device__ __forceinline__ bool subset(const Mask& a, const Mask& b)
{
    return (a.w[0] & ~b.w[0]) == 0 && (a.w[1] & ~b.w[1]) == 0;
}

// a before b in lexicographic order of the sorted index tuples (equal orders): the lowest variable
// in which they differ belongs to a
__device__ __forceinline__ bool lex_less(const Mask& a, const Mask& b)
{
    const uint64_t x0 = a.w[0] ^ b.w[0];
    if (x0) return (a.w[0] >> __builtin_ctzll(x0)) & 1ull;
    const uint64_t x1 = a.w[1] ^ b.w[1];
    if (x1) return (a.w[1] >> __builtin_ctzll(x1)) & 1ull;
    return false;
}

// total order on doubles as uint64 (-0.0 folded onto +0.0)
__device__ __forceinline__ uint64_t okey(double x)
{
    if (x == 0.0) x = 0.0;
    const uint64_t u = (uint64_t)__double_as_longlong(x);
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

struct GreedyArgs {
    const double* Sigma;    // [D][N][N]
    int D;
    int N;
    int kappa;
    int measure;            // 0 TC, 1 DTC, 2 Omega, 3 S
    int kind;               // THOI_OBJ_MEAN or THOI_OBJ_PAIRED_EFFECT over the D datasets
    double sign;            // +1: keep the largest objective, -1: the smallest
    Mask* sols;             // [steps + 1][kappa]; slot 0 holds the first order's solutions
    double* vals;           // [steps + 1][kappa]
    int32_t* count;         // [steps + 1]
    Mask* cmask;            // [kappa * N] candidates of the current step
    double* meas;           // [D][kappa * N] their measure (NaN: not a candidate or not positive definite)
};

// grid (kappa * N, D), block 64: candidate (p, v) = blockIdx.x / N, % N of step s (order k + 1)
// in dataset blockIdx.y.  Dynamic LDS: the factorisation block, kc rows of stride kc + 1 for the
// step's order kc (sized per step, so that short orders leave room for more wavefronts per CU).
__global__ __launch_bounds__(64) void k_greedy_eval(GreedyArgs g, int s, int kc)
{
    extern __shared__ double sM[];
    const int ks = kc + 1;
    __shared__ double sInv[64], sIsd[64], sSeq[128];
    __shared__ int cidx[64];
    const int N = g.N;
    const int p = blockIdx.x / N, v = blockIdx.x % N;
    const int lane = threadIdx.x;
    const int d = blockIdx.y;
    const int64_t slot = blockIdx.x;
    double* meas = g.meas + (int64_t)d * g.kappa * N;
    const double* Sig = g.Sigma + (int64_t)d * N * N;
    const int cnt = g.count[s];
    const Mask* sol = g.sols + (int64_t)s * g.kappa;
    // uniform in the workgroup: a parent that exists, a variable it lacks, and no earlier parent
    // reaching the same n-plet
    bool use = p < cnt && !has(sol[p], v);
    Mask C{};
    if (use) {
        C = sol[p];
        C.w[v >> 6] |= 1ull << (v & 63);
        for (int q = lane; q < p; q += 64) use = use && !subset(sol[q], C);
        use = __all(use);                      // __all over the wavefront: every earlier parent checked
        use = use && popc(C) <= kc;            // the step's order by construction; the block holds no more
    }
    if (!use) {
        if (lane == 0) meas[slot] = __builtin_nan("");
        return;
    }
    int k = popc(C);
    k = k < 64 ? k : 64;
    int ci = 0;
    if (lane < k) {
        // lane j takes the (j+1)-th member
        Mask m = C;
        int n = lane;
        ci = 0;
        for (int h = 0; h < 2; ++h) {
            const int c = __popcll(m.w[h]);
            if (n < c) {
                uint64_t x = m.w[h];
                for (int i = 0; i < n; ++i) x &= x - 1;
                ci = 64 * h + __builtin_ctzll(x);
                break;
            }
            n -= c;
        }
        cidx[lane] = ci;
        const double dj = Sig[(int64_t)ci * N + ci];
        sIsd[lane] = dj > 0.0 ? 1.0 / sqrt(dj) : __builtin_nan("");
    }
    __syncthreads();
    if (lane < k) gather_row(Sig + (int64_t)ci * N, cidx, sIsd, lane, sM + lane * ks);
    __syncthreads();
    const FactorOut<double> f = wave_factor_core(k, sM, ks, sInv, sSeq);
    if (lane == 0) {
        const bool ok = f.ok && isfinite(f.ld) && isfinite(f.sa);
        const double TC = -0.5 * f.ld, DTC = 0.5 * (f.ld + f.sa);
        const double m = g.measure == 0 ? TC : g.measure == 1 ? DTC : g.measure == 2 ? TC - DTC : TC + DTC;
        if (d == 0) g.cmask[slot] = C;
        meas[slot] = ok ? m : __builtin_nan("");
    }
}

// grid (ceil(kappa * N / 2), D), block 64: two candidate slots per wavefront (half-wave h takes
// slot 2 blockIdx.x + h), factored with the rows in registers; for steps whose order is at most
// kW2Max.  The same candidates, measures and sums in variable order as k_greedy_eval.
__global__ __launch_bounds__(64) void k_greedy_eval_pair(GreedyArgs g, int s)
{
    __shared__ double scol[2 * 2 * kW2Max], swrow[2 * 2 * kW2Max];
    __shared__ int sch[2 * kW2Max];
    const int N = g.N;
    const int lane = threadIdx.x, h = lane >> 5, i = lane & 31;
    const int64_t slot = 2 * (int64_t)blockIdx.x + h;
    const int64_t nslot = (int64_t)g.kappa * N;
    const int d = blockIdx.y;
    double* meas = g.meas + (int64_t)d * nslot;
    const double* Sig = g.Sigma + (int64_t)d * N * N;
    const int cnt = g.count[s];
    const Mask* sol = g.sols + (int64_t)s * g.kappa;
    const int p = slot < nslot ? (int)(slot / N) : 0, v = slot < nslot ? (int)(slot % N) : 0;
    // uniform in the half-wave: a slot that exists, a parent that exists, a variable it lacks, and
    // no earlier parent reaching the same n-plet
    bool use = slot < nslot && p < cnt && !has(sol[p], v);
    Mask C{};
    if (use) {
        C = sol[p];
        C.w[v >> 6] |= 1ull << (v & 63);
    }
    bool lane_ok = true;
    if (use)
        for (int q = i; q < p; q += 32) lane_ok = lane_ok && !subset(sol[q], C);
    const uint64_t bad = __ballot(!lane_ok);               // whole wavefront active
    use = use && ((bad >> (32 * h)) & 0xffffffffull) == 0;
    int kh = use ? popc(C) : 0;
    kh = kh < kW2Max ? kh : kW2Max;
    int* ch = sch + h * kW2Max;
    if (i < kh) {
        Mask m = C;
        int n = i, ci = 0;
        for (int hw = 0; hw < 2; ++hw) {
            const int c = __popcll(m.w[hw]);
            if (n < c) {
                uint64_t x = m.w[hw];
                for (int t = 0; t < n; ++t) x &= x - 1;
                ci = 64 * hw + __builtin_ctzll(x);
                break;
            }
            n -= c;
        }
        ch[i] = ci;
    }
    wave_sync();
    const int k0 = __shfl(kh, 0), k1 = __shfl(kh, 32);
    const FactorOut<double> f = pair_factor<true, true>(Sig, N, ch, k0 > k1 ? k0 : k1, kh, scol + h * 2 * kW2Max,
                                                        swrow + h * 2 * kW2Max);
    if (i == 0 && slot < nslot) {
        if (!use) {
            meas[slot] = __builtin_nan("");
        } else {
            const bool ok = f.ok && isfinite(f.ld) && isfinite(f.sa);
            const double TC = -0.5 * f.ld, DTC = 0.5 * (f.ld + f.sa);
            const double m = g.measure == 0 ? TC : g.measure == 1 ? DTC : g.measure == 2 ? TC - DTC : TC + DTC;
            if (d == 0) g.cmask[slot] = C;
            meas[slot] = ok ? m : __builtin_nan("");
        }
    }
}

constexpr int kSelChunk = 128;         // entries one wavefront sorts on its own (two per lane)

// Entry (kx, ix) goes before entry (ky, iy): the smaller key, or equal valid keys and the
// lexicographically smaller n-plet (valid slots hold distinct n-plets, so the order is strict there).
__device__ __forceinline__ bool sel_before(uint64_t kx, int ix, uint64_t ky, int iy, const Mask* msk)
{
    if (kx != ky) return kx < ky;
    return ky != ~0ull && lex_less(msk[ix], msk[iy]);
}

// grid 1, block kSelThreads: the objective of each of the ncand = kappa * N slots of step s, then
// order them and keep the kappa best distinct n-plets as step s + 1.
//
// Bitonic sort in LDS of the P >= ncand (a power of two) keys and slot indices.  Thread
// 1024 j + 64 w + r of a stage with stride <= 64 exchanges entries of the 128-entry chunk
// 2048 j + 128 w only, so between two such stages wavefront w waits for itself alone; a stage that
// follows or precedes one with a wider stride (or the fill) waits for the block.  When kappa <= 128
// only the best 128 entries are needed: once every chunk is sorted (chunk c ascending when c is
// even, else descending), pairs of chunks are merged keeping the lower half only.  Entry-wise
// minimum of an ascending and a descending chunk is the 128 smallest of the two as a bitonic
// sequence; one wavefront sorts it (strides 64..1) ascending or descending as the next merge needs,
// and the number of chunks halves, until chunk 0 holds the best 128 in order.
__global__ __launch_bounds__(kSelThreads) void k_greedy_select(GreedyArgs g, int s)
{
    __shared__ uint64_t key[kSelMax];
    __shared__ int idx[kSelMax];
    __shared__ Mask msk[kSelMax];           // the n-plets by slot, read for the lexicographic ties
    const int ncand = g.kappa * g.N;
    int P = 1;
    while (P < ncand) P <<= 1;
    for (int i = threadIdx.x; i < P; i += kSelThreads) {
        const double o = i < ncand ? objective_of<double>(g.meas, g.D, ncand, i, g.kind) : __builtin_nan("");
        // ascending key = better first; invalid slots last
        key[i] = isnan(o) ? ~0ull : (g.sign > 0.0 ? ~okey(o) : okey(o));
        idx[i] = i < ncand ? i : -1;
        msk[i] = isnan(o) ? Mask{{0ull, 0ull}} : g.cmask[i];
    }
    const bool topk = g.kappa <= kSelChunk && P > kSelChunk;
    const int top = topk ? kSelChunk : P;
    bool wide = true;
    for (int size = 2; size <= top; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            const bool w = stride > 64;
            if (w || wide) __syncthreads();
            else wave_sync();
            wide = w;
            for (int i = threadIdx.x; i < (P >> 1); i += kSelThreads) {
                const int lo = 2 * i - (i & (stride - 1)), hi = lo + stride;
                const bool asc = (lo & size) == 0;
                const uint64_t ka = key[lo], kb = key[hi];
                const int ia = idx[lo], ib = idx[hi];
                if (sel_before(kb, ib, ka, ia, msk) == asc) { key[lo] = kb; key[hi] = ka; idx[lo] = ib; idx[hi] = ia; }
            }
        }
    }
    if (topk) {
        // P / 128 <= 32 chunks; merge r pairs chunk 2^r w (ascending) with chunk 2^r w + 2^(r-1)
        // (descending) in wavefront w, for w below the number of chunks left
        const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
        const int nch = P / kSelChunk;
        for (int r = 1; (1 << r) <= nch; ++r) {
            __syncthreads();
            if (wv < (nch >> r)) {
                const int a = (wv << r) * kSelChunk, b = a + (1 << (r - 1)) * kSelChunk;
                const bool asc = (wv & 1) == 0;
                for (int j = ln; j < kSelChunk; j += 64) {
                    const uint64_t ka = key[a + j], kb = key[b + j];
                    const int ia = idx[a + j], ib = idx[b + j];
                    if (sel_before(kb, ib, ka, ia, msk)) { key[a + j] = kb; idx[a + j] = ib; }
                }
                for (int stride = 64; stride > 0; stride >>= 1) {
                    wave_sync();
                    const int lo = a + 2 * ln - (ln & (stride - 1)), hi = lo + stride;
                    const uint64_t ka = key[lo], kb = key[hi];
                    const int ia = idx[lo], ib = idx[hi];
                    if (sel_before(kb, ib, ka, ia, msk) == asc) {
                        key[lo] = kb; key[hi] = ka; idx[lo] = ib; idx[hi] = ia;
                    }
                }
            }
        }
    }
    __syncthreads();
    // the valid slots come first and are distinct n-plets: the first min(kappa, valid) are kept,
    // one thread each
    const int t = threadIdx.x;
    const int n = __syncthreads_count(t < g.kappa && t < P && key[t] != ~0ull);
    if (t < n) {
        const int i = idx[t];
        g.sols[(int64_t)(s + 1) * g.kappa + t] = msk[i];
        g.vals[(int64_t)(s + 1) * g.kappa + t] = objective_of<double>(g.meas, g.D, ncand, i, g.kind);
    }
    if (t == 0) g.count[s + 1] = n;
}

}  // namespace

size_t greedy_ws_bytes(int64_t D, int32_t N, int32_t kappa)
{
    return (size_t)kappa * N * (sizeof(Mask) + 8 * (size_t)D) + 256;
}

int greedy_select_max() { return kSelMax; }

thoi_status launch_greedy(const double* Sigma, int64_t D, int32_t N, int32_t k_first, int32_t kappa, int32_t steps,
                          int32_t measure, int32_t kind, int32_t maximize, uint64_t* sols, double* vals, int32_t* count,
                          void* ws, hipStream_t s)
{
    GreedyArgs g{};
    g.Sigma = Sigma;
    g.D = (int)D;
    g.N = N;
    g.kappa = kappa;
    g.measure = measure;
    g.kind = kind;
    g.sign = maximize ? 1.0 : -1.0;
    g.sols = reinterpret_cast<Mask*>(sols);
    g.vals = vals;
    g.count = count;
    char* base = static_cast<char*>(ws);
    g.cmask = reinterpret_cast<Mask*>(base);
    g.meas = reinterpret_cast<double*>(base + (size_t)kappa * N * sizeof(Mask));
    for (int32_t t = 0; t < steps; ++t) {
        // step t builds order k_first + t + 1
        if (k_first + t + 1 <= kW2Max)
            hipLaunchKernelGGL(k_greedy_eval_pair, dim3((unsigned)((kappa * N + 1) / 2), (unsigned)D), dim3(64), 0, s, g,
                               (int)t);
        else {
            const int kc = k_first + t + 1;
            const size_t lds = (size_t)kc * (size_t)(kc + 1) * sizeof(double);
            hipLaunchKernelGGL(k_greedy_eval, dim3((unsigned)(kappa * N), (unsigned)D), dim3(64), lds, s, g, (int)t, kc);
        }
        hipLaunchKernelGGL(k_greedy_select, dim3(1), dim3(kSelThreads), 0, s, g, (int)t);
    }
    return hip_status(hipGetLastError());
}

}  // namespace thoi
