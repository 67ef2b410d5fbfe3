// Gaussian-copula transform on gfx950 (Supplementary, "Estimation of entropy via Gaussian
// copulas", Eq. gaussian_copula_covariance_estimator): every variable of every dataset is
// replaced by Phi^{-1}(r / (T+1)), r its 1-based ordinal rank, equal values ranked by sample
// index.
//
// Design: a column is cut into chunks of kChunk samples.  One workgroup of kChunk threads sorts
// one chunk of (orderable key, sample index) pairs with a bitonic network held in registers:
// partners inside a wavefront are exchanged by cross-lane shuffles, larger distances through LDS.  With a single chunk the sorted position is the rank.  Otherwise the
// sorted chunks go to the workspace and a merge workgroup per chunk adds, for each of its
// elements, the number of entries before it in every chunk of the column (its own included).
// Every kernel issues its global loads in batches, all in flight together: at these sizes the
// cost is round trips to memory, not bandwidth.
#include "thoi_internal.hpp"

namespace thoi {
namespace {

constexpr int kChunk = 1024;                       // samples per sorted chunk
constexpr int kSortThreads = 1024;
constexpr int kSortReg = kChunk / kSortThreads;    // elements per thread in the sort (one)
constexpr int kMergeThreads = 1024;
constexpr int kMergeReg = kChunk / kMergeThreads;  // elements per thread in the merge
constexpr int kMergeStage = 16;                    // chunks staged in LDS at a time (128 KB of values)

// Monotone map of a double onto uint64 (total order; -0.0 is folded onto +0.0).
__device__ __forceinline__ uint64_t order_key(double x)
{
    if (x == 0.0) x = 0.0;
    uint64_t u = (uint64_t)__double_as_longlong(x);
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

// Phi^{-1}(r/(T+1)); the upper half uses the exact integer complement, so score(r) = -score(T+1-r).
// One call per score (lanes of a wave would otherwise run both inlined copies).
__device__ __forceinline__ double normal_score(int64_t r, int64_t T)
{
    const int64_t den = T + 1;
    const bool lower = 2 * r <= den;
    const double z = normcdfinv((double)(lower ? r : den - r) / (double)den);
    return lower ? z : -z;
}

template <typename ZT>
__device__ __forceinline__ void store_z(void* Z, int64_t off, double z)
{
    static_cast<ZT*>(Z)[off] = (ZT)z;
}

__device__ __forceinline__ bool pair_less(uint64_t ka, uint32_t ia, uint64_t kb, uint32_t ib)
{
    return ka < kb || (ka == kb && ia < ib);
}

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int m)
{
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, m);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), m);
    return ((uint64_t)hi << 32) | lo;
}

// One stage (block size SIZE, partner distance S) of the bitonic network over the kChunk elements
// of a workgroup, element i = kSortReg * tid + e.  Partners at distance below kSortReg sit in the
// same thread; up to a wavefront's span they are exchanged by cross-lane shuffles; beyond it through
// LDS.
template <int SIZE, int S>
__device__ __forceinline__ void bitonic_stage(uint64_t (&k)[kSortReg], uint32_t (&x)[kSortReg], int tid,
                                              uint64_t* skey, uint32_t* sidx)
{
    if constexpr (S < kSortReg) {
#pragma unroll
        for (int e = 0; e < kSortReg; ++e) {
            if ((e & S) == 0) {
                const bool asc = (((tid * kSortReg) | e) & SIZE) == 0;
                const bool swap = pair_less(k[e | S], x[e | S], k[e], x[e]) == asc;
                const uint64_t ka = k[e], kb = k[e | S];
                const uint32_t ia = x[e], ib = x[e | S];
                k[e] = swap ? kb : ka; k[e | S] = swap ? ka : kb;
                x[e] = swap ? ib : ia; x[e | S] = swap ? ia : ib;
            }
        }
    } else {
        constexpr int m = S / kSortReg;
        uint64_t pk[kSortReg];
        uint32_t px[kSortReg];
        if constexpr (m < 64) {
#pragma unroll
            for (int e = 0; e < kSortReg; ++e) {
                pk[e] = shfl_xor_u64(k[e], m);
                px[e] = (uint32_t)__shfl_xor((int)x[e], m);
            }
        } else {
            __syncthreads();                       // earlier readers of the exchange buffer are done
#pragma unroll
            for (int e = 0; e < kSortReg; ++e) {
                skey[tid * kSortReg + e] = k[e];
                sidx[tid * kSortReg + e] = x[e];
            }
            __syncthreads();
#pragma unroll
            for (int e = 0; e < kSortReg; ++e) {
                pk[e] = skey[(tid ^ m) * kSortReg + e];
                px[e] = sidx[(tid ^ m) * kSortReg + e];
            }
        }
        const bool lower = (tid & m) == 0;
#pragma unroll
        for (int e = 0; e < kSortReg; ++e) {
            const bool asc = (((tid * kSortReg) | e) & SIZE) == 0;
            // the lower element of the pair keeps the smaller one when ascending
            const bool keep = pair_less(k[e], x[e], pk[e], px[e]) == (lower == asc);
            k[e] = keep ? k[e] : pk[e];
            x[e] = keep ? x[e] : px[e];
        }
    }
    if constexpr (S > 1) bitonic_stage<SIZE, S / 2>(k, x, tid, skey, sidx);
}

template <int SIZE>
__device__ __forceinline__ void bitonic_sort(uint64_t (&k)[kSortReg], uint32_t (&x)[kSortReg], int tid,
                                             uint64_t* skey, uint32_t* sidx)
{
    bitonic_stage<SIZE, SIZE / 2>(k, x, tid, skey, sidx);
    if constexpr (SIZE < kChunk) bitonic_sort<SIZE * 2>(k, x, tid, skey, sidx);
}

// grid (nchunks, N, D), block kSortThreads: sorts chunk q of column (d, c).
template <typename ZT>
__global__ __launch_bounds__(kSortThreads) void k_copula_sort(const double* __restrict__ X, int64_t T, int64_t N,
                                                              void* __restrict__ Z, uint64_t* __restrict__ wkey,
                                                              uint32_t* __restrict__ widx,
                                                              int32_t* __restrict__ nanflag, WsHeader* hdr)
{
    __shared__ uint64_t skey[kChunk];
    __shared__ uint32_t sidx[kChunk];
    const int tid = threadIdx.x;
    const int64_t q = blockIdx.x, c = blockIdx.y, d = blockIdx.z;
    const int64_t nchunks = gridDim.x;
    const int64_t t0 = q * kChunk;
    const int n = (int)min<int64_t>(kChunk, T - t0);

    // load: register e of thread j takes sample t0 + kSortThreads e + j (consecutive threads read
    // consecutive rows); all loads are issued before the first use
    const double* Xd = X + d * T * N;
    double v[kSortReg];
#pragma unroll
    for (int e = 0; e < kSortReg; ++e) {
        const int i = kSortThreads * e + tid;
        v[e] = i < n ? Xd[(t0 + i) * N + c] : 0.0;
    }
    uint64_t k[kSortReg];
    uint32_t x[kSortReg];
    int has_nan = 0;
#pragma unroll
    for (int e = 0; e < kSortReg; ++e) {
        const int i = kSortThreads * e + tid;
        const bool in = i < n;
        has_nan |= in && isnan(v[e]);
        k[e] = in ? order_key(v[e]) : ~0ull;
        x[e] = in ? (uint32_t)(t0 + i) : 0xffffffffu;
    }
    const bool bad = __syncthreads_or(has_nan) != 0;
    bitonic_sort<2>(k, x, tid, skey, sidx);

    if (nchunks == 1) {
        if (bad && tid == 0) raise_status(hdr, THOI_EINVAL_DATA);
#pragma unroll
        for (int e = 0; e < kSortReg; ++e) {
            const int p = tid * kSortReg + e;
            if (p < n) store_z<ZT>(Z, (d * T + x[e]) * N + c, bad ? __builtin_nan("") : normal_score(p + 1, T));
        }
    } else {
        // the merge raises the status, after this kernel: clear the header here
        if (q == 0 && c == 0 && d == 0 && tid < (int)(kWsHeader / 4)) reinterpret_cast<int32_t*>(hdr)[tid] = 0;
        const int64_t base = ((d * N + c) * nchunks + q) * (int64_t)kChunk + tid * kSortReg;
#pragma unroll
        for (int e = 0; e < kSortReg; ++e) {
            wkey[base + e] = k[e];      // padding slots too: the merge searches whole chunks
            widx[base + e] = x[e];
        }
        if (tid == 0) nanflag[(d * N + c) * nchunks + q] = bad ? 1 : 0;   // every chunk writes its own flag
    }
}

// grid (nchunks, N*D), block kMergeThreads: the rank of element j of sorted chunk q of column (d, c)
// is its position in chunk q plus, for every other chunk o, the number of entries of o before it.
// Chunks hold contiguous ranges of samples, so an entry of o with an equal value comes before it
// exactly when o < q: the count is a search on the values alone (no sample indices in LDS).
// Chunks are staged kMergeStage at a time in LDS (all loads of a stage in flight together) and
// every element does a branchless fixed-step search in every staged chunk; the searches are
// independent, so a thread keeps many LDS reads in flight.
template <typename ZT>
__global__ __launch_bounds__(kMergeThreads) void k_copula_merge(int64_t T, int64_t N, int nchunks,
                                                                void* __restrict__ Z,
                                                                const uint64_t* __restrict__ wkey,
                                                                const uint32_t* __restrict__ widx,
                                                                const int32_t* __restrict__ nanflag, WsHeader* hdr)
{
    __shared__ uint64_t okey[kMergeStage][kChunk];
    const int tid = threadIdx.x;
    // XCD-aware order: workgroups are dealt round-robin to the 8 XCDs; give consecutive work items
    // (the chunks of one column, which read the same staged chunks) to the same XCD
    const int64_t G = (int64_t)gridDim.x * gridDim.y, b = blockIdx.x + (int64_t)gridDim.x * blockIdx.y;
    const int64_t xcd = b % 8, q8 = G / 8, r8 = G % 8;
    const int64_t w = xcd * q8 + (xcd < r8 ? xcd : r8) + b / 8;
    const int q = (int)(w % nchunks);
    const int64_t cd = w / nchunks;
    const int64_t c = cd % N, d = cd / N;
    const int64_t col = (d * N + c) * nchunks;
    const int nq = (int)min<int64_t>(kChunk, T - (int64_t)q * kChunk);
    // the flags, the thread's own entries and the first stage's chunks are loaded together
    int f = 0;
    for (int o = tid; o < nchunks; o += kMergeThreads) f |= nanflag[col + o];
    bool bad = false;

    const int p0 = tid * kMergeReg;
    uint64_t mk[kMergeReg];
    uint32_t mi[kMergeReg];
    uint32_t rank[kMergeReg];
#pragma unroll
    for (int e = 0; e < kMergeReg; ++e) {
        mk[e] = wkey[(col + q) * (int64_t)kChunk + p0 + e];
        mi[e] = widx[(col + q) * (int64_t)kChunk + p0 + e];
        rank[e] = p0 + e;                                  // entries of its own chunk before it
    }
    for (int o0 = 0; o0 < nchunks; o0 += kMergeStage) {
        // stage chunks o0 .. o0+kMergeStage-1 other than q; slots past the last chunk and chunk q
        // itself are neither loaded nor searched (uniform branches)
        uint64_t lk[kMergeStage][kChunk / kMergeThreads];
#pragma unroll
        for (int s = 0; s < kMergeStage; ++s) {
            if (o0 + s < nchunks && o0 + s != q) {
                const int64_t src = (col + o0 + s) * (int64_t)kChunk;
#pragma unroll
                for (int e = 0; e < kChunk / kMergeThreads; ++e) lk[s][e] = wkey[src + e * kMergeThreads + tid];
            }
        }
        if (o0 == 0) bad = __syncthreads_or(f) != 0;     // uniform
        else __syncthreads();                      // the previous stage's searches are done
#pragma unroll
        for (int s = 0; s < kMergeStage; ++s) {
            if (o0 + s < nchunks && o0 + s != q) {
#pragma unroll
                for (int e = 0; e < kChunk / kMergeThreads; ++e) okey[s][e * kMergeThreads + tid] = lk[s][e];
            }
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < kMergeStage; ++s) {
            if (o0 + s >= nchunks || o0 + s == q) continue;
            const bool le = o0 + s < q;           // equal values of an earlier chunk come first
#pragma unroll
            for (int e = 0; e < kMergeReg; ++e) {
                // count of entries before x (v < x, or v <= x for an earlier chunk: v < x + 1; a
                // real key is below ~0, and the padding slots' ranks are never stored): binary
                // digits from the top, then the last entry
                const uint64_t xs = le ? mk[e] + 1 : mk[e];
                int pos = 0;
#pragma unroll
                for (int b = kChunk / 2; b >= 1; b >>= 1) pos += okey[s][pos + b - 1] < xs ? b : 0;
                pos += okey[s][pos] < xs ? 1 : 0;
                rank[e] += pos;
            }
        }
    }
    if (bad && q == 0 && tid == 0) raise_status(hdr, THOI_EINVAL_DATA);
#pragma unroll
    for (int e = 0; e < kMergeReg; ++e) {
        if (p0 + e < nq) {
            const double z = bad ? __builtin_nan("") : normal_score((int64_t)rank[e] + 1, T);
            store_z<ZT>(Z, (d * T + (int64_t)mi[e]) * N + c, z);
        }
    }
}

__global__ void k_zero_i32(int32_t* p, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

struct CopulaWs {
    size_t key_off, idx_off, nan_off, total;
};

CopulaWs copula_layout(int64_t D, int64_t T, int64_t N)
{
    CopulaWs w{};
    const int64_t nchunks = (T + kChunk - 1) / kChunk;
    size_t off = kWsHeader;
    if (nchunks > 1) {
        const size_t slots = (size_t)D * N * nchunks * kChunk;
        w.key_off = off; off = align_up(off + slots * 8, 256);
        w.idx_off = off; off = align_up(off + slots * 4, 256);
        w.nan_off = off; off = align_up(off + (size_t)D * N * nchunks * 4, 256);
    }
    w.total = off;
    return w;
}

}  // namespace

size_t copulize_ws_bytes(int64_t D, int64_t T, int64_t N) { return copula_layout(D, T, N).total; }

thoi_status launch_copulize(const double* X, int64_t D, int64_t T, int64_t N, int32_t z_dtype, void* Z, void* ws,
                            hipStream_t s)
{
    const CopulaWs w = copula_layout(D, T, N);
    char* base = static_cast<char*>(ws);
    WsHeader* hdr = reinterpret_cast<WsHeader*>(base);
    const int64_t nchunks = (T + kChunk - 1) / kChunk;
    uint64_t* wkey = nchunks > 1 ? reinterpret_cast<uint64_t*>(base + w.key_off) : nullptr;
    uint32_t* widx = nchunks > 1 ? reinterpret_cast<uint32_t*>(base + w.idx_off) : nullptr;
    int32_t* nanf = nchunks > 1 ? reinterpret_cast<int32_t*>(base + w.nan_off) : nullptr;

    // the header starts at zero: a fill kernel where the sort itself raises the status (one chunk),
    // else the sort clears it and the merge raises (no memset node, so the call can be captured)
    if (nchunks <= 1 || D * N == 0)
        hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, s, reinterpret_cast<int32_t*>(hdr), (int64_t)(kWsHeader / 4));
    if (D * N == 0 || T == 0) return hip_status(hipGetLastError());

    dim3 g1((unsigned)nchunks, (unsigned)N, (unsigned)D);
    if (z_dtype == THOI_DTYPE_F64)
        hipLaunchKernelGGL(k_copula_sort<double>, g1, dim3(kSortThreads), 0, s, X, T, N, Z, wkey, widx, nanf, hdr);
    else
        hipLaunchKernelGGL(k_copula_sort<float>, g1, dim3(kSortThreads), 0, s, X, T, N, Z, wkey, widx, nanf, hdr);
    if (nchunks > 1) {
        dim3 g2((unsigned)nchunks, (unsigned)(N * D));
        if (z_dtype == THOI_DTYPE_F64)
            hipLaunchKernelGGL(k_copula_merge<double>, g2, dim3(kMergeThreads), 0, s, T, N, (int)nchunks, Z, wkey, widx,
                               nanf, hdr);
        else
            hipLaunchKernelGGL(k_copula_merge<float>, g2, dim3(kMergeThreads), 0, s, T, N, (int)nchunks, Z, wkey, widx,
                               nanf, hdr);
    }
    return hip_status(hipGetLastError());
}

}  // namespace thoi
