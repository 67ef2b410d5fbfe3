// Gaussian-copula transform on gfx950 (Supplementary, "Estimation of entropy via Gaussian
// copulas", Eq. gaussian_copula_covariance_estimator): every variable of every dataset is
// replaced by Phi^{-1}(r / (T+1)), r its 1-based ordinal rank, equal values ranked by sample
// index.
//
// Design: a column is cut into chunks of kChunk samples.  One workgroup sorts one chunk of
// (orderable key, sample index) pairs with a bitonic network in LDS.  With a single chunk the
// sorted position is the rank.  Otherwise the sorted chunks go to the workspace and a merge
// workgroup per chunk ranks its elements against every other chunk of the column: the other
// chunk is staged in LDS and each thread, owning kPerThread consecutive sorted elements, does one
// binary search and walks forward for the rest (the positions are monotone).
#include "thoi_internal.hpp"

namespace thoi {
namespace {

constexpr int kChunk = 1024;          // samples per LDS sort
constexpr int kSortThreads = 256;
constexpr int kPerThread = kChunk / kSortThreads;

// Monotone map of a double onto uint64 (total order; -0.0 is folded onto +0.0).
__device__ __forceinline__ uint64_t order_key(double x)
{
    if (x == 0.0) x = 0.0;
    uint64_t u = (uint64_t)__double_as_longlong(x);
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

// Phi^{-1}(r/(T+1)); the upper half uses the exact integer complement, so score(r) = -score(T+1-r).
__device__ __forceinline__ double normal_score(int64_t r, int64_t T)
{
    const int64_t den = T + 1;
    if (2 * r <= den) return normcdfinv((double)r / (double)den);
    return -normcdfinv((double)(den - r) / (double)den);
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

// grid (nchunks, N, D), block kSortThreads.
template <typename ZT>
__global__ __launch_bounds__(kSortThreads) void k_copula_sort(const double* __restrict__ X, int64_t T, int64_t N,
                                                               void* __restrict__ Z, uint64_t* __restrict__ wkey,
                                                               uint32_t* __restrict__ widx,
                                                               int32_t* __restrict__ nanflag, WsHeader* hdr)
{
    __shared__ uint64_t skey[kChunk];
    __shared__ uint32_t sidx[kChunk];
    __shared__ int snan;

    const int64_t q = blockIdx.x, c = blockIdx.y, d = blockIdx.z;
    const int64_t nchunks = gridDim.x;
    const int64_t t0 = q * kChunk;
    const int n = (int)min<int64_t>(kChunk, T - t0);
    int P = 1;
    while (P < n) P <<= 1;
    if (threadIdx.x == 0) snan = 0;
    __syncthreads();

    const double* Xd = X + d * T * N;
    bool has_nan = false;
    for (int i = threadIdx.x; i < P; i += blockDim.x) {
        if (i < n) {
            const double x = Xd[(t0 + i) * N + c];
            has_nan |= isnan(x);
            skey[i] = order_key(x);
            sidx[i] = (uint32_t)(t0 + i);
        } else {
            skey[i] = ~0ull;
            sidx[i] = 0xffffffffu;
        }
    }
    if (has_nan) atomicOr(&snan, 1);

    for (int size = 2; size <= P; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            __syncthreads();
            for (int i = threadIdx.x; i < (P >> 1); i += blockDim.x) {
                const int lo = 2 * i - (i & (stride - 1));
                const int hi = lo + stride;
                const bool asc = (lo & size) == 0;
                const uint64_t ka = skey[lo], kb = skey[hi];
                const uint32_t ia = sidx[lo], ib = sidx[hi];
                if (pair_less(kb, ib, ka, ia) == asc) {
                    skey[lo] = kb; skey[hi] = ka;
                    sidx[lo] = ib; sidx[hi] = ia;
                }
            }
        }
    }
    __syncthreads();

    if (nchunks == 1) {
        const bool bad = snan != 0;
        if (bad && threadIdx.x == 0) raise_status(hdr, THOI_EINVAL_DATA);
        for (int p = threadIdx.x; p < n; p += blockDim.x) {
            const int64_t t = sidx[p];
            const double z = bad ? __builtin_nan("") : normal_score(p + 1, T);
            store_z<ZT>(Z, (d * T + t) * N + c, z);
        }
    } else {
        const int64_t base = ((d * N + c) * nchunks + q) * (int64_t)kChunk;
        for (int p = threadIdx.x; p < n; p += blockDim.x) {
            wkey[base + p] = skey[p];
            widx[base + p] = sidx[p];
        }
        if (threadIdx.x == 0) nanflag[(d * N + c) * nchunks + q] = snan;   // every chunk writes its own flag
    }
}

// grid (nchunks, N*D), block kSortThreads: ranks of sorted chunk q of column (d, c).
template <typename ZT>
__global__ __launch_bounds__(kSortThreads) void k_copula_merge(int64_t T, int64_t N, int nchunks, void* __restrict__ Z,
                                                               const uint64_t* __restrict__ wkey,
                                                               const uint32_t* __restrict__ widx,
                                                               const int32_t* __restrict__ nanflag, WsHeader* hdr)
{
    __shared__ uint64_t okey[kChunk];
    __shared__ uint32_t oidx[kChunk];
    __shared__ int sbad;
    const int q = blockIdx.x;
    const int64_t c = blockIdx.y % N, d = blockIdx.y / N;
    const int64_t col = (d * N + c) * nchunks;
    const int nq = (int)min<int64_t>(kChunk, T - (int64_t)q * kChunk);
    if (threadIdx.x == 0) {
        int bad = 0;
        for (int o = 0; o < nchunks; ++o) bad |= nanflag[col + o];
        sbad = bad;
        if (bad && q == 0) raise_status(hdr, THOI_EINVAL_DATA);
    }
    // this thread's elements: sorted positions p0 .. p0 + kPerThread - 1 of chunk q
    const int p0 = threadIdx.x * kPerThread;
    uint64_t mk[kPerThread];
    uint32_t mi[kPerThread];
    int64_t rank[kPerThread];
#pragma unroll
    for (int e = 0; e < kPerThread; ++e) {
        const int p = p0 + e;
        mk[e] = p < nq ? wkey[(col + q) * (int64_t)kChunk + p] : ~0ull;
        mi[e] = p < nq ? widx[(col + q) * (int64_t)kChunk + p] : 0xffffffffu;
        rank[e] = p;
    }
    for (int o = 0; o < nchunks; ++o) {
        if (o == q) continue;
        const int no = (int)min<int64_t>(kChunk, T - (int64_t)o * kChunk);
        __syncthreads();
        for (int i = threadIdx.x; i < no; i += blockDim.x) {
            okey[i] = wkey[(col + o) * (int64_t)kChunk + i];
            oidx[i] = widx[(col + o) * (int64_t)kChunk + i];
        }
        __syncthreads();
        // lower bound of the first element, then a forward walk for the others
        int lo = 0, hi = no;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (pair_less(okey[mid], oidx[mid], mk[0], mi[0])) lo = mid + 1; else hi = mid;
        }
#pragma unroll
        for (int e = 0; e < kPerThread; ++e) {
            while (lo < no && pair_less(okey[lo], oidx[lo], mk[e], mi[e])) ++lo;
            rank[e] += lo;
        }
    }
    __syncthreads();
    const bool bad = sbad != 0;
#pragma unroll
    for (int e = 0; e < kPerThread; ++e) {
        if (p0 + e < nq) {
            const double z = bad ? __builtin_nan("") : normal_score(rank[e] + 1, T);
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

    // the header starts at zero (a fill kernel, so the call can be graph-captured)
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
            hipLaunchKernelGGL(k_copula_merge<double>, g2, dim3(kSortThreads), 0, s, T, N, (int)nchunks, Z, wkey, widx,
                               nanf, hdr);
        else
            hipLaunchKernelGGL(k_copula_merge<float>, g2, dim3(kSortThreads), 0, s, T, N, (int)nchunks, Z, wkey, widx,
                               nanf, hdr);
    }
    return hip_status(hipGetLastError());
}

}  // namespace thoi
