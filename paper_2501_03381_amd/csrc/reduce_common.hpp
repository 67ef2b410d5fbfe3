// Streaming per-(dataset, order) reduction of Omega on gfx950: exact top-K (largest) and bottom-K
// (smallest) lists with (value, global index) ordering, and a histogram with under/overflow
// counts.  This replaces the paper's per-batch custom function aggregated on the fly (Figure 1A)
// so that exhaustive runs never store exponentially many results.
//
// Each workgroup covers n-plets of one (d, k) and keeps two running sorted lists in LDS.  Values
// that beat the current K-th entry are compacted, sorted (bitonic, small) and merged in (merge
// path).  At the end the workgroup writes its lists as one "segment" to the workspace and adds
// its LDS histogram to the global one.  A final kernel merges, per (d, k), the accumulated lists
// of earlier calls, every segment of this call, and the FP64-refined values (queued separately).
#pragma once

#include "thoi_internal.hpp"

namespace thoi {

constexpr int kRedMaxK = 256;
constexpr int kRedMaxBins = 4096;

struct SegHdr {
    int32_t d, k;
};

struct LateEntry {          // an FP64-refined value for the final merge
    int32_t d, k;
    int64_t g;
    double v;
};

struct RedArgs {
    int32_t active, topk, bins, kmax;
    double* top_val;                 // [D][kmax+1][2][topk]
    int64_t* top_g;
    unsigned long long* hist;        // [D][kmax+1][bins+2]
    uint64_t* seg_key;               // [seg_cap][2][topk]
    int64_t* seg_g;
    SegHdr* seg_hdr;                 // [seg_cap]
    uint32_t* seg_next;              // segment counter (in the workspace header)
    uint32_t seg_cap;
    LateEntry* late;                 // [late_cap]
    uint32_t* late_next;
    uint32_t late_cap;
    double lo[THOI_MAX_K + 1], hi[THOI_MAX_K + 1];
};

// The reducer's LDS, sized by the call's K and bin count: views into a workgroup's shared memory.
// Layout from a 16-byte aligned base: key [2 lists][2 buffers][K] u64 | g [2][2][K] i64 |
// candidates ck, cg [kRedCand] | hist [bins + 2] u32 | cur [2], nc.
constexpr int kRedCand = 256;        // candidates per offer: at most one per thread of a workgroup
struct RedLds {
    uint64_t* key;
    int64_t* g;
    uint64_t* ck;
    int64_t* cg;
    unsigned int* hist;
    int* cur;
    int* nc;
    int K;
    __device__ __forceinline__ uint64_t* keys(int l, int b) const { return key + (2 * l + b) * K; }
    __device__ __forceinline__ int64_t* gs(int l, int b) const { return g + (2 * l + b) * K; }
};

__host__ __device__ constexpr size_t red_lds_bytes(int K, int bins)
{
    const size_t lists = (size_t)4 * (K > 0 ? K : 1) * 16;
    const size_t b = lists + (size_t)kRedCand * 16 + (size_t)(bins + 2) * 4 + 16;
    return (b + 15) / 16 * 16;
}

__device__ __forceinline__ RedLds red_view(unsigned char* base, int K, int bins)
{
    RedLds S;
    const int Kc = K > 0 ? K : 1;
    S.K = Kc;
    S.key = reinterpret_cast<uint64_t*>(base);
    S.g = reinterpret_cast<int64_t*>(S.key + 4 * Kc);
    S.ck = reinterpret_cast<uint64_t*>(S.g + 4 * Kc);
    S.cg = reinterpret_cast<int64_t*>(S.ck + kRedCand);
    S.hist = reinterpret_cast<unsigned int*>(S.cg + kRedCand);
    S.cur = reinterpret_cast<int*>(S.hist + bins + 2);
    S.nc = S.cur + 2;
    return S;
}

// total order on doubles as uint64 (-0.0 folded onto +0.0)
__device__ __forceinline__ uint64_t red_okey(double x)
{
    if (x == 0.0) x = 0.0;
    const uint64_t u = (uint64_t)__double_as_longlong(x);
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}
__device__ __forceinline__ double red_unkey(uint64_t k)
{
    const uint64_t u = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
    return __longlong_as_double((long long)u);
}
__device__ __forceinline__ bool red_less(uint64_t ka, int64_t ga, uint64_t kb, int64_t gb)
{
    return ka < kb || (ka == kb && ga < gb);
}
constexpr uint64_t kKeyEmpty = ~0ull;
constexpr int64_t kGEmpty = INT64_MAX;

// list 0 keeps the largest Omega (key = ~okey), list 1 the smallest (key = okey)
__device__ __forceinline__ uint64_t red_list_key(int list, double v)
{
    return list == 0 ? ~red_okey(v) : red_okey(v);
}
__device__ __forceinline__ double red_list_val(int list, uint64_t key)
{
    return red_unkey(list == 0 ? ~key : key);
}

// Whole workgroup: empty lists and histogram.
__device__ __forceinline__ void red_begin(RedLds& S, int K, int bins)
{
    for (int i = threadIdx.x; i < 2 * 2 * K; i += blockDim.x) {
        S.key[i] = kKeyEmpty;
        S.g[i] = kGEmpty;
    }
    for (int i = threadIdx.x; i < bins + 2; i += blockDim.x) S.hist[i] = 0;
    if (threadIdx.x == 0) { S.cur[0] = S.cur[1] = 0; }
    __syncthreads();
}

// Whole workgroup: merge the sorted run (ck, cg)[0..nb) into list `l`, keeping K.
__device__ __forceinline__ void red_merge_sorted(RedLds& S, int l, int K, const uint64_t* bk, const int64_t* bg, int nb)
{
    const int c = S.cur[l];
    const uint64_t* ak = S.keys(l, c);
    const int64_t* ag = S.gs(l, c);
    uint64_t* ok = S.keys(l, c ^ 1);
    int64_t* og = S.gs(l, c ^ 1);
    const int na = K;
    for (int i = threadIdx.x; i < K; i += blockDim.x) {
        // co-rank: a = how many of the first i outputs come from A
        int lo = i - nb > 0 ? i - nb : 0, hi = i < na ? i : na;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (red_less(ak[mid], ag[mid], bk[i - 1 - mid], bg[i - 1 - mid])) lo = mid + 1; else hi = mid;
        }
        const int a = lo, b = i - a;
        const bool takeA = (b >= nb) || (a < na && red_less(ak[a], ag[a], bk[b], bg[b]));
        ok[i] = takeA ? ak[a] : bk[b];
        og[i] = takeA ? ag[a] : bg[b];
    }
    __syncthreads();
    if (threadIdx.x == 0) S.cur[l] = c ^ 1;
    __syncthreads();
}

// Whole workgroup: offer one (key, g) per thread (valid == false: nothing) to list l.
__device__ __forceinline__ void red_offer(RedLds& S, int l, int K, bool valid, uint64_t key, int64_t g)
{
    const int c = S.cur[l];
    const bool cand = valid && red_less(key, g, S.keys(l, c)[K - 1], S.gs(l, c)[K - 1]);
    if (!__syncthreads_or(cand)) return;
    if (threadIdx.x == 0) *S.nc = 0;
    __syncthreads();
    if (cand) {
        const int slot = atomicAdd(S.nc, 1);
        S.ck[slot] = key;
        S.cg[slot] = g;
    }
    __syncthreads();
    const int nc = *S.nc;
    int P = 1;
    while (P < nc) P <<= 1;
    for (int i = nc + threadIdx.x; i < P; i += blockDim.x) { S.ck[i] = kKeyEmpty; S.cg[i] = kGEmpty; }
    for (int size = 2; size <= P; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            __syncthreads();
            for (int i = threadIdx.x; i < (P >> 1); i += blockDim.x) {
                const int lo = 2 * i - (i & (stride - 1)), hi = lo + stride;
                const bool asc = (lo & size) == 0;
                const uint64_t ka = S.ck[lo], kb = S.ck[hi];
                const int64_t ga = S.cg[lo], gb = S.cg[hi];
                if (red_less(kb, gb, ka, ga) == asc) { S.ck[lo] = kb; S.ck[hi] = ka; S.cg[lo] = gb; S.cg[hi] = ga; }
            }
        }
    }
    __syncthreads();
    red_merge_sorted(S, l, K, S.ck, S.cg, nc < K ? nc : K);
}

// Bin of a value in [lo, hi] with `bins` equal bins; bins = under, bins + 1 = over.
__device__ __forceinline__ int red_bin(double v, double lo, double hi, int bins)
{
    if (v < lo) return bins;
    if (v > hi) return bins + 1;
    const int b = (int)floor((v - lo) / (hi - lo) * (double)bins);
    return b < bins - 1 ? b : bins - 1;
}

// Whole workgroup: every thread contributes at most one Omega of order k.
__device__ __forceinline__ void red_push(RedLds& S, const RedArgs& r, int k, bool valid, double v, int64_t g)
{
    if (r.bins > 0 && valid) atomicAdd(&S.hist[red_bin(v, r.lo[k], r.hi[k], r.bins)], 1u);
    if (r.topk > 0) {
        red_offer(S, 0, r.topk, valid, red_list_key(0, v), g);
        red_offer(S, 1, r.topk, valid, red_list_key(1, v), g);
    }
}

// Whole workgroup: write the lists as one segment and flush the histogram.
__device__ __forceinline__ void red_end(RedLds& S, const RedArgs& r, WsHeader* hdr, int d, int k)
{
    __syncthreads();
    const int K = r.topk;
    if (K > 0) {
        __shared__ uint32_t slot;
        if (threadIdx.x == 0) {
            // an all-empty segment is skipped
            const bool any = S.keys(0, S.cur[0])[0] != kKeyEmpty;
            slot = any ? atomicAdd(r.seg_next, 1u) : 0xffffffffu;
            if (any && slot >= r.seg_cap) raise_status(hdr, THOI_EWORKSPACE);
        }
        __syncthreads();
        const uint32_t s = slot;
        if (s < r.seg_cap) {
            if (threadIdx.x == 0) { r.seg_hdr[s].d = d; r.seg_hdr[s].k = k; }
            for (int i = threadIdx.x; i < 2 * K; i += blockDim.x) {
                const int l = i / K, j = i % K;
                r.seg_key[((int64_t)s * 2 + l) * K + j] = S.keys(l, S.cur[l])[j];
                r.seg_g[((int64_t)s * 2 + l) * K + j] = S.gs(l, S.cur[l])[j];
            }
        }
    }
    if (r.bins > 0) {
        unsigned long long* h = r.hist + ((int64_t)d * (r.kmax + 1) + k) * (r.bins + 2);
        for (int i = threadIdx.x; i < r.bins + 2; i += blockDim.x)
            if (S.hist[i]) atomicAdd(&h[i], (unsigned long long)S.hist[i]);
    }
    __syncthreads();
}

// One thread: queue an FP64-refined value for the final merge and count it in the histogram.
__device__ __forceinline__ void red_late(const RedArgs& r, WsHeader* hdr, int d, int k, int64_t g, double v)
{
    if (r.bins > 0) {
        unsigned long long* h = r.hist + ((int64_t)d * (r.kmax + 1) + k) * (r.bins + 2);
        atomicAdd(&h[red_bin(v, r.lo[k], r.hi[k], r.bins)], 1ull);
    }
    if (r.topk > 0) {
        const uint32_t s = atomicAdd(r.late_next, 1u);
        if (s < r.late_cap) r.late[s] = LateEntry{d, k, g, v};
        else raise_status(hdr, THOI_EWORKSPACE);
    }
}

}  // namespace thoi
