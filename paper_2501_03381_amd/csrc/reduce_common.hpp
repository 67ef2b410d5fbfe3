// Streaming per-(dataset, order) reduction of Omega on gfx950: exact top-K (largest) and bottom-K
// (smallest) lists with (value, global index) ordering, and a histogram with under/overflow
// counts.  This replaces the paper's per-batch custom function aggregated on the fly (Figure 1A)
// so that exhaustive runs never store exponentially many results.
//
// Each workgroup covers n-plets of one (d, k); each of its wavefronts keeps two running sorted
// lists in LDS and merges the values that beat its admission bound (merge path).  At the end the
// workgroup folds its wavefront lists into one "segment" in the workspace, publishes the
// segment's K-th keys as admission bounds for later workgroups of the same (d, k), and adds its
// LDS histogram to the global one.  A final kernel merges, per (d, k), the accumulated lists of
// earlier calls, every segment of this call, and the FP64-refined values (queued separately).
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
    unsigned long long* bound;       // [D][kmax+1][2] admission bounds, ~key (0 = none); or null
    double lo[THOI_MAX_K + 1], hi[THOI_MAX_K + 1];
};

// Producers reduce with per-wavefront lists: a value enters a wavefront's list when it beats the
// list's admission bound (the tighter of the list's K-th entry and a bound shared by the (d, k));
// the wavefront ranks its candidates among themselves with lane reads and merges them into its
// list with a merge path, with no workgroup barrier.  The wavefront lists are folded into one
// segment when the workgroup ends.  Every thread of a producing workgroup calls red_push the same
// number of times with its whole wavefront active; a workgroup has at most kRedWaves wavefronts.
constexpr int kRedWaves = 4;

struct __align__(16) RedItem {
    uint64_t k;
    int64_t g;
};

// Layout from a 16-byte aligned base: list [kRedWaves][2 lists][K] | stage [kRedWaves][64] |
// hist [bins + 2] u32 | slot u32.
struct RedLds {
    RedItem* list;
    RedItem* stage;
    unsigned int* hist;
    uint32_t* slot;
    int K;
    int w;                   // this thread's wavefront
    uint64_t tk[2];          // admission bound of each list (uniform in the wavefront)
    int64_t tg[2];
    __device__ __forceinline__ RedItem* L(int wave, int l) const { return list + (wave * 2 + l) * K; }
};

__host__ __device__ constexpr size_t red_lds_bytes(int K, int bins)
{
    const size_t lists = (size_t)kRedWaves * 2 * (K > 0 ? K : 1) * 16;
    const size_t b = lists + (size_t)kRedWaves * 64 * 16 + (size_t)(bins + 2) * 4 + 16;
    return (b + 15) / 16 * 16;
}

__device__ __forceinline__ RedLds red_view(unsigned char* base, int K, int bins)
{
    RedLds S;
    const int Kc = K > 0 ? K : 1;
    S.K = Kc;
    S.list = reinterpret_cast<RedItem*>(base);
    S.stage = S.list + kRedWaves * 2 * Kc;
    S.hist = reinterpret_cast<unsigned int*>(S.stage + kRedWaves * 64);
    S.slot = S.hist + bins + 2;
    S.w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    S.tk[0] = S.tk[1] = ~0ull;
    S.tg[0] = S.tg[1] = INT64_MAX;
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

__device__ __forceinline__ bool red_less(const RedItem& a, const RedItem& b) { return red_less(a.k, a.g, b.k, b.g); }

__device__ __forceinline__ void red_wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint64_t red_readlane(uint64_t x, int j)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, j);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), j);
    return ((uint64_t)hi << 32) | lo;
}

// A value the wavefront holds in every lane, moved to scalar registers.
__device__ __forceinline__ uint64_t red_uniform(uint64_t x)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(x >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Output i (< na + nb) of the merge of the sorted runs A[0..na) and B[0..nb): the co-rank a (how
// many of the first i outputs come from A) by binary search over the window the run lengths allow.
__device__ __forceinline__ RedItem red_merge_at(const RedItem* A, int na, const RedItem* B, int nb, int i)
{
    int lo = i - nb > 0 ? i - nb : 0, hi = i < na ? i : na;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (red_less(A[mid], B[i - 1 - mid])) lo = mid + 1; else hi = mid;
    }
    const int a = lo, b = i - a;
    const bool takeA = (b >= nb) || (a < na && red_less(A[a], B[b]));
    return takeA ? A[a] : B[b];
}

// Bin of a value in [lo, hi] with `bins` equal bins; bins = under, bins + 1 = over.
__device__ __forceinline__ int red_bin(double v, double lo, double hi, int bins)
{
    if (v < lo) return bins;
    if (v > hi) return bins + 1;
    const int b = (int)floor((v - lo) / (hi - lo) * (double)bins);
    return b < bins - 1 ? b : bins - 1;
}

// Whole workgroup: empty the wavefront lists and the histogram, and take the admission bounds
// that (d, k) has published so far.
__device__ __forceinline__ void red_begin(RedLds& S, const RedArgs& r, int d, int k)
{
    const int K = r.topk;
    for (int i = threadIdx.x; i < kRedWaves * 2 * K; i += blockDim.x) S.list[i] = RedItem{kKeyEmpty, kGEmpty};
    for (int i = threadIdx.x; i < r.bins + 2; i += blockDim.x) S.hist[i] = 0;
    S.tk[0] = S.tk[1] = kKeyEmpty;
    S.tg[0] = S.tg[1] = kGEmpty;
    if (K > 0 && r.bound) {
        unsigned long long* b = r.bound + ((int64_t)d * (r.kmax + 1) + k) * 2;
#pragma unroll
        for (int l = 0; l < 2; ++l) {
            const unsigned long long v = __hip_atomic_load(b + l, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            S.tk[l] = red_uniform(~(uint64_t)v);     // stored complemented: 0 = no bound yet
        }
    }
    __syncthreads();
}

// Whole wavefront: merge the candidates of mask m (this lane's: cand, key, g) into list l of the
// wavefront and tighten its admission bound.
__device__ __forceinline__ void red_wave_insert(RedLds& S, int l, int K, uint64_t m, bool cand, uint64_t key, int64_t g)
{
    const int lane = (int)(threadIdx.x & 63);
    const int n = __popcll(m);
    // rank among the candidates (their (key, g) are distinct)
    int rank = 0;
    for (uint64_t mm = m; mm; mm &= mm - 1) {
        const int j = __builtin_ctzll(mm);
        rank += red_less(red_readlane(key, j), (int64_t)red_readlane((uint64_t)g, j), key, g) ? 1 : 0;
    }
    RedItem* B = S.stage + S.w * 64;
    RedItem* A = S.L(S.w, l);
    if (cand) B[rank] = RedItem{key, g};
    red_wave_sync();
    // In place, 64 outputs at a time from the back: output i only reads A[0..i], so a block of
    // outputs never reads what the blocks after it have written.
    const int nb = n < K ? n : K;
    for (int r = (K - 1) >> 6; r >= 0; --r) {
        const int i = lane + 64 * r;
        RedItem o{};
        if (i < K) o = red_merge_at(A, K, B, nb, i);
        red_wave_sync();
        if (i < K) A[i] = o;
        red_wave_sync();
    }
    const RedItem t = A[K - 1];
    if (red_less(t.k, t.g, S.tk[l], S.tg[l])) { S.tk[l] = red_uniform(t.k); S.tg[l] = (int64_t)red_uniform((uint64_t)t.g); }
}

// Whole workgroup (see above): every thread contributes at most one Omega of order k.
__device__ __forceinline__ void red_push(RedLds& S, const RedArgs& r, int k, bool valid, double v, int64_t g)
{
    if (r.bins > 0 && valid) atomicAdd(&S.hist[red_bin(v, r.lo[k], r.hi[k], r.bins)], 1u);
    if (r.topk > 0) {
#pragma unroll
        for (int l = 0; l < 2; ++l) {
            const uint64_t key = red_list_key(l, v);
            const bool cand = valid && red_less(key, g, S.tk[l], S.tg[l]);
            const uint64_t m = __ballot(cand);
            if (m) red_wave_insert(S, l, r.topk, m, cand, key, g);      // uniform in the wavefront
        }
    }
}

// Whole workgroup: fold the wavefront lists into one segment, publish its K-th keys as admission
// bounds of (d, k), and flush the histogram.  A published key b comes from a segment holding K
// entries with keys <= b, all of which reach the final merge, so a later value whose key exceeds b
// has K better entries ahead of it and is not needed; a value with key == b is still admitted
// (ties are ordered by index).
__device__ __forceinline__ void red_end(RedLds& S, const RedArgs& r, WsHeader* hdr, int d, int k)
{
    __syncthreads();
    const int K = r.topk;
    if (K > 0) {
        const int nw = (int)((blockDim.x + 63) >> 6);
        for (int w = 1; w < nw; ++w) {
            // both lists at once: thread t owns outputs t, t + blockDim, ... of the 2K
            constexpr int kPer = 2 * kRedMaxK / 128;     // nw >= 2 means blockDim >= 128
            RedItem o[kPer];
#pragma unroll
            for (int r2 = 0; r2 < kPer; ++r2) {
                const int i = (int)threadIdx.x + r2 * (int)blockDim.x;
                if (i < 2 * K) {
                    const int l = i / K;
                    o[r2] = red_merge_at(S.L(0, l), K, S.L(w, l), K, i - l * K);
                }
            }
            __syncthreads();
#pragma unroll
            for (int r2 = 0; r2 < kPer; ++r2) {
                const int i = (int)threadIdx.x + r2 * (int)blockDim.x;
                if (i < 2 * K) {
                    const int l = i / K;
                    S.L(0, l)[i - l * K] = o[r2];
                }
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            // an all-empty segment is skipped
            const bool any = S.L(0, 0)[0].k != kKeyEmpty || S.L(0, 1)[0].k != kKeyEmpty;
            const uint32_t slot = any ? atomicAdd(r.seg_next, 1u) : 0xffffffffu;
            if (any && slot >= r.seg_cap) raise_status(hdr, THOI_EWORKSPACE);
            *S.slot = slot;
            if (r.bound && slot < r.seg_cap) {
                unsigned long long* b = r.bound + ((int64_t)d * (r.kmax + 1) + k) * 2;
                for (int l = 0; l < 2; ++l) {
                    const uint64_t t = S.L(0, l)[K - 1].k;
                    if (t != kKeyEmpty) atomicMax(b + l, (unsigned long long)~t);
                }
            }
        }
        __syncthreads();
        const uint32_t s = *S.slot;
        if (s < r.seg_cap) {
            if (threadIdx.x == 0) { r.seg_hdr[s].d = d; r.seg_hdr[s].k = k; }
            for (int i = threadIdx.x; i < 2 * K; i += blockDim.x) {
                const int l = i / K, j = i % K;
                const RedItem e = S.L(0, l)[j];
                r.seg_key[((int64_t)s * 2 + l) * K + j] = e.k;
                r.seg_g[((int64_t)s * 2 + l) * K + j] = e.g;
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

// ------------------------------------------------------------------------------------------------
// Final merge (one workgroup per (order, dataset)): two double-buffered lists in LDS.
// ------------------------------------------------------------------------------------------------
struct RedFinal {
    uint64_t key[2][2][kRedMaxK];
    int64_t g[2][2][kRedMaxK];
    uint64_t ck[256];
    int64_t cg[256];
    int cur[2];
    int nc;
};

// Whole workgroup: merge the sorted run (bk, bg)[0..nb) into list `l`, keeping K.
__device__ __forceinline__ void red_final_merge(RedFinal& S, int l, int K, const uint64_t* bk, const int64_t* bg, int nb)
{
    const int c = S.cur[l];
    const uint64_t* ak = S.key[l][c];
    const int64_t* ag = S.g[l][c];
    uint64_t* ok = S.key[l][c ^ 1];
    int64_t* og = S.g[l][c ^ 1];
    const int na = K;
    for (int i = threadIdx.x; i < K; i += blockDim.x) {
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

// Whole workgroup (blockDim <= 256): offer one (key, g) per thread (valid == false: nothing) to
// list l; the candidates are compacted, sorted (bitonic) and merged.
__device__ __forceinline__ void red_final_offer(RedFinal& S, int l, int K, bool valid, uint64_t key, int64_t g)
{
    const int c = S.cur[l];
    const bool cand = valid && red_less(key, g, S.key[l][c][K - 1], S.g[l][c][K - 1]);
    if (!__syncthreads_or(cand)) return;
    if (threadIdx.x == 0) S.nc = 0;
    __syncthreads();
    if (cand) {
        const int slot = atomicAdd(&S.nc, 1);
        S.ck[slot] = key;
        S.cg[slot] = g;
    }
    __syncthreads();
    const int nc = S.nc;
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
    red_final_merge(S, l, K, S.ck, S.cg, nc < K ? nc : K);
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
