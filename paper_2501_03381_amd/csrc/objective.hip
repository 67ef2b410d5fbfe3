// Objectives over datasets: one FP64 value per n-plet from its measure in D datasets (mean, or the
// paired effect size between two conditions), written out and/or streamed into the top-K /
// histogram reducer (one list, order slot 0).  A function of the measures optimised across
// datasets is what the paper's searches take as their objective (Discussion; Methods, "Greedy
// Algorithm").
#include "nplets_fwd_common.hpp"
#include "objective_common.hpp"

namespace thoi {
namespace {

constexpr int kObjTile = 256;
constexpr int kObjMaxBlocks = 4096;
static_assert(kObjTile <= 64 * kRedWaves, "the reducer keeps lists for at most kRedWaves wavefronts");

// grid (blocks), block kObjTile: tiles [blk * per_blk, (blk + 1) * per_blk) of n-plets.
template <typename VT, bool RED>
__global__ __launch_bounds__(kObjTile) void k_objective(const void* __restrict__ vals, int64_t D, int64_t B, int kind,
                                                        int64_t per_blk, double* __restrict__ obj, RedArgs red,
                                                        WsHeader* hdr)
{
    const VT* v = static_cast<const VT*>(vals);
    __shared__ __align__(16) unsigned char sred[red_lds_bytes(kRedMaxK, kRedMaxBins)];
    RedLds S = red_view(sred, red.topk, red.bins);
    if constexpr (RED) red_begin(S, red, 0, 0);
    const int64_t b0 = (int64_t)blockIdx.x * per_blk;
    const int64_t b1 = min(B, b0 + per_blk);
    for (int64_t t = b0; t < b1; t += kObjTile) {          // uniform trip count in the workgroup
        const int64_t b = t + threadIdx.x;
        double o = __builtin_nan("");
        if (b < b1) {
            o = objective_of<VT>(v, D, B, b, kind);
            if (obj) obj[b] = o;
        }
        if constexpr (RED) red_push(S, red, 0, b < b1 && !isnan(o), o, b);
    }
    if constexpr (RED) red_end(S, red, hdr, 0, 0);
}

struct ObjWs {
    size_t key_off, g_off, hdr_off, bound_off, clear_end, total;
    int64_t blocks, per_blk;
};

ObjWs obj_layout(int64_t B, int topk)
{
    ObjWs w{};
    const int64_t tiles = (B + kObjTile - 1) / kObjTile;
    const int64_t tpb = (tiles + kObjMaxBlocks - 1) / kObjMaxBlocks;
    w.per_blk = (tpb > 0 ? tpb : 1) * kObjTile;
    w.blocks = (B + w.per_blk - 1) / w.per_blk;
    size_t off = kWsHeader;
    if (topk > 0) {
        w.bound_off = off;             // admission bounds of the one list pair, cleared with the header
        off = align_up(off + 16, 256);
    }
    w.clear_end = off;
    if (topk > 0) {
        const size_t segs = (size_t)(w.blocks > 0 ? w.blocks : 1);
        w.key_off = off; off = align_up(off + segs * 2 * topk * 8, 256);
        w.g_off = off; off = align_up(off + segs * 2 * topk * 8, 256);
        w.hdr_off = off; off = align_up(off + segs * sizeof(SegHdr), 256);
    }
    w.total = off;
    return w;
}

}  // namespace

size_t objective_ws_bytes(int64_t D, int64_t B, const thoi_reduce* red)
{
    (void)D;
    return obj_layout(B, red ? red->topk : 0).total;
}

thoi_status launch_objective(const void* vals, int32_t val_dtype, int64_t D, int64_t B, int32_t kind, double* obj,
                             const thoi_reduce* red, void* ws, hipStream_t s)
{
    const ObjWs w = obj_layout(B, red ? red->topk : 0);
    char* base = static_cast<char*>(ws);
    WsHeader* hdr = reinterpret_cast<WsHeader*>(base);
    ws_clear(base, w.clear_end, s);
    RedArgs ra{};
    if (red) {
        ra.active = 1;
        ra.topk = red->topk;
        ra.bins = red->hist_bins;
        ra.kmax = 0;
        ra.top_val = red->top_val;
        ra.top_g = red->top_g;
        ra.hist = reinterpret_cast<unsigned long long*>(red->hist);
        if (red->topk > 0) {
            ra.seg_key = reinterpret_cast<uint64_t*>(base + w.key_off);
            ra.seg_g = reinterpret_cast<int64_t*>(base + w.g_off);
            ra.seg_hdr = reinterpret_cast<SegHdr*>(base + w.hdr_off);
            ra.seg_cap = (uint32_t)(w.blocks > 0 ? w.blocks : 1);
            ra.bound = reinterpret_cast<unsigned long long*>(base + w.bound_off);
        }
        ra.seg_next = &hdr->seg_next;
        ra.late_next = &hdr->late_next;
        if (red->hist_bins > 0) { ra.lo[0] = red->hist_lo_hi[0]; ra.hi[0] = red->hist_lo_hi[1]; }
    }
    if (B > 0) {
        typedef void (*ObjKernel)(const void*, int64_t, int64_t, int, int64_t, double*, RedArgs, WsHeader*);
        const bool r = red != nullptr;
        const bool f64 = val_dtype == THOI_DTYPE_F64;
        const ObjKernel kern = f64 ? (r ? (ObjKernel)k_objective<double, true> : (ObjKernel)k_objective<double, false>)
                                   : (r ? (ObjKernel)k_objective<float, true> : (ObjKernel)k_objective<float, false>);
        hipLaunchKernelGGL(kern, dim3((unsigned)w.blocks), dim3(kObjTile), 0, s, vals, D, B, (int)kind, w.per_blk, obj,
                           ra, hdr);
    }
    if (red && red->topk > 0) hipLaunchKernelGGL(k_red_final, dim3(1, 1), dim3(256), 0, s, ra, hdr);
    return hip_status(hipGetLastError());
}

}  // namespace thoi
