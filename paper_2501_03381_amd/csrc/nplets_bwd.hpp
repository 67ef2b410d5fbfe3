// Types and launchers shared by the translation units of the adjoint (nplets_bwd*.hip).
#pragma once

#include "thoi_internal.hpp"

namespace thoi {

constexpr int kBwdMaxPieces = 24;      // RANGE: orders per lane-engine class

// Lane-engine classes: orders [lo, hi] evaluated by one launch (one register footprint).
struct BwdClass { int lo, hi; };
constexpr BwdClass kBwdClasses[] = {{0, 8}, {9, 12}, {13, 16}, {17, 20}};
constexpr int kBwdNClasses = (int)(sizeof(kBwdClasses) / sizeof(BwdClass));
constexpr int kBwdLaneMax = 20;
// Threads per workgroup (= n-plets per tile) of each class.  Orders 0..8 use 64 VGPRs and run four
// waves per SIMD in one workgroup; for the larger classes 1024- and 512-thread workgroups measured
// slower than 256 at N = 100 (latent_100 adjoint: 200 / 170 us against 123 / 135 us per class).
constexpr int kBwdClassThreads[] = {1024, 256, 256, 256};
static_assert(sizeof(kBwdClassThreads) / sizeof(int) == kBwdNClasses, "one size per class");

// RANGE: the n-plets of one order inside the call's range, and the first tile they occupy inside
// their class's launch.
struct BwdPiece {
    int32_t k;
    int32_t pad;
    int64_t first;   // first lexicographic rank inside C(N, k)
    int64_t pos0;    // output position of `first`
    int64_t cnt;     // n-plets
    int64_t tile0;   // first tile
};
struct BwdTiles {
    int32_t n;
    int32_t pad;
    BwdPiece p[kBwdMaxPieces];
};

struct BwdArgs {
    const double* Sigma;        // [D][N][N]
    int32_t N, D;
    int64_t B;                  // output positions per dataset
    const float* grad_out;      // [4][D][B]
    float* grad_Sigma;          // [D][N][N]
    int32_t mode;               // THOI_SEL_*
    int32_t lane_max;           // largest order of the lane engine (kBwdLaneMax, or 0 when its staged
                                // matrix does not fit in LDS); larger orders go to the wave engine
    int64_t g_begin;            // RANGE
    int64_t ostart[THOI_MAX_K + 2];   // RANGE: global index of the first n-plet of order k
    int32_t kmin, kmax;         // RANGE
    const int32_t* idx;         // LIST
    int32_t kmax_list;
    int32_t pad;
    const uint64_t* mask;       // MASK
    const int64_t* perm;        // LIST / MASK: positions sorted by order
    const int64_t* lcnt;        // LIST / MASK: rows per order
    const int64_t* lbase;       // LIST / MASK: first slot of each order in perm
};

__host__ __device__ inline size_t bwd_align16(size_t x) { return (x + 15) / 16 * 16; }

// The lane engine stages the FP64 correlation matrix in LDS when it is small (N <= 64: 32 KB);
// larger matrices are read from global memory (they stay in L2), so that LDS does not cap the
// workgroups per compute unit.
__host__ __device__ inline bool bwd_stage_matrix(int N) { return N <= 64; }

// LDS of the lane engine: sR [N*N] f64 (staged only) | sIsd [N] f64 | sLogd [N] f64 |
// sBin [N*kb] u64 (RANGE) | sAcc [N (N+1) / 2] f32
__host__ __device__ inline size_t bwd_lane_lds_bytes(int N, int kb)
{
    const size_t r = bwd_stage_matrix(N) ? bwd_align16((size_t)N * N * 8) : 0;
    return bwd_align16(r + (size_t)N * 16 + (size_t)N * kb * 8) + bwd_align16((size_t)N * (N + 1) / 2 * 4);
}

// Launch lane-engine class `cls` (nplets_bwd_lane_lo.hip: classes 0..2, nplets_bwd_lane_hi.hip:
// class 3) and the number of its workgroups one compute unit holds at `lds` bytes of LDS.
void bwd_lane_launch_lo(int cls, const BwdArgs& a, const BwdTiles& t, int64_t ntiles, dim3 grid, size_t lds,
                        hipStream_t s);
void bwd_lane_launch_hi(int cls, const BwdArgs& a, const BwdTiles& t, int64_t ntiles, dim3 grid, size_t lds,
                        hipStream_t s);
int bwd_lane_blocks_per_cu_lo(int cls, size_t lds);
int bwd_lane_blocks_per_cu_hi(int cls, size_t lds);

}  // namespace thoi
