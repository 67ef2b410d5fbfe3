// Prefix-sharing engine of the exhaustive evaluation (nplets_prefix.hip): host-side interface.
#pragma once

#include "nplets_fwd_common.hpp"

namespace thoi {

// Orders handled by the prefix engine, grouped into launch classes by register footprint.
struct PfxClass { int lo, hi; };
constexpr PfxClass kPfxF32Classes[] = {{3, 8}, {9, 12}, {13, 16}};
constexpr PfxClass kPfxF64Classes[] = {{3, 8}, {9, 12}};
constexpr int kPfxF32Max = 16;
constexpr int kPfxF64Max = 12;
constexpr int kPfxThreads = 256;   // threads per workgroup: 4 wavefronts, same last prefix variable
constexpr int kPfxMaxTails = 16;   // largest number of consecutive tails walked by one lane
constexpr int64_t kPfxMaxGroups = 2048;   // persistent workgroups per order and dataset

// One whole order k of a RANGE call: output position of its first n-plet, tails per lane, and the
// persistent workgroups [blk0, blk0 + nphys) of its class launch that walk its nblk blocks.
struct PfxPiece {
    int32_t k;
    int32_t L;
    int64_t pos0;
    int64_t blk0;
    int64_t nphys;
    int64_t nblk;
};
struct PfxTable {
    int32_t n;
    int32_t pad;
    PfxPiece p[kMaxPieces];
};

// Tails per lane for order k over N variables and D datasets: as many as keep about 2^18 lanes
// busy (a power of two in 1..kPfxMaxTails).
int pfx_tails(int N, int k, int64_t D);
// Blocks (4 units of 64 prefixes x L tails) of order k over N variables.
int64_t pfx_blocks(int N, int k, int L);
// LDS bytes of a prefix-engine workgroup (red_bytes: the reducer's share, 0 without reduction).
size_t pfx_lds_bytes(int N, int fsize, size_t red_bytes);
// Launch prefix class `cls` (FP64 when f64) over D datasets.
void pfx_launch(bool f64, int cls, bool reduce, const EvalArgs& a, const PfxTable& t, const RedArgs& red,
                int64_t nblk, int D, hipStream_t s);

}  // namespace thoi
