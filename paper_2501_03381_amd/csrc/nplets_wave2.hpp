// Pair engine (nplets_wave2.hip): FP64 evaluation of orders above the register classes up to
// kW2Max, two n-plets per wavefront.  Host-side interface.
#pragma once

#include "nplets_fwd_common.hpp"

namespace thoi {

constexpr int kW2Max = 32;   // largest order of the pair engine
constexpr int kPairThreads = 256;                 // threads per pair-engine workgroup
constexpr int kPairHalves = kPairThreads / 32;    // n-plets factored at once per workgroup

// LDS bytes of a pair-engine workgroup (red_bytes: the reducer's share, 0 without reduction).
size_t pair_lds_bytes(int N, size_t red_bytes);
// Launch the pair engine over nblk workgroups per dataset: a.wave_tile n-plets of one order per
// workgroup (RANGE pieces of t, LIST / MASK buckets) of orders klo..kmax.
void pair_launch(int mode, bool reduce, const EvalArgs& a, const PieceTable& t, const RedArgs& red, int klo, int kmax,
                 int64_t nblk, hipStream_t s);

// FP64 re-evaluation of the refinement queue of a call, replacing the FP32 results of the queued
// n-plets (orders up to 16 one per lane, the others up to kW2Max two per wavefront).
void refine_launch(int mode, const EvalArgs& a, const RangeOrders& ro, const RedArgs& red, hipStream_t s);

}  // namespace thoi
