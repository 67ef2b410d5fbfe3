// Adjoint lane engine, register classes of orders 0..8, 9..12 and 13..16 (see nplets_bwd_lane.hpp).
#include "nplets_bwd_lane.hpp"

namespace thoi {

void bwd_lane_launch_lo(int cls, const BwdArgs& a, const BwdTiles& t, int64_t ntiles, dim3 grid, size_t lds,
                        hipStream_t s)
{
    static_assert(kBwdClasses[0].lo == 0 && kBwdClasses[0].hi == 8 && kBwdClasses[1].hi == 12 &&
                      kBwdClasses[2].hi == 16, "class table");
    if (cls == 0) bwd_lane_launch_one<0, 8, kBwdClassThreads[0]>(a, t, ntiles, grid, lds, s);
    else if (cls == 1) bwd_lane_launch_one<9, 12, kBwdClassThreads[1]>(a, t, ntiles, grid, lds, s);
    else bwd_lane_launch_one<13, 16, kBwdClassThreads[2]>(a, t, ntiles, grid, lds, s);
}

int bwd_lane_blocks_per_cu_lo(int cls, size_t lds)
{
    if (cls == 0) return bwd_lane_blocks_one<0, 8, kBwdClassThreads[0]>(lds);
    if (cls == 1) return bwd_lane_blocks_one<9, 12, kBwdClassThreads[1]>(lds);
    return bwd_lane_blocks_one<13, 16, kBwdClassThreads[2]>(lds);
}

}  // namespace thoi
