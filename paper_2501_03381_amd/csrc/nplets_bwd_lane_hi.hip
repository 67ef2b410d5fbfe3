// Adjoint lane engine, register class of orders 17..20 (see nplets_bwd_lane.hpp).
#include "nplets_bwd_lane.hpp"

namespace thoi {

void bwd_lane_launch_hi(int cls, const BwdArgs& a, const BwdTiles& t, int64_t ntiles, dim3 grid, size_t lds,
                        hipStream_t s)
{
    static_assert(kBwdClasses[3].lo == 17 && kBwdClasses[3].hi == 20 && kBwdLaneMax == 20, "class table");
    (void)cls;
    bwd_lane_launch_one<17, 20, kBwdClassThreads[3]>(a, t, ntiles, grid, lds, s);
}

int bwd_lane_blocks_per_cu_hi(int cls, size_t lds)
{
    (void)cls;
    return bwd_lane_blocks_one<17, 20, kBwdClassThreads[3]>(lds);
}

}  // namespace thoi
