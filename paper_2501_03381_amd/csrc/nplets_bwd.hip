// Adjoint of the n-plet evaluation (placeholder until the adjoint kernel lands).
#include "nplets_common.hpp"

namespace thoi {

size_t backward_ws_bytes(int64_t D, int32_t N, const thoi_nplets* sel, const thoi_eval_opts* opts)
{
    (void)D; (void)N; (void)sel; (void)opts;
    return kWsHeader;
}

thoi_status launch_backward(const double* Sigma, int64_t D, int32_t N, const thoi_nplets* sel,
                            const thoi_eval_opts* opts, const float* grad_out, float* grad_Sigma, void* ws,
                            size_t ws_bytes, hipStream_t s)
{
    (void)Sigma; (void)D; (void)N; (void)sel; (void)opts; (void)grad_out; (void)grad_Sigma; (void)ws; (void)ws_bytes; (void)s;
    return THOI_EUNSUPPORTED;
}

}  // namespace thoi
