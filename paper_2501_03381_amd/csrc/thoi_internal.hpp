// Internal declarations shared by the libthoi.so translation units (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "thoi.h"

namespace thoi {

// ---------------------------------------------------------------------------------------------
// Workspace: every call that takes a workspace starts it with this 256-byte header.
// ---------------------------------------------------------------------------------------------
struct WsHeader {
    int32_t status;          // THOI_OK or a thoi_status raised on the device
    uint32_t refine_count;   // FP32_REFINE: number of n-plets appended to the refine list
    uint32_t seg_next;       // streaming reduction: segments written
    uint32_t late_next;      // streaming reduction: FP64-refined values queued
    uint64_t reserved[30];
};
static_assert(sizeof(WsHeader) == 256, "workspace header is 256 bytes");
constexpr size_t kWsHeader = 256;

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Record a device-side error in the status word (first error wins).
__device__ __forceinline__ void raise_status(WsHeader* h, int32_t code)
{
    atomicCAS(&h->status, 0, code);
}

// ---------------------------------------------------------------------------------------------
// Host-side helpers (api.cpp).
// ---------------------------------------------------------------------------------------------
thoi_status hip_status(hipError_t e);
// C(n, m) for 0 <= m <= n <= 64, exact in uint64 (0 outside that range).
uint64_t binom_u64(int n, int m);
// Bias offsets of order k (see thoi_bias_offsets).
void bias_offsets(int k, int T, double* d_tc, double* d_dtc, double* eta);
// psi((T-1)/2) and psi((T-2)/2), the seeds of the device-side recurrence for the offsets.
void bias_psi_seeds(int T, double* psi1, double* psi2);

// Fork/join over per-device side streams for independent launches (see fan.cpp).  Branch 0 is the
// caller's stream; branches beyond the side streams wrap around.
constexpr int kFanSide = 6;
class FanScope {
public:
    FanScope(hipStream_t s, int branches);
    ~FanScope();
    FanScope(const FanScope&) = delete;
    FanScope& operator=(const FanScope&) = delete;
    hipStream_t stream(int branch) const;

private:
    hipStream_t s_;
    void* fan_ = nullptr;
    int nside_ = 0;
    std::unique_lock<std::mutex> lock_;
};

// Launchers implemented in the kernel translation units.
thoi_status launch_copulize(const double* X, int64_t D, int64_t T, int64_t N, int32_t z_dtype, void* Z,
                            void* ws, hipStream_t s);
size_t copulize_ws_bytes(int64_t D, int64_t T, int64_t N);
thoi_status launch_cov(const void* Z, int32_t z_dtype, int64_t D, int64_t T, int64_t N, double* Sigma,
                       void* ws, hipStream_t s);
size_t cov_ws_bytes(int64_t D, int64_t T, int64_t N);
// serial: every launch goes to `s` (no side streams are created or used)
thoi_status launch_eval(const double* Sigma, int64_t D, int32_t N, const thoi_nplets* sel,
                        const thoi_eval_opts* opts, void* out, uint8_t* flags, void* ws, size_t ws_bytes,
                        hipStream_t s, bool serial = false);
// Host argument checks of thoi_nplets_eval (forward) and thoi_nplets_eval_backward (api.cpp).
thoi_status check_eval(const double* Sigma, int64_t D, int32_t N, const thoi_nplets* sel,
                       const thoi_eval_opts* opts, bool forward, const void* out);
size_t eval_ws_bytes(int64_t D, int32_t N, const thoi_nplets* sel, const thoi_eval_opts* opts);
size_t eval_lds_bytes(int32_t N, const thoi_nplets* sel, const thoi_eval_opts* opts);
void eval_launch_shape(int32_t N, const thoi_nplets* sel, const thoi_eval_opts* opts, int32_t* n_launches,
                       int64_t* max_items_x);
thoi_status launch_backward(const double* Sigma, int64_t D, int32_t N, const thoi_nplets* sel,
                            const thoi_eval_opts* opts, const float* grad_out, float* grad_Sigma, void* ws,
                            size_t ws_bytes, hipStream_t s);
size_t backward_ws_bytes(int64_t D, int32_t N, const thoi_nplets* sel, const thoi_eval_opts* opts);
size_t backward_lds_bytes(int32_t N, const thoi_nplets* sel);
thoi_status launch_reduce_init(const thoi_reduce* red, int64_t D, int32_t kmax, hipStream_t s);
thoi_status launch_multi(const double* Sigma, const int32_t* N_d, const int32_t* T_d, int64_t D, int32_t kmin,
                         int32_t kmax, const thoi_eval_opts* opts, void* out, uint8_t* flags, void* ws,
                         size_t ws_bytes, hipStream_t s);
size_t multi_ws_bytes(const int32_t* N_d, int64_t D, int32_t kmin, int32_t kmax, const thoi_eval_opts* opts);
size_t multi_lds_bytes(int32_t nmax, int32_t kmax, const thoi_eval_opts* opts);
int multi_lane_max(int32_t precision);
thoi_status launch_objective(const void* vals, int32_t val_dtype, int64_t D, int64_t B, int32_t kind, double* obj,
                             const thoi_reduce* red, void* ws, hipStream_t s);
size_t objective_ws_bytes(int64_t D, int64_t B, const thoi_reduce* red);
size_t greedy_ws_bytes(int64_t D, int32_t N, int32_t kappa);
int greedy_select_max();
thoi_status launch_greedy(const double* Sigma, int64_t D, int32_t N, int32_t k_first, int32_t kappa, int32_t steps,
                          int32_t measure, int32_t kind, int32_t maximize, uint64_t* sols, double* vals, int32_t* count,
                          void* ws, hipStream_t s);
thoi_status launch_anneal(const double* Sigma, int32_t N, const uint64_t* masks0, int32_t kappa, int32_t iters,
                          const double* draw_move, const double* draw_a, const double* draw_b, const double* draw_u,
                          double T0, double alpha, int32_t maximize, int32_t across, int32_t k_min, int32_t k_max,
                          uint64_t* cur_mask, double* cur_omega, uint64_t* best_mask, double* best_omega,
                          int64_t* accepted, hipStream_t s);

}  // namespace thoi
