// thoi_nplets_eval_noalloc: the n-plet evaluation with a library-owned workspace, for callers
// that cannot allocate device memory.
//
// The workspace is `scratch`, a file-scope device array (one per GPU, alive until the process
// ends).  Host code never passes the array's name to a kernel: its device address is looked up
// once per device with hipGetSymbolAddress, with that device current, and kept in a per-device
// table; the kernels receive that address exactly as they receive a caller's workspace.  The
// evaluation itself is thoi_nplets_eval's (same kernels, launched on the caller's stream only).
#include "thoi_internal.hpp"

#include <mutex>

namespace thoi {
namespace {

constexpr size_t kScratchBytes = THOI_NOALLOC_SCRATCH_BYTES;
static_assert(kScratchBytes % 256 == 0, "scratch size is a multiple of its alignment");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];   // device address of `scratch` on each device, once looked up

// The status word of the workspace header, copied to the caller's buffer after the evaluation.
__global__ void k_copy_status(const WsHeader* hdr, int32_t* status)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *status = hdr->status;
}

// Address of `scratch` on the device of stream s (looked up on the first call on that device).
thoi_status scratch_for(hipStream_t s, void** ptr)
{
    int dev = 0;
    if (hipStreamGetDevice(s, &dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return THOI_EHIP;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        int cur = 0;
        if (hipGetDevice(&cur) != hipSuccess) return THOI_EHIP;
        if (cur != dev && hipSetDevice(dev) != hipSuccess) return THOI_EHIP;
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) (void)hipSetDevice(cur);
        if (e != hipSuccess || p == nullptr) return THOI_EHIP;
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return THOI_OK;
}

}  // namespace
}  // namespace thoi

using namespace thoi;

extern "C" thoi_status thoi_nplets_eval_noalloc(const double* Sigma, int64_t D, int32_t N, const thoi_nplets* sel,
                                                const thoi_eval_opts* opts, void* out, uint8_t* flags,
                                                int32_t* status, void* stream)
{
    const thoi_status st = check_eval(Sigma, D, N, sel, opts, true, out);
    if (st != THOI_OK) return st;
    const size_t need = eval_ws_bytes(D, N, sel, opts);
    if (need > kScratchBytes) return THOI_EWORKSPACE;
    const hipStream_t s = (hipStream_t)stream;
    void* ws = nullptr;
    const thoi_status sst = scratch_for(s, &ws);
    if (sst != THOI_OK) return sst;
    const thoi_status lst = launch_eval(Sigma, D, N, sel, opts, out, flags, ws, kScratchBytes, s, true);
    if (lst != THOI_OK || status == nullptr) return lst;
    hipLaunchKernelGGL(k_copy_status, dim3(1), dim3(64), 0, s, static_cast<const WsHeader*>(ws), status);
    return hip_status(hipGetLastError());
}
