// Covariance operator of Eq. (gaussian_copula_covariance_estimator) on gfx950:
// Sigma_d = (Z_d - mean_d)^T (Z_d - mean_d) / (T - 1), FP64 throughout.
//
// The contraction over samples runs on the matrix cores (v_mfma_f64_16x16x4_f64).  Each wave
// owns one 16x16 output tile (a0, b0) with b0 >= a0 and one slab of samples; the four waves of a
// workgroup split the slab and sum their tiles through LDS.  Slab partials go to the workspace
// and a final kernel sums them in a fixed order (bitwise reproducible), divides by T-1 and
// mirrors the upper tiles so Sigma is exactly symmetric.
#include "thoi_internal.hpp"

namespace thoi {
namespace {

typedef double double4_t __attribute__((ext_vector_type(4)));

constexpr int kCovWaves = 4;
constexpr int kSlab = 512;        // samples per workgroup

template <typename ZT>
__device__ __forceinline__ double ld_z(const void* Z, int64_t off) { return (double)static_cast<const ZT*>(Z)[off]; }

// grid (nslabs, D), block 256: per-slab column sums.  Thread t owns column t % N and every
// (256 / N)-th row of the slab (N <= 256; wider matrices loop over column groups), so the loads
// of a row are coalesced; the per-thread partials are added in a fixed order (reproducible).
template <typename ZT>
__global__ __launch_bounds__(256) void k_col_sums(const void* __restrict__ Z, int64_t T, int64_t N,
                                                  double* __restrict__ part)
{
    __shared__ double red[256];
    const int64_t d = blockIdx.y;
    const int slab = blockIdx.x, nslabs = gridDim.x;
    const int64_t s0 = (int64_t)slab * kSlab, s1 = min<int64_t>(T, s0 + kSlab);
    for (int64_t c0 = 0; c0 < N; c0 += 256) {
        const int64_t nc = min<int64_t>(256, N - c0);
        const int groups = (int)(256 / nc);
        const int g = threadIdx.x / (int)nc, c = threadIdx.x % (int)nc;
        double s = 0.0;
        if (g < groups)
            for (int64_t t = s0 + g; t < s1; t += groups) s += ld_z<ZT>(Z, (d * T + t) * N + c0 + c);
        red[threadIdx.x] = s;
        __syncthreads();
        if (threadIdx.x < nc) {
            double acc = 0.0;
            for (int gg = 0; gg < groups; ++gg) acc += red[gg * nc + threadIdx.x];
            part[((int64_t)d * nslabs + slab) * N + c0 + threadIdx.x] = acc;
        }
        __syncthreads();
    }
}

// grid (ceil(N/256), D), block 256: mean = (sum of the slab sums in slab order) / T.
__global__ __launch_bounds__(256) void k_col_mean(const double* __restrict__ part, int nslabs, int64_t T, int64_t N,
                                                  double* __restrict__ mean)
{
    const int64_t d = blockIdx.y;
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= N) return;
    double s = 0.0;
    for (int sl = 0; sl < nslabs; ++sl) s += part[((int64_t)d * nslabs + sl) * N + c];
    mean[d * N + c] = s / (double)T;
}

// grid (ntile_pairs, nslabs, D), block 64*kCovWaves.  partial: [D][nslabs][Np][Np].
template <typename ZT>
__global__ __launch_bounds__(64 * kCovWaves) void k_cov_tiles(const void* __restrict__ Z, int64_t T, int64_t N, int64_t Np,
                                                             const double* __restrict__ mean,
                                                             double* __restrict__ partial)
{
    __shared__ double red[kCovWaves][256];
    const int64_t d = blockIdx.z;
    const int slab = blockIdx.y, nslabs = gridDim.y;
    // tile pair index -> (ta, tb) with ta <= tb
    const int nt = (int)(Np / 16);
    int p = blockIdx.x, ta = 0;
    while (p >= nt - ta) { p -= nt - ta; ++ta; }
    const int tb = ta + p;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t ca = ta * 16 + (lane & 15), cb = tb * 16 + (lane & 15);
    const int kk = lane >> 4;  // 0..3: sample within a step of 4
    const double ma = ca < N ? mean[d * N + ca] : 0.0;
    const double mb = cb < N ? mean[d * N + cb] : 0.0;

    const int64_t s0 = (int64_t)slab * kSlab, s1 = min<int64_t>(T, s0 + kSlab);
    double4_t acc = {0.0, 0.0, 0.0, 0.0};
    // t0 depends on the wave only, so every lane of a wave issues the same MFMAs; lanes whose
    // sample falls past the slab contribute zeros.
    for (int64_t t0 = s0 + 4 * w; t0 < s1; t0 += 4 * kCovWaves) {
        const int64_t t = t0 + kk;
        const bool in = t < s1;
        const double a = (in && ca < N) ? ld_z<ZT>(Z, (d * T + t) * N + ca) - ma : 0.0;
        const double b = (in && cb < N) ? ld_z<ZT>(Z, (d * T + t) * N + cb) - mb : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
    // Output layout of the 16x16x4 FP64 MFMA: lane holds D[lane/16 + 4v][lane%16], v = 0..3
    // (checked on gfx950 against the CPU covariance).
#pragma unroll
    for (int v = 0; v < 4; ++v) red[w][((lane >> 4) + 4 * v) * 16 + (lane & 15)] = acc[v];
    __syncthreads();
    for (int e = threadIdx.x; e < 256; e += blockDim.x) {
        double s = ((red[0][e] + red[1][e]) + red[2][e]) + red[3][e];
        const int i = e >> 4, j = e & 15;
        partial[((d * nslabs + slab) * Np + (ta * 16 + i)) * Np + (tb * 16 + j)] = s;
    }
}

// grid (ceil(Np*Np/256), D): Sigma = sum over slabs / (T-1), mirrored from the upper tiles.
__global__ __launch_bounds__(256) void k_cov_finish(const double* __restrict__ partial, int nslabs, int64_t T, int64_t N,
                                                    int64_t Np, double* __restrict__ Sigma)
{
    const int64_t d = blockIdx.y;
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= N * N) return;
    int64_t a = e / N, b = e % N;
    // both (a, b) and (b, a) read the upper-triangle entry, so Sigma is exactly symmetric
    const int64_t ra = a < b ? a : b, rb = a < b ? b : a;
    double s = 0.0;
    for (int sl = 0; sl < nslabs; ++sl) s += partial[((d * nslabs + sl) * Np + ra) * Np + rb];
    Sigma[(d * N + a) * N + b] = s / (double)(T - 1);
}

}  // namespace

size_t cov_ws_bytes(int64_t D, int64_t T, int64_t N)
{
    const int64_t Np = (N + 15) / 16 * 16;
    const int64_t nslabs = (T + kSlab - 1) / kSlab;
    size_t off = kWsHeader;
    off = align_up(off + (size_t)D * N * 8, 256);                      // means
    off = align_up(off + (size_t)D * nslabs * N * 8, 256);             // slab column sums
    off = align_up(off + (size_t)D * nslabs * Np * Np * 8, 256);       // slab products
    return off;
}

thoi_status launch_cov(const void* Z, int32_t z_dtype, int64_t D, int64_t T, int64_t N, double* Sigma, void* ws,
                       hipStream_t s)
{
    const int64_t Np = (N + 15) / 16 * 16;
    const int64_t nslabs = (T + kSlab - 1) / kSlab;
    char* base = static_cast<char*>(ws);
    size_t off = kWsHeader;
    double* mean = reinterpret_cast<double*>(base + off);
    off = align_up(off + (size_t)D * N * 8, 256);
    double* colsum = reinterpret_cast<double*>(base + off);
    off = align_up(off + (size_t)D * nslabs * N * 8, 256);
    double* partial = reinterpret_cast<double*>(base + off);
    if (D * N == 0) return THOI_OK;
    dim3 gs((unsigned)nslabs, (unsigned)D);
    dim3 gm((unsigned)((N + 255) / 256), (unsigned)D);
    const int nt = (int)(Np / 16);
    dim3 gt((unsigned)(nt * (nt + 1) / 2), (unsigned)nslabs, (unsigned)D);
    dim3 gf((unsigned)((N * N + 255) / 256), (unsigned)D);
    if (z_dtype == THOI_DTYPE_F64) {
        hipLaunchKernelGGL(k_col_sums<double>, gs, dim3(256), 0, s, Z, T, N, colsum);
        hipLaunchKernelGGL(k_col_mean, gm, dim3(256), 0, s, colsum, (int)nslabs, T, N, mean);
        hipLaunchKernelGGL(k_cov_tiles<double>, gt, dim3(64 * kCovWaves), 0, s, Z, T, N, Np, mean, partial);
    } else {
        hipLaunchKernelGGL(k_col_sums<float>, gs, dim3(256), 0, s, Z, T, N, colsum);
        hipLaunchKernelGGL(k_col_mean, gm, dim3(256), 0, s, colsum, (int)nslabs, T, N, mean);
        hipLaunchKernelGGL(k_cov_tiles<float>, gt, dim3(64 * kCovWaves), 0, s, Z, T, N, Np, mean, partial);
    }
    hipLaunchKernelGGL(k_cov_finish, gf, dim3(256), 0, s, partial, (int)nslabs, T, N, Np, Sigma);
    return hip_status(hipGetLastError());
}

}  // namespace thoi
