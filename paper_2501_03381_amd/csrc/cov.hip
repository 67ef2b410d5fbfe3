// Covariance operator of Eq. (gaussian_copula_covariance_estimator) on gfx950:
// Sigma_d = (Z_d - mean_d)^T (Z_d - mean_d) / (T - 1), FP64 throughout.
//
// Samples are cut into slabs of kSlab rows.  A workgroup owns one slab and one 16x16 output tile
// (a0, b0) with b0 >= a0: it stages the slab's 32 columns in LDS (all loads in flight at once),
// takes their slab means, then contracts the slab-centred columns on the matrix cores
// (v_mfma_f64_16x16x4_f64), its four waves splitting the slab and summing their tiles through LDS.  The finish kernel combines the slabs with the exact
// pairwise update of centred sums (Chan, Golub and LeVeque):
//   C = sum_s C_s + sum_s n_s (m_s - m)(m_s - m)^T,   m = sum_s n_s m_s / T,
// with one wavefront per output entry, lanes over slabs and a fixed reduction tree (bitwise
// reproducible); it divides by T-1 and writes both mirror entries, so Sigma is exactly symmetric.  Both passes are centred, so there is no cancellation of large means.
#include "thoi_internal.hpp"

namespace thoi {
namespace {

typedef double double4_t __attribute__((ext_vector_type(4)));

constexpr int kCovThreads = 256;   // four waves
constexpr int kSlab = 128;         // samples per workgroup
constexpr int kStageLd = kSlab * 32 / kCovThreads;   // staged values per thread
constexpr int kFinReg = 4;          // slabs per lane held in registers by the finish (T <= 32768)

template <typename ZT>
__device__ __forceinline__ double ld_z(const void* Z, int64_t off) { return (double)static_cast<const ZT*>(Z)[off]; }

// grid (nslabs, ntile_pairs, D), block kCovThreads.
// partial: [D][nslabs][Np][Np] centred slab products; smean: [D][nslabs][N] slab means (written by
// the diagonal tiles, which are the only blocks covering each column once).
template <typename ZT>
__global__ __launch_bounds__(kCovThreads) void k_cov_slab(const void* __restrict__ Z, int64_t T, int64_t N,
                                                          int64_t Np, double* __restrict__ smean,
                                                          double* __restrict__ partial)
{
    __shared__ double zs[kSlab][33];          // the slab's rows x (16 columns of tile a | 16 of tile b)
    __shared__ double red[4][256];
    __shared__ double mcol[32];
    const int64_t d = blockIdx.z;
    const int slab = blockIdx.x, nslabs = gridDim.x;
    // tile pair index -> (ta, tb) with ta <= tb
    const int nt = (int)(Np / 16);
    int p = blockIdx.y, ta = 0;
    while (p >= nt - ta) { p -= nt - ta; ++ta; }
    const int tb = ta + p;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t s0 = (int64_t)slab * kSlab;
    const int rows = (int)min<int64_t>(kSlab, T - s0);

    // stage the slab: all loads in flight together; zero outside the matrix
    double v[kStageLd];
#pragma unroll
    for (int e = 0; e < kStageLd; ++e) {
        const int i = e * kCovThreads + tid, r = i >> 5, cs = i & 31;
        const int64_t col = cs < 16 ? ta * 16 + cs : tb * 16 + (cs - 16);
        v[e] = (r < rows && col < N) ? ld_z<ZT>(Z, (d * T + s0 + r) * N + col) : 0.0;
    }
#pragma unroll
    for (int e = 0; e < kStageLd; ++e) {
        const int i = e * kCovThreads + tid;
        zs[i >> 5][i & 31] = v[e];
    }
    __syncthreads();
    // slab means: 8 threads per column, 16 rows each, combined in a fixed order
    {
        const int cs = tid & 31, part = tid >> 5;
        double acc = 0.0;
        for (int r = part * (kSlab / 8); r < (part + 1) * (kSlab / 8); ++r) acc += zs[r][cs];
        red[0][tid] = acc;
    }
    __syncthreads();
    if (tid < 32) {
        double acc = 0.0;
        for (int part = 0; part < 8; ++part) acc += red[0][part * 32 + tid];
        const double m = acc / (double)rows;
        mcol[tid] = m;
        if (tid < 16 && ta == tb && ta * 16 + tid < N) smean[((int64_t)d * nslabs + slab) * N + ta * 16 + tid] = m;
    }
    __syncthreads();
    // centred contraction on the matrix cores: wave w takes rows w*32 .. w*32+31, four per MFMA
    const int kk = lane >> 4, cl = lane & 15;
    const double ma = mcol[cl], mb = mcol[16 + cl];
    double4_t acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int st = 0; st < kSlab / 4 / 4; ++st) {
        const int r = w * (kSlab / 4) + 4 * st + kk;
        const bool in = r < rows;
        const double a = in ? zs[r][cl] - ma : 0.0;
        const double b = in ? zs[r][16 + cl] - mb : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
    // Output layout of the 16x16x4 FP64 MFMA: lane holds D[lane/16 + 4v][lane%16], v = 0..3
    // (checked on gfx950 against the CPU covariance).
#pragma unroll
    for (int q = 0; q < 4; ++q) red[w][(kk + 4 * q) * 16 + cl] = acc[q];
    __syncthreads();
    {
        const double sum = ((red[0][tid] + red[1][tid]) + red[2][tid]) + red[3][tid];
        const int i = tid >> 4, j = tid & 15;
        partial[((d * nslabs + slab) * Np + (ta * 16 + i)) * Np + (tb * 16 + j)] = sum;
    }
}

// Sum over the 64 lanes in a fixed order; lane 0's value is returned to every lane.
__device__ __forceinline__ double wave_sum_fixed(double v)
{
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    return __shfl(v, 0);
}

// grid (ceil(npairs/4), D), block 256: one wave per upper-triangle entry (a <= b); lanes take slabs.
__global__ __launch_bounds__(256) void k_cov_finish(const double* __restrict__ partial,
                                                    const double* __restrict__ smean, int nslabs, int64_t T,
                                                    int64_t N, int64_t Np, double* __restrict__ Sigma)
{
    const int64_t d = blockIdx.y;
    const int lane = threadIdx.x & 63;
    int64_t e = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (e >= N * (N + 1) / 2) return;
    // e -> (a, b), a <= b, row-major over the upper triangle
    int64_t a = 0;
    while (e >= N - a) { e -= N - a; ++a; }
    const int64_t b = a + e;
    const double* ms = smean + (int64_t)d * nslabs * N;
    auto cnt = [&](int sl) { return (double)(min<int64_t>(T, (int64_t)(sl + 1) * kSlab) - (int64_t)sl * kSlab); };
    double ma = 0.0, mb = 0.0, s = 0.0;
    if (nslabs <= 64 * kFinReg) {
        // every load of the lane in flight together; the sums run in the same order as below
        double pa[kFinReg], pb[kFinReg], pp[kFinReg];
#pragma unroll
        for (int r = 0; r < kFinReg; ++r) {
            const int sl = lane + 64 * r;
            const bool in = sl < nslabs;
            pa[r] = in ? ms[sl * N + a] : 0.0;
            pb[r] = in ? ms[sl * N + b] : 0.0;
            pp[r] = in ? partial[((d * nslabs + sl) * Np + a) * Np + b] : 0.0;
        }
#pragma unroll
        for (int r = 0; r < kFinReg; ++r) {
            const int sl = lane + 64 * r;
            if (sl < nslabs) {
                ma += cnt(sl) * pa[r];
                mb += cnt(sl) * pb[r];
            }
        }
        ma = wave_sum_fixed(ma) / (double)T;
        mb = wave_sum_fixed(mb) / (double)T;
#pragma unroll
        for (int r = 0; r < kFinReg; ++r) {
            const int sl = lane + 64 * r;
            if (sl < nslabs) s += pp[r] + cnt(sl) * (pa[r] - ma) * (pb[r] - mb);
        }
    } else {
        for (int sl = lane; sl < nslabs; sl += 64) {
            ma += cnt(sl) * ms[sl * N + a];
            mb += cnt(sl) * ms[sl * N + b];
        }
        ma = wave_sum_fixed(ma) / (double)T;
        mb = wave_sum_fixed(mb) / (double)T;
        for (int sl = lane; sl < nslabs; sl += 64)
            s += partial[((d * nslabs + sl) * Np + a) * Np + b] + cnt(sl) * (ms[sl * N + a] - ma) * (ms[sl * N + b] - mb);
    }
    s = wave_sum_fixed(s) / (double)(T - 1);
    if (lane == 0) {
        Sigma[(d * N + a) * N + b] = s;
        Sigma[(d * N + b) * N + a] = s;     // the same value: Sigma is exactly symmetric
    }
}

}  // namespace

size_t cov_ws_bytes(int64_t D, int64_t T, int64_t N)
{
    const int64_t Np = (N + 15) / 16 * 16;
    const int64_t nslabs = (T + kSlab - 1) / kSlab;
    size_t off = kWsHeader;
    off = align_up(off + (size_t)D * nslabs * N * 8, 256);             // slab means
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
    double* smean = reinterpret_cast<double*>(base + off);
    off = align_up(off + (size_t)D * nslabs * N * 8, 256);
    double* partial = reinterpret_cast<double*>(base + off);
    if (D * N == 0) return THOI_OK;
    const int nt = (int)(Np / 16);
    dim3 gt((unsigned)nslabs, (unsigned)(nt * (nt + 1) / 2), (unsigned)D);
    dim3 gf((unsigned)((N * (N + 1) / 2 + 3) / 4), (unsigned)D);
    if (z_dtype == THOI_DTYPE_F64)
        hipLaunchKernelGGL(k_cov_slab<double>, gt, dim3(kCovThreads), 0, s, Z, T, N, Np, smean, partial);
    else
        hipLaunchKernelGGL(k_cov_slab<float>, gt, dim3(kCovThreads), 0, s, Z, T, N, Np, smean, partial);
    hipLaunchKernelGGL(k_cov_finish, gf, dim3(256), 0, s, partial, smean, (int)nslabs, T, N, Np, Sigma);
    return hip_status(hipGetLastError());
}

}  // namespace thoi
