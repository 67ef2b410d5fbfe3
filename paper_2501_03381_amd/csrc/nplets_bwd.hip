// Adjoint of the n-plet evaluation on gfx950:
//   grad_Sigma[d] += sum_b sum_m w_m(b, d) d measure_m(b, d) / d Sigma_d
// with the entries of Sigma treated as independent.
//
// For an n-plet S with sub-matrix Sigma_S, A = Sigma_S^-1, a_j = A_jj, d_j = Sigma_jj, the
// Gaussian entropy (Supplementary, Eq. gaussian_differential_entropy) and the cofactor form of
// the leave-one-out determinants give TC = 1/2[sum log d_j - log det Sigma_S] and
// DTC = 1/2[log det Sigma_S + sum log a_j], hence (d log det / d Sigma = A,
// d a_j / d Sigma_pq = -A_jp A_qj):
//   dTC/dSigma_S  = 1/2 [diag(1/d) - A]
//   dDTC/dSigma_S = 1/2 [A - A diag(1/a) A]
// and Omega = TC - DTC, S = TC + DTC (Eqs. O-info, S-info).  In terms of the correlation
// inverse P = R_S^-1 (p_j = P_jj): A_ij = P_ij / sqrt(d_i d_j) and
// (A diag(1/a) A)_ij = (P diag(1/p) P)_ij / sqrt(d_i d_j), so with c_T = w_TC + w_O + w_S and
// c_D = w_DTC - w_O + w_S:
//   G_ij = { c_T/2 (delta_ij - P_ij) + c_D/2 (P_ij - (P diag(1/p) P)_ij) } / sqrt(d_i d_j).
//
// Work decomposition: one wavefront per n-plet (FP64, runtime order, so LIST rows need no
// bucketing); P = W^T W from the triangular inverse W = L^-1 that the factorisation leaves in
// LDS.  Each workgroup accumulates its n-plets' contributions in an LDS N x N FP32 tile (lane i
// owns row c_i, so the adds of one wavefront never collide) and flushes it once with hardware
// float atomics.
#include "nplets_common.hpp"

namespace thoi {
namespace {

constexpr int64_t kBwdTileMin = 16;     // n-plets per workgroup, bounds of the host's choice
constexpr int64_t kBwdTileMax = 4096;
constexpr int64_t kLdsPerCu = 160 * 1024;
constexpr int64_t kCus = 256;

struct BwdArgs {
    const double* Sigma;
    int32_t N, D;
    int64_t B;
    const float* grad_out;      // [4][D][B]
    float* grad_Sigma;          // [D][N][N]
    int32_t mode;
    int32_t kmin, kmax;         // RANGE
    int64_t g_begin;
    int64_t ostart[THOI_MAX_K + 2];
    const int32_t* idx;
    int32_t kmax_list;
    const uint64_t* mask;
    int32_t ks;                 // LDS row stride (>= largest order + 1)
    int64_t tile;               // n-plets per workgroup
};

// LDS: sIsd [N] f64 | sBin [N*64] u64 (RANGE) | sM [64*ks] f64 | sP [64*ks] f64 | sInv [64] f64 |
//      sAcc [N*N] f32 | cidx [64] i32
__host__ __device__ inline size_t bwd_lds_bytes(int N, int ks, bool range)
{
    size_t off = (size_t)N * 8 + (range ? (size_t)N * 64 * 8 : 0);
    off += 2 * (size_t)64 * ks * 8 + 64 * 8;
    off += (size_t)N * N * 4 + 64 * 4;
    return off;
}

template <int MODE>
__global__ __launch_bounds__(64) void k_backward(BwdArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int N = a.N, ks = a.ks;
    const int d = blockIdx.y;
    const int lane = threadIdx.x;
    double* sIsd = reinterpret_cast<double*>(smem);
    uint64_t* sBin = reinterpret_cast<uint64_t*>(sIsd + N);
    double* sM = reinterpret_cast<double*>(sBin + (MODE == THOI_SEL_RANGE ? N * 64 : 0));
    double* sP = sM + 64 * ks;
    double* sInv = sP + 64 * ks;
    float* sAcc = reinterpret_cast<float*>(sInv + 64);
    int* cidx = reinterpret_cast<int*>(sAcc + N * N);
    __shared__ int sk;

    const double* Sig = a.Sigma + (int64_t)d * N * N;
    for (int j = lane; j < N; j += 64) {
        const double dj = Sig[(int64_t)j * N + j];
        sIsd[j] = dj > 0.0 ? 1.0 / sqrt(dj) : __builtin_nan("");
    }
    for (int e = lane; e < N * N; e += 64) sAcc[e] = 0.0f;
    if constexpr (MODE == THOI_SEL_RANGE) stage_binomials(N, 64, sBin);
    __syncthreads();

    const int64_t b0 = (int64_t)blockIdx.x * a.tile;
    const int64_t b1 = b0 + a.tile < a.B ? b0 + a.tile : a.B;
    bool touched = false;
    for (int64_t pos = b0; pos < b1; ++pos) {
        const int64_t o = (int64_t)d * a.B + pos;
        const float wTC = a.grad_out[o], wDTC = a.grad_out[(int64_t)a.D * a.B + o];
        const float wO = a.grad_out[2 * (int64_t)a.D * a.B + o], wS = a.grad_out[3 * (int64_t)a.D * a.B + o];
        const double cT = (double)wTC + (double)wO + (double)wS;
        const double cD = (double)wDTC - (double)wO + (double)wS;
        if (cT == 0.0 && cD == 0.0) continue;   // uniform across the wave
        if (lane == 0) {
            int k = 0;
            if constexpr (MODE == THOI_SEL_RANGE) {
                const int64_t g = a.g_begin + pos;
                k = a.kmin;
                while (k < a.kmax && g >= a.ostart[k + 1]) ++k;
                unrank_lex_rt((uint64_t)(g - a.ostart[k]), N, k, sBin, 64, cidx);
            } else if constexpr (MODE == THOI_SEL_LIST) {
                const int32_t* row = a.idx + pos * a.kmax_list;
                bool ok = true;
                int prev = -1;
                while (k < a.kmax_list && row[k] >= 0) {
                    ok = ok && row[k] > prev && row[k] < N;
                    prev = row[k];
                    cidx[k] = row[k];
                    ++k;
                }
                if (!ok || k > 64) k = -1;   // invalid rows contribute nothing
            } else {
                uint64_t m = a.mask[pos];
                if (N < 64 && (m >> N) != 0) m = 0, k = -1;
                while (m) { cidx[k++] = __builtin_ctzll(m); m &= m - 1; }
            }
            sk = k;
        }
        __syncthreads();
        const int k = sk;
        if (k <= 0) { __syncthreads(); continue; }
        // correlation sub-matrix rows, lane i owns row i
        if (lane < k) {
            const int ci = cidx[lane];
            for (int j = 0; j < lane; ++j) {
                const int cj = cidx[j];
                sM[lane * ks + j] = Sig[(int64_t)ci * N + cj] * sIsd[ci] * sIsd[cj];
            }
            sM[lane * ks + lane] = 1.0;
        }
        __syncthreads();
        // Cholesky (right-looking) and W = L^-1: same steps as the forward wave engine
        bool ok = true;
        for (int j = 0; j < k; ++j) {
            const double p = sM[j * ks + j];
            ok = ok && (p > 0.0);
            const double r = rsqrt(p);
            if (lane == j) sInv[j] = r;
            if (lane > j && lane < k) sM[lane * ks + j] *= r;
            __syncthreads();
            if (lane > j && lane < k) {
                const double l = sM[lane * ks + j];
                for (int m = j + 1; m <= lane; ++m) sM[lane * ks + m] -= l * sM[m * ks + j];
            }
            __syncthreads();
        }
        if (!ok) { __syncthreads(); continue; }   // not positive definite: no contribution
        if (lane < k) {
            const int j = lane;
            const double wjj = sInv[j];
            for (int i = j + 1; i < k; ++i) {
                double s = sM[i * ks + j] * wjj;
                for (int m = j + 1; m < i; ++m) s += sM[i * ks + m] * sM[j * ks + m];
                sM[j * ks + i] = -s * sInv[i];     // W_ij kept in row j, column i > j
            }
            sM[j * ks + j] = wjj;                  // row j now holds W_jj .. W_{k-1,j}
        }
        __syncthreads();
        // P = W^T W: P_ij = sum_{r >= max(i,j)} W_ri W_rj
        if (lane < k) {
            const int i = lane;
            for (int j = i; j < k; ++j) {
                double s = 0.0;
                for (int r = j; r < k; ++r) s += sM[i * ks + r] * sM[j * ks + r];
                sP[i * ks + j] = s;
                sP[j * ks + i] = s;
            }
        }
        __syncthreads();
        // U = P diag(1/p) in the rows of sM (W is no longer needed): one reciprocal per column,
        // then (P diag(1/p) P)_ij = sum_m U_im P_jm (P symmetric; row j is the same for every lane)
        if (lane < k) sInv[lane] = 1.0 / sP[lane * ks + lane];
        __syncthreads();
        if (lane < k) {
            for (int m = 0; m < k; ++m) sM[lane * ks + m] = sP[lane * ks + m] * sInv[m];
        }
        // G row i, scattered into the accumulator row c_i (lane i reads only its own row of U)
        if (lane < k) {
            const int i = lane;
            const int ci = cidx[i];
            for (int j = 0; j < k; ++j) {
                double q = 0.0;
                for (int m = 0; m < k; ++m) q += sM[i * ks + m] * sP[j * ks + m];
                const double pij = sP[i * ks + j];
                const double g = 0.5 * cT * ((i == j ? 1.0 : 0.0) - pij) + 0.5 * cD * (pij - q);
                const int cj = cidx[j];
                sAcc[ci * N + cj] += (float)(g * sIsd[ci] * sIsd[cj]);
            }
        }
        touched = true;
        __syncthreads();
    }
    __syncthreads();
    if (touched) {
        float* G = a.grad_Sigma + (int64_t)d * N * N;
        for (int e = lane; e < N * N; e += 64) {
            const float v = sAcc[e];
            if (v != 0.0f) unsafeAtomicAdd(&G[e], v);
        }
    }
}

}  // namespace

size_t backward_ws_bytes(int64_t D, int32_t N, const thoi_nplets* sel, const thoi_eval_opts* opts)
{
    (void)D; (void)N; (void)sel; (void)opts;
    return 0;
}

size_t backward_lds_bytes(int32_t N, const thoi_nplets* sel)
{
    const int kmax = sel->mode == THOI_SEL_RANGE ? sel->kmax : (sel->mode == THOI_SEL_LIST ? sel->kmax_list : N);
    const int ks = (kmax < 64 ? kmax : 64) + 1;
    return bwd_lds_bytes(N, ks, sel->mode == THOI_SEL_RANGE);
}

thoi_status launch_backward(const double* Sigma, int64_t D, int32_t N, const thoi_nplets* sel,
                            const thoi_eval_opts* opts, const float* grad_out, float* grad_Sigma, void* ws,
                            size_t ws_bytes, hipStream_t s)
{
    (void)opts; (void)ws; (void)ws_bytes;
    BwdArgs a{};
    a.Sigma = Sigma;
    a.N = N;
    a.D = (int32_t)D;
    a.B = sel->mode == THOI_SEL_RANGE ? sel->g_count : sel->B;
    a.grad_out = grad_out;
    a.grad_Sigma = grad_Sigma;
    a.mode = sel->mode;
    a.idx = sel->idx;
    a.kmax_list = sel->kmax_list;
    a.mask = sel->mask;
    int kmax;
    if (sel->mode == THOI_SEL_RANGE) {
        a.kmin = sel->kmin;
        a.kmax = sel->kmax;
        a.g_begin = sel->g_begin;
        int64_t g = 0;
        for (int k = sel->kmin; k <= sel->kmax + 1 && k <= THOI_MAX_K + 1; ++k) {
            a.ostart[k] = g;
            if (k <= sel->kmax) g += (int64_t)binom_u64(N, k);
        }
        kmax = sel->kmax;
    } else if (sel->mode == THOI_SEL_LIST) {
        kmax = sel->kmax_list;
    } else {
        kmax = N;
    }
    a.ks = (kmax < 64 ? kmax : 64) + 1;
    if (D == 0 || a.B == 0) return THOI_OK;
    const size_t lds = bwd_lds_bytes(N, a.ks, sel->mode == THOI_SEL_RANGE);
    // one round of workgroups: as many per dataset as the LDS footprint lets the CUs hold at once
    // (each workgroup flushes its accumulator tile once, so fewer, longer workgroups also mean
    // fewer atomics)
    const int64_t per_cu = (int64_t)(kLdsPerCu / (int64_t)(lds > 0 ? lds : 1));
    const int64_t resident = kCus * (per_cu > 0 ? per_cu : 1);
    const int64_t per_d = (resident + D - 1) / D;
    int64_t tile = (a.B + per_d - 1) / per_d;
    tile = tile < kBwdTileMin ? kBwdTileMin : (tile > kBwdTileMax ? kBwdTileMax : tile);
    a.tile = tile;
    const int64_t nblk = (a.B + tile - 1) / tile;
    if (nblk > 0x7fffffff) return THOI_EUNSUPPORTED;
    dim3 grid((unsigned)nblk, (unsigned)D);
    if (sel->mode == THOI_SEL_RANGE) hipLaunchKernelGGL(k_backward<THOI_SEL_RANGE>, grid, dim3(64), lds, s, a);
    else if (sel->mode == THOI_SEL_LIST) hipLaunchKernelGGL(k_backward<THOI_SEL_LIST>, grid, dim3(64), lds, s, a);
    else hipLaunchKernelGGL(k_backward<THOI_SEL_MASK>, grid, dim3(64), lds, s, a);
    return hip_status(hipGetLastError());
}

}  // namespace thoi
