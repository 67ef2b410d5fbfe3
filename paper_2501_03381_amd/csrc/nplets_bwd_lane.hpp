// Lane engine of the adjoint (included by nplets_bwd_lane_lo.hip and nplets_bwd_lane_hi.hip, which
// instantiate its register classes).
//
// grad_Sigma[d] += sum_b sum_m w_m(b, d) d measure_m(b, d) / d Sigma_d, entries of Sigma
// independent.  For an n-plet S with correlation sub-matrix R_S, P = R_S^-1, p_j = P_jj,
// d_j = Sigma_jj and c_T = w_TC + w_O + w_S, c_D = w_DTC - w_O + w_S (Eqs. O-info, S-info), the
// derivatives of TC = -1/2 log det R_S and DTC = 1/2 (log det R_S + sum log p_j) (Supplementary,
// Eq. gaussian_differential_entropy, with the cofactor form of the leave-one-out determinants) are
//   G_ij = { c_T/2 (delta_ij - P_ij) + c_D/2 (P_ij - (P diag(1/p) P)_ij) } / sqrt(d_i d_j).
// With t_i = sqrt(p_i) and the unit-diagonal Z = diag(1/t) P diag(1/t) (negated partial
// correlations), P = diag(t) Z diag(t) and P diag(1/p) P = diag(t) Z^2 diag(t), so
//   G_ij = c_T/2 delta_ij / d_i + u_i u_j [ (c_D - c_T)/2 Z_ij - c_D/2 (Z^2)_ij ],  u_i = t_i / sqrt(d_i),
// one length-k dot product per pair i >= j.
//
// One lane owns one n-plet, gathered from the correlation matrix staged in LDS (N <= 64) or from
// the covariance in global memory (larger N, scaled on the fly: LDS then holds only the
// accumulator and does not cap the occupancy).  L = chol(R_S), W = L^-1 and P = W^T W overwrite one packed FP64
// triangle in registers; Z, whose entries lie in [-1, 1], is then rounded to FP32 for the quadratic
// part (that rounding, about 6e-8 of the diagonal terms of G, is the size of the FP32 accumulation
// of the result), which halves the live state of the widest phase.  Contributions go with LDS
// atomics into the packed lower triangle of an N x N FP32 tile per workgroup (n-plet indices
// ascend, so c_i >= c_j); each workgroup flushes its tile once with float atomics.  Workgroups are
// persistent over the tiles (one n-plet per thread, one order per tile) of their class.
#pragma once

#include "nplets_bwd.hpp"
#include "nplets_common.hpp"

namespace thoi {
namespace {

__device__ __forceinline__ int ptri(int i, int j) { return i * (i + 1) / 2 + j; }   // i >= j

template <int K>
__device__ __forceinline__ void lane_adjoint(const int (&c)[K > 0 ? K : 1], const double* __restrict__ sR,
                                             const double* __restrict__ Sig, int N, const double* __restrict__ sIsd,
                                             double cT, double cD, float* __restrict__ sAcc)
{
    constexpr int NT = K * (K + 1) / 2;
    double a[NT > 0 ? NT : 1];
    // gather R_S (strict lower triangle; unit diagonal): from the staged correlation matrix, or
    // from the covariance in global memory scaled by 1/sqrt(Sigma_ii Sigma_jj)
    if (bwd_stage_matrix(N)) {
#pragma unroll
        for (int i = 0; i < K; ++i) {
            const double* row = sR + c[i] * N;
#pragma unroll
            for (int j = 0; j < i; ++j) a[tri(i, j)] = row[c[j]];
            a[tri(i, i)] = 1.0;
        }
    } else {
#pragma unroll
        for (int i = 0; i < K; ++i) {
            const int ri = c[i] * N;
            const double si = sIsd[c[i]];
#pragma unroll
            for (int j = 0; j < i; ++j) a[tri(i, j)] = Sig[ri + c[j]] * si * sIsd[c[j]];
            a[tri(i, i)] = 1.0;
        }
    }
    // Cholesky R_S = L L^T; the diagonal slot keeps 1 / L_jj
    bool ok = true;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const double p = a[tri(j, j)];
        ok = ok && (p > 0.0);
        const double r = rsqrt(p);
        a[tri(j, j)] = r;
#pragma unroll
        for (int i = j + 1; i < K; ++i) a[tri(i, j)] *= r;
#pragma unroll
        for (int i = j + 1; i < K; ++i) {
            const double lij = a[tri(i, j)];
#pragma unroll
            for (int m = j + 1; m <= i; ++m) a[tri(i, m)] -= lij * a[tri(m, j)];
        }
    }
    if (!ok) return;   // not positive definite: no contribution
    // W = L^-1 in place, column by column (W_jj = 1 / L_jj is already in the diagonal slot)
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const double wjj = a[tri(j, j)];
#pragma unroll
        for (int i = j + 1; i < K; ++i) {
            double s = a[tri(i, j)] * wjj;
#pragma unroll
            for (int m = j + 1; m < i; ++m) s += a[tri(i, m)] * a[tri(m, j)];
            a[tri(i, j)] = -s * a[tri(i, i)];
        }
    }
    // P = W^T W in place: P_ij (i >= j) = sum_{r >= i} W_ri W_rj.  Columns ascend and rows ascend
    // inside a column, so every W entry is read before it is overwritten.
    sfor<0, K>([&](auto J) {
        constexpr int j = J;
        sfor<j, K>([&](auto I) {
            constexpr int i = I;
            double s = a[tri(i, i)] * a[tri(i, j)];
            sfor<i + 1, K>([&](auto R) { s += a[tri(R, i)] * a[tri(R, j)]; });
            a[tri(i, j)] = s;
        });
    });
    // Z (rounded to FP32) and u
    float z[NT > 0 ? NT : 1];
    float u[K > 0 ? K : 1];
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const double r = rsqrt(a[tri(i, i)]);
#pragma unroll
        for (int j = 0; j < i; ++j) a[tri(i, j)] *= r;
#pragma unroll
        for (int m = i + 1; m < K; ++m) a[tri(m, i)] *= r;
        u[i] = (float)(a[tri(i, i)] * r * sIsd[c[i]]);
    }
#pragma unroll
    for (int e = 0; e < NT; ++e) z[e] = (float)a[e];
    const float hT = (float)(0.5 * cT), hDT = (float)(0.5 * (cD - cT)), hD = (float)(0.5 * cD);
    sfor<0, K>([&](auto I) {
        constexpr int i = I;
        const int rowi = ptri(c[i], 0);
        sfor<0, i + 1>([&](auto J) {
            constexpr int j = J;
            // (Z^2)_ij = sum_m Z_im Z_jm with Z_mm = 1
            float q = 0.0f;
            sfor<0, K>([&](auto M) {
                constexpr int m = M;
                const float zim = m == i ? 1.0f : (m < i ? z[tri(i, m)] : z[tri(m, i)]);
                const float zjm = m == j ? 1.0f : (m < j ? z[tri(j, m)] : z[tri(m, j)]);
                q = fmaf(zim, zjm, q);
            });
            const float zij = i == j ? 1.0f : z[tri(i, j)];
            // every product below depends on q, so none is computed ahead of its pair
            float g = fmaf(hDT, zij, -(hD * q));
            g = (g * u[j]) * u[i];
            if constexpr (i == j) {
                const double sd = sIsd[c[i]];
                g += (float)((double)hT * sd * sd);
            }
            atomicAdd(&sAcc[rowi + c[j]], g);
        });
    });
}

// Weights of one output position: c_T, c_D as above.  Returns false when both vanish.
__device__ __forceinline__ bool bwd_lane_weights(const BwdArgs& a, int d, int64_t pos, double& cT, double& cD)
{
    const int64_t o = (int64_t)d * a.B + pos;
    const int64_t plane = (int64_t)a.D * a.B;
    const double wTC = a.grad_out[o], wDTC = a.grad_out[plane + o];
    const double wO = a.grad_out[2 * plane + o], wS = a.grad_out[3 * plane + o];
    cT = wTC + wO + wS;
    cD = wDTC - wO + wS;
    return cT != 0.0 || cD != 0.0;
}

template <int K>
__device__ __forceinline__ void bwd_lane_task(const BwdArgs& a, int d, const double* __restrict__ sR,
                                              const double* __restrict__ Sig, const double* __restrict__ sIsd, const uint64_t* __restrict__ sBin,
                                              int kb, float* __restrict__ sAcc, int64_t first, int64_t pos0,
                                              int64_t local)
{
    int c[K > 0 ? K : 1];
    int64_t pos;
    if (a.mode == THOI_SEL_RANGE) {
        pos = pos0 + local;
        unrank_lex<K>((uint64_t)(first + local), a.N, sBin, kb, c);
    } else {
        pos = a.perm[first + local];
        if (a.mode == THOI_SEL_LIST) {
            const int32_t* row = a.idx + pos * a.kmax_list;
#pragma unroll
            for (int i = 0; i < K; ++i) c[i] = row[i];
        } else {
            uint64_t m = a.mask[pos];
#pragma unroll
            for (int i = 0; i < K; ++i) { c[i] = __builtin_ctzll(m); m &= m - 1; }
        }
    }
    double cT, cD;
    if (!bwd_lane_weights(a, d, pos, cT, cD)) return;
    lane_adjoint<K>(c, sR, Sig, a.N, sIsd, cT, cD, sAcc);
}

template <int K, int KHI>
__device__ __forceinline__ void bwd_lane_dispatch(int k, const BwdArgs& a, int d, const double* sR, const double* Sig,
                                                  const double* sIsd, const uint64_t* sBin, int kb, float* sAcc,
                                                  int64_t first, int64_t pos0, int64_t local)
{
    if (k == K) bwd_lane_task<K>(a, d, sR, Sig, sIsd, sBin, kb, sAcc, first, pos0, local);
    else if constexpr (K < KHI)
        bwd_lane_dispatch<K + 1, KHI>(k, a, d, sR, Sig, sIsd, sBin, kb, sAcc, first, pos0, local);
}

// grid (workgroups, D), block BS; workgroup x walks tiles (BS n-plets of one order) x, x + gridDim.x,
// ... of its class.
// RANGE: tab.p[i].tile0 is the piece's first tile and ntiles_range the class's tile count;
// LIST / MASK: tiles follow the per-order buckets of orders KLO..KHI.
template <int KLO, int KHI, int BS>
__global__ __launch_bounds__(BS) void k_bwd_lane(BwdArgs a, BwdTiles tab, int64_t ntiles_range)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int N = a.N;
    const int d = blockIdx.y;
    const bool range = a.mode == THOI_SEL_RANGE;
    const int kb = range ? KHI : 0;
    const bool staged = bwd_stage_matrix(N);
    double* sR = reinterpret_cast<double*>(smem);
    const size_t off = staged ? bwd_align16((size_t)N * N * 8) : 0;
    double* sIsd = reinterpret_cast<double*>(smem + off);
    double* sLogd = sIsd + N;
    uint64_t* sBin = reinterpret_cast<uint64_t*>(sLogd + N);
    float* sAcc = reinterpret_cast<float*>(smem + bwd_align16(off + (size_t)N * 16 + (size_t)N * kb * 8));
    const int NTN = N * (N + 1) / 2;
    for (int e = threadIdx.x; e < NTN; e += blockDim.x) sAcc[e] = 0.0f;
    const double* Sig = a.Sigma + (int64_t)d * N * N;
    if (staged) {
        stage_corr<double>(Sig, N, sR, sIsd, sLogd, range ? sBin : nullptr, kb);
    } else {
        for (int j = threadIdx.x; j < N; j += blockDim.x) {
            const double dj = Sig[(int64_t)j * N + j];
            sIsd[j] = dj > 0.0 ? 1.0 / sqrt(dj) : __builtin_nan("");
        }
        if (range) stage_binomials(N, kb, sBin);
        __syncthreads();
    }

    int64_t ntiles = ntiles_range;
    if (!range) {
        ntiles = 0;
        for (int kk = KLO; kk <= KHI; ++kk) ntiles += (a.lcnt[kk] + BS - 1) / BS;
    }
    bool any = false;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        int k = -1;
        int64_t first = 0, pos0 = 0, cnt = 0, tb = 0;
        if (range) {
            for (int p = 0; p < tab.n; ++p) {
                const int64_t nt = (tab.p[p].cnt + BS - 1) / BS;
                if (t >= tab.p[p].tile0 && t < tab.p[p].tile0 + nt) {
                    k = tab.p[p].k; first = tab.p[p].first; pos0 = tab.p[p].pos0; cnt = tab.p[p].cnt;
                    tb = (t - tab.p[p].tile0) * BS;
                }
            }
        } else {
            int64_t t0 = 0;
            for (int kk = KLO; kk <= KHI; ++kk) {
                const int64_t c = a.lcnt[kk];
                const int64_t nt = (c + BS - 1) / BS;
                if (t >= t0 && t < t0 + nt) { k = kk; first = a.lbase[kk]; cnt = c; tb = (t - t0) * BS; }
                t0 += nt;
            }
        }
        if (k < 0) continue;   // uniform
        any = true;
        const int64_t local = tb + threadIdx.x;
        if (local < cnt) bwd_lane_dispatch<KLO, KHI>(k, a, d, sR, Sig, sIsd, sBin, kb, sAcc, first, pos0, local);
    }
    __syncthreads();
    if (!any) return;   // uniform
    float* G = a.grad_Sigma + (int64_t)d * N * N;
    for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
        const int r = e / N, s = e - r * N;
        const float v = sAcc[r >= s ? ptri(r, s) : ptri(s, r)];
        if (v != 0.0f) unsafeAtomicAdd(&G[e], v);
    }
}

template <int KLO, int KHI, int BS>
void bwd_lane_launch_one(const BwdArgs& a, const BwdTiles& t, int64_t ntiles, dim3 grid, size_t lds, hipStream_t s)
{
    hipLaunchKernelGGL((k_bwd_lane<KLO, KHI, BS>), grid, dim3(BS), lds, s, a, t, ntiles);
}

template <int KLO, int KHI, int BS>
int bwd_lane_blocks_one(size_t lds)
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(k_bwd_lane<KLO, KHI, BS>),
                                                     BS, lds) != hipSuccess || n < 1)
        n = 1;
    return n;
}

}  // namespace
}  // namespace thoi
