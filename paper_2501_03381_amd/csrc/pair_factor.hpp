// Two n-plets per wavefront, rows in registers: the factorisation of the pair engine (orders up to
// kW2Max), shared by the evaluation, refinement and search kernels.  Each half-wave (32 lanes)
// factors one n-plet; lane i keeps row i of the sub-matrix in registers, indexed by compile-time
// constants only.  Only the lanes of one wavefront exchange data through LDS, so no workgroup
// barrier is needed: LDS operations of one wavefront complete in issue order, and a
// wavefront-scope fence keeps the compiler from reordering them.
#pragma once

#include "nplets_wave2.hpp"

namespace thoi {

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double half_sum(double v)
{
#pragma unroll
    for (int o = 16; o > 0; o >>= 1) v += __shfl_xor(v, o, 32);
    return v;
}
__device__ __forceinline__ double half_max(double v)
{
#pragma unroll
    for (int o = 16; o > 0; o >>= 1) {
        const double u = __shfl_xor(v, o, 32);
        v = v > u ? v : u;
    }
    return v;
}

// Factor the n-plet cidx[0..kh-1] of this half-wave (lane i = row i).  Both halves of the
// wavefront pass the same k (>= the kh of each): the loops run to k.  GLOBAL: entries from the
// covariance Sig in global memory, scaled by 1/sqrt(Sigma_ii Sigma_jj) (each half may have its
// own dataset); otherwise from the staged correlation matrix sR.  col and wrow: two buffers of 32
// doubles each, per half.  Returns the FactorOut in every lane.  SEQ: the two log sums are taken
// by the half's lane 0 in row order instead of by a lane tree, so inserting an independent
// variable (a zero row and column) changes no bit of them.
template <bool GLOBAL, bool SEQ = false>
__device__ __forceinline__ FactorOut<double> pair_factor(const double* __restrict__ sR, int N,
                                                         const int* __restrict__ cidx, int k_in, int kh,
                                                         double* __restrict__ col, double* __restrict__ wrow)
{
    const int k = __builtin_amdgcn_readfirstlane(k_in);   // uniform: scalar loop guards
    const int i = threadIdx.x & 31;
    const bool mine = i < kh;
    const int ci = mine ? cidx[i] : 0;
    double r[kW2Max];
    double si = 1.0;
    if constexpr (GLOBAL) {
        // lane i scales its row by 1/sqrt(Sigma_ii) and publishes the factor for the columns
        const double di = sR[(int64_t)ci * N + ci];
        si = di > 0.0 ? 1.0 / sqrt(di) : __builtin_nan("");
        wrow[i] = si;
        wave_sync();
    }
    // Gather: every load of a group of four columns is issued before any is used (an unused
    // lane reads a valid entry and discards it); r[] is indexed by constants only.
    sfor<0, kW2Max>([&](auto M) {
        constexpr int m = M;
        r[m] = (m == i && mine) ? 1.0 : 0.0;
    });
    sfor<0, kW2Max / 4>([&](auto G) {
        constexpr int g = G;
        if (4 * g < k) {
            double e[4];
            sfor<0, 4>([&](auto U) {
                constexpr int u = U;
                const int cm = 4 * g + u < kh ? cidx[4 * g + u] : 0;
                if constexpr (GLOBAL) e[u] = sR[(int64_t)ci * N + cm];
                else e[u] = sR[ci * N + cm];
            });
            sfor<0, 4>([&](auto U) {
                constexpr int u = U, m = 4 * g + u;
                if constexpr (GLOBAL) e[u] *= si * wrow[m];
                if (m < i && mine) r[m] = e[u];
            });
        }
    });
    if constexpr (GLOBAL) wave_sync();          // wrow is reused below
    // Right-looking Cholesky.  Lane i's entries r[m] with m > i, and every entry of a lane beyond
    // the order, are never read for the result; the updates below run on them too, so that the
    // inner loops need no per-lane condition (column entries beyond the order are stale but in
    // bounds).  The update loops are guarded in groups of four columns by the uniform order.
    double piv = 1.0;
    sfor<0, kW2Max>([&](auto J) {
        constexpr int j = J;
        if (j < k) {
            double* cl = col + (j & 1) * kW2Max;
            cl[i] = r[j];                                 // a_ij of the current Schur complement
            wave_sync();
            const double p = cl[j];
            const double rs = rsqrt(p);
            const double aij = r[j];
            const double t = aij * rs * rs;               // a_ij / a_jj
            piv = i == j ? p : piv;
            r[j] = i == j ? rs : aij * rs;                // 1 / L_jj on the diagonal, L_ij below
            sfor<(j + 1) / 4, kW2Max / 4>([&](auto G) {
                constexpr int g = G;
                if (4 * g < k) {
                    sfor<4 * g, 4 * g + 4>([&](auto M) {
                        constexpr int m = M;
                        if constexpr (m > j) r[m] -= t * cl[m];
                    });
                }
            });
        }
    });
    // W = L^-1 row by row.  Lane i holds L_im in r[m] (m < i) and 1 / L_ii in r[i]; at step t it
    // adds L_it W_t to the running sum of its row, stored in r[0..t] as L_it is consumed (a lane
    // whose row is published no longer needs its registers).  Column norms accumulate in aj.
    double aj = 0.0;
    sfor<0, kW2Max>([&](auto T) {
        constexpr int t = T;
        if (t < k) {
            double* wr = wrow + (t & 1) * kW2Max;
            if (i == t) {
                sfor<0, t + 1>([&](auto M) {
                    constexpr int m = M;
                    wr[m] = m < t ? -r[m] * r[t] : r[t];
                });
            }
            wave_sync();
            const double w = wr[i];
            aj += (i <= t && t < kh) ? w * w : 0.0;      // rows of this half's own n-plet only
            const double lit = r[t];
            sfor<0, t>([&](auto M) {
                constexpr int m = M;
                r[m] += lit * wr[m];
            });
            r[t] = lit * wr[t];
        }
    });
    FactorOut<double> o;
    if constexpr (SEQ) {
        wave_sync();                                      // every lane has read its last W row
        wrow[i] = mine ? log(piv) : 0.0;
        wrow[kW2Max + i] = mine ? log(aj) : 0.0;
        wave_sync();
        double s1 = 0.0, s2 = 0.0;
        if (i == 0) {
            for (int m = 0; m < kh; ++m) { s1 += wrow[m]; s2 += wrow[kW2Max + m]; }
        }
        o.ld = __shfl(s1, 0, 32);
        o.sa = __shfl(s2, 0, 32);
    } else {
        o.ld = half_sum(mine ? log(piv) : 0.0);
        o.sa = half_sum(mine ? log(aj) : 0.0);
    }
    o.vmax = half_max(mine ? aj : 0.0);
    o.ok = half_sum((mine && !(piv > 0.0)) ? 1.0 : 0.0) == 0.0;
    wave_sync();
    return o;
}

}  // namespace thoi
