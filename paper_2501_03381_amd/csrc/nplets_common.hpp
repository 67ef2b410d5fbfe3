// Device building blocks of the n-plet evaluation (forward and adjoint), gfx950.
//
// Per n-plet S of order k the measures need log det Sigma_S, every leave-one-out
// log det Sigma_{S\j} and the variances Sigma_jj (Methods, "Parallel and batched computation of
// HOI").  All four measures are invariant to rescaling each variable, so the kernels work on
// the correlation matrix R = D^-1/2 Sigma D^-1/2 (unit diagonal) and use one Cholesky
// factorisation R_S = L L^T per n-plet:
//   ld   = log det R_S            = sum_j log L_jj^2
//   a_j  = (R_S^-1)_jj            = sum_{r>=j} (L^-1)_rj^2    (variance-inflation factor VIF_j)
//   log det R_{S\j} = ld + log a_j                             (cofactor identity)
// so that, from the Gaussian entropy (Supplementary, Eq. gaussian_differential_entropy) and
// Eqs. (TC), (DTC), (O-info), (S-info):
//   TC = -ld/2,  DTC = (ld + sum_j log a_j)/2,  Omega = TC - DTC,  S = TC + DTC.
#pragma once

#include <type_traits>

#include "thoi_internal.hpp"

namespace thoi {

constexpr double kLn2 = 0.69314718055994530942;
constexpr double kLog2PiE = 2.8378770664093454836;   // log(2 pi e)

// ------------------------------------------------------------------------------------------------
// Precision traits
// ------------------------------------------------------------------------------------------------
template <typename F> struct Num;
template <> struct Num<float> {
    static __device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
    static __device__ __forceinline__ float mant(float x) { return __builtin_amdgcn_frexp_mantf(x); }
    static __device__ __forceinline__ int expo(float x) { return __builtin_amdgcn_frexp_expf(x); }
    static __device__ __forceinline__ float log2m(float m) { return __builtin_amdgcn_logf(m); }   // m in [1/2, 1)
};
template <> struct Num<double> {
    static __device__ __forceinline__ double rsq(double x) { return rsqrt(x); }
    static __device__ __forceinline__ double mant(double x) { return __builtin_amdgcn_frexp_mant(x); }
    static __device__ __forceinline__ int expo(double x) { return __builtin_amdgcn_frexp_exp(x); }
    static __device__ __forceinline__ double log2m(double m) { return log2(m); }
};

// Compile-time loop: fn(integral_constant<int, B>), ..., fn(integral_constant<int, E - 1>).  Used
// for the nests whose inner trip counts depend on the outer index: #pragma unroll does not always
// unroll them fully, which would leave the triangle dynamically indexed, i.e. in scratch memory.
template <int B, int E, typename Fn>
__device__ __forceinline__ void sfor(Fn&& fn)
{
    if constexpr (B < E) {
        fn(std::integral_constant<int, B>{});
        sfor<B + 1, E>(fn);
    }
}

// Running product kept as mantissa * 2^exponent, so products of up to 64 pivots or VIFs never
// leave the normal range.
template <typename F> struct LogProd {
    F m = F(1);
    int e = 0;
    __device__ __forceinline__ void mul(F x) { m *= x; }
    __device__ __forceinline__ void renorm() { e += Num<F>::expo(m); m = Num<F>::mant(m); }
    __device__ __forceinline__ F log() const { return (Num<F>::log2m(Num<F>::mant(m)) + F(e + Num<F>::expo(m))) * F(kLn2); }
};

// Pascal's triangle C(n, m), n, m < 64, exact in uint64 (C(63, 31) < 2^60), built at compile time.
struct PascalTable {
    uint64_t v[64][64];
};
constexpr PascalTable make_pascal()
{
    PascalTable t{};
    for (int n = 0; n < 64; ++n)
        for (int m = 0; m < 64; ++m)
            t.v[n][m] = m == 0 ? 1ull : (n == 0 ? 0ull : t.v[n - 1][m - 1] + t.v[n - 1][m]);
    return t;
}
__device__ constexpr PascalTable kPascal = make_pascal();

// 1/n for n = 1..63 (entry 0 is 0), correctly rounded at compile time.
struct RecipTable {
    double v[64];
};
constexpr RecipTable make_recip()
{
    RecipTable t{};
    t.v[0] = 0.0;
    for (int n = 1; n < 64; ++n) t.v[n] = 1.0 / n;
    return t;
}
__device__ constexpr RecipTable kRecip = make_recip();

// ------------------------------------------------------------------------------------------------
// Staging of one dataset into LDS: R (precision F), 1/sqrt(Sigma_jj) and log Sigma_jj (FP64).
// Must be called by the whole block (after a barrier if the block has used the LDS before); ends
// with a barrier.  Each thread issues the loads of its first 8 entries together with its diagonal
// load; N threads compute 1/sqrt(Sigma_jj) and log Sigma_jj once into LDS, and after a barrier
// every entry is scaled by two of them (entries beyond the first 8 * blockDim are loaded in
// further batches of 8).
// ------------------------------------------------------------------------------------------------
// With sBin, the block also copies C(n, m), n < N, m < kb, into sBin[n * kb + m]; the first
// entries' loads go out with the correlation loads.
template <typename F>
__device__ __forceinline__ void stage_corr(const double* __restrict__ Sig, int N, F* __restrict__ sR,
                                           double* __restrict__ sIsd, double* __restrict__ sLogd,
                                           uint64_t* __restrict__ sBin = nullptr, int kb = 0)
{
    const int NN = N * N;
    const int bd = (int)blockDim.x;
    const int nbin = sBin ? N * kb : 0;
    const int tid = (int)threadIdx.x;
    const uint64_t b0 = tid < nbin ? kPascal.v[tid / kb][tid % kb] : 0ull;
    // first batch of entries and the diagonal in flight together
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int e = tid + u * bd;
        v[u] = e < NN ? Sig[e] : 0.0;
    }
    // one reciprocal square root and one log per variable
    for (int j = tid; j < N; j += bd) {
        const double dj = Sig[(int64_t)j * N + j];
        sIsd[j] = dj > 0.0 ? 1.0 / sqrt(dj) : __builtin_nan("");
        sLogd[j] = log(dj);
    }
    if (tid < nbin) sBin[tid] = b0;
    for (int e = tid + bd; e < nbin; e += bd) sBin[e] = kPascal.v[e / kb][e % kb];
    __syncthreads();
    for (int e0 = tid; e0 < NN; e0 += 8 * bd) {
        if (e0 != tid) {
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int e = e0 + u * bd;
                v[u] = e < NN ? Sig[e] : 0.0;
            }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = e0 + u * bd;
            if (e < NN) {
                const int i = e / N, j = e - i * N;
                const double si = sIsd[i], sj = sIsd[j];
                sR[e] = (F)((i == j) ? (si == si ? 1.0 : __builtin_nan("")) : v[u] * si * sj);
            }
        }
    }
    __syncthreads();
}

// C(n, m), n < N, m < kb, into LDS at [n * kb + m] (kb <= 64), copied from the compile-time table
// with all loads of a thread in flight together.  Caller synchronises afterwards.
__device__ __forceinline__ void stage_binomials(int N, int kb, uint64_t* __restrict__ sBin)
{
    const int tot = N * kb;
    const int bd = (int)blockDim.x;
    for (int e0 = threadIdx.x; e0 < tot; e0 += 8 * bd) {
        uint64_t v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = e0 + u * bd;
            v[u] = e < tot ? kPascal.v[e / kb][e % kb] : 0ull;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = e0 + u * bd;
            if (e < tot) sBin[e] = v[u];
        }
    }
}

// Lexicographic unranking: rank r (0 <= r < C(N, K)) -> the r-th K-subset of {0..N-1} in the
// order of Python's itertools.combinations.  sBin holds C(n, m) at [n * kb + m], m < kb, kb >= K.
template <int K>
__device__ __forceinline__ void unrank_lex(uint64_t r, int N, const uint64_t* __restrict__ sBin, int kb,
                                           int (&c)[K > 0 ? K : 1])
{
    if (N <= 33) {
        // One pass over the candidate values x = 0..N-1, the same number of steps in every lane.
        // b = C(N-1-x, m) (m: binomial column of the next free position) is carried in FP64 and
        // updated by C(n-1, m) = C(n, m) (n-m) / n after a skip and C(n-1, m-1) = C(n, m) m / n
        // after a take.  With n < 33 every C(n, m) is below 2^32 and every product b * f below
        // 2^37, so b * f * (1/n) lies within 2^-15 of the integer quotient and rounding recovers it
        // exactly; the taken values are collected in a bit mask.
        if constexpr (K >= 1) {
            double rr = (double)(uint32_t)r;
            double b = (double)(uint32_t)kPascal.v[N - 1][K - 1];
            int m = K - 1;
            uint64_t mask = 0;
            for (int x = 0; x < N; ++x) {
                const int n = N - 1 - x;
                const double inv = kRecip.v[n];
                const bool take = rr < b;
                const double bt = rint(b * (double)m * inv);
                const double bs = rint(b * (double)(n - m) * inv);
                rr = take ? rr : rr - b;
                b = take ? bt : bs;
                m -= take ? 1 : 0;
                mask |= take ? (1ull << x) : 0ull;
            }
#pragma unroll
            for (int i = 0; i < K; ++i) {
                c[i] = __builtin_ctzll(mask);
                mask &= mask - 1;
            }
        }
        return;
    }
    int x = 0;
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const int m = K - 1 - i;
        if (m == 0) {
            c[i] = x + (int)r;
        } else {
            while (x < N) {
                const uint64_t b = sBin[(N - 1 - x) * kb + m];
                if (r < b) break;
                r -= b;
                ++x;
            }
            c[i] = x;
            ++x;
        }
    }
}

// Runtime-order version of the same unranking (one lane).
__device__ __forceinline__ int unrank_lex_rt(uint64_t r, int N, int k, const uint64_t* __restrict__ sBin, int kb,
                                             int* __restrict__ c)
{
    int x = 0;
    for (int i = 0; i < k; ++i) {
        const int m = k - 1 - i;
        if (m == 0) {
            c[i] = x + (int)r;
        } else {
            while (x < N) {
                const uint64_t b = sBin[(N - 1 - x) * kb + m];
                if (r < b) break;
                r -= b;
                ++x;
            }
            c[i] = x;
            ++x;
        }
    }
    return k;
}

// ------------------------------------------------------------------------------------------------
// Lane engine: one lane factors one n-plet of compile-time order K held in registers.
// ------------------------------------------------------------------------------------------------
template <typename F>
struct FactorOut {
    F ld;      // log det R_S
    F sa;      // sum_j log a_j
    F vmax;    // max_j a_j
    bool ok;   // every pivot > 0
};

constexpr int tri(int i, int j) { return i * (i + 1) / 2 + j; }

// packed lower triangle of an order-K matrix (at least one slot)
template <int K> constexpr int kTri = K * (K + 1) / 2 > 0 ? K * (K + 1) / 2 : 1;

// Factor R_S in registers; entry(i, j) (j < i) returns its (i, j) entry, the diagonal is 1.  The
// gather is part of this function so that the register allocation sees gather and factorisation
// together.
template <typename F, int K, typename Entry>
__device__ __forceinline__ FactorOut<F> lane_factor_by(Entry&& entry)
{
    F a[kTri<K>];
#pragma unroll
    for (int i = 0; i < K; ++i) {
#pragma unroll
        for (int j = 0; j < i; ++j) a[tri(i, j)] = entry(i, j);
        a[tri(i, i)] = F(1);
    }
    LogProd<F> det;
    bool ok = true;
    // right-looking Cholesky, L overwrites the strict lower triangle and the diagonal slot j
    // keeps 1 / L_jj (the pivot itself is not needed again)
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const F p = a[tri(j, j)];
        ok = ok && (p > F(0));
        const F r = Num<F>::rsq(p);
        a[tri(j, j)] = r;
        det.mul(p);
        if ((j & 3) == 3) det.renorm();
#pragma unroll
        for (int i = j + 1; i < K; ++i) a[tri(i, j)] *= r;
#pragma unroll
        for (int i = j + 1; i < K; ++i) {
            const F lij = a[tri(i, j)];
#pragma unroll
            for (int m = j + 1; m <= i; ++m) a[tri(i, m)] -= lij * a[tri(m, j)];
        }
    }
    // W = L^-1 column by column, in place (column j of W replaces column j of L), and the
    // squared column norms a_j = (R_S^-1)_jj.
    LogProd<F> va;
    F vmax = F(0);
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const F wjj = a[tri(j, j)];
        F acc = wjj * wjj;
#pragma unroll
        for (int i = j + 1; i < K; ++i) {
            F s = a[tri(i, j)] * wjj;
#pragma unroll
            for (int m = j + 1; m < i; ++m) s += a[tri(i, m)] * a[tri(m, j)];
            const F w = -s * a[tri(i, i)];
            a[tri(i, j)] = w;
            acc += w * w;
        }
        vmax = vmax > acc ? vmax : acc;
        va.mul(acc);
        if ((j & 3) == 3) va.renorm();
    }
    FactorOut<F> o;
    o.ld = det.log();
    o.sa = va.log();
    o.vmax = vmax;
    o.ok = ok;
    return o;
}

// Gather R_S of the index set c from the staged correlation matrix sR and factor it.
template <typename F, int K>
__device__ __forceinline__ FactorOut<F> lane_factor(const int (&c)[K > 0 ? K : 1], const F* __restrict__ sR, int N)
{
    return lane_factor_by<F, K>([&](int i, int j) { return sR[c[i] * N + c[j]]; });
}

// ------------------------------------------------------------------------------------------------
// Wave engine: one wavefront factors one n-plet of runtime order k <= 64 in FP64, the matrix in
// LDS.  Lane i owns row i.  sM: [64 * ks] doubles with row stride ks >= k + 1; sAux: [2*64].
// The block must consist of this single wavefront (barriers are block barriers).
// Returns the FactorOut in every lane.
// ------------------------------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) { const double u = __shfl_xor(v, o, 64); v = v > u ? v : u; }
    return v;
}

// Row `lane` of a correlation block gathered from the covariance row Sig[ci][.] (global memory):
// out[j] = (Sigma_{ci, c_j} / sqrt(Sigma_ii)) / sqrt(Sigma_jj) for j < lane, out[lane] = 1, with
// isd[j] = 1 / sqrt(Sigma_{c_j c_j}).  The loads go out eight at a time, all in flight together.
__device__ __forceinline__ void gather_row(const double* __restrict__ row, const int* __restrict__ cidx,
                                           const double* __restrict__ isd, int lane, double* __restrict__ out)
{
    const double si = isd[lane];
    for (int j0 = 0; j0 < lane; j0 += 8) {
        double e[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) e[u] = j0 + u < lane ? row[cidx[j0 + u]] : 0.0;
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (j0 + u < lane) out[j0 + u] = e[u] * si * isd[j0 + u];
    }
    out[lane] = 1.0;
}

// Factorisation of the k x k block already gathered into the lower triangle of sM (row stride
// ks, unit diagonal), one wavefront: log det, sum of log a_j and max a_j.  With sSeq (128
// doubles of LDS) the two sums are taken by lane 0 in variable order instead of by a lane tree, so
// inserting an independent variable (a zero row and column) changes no bit of the result.
__device__ __forceinline__ FactorOut<double> wave_factor_core(int k, double* __restrict__ sM, int ks,
                                                              double* __restrict__ sInv, double* __restrict__ sSeq = nullptr)
{
    const int lane = threadIdx.x & 63;
    bool ok = true;
    double pv = 1.0;   // this lane's pivot (lane j holds L_jj^2); its log is taken after the loop
    for (int j = 0; j < k; ++j) {
        const double p = sM[j * ks + j];
        ok = ok && (p > 0.0);
        const double r = rsqrt(p);
        if (lane == j) { sInv[j] = r; pv = p; }
        if (lane > j && lane < k) sM[lane * ks + j] *= r;
        __syncthreads();
        if (lane > j && lane < k) {
            const double l = sM[lane * ks + j];
            for (int m = j + 1; m <= lane; ++m) sM[lane * ks + m] -= l * sM[m * ks + j];
        }
        __syncthreads();
    }
    const double lp = lane < k ? log(pv) : 0.0;   // log L_jj^2 in lane j
    double la = 0.0, acc = 0.0;
    if (lane < k) {
        // column `lane` of W = L^-1 by forward substitution; W_mj is kept in the (unused) upper
        // triangle of row j = lane.
        const int j = lane;
        const double wjj = sInv[j];
        acc = wjj * wjj;
        for (int i = j + 1; i < k; ++i) {
            double s = sM[i * ks + j] * wjj;
            for (int m = j + 1; m < i; ++m) s += sM[i * ks + m] * sM[j * ks + m];
            const double w = -s * sInv[i];
            sM[j * ks + i] = w;
            acc += w * w;
        }
        la = log(acc);
    }
    FactorOut<double> o;
    if (sSeq) {
        if (lane < k) { sSeq[lane] = lp; sSeq[64 + lane] = la; }
        __syncthreads();
        double s1 = 0.0, s2 = 0.0;
        if (lane == 0) {
            for (int j = 0; j < k; ++j) { s1 += sSeq[j]; s2 += sSeq[64 + j]; }
        }
        o.ld = __shfl(s1, 0, 64);
        o.sa = __shfl(s2, 0, 64);
    } else {
        o.ld = wave_sum(lane < k ? lp : 0.0);
        o.sa = wave_sum(la);
    }
    o.vmax = wave_max(acc);
    o.ok = ok;
    __syncthreads();
    return o;
}

__device__ __forceinline__ FactorOut<double> wave_factor(const double* __restrict__ sR, int N, const int* __restrict__ cidx,
                                                         int k, double* __restrict__ sM, int ks,
                                                         double* __restrict__ sInv)
{
    const int lane = threadIdx.x & 63;
    if (lane < k) {
        const double* row = sR + cidx[lane] * N;
        for (int j = 0; j < lane; ++j) sM[lane * ks + j] = row[cidx[j]];
        sM[lane * ks + lane] = 1.0;
    }
    __syncthreads();
    return wave_factor_core(k, sM, ks, sInv);
}

}  // namespace thoi
