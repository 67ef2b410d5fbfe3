// Prefix-sharing engine: exhaustive evaluation of whole orders with the factorisation of each
// shared prefix done once.
//
// What drives the cost of the exhaustive search is one k x k factorisation per n-plet for every
// one of the C(N, k) n-plets of each order (Supplementary, "The combinatorial explosion",
// Eq. comb).  In lexicographic order the n-plets that share their first k - 2 variables P are
// consecutive, and each of them is P plus a pair x1 < x2 drawn from the variables after max P.
// A lane owns one prefix P: it factors R_P = L L^T once (W = L^-1, the inverse diagonal
// a_j = (R_P^-1)_jj = sum_r W_rj^2 and the pivot product), then walks the pairs in lexicographic
// order, bordering the factor with one variable at a time.  Bordering R_Q (size r) with a
// variable x, v = R[x, Q]:
//   l = W v,  s = 1 - l.l  (the new pivot, so log det R_{Q+x} = log det R_Q + log s),
//   w = W^T l = R_Q^-1 v,  (R_{Q+x}^-1)_jj = a_j + w_j^2 / s,  (R_{Q+x}^-1)_xx = 1 / s,
//   new row of W: (-w^T, 1) / sqrt(s)
// (block inverse with the Schur complement s).  The first bordering (x1) is shared by all the
// pairs that start with it; the second (x2) completes one n-plet.  Per n-plet that is about
// 2 (k-1)^2 multiply-adds instead of the 2 (k^3 - k)/3 + k (k+1) flops of a full factorisation
// (plus the shared parts), and the measures follow from log det and the inverse diagonal exactly
// as in the lane engine.
//
// Work decomposition: order k's prefixes are grouped by their last variable q (the C(q, k-3)
// subsets of {0..q-1} plus q); a workgroup takes 256 prefixes with the same q, so every lane runs
// the same pair loops (x1 in q+1..N-2, x2 in x1+1..N-1) and the streaming reducer's workgroup-wide
// steps stay uniform.  A lane's n-plets are consecutive global indices, starting at the
// lexicographic rank of P + {q+1, q+2}.  FP32 with FP64 re-evaluation of flagged n-plets, or FP64,
// as in the lane engine.
#include "nplets_prefix.hpp"

namespace thoi {
static_assert(kPfxThreads <= 64 * kRedWaves, "the reducer keeps lists for at most kRedWaves wavefronts");
namespace {

// Tail depth for order K: the variables appended to a shared prefix of K - S variables.
template <int K>
__host__ __device__ constexpr int pfx_tail(){ return K >= 4 ? 3 : 2; }

// lexicographic rank of the first n-plet P + {q+1, ..., q+S} of prefix P (K - S sorted variables,
// the last being q) among the K-subsets of {0..N-1}: over the prefix positions i, the K-subsets
// that agree before i and are smaller at i number C(N - c_{i-1} - 1, K - i) - C(N - c_i, K - i)
// (hockey-stick sum, c_{-1} = -1); the consecutive tail variables add nothing.
template <int K>
__device__ __forceinline__ uint64_t pfx_first_rank(const int (&c)[K], int N)
{
    constexpr int M = K - pfx_tail<K>();
    uint64_t r = 0;
    int prev = -1;
#pragma unroll
    for (int i = 0; i < M; ++i) {
        r += kPascal.v[N - prev - 1][K - i] - kPascal.v[N - c[i]][K - i];
        prev = c[i];
    }
    return r;
}

// Border the factor of the first R variables of c (W rows 0..R-1, inverse diagonal ain, pivot
// product din) with variable x = c[R]: l = W v, s = 1 - l.l, w = W^T l.  Interior levels write W
// row R, the inverse diagonal aout[0..R] and dout; the caller of the last level uses l, w, s.
template <typename F, int K, int R, bool LEAF>
__device__ __forceinline__ F pfx_border(F (&W)[K * (K + 1) / 2], const F* __restrict__ sR, int N,
                                        const int (&c)[K], const F (&ain)[K], F (&aout)[K], const LogProd<F>& din,
                                        LogProd<F>& dout, F (&w)[K])
{
    const F* row = sR + c[R] * N;
    F l[R > 0 ? R : 1];
    F s = F(1);
#pragma unroll
    for (int i = 0; i < R; ++i) {
        F t = W[tri(i, 0)] * row[c[0]];
#pragma unroll
        for (int j = 1; j <= i; ++j) t += W[tri(i, j)] * row[c[j]];
        l[i] = t;
        s -= t * t;
    }
#pragma unroll
    for (int j = 0; j < R; ++j) {
        F t = W[tri(j, j)] * l[j];
#pragma unroll
        for (int i = j + 1; i < R; ++i) t += W[tri(i, j)] * l[i];
        w[j] = t;
    }
    if constexpr (!LEAF) {
        const F rs = Num<F>::rsq(s);
        const F is = rs * rs;
#pragma unroll
        for (int j = 0; j < R; ++j) {
            W[tri(R, j)] = -w[j] * rs;
            aout[j] = ain[j] + w[j] * w[j] * is;
        }
        W[tri(R, R)] = rs;
        aout[R] = is;
        dout = din;
        dout.mul(s);
        dout.renorm();
    }
    return s;
}

// One lane: prefix P (rank r among the (M-1)-subsets of {0..q-1}, then q), the tails of ranks
// t0 .. t0 + L - 1 (lexicographic S-subsets of {q+1..N-1}; ranks >= ntail do nothing).  The tail
// sequence is the same for every lane of the wave, so which levels are re-bordered after each step
// is uniform.
template <typename F, int K, bool RED>
__device__ __forceinline__ void pfx_lane(const EvalArgs& a, RedLds& Rl, const RedArgs& red, int d, const F* sR,
                                         const double* sLogd, int q, uint64_t r, bool active, uint64_t t0, int L,
                                         uint64_t ntail, int64_t pos0, double dtc, double ddtc, double eta)
{
    constexpr int S = pfx_tail<K>();
    constexpr int M = K - S;                   // prefix size, >= 1
    constexpr int NT = K * (K + 1) / 2;
    const int N = a.N;
    int c[K];
    {
        int x = 0;
#pragma unroll
        for (int i = 0; i < M - 1; ++i) {
            const int m = M - 2 - i;
            while (x < q) {
                const uint64_t b = kPascal.v[q - 1 - x][m];
                if (r < b) break;
                r -= b;
                ++x;
            }
            c[i] = x++;
        }
        c[M - 1] = q;
    }
    const int64_t pbase = pos0 + (int64_t)pfx_first_rank<K>(c, N);
    // the first tail: rank t0 among the S-subsets of the nt = N - 1 - q variables after q
    {
        const int nt = N - 1 - q;
        uint64_t rt = t0 < ntail ? t0 : 0;
        int x = 0;
#pragma unroll
        for (int i = 0; i < S; ++i) {
            const int m = S - 1 - i;
            while (x < nt) {
                const uint64_t b = kPascal.v[nt - 1 - x][m];
                if (rt < b) break;
                rt -= b;
                ++x;
            }
            c[M + i] = q + 1 + x++;
        }
    }

    // factor the prefix: Cholesky (the diagonal slot keeps 1 / L_jj), W = L^-1 in place, inverse
    // diagonal = column norms of W, pivot product
    F W[NT];
#pragma unroll
    for (int i = 0; i < M; ++i) {
        const F* row = sR + c[i] * N;
#pragma unroll
        for (int j = 0; j < i; ++j) W[tri(i, j)] = row[c[j]];
        W[tri(i, i)] = F(1);
    }
    F al[S][K];           // inverse diagonal after levels 0 (prefix) .. S-1
    LogProd<F> det[S];
    bool ok0 = true;
#pragma unroll
    for (int j = 0; j < M; ++j) {
        const F p = W[tri(j, j)];
        ok0 = ok0 && (p > F(0));
        const F rs = Num<F>::rsq(p);
        W[tri(j, j)] = rs;
        det[0].mul(p);
        if ((j & 3) == 3) det[0].renorm();
#pragma unroll
        for (int i = j + 1; i < M; ++i) W[tri(i, j)] *= rs;
#pragma unroll
        for (int i = j + 1; i < M; ++i) {
            const F lij = W[tri(i, j)];
#pragma unroll
            for (int m = j + 1; m <= i; ++m) W[tri(i, m)] -= lij * W[tri(m, j)];
        }
    }
    det[0].renorm();
#pragma unroll
    for (int j = 0; j < M; ++j) {
        const F wjj = W[tri(j, j)];
#pragma unroll
        for (int i = j + 1; i < M; ++i) {
            F s = W[tri(i, j)] * wjj;
#pragma unroll
            for (int m = j + 1; m < i; ++m) s += W[tri(i, m)] * W[tri(m, j)];
            W[tri(i, j)] = -s * W[tri(i, i)];
        }
    }
#pragma unroll
    for (int j = 0; j < M; ++j) {
        F t = W[tri(j, j)] * W[tri(j, j)];
#pragma unroll
        for (int i = j + 1; i < M; ++i) t += W[tri(i, j)] * W[tri(i, j)];
        al[0][j] = t;
    }
    // interior levels 1..S-1 for the first tail; pivots of every level must be positive
    F w[K];
    bool okl[S];
    okl[0] = ok0;
    sfor<1, S>([&](auto D) {
        constexpr int lv = D;
        const F s = pfx_border<F, K, M + lv - 1, false>(W, sR, N, c, al[lv - 1], al[lv], det[lv - 1], det[lv], w);
        okl[lv] = okl[lv - 1] && (s > F(0));
    });

    for (int it = 0; it < L; ++it) {
        const uint64_t tr = t0 + (uint64_t)it;
        // leaf: border with the last tail variable
        LogProd<F> dl;
        const F s = pfx_border<F, K, K - 1, true>(W, sR, N, c, al[S - 1], al[S - 1], det[S - 1], dl, w);
        const bool ok = okl[S - 1] && (s > F(0));
        const F is = F(1) / s;
        LogProd<F> va;
        F vmax = is;
#pragma unroll
        for (int j = 0; j < K - 1; ++j) {
            const F aj = al[S - 1][j] + w[j] * w[j] * is;
            vmax = vmax > aj ? vmax : aj;
            va.mul(aj);
            if ((j & 3) == 3) va.renorm();
        }
        va.mul(is);
        LogProd<F> dt = det[S - 1];
        dt.mul(s);
        FactorOut<F> fo;
        fo.ld = dt.log();
        fo.sa = va.log();
        fo.vmax = vmax;
        fo.ok = ok;
        double omega = 0.0;
        bool valid = false;
        const int64_t pos = pbase + (int64_t)tr;
        if (active && tr < ntail) {
            double sld = 0.0;
            if (a.write_H) {
#pragma unroll
                for (int i = 0; i < K; ++i) sld += sLogd[c[i]];
            }
            valid = store_result<F>(a, RED, d, pos, K, fo, sld, dtc, ddtc, eta, false, omega);
        }
        if constexpr (RED) red_push(Rl, red, K, valid, omega, a.g_begin + pos);
        // next tail in lexicographic order: the last tail position that can still grow grows by
        // one, the positions after it follow it; levels from that position on are re-bordered
        if (it + 1 < L && tr + 1 < ntail) {
            int piv = 0;
#pragma unroll
            for (int i = 0; i < S; ++i) piv = c[M + i] < N - S + i ? i : piv;
#pragma unroll
            for (int i = 0; i < S; ++i) {
                if (i == piv) c[M + i] += 1;
                else if (i > piv) c[M + i] = c[M + i - 1] + 1;
            }
            sfor<1, S>([&](auto D) {
                constexpr int lv = D;
                if (piv <= lv - 1) {
                    const F sb = pfx_border<F, K, M + lv - 1, false>(W, sR, N, c, al[lv - 1], al[lv], det[lv - 1],
                                                                     det[lv], w);
                    okl[lv] = okl[lv - 1] && (sb > F(0));
                }
            });
        }
    }
}

template <typename F, int K, int KHI, bool RED>
__device__ __forceinline__ void pfx_dispatch(int k, const EvalArgs& a, RedLds& Rl, const RedArgs& red, int d,
                                             const F* sR, const double* sLogd, int q, uint64_t r, bool active,
                                             uint64_t t0, int L, uint64_t ntail, int64_t pos0, double dtc,
                                             double ddtc, double eta)
{
    if (k == K) pfx_lane<F, K, RED>(a, Rl, red, d, sR, sLogd, q, r, active, t0, L, ntail, pos0, dtc, ddtc, eta);
    else if constexpr (K < KHI)
        pfx_dispatch<F, K + 1, KHI, RED>(k, a, Rl, red, d, sR, sLogd, q, r, active, t0, L, ntail, pos0, dtc, ddtc,
                                         eta);
}

// Work units of order k with last prefix variable q: blocks of 64 prefixes x chunks of L tails.
__host__ __device__ inline void pfx_units(int N, int k, int q, int L, uint64_t& npref, uint64_t& ntail,
                                          uint64_t& nchunk, uint64_t& nunits)
{
    const int S = k >= 4 ? 3 : 2;
    const int M = k - S;
#ifdef __HIP_DEVICE_COMPILE__
    npref = kPascal.v[q][M - 1];
    ntail = kPascal.v[N - 1 - q][S];
#else
    npref = binom_u64(q, M - 1);
    ntail = binom_u64(N - 1 - q, S);
#endif
    nchunk = (ntail + L - 1) / L;
    nunits = (npref + 63) / 64 * nchunk;
}

// LDS: sR [N*N] F | sIsd [N] f64 | sLogd [N] f64 | (reduce) RedLds
__host__ __device__ inline size_t pfx_stage_bytes(int N, int fsize)
{
    size_t off = ((size_t)N * N * fsize + 15) / 16 * 16;
    off += (size_t)N * 16;
    return (off + 15) / 16 * 16;
}

// grid (workgroups, D), block kPfxThreads.
template <typename F, int KLO, int KHI, bool RED>
__global__ __launch_bounds__(kPfxThreads) void k_eval_prefix(EvalArgs a, PfxTable tab, RedArgs red)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double sbias[3];
    const int N = a.N;
    const int d = blockIdx.y;
    const int64_t blk = blockIdx.x;
    // order k of this workgroup (persistent over the blocks of one order)
    int k = -1, L = 1;
    int64_t pos0 = 0, vb0 = 0, nphys = 1, nblk = 0;
    for (int p = 0; p < tab.n; ++p) {
        if (blk >= tab.p[p].blk0 && blk < tab.p[p].blk0 + tab.p[p].nphys) {
            k = tab.p[p].k;
            L = tab.p[p].L;
            pos0 = tab.p[p].pos0;
            vb0 = blk - tab.p[p].blk0;
            nphys = tab.p[p].nphys;
            nblk = tab.p[p].nblk;
        }
    }
    if (k < 0) return;
    F* sR = reinterpret_cast<F*>(smem);
    const size_t off = ((size_t)N * N * sizeof(F) + 15) / 16 * 16;
    double* sIsd = reinterpret_cast<double*>(smem + off);
    double* sLogd = sIsd + N;
    RedLds Rl = red_view(smem + pfx_stage_bytes(N, sizeof(F)), red.topk, red.bins);
    if (threadIdx.x == 0) bias_for(a.bias, k, sbias[0], sbias[1], sbias[2]);
    stage_corr<F>(a.Sigma + (int64_t)d * N * N, N, sR, sIsd, sLogd);
    if constexpr (RED) red_begin(Rl, red, d, k);
    const int S = k >= 4 ? 3 : 2;
    for (int64_t vb = vb0; vb < nblk; vb += nphys) {
        // the prefixes' last variable q: the blocks of each q in turn (4 units of 64 prefixes x
        // L tails each); everything below is uniform in the workgroup
        int64_t lb = vb;
        int q = k - S - 1;
        uint64_t npref = 0, ntail = 0, nchunk = 0, nunits = 0;
        for (; q <= N - 1 - S; ++q) {
            pfx_units(N, k, q, L, npref, ntail, nchunk, nunits);
            const int64_t nb = (int64_t)((nunits + 3) / 4);
            if (lb < nb) break;
            lb -= nb;
        }
        if (q > N - 1 - S) break;
        const uint64_t unit = (uint64_t)lb * 4 + threadIdx.x / 64;
        const uint64_t pb = unit / nchunk, ch = unit % nchunk;
        const uint64_t r = pb * 64 + (threadIdx.x & 63);
        const bool active = unit < nunits && r < npref;
        pfx_dispatch<F, KLO, KHI, RED>(k, a, Rl, red, d, sR, sLogd, q, active ? r : 0, active,
                                       unit < nunits ? ch * (uint64_t)L : 0, L, ntail, pos0, sbias[0], sbias[1],
                                       sbias[2]);
    }
    if constexpr (RED) red_end(Rl, red, a.hdr, d, k);
}

template <typename F, int KLO, int KHI>
void pfx_launch_one(bool reduce, const EvalArgs& a, const PfxTable& t, const RedArgs& red, int64_t nblk, int D,
                    size_t lds, hipStream_t s)
{
    const dim3 grid((unsigned)nblk, (unsigned)D);
    if (reduce) hipLaunchKernelGGL((k_eval_prefix<F, KLO, KHI, true>), grid, dim3(kPfxThreads), lds, s, a, t, red);
    else hipLaunchKernelGGL((k_eval_prefix<F, KLO, KHI, false>), grid, dim3(kPfxThreads), lds, s, a, t, red);
}

}  // namespace

int pfx_tails(int N, int k, int64_t D)
{
    const double want = (double)binom_u64(N, k) * (double)(D > 0 ? D : 1) / 262144.0;
    int L = 1;
    while (L < kPfxMaxTails && 2.0 * L <= want) L *= 2;
    return L;
}

int64_t pfx_blocks(int N, int k, int L)
{
    const int S = k >= 4 ? 3 : 2;
    int64_t nb = 0;
    for (int q = k - S - 1; q <= N - 1 - S; ++q) {
        uint64_t npref, ntail, nchunk, nunits;
        pfx_units(N, k, q, L, npref, ntail, nchunk, nunits);
        nb += (int64_t)((nunits + 3) / 4);
    }
    return nb;
}

size_t pfx_lds_bytes(int N, int fsize, size_t red_bytes)
{
    return pfx_stage_bytes(N, fsize) + red_bytes;
}

void pfx_launch(bool f64, int cls, bool reduce, const EvalArgs& a, const PfxTable& t, const RedArgs& red,
                int64_t nblk, int D, hipStream_t s)
{
    const size_t lds = pfx_lds_bytes(a.N, f64 ? 8 : 4, red_lds(red));
    static_assert(kPfxF32Classes[0].lo == 3 && kPfxF32Classes[0].hi == 8 && kPfxF32Classes[1].hi == 12 &&
                      kPfxF32Classes[2].hi == 16 && kPfxF64Classes[1].hi == 12,
                  "class table");
    if (f64) {
        if (cls == 0) pfx_launch_one<double, 3, 8>(reduce, a, t, red, nblk, D, lds, s);
        else pfx_launch_one<double, 9, 12>(reduce, a, t, red, nblk, D, lds, s);
    } else {
        if (cls == 0) pfx_launch_one<float, 3, 8>(reduce, a, t, red, nblk, D, lds, s);
        else if (cls == 1) pfx_launch_one<float, 9, 12>(reduce, a, t, red, nblk, D, lds, s);
        else pfx_launch_one<float, 13, 16>(reduce, a, t, red, nblk, D, lds, s);
    }
}

}  // namespace thoi
