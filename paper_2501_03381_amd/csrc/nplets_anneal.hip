// Batched simulated annealing run on the device (Methods, "Heuristics", "Simulated Annealing
// Algorithm").  Each iteration is one kernel launch in which every chain proposes a neighbour,
// evaluates its O-information (Eq. O-info with TC and DTC from one Cholesky factorisation) and
// applies the Metropolis rule, so a whole run is enqueued without a host round trip.
//
// Orders up to 32: two chains per 64-lane wavefront, each half-wave factoring its chain's
// neighbour with the rows in registers (the pair factorisation, entries read from Sigma in global
// memory).  Larger orders (up to 64): one wavefront per chain, the block gathered into LDS.  In
// both, the lane that owns a chain forms its neighbour from the chain's mask and draws, and takes
// the decision and updates the chain's state.  Masks are two 64-bit words (N <= 128).  The random
// numbers are inputs (one row of draws per iteration), so a run is reproducible bit for bit.
#include "thoi_internal.hpp"
#include "nplets_common.hpp"
#include "pair_factor.hpp"

namespace thoi {
namespace {


struct Mask {
    uint64_t w[2];
};

struct AnnealArgs {
    const double* Sigma;
    int N;
    int kappa;
    int across;
    int kmin, kmax;
    double sign;                   // +1: maximise Omega, -1: minimise
    const double* move;            // [iters][kappa] (across orders only)
    const double* a;               // [iters][kappa] which member leaves
    const double* b;               // [iters][kappa] which outsider enters
    const double* u;               // [iters][kappa] acceptance draw
    Mask* cur;
    double* cur_om;
    Mask* best;
    double* best_om;
    int64_t* acc;
};

__device__ __forceinline__ int popc(const Mask& m) { return __popcll(m.w[0]) + __popcll(m.w[1]); }

// Index of the (n+1)-th set bit of m counted from bit 0, or 0 when m has fewer set bits.
__device__ __forceinline__ int nth_set(Mask m, int n)
{
    for (int h = 0; h < 2; ++h) {
        const int c = __popcll(m.w[h]);
        if (n < c) {
            uint64_t x = m.w[h];
            for (int i = 0; i < n; ++i) x &= x - 1;
            return 64 * h + __builtin_ctzll(x);
        }
        n -= c;
    }
    return 0;
}

__device__ __forceinline__ Mask full_mask(int N)
{
    Mask f;
    f.w[0] = N >= 64 ? ~0ull : ((1ull << N) - 1ull);
    f.w[1] = N >= 128 ? ~0ull : (N > 64 ? ((1ull << (N - 64)) - 1ull) : 0ull);
    return f;
}

// The neighbour of mask `cur` (Methods, "Simulated Annealing Algorithm"): within an order a member
// is swapped for an outsider; across orders a member is added (move < 1/3), removed
// (1/3 <= move < 2/3) or swapped, a swap also replacing a move that would leave [kmin, kmax].  The
// member is the floor(a k)-th set bit and the outsider the floor(b (N - k))-th clear bit, both in
// ascending order.
__device__ __forceinline__ Mask propose(Mask cur, int N, bool across, int kmin, int kmax, double move, double a,
                                        double b)
{
    const Mask full = full_mask(N);
    const int k = popc(cur);
    const bool add = across && move < 1.0 / 3.0 && k < kmax;
    const bool rem = across && move >= 1.0 / 3.0 && move < 2.0 / 3.0 && k > kmin;
    const bool swap = !(add || rem);
    Mask out;
    out.w[0] = ~cur.w[0] & full.w[0];
    out.w[1] = ~cur.w[1] & full.w[1];
    const int drop = nth_set(cur, (int)(int64_t)(a * (double)k));
    const int take = nth_set(out, (int)(int64_t)(b * (double)(N - k)));
    Mask p = cur;
    if (swap || rem) p.w[drop >> 6] &= ~(1ull << (drop & 63));
    if (swap || add) p.w[take >> 6] |= 1ull << (take & 63);
    return p;
}

// The chain's starting state, or one iteration's neighbour p, chosen for chain c.
__device__ __forceinline__ Mask chain_neighbour(const AnnealArgs& g, bool init, const Mask* __restrict__ masks0,
                                                int c, int64_t t)
{
    if (init) {
        const Mask full = full_mask(g.N);
        Mask p;
        p.w[0] = masks0[c].w[0] & full.w[0];
        p.w[1] = masks0[c].w[1] & full.w[1];
        return p;
    }
    const int64_t e = t * g.kappa + c;
    return propose(g.cur[c], g.N, g.across != 0, g.kmin, g.kmax, g.across ? g.move[e] : 0.0, g.a[e], g.b[e]);
}

// One thread per chain: the starting state (init), or the Metropolis decision on neighbour p.
__device__ __forceinline__ void chain_update(const AnnealArgs& g, bool init, int c, int64_t t, double temp,
                                             const Mask& p, const FactorOut<double>& f)
{
    // Omega = TC - DTC with TC = -ld/2 and DTC = (ld + sum_j log a_j)/2; NaN if not positive definite
    const bool ok = f.ok && isfinite(f.ld) && isfinite(f.sa);
    const double TC = -0.5 * f.ld, DTC = 0.5 * (f.ld + f.sa);
    const double om = ok ? TC - DTC : __builtin_nan("");
    if (init) {
        g.cur[c] = p;
        g.cur_om[c] = om;
        g.best[c] = p;
        g.best_om[c] = om;
        g.acc[c] = 0;
        return;
    }
    // energy E = sign * Omega; the neighbour is taken when dE > 0, else with probability
    // exp(dE / temp); a neighbour that is not positive definite is never taken
    const int64_t e = t * g.kappa + c;
    const double E = g.sign * g.cur_om[c];
    const double Ep = g.sign * om;
    const double dE = Ep - E;
    const bool take = ((dE > 0.0) || (g.u[e] < exp(dE / temp))) && !isnan(Ep);
    Mask m = g.cur[c];
    double mo = g.cur_om[c];
    if (take) {
        m = p;
        mo = om;
        g.cur[c] = p;
        g.cur_om[c] = om;
        g.acc[c] += 1;
    }
    if (g.sign * mo > g.sign * g.best_om[c]) {
        g.best[c] = m;
        g.best_om[c] = mo;
    }
}

// grid (ceil(kappa / 2)), block 64: chain 2 blockIdx.x + h in half-wave h, orders up to kW2Max.
template <bool INIT>
__global__ __launch_bounds__(64) void k_anneal_pair(AnnealArgs g, const Mask* __restrict__ masks0, int64_t t,
                                                    double temp)
{
    __shared__ double scol[2 * 2 * kW2Max], swrow[2 * 2 * kW2Max];
    __shared__ int sch[2 * kW2Max];
    __shared__ Mask sprop[2];
    const int lane = threadIdx.x, h = lane >> 5, i = lane & 31;
    const int c = 2 * blockIdx.x + h;
    const bool live = c < g.kappa;
    if (i == 0) sprop[h] = live ? chain_neighbour(g, INIT, masks0, c, t) : Mask{{0ull, 0ull}};
    wave_sync();
    const Mask p = sprop[h];
    int kh = popc(p);
    kh = kh < kW2Max ? kh : kW2Max;
    int* ch = sch + h * kW2Max;
    if (i < kh) ch[i] = nth_set(p, i);
    wave_sync();
    // every shuffle runs with the whole wavefront active
    const int k0 = __shfl(kh, 0), k1 = __shfl(kh, 32);
    const FactorOut<double> f = pair_factor<true>(g.Sigma, g.N, ch, k0 > k1 ? k0 : k1, kh, scol + h * 2 * kW2Max,
                                                  swrow + h * 2 * kW2Max);
    if (i == 0 && live) chain_update(g, INIT, c, t, temp, p, f);
}

// grid (kappa), block 64.  INIT: evaluate the starting masks; else iteration t at temperature temp.
// Dynamic LDS: the factorisation block, kmax rows of stride kmax + 1 (sized for the largest order a
// chain reaches, so that smaller maxima leave room for more wavefronts per CU); static: sInv [64] |
// sIsd [64] | cidx [64] | prop.
template <bool INIT>
__global__ __launch_bounds__(64) void k_anneal(AnnealArgs g, const Mask* __restrict__ masks0, int64_t t,
                                               double temp)
{
    extern __shared__ double sM[];
    const int ks = g.kmax + 1;
    __shared__ double sInv[64], sIsd[64];
    __shared__ int cidx[64];
    __shared__ Mask sprop;
    const int N = g.N;
    const int c = blockIdx.x;
    const int lane = threadIdx.x;

    if (lane == 0) sprop = chain_neighbour(g, INIT, masks0, c, t);
    __syncthreads();
    const Mask p = sprop;
    // every state holds k_min..k_max members; the clamp keeps a starting mask outside that range
    // in bounds of the block
    int k = popc(p);
    k = k < g.kmax ? k : g.kmax;
    // the block's variables and 1/sqrt of their variances, then the correlation block row by row:
    // R_ij = (Sigma_ij / sqrt(Sigma_ii)) / sqrt(Sigma_jj), unit diagonal
    int ci = 0;
    if (lane < k) {
        ci = nth_set(p, lane);
        cidx[lane] = ci;
        const double dj = g.Sigma[(int64_t)ci * N + ci];
        sIsd[lane] = dj > 0.0 ? 1.0 / sqrt(dj) : __builtin_nan("");
    }
    __syncthreads();
    if (lane < k) gather_row(g.Sigma + (int64_t)ci * N, cidx, sIsd, lane, sM + lane * ks);
    __syncthreads();
    const FactorOut<double> f = wave_factor_core(k, sM, ks, sInv);
    if (lane == 0) chain_update(g, INIT, c, t, temp, p, f);
}

}  // namespace

thoi_status launch_anneal(const double* Sigma, int32_t N, const uint64_t* masks0, int32_t kappa, int32_t iters,
                          const double* draw_move, const double* draw_a, const double* draw_b, const double* draw_u,
                          double T0, double alpha, int32_t maximize, int32_t across, int32_t k_min, int32_t k_max,
                          uint64_t* cur_mask, double* cur_omega, uint64_t* best_mask, double* best_omega,
                          int64_t* accepted, hipStream_t s)
{
    AnnealArgs g{};
    g.Sigma = Sigma;
    g.N = N;
    g.kappa = kappa;
    g.across = across ? 1 : 0;
    g.kmin = k_min;
    g.kmax = k_max;
    g.sign = maximize ? 1.0 : -1.0;
    g.move = draw_move;
    g.a = draw_a;
    g.b = draw_b;
    g.u = draw_u;
    g.cur = reinterpret_cast<Mask*>(cur_mask);
    g.cur_om = cur_omega;
    g.best = reinterpret_cast<Mask*>(best_mask);
    g.best_om = best_omega;
    g.acc = accepted;
    const Mask* m0 = reinterpret_cast<const Mask*>(masks0);
    // every order a chain can reach is at most k_max: the pair factorisation when it fits
    const bool pair = k_max <= kW2Max;
    const dim3 grid(pair ? (unsigned)((kappa + 1) / 2) : (unsigned)kappa);
    const size_t lds = pair ? 0 : (size_t)k_max * (size_t)(k_max + 1) * sizeof(double);
    if (pair) hipLaunchKernelGGL(k_anneal_pair<true>, grid, dim3(64), 0, s, g, m0, (int64_t)0, 0.0);
    else hipLaunchKernelGGL(k_anneal<true>, grid, dim3(64), lds, s, g, m0, (int64_t)0, 0.0);
    // the temperature of iteration t is T0 multiplied by alpha t times, one product at a time
    double temp = T0;
    for (int32_t t = 0; t < iters; ++t) {
        if (pair) hipLaunchKernelGGL(k_anneal_pair<false>, grid, dim3(64), 0, s, g, m0, (int64_t)t, temp);
        else hipLaunchKernelGGL(k_anneal<false>, grid, dim3(64), lds, s, g, m0, (int64_t)t, temp);
        temp *= alpha;
    }
    return hip_status(hipGetLastError());
}

}  // namespace thoi
