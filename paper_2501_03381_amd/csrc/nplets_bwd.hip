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
// Orders up to kBwdLaneMax run on the lane engine (one lane per n-plet, registers;
// nplets_bwd_lane.hpp), larger orders on the wave engine below (one wavefront per n-plet, LDS).
// LIST / MASK rows are first bucketed by order on the device.  This file holds the wave engine
// and the host side.
#include "nplets_bwd.hpp"
#include "nplets_fwd_common.hpp"

namespace thoi {
namespace {

constexpr int kCus = 256;
constexpr int64_t kLdsPerCu = 160 * 1024;
constexpr size_t kLdsLimit = 160 * 1024;

__device__ __forceinline__ bool bwd_wave_weights(const BwdArgs& a, int d, int64_t pos, double& cT, double& cD)
{
    const int64_t o = (int64_t)d * a.B + pos;
    const int64_t plane = (int64_t)a.D * a.B;
    const double wTC = a.grad_out[o], wDTC = a.grad_out[plane + o];
    const double wO = a.grad_out[2 * plane + o], wS = a.grad_out[3 * plane + o];
    cT = wTC + wO + wS;
    cD = wDTC - wO + wS;
    return cT != 0.0 || cD != 0.0;
}

// ------------------------------------------------------------------------------------------------
// Wave engine: orders above the lane engine's, one wavefront per n-plet, FP64 in LDS.
// grid (workgroups, D), block 64; each workgroup walks n-plets blockIdx.x, + gridDim.x, ... of
// the slots [s0, s1): RANGE positions [s0_range, s1_range) (the orders above the lane engine);
// LIST / MASK slots of perm from the bucket of order lane_max + 1 on.
// LDS: sIsd [N] f64 | sBin [N*64] u64 (RANGE) | sM [64*ks] f64 | sP [64*ks] f64 | sInv [64] f64 |
//      sAcc [N*N] f32 | cidx [64] i32
// ------------------------------------------------------------------------------------------------
__host__ __device__ inline size_t bwd_wave_lds_bytes(int N, int ks, bool range)
{
    size_t off = (size_t)N * 8 + (range ? (size_t)N * 64 * 8 : 0);
    off += 2 * (size_t)64 * ks * 8 + 64 * 8;
    off += (size_t)N * N * 4 + 64 * 4;
    return off;
}

template <int MODE>
__global__ __launch_bounds__(64) void k_bwd_wave(BwdArgs a, int ks, int64_t s0_range, int64_t s1_range)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int N = a.N;
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

    int64_t s0 = s0_range, s1 = s1_range;
    if constexpr (MODE != THOI_SEL_RANGE) {
        s0 = a.lbase[a.lane_max + 1];
        s1 = a.lbase[THOI_MAX_K + 1];
    }
    if (s0 + (int64_t)blockIdx.x >= s1) return;   // uniform: nothing for this workgroup

    const double* Sig = a.Sigma + (int64_t)d * N * N;
    for (int j = lane; j < N; j += 64) {
        const double dj = Sig[(int64_t)j * N + j];
        sIsd[j] = dj > 0.0 ? 1.0 / sqrt(dj) : __builtin_nan("");
    }
    for (int e = lane; e < N * N; e += 64) sAcc[e] = 0.0f;
    if constexpr (MODE == THOI_SEL_RANGE) stage_binomials(N, 64, sBin);
    __syncthreads();

    bool touched = false;
    for (int64_t slot = s0 + blockIdx.x; slot < s1; slot += gridDim.x) {
        const int64_t pos = MODE == THOI_SEL_RANGE ? slot : a.perm[slot];
        double cT, cD;
        if (!bwd_wave_weights(a, d, pos, cT, cD)) continue;   // uniform across the wave
        if (lane == 0) {
            int k = 0;
            if constexpr (MODE == THOI_SEL_RANGE) {
                const int64_t g = a.g_begin + pos;
                k = a.kmin;
                while (k < a.kmax && g >= a.ostart[k + 1]) ++k;
                unrank_lex_rt((uint64_t)(g - a.ostart[k]), N, k, sBin, 64, cidx);
            } else if constexpr (MODE == THOI_SEL_LIST) {
                const int32_t* row = a.idx + pos * a.kmax_list;
                while (k < a.kmax_list && row[k] >= 0) { cidx[k] = row[k]; ++k; }
            } else {
                uint64_t m = a.mask[pos];
                while (m) { cidx[k++] = __builtin_ctzll(m); m &= m - 1; }
            }
            sk = k;
        }
        __syncthreads();
        const int k = sk;
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
        // Cholesky (right-looking) and W = L^-1
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
        if (!ok) continue;   // not positive definite: no contribution (uniform)
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
        // U = P diag(1/p) in the rows of sM, then (P diag(1/p) P)_ij = sum_m U_im P_jm
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

// ------------------------------------------------------------------------------------------------
// Host side
// ------------------------------------------------------------------------------------------------
int bwd_class_of(int k)
{
    int c = 0;
    while (c < kBwdNClasses - 1 && k > kBwdClasses[c].hi) ++c;
    return c;
}

// Largest order of the lane engine for N variables: its LDS (staged matrix when N <= 64, the
// accumulator tile) must fit; otherwise every order goes to the wave engine.
int bwd_lane_max(int N) { return bwd_lane_lds_bytes(N, kBwdLaneMax) <= kLdsLimit ? kBwdLaneMax : 0; }

void bwd_lane_launch(int cls, const BwdArgs& a, const BwdTiles& t, int64_t ntiles, dim3 grid, size_t lds,
                     hipStream_t s)
{
    if (cls < kBwdNClasses - 1) bwd_lane_launch_lo(cls, a, t, ntiles, grid, lds, s);
    else bwd_lane_launch_hi(cls, a, t, ntiles, grid, lds, s);
}

int bwd_lane_blocks_per_cu(int cls, size_t lds)
{
    return cls < kBwdNClasses - 1 ? bwd_lane_blocks_per_cu_lo(cls, lds) : bwd_lane_blocks_per_cu_hi(cls, lds);
}

struct BwdWs {
    size_t korder_off, cnt_off, base_off, blk0_off, cursor_off, perm_off, total;
};

BwdWs bwd_layout(const thoi_nplets* sel)
{
    BwdWs w{};
    if (sel->mode == THOI_SEL_RANGE) return w;   // RANGE needs no workspace
    size_t off = kWsHeader;
    const int64_t B = sel->B;
    w.korder_off = off; off = align_up(off + (size_t)B, 256);
    w.cnt_off = off; off = align_up(off + kListOrders * 8, 256);
    w.base_off = off; off = align_up(off + kListOrders * 8, 256);
    w.blk0_off = off; off = align_up(off + kListOrders * 8, 256);
    w.cursor_off = off; off = align_up(off + kListOrders * 8, 256);
    w.perm_off = off; off = align_up(off + (size_t)B * 8, 256);
    w.total = off;
    return w;
}

void launch_bwd_engines(BwdArgs& a, const thoi_nplets* sel, hipStream_t s)
{
    const int N = a.N;
    const int64_t D = a.D;
    const int lane_max = a.lane_max;
    const bool range = a.mode == THOI_SEL_RANGE;
    BwdTiles tabs[kBwdNClasses] = {};
    int64_t ntiles[kBwdNClasses] = {0};
    int64_t wave_s0 = 0, wave_cnt = 0;
    int wave_kmax = 0;
    if (range) {
        int64_t g = 0;
        const int64_t gb = sel->g_begin, ge = sel->g_begin + sel->g_count;
        bool wave_start = false;
        for (int k = sel->kmin; k <= sel->kmax; ++k) {
            const int64_t ck = (int64_t)binom_u64(N, k);
            const int64_t lo = gb > g ? gb : g, hi = ge < g + ck ? ge : g + ck;
            if (hi > lo) {
                if (k <= lane_max) {
                    const int c = bwd_class_of(k);
                    BwdPiece p{};
                    p.k = k;
                    p.first = lo - g;
                    p.pos0 = lo - gb;
                    p.cnt = hi - lo;
                    p.tile0 = ntiles[c];
                    ntiles[c] += (p.cnt + kBwdClassThreads[c] - 1) / kBwdClassThreads[c];
                    tabs[c].p[tabs[c].n++] = p;
                } else {
                    if (!wave_start) { wave_s0 = lo - gb; wave_start = true; }
                    wave_cnt += hi - lo;
                    wave_kmax = k;
                }
            }
            g += ck;
        }
    } else {
        const int kcap = sel_kmax(sel, N);
        for (int c = 0; c < kBwdNClasses; ++c) {
            if (kBwdClasses[c].lo <= kcap && kBwdClasses[c].lo <= lane_max)
                ntiles[c] = (a.B + kBwdClassThreads[c] - 1) / kBwdClassThreads[c];
        }
        if (kcap > lane_max) { wave_cnt = a.B; wave_kmax = kcap; }
    }
    int nl = wave_cnt > 0 ? 1 : 0;
    for (int c = 0; c < kBwdNClasses; ++c) nl += ntiles[c] > 0;
    FanScope fan(s, nl);
    int b = 0;
    for (int c = kBwdNClasses - 1; c >= 0; --c) {   // longest lanes first
        if (ntiles[c] == 0) continue;
        const size_t lds = bwd_lane_lds_bytes(N, range ? kBwdClasses[c].hi : 0);
        // persistent: one round of workgroups (registers and LDS decide how many a CU holds),
        // shared among the datasets
        const int64_t res = (int64_t)kCus * bwd_lane_blocks_per_cu(c, lds);
        const int64_t per_d = (res + D - 1) / D;
        const int64_t gx = ntiles[c] < per_d ? ntiles[c] : per_d;
        bwd_lane_launch(c, a, tabs[c], ntiles[c], dim3((unsigned)gx, (unsigned)D), lds, fan.stream(b++));
    }
    if (wave_cnt > 0) {
        const int ks = (wave_kmax < 64 ? wave_kmax : 64) + 1;
        const size_t lds = bwd_wave_lds_bytes(N, ks, range);
        const int64_t per_cu = kLdsPerCu / (int64_t)lds > 0 ? kLdsPerCu / (int64_t)lds : 1;
        const int64_t per_d = (kCus * per_cu + D - 1) / D;
        const int64_t gx = wave_cnt < per_d ? wave_cnt : per_d;
        const dim3 grid((unsigned)gx, (unsigned)D);
        if (a.mode == THOI_SEL_RANGE)
            hipLaunchKernelGGL(k_bwd_wave<THOI_SEL_RANGE>, grid, dim3(64), lds, fan.stream(b++), a, ks, wave_s0,
                               wave_s0 + wave_cnt);
        else if (a.mode == THOI_SEL_LIST)
            hipLaunchKernelGGL(k_bwd_wave<THOI_SEL_LIST>, grid, dim3(64), lds, fan.stream(b++), a, ks, (int64_t)0,
                               (int64_t)0);
        else
            hipLaunchKernelGGL(k_bwd_wave<THOI_SEL_MASK>, grid, dim3(64), lds, fan.stream(b++), a, ks, (int64_t)0,
                               (int64_t)0);
    }
}

}  // namespace

size_t backward_ws_bytes(int64_t D, int32_t N, const thoi_nplets* sel, const thoi_eval_opts* opts)
{
    (void)D; (void)N; (void)opts;
    return bwd_layout(sel).total;
}

size_t backward_lds_bytes(int32_t N, const thoi_nplets* sel)
{
    const bool range = sel->mode == THOI_SEL_RANGE;
    const int kmax = range ? sel->kmax : (sel->mode == THOI_SEL_LIST ? sel->kmax_list : N);
    const int lane_max = bwd_lane_max(N);
    size_t need = lane_max > 0 ? bwd_lane_lds_bytes(N, range ? kBwdLaneMax : 0) : 0;
    if (kmax > lane_max) {
        const int ks = (kmax < 64 ? kmax : 64) + 1;
        const size_t w = bwd_wave_lds_bytes(N, ks, range);
        need = need > w ? need : w;
    }
    return need;
}

thoi_status launch_backward(const double* Sigma, int64_t D, int32_t N, const thoi_nplets* sel,
                            const thoi_eval_opts* opts, const float* grad_out, float* grad_Sigma, void* ws,
                            size_t ws_bytes, hipStream_t s)
{
    (void)opts;
    const BwdWs w = bwd_layout(sel);
    if (w.total > 0 && (ws == nullptr || ws_bytes < w.total)) return THOI_EWORKSPACE;
    BwdArgs a{};
    a.Sigma = Sigma;
    a.N = N;
    a.D = (int32_t)D;
    a.B = sel_B(sel);
    a.grad_out = grad_out;
    a.grad_Sigma = grad_Sigma;
    a.mode = sel->mode;
    a.lane_max = bwd_lane_max(N);
    a.idx = sel->idx;
    a.kmax_list = sel->kmax_list;
    a.mask = sel->mask;
    if (sel->mode == THOI_SEL_RANGE) {
        a.kmin = sel->kmin;
        a.kmax = sel->kmax;
        a.g_begin = sel->g_begin;
        int64_t g = 0;
        for (int k = sel->kmin; k <= sel->kmax + 1 && k <= THOI_MAX_K + 1; ++k) {
            a.ostart[k] = g;
            if (k <= sel->kmax) g += (int64_t)binom_u64(N, k);
        }
    }
    if (D == 0 || a.B == 0) return THOI_OK;
    if (sel->mode == THOI_SEL_RANGE) {
        launch_bwd_engines(a, sel, s);
        return hip_status(hipGetLastError());
    }
    // LIST / MASK: bucket the rows by order on the device (invalid rows go to the last bucket,
    // contribute nothing and raise THOI_EINVAL_DATA in the status word)
    char* base = static_cast<char*>(ws);
    WsHeader* hdr = reinterpret_cast<WsHeader*>(base);
    uint8_t* korder = reinterpret_cast<uint8_t*>(base + w.korder_off);
    unsigned long long* cnt = reinterpret_cast<unsigned long long*>(base + w.cnt_off);
    int64_t* lbase = reinterpret_cast<int64_t*>(base + w.base_off);
    int64_t* lblk0 = reinterpret_cast<int64_t*>(base + w.blk0_off);
    unsigned long long* cursor = reinterpret_cast<unsigned long long*>(base + w.cursor_off);
    int64_t* perm = reinterpret_cast<int64_t*>(base + w.perm_off);
    a.perm = perm;
    a.lcnt = reinterpret_cast<const int64_t*>(cnt);
    a.lbase = lbase;
    EvalArgs ea{};
    ea.N = N;
    ea.D = (int32_t)D;
    ea.B = a.B;
    ea.hdr = hdr;
    ea.idx = sel->idx;
    ea.kmax_list = sel->kmax_list;
    ea.mask = sel->mask;
    hipLaunchKernelGGL(k_ws_clear, dim3(1), dim3(64), 0, s, reinterpret_cast<uint32_t*>(base), (int64_t)(kWsHeader / 4));
    hipLaunchKernelGGL(k_ws_clear, dim3(1), dim3(256), 0, s, reinterpret_cast<uint32_t*>(cnt), (int64_t)kListOrders * 2);
    const unsigned nb = (unsigned)((a.B + 255) / 256);
    ClassMap cm{};
    for (int k = 0; k < kListOrders; ++k) {
        cm.wave[k] = k > a.lane_max ? 1 : 0;
        cm.cls[k] = (int8_t)bwd_class_of(k <= kBwdLaneMax ? k : kBwdLaneMax);
    }
    if (sel->mode == THOI_SEL_LIST)
        hipLaunchKernelGGL(k_list_classify<THOI_SEL_LIST>, dim3(nb), dim3(256), 0, s, ea, 1, a.B, korder, cnt);
    else
        hipLaunchKernelGGL(k_list_classify<THOI_SEL_MASK>, dim3(nb), dim3(256), 0, s, ea, 1, a.B, korder, cnt);
    hipLaunchKernelGGL(k_list_scan, dim3(1), dim3(64), 0, s, cnt, lbase, lblk0, cursor, cm, (int64_t)1, (int64_t)1,
                       (int64_t)1);
    hipLaunchKernelGGL(k_list_scatter, dim3(nb), dim3(256), 0, s, a.B, korder, lbase, cursor, perm);
    launch_bwd_engines(a, sel, s);
    return hip_status(hipGetLastError());
}

}  // namespace thoi
