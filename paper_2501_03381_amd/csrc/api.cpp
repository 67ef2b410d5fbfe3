// Host side of the libthoi.so C ABI: argument checking, workspace sizing and pure host helpers.
// Every entry point validates its arguments before enqueuing anything.
#include <hip/hip_runtime.h>

#include <math.h>
#include <mutex>

#include "thoi_internal.hpp"

#include <cmath>

namespace thoi {

thoi_status hip_status(hipError_t e) { return e == hipSuccess ? THOI_OK : THOI_EHIP; }

uint64_t binom_u64(int n, int m)
{
    if (m < 0 || n < 0 || m > n) return 0;
    if (m > n - m) m = n - m;
    // exact for n <= 64: the running value is C(n - m + i, i) and the division is exact
    unsigned __int128 c = 1;
    for (int i = 1; i <= m; ++i) c = c * (unsigned __int128)(n - m + i) / (unsigned __int128)i;
    return (uint64_t)c;
}

namespace {

// psi at x = (T - j) / 2 for j = 1 .. 65, from the exact finite sums
//   psi(n)       = -gamma + sum_{i=1}^{n-1} 1/i
//   psi(n + 1/2) = -gamma - 2 log 2 + sum_{i=1}^{n} 2/(2i - 1)
// evaluated at the two largest arguments and stepped down with psi(x) = psi(x + 1) - 1/x.
struct PsiCache {
    int T = -1;
    double psi[THOI_MAX_K + 2];  // psi[j] = psi((T - j)/2), j >= 1
};
std::mutex g_psi_mu;
PsiCache g_psi;

double psi_integer_or_half(int twice_x)
{
    const double gamma = 0.57721566490153286061;
    // Kahan-compensated sums, small terms first
    double s = 0.0, comp = 0.0;
    auto add = [&](double v) {
        double y = v - comp;
        double t = s + y;
        comp = (t - s) - y;
        s = t;
    };
    if (twice_x % 2 == 0) {
        const int n = twice_x / 2;
        for (int i = n - 1; i >= 1; --i) add(1.0 / i);
        return -gamma + s;
    }
    const int n = (twice_x - 1) / 2;
    for (int i = n; i >= 1; --i) add(2.0 / (2.0 * i - 1.0));
    return -gamma - 2.0 * log(2.0) + s;
}

void fill_psi(int T)
{
    std::lock_guard<std::mutex> lk(g_psi_mu);
    if (g_psi.T == T) return;
    const int jmax = THOI_MAX_K + 1;
    for (int j = 1; j <= jmax && j < T; ++j) {
        if (j <= 2) g_psi.psi[j] = psi_integer_or_half(T - j);
        else g_psi.psi[j] = g_psi.psi[j - 2] - 2.0 / (double)(T - j);   // psi(x) = psi(x+1) - 1/x
    }
    g_psi.T = T;
}

}  // namespace

void bias_offsets(int k, int T, double* d_tc, double* d_dtc, double* eta)
{
    *d_tc = *d_dtc = *eta = 0.0;
    if (k <= 0) return;
    fill_psi(T);
    double P = 0.0, Pkm1 = 0.0;
    for (int j = 1; j <= k; ++j) {
        if (j == k) Pkm1 = P;
        P += g_psi.psi[j];
    }
    const double psi1 = g_psi.psi[1], psik = g_psi.psi[k];
    *d_tc = 0.5 * (P - k * psi1);
    *d_dtc = 0.5 * ((k - 1) * psik - Pkm1);
    *eta = 0.5 * (k * log(2.0 / (double)(T - 1)) + P);
}

void bias_psi_seeds(int T, double* psi1, double* psi2)
{
    fill_psi(T);
    *psi1 = g_psi.psi[1];
    *psi2 = T > 2 ? g_psi.psi[2] : 0.0;
}

}  // namespace thoi

using namespace thoi;

namespace {

int64_t count_orders(int N, int kmin, int kmax)
{
    if (N < 0 || N > 64) return -1;
    unsigned __int128 s = 0;
    for (int k = kmin < 0 ? 0 : kmin; k <= kmax && k <= N; ++k) s += binom_u64(N, k);
    if (s > (unsigned __int128)INT64_MAX) return -1;
    return (int64_t)s;
}

bool valid_dtype(int32_t t) { return t == THOI_DTYPE_F64 || t == THOI_DTYPE_F32; }
constexpr size_t kLdsLimit = 160 * 1024;

}  // namespace

thoi_status thoi::check_eval(const double* Sigma, int64_t D, int32_t N, const thoi_nplets* sel, const thoi_eval_opts* opts,
                       bool forward, const void* out)
{
    if (!sel || !opts) return THOI_EINVAL;
    if (D < 0 || N < 1) return THOI_EINVAL;
    if (D > 65535 || N > THOI_MAX_N) return THOI_EUNSUPPORTED;
    if (opts->precision != THOI_FP64 && opts->precision != THOI_FP32 && opts->precision != THOI_FP32_REFINE)
        return THOI_EINVAL;
    if (!valid_dtype(opts->out_dtype)) return THOI_EINVAL;
    int kmax = 0;
    int64_t B = 0;
    switch (sel->mode) {
        case THOI_SEL_RANGE: {
            if (N > THOI_MAX_N_RANGE) return THOI_EUNSUPPORTED;
            if (sel->kmin < 0 || sel->kmax < sel->kmin || sel->kmax > N) return THOI_EINVAL;
            if (sel->kmax > THOI_MAX_K) return THOI_EUNSUPPORTED;
            const int64_t total = count_orders(N, sel->kmin, sel->kmax);
            if (total < 0) return THOI_EUNSUPPORTED;
            if (sel->g_begin < 0 || sel->g_count < 0 || sel->g_begin > total || sel->g_count > total - sel->g_begin)
                return THOI_EINVAL;
            kmax = sel->kmax;
            B = sel->g_count;
            break;
        }
        case THOI_SEL_LIST:
            if (sel->B < 0 || sel->kmax_list < 1) return THOI_EINVAL;
            if (sel->kmax_list > THOI_MAX_K) return THOI_EUNSUPPORTED;
            if (sel->B > 0 && !sel->idx) return THOI_EINVAL;
            kmax = sel->kmax_list;
            B = sel->B;
            break;
        case THOI_SEL_MASK:
            if (sel->B < 0) return THOI_EINVAL;
            if (N > 64) return THOI_EUNSUPPORTED;
            if (sel->B > 0 && !sel->mask) return THOI_EINVAL;
            kmax = N;
            B = sel->B;
            break;
        default:
            return THOI_EINVAL;
    }
    if (D * B > 0 && !Sigma) return THOI_EINVAL;
    if (B > ((int64_t)1 << 40) || D * B > ((int64_t)1 << 42)) return THOI_EUNSUPPORTED;
    if (opts->bias_correct) {
        if (opts->bias_correct != 1) return THOI_EINVAL;
        if (opts->T < kmax + 2 || opts->T < 3) return THOI_EINVAL;
    }
    if (opts->write_entropy != 0 && opts->write_entropy != 1) return THOI_EINVAL;
    if (opts->seg_tiles < 0 || opts->grid_blocks < 0) return THOI_EINVAL;
    if (opts->engine < THOI_ENGINE_AUTO || opts->engine > THOI_ENGINE_PREFIX) return THOI_EINVAL;
    if (opts->seg_tiles > 4096) return THOI_EUNSUPPORTED;
    for (int c = 0; c < 8; ++c) {
        if (opts->class_seg_tiles[c] < 0 || opts->class_lanes[c] < 0 || opts->class_lanes[c] > 2) return THOI_EINVAL;
        if (opts->class_seg_tiles[c] > 4096) return THOI_EUNSUPPORTED;
    }
    if (forward) {
        if (opts->reduce) {
            const thoi_reduce* r = opts->reduce;
            if (r->topk < 0 || r->hist_bins < 0 || (r->topk == 0 && r->hist_bins == 0)) return THOI_EINVAL;
            if (r->topk > 256 || r->hist_bins > 4096) return THOI_EUNSUPPORTED;
            if (r->topk > 0 && (!r->top_val || !r->top_g)) return THOI_EINVAL;
            if (r->hist_bins > 0) {
                if (!r->hist || !r->hist_lo_hi) return THOI_EINVAL;
                for (int k = 0; k <= kmax; ++k) {
                    const double lo = r->hist_lo_hi[2 * k], hi = r->hist_lo_hi[2 * k + 1];
                    if (!(lo < hi) || !isfinite(lo) || !isfinite(hi)) return THOI_EINVAL;
                }
            }
        } else if (D * B > 0 && !out) {
            return THOI_EINVAL;
        }
    } else {
        if (opts->reduce) return THOI_EINVAL;
    }
    if (forward && eval_lds_bytes(N, sel, opts) > kLdsLimit) return THOI_EUNSUPPORTED;
    if (!forward && backward_lds_bytes(N, sel) > kLdsLimit) return THOI_EUNSUPPORTED;
    return THOI_OK;
}

extern "C" {

thoi_status thoi_copulize(const double* X, int64_t D, int64_t T, int64_t N, int32_t z_dtype, void* Z, void* ws,
                          size_t ws_bytes, void* stream)
{
    if (D < 0 || N < 1 || T < 2 || !valid_dtype(z_dtype)) return THOI_EINVAL;
    if (T > INT32_MAX - 1 || D > 65535 || N > 65535 || D * N > 65535) return THOI_EUNSUPPORTED;
    if (D > 0 && (!X || !Z)) return THOI_EINVAL;
    const size_t need = copulize_ws_bytes(D, T, N);
    if (!ws || ws_bytes < need) return THOI_EWORKSPACE;
    return launch_copulize(X, D, T, N, z_dtype, Z, ws, (hipStream_t)stream);
}

thoi_status thoi_cov(const void* Z, int32_t z_dtype, int64_t D, int64_t T, int64_t N, double* Sigma, void* ws,
                     size_t ws_bytes, void* stream)
{
    if (D < 0 || N < 1 || T < 2 || !valid_dtype(z_dtype)) return THOI_EINVAL;
    if (D > 65535 || N > 4096 || T > INT32_MAX) return THOI_EUNSUPPORTED;
    if (D > 0 && (!Z || !Sigma)) return THOI_EINVAL;
    const size_t need = cov_ws_bytes(D, T, N);
    if (!ws || ws_bytes < need) return THOI_EWORKSPACE;
    return launch_cov(Z, z_dtype, D, T, N, Sigma, ws, (hipStream_t)stream);
}

thoi_status thoi_nplets_eval(const double* Sigma, int64_t D, int32_t N, const thoi_nplets* sel,
                             const thoi_eval_opts* opts, void* out, uint8_t* flags, void* ws, size_t ws_bytes,
                             void* stream)
{
    const thoi_status st = check_eval(Sigma, D, N, sel, opts, true, out);
    if (st != THOI_OK) return st;
    return launch_eval(Sigma, D, N, sel, opts, out, flags, ws, ws_bytes, (hipStream_t)stream);
}

thoi_status thoi_eval_launch_shape(int32_t N, const thoi_nplets* sel, const thoi_eval_opts* opts,
                                   int32_t* n_launches, int64_t* max_items_x)
{
    if (!n_launches || !max_items_x) return THOI_EINVAL;
    // D = 0: the same checks as thoi_nplets_eval except those of Sigma and out
    const thoi_status st = check_eval(nullptr, 0, N, sel, opts, true, nullptr);
    if (st != THOI_OK) return st;
    eval_launch_shape(N, sel, opts, n_launches, max_items_x);
    return THOI_OK;
}

thoi_status thoi_nplets_eval_backward(const double* Sigma, int64_t D, int32_t N, const thoi_nplets* sel,
                                      const thoi_eval_opts* opts, const float* grad_out, float* grad_Sigma, void* ws,
                                      size_t ws_bytes, void* stream)
{
    const thoi_status st = check_eval(Sigma, D, N, sel, opts, false, nullptr);
    if (st != THOI_OK) return st;
    const int64_t B = sel->mode == THOI_SEL_RANGE ? sel->g_count : sel->B;
    if (D * B > 0 && (!grad_out || !grad_Sigma)) return THOI_EINVAL;
    return launch_backward(Sigma, D, N, sel, opts, grad_out, grad_Sigma, ws, ws_bytes, (hipStream_t)stream);
}

static thoi_status check_multi(const int32_t* N_d, const int32_t* T_d, int64_t D, int32_t kmin, int32_t kmax,
                               const thoi_eval_opts* opts, int64_t* total)
{
    if (!opts || D < 0 || (D > 0 && !N_d)) return THOI_EINVAL;
    if (opts->precision != THOI_FP64 && opts->precision != THOI_FP32 && opts->precision != THOI_FP32_REFINE)
        return THOI_EINVAL;
    if (!valid_dtype(opts->out_dtype) || opts->seg_tiles < 0 || opts->grid_blocks < 0) return THOI_EINVAL;
    if (opts->write_entropy != 0 && opts->write_entropy != 1) return THOI_EINVAL;
    if (kmin < 0 || kmax < kmin) return THOI_EINVAL;
    if (kmax > multi_lane_max(opts->precision) || opts->seg_tiles > 4096) return THOI_EUNSUPPORTED;
    if (opts->bias_correct && !T_d) return THOI_EINVAL;
    int nmax = 0;
    int64_t s = 0;
    for (int64_t d = 0; d < D; ++d) {
        if (N_d[d] < 1) return THOI_EINVAL;
        if (N_d[d] > THOI_MAX_N_RANGE) return THOI_EUNSUPPORTED;
        if (opts->bias_correct && (T_d[d] < kmax + 2 || T_d[d] < 3)) return THOI_EINVAL;
        nmax = N_d[d] > nmax ? N_d[d] : nmax;
        const int64_t c = count_orders(N_d[d], kmin, kmax);
        if (c < 0 || s > ((int64_t)1 << 42) - c) return THOI_EUNSUPPORTED;
        s += c;
    }
    if (opts->reduce) {
        const thoi_reduce* r = opts->reduce;
        if (r->topk < 0 || r->hist_bins < 0 || (r->topk == 0 && r->hist_bins == 0)) return THOI_EINVAL;
        if (r->topk > 256 || r->hist_bins > 4096) return THOI_EUNSUPPORTED;
        if (r->topk > 0 && (!r->top_val || !r->top_g)) return THOI_EINVAL;
        if (r->hist_bins > 0) {
            if (!r->hist || !r->hist_lo_hi) return THOI_EINVAL;
            for (int k = 0; k <= kmax; ++k) {
                const double lo = r->hist_lo_hi[2 * k], hi = r->hist_lo_hi[2 * k + 1];
                if (!(lo < hi) || !isfinite(lo) || !isfinite(hi)) return THOI_EINVAL;
            }
        }
    }
    if (D > 0 && multi_lds_bytes(nmax, kmax, opts) > kLdsLimit) return THOI_EUNSUPPORTED;
    *total = s;
    return THOI_OK;
}

thoi_status thoi_nplets_eval_multi(const double* Sigma, const int32_t* N_d, const int32_t* T_d, int64_t D,
                                   int32_t kmin, int32_t kmax, const thoi_eval_opts* opts, void* out,
                                   uint8_t* flags, void* ws, size_t ws_bytes, void* stream)
{
    int64_t total = 0;
    const thoi_status st = check_multi(N_d, T_d, D, kmin, kmax, opts, &total);
    if (st != THOI_OK) return st;
    if (total > 0 && !Sigma) return THOI_EINVAL;
    if (total > 0 && !opts->reduce && !out) return THOI_EINVAL;
    if (total == 0) return THOI_OK;
    return launch_multi(Sigma, N_d, T_d, D, kmin, kmax, opts, out, flags, ws, ws_bytes, (hipStream_t)stream);
}

thoi_status thoi_multi_offsets(const int32_t* N_d, int64_t D, int32_t kmin, int32_t kmax, int64_t* out_off)
{
    if (D < 0 || (D > 0 && !N_d) || !out_off || kmin < 0 || kmax < kmin) return THOI_EINVAL;
    int64_t s = 0;
    for (int64_t d = 0; d < D; ++d) {
        if (N_d[d] < 1 || N_d[d] > 64) return THOI_EINVAL;
        out_off[d] = s;
        const int64_t c = count_orders(N_d[d], kmin, kmax);
        if (c < 0) return THOI_EUNSUPPORTED;
        s += c;
    }
    out_off[D] = s;
    return THOI_OK;
}

size_t thoi_multi_workspace_bytes(const int32_t* N_d, int64_t D, int32_t kmin, int32_t kmax,
                                  const thoi_eval_opts* opts)
{
    int64_t total = 0;
    if (check_multi(N_d, nullptr, D, kmin, kmax, opts, &total) != THOI_OK && !(opts && opts->bias_correct)) return 0;
    return multi_ws_bytes(N_d, D, kmin, kmax, opts);
}

thoi_status thoi_reduce_init(const thoi_reduce* red, int64_t D, int32_t kmax, void* stream)
{
    if (!red || D < 0 || kmax < 0 || kmax > THOI_MAX_K) return THOI_EINVAL;
    if (red->topk < 0 || red->hist_bins < 0) return THOI_EINVAL;
    if (red->topk > 256 || red->hist_bins > 4096) return THOI_EUNSUPPORTED;
    if (D > 0 && red->topk > 0 && (!red->top_val || !red->top_g)) return THOI_EINVAL;
    if (D > 0 && red->hist_bins > 0 && !red->hist) return THOI_EINVAL;
    return launch_reduce_init(red, D, kmax, (hipStream_t)stream);
}

thoi_status thoi_objective(const void* vals, int32_t val_dtype, int64_t D, int64_t B, int32_t kind, double* obj,
                           const thoi_reduce* red, void* ws, size_t ws_bytes, void* stream)
{
    if (D < 1 || B < 0 || !valid_dtype(val_dtype)) return THOI_EINVAL;
    if (kind != THOI_OBJ_MEAN && kind != THOI_OBJ_PAIRED_EFFECT) return THOI_EINVAL;
    if (kind == THOI_OBJ_PAIRED_EFFECT && (D % 2 != 0 || D < 4)) return THOI_EINVAL;
    if (!obj && !red) return THOI_EINVAL;
    if (D > 65535 || B > ((int64_t)1 << 40)) return THOI_EUNSUPPORTED;
    if (B > 0 && !vals) return THOI_EINVAL;
    if (red) {
        if (red->topk < 0 || red->hist_bins < 0 || (red->topk == 0 && red->hist_bins == 0)) return THOI_EINVAL;
        if (red->topk > 256 || red->hist_bins > 4096) return THOI_EUNSUPPORTED;
        if (red->topk > 0 && (!red->top_val || !red->top_g)) return THOI_EINVAL;
        if (red->hist_bins > 0) {
            if (!red->hist || !red->hist_lo_hi) return THOI_EINVAL;
            const double lo = red->hist_lo_hi[0], hi = red->hist_lo_hi[1];
            if (!(lo < hi) || !std::isfinite(lo) || !std::isfinite(hi)) return THOI_EINVAL;
        }
    }
    if (!ws || ws_bytes < objective_ws_bytes(D, B, red)) return THOI_EWORKSPACE;
    return launch_objective(vals, val_dtype, D, B, kind, obj, red, ws, (hipStream_t)stream);
}

thoi_status thoi_anneal(const double* Sigma, int32_t N, const uint64_t* masks0, int32_t kappa, int32_t iters,
                        const double* draw_move, const double* draw_a, const double* draw_b, const double* draw_accept,
                        double T0, double alpha, int32_t maximize, int32_t across, int32_t k_min, int32_t k_max,
                        uint64_t* cur_mask, double* cur_omega, uint64_t* best_mask, double* best_omega,
                        int64_t* accepted, void* stream)
{
    if (N < 2 || N > 128 || kappa < 1 || iters < 0) return THOI_EINVAL;
    if (kappa > (1 << 20) || (int64_t)iters * kappa > ((int64_t)1 << 40)) return THOI_EUNSUPPORTED;
    if (k_min < 1 || k_min > k_max || k_max > N - 1) return THOI_EINVAL;
    if (k_max > 64) return THOI_EUNSUPPORTED;
    if (!(T0 > 0.0) || !std::isfinite(T0) || !(alpha > 0.0) || !std::isfinite(alpha)) return THOI_EINVAL;
    if (!Sigma || !masks0 || !cur_mask || !cur_omega || !best_mask || !best_omega || !accepted) return THOI_EINVAL;
    if (iters > 0 && (!draw_a || !draw_b || !draw_accept || (across && !draw_move))) return THOI_EINVAL;
    return launch_anneal(Sigma, N, masks0, kappa, iters, draw_move, draw_a, draw_b, draw_accept, T0, alpha, maximize,
                         across, k_min, k_max, cur_mask, cur_omega, best_mask, best_omega, accepted,
                         (hipStream_t)stream);
}

thoi_status thoi_greedy(const double* Sigma, int64_t D, int32_t N, int32_t k_first, int32_t steps, int32_t kappa,
                        int32_t measure, int32_t kind, int32_t maximize, uint64_t* sols, double* vals, int32_t* count,
                        void* ws, size_t ws_bytes, void* stream)
{
    if (D < 1 || N < 2 || N > 128 || k_first < 1 || steps < 0 || kappa < 1 || kappa > 256) return THOI_EINVAL;
    if (measure < 0 || measure > 3) return THOI_EINVAL;
    if (kind != THOI_OBJ_MEAN && kind != THOI_OBJ_PAIRED_EFFECT) return THOI_EINVAL;
    if (kind == THOI_OBJ_PAIRED_EFFECT && (D % 2 != 0 || D < 4)) return THOI_EINVAL;
    if (k_first + steps > N) return THOI_EINVAL;
    if (D > 65535 || k_first + steps > 64 || (int64_t)kappa * N > greedy_select_max()) return THOI_EUNSUPPORTED;
    if (!Sigma || !sols || !vals || !count) return THOI_EINVAL;
    if (steps == 0) return THOI_OK;
    if (!ws || ws_bytes < greedy_ws_bytes(D, N, kappa)) return THOI_EWORKSPACE;
    return launch_greedy(Sigma, D, N, k_first, kappa, steps, measure, kind, maximize, sols, vals, count, ws,
                         (hipStream_t)stream);
}

size_t thoi_greedy_workspace_bytes(int64_t D, int32_t N, int32_t kappa)
{
    return (D >= 1 && N >= 1 && kappa >= 1) ? greedy_ws_bytes(D, N, kappa) : 0;
}

size_t thoi_objective_workspace_bytes(int64_t D, int64_t B, const thoi_reduce* red)
{
    return (D >= 1 && B >= 0) ? objective_ws_bytes(D, B, red) : 0;
}

size_t thoi_workspace_bytes(int32_t which, int64_t D, int64_t T, int32_t N, const thoi_nplets* sel,
                            const thoi_eval_opts* opts)
{
    switch (which) {
        case THOI_WS_COPULIZE: return (D >= 0 && T >= 1 && N >= 1) ? copulize_ws_bytes(D, T, N) : 0;
        case THOI_WS_COV: return (D >= 0 && T >= 1 && N >= 1) ? cov_ws_bytes(D, T, N) : 0;
        case THOI_WS_EVAL: return (sel && opts && D >= 0) ? eval_ws_bytes(D, N, sel, opts) : 0;
        case THOI_WS_BACKWARD: return (sel && opts && D >= 0) ? backward_ws_bytes(D, N, sel, opts) : 0;
        default: return 0;
    }
}

size_t thoi_ws_status_offset(void) { return 0; }

int64_t thoi_count(int32_t N, int32_t kmin, int32_t kmax) { return count_orders(N, kmin, kmax); }

thoi_status thoi_unrank_host(int32_t N, int32_t kmin, int64_t g, int32_t* out_k, int32_t* out_idx)
{
    if (N < 1 || N > 64 || kmin < 0 || kmin > N || g < 0 || !out_k || !out_idx) return THOI_EINVAL;
    int k = kmin;
    uint64_t r = (uint64_t)g;
    while (k <= N && r >= binom_u64(N, k)) { r -= binom_u64(N, k); ++k; }
    if (k > N) return THOI_EINVAL;
    int x = 0;
    for (int i = 0; i < k; ++i) {
        const int m = k - 1 - i;
        while (r >= binom_u64(N - 1 - x, m)) { r -= binom_u64(N - 1 - x, m); ++x; }
        out_idx[i] = x++;
    }
    *out_k = k;
    return THOI_OK;
}

thoi_status thoi_bias_offsets(int32_t k, int32_t T, double* d_tc, double* d_dtc, double* eta_k)
{
    if (k < 0 || k > THOI_MAX_K || T < k + 2 || T < 3 || !d_tc || !d_dtc || !eta_k) return THOI_EINVAL;
    bias_offsets(k, T, d_tc, d_dtc, eta_k);
    return THOI_OK;
}

const char* thoi_status_string(thoi_status s)
{
    switch (s) {
        case THOI_OK: return "ok";
        case THOI_EINVAL: return "invalid argument";
        case THOI_EUNSUPPORTED: return "unsupported size or option";
        case THOI_EWORKSPACE: return "workspace missing or too small";
        case THOI_EHIP: return "HIP runtime error";
        case THOI_EINVAL_DATA: return "invalid data (NaN in X or bad n-plet row)";
        default: return "unknown status";
    }
}

const char* thoi_version(void) { return "thoi-mi355x 0.1 (gfx950)"; }

}  // extern "C"
