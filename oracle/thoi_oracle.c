/*
 * thoi_oracle.c -- plain, slow, FP64 CPU oracle for the Gaussian-copula
 * higher-order-interaction measures (TC, DTC, O-information, S-information)
 * of THOI (arXiv 2501.03381).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or constant
 * generator with the HIP library.
 *
 * Every function computes the plain definition written in the paper:
 *   - Gaussian-copula covariance: Supplementary "Estimation of entropy via
 *     Gaussian copulas", Eq. (gaussian_copula_covariance_estimator):
 *     rank each variable, map rank/(T+1) through the inverse standard-normal
 *     CDF, take the covariance of the result.
 *   - Gaussian entropy: Supplementary "Entropy analytical expression for
 *     multivariate Gaussian variables", Eq. (gaussian_differential_entropy):
 *     H = 1/2 log((2 pi e)^n det Sigma).
 *   - Finite-sample bias corrector, Eq. (bias_corrector), with the reading
 *     eta(n) = 1/2 [ n log(2/(T-1)) + sum_{j=1..n} psi((T-j)/2) ].
 *   - TC, DTC, Omega, S: Methods "Generalizations of the mutual information",
 *     Eqs. (TC), (DTC), (O-info), (S-info), evaluated literally from the
 *     entropies H(X_j), H(X^n) and H(X^n_{-j}) that Methods "Parallel and
 *     batched computation of HOI" lists.  Every determinant -- the joint one
 *     and each of the n leave-one-out ones -- is a separate LU factorisation
 *     with partial pivoting.  No inverse-diagonal identity is used.
 *   - n-plet enumeration: all k-subsets of {0..N-1} for k = kmin..kmax in
 *     ascending order, lexicographic within an order (Supplementary "The
 *     combinatorial explosion", Eq. (comb) gives their count).
 *   - Gradient of the measures with respect to the covariance entries:
 *     derivative of log det (matrix inverse) and of the inverse-matrix
 *     diagonal, formed from an explicit inverse; checked in the tests against
 *     central finite differences of the literal measures.
 *
 * Precision: FP64 throughout.  Parity status: every function here is pinned
 * by tests against closed forms, library routines or brute force; none is
 * "parity unpinned".
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_LOG_2PIE 2.8378770664093454836 /* log(2 pi e) */
#define OR_FLAG_NOT_PD 2

/* ------------------------------------------------------------------------ */
/* Standard normal CDF / PDF from the C library's erfc.                       */
/* ------------------------------------------------------------------------ */
static double or_phi_cdf(double x) { return 0.5 * erfc(-x / sqrt(2.0)); }
static double or_phi_pdf(double x) { return exp(-0.5 * x * x) / sqrt(2.0 * M_PI); }

/* Quantile of the lower half: the x <= 0 with Phi(x) = p, for 0 < p <= 1/2.
 * Starting guess: Abramowitz & Stegun 26.2.23 (|error| < 4.5e-4); then
 * safeguarded Newton steps on Phi(x) - p inside a shrinking bracket. */
static double or_lower_quantile(double p)
{
    double t = sqrt(-2.0 * log(p));
    double x = -(t - (2.515517 + 0.802853 * t + 0.010328 * t * t) /
                     (1.0 + 1.432788 * t + 0.189269 * t * t + 0.001308 * t * t * t));
    double lo = -40.0, hi = 0.0;
    if (x > hi) x = hi;
    if (x < lo) x = lo;
    for (int it = 0; it < 200; ++it) {
        double f = or_phi_cdf(x) - p;
        if (f == 0.0) break;
        if (f > 0.0) hi = x; else lo = x;
        double xn = x - f / or_phi_pdf(x);
        if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
        double step = fabs(xn - x);
        x = xn;
        if (step <= 1e-17 * (1.0 + fabs(x))) break;
        if (hi - lo <= 4e-16 * (1.0 + fabs(x))) break;
    }
    return x;
}

/* Inverse standard-normal CDF for 0 < p < 1 (used for checking only). */
double or_ndtri(double p)
{
    if (!(p > 0.0 && p < 1.0)) return NAN;
    if (p <= 0.5) return or_lower_quantile(p);
    return -or_lower_quantile(1.0 - p); /* 1-p is exact for p in [1/2, 1) */
}

/* Normal score of rank r in 1..T: Phi^{-1}(r/(T+1)).  The upper half uses
 * the exact integer complement so that score(r) = -score(T+1-r). */
double or_normal_score(int64_t r, int64_t T)
{
    int64_t den = T + 1;
    if (2 * r <= den) return or_lower_quantile((double)r / (double)den);
    return -or_lower_quantile((double)(den - r) / (double)den);
}

/* ------------------------------------------------------------------------ */
/* Digamma: recurrence psi(x) = psi(x+1) - 1/x up to x >= 10, then the       */
/* asymptotic series ln x - 1/(2x) - sum B_2n / (2n x^2n).                    */
/* ------------------------------------------------------------------------ */
double or_digamma(double x)
{
    if (!(x > 0.0)) return NAN;
    double acc = 0.0;
    while (x < 10.0) { acc -= 1.0 / x; x += 1.0; }
    double r = 1.0 / (x * x);
    /* B2/2 = 1/12, B4/4 = -1/120, B6/6 = 1/252, B8/8 = -1/240, B10/10 = 1/132,
     * B12/12 = -691/32760 */
    double series = r * (1.0 / 12 - r * (1.0 / 120 - r * (1.0 / 252 - r * (1.0 / 240 - r * (1.0 / 132 - r * (691.0 / 32760))))));
    return acc + log(x) - 0.5 / x - series;
}

/* Bias corrector eta(n) for an n-variate entropy from T samples. */
double or_bias_eta(int n, int64_t T)
{
    if (n <= 0) return 0.0;
    double s = 0.5 * n * log(2.0 / (double)(T - 1));
    double ps = 0.0;
    for (int j = 1; j <= n; ++j) ps += or_digamma(0.5 * (double)(T - j));
    return s + 0.5 * ps;
}

/* ------------------------------------------------------------------------ */
/* Gaussian copula of one dataset X [T][N] (sample-major) -> Z [T][N].       */
/* Ranks are 1-based ordinal ranks; equal values are ranked by sample index. */
/* ------------------------------------------------------------------------ */
typedef struct { double v; int64_t i; } or_keyed;

static int or_keyed_cmp(const void* a, const void* b)
{
    const or_keyed* x = (const or_keyed*)a;
    const or_keyed* y = (const or_keyed*)b;
    if (x->v < y->v) return -1;
    if (x->v > y->v) return 1;
    return (x->i < y->i) ? -1 : (x->i > y->i) ? 1 : 0;
}

/* Returns 0, or -1 if X holds a NaN or T < 2. */
int or_copula(const double* X, int64_t T, int64_t N, double* Z)
{
    if (T < 2) return -1;
    for (int64_t t = 0; t < T * N; ++t)
        if (isnan(X[t])) return -1;
    or_keyed* buf = (or_keyed*)malloc(sizeof(or_keyed) * (size_t)T);
    for (int64_t c = 0; c < N; ++c) {
        for (int64_t t = 0; t < T; ++t) { buf[t].v = X[t * N + c]; buf[t].i = t; }
        qsort(buf, (size_t)T, sizeof(or_keyed), or_keyed_cmp);
        for (int64_t p = 0; p < T; ++p)
            Z[buf[p].i * N + c] = or_normal_score(p + 1, T);
    }
    free(buf);
    return 0;
}

/* Sample covariance with mean-centring and 1/(T-1): S [N][N]. */
void or_covariance(const double* Z, int64_t T, int64_t N, double* S)
{
    double* mean = (double*)calloc((size_t)N, sizeof(double));
    for (int64_t t = 0; t < T; ++t)
        for (int64_t c = 0; c < N; ++c) mean[c] += Z[t * N + c];
    for (int64_t c = 0; c < N; ++c) mean[c] /= (double)T;
    for (int64_t a = 0; a < N; ++a)
        for (int64_t b = 0; b < N; ++b) {
            double s = 0.0;
            for (int64_t t = 0; t < T; ++t)
                s += (Z[t * N + a] - mean[a]) * (Z[t * N + b] - mean[b]);
            S[a * N + b] = s / (double)(T - 1);
        }
    free(mean);
}

/* ------------------------------------------------------------------------ */
/* Dense linear algebra on small matrices.                                    */
/* ------------------------------------------------------------------------ */

/* log|det A| and sign by LU with partial pivoting; A [n][n] is overwritten.
 * The empty matrix has determinant 1. */
double or_lu_logdet(double* A, int n, int* sign)
{
    int s = 1;
    double acc = 0.0;
    for (int c = 0; c < n; ++c) {
        int piv = c;
        double best = fabs(A[c * n + c]);
        for (int r = c + 1; r < n; ++r)
            if (fabs(A[r * n + c]) > best) { best = fabs(A[r * n + c]); piv = r; }
        if (!(best > 0.0)) { *sign = 0; return -INFINITY; }
        if (piv != c) {
            for (int j = 0; j < n; ++j) {
                double tmp = A[c * n + j]; A[c * n + j] = A[piv * n + j]; A[piv * n + j] = tmp;
            }
            s = -s;
        }
        double u = A[c * n + c];
        if (u < 0) s = -s;
        acc += log(fabs(u));
        for (int r = c + 1; r < n; ++r) {
            double m = A[r * n + c] / u;
            for (int j = c; j < n; ++j) A[r * n + j] -= m * A[c * n + j];
        }
    }
    *sign = s;
    return acc;
}

/* Positive definiteness of a symmetric matrix (Sylvester's criterion): the
 * pivots of Gaussian elimination without row exchanges are the ratios of
 * consecutive leading principal minors, so all must be > 0. */
int or_is_pd(const double* A0, int n)
{
    double* A = (double*)malloc(sizeof(double) * (size_t)(n * n > 0 ? n * n : 1));
    memcpy(A, A0, sizeof(double) * (size_t)(n * n));
    int ok = 1;
    for (int c = 0; c < n && ok; ++c) {
        double u = A[c * n + c];
        if (!(u > 0.0) || !isfinite(u)) { ok = 0; break; }
        for (int r = c + 1; r < n; ++r) {
            double m = A[r * n + c] / u;
            for (int j = c; j < n; ++j) A[r * n + j] -= m * A[c * n + j];
        }
    }
    free(A);
    return ok;
}

/* Explicit inverse by Gauss-Jordan elimination with partial pivoting.
 * Returns 0 on success. */
int or_inverse(const double* A0, int n, double* Ainv)
{
    int w = 2 * n;
    double* M = (double*)malloc(sizeof(double) * (size_t)(n * w));
    for (int r = 0; r < n; ++r)
        for (int j = 0; j < w; ++j)
            M[r * w + j] = (j < n) ? A0[r * n + j] : (j - n == r ? 1.0 : 0.0);
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (fabs(M[r * w + c]) > fabs(M[piv * w + c])) piv = r;
        if (!(fabs(M[piv * w + c]) > 0.0)) { free(M); return -1; }
        if (piv != c)
            for (int j = 0; j < w; ++j) { double t = M[c * w + j]; M[c * w + j] = M[piv * w + j]; M[piv * w + j] = t; }
        double u = M[c * w + c];
        for (int j = 0; j < w; ++j) M[c * w + j] /= u;
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            double m = M[r * w + c];
            if (m == 0.0) continue;
            for (int j = 0; j < w; ++j) M[r * w + j] -= m * M[c * w + j];
        }
    }
    for (int r = 0; r < n; ++r)
        for (int j = 0; j < n; ++j) Ainv[r * n + j] = M[r * w + n + j];
    free(M);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Measures of one n-plet, literally from entropies.                         */
/* ------------------------------------------------------------------------ */

/* Gaussian entropy of the sub-matrix of S [N][N] on indices idx[0..m-1];
 * sets *ok = 0 if its determinant is not positive. */
static double or_subset_entropy(const double* S, int N, const int* idx, int m, int* ok)
{
    if (m == 0) { *ok = 1; return 0.0; }
    double* A = (double*)malloc(sizeof(double) * (size_t)(m * m));
    for (int a = 0; a < m; ++a)
        for (int b = 0; b < m; ++b) A[a * m + b] = S[idx[a] * N + idx[b]];
    int sign = 0;
    double ld = or_lu_logdet(A, m, &sign);
    free(A);
    *ok = (sign > 0) && isfinite(ld);
    return 0.5 * (m * OR_LOG_2PIE + ld);
}

/*
 * Measures of the n-plet idx[0..k-1] of covariance S [N][N].
 * out4 = {TC, DTC, Omega, S}; *Hout = H(X^n) (bias-corrected if asked).
 * bias != 0 subtracts eta(m) from every m-variate entropy (T samples).
 * Returns 0, or OR_FLAG_NOT_PD (outputs NaN) if the sub-matrix is not
 * positive definite, or -1 if the two printed forms of Omega disagree.
 */
int or_measures(const double* S, int N, const int* idx, int k, int bias, int64_t T,
                double* out4, double* Hout)
{
    double* sub = (double*)malloc(sizeof(double) * (size_t)(k * k > 0 ? k * k : 1));
    for (int a = 0; a < k; ++a)
        for (int b = 0; b < k; ++b) sub[a * k + b] = S[idx[a] * N + idx[b]];
    int pd = or_is_pd(sub, k);
    free(sub);
    if (!pd) {
        for (int m = 0; m < 4; ++m) out4[m] = NAN;
        if (Hout) *Hout = NAN;
        return OR_FLAG_NOT_PD;
    }
    int ok = 1, okj = 1;
    double e_k = bias ? or_bias_eta(k, T) : 0.0;
    double e_1 = bias ? or_bias_eta(1, T) : 0.0;
    double e_km1 = bias ? or_bias_eta(k - 1, T) : 0.0;

    double Hn = or_subset_entropy(S, N, idx, k, &ok) - e_k;          /* H(X^n) */
    double sumHj = 0.0, sumHloo = 0.0, sumCond = 0.0;
    int* rest = (int*)malloc(sizeof(int) * (size_t)(k > 1 ? k - 1 : 1));
    for (int j = 0; j < k; ++j) {
        double Hj = 0.5 * (OR_LOG_2PIE + log(S[idx[j] * N + idx[j]])) - e_1;   /* H(X_j) */
        int m = 0;
        for (int a = 0; a < k; ++a) if (a != j) rest[m++] = idx[a];
        double Hloo = or_subset_entropy(S, N, rest, k - 1, &okj) - e_km1;    /* H(X^n_{-j}) */
        ok = ok && okj;
        sumHj += Hj;
        sumHloo += Hloo;
        sumCond += Hn - Hloo;                                                 /* H(X_j | X^n_{-j}) */
    }
    free(rest);
    if (!ok) {
        for (int m = 0; m < 4; ++m) out4[m] = NAN;
        if (Hout) *Hout = NAN;
        return OR_FLAG_NOT_PD;
    }
    double TC = sumHj - Hn;                 /* Eq. (TC)     */
    double DTC = Hn - sumCond;              /* Eq. (DTC)    */
    double Om = TC - DTC;                   /* Eq. (O-info), first form  */
    double Si = TC + DTC;                   /* Eq. (S-info) */
    double Om2 = (k - 2) * Hn + (sumHj - sumHloo);   /* Eq. (O-info), second form */
    out4[0] = TC; out4[1] = DTC; out4[2] = Om; out4[3] = Si;
    if (Hout) *Hout = Hn;
    double scale = 1.0 + fabs(Hn) * k + fabs(sumHj) + fabs(sumHloo);
    if (fabs(Om - Om2) > 1e-11 * scale) return -1;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Batched evaluation over an explicit n-plet list.                          */
/* idx [B][kmax]: sorted ascending, padded with -1.  out [4][B], H [B],       */
/* flags [B].  nthreads <= 0 uses the OpenMP default.                        */
/* ------------------------------------------------------------------------ */
int or_eval_list(const double* S, int N, const int32_t* idx, int64_t B, int kmax,
                 int bias, int64_t T, double* out, double* H, uint8_t* flags, int nthreads)
{
    int bad = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 64) reduction(| : bad)
#endif
    for (int64_t b = 0; b < B; ++b) {
        int tuple[128];
        int k = 0;
        for (int j = 0; j < kmax && j < 128; ++j) {
            int v = idx[b * kmax + j];
            if (v < 0) break;
            tuple[k++] = v;
        }
        double o[4], h;
        int rc = or_measures(S, N, tuple, k, bias, T, o, &h);
        if (rc < 0) bad = 1;
        for (int m = 0; m < 4; ++m) out[m * B + b] = o[m];
        if (H) H[b] = h;
        if (flags) flags[b] = (uint8_t)(rc == OR_FLAG_NOT_PD ? OR_FLAG_NOT_PD : 0);
    }
    return bad ? -1 : 0;
}

/* Number of threads the OpenMP runtime would use. */
int or_max_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
    return omp_get_max_threads();
#else
    (void)nthreads;
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Enumeration: all k-subsets, k = kmin..kmax, lexicographic within an order. */
/* Writes [count][kmax] padded with -1 if out != NULL; returns the count.     */
/* ------------------------------------------------------------------------ */
int64_t or_enumerate(int N, int kmin, int kmax, int32_t* out)
{
    int64_t n = 0;
    int c[128];
    for (int k = kmin; k <= kmax; ++k) {
        if (k > N || k < 0) continue;
        for (int j = 0; j < k; ++j) c[j] = j;
        for (;;) {
            if (out) {
                for (int j = 0; j < kmax; ++j) out[n * kmax + j] = (j < k) ? c[j] : -1;
            }
            ++n;
            /* next k-subset in lexicographic order */
            int j = k - 1;
            while (j >= 0 && c[j] == N - k + j) --j;
            if (j < 0) break;
            ++c[j];
            for (int i = j + 1; i < k; ++i) c[i] = c[i - 1] + 1;
        }
    }
    return n;
}

/* ------------------------------------------------------------------------ */
/* Gradient: G [N][N] += sum_b sum_m w[m][b] d(measure_m of n-plet b)/dS.    */
/* Entries of S are treated as independent (G is symmetric).                  */
/*   d log det(S_b)/dS_pq  = (S_b^{-1})_pq                                    */
/*   d a_j / dS_pq         = -(A)_jp (A)_qj   with A = S_b^{-1}, a_j = A_jj  */
/* TC = 1/2[sum log d_j - log det], DTC = 1/2[log det + sum log a_j] follow  */
/* from the Gaussian entropy and the cofactor expansion of the leave-one-out */
/* determinants; the tests check this gradient against finite differences  */
/* of or_measures, which never uses that expansion.                          */
/* ------------------------------------------------------------------------ */
int or_grad_list(const double* S, int N, const int32_t* idx, int64_t B, int kmax,
                 const double* w /* [4][B] */, double* G)
{
    int bad = 0;
    for (int64_t b = 0; b < B; ++b) {
        int t[128], k = 0;
        for (int j = 0; j < kmax && j < 128; ++j) { int v = idx[b * kmax + j]; if (v < 0) break; t[k++] = v; }
        if (k == 0) continue;
        double* sub = (double*)malloc(sizeof(double) * (size_t)(k * k));
        double* A = (double*)malloc(sizeof(double) * (size_t)(k * k));
        for (int p = 0; p < k; ++p)
            for (int q = 0; q < k; ++q) sub[p * k + q] = S[t[p] * N + t[q]];
        if (!or_is_pd(sub, k) || or_inverse(sub, k, A) != 0) { bad = 1; free(sub); free(A); continue; }
        double wTC = w[0 * B + b], wDTC = w[1 * B + b], wO = w[2 * B + b], wS = w[3 * B + b];
        /* coefficient of each building block:
         *   dTC  = 1/2 [diag(1/d) - A]
         *   dDTC = 1/2 [A - A diag(1/a) A]
         *   Omega = TC - DTC,  S = TC + DTC                                  */
        double cT = wTC + wO + wS;   /* total weight on dTC  */
        double cD = wDTC - wO + wS;  /* total weight on dDTC */
        for (int p = 0; p < k; ++p)
            for (int q = 0; q < k; ++q) {
                double AdA = 0.0;
                for (int j = 0; j < k; ++j) AdA += A[p * k + j] * A[j * k + q] / A[j * k + j];
                double dTC = 0.5 * ((p == q ? 1.0 / sub[p * k + p] : 0.0) - A[p * k + q]);
                double dDTC = 0.5 * (A[p * k + q] - AdA);
                G[t[p] * N + t[q]] += cT * dTC + cD * dDTC;
            }
        free(sub);
        free(A);
    }
    return bad ? -1 : 0;
}
