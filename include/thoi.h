/*
 * thoi.h -- C ABI of libthoi.so: Gaussian-copula higher-order-interaction
 * measures over batches of n-plets on AMD Instinct MI355X (gfx950).
 *
 * Method: THOI (arXiv 2501.03381).  For data X with T samples of N variables
 * the Gaussian-copula covariance Sigma (Supplementary, "Estimation of entropy
 * via Gaussian copulas", Eq. gaussian_copula_covariance_estimator) gives the
 * Gaussian entropy of any subset S of variables in closed form
 * (Supplementary, Eq. gaussian_differential_entropy).  For every selected
 * n-plet S the library returns the total correlation, dual total correlation,
 * O-information and S-information (Methods, Eqs. TC, DTC, O-info, S-info),
 * pairing each n-plet with each of D covariance matrices (Methods, "Parallel
 * and batched computation of HOI").
 *
 * Conventions shared by every call
 *  - Pointers documented as "device" are HIP device pointers owned by the
 *    caller; "host" pointers are ordinary host memory read during the call.
 *    The library keeps no device memory between calls.
 *  - `stream` is a hipStream_t (NULL = the null stream).  Device work is
 *    enqueued on it and the call returns without synchronising.
 *  - Argument errors are detected on the host before anything is enqueued and
 *    returned as a negative thoi_status; nothing is written in that case.
 *  - Errors found in the data on the device (NaN in X, too many n-plets to
 *    refine for the workspace) are reported through the int32 status word at
 *    the start of the workspace (see thoi_ws_status_offset), read by the
 *    caller after synchronising; it holds THOI_OK or a thoi_status.
 *  - Numerical failure of one n-plet (a sub-matrix that is not positive
 *    definite) is not an API error: its outputs are NaN and its flag byte
 *    has THOI_NPLET_NOT_PD.
 *  - Units are nats.  Layouts are C order (last index fastest).
 */
#ifndef THOI_H_
#define THOI_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    THOI_OK = 0,
    THOI_EINVAL = -1,        /* bad argument: shape, pointer, mode or option        */
    THOI_EUNSUPPORTED = -2,  /* valid request outside the built limits (N, k, T)     */
    THOI_EWORKSPACE = -3,    /* workspace missing or too small                       */
    THOI_EHIP = -4,          /* the HIP runtime reported an error on launch          */
    THOI_EINVAL_DATA = -5    /* device-detected: NaN in the data                     */
} thoi_status;

/* precision of the per-n-plet evaluation */
enum { THOI_FP64 = 0, THOI_FP32 = 1, THOI_FP32_REFINE = 2 };
/* element type of Z or of the output planes */
enum { THOI_DTYPE_F64 = 0, THOI_DTYPE_F32 = 1 };
/* n-plet selection */
enum { THOI_SEL_RANGE = 0, THOI_SEL_LIST = 1, THOI_SEL_MASK = 2 };
/* per-n-plet flag bits */
enum { THOI_NPLET_REFINED = 1, THOI_NPLET_NOT_PD = 2 };
/* which call a workspace is for */
enum { THOI_WS_COPULIZE = 0, THOI_WS_COV = 1, THOI_WS_EVAL = 2, THOI_WS_BACKWARD = 3 };

/* Built limits. */
#define THOI_MAX_N_RANGE 62   /* RANGE mode: global indices are int64 and binomials exact in uint64 */
#define THOI_MAX_N 128        /* variables per covariance matrix (the matrix is staged in LDS)       */
#define THOI_MAX_K 64         /* largest n-plet order                                              */

/*
 * Which n-plets to evaluate.  Output position b (0 <= b < B) is:
 *  RANGE: b-th n-plet of the global enumeration restricted to [g_begin,
 *         g_begin + g_count).  The global enumeration lists orders kmin..kmax
 *         in ascending order and, within an order, the k-subsets of
 *         {0..N-1} in lexicographic order (the order of Python's
 *         itertools.combinations); g is its 0-based int64 position.  B =
 *         g_count.  Requires N <= THOI_MAX_N_RANGE.  The count of orders 3..N
 *         is 2^N - 1 - N - N(N-1)/2 (Supplementary, Eq. comb).
 *  LIST:  row b of idx (device, [B][kmax_list] int32): strictly ascending
 *         variable indices in [0, N), then -1 padding.  The order of row b is
 *         its number of non-negative entries (1 <= k <= THOI_MAX_K).
 *  MASK:  bit j of mask[b] (device, [B] uint64) selects variable j; N <= 64.
 */
typedef struct {
    int32_t mode;
    int32_t kmin, kmax;          /* RANGE */
    int64_t g_begin, g_count;    /* RANGE */
    const int32_t* idx;          /* LIST, device */
    int32_t kmax_list;           /* LIST */
    const uint64_t* mask;        /* MASK, device */
    int64_t B;                   /* LIST / MASK: number of n-plets */
} thoi_nplets;

/*
 * Optional streaming reduction of Omega per (dataset d, order k), replacing
 * the full output planes (Figure 1A: a per-batch custom function, e.g. the
 * minimum Omega, aggregated on the fly).  All device arrays are accumulated
 * across calls (+= / merge), so a long enumeration can be split into RANGE
 * pieces; the caller initialises them with thoi_reduce_init.
 *   top_val/top_g: device [D][kmax+1][2][topk]; slot [..][0][..] holds the
 *     topk largest Omega in descending order, [..][1][..] the topk smallest
 *     in ascending order; ties are ordered by the lower global index g;
 *     unused slots have g = -1.
 *   hist: device [D][kmax+1][hist_bins+2] uint64: bin i counts Omega in
 *     [lo + i w, lo + (i+1) w) with w = (hi-lo)/hist_bins (Omega == hi goes
 *     to the last bin), then the counts below lo and above hi.  NaN results
 *     (not positive definite) are not counted.
 *   hist_lo_hi: host [kmax+1][2] range per order (lo < hi, finite).
 * kmax is the selection's largest order: RANGE kmax, LIST kmax_list, MASK N.
 * In reduce mode no output planes are written (out may be NULL) and the
 * entropy plane is not produced; n-plets refined in FP64 enter with their
 * FP64 value.  The workspace must be sized with the same thoi_reduce.
 */
typedef struct {
    int32_t topk;                /* 0 = off; at most 256 */
    int32_t hist_bins;           /* 0 = off; at most 4096 */
    const double* hist_lo_hi;    /* host */
    double* top_val;             /* device */
    int64_t* top_g;              /* device */
    uint64_t* hist;              /* device */
} thoi_reduce;

typedef struct {
    int32_t precision;           /* THOI_FP64, THOI_FP32, THOI_FP32_REFINE                      */
    int32_t out_dtype;           /* THOI_DTYPE_F64 or THOI_DTYPE_F32 for the output planes      */
    double vif_tau;              /* FP32_REFINE: re-evaluate in FP64 if max_j VIF_j > vif_tau   */
                                 /* (VIF_j = Sigma_jj (Sigma_S^-1)_jj); <= 0 selects 1e3       */
    int32_t bias_correct;        /* 1: subtract eta(m) of Eq. bias_corrector from every          */
                                 /* m-variate entropy, read as 1/2[m log(2/(T-1)) + sum psi]   */
    int32_t T;                   /* samples per dataset (bias correction only)                  */
    int32_t write_entropy;       /* 1: a fifth output plane with H(X^n)                          */
    const thoi_reduce* reduce;   /* host; NULL = write the full output planes                    */
    int32_t seg_tiles;           /* tuning: tiles of 256 n-plets per workgroup; 0 = library choice */
    int32_t grid_blocks;         /* tuning: workgroups of a persistent launch; 0 = library choice  */
    int32_t engine;              /* THOI_ENGINE_*: how whole orders of a RANGE selection are       */
                                 /* factored (same results to rounding; other selections ignore it) */
    /* tuning per register class of a RANGE selection (index: the precision's class table, FP32  */
    /* orders {0-8, 9-12, 13-16, 17-20, 21-24}, FP64 {0-6, 7-10, 11-14, 15-18}); 0 = seg_tiles /  */
    /* library choice.  Work split only: results are the same for every value.                   */
    int32_t class_seg_tiles[8];  /* tiles of 256 lanes per workgroup                               */
    int32_t class_lanes[8];      /* n-plets per lane: 1, or 2 where the class has register room   */
} thoi_eval_opts;

/*
 * Engines for the orders of a RANGE selection that the call covers completely:
 *  THOI_ENGINE_FACTOR: one Cholesky factorisation per n-plet (every order).
 *  THOI_ENGINE_PREFIX: prefix sharing (Supplementary, "The combinatorial explosion": the cost is
 *    one factorisation per n-plet of every order).  In lexicographic order the n-plets that share
 *    their first k - 2 variables are consecutive; each prefix is factored once and its factor is
 *    bordered with the remaining two variables, x1 then x2 (the first bordering shared by all
 *    pairs starting with x1): about 2 (k-1)^2 multiply-adds per n-plet instead of 2 (k^3-k)/3 +
 *    k(k+1) flops.  Orders 3..16 in FP32, 3..12 in FP64; others use the factorisation engine.
 *  THOI_ENGINE_AUTO (0): the library's choice: the prefix engine for orders 7..12 of an FP64
 *    streaming reduction with at least 4 tails per lane (C(N, k) D >= 2^20), where it measured
 *    faster; the factorisation engine otherwise.
 */
enum { THOI_ENGINE_AUTO = 0, THOI_ENGINE_FACTOR = 1, THOI_ENGINE_PREFIX = 2 };

/*
 * Gaussian-copula transform (Supplementary, Eq. gaussian_copula_covariance_estimator):
 * for each dataset and variable, z_t = Phi^{-1}(r_t / (T+1)) with r_t the
 * 1-based ordinal rank of x_t among the T samples; equal values are ranked by
 * sample index (-0.0 equals +0.0).
 *   X: device [D][T][N] FP64.  Z: device [D][T][N], z_dtype F64 or F32.
 *   ws: device, >= thoi_workspace_bytes(THOI_WS_COPULIZE, D, T, N, NULL, NULL).
 * A NaN in column (d, n) writes NaN to that column of Z and THOI_EINVAL_DATA to
 * the workspace status word.  Requires 2 <= T <= 2^31 - 1.
 */
thoi_status thoi_copulize(const double* X, int64_t D, int64_t T, int64_t N, int32_t z_dtype,
                          void* Z, void* ws, size_t ws_bytes, void* stream);

/*
 * Covariance operator of the same equation: Sigma_d = (Z_d - mean)^T (Z_d - mean) / (T-1),
 * accumulated in FP64 on the matrix cores.
 *   Z: device [D][T][N] (z_dtype).  Sigma: device [D][N][N] FP64 (overwritten).
 *   ws: device, >= thoi_workspace_bytes(THOI_WS_COV, D, T, N, NULL, NULL).
 * Requires 2 <= T <= 2^31 - 1, N <= 4096, D <= 65535 (else THOI_EUNSUPPORTED).
 */
thoi_status thoi_cov(const void* Z, int32_t z_dtype, int64_t D, int64_t T, int64_t N,
                     double* Sigma, void* ws, size_t ws_bytes, void* stream);

/*
 * Measures of every selected n-plet against every covariance matrix.
 *   Sigma: device [D][N][N] FP64, symmetric.
 *   out: device [P][D][B] of opts->out_dtype with P = 4 (+1 if write_entropy):
 *        planes TC, DTC, Omega, S-information (, H(X^n)).  Ignored (may be
 *        NULL) when opts->reduce is set.
 *   flags: device [D][B] uint8 (THOI_NPLET_* bits) or NULL.
 *   ws: device, >= thoi_workspace_bytes(THOI_WS_EVAL, D, 0, N, sel, opts); its
 *       first 256 bytes are overwritten by the status word and counters.
 * The per-n-plet work is one Cholesky factorisation of the sub-matrix: the
 * joint log-determinant and every leave-one-out log-determinant
 * (log det Sigma_{S\j} = log det Sigma_S + log (Sigma_S^-1)_jj) come from it.
 */
thoi_status thoi_nplets_eval(const double* Sigma, int64_t D, int32_t N, const thoi_nplets* sel,
                             const thoi_eval_opts* opts, void* out, uint8_t* flags,
                             void* ws, size_t ws_bytes, void* stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): thoi_nplets_eval without a workspace argument.  Same
 * arguments (minus ws), checks, kernels and results as thoi_nplets_eval; the workspace is a
 * fixed device array of THOI_NOALLOC_SCRATCH_BYTES owned by the library, one per GPU, held until
 * the process ends.  The call allocates nothing (no hipMalloc, no stream or event creation): all
 * of its kernels go to `stream`, one after the other.
 *   status: device int32 or NULL; receives the call's device status word (THOI_OK, or the
 *           thoi_status a kernel raised: THOI_EINVAL_DATA for bad LIST / MASK rows,
 *           THOI_EWORKSPACE when the FP64 refinement queue overflowed) once the call's kernels
 *           have run.
 * Errors: THOI_EWORKSPACE, before anything is enqueued, when the call needs more workspace than
 * THOI_NOALLOC_SCRATCH_BYTES (thoi_workspace_bytes(THOI_WS_EVAL, D, 0, N, sel, opts) tells);
 * THOI_EHIP when the array's address cannot be obtained on the stream's device; otherwise those
 * of thoi_nplets_eval.
 * Every call on one GPU uses that GPU's array, which keeps what the last call left in it (each
 * call clears what it needs at its start).  Calls that overlap in time on one GPU (two streams,
 * two host threads) race on it and give undefined results: the caller serialises them.
 */
#define THOI_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
thoi_status thoi_nplets_eval_noalloc(const double* Sigma, int64_t D, int32_t N, const thoi_nplets* sel,
                                     const thoi_eval_opts* opts, void* out, uint8_t* flags,
                                     int32_t* status, void* stream);

/*
 * Host, pure: the launches thoi_nplets_eval would enqueue for the evaluation engines of this
 * selection on one dataset (the class launches and the large-order engine; not the small
 * bookkeeping kernels), and the largest number of work-items along x among them.  Every grid is
 * kept below 2^30 work-items along x (the dispatch limit is 2^32) by giving each workgroup more
 * n-plets.  Same argument checks as thoi_nplets_eval except those of Sigma and out (no pointer is
 * dereferenced; LIST and MASK selections still need their non-NULL device pointer).
 */
thoi_status thoi_eval_launch_shape(int32_t N, const thoi_nplets* sel, const thoi_eval_opts* opts,
                                   int32_t* n_launches, int64_t* max_items_x);

/*
 * Adjoint of thoi_nplets_eval: grad_Sigma[d] += sum_b sum_m grad_out[m][d][b] *
 * d measure_m(b, d) / d Sigma_d, with the entries of Sigma treated as
 * independent (the result is symmetric).  FP64 factorisation, inverse and P = R_S^-1; the
 * quadratic part (P diag(1/p) P, from the unit-diagonal rescaling of P) and the accumulation in FP32.
 *   grad_out: device [4][D][B] FP32 (planes TC, DTC, Omega, S).
 *   grad_Sigma: device [D][N][N] FP32, accumulated.
 * The bias correction adds constants and has no gradient.  n-plets whose
 * sub-matrix is not positive definite contribute nothing.  opts->reduce must be NULL.
 */
thoi_status thoi_nplets_eval_backward(const double* Sigma, int64_t D, int32_t N, const thoi_nplets* sel,
                                      const thoi_eval_opts* opts, const float* grad_out,
                                      float* grad_Sigma, void* ws, size_t ws_bytes, void* stream);

/*
 * Many datasets of uneven size in one call (Methods, "Parallel and batched computation of HOI":
 * several datasets; here each with its own number of variables and samples): every n-plet of
 * orders kmin..kmax of every dataset.
 *   Sigma: device, the D matrices back to back; matrix d is [N_d][N_d] FP64 and starts at
 *          element sum_{e<d} N_e^2.
 *   N_d: host [D], 1 <= N_d <= THOI_MAX_N_RANGE.  T_d: host [D] sample counts, needed only with
 *        bias correction (opts->T is ignored), else may be NULL.
 *   Output position of the b-th n-plet of dataset d (in that dataset's RANGE order) is
 *   out_off[d] + b, out_off being the exclusive prefix sum of thoi_count(N_d, kmin, kmax)
 *   (thoi_multi_offsets); out: device [P][total] (P = 4, or 5 with write_entropy); flags:
 *   device [total] or NULL.  With opts->reduce the reducer arrays are [D][kmax+1]... as in
 *   thoi_nplets_eval and g is the index inside dataset d.
 *   kmax must not exceed the register-resident orders (24 in FP32, 18 in FP64).
 * The sizes travel to the device in kernel arguments (512 datasets per small upload launch); one
 * planning kernel derives the per-dataset offsets and work-unit tables in the workspace; then one
 * persistent launch per register class covers every dataset, each workgroup walking a contiguous
 * range of (dataset, order, tile) units.
 */
thoi_status thoi_nplets_eval_multi(const double* Sigma, const int32_t* N_d, const int32_t* T_d, int64_t D,
                                   int32_t kmin, int32_t kmax, const thoi_eval_opts* opts, void* out,
                                   uint8_t* flags, void* ws, size_t ws_bytes, void* stream);
/* Host, pure: out_off[0..D] (exclusive prefix sums of per-dataset n-plet counts, out_off[D] = total). */
thoi_status thoi_multi_offsets(const int32_t* N_d, int64_t D, int32_t kmin, int32_t kmax, int64_t* out_off);
/* Device workspace bytes for thoi_nplets_eval_multi. */
size_t thoi_multi_workspace_bytes(const int32_t* N_d, int64_t D, int32_t kmin, int32_t kmax,
                                  const thoi_eval_opts* opts);

/*
 * Objectives over datasets (Discussion: functions of the measures, such as effect sizes,
 * optimised across datasets; Methods, "Greedy Algorithm": a function over a sequence of
 * datasets).  One FP64 value per n-plet b from its values v[d][b] in D datasets:
 *   THOI_OBJ_MEAN           mean over d = 0..D-1 (summed in ascending d).
 *   THOI_OBJ_PAIRED_EFFECT  D = 2P datasets, dataset p paired with P + p: x_p = v[p][b] - v[P+p][b],
 *                           objective = mean(x) / sd(x) with sd on P - 1 degrees of freedom
 *                           (P >= 2); NaN when sd = 0.
 * A NaN among the inputs gives NaN.
 *   vals: device [D][B], val_dtype THOI_DTYPE_F64 or F32 (e.g. one plane of thoi_nplets_eval's out,
 *         which is [P][D][B]: pass out + m*D*B for measure m).
 *   obj:  device [B] FP64, or NULL.
 *   red:  NULL, or a reducer with kmax = 0 (one list: top_val/top_g [1][1][2][topk], hist
 *         [1][1][hist_bins+2], hist_lo_hi host [1][2]); it receives (objective, b) with ties
 *         ordered by the lower b, NaN objectives not counted, and is merged into across calls
 *         (initialise it with thoi_reduce_init(red, 1, 0, stream)).
 *   ws:   device, >= thoi_objective_workspace_bytes(D, B, red).
 * Needs obj or red.  D <= 65535 (PAIRED_EFFECT: even D >= 4), B <= 2^40.
 */
enum { THOI_OBJ_MEAN = 0, THOI_OBJ_PAIRED_EFFECT = 1 };
thoi_status thoi_objective(const void* vals, int32_t val_dtype, int64_t D, int64_t B, int32_t kind, double* obj,
                           const thoi_reduce* red, void* ws, size_t ws_bytes, void* stream);
size_t thoi_objective_workspace_bytes(int64_t D, int64_t B, const thoi_reduce* red);

/*
 * Batched simulated annealing over n-plets, run on the device (Methods, "Heuristics", "Simulated
 * Annealing Algorithm").  kappa chains, each an n-plet as a bit mask of the N <= 128 variables
 * (two 64-bit words per chain: variable i is bit i % 64 of word i / 64), start from masks0.  Iteration t (t = 0 .. iters-1), per chain c:
 *   neighbour: within an order (across = 0) the floor(a k)-th member (ascending) is swapped for the
 *     floor(b (N - k))-th outsider; across orders (across = 1) the n-plet instead gains that
 *     outsider when move < 1/3 and k < k_max, or loses that member when 1/3 <= move < 2/3 and
 *     k > k_min, and is swapped otherwise (k = order of the current n-plet; a, b, move are
 *     draw_a, draw_b, draw_move [t][c]);
 *   energy E = Omega (maximize != 0) or -Omega; dE = E(neighbour) - E(current); the neighbour is
 *     taken when dE > 0 or draw_accept[t][c] < exp(dE / temp_t), and never when it is not positive
 *     definite (its Omega is NaN); temp_0 = T0 and temp_{t+1} = temp_t * alpha;
 *   the best state seen so far is kept (a later state replaces it only with a strictly larger E).
 * Omega is evaluated in FP64 from the correlation of Sigma (N x N, device, row-major).
 *   masks0: device [kappa][2] uint64; orders in [k_min, k_max]; bits at N and above are ignored.
 *   draw_*: device [iters][kappa] FP64 in [0, 1); draw_move is needed only when across = 1.
 *   cur_mask, best_mask: device [kappa][2] uint64; cur_omega, best_omega: device [kappa] FP64;
 *     accepted: device [kappa] int64 (the final state, the best state and the number of accepted
 *     moves per chain).
 * 1 <= k_min <= k_max <= min(N - 1, 64); T0 > 0, alpha > 0.  Every iteration is one kernel launch on
 * `stream`; nothing is allocated and the host does not wait.
 */
thoi_status thoi_anneal(const double* Sigma, int32_t N, const uint64_t* masks0, int32_t kappa, int32_t iters,
                        const double* draw_move, const double* draw_a, const double* draw_b, const double* draw_accept,
                        double T0, double alpha, int32_t maximize, int32_t across, int32_t k_min, int32_t k_max,
                        uint64_t* cur_mask, double* cur_omega, uint64_t* best_mask, double* best_omega,
                        int64_t* accepted, void* stream);

/*
 * Greedy growth run on the device (Methods, "Heuristics", "Greedy Algorithm").  Slot 0 holds the
 * starting solutions: count[0] <= kappa distinct n-plets of order k_first, as masks of the
 * N <= 128 variables (two 64-bit words each: variable i is bit i % 64 of word i / 64).  Step
 * s = 0 .. steps-1 extends every solution of slot s by every variable it lacks, evaluates each
 * distinct candidate of order k_first + s + 1 in the D datasets (FP64) and writes the kappa best to
 * slot s + 1, best first: the largest objective (maximize != 0) or the smallest, equal values
 * ordered by the n-plet in lexicographic order (the smaller first).  The objective is the
 * measure (0 TC, 1 DTC, 2 Omega, 3 S) combined over the datasets as thoi_objective does (`kind`:
 * THOI_OBJ_MEAN, or THOI_OBJ_PAIRED_EFFECT with even D >= 4); a candidate whose objective is NaN
 * (not positive definite in some dataset, or a zero spread) is dropped.  With D = 1 and
 * THOI_OBJ_MEAN the objective is the measure itself.
 *   Sigma: device [D][N][N] FP64.
 *   sols:  device [steps+1][kappa][2] uint64; vals: device [steps+1][kappa] FP64;
 *   count: device [steps+1] int32 (solutions in each slot); slot 0 (sols, vals, count) is input.
 *   ws:    device, >= thoi_greedy_workspace_bytes(D, N, kappa).
 * k_first + steps <= min(N, 64), kappa <= 256, kappa * N <= 4096, D <= 65535.  Two kernel
 * launches per step on `stream`; nothing is allocated and the host does not wait.
 */
thoi_status thoi_greedy(const double* Sigma, int64_t D, int32_t N, int32_t k_first, int32_t steps, int32_t kappa,
                        int32_t measure, int32_t kind, int32_t maximize, uint64_t* sols, double* vals, int32_t* count,
                        void* ws, size_t ws_bytes, void* stream);
size_t thoi_greedy_workspace_bytes(int64_t D, int32_t N, int32_t kappa);

/* Initialise reducer arrays for D datasets (top_g = -1, hist = 0). */
thoi_status thoi_reduce_init(const thoi_reduce* red, int64_t D, int32_t kmax, void* stream);

/* Device workspace bytes needed by the call `which` (THOI_WS_*); 0 if none. */
size_t thoi_workspace_bytes(int32_t which, int64_t D, int64_t T, int32_t N,
                            const thoi_nplets* sel, const thoi_eval_opts* opts);
/* Offset in bytes of the int32 device status word inside a workspace. */
size_t thoi_ws_status_offset(void);

/* Host, pure: number of n-plets of orders kmin..kmax of N variables; -1 if it exceeds int64. */
int64_t thoi_count(int32_t N, int32_t kmin, int32_t kmax);
/* Host, pure: the n-plet at global index g of the RANGE enumeration (orders kmin..);
 * writes its order to *out_k and its indices to out_idx[0..k-1]. */
thoi_status thoi_unrank_host(int32_t N, int32_t kmin, int64_t g, int32_t* out_k, int32_t* out_idx);
/* Host, pure: bias-correction offsets added to TC and DTC at order k for T samples. */
thoi_status thoi_bias_offsets(int32_t k, int32_t T, double* d_tc, double* d_dtc, double* eta_k);

const char* thoi_status_string(thoi_status s);
const char* thoi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* THOI_H_ */
