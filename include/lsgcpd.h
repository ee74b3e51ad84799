/*
 * lsgcpd.h -- C ABI of the MI355X (gfx950) LSG-CPD library.
 *
 * LSG-CPD (Liu, Wu, Chirikjian, ICCV 2021) registers a source cloud X (N x 3)
 * to a target cloud Y (M x 3) by EM on a Gaussian mixture built on the target:
 * one component per target point with inverse covariance
 * sigma^-2 (alpha_m n_m n_m^T + I) (Sec. 3.1, Eq. 2), alpha_m set from the local
 * surface variation (Eq. 3), plus a uniform outlier component (Eq. 1).
 *
 * Conventions shared by every call:
 *  - Arrays named X, Y, P (points), normals, kappa, alpha, pi, w, phi, phi_x,
 *    phi_y and colstats are DEVICE pointers owned by the caller (hipMalloc'd or
 *    torch CUDA tensors), row-major and contiguous (lsgcpd_register_batch takes
 *    host arrays of such pointers).  Point clouds are float32 [n][3].  Structs (poses,
 *    parameters, results, reports) are HOST memory owned by the caller.
 *  - The library owns only the workspace inside an lsgcpd_ctx; it grows on
 *    demand, is reused across calls and is released by lsgcpd_ctx_destroy.
 *    No caller pointer is retained after a call returns.
 *  - Every call returns an lsgcpd_status; nothing throws across the ABI.  On
 *    a non-OK status the outputs are unspecified and lsgcpd_last_error(ctx)
 *    holds a message.  Invalid arguments are rejected before any GPU work.
 *  - `stream` is a hipStream_t (NULL = the default stream).  lsgcpd_normals and
 *    lsgcpd_depth_confidence are asynchronous on it; the calls with host outputs
 *    (lsgcpd_estep, lsgcpd_register*, lsgcpd_autotune) synchronise it before
 *    filling them.
 *  - A context is not thread-safe: use one context per host thread.
 *  - The pose g = (R, t) maps the source into the target frame,
 *    g(x) = R x + t, with R row-major.
 */
#ifndef LSGCPD_H
#define LSGCPD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LSGCPD_ABI_VERSION 6

typedef struct lsgcpd_ctx lsgcpd_ctx;
typedef void *lsgcpd_stream;  /* a hipStream_t */

typedef enum {
  LSGCPD_OK = 0,
  LSGCPD_E_INVALID = 1,     /* bad argument (NULL pointer, size, range)      */
  LSGCPD_E_HIP = 2,         /* a HIP runtime call failed (no device, launch) */
  LSGCPD_E_NOMEM = 3,       /* workspace allocation failed                   */
  LSGCPD_E_NUMERIC = 4,     /* non-finite variance or pose                   */
  LSGCPD_E_UNSUPPORTED = 5  /* size or option the library does not handle    */
} lsgcpd_status;

/* Flags for lsgcpd_estep / lsgcpd_params.flags */
#define LSGCPD_EXACT_NORMALIZER 1u  /* multiply each component by sqrt(1+alpha_m),
                                       the determinant factor of Eq. 2 that the
                                       printed E step (Eq. 9-10) leaves out */
#define LSGCPD_PAIRS_LDS 2u         /* pair kernel stages target records in LDS
                                       instead of reading them through the
                                       scalar cache (comparison only)           */
#define LSGCPD_PAIRS_MFMA 4u        /* pair kernel accumulates on the FP64
                                       matrix cores (comparison only)           */
#define LSGCPD_DENSE 8u             /* evaluate every pair.  By default the
                                       pair kernel drops (source group, target
                                       tile) blocks whose bounding boxes prove
                                       that every exponential is an exact zero
                                       in float32, and lsgcpd_register first
                                       puts both clouds in spatial order; the
                                       dropped terms are exact zeros, so the
                                       results differ only in the rounding order
                                       of the sums */
#define LSGCPD_GRAPH 16u            /* lsgcpd_register* only: record the EM
                                       iterations once as a HIP graph and
                                       replay it; the recording is kept in the
                                       context and replayed by later calls of
                                       the same sizes and parameters (ignored
                                       while kernel timing is on) */
#define LSGCPD_BF16_CROSS 32u       /* E steps at large sigma^2 evaluate the
                                       exponent on the matrix cores: c d_mn as
                                       the product of lifted quadratic features
                                       (Eq. 10's bilinear structure), each split
                                       into BF16 high and low parts, FP32 sums,
                                       and the accumulation as a second BF16
                                       product.  An E step takes this path only
                                       while its exponent error bound,
                                       |dz| <= 4.96e-5 (1 + alpha_m)(|u| + |v|)^2
                                       with u, v the source and target in units
                                       of sqrt(2 sigma^2 / log2 e) about the box
                                       centre of 64 neighbouring sources, stays
                                       below 1/32 for every pair within distance
                                       2 of the sources' box (the early, large-
                                       sigma^2 iterations; typical errors are
                                       1e-4); the others run the FP64 kernel.
                                       Not with LSGCPD_DENSE, _PAIRS_LDS or
                                       _PAIRS_MFMA (LSGCPD_E_INVALID) */

typedef struct {
  double R[9]; /* row-major rotation */
  double t[3];
} lsgcpd_pose;

/* ---- context ---------------------------------------------------------- */

/* Creates a context on HIP device `device` (it becomes current on this host
 * thread).  Returns LSGCPD_E_HIP if the device cannot be opened. */
lsgcpd_status lsgcpd_ctx_create(int device, lsgcpd_ctx **out);
/* Frees the workspace and the context.  NULL is a no-op. */
void lsgcpd_ctx_destroy(lsgcpd_ctx *ctx);
/* Message for the last failed call on ctx ("" if none).  Owned by ctx. */
const char *lsgcpd_last_error(const lsgcpd_ctx *ctx);
/* Static name of a status code. */
const char *lsgcpd_status_string(lsgcpd_status s);
int lsgcpd_abi_version(void);

/* ---- target geometry (Sec. 3.1, Eq. 3) --------------------------------- */

/* Surface normal n_m, surface variation kappa_m and penalty alpha_m of every
 * target point.  The neighbourhood of y_m is its k nearest points of Y by
 * Euclidean distance (itself included, ties to the lower index, distances
 * compared in float32); its covariance about the neighbourhood mean (weight
 * 1/k) is eigen-decomposed in FP64: n_m = unit eigenvector of the smallest
 * eigenvalue (sign arbitrary), kappa_m = smallest eigenvalue / trace (in
 * [0, 1/3]; 1/3 and n = e_z for a zero trace), and
 * alpha_m = alpha_max (1 - e^{lambda(3 - 1/kappa)}) / (1 + e^{lambda(3 - 1/kappa)})
 * (alpha_max at kappa = 0, never negative).
 * Y: M x 3 float32.  Outputs: normals M x 3, kappa M (may be NULL), alpha M,
 * all float32.  Requires 1 <= k <= min(M, 32), alpha_max >= 0, lambda > 0.
 * Asynchronous on `stream`. */
lsgcpd_status lsgcpd_normals(lsgcpd_ctx *ctx, const float *Y, int64_t M, int32_t k,
                             double alpha_max, double lambda, float *normals,
                             float *kappa, float *alpha, lsgcpd_stream stream);

/* ---- one E step (Sec. 3.1 Eq. 5, Sec. 3.4 Eq. 9) ------------------------ */

/* Sufficient statistics of the posterior.  With x~_n = (x_n, 1),
 * M_m = I + alpha_m n_m n_m^T, and per source n
 *   p_n = sum_m P_mn,  W_n = sum_m P_mn alpha_m n_m n_m^T,
 *   B_n = sum_m P_mn M_m y_m,  C_n = sum_m P_mn y_m^T M_m y_m,
 * the array `stats` holds, in this order (FP64):
 *   [0..9]    S0 = sum_n p_n x~ x~^T         upper triangle of the 4x4, rows
 *                                             (00 01 02 03 11 12 13 22 23 33)
 *   [10..69]  S1[ab] = sum_n W_n[a][b] x~ x~^T for ab = 00 01 02 11 12 22,
 *                                             10 values each, same order
 *   [70..81]  S2 = sum_n B_n x~^T            3x4 row-major
 *   [82]      S3 = sum_n C_n
 *   [83]      sum_n log(sum_m K_mn + gamma)
 *   [84]      sum_n gamma / (sum_m K_mn + gamma)     (expected outliers)
 *   [85]      sum_n log w_n
 * For G = [R | t] (3x4) the M-step objective is the quadratic
 *   sum_mn P_mn d_mn(G) = sum_ab G_a^T (delta_ab S0 + S1[ab]) G_b
 *                          - 2 <S2, G> + S3,
 * d_mn(G) = (G x~_n - y_m)^T M_m (G x~_n - y_m). */
#define LSGCPD_NSTATS 86

typedef struct {
  double sigma2, gamma, V;   /* values used; gamma = (2 pi sigma2)^{3/2} / V   */
  double sumP;               /* N_P = sum_mn P_mn                              */
  double outlier_mass;       /* sum_n gamma / (sum_m K_mn + gamma)            */
  double nll;                /* Eq. 4 at the given pose                        */
  double pd;                 /* sum_mn P_mn d_mn at the given pose             */
  double stats[LSGCPD_NSTATS];
  double grad[6];            /* Eq. 11 at the given pose (right derivatives of
                                sum P d / sigma2, basis: rotations about x, y,
                                z, then translations along x, y, z)            */
  double hess[36];           /* (H + H^T)/2 of Eq. 12, row-major               */
  lsgcpd_pose pose_next;     /* M step (Sec. 3.5) from the given pose          */
  double sigma2_next;        /* sigma^2 after that M step                      */
  int32_t newton_iters;
  int32_t gn_fallbacks;
  int32_t bf16_cross;        /* 1 if the LSGCPD_BF16_CROSS path ran this E step */
  int32_t pad;
} lsgcpd_estep_out;

/* One E step at pose g and variance sigma2, plus the M step it implies.
 *   X: N x 3, Y: M x 3, normals: M x 3 (unit), alpha: M (>= 0), float32.
 *   pi: M priors (NULL => 1/M), w: N outlier weights in (0,1) (NULL => w0).
 *   V > 0 working volume (<= 0 => target box volume, edges floored at 1e-3 of
 *   its diagonal).  flags: LSGCPD_EXACT_NORMALIZER, LSGCPD_PAIRS_LDS or LSGCPD_PAIRS_MFMA.
 *   Posterior P_mn = K_mn / (sum_m K_mn + gamma), K_mn = (1-w_n)/w_n pi_m
 *   exp(-d_mn / (2 sigma2)) with d_mn = |g(x_n) - y_m|^2 + alpha_m (n_m .
 *   (g(x_n) - y_m))^2 (Eq. 9-10).  The M x N matrix is never formed unless
 *   `P` is non-NULL (testing aid: float32 M x N, row m = component).
 *   colstats: NULL or N x 16 FP64 per-source values
 *   [sum_m K_mn/rho_n, sum_m K_mn, p_n, W_n (00 01 02 11 12 22), B_n (3), C_n,
 *    log(sum_m K_mn + gamma), gamma/(sum_m K_mn + gamma), 0]
 *   with rho_n = (1 - w_n)/w_n.
 * Requires M, N >= 1, 0 < w0 < 1 when w is NULL, finite sigma2 > 0, R a
 * rotation (|R^T R - I| <= 1e-6).  Synchronises `stream`. */
lsgcpd_status lsgcpd_estep(lsgcpd_ctx *ctx, const float *X, int64_t N, const float *Y,
                           const float *normals, const float *alpha, int64_t M,
                           const float *pi, const float *w, double w0, double V,
                           const lsgcpd_pose *g, double sigma2, uint32_t flags,
                           lsgcpd_estep_out *out, float *P, double *colstats,
                           lsgcpd_stream stream);

/* The E step of lsgcpd_estep (same arguments, meaning, layouts, outputs and
 * errors) without allocating memory, for callers that cannot allocate: code
 * that runs while a stream is being captured into a HIP graph, serving loops
 * that must not call hipMalloc, harnesses that forbid it.  It calls no
 * hipMalloc, hipFree or hipHostMalloc: its device workspace is a static
 * array of 36 MiB that each GPU holds from the first lsgcpd_ctx_create on it
 * until the process ends, and its plan tables and state are copied from
 * host stack/heap memory.  Limits: M, N <= 65,536 (LSGCPD_E_UNSUPPORTED
 * beyond, and for LSGCPD_PAIRS_LDS / LSGCPD_PAIRS_MFMA); the work is split
 * into about 1,024 work items whatever lsgcpd_autotune chose, so results
 * equal lsgcpd_estep's up to the grouping of the FP64 sums.  Every call on a
 * GPU uses that GPU's one array: calls that overlap on one GPU (other host
 * threads, other streams) race and give wrong results; successive calls on
 * one stream are safe.  Synchronises `stream`. */
lsgcpd_status lsgcpd_estep_noalloc(lsgcpd_ctx *ctx, const float *X, int64_t N, const float *Y,
                                   const float *normals, const float *alpha, int64_t M,
                                   const float *pi, const float *w, double w0, double V,
                                   const lsgcpd_pose *g, double sigma2, uint32_t flags,
                                   lsgcpd_estep_out *out, float *P, double *colstats,
                                   lsgcpd_stream stream);

/* ---- full registration (Sec. 3) ----------------------------------------- */

typedef struct {
  int32_t k;             /* neighbourhood size for the normals (<= 32)       */
  double alpha_max;      /* Eq. 3 upper bound                                 */
  double lambda;         /* Eq. 3 sensitivity                                 */
  double w0;             /* uniform outlier weight, 0 < w0 < 1                */
  double V;              /* working volume; <= 0 => target box volume         */
  int32_t max_iter;      /* EM iterations                                      */
  double tol;            /* > 0: stop once |L_i - L_{i-1}| <= tol |L_i|       */
  double sigma2_init;    /* <= 0 => sum_mn |g0(x_n) - y_m|^2 / (3 M N)        */
  int32_t newton_max;    /* Newton steps per M step (>= 1)                     */
  uint32_t flags;        /* as for lsgcpd_estep                                 */
  double eta;            /* outlier ratio (Sec. 3.2).  0 < eta < 1: w0 is set
                            to w_max = eta V S / ((1 - eta) + eta V S),
                            S = sum_m pi(m) c_m, with c_m the peak of the
                            component density (Eq. 2) as the E step evaluates
                            it -- (2 pi sigma2)^{-3/2}, times sqrt(1 + alpha_m)
                            with LSGCPD_EXACT_NORMALIZER -- taken once, at the
                            initial sigma2, and kept; the w0 field is then
                            ignored.  <= 0: w0 as given                      */
} lsgcpd_params;

typedef struct {
  int32_t iters;         /* M steps taken                                      */
  int32_t converged;     /* 1 if the tol criterion stopped EM                  */
  int32_t gn_fallbacks;  /* M-step Newton steps that used the Gauss-Newton term */
  double sigma2;         /* final sigma^2                                      */
  double nll_first, nll_last;
  double V;
  double w0;             /* uniform outlier weight used (w_max when eta > 0)  */
  int64_t n_used;        /* source / target points registered (after the     */
  int64_t m_used;        /* truncation of lsgcpd_register_cf)                */
  int32_t bf16_steps;    /* E steps that took the LSGCPD_BF16_CROSS path      */
  int32_t pad;
} lsgcpd_report;

/* Fills p with the defaults used by the examples: k=10, alpha_max=30,
 * lambda=0.2, w0=0.1, V=0, max_iter=50, tol=0, sigma2_init=0, newton_max=20,
 * flags=0, eta=0. */
void lsgcpd_params_default(lsgcpd_params *p);

/* Registers X (N x 3) to Y (M x 3): normals from Y (lsgcpd_normals), then EM
 * from `init` (NULL => identity).  `out` receives the final pose.  nll_trace:
 * NULL or a host array of max_iter doubles receiving Eq. 4 at each E step
 * (entries after the last E step are left untouched).  Synchronises
 * `stream`. */
lsgcpd_status lsgcpd_register(lsgcpd_ctx *ctx, const float *X, int64_t N, const float *Y,
                              int64_t M, const lsgcpd_params *p, const lsgcpd_pose *init,
                              lsgcpd_pose *out, lsgcpd_report *report, double *nll_trace,
                              lsgcpd_stream stream);

/* Registers npairs independent pairs (X[i], N[i]) to (Y[i], M[i]) with the
 * same parameters, as lsgcpd_register does each of them, but in one pipeline:
 * every EM iteration runs the E steps and M steps of all pairs in the same
 * kernel launches, with the work items of the pair kernel shared out in
 * proportion to M[i] N[i].  X, N, Y, M, init (NULL => identity for every
 * pair), out and reports (may be NULL) are HOST arrays of npairs entries;
 * X[i] and Y[i] are device pointers.  Each pair stops on its own tol test.
 * Results equal lsgcpd_register's up to the grouping of the sums (the work
 * items differ).  Requires 1 <= npairs <= 65536, sum of N[i] + M[i] at most
 * 2^27, k <= M[i], and the default pair kernel (LSGCPD_PAIRS_LDS / _MFMA give
 * LSGCPD_E_UNSUPPORTED for npairs > 1).  The set-up of the clouds (sorting,
 * neighbours, records) of pair i runs on `stream` when i % 4 == 0 and else
 * on one of three streams of the context, which start after the work queued
 * on `stream` and which `stream` waits for (events) before the EM loop.
 * Synchronises `stream`. */
lsgcpd_status lsgcpd_register_batch(lsgcpd_ctx *ctx, int32_t npairs, const float *const *X,
                                    const int64_t *N, const float *const *Y, const int64_t *M,
                                    const lsgcpd_params *p, const lsgcpd_pose *init,
                                    lsgcpd_pose *out, lsgcpd_report *reports,
                                    lsgcpd_stream stream);

/* ---- tuning --------------------------------------------------------------- */

/* Picks the work-item count of the default pair kernel by measurement: runs
 * the registration lsgcpd_register(X, Y, p) would run (outputs discarded)
 * with each of 1024, 2048, 4096, 8192, 16384 and 32768 work items per E step
 * (twice each; the second run is timed with HIP events on `stream`) and keeps
 * the fastest for the size class of the pair (floor(log2(M N))) in ctx:
 * later lsgcpd_estep / lsgcpd_register / lsgcpd_register_cf calls and batches
 * whose sum of M N falls in that class use it (default: 1024 up to 1.6e8
 * pairs, 4096 up to 1.6e9, 8192 above; or the LSGCPD_WORK_ITEMS environment
 * variable).  The count changes how the pair
 * sums are grouped, so results differ at the rounding level only.  *items_out
 * (may be NULL) receives the choice.  Argument rules as lsgcpd_register.
 * Synchronises `stream`. */
lsgcpd_status lsgcpd_autotune(lsgcpd_ctx *ctx, const float *X, int64_t N, const float *Y,
                              int64_t M, const lsgcpd_params *p, int32_t *items_out,
                              lsgcpd_stream stream);

/* ---- confidence filtering (Sec. 3.3) ------------------------------------ */

/* Measurement confidence of points seen by a depth sensor (Sec. 3.3):
 * phi = e_min / e(z) with the error model e(z) = coef[0] + coef[1] z +
 * coef[2] z^2 of the depth z = P[i][2] (points in the sensor frame), and
 * phi = 1 where e(z) <= e_min (e_min: the smallest error over the sensor's
 * range).  Evaluated in FP64, written as float32.  P: n x 3 float32 device
 * array; phi: n float32 device array; coef: HOST array of 3 finite doubles;
 * e_min > 0.  Asynchronous on `stream`. */
lsgcpd_status lsgcpd_depth_confidence(lsgcpd_ctx *ctx, const float *P, int64_t n,
                                      const double *coef, double e_min, float *phi,
                                      lsgcpd_stream stream);

/* lsgcpd_register with confidence filtering (Sec. 3.3).  phi_x (N) and
 * phi_y (M) are float32 device arrays of confidences in (0, 1] (NULL => 1
 * for that cloud; values are not checked).  If threshold > 0, the points of a
 * cloud whose confidence is below it are dropped first (order kept; the
 * normals, V and the initial sigma2 then come from the points kept, and
 * report->n_used / m_used give their numbers).  Then EM runs with priors
 * pi(m) = phi(y_m) / sum phi(y) and outlier weights
 * w_n = 1 - (1 - w0) phi(x_n), w0 from p (or w_max with p->eta > 0).
 * LSGCPD_E_INVALID if no point of a cloud, or fewer than k targets, remain.
 * Synchronises `stream` (once more after the truncation). */
lsgcpd_status lsgcpd_register_cf(lsgcpd_ctx *ctx, const float *X, const float *phi_x, int64_t N,
                                 const float *Y, const float *phi_y, int64_t M, double threshold,
                                 const lsgcpd_params *p, const lsgcpd_pose *init,
                                 lsgcpd_pose *out, lsgcpd_report *report, double *nll_trace,
                                 lsgcpd_stream stream);

/* ---- kernel timing (benchmarks) ----------------------------------------- */

/* Event-based timing of the E step inside lsgcpd_estep / lsgcpd_register.
 * While enabled, every E step records HIP events on the call's stream around
 * (a) the pair kernel alone (exponents + feature accumulation) and (b) the
 * whole E step (work-item plan, pair kernel, per-source finalisation and the
 * block statistics; the M step is not included).  Elapsed times are summed
 * when the call synchronises.  Off by default. */
typedef struct {
  int64_t launches;        /* E steps timed                                 */
  int64_t pairs;           /* sum of M * N over those E steps               */
  double pair_kernel_ms;   /* total time of (a)                             */
  double estep_ms;         /* total time of (b)                             */
  int64_t evaluated_pairs; /* pairs (a) evaluated after dropping the blocks
                              of exact zeros (<= pairs)                     */
} lsgcpd_profile;

lsgcpd_status lsgcpd_profile_enable(lsgcpd_ctx *ctx, int on);
/* Copies the totals into *out (may be NULL) and, if reset != 0, zeroes them
 * and forgets the per-launch times below. */
lsgcpd_status lsgcpd_profile_read(lsgcpd_ctx *ctx, lsgcpd_profile *out, int reset);
/* The times (a) and (b), in microseconds, of every timed E step since the
 * last reset, in launch order: the first min(cap, *count) go to the HOST
 * arrays pair_us and estep_us; *count (may be NULL) receives how many there
 * are. */
lsgcpd_status lsgcpd_profile_launches(lsgcpd_ctx *ctx, double *pair_us, double *estep_us,
                                      int64_t cap, int64_t *count);

/* ---- learned initial-pose proposal ------------------------------------- */
/* LSG-CPD converges from starts inside its basin (Sec. 1 and 5 of the paper
 * on initialisation); these calls run a small point-set encoder that
 * predicts the rigid motion of a cloud pair, to start registrations from.
 * Inputs: P points of each cloud (indices floor((2k + 1) N / (2P)), k =
 * 0..P-1), each cloud centred on the mean of its samples and expressed in
 * its principal-axis frame F = [e0 e1 e2] (eigenvectors of the samples'
 * covariance, decreasing eigenvalues; e0, e1 signed so that the samples'
 * third moment along them is >= 0, or their largest component positive if
 * it is 0; e2 = e0 x e1; F = I for a zero covariance), both divided by the
 * RMS radius s of the target's samples (1 if that is 0).  The inputs do not
 * change when a cloud is rotated; the encoder predicts the rotation R_c and
 * translation t^ between the two frames.
 * Model: each cloud's inputs pass a shared per-point MLP 3 -> 64 -> 128 ->
 * 256 (ReLU after each layer) and a max-pool (ties to the lower point); the
 * source's and the target's 256-vectors side by side pass 512 -> 128 (ReLU)
 * -> 9; outputs 0..5 are two 3-vectors made a rotation by Gram-Schmidt
 * (columns: the first normalised, the second's part orthogonal to it
 * normalised, their cross product), outputs 6..8 the translation t^.  The
 * pose is R = F_Y R_c F_X^T, t = mu_Y + s F_Y t^ - R mu_X.  theta:
 * LSGCPD_PROPOSAL_PARAMS float32 in device memory, layer by layer, each W
 * row-major [out][in] then its b:
 *   W1 64x3, b1 64, W2 128x64, b2 128, W3 256x128, b3 256,
 *   W4 128x512, b4 128, W5 9x128, b5 9.
 * P <= 4096 points per cloud. */
#define LSGCPD_PROPOSAL_PARAMS 108425
#define LSGCPD_PROPOSAL_NORM 25  /* doubles of normalisation per pair */

/* Encoder inputs of npairs pairs.  X[i] (N[i] x 3) and Y[i] (M[i] x 3):
 * float32 device clouds (the arrays of pointers and sizes are host memory);
 * the sources are first rotated by Q[9i..] (host, row-major; may be NULL).
 * Outputs (device): Xn, Yn (npairs x P x 3 float32) and norm[25i..] =
 * (mu_X, mu_Y, s, F_X, F_Y) FP64, frames row-major.  Synchronises `stream`. */
lsgcpd_status lsgcpd_proposal_inputs(lsgcpd_ctx *ctx, int32_t npairs, const float *const *X,
                                     const int64_t *N, const float *const *Y, const int64_t *M,
                                     const double *Q, int32_t P, float *Xn, float *Yn,
                                     double *norm, lsgcpd_stream stream);

/* Predicted poses of npairs pairs of inputs (device): pose[12i..] = (R
 * row-major, t) in world units, g(x) = R x + t mapping the source onto the
 * target.  Asynchronous on `stream`. */
lsgcpd_status lsgcpd_proposal_forward(lsgcpd_ctx *ctx, const float *theta, int32_t npairs,
                                      int32_t P, const float *Xn, const float *Yn,
                                      const double *norm, double *pose, lsgcpd_stream stream);

/* One training step: the mean over the batch of |a1 - R_l e_x|^2 +
 * |a2 - R_l e_y|^2 + |t^ - t_l|^2 (a1, a2: the two output 3-vectors), with
 * the label in the pair's frames (R_l = F_Y^T R F_X, t_l = F_Y^T (R mu_X +
 * t - mu_Y) / s), its gradient and one Adam update
 * (beta1 0.9, beta2 0.999, eps 1e-8, bias correction at step `step` >= 1,
 * learning rate lr) of theta with moments m and v (device float32,
 * LSGCPD_PROPOSAL_PARAMS each, zero at step 1).  Xn, Yn, norm (device) hold
 * nstored pairs of inputs; pair b of the batch is stored pair index[b] (host
 * int32, each in [0, nstored), else LSGCPD_E_INVALID; NULL: b);
 * label[12b..] (host) its pose (R row-major, t; world units, source onto
 * target).  Outputs (device): loss[b] per pair (FP64); argmax (NULL or
 * npairs x 2 x 256 int32: the pooled point of each channel, source first)
 * and grad (NULL or LSGCPD_PROPOSAL_PARAMS float32: the gradient applied)
 * are test aids.  Synchronises `stream`. */
lsgcpd_status lsgcpd_proposal_train_step(lsgcpd_ctx *ctx, float *theta, float *m, float *v,
                                         int32_t step, double lr, int32_t npairs, int32_t P,
                                         const float *Xn, const float *Yn, const double *norm,
                                         int32_t nstored, const int32_t *index,
                                         const double *label, double *loss, int32_t *argmax,
                                         float *grad, lsgcpd_stream stream);

/* Registration of npairs pairs started from the proposal, with multi-start
 * EM as its fallback and judge:
 *   1. the encoder's pose of every pair (theta, P points per cloud);
 *   2. LSG-CPD (params) from each, all pairs in one batch;
 *   3. a pair is accepted if its final sigma (sqrt of sigma2) is at most
 *      accept times the RMS radius s of its target's samples;
 *   4. every other pair is registered again from R = F_Y G F_X^T (the
 *      pair's principal-axis frames) with t aligning the sampled centroids,
 *      G first the 4 sign changes of the axes, then, for pairs still not
 *      accepted, the other 20 rotations of the cube; the run with the
 *      lowest final NLL (Eq. 4), the proposal's included, is kept.
 * Clouds as for lsgcpd_register_batch (host arrays of device pointers and
 * sizes).  Outputs (host): out[i], reports[i] (NULL ok) of the run kept,
 * fallback[i] (NULL ok): 1 if step 4 ran for pair i.  Synchronises
 * `stream`. */
lsgcpd_status lsgcpd_register_proposed(lsgcpd_ctx *ctx, int32_t npairs, const float *const *X,
                                       const int64_t *N, const float *const *Y,
                                       const int64_t *M, const lsgcpd_params *p,
                                       const float *theta, int32_t P, double accept,
                                       lsgcpd_pose *out, lsgcpd_report *reports,
                                       int32_t *fallback, lsgcpd_stream stream);

#ifdef __cplusplus
}
#endif
#endif /* LSGCPD_H */
