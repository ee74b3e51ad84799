// Internal declarations shared by the HIP sources of liblsgcpd (device state,
// record layouts, kernel launchers).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lsg {

// Per-target record read by the E-step kernels (FP64, 144 bytes):
//   y     target point
//   a     sqrt(alpha_m) n_m
//   l     log2(pi_m [* sqrt(1 + alpha_m)])
//   f     accumulation features 1..10 (feature 0 is the constant 1):
//         alpha n n^T (00 01 02 11 12 22), M_m y_m, y_m^T M_m y_m
struct TRec {
  double y[3];
  double a[3];
  double l;
  double f[10];
  double pad;
};
constexpr int kRecDoubles = 18;

// Bounding box of a tile of kCullTile consecutive target records and their
// largest log-prior (for exact culling in the pair kernel).
struct TBox {
  double lo[3];
  double hi[3];
  double lmax;
  double pad;
};
constexpr int kCullTile = 64;

// Position and log-prior of a target record, packed for the culling tests.
struct TPt {
  double y[3];
  double l;
};
constexpr int kFeatUsed = 11;   // feature 0 (= 1) and f[0..9]
constexpr int kStats = 86;
constexpr int kColStats = 16;

// Device-resident EM state.  Written by the set-up kernels and the M-step
// kernel, read by every E-step kernel, so that an EM iteration needs no host
// round trip.
struct DevState {
  double R[9];
  double t[3];
  double sigma2;
  double V;
  double sigma2_floor;
  double w0;          // used when no per-source weights are given
  double tol;
  double nll_prev;
  double stats[kStats];
  // outputs of the last M step / derivatives at the E-step pose
  double grad[6];
  double hess[36];
  double R_next[9];
  double t_next[3];
  double sigma2_next;
  double pd;          // sum P d at the E-step pose
  double nll;         // Eq. 4 at the E-step pose
  double gamma;
  int64_t evaluated_pairs;  // pairs the pair kernel evaluated (scalar back end)
  int32_t iter;       // M steps taken
  int32_t done;       // 1 once tol stopped EM (later kernels return at once)
  int32_t converged;
  int32_t gn_fallbacks;
  int32_t newton_iters;
  int32_t numeric_error;
  int32_t newton_max;
  int32_t max_iter;
};

// ---------------------------------------------------------------- launchers
// All launchers enqueue on `st` and return the hipError_t of the launch.

// Normals: k nearest neighbours over the Morton-sorted copy Ys (x, y, z,
// original index bits; perm[i] = original index of Ys[i]) + PCA + alpha,
// written in the original order of Y.
size_t knn_workspace_bytes(int64_t M, int k);
hipError_t launch_normals(const float *Y, int64_t M, const float4 *Ys, const uint32_t *perm,
                          int k, double alpha_max, double lambda, float *normals, float *kappa,
                          float *alpha, void *work, hipStream_t st);

// Bounding box and first/second moments of a cloud, optionally after the
// state's pose: out[0..2]=sum x', out[3]=sum |x'|^2, out[4..6]=min, out[7..9]=max.
hipError_t launch_moments(const float *P, int64_t n, const DevState *pose, double *partials,
                          int nblk, double *out, hipStream_t st);
int moments_blocks(int64_t n);

// Working volume, sigma^2 floor and (optionally) the initial sigma^2 from the
// moments of Y and of X at the initial pose.
hipError_t launch_init_state(DevState *s, const double *ymom, const double *xmom, int64_t M,
                             int64_t N, int v_auto, int s2_auto, hipStream_t st);

// Points sorted by a Morton code of their position (box = moments of the
// cloud): writes the permuted cloud to out3 (x, y, z) and/or out4 (x, y, z,
// original index bits), and the permutation (sorted position -> original
// index) to perm; any of them may be null.
size_t morton_workspace_bytes(int64_t n);
hipError_t launch_morton_order(const float *P, int64_t n, const double *box, void *work,
                               size_t work_bytes, float *out3, float4 *out4, uint32_t *perm,
                               hipStream_t st);

// Target records.
// Record i describes target perm[i] (perm may be null); rec[M] is a sentinel
// whose exponent is -inf (rec holds M + 1 records); boxes gets one TBox per
// tile of kCullTile records.
hipError_t launch_prep_targets(const float *Y, const float *normals, const float *alpha,
                               const float *pi, const uint32_t *perm, int64_t M, int exact,
                               TRec *rec, TPt *pts, TBox *boxes, hipStream_t st);

// E step: fused exponent + accumulation (over live target tiles in balanced
// work items, or over target chunks), then per-source finalisation + lift to
// the 86 statistics, then the deterministic reduction.
constexpr int kBackendScalar = 0;  // target records via the scalar cache (default)
constexpr int kBackendLds = 1;     // target records staged in LDS
constexpr int kBackendMfma = 2;    // FP64 matrix-core accumulation
constexpr int kPairS = 2;          // sources per thread in the LDS back end

struct EstepPlan {
  int backend;
  // scalar back end (work items over live tiles)
  int cull;          // drop target tiles whose exponentials are all exact zeros
  int ngroups;       // source groups of 256
  int ntiles;        // target tiles of kCullTile records
  int target_items;  // about this many work items per E step
  int cap_items;     // upper bound on the work items (grid of the pair kernel)
  // LDS and MFMA back ends (target chunks)
  int nsplit;        // target chunks
  int64_t mchunk;    // targets per chunk
  int nsrc_blocks;   // source blocks of the accumulation kernel
  int nfin_blocks;   // blocks of the finalisation kernel
};

// Written on the device by each E step of the scalar back end.
struct CullHdr {
  int items;           // work items of the pair kernel
  int tiles_per_item;
};

EstepPlan estep_plan(int64_t N, int64_t M, int backend, int cull, int target_items);
size_t estep_partial_bytes(const EstepPlan &pl, int64_t N);

// Device workspace of the work-item plan, and the counter of evaluated pairs
// inside it (scalar back end; null otherwise).
size_t estep_plan_bytes(const EstepPlan &pl);
unsigned long long *estep_plan_counter(const EstepPlan &pl, void *plan_ws);

// The work-item plan of the scalar back end (no-op for the others), then the
// pair kernel.
hipError_t launch_estep_plan(const EstepPlan &pl, const float *X, int64_t N, const TBox *boxes,
                             DevState *s, void *plan_ws, hipStream_t st);
hipError_t launch_estep_pairs(const EstepPlan &pl, const float *X, int64_t N, const TRec *rec,
                              const TPt *pts, int64_t M, DevState *s, void *plan_ws,
                              double *partial, hipStream_t st);
hipError_t launch_finalize(const EstepPlan &pl, const float *X, int64_t N, const float *w,
                           const DevState *s, const void *plan_ws, const double *partial,
                           double *blockstats, double *colS, double *colstats, hipStream_t st);
hipError_t launch_dump_P(const float *X, int64_t N, const TRec *rec, int64_t M, const float *w,
                         const DevState *s, const double *colS, float *P, hipStream_t st);

// Reduce the block statistics and run the M step.  mode 0: derive only
// (gradient, Hessian, next pose into the *_next fields); mode 1: EM update of
// the state (pose, sigma2, iteration, convergence).
// evcount (may be null): pairs the pair kernel evaluated, added to
// s->evaluated_pairs.
hipError_t launch_reduce_mstep(double *blockstats, int nblk, int64_t N, DevState *s,
                               double *nll_trace, const unsigned long long *evcount, int mode,
                               hipStream_t st);

}  // namespace lsg
