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

// Normals: k nearest neighbours (split over target ranges) + PCA + alpha.
size_t knn_workspace_bytes(int64_t M, int nsplit);
int knn_choose_splits(int64_t M);
hipError_t launch_normals(const float *Y, int64_t M, int k, double alpha_max, double lambda,
                          float *normals, float *kappa, float *alpha, void *work, int nsplit,
                          hipStream_t st);

// Bounding box and first/second moments of a cloud, optionally after the
// state's pose: out[0..2]=sum x', out[3]=sum |x'|^2, out[4..6]=min, out[7..9]=max.
hipError_t launch_moments(const float *P, int64_t n, const DevState *pose, double *partials,
                          int nblk, double *out, hipStream_t st);
int moments_blocks(int64_t n);

// Working volume, sigma^2 floor and (optionally) the initial sigma^2 from the
// moments of Y and of X at the initial pose.
hipError_t launch_init_state(DevState *s, const double *ymom, const double *xmom, int64_t M,
                             int64_t N, int v_auto, int s2_auto, hipStream_t st);

// Target records.
hipError_t launch_prep_targets(const float *Y, const float *normals, const float *alpha,
                               const float *pi, int64_t M, int exact, TRec *rec, hipStream_t st);

// E step: fused exponent + accumulation over target chunks, then per-source
// finalisation + lift to the 86 statistics, then the deterministic reduction.
constexpr int kBackendScalar = 0;  // target records via the scalar cache (default)
constexpr int kBackendLds = 1;     // target records staged in LDS
constexpr int kBackendMfma = 2;    // FP64 matrix-core accumulation
constexpr int kPairS = 2;          // sources per lane in the VALU back ends

struct EstepPlan {
  int backend;
  int srcs_per_lane;  // sources per lane of the VALU back ends (2 or 4)
  int parts;          // target sub-ranges per block of the scalar back end (1, 2, 4)
  int nsplit;      // target chunks
  int64_t mchunk;  // targets per chunk (multiple of the tile)
  int nsrc_blocks; // source blocks of the accumulation kernel
  int nfin_blocks; // blocks of the finalisation kernel
};
EstepPlan estep_plan(int64_t N, int64_t M, int backend, int srcs_per_lane, int parts);
size_t estep_partial_bytes(const EstepPlan &pl, int64_t N);

hipError_t launch_estep(const EstepPlan &pl, const float *X, int64_t N, const TRec *rec,
                        int64_t M, const DevState *s, double *partial, hipStream_t st);
hipError_t launch_finalize(const EstepPlan &pl, const float *X, int64_t N, const float *w,
                           const DevState *s, const double *partial, double *blockstats,
                           double *colS, double *colstats, hipStream_t st);
hipError_t launch_dump_P(const float *X, int64_t N, const TRec *rec, int64_t M, const float *w,
                         const DevState *s, const double *colS, float *P, hipStream_t st);

// Reduce the block statistics and run the M step.  mode 0: derive only
// (gradient, Hessian, next pose into the *_next fields); mode 1: EM update of
// the state (pose, sigma2, iteration, convergence).
hipError_t launch_reduce_mstep(double *blockstats, int nblk, int64_t N, DevState *s,
                               double *nll_trace, int mode, hipStream_t st);

}  // namespace lsg
