// Internal declarations shared by the HIP sources of liblsgcpd (device state,
// record layouts, kernel launchers).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>
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
constexpr int kGroup = 128;     // sources per group of the scalar pair kernel
constexpr int kFinBlock = 64;   // sources per finalisation block

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
  // outlier weight from the outlier ratio (eta > 0: w0 = w_max at the initial
  // sigma^2) and the target sums it and the confidence priors use
  double eta;
  double pi_sum;      // sum_m phi(y_m) (prior normaliser)
  double pic;         // sum_m pi(m) c_m (2 pi sigma^2)^{3/2}
  int64_t evaluated_pairs;  // pairs the pair kernel evaluated (scalar back end)
  int32_t iter;       // M steps taken
  int32_t done;       // 1 once tol stopped EM (later kernels return at once)
  int32_t converged;
  int32_t gn_fallbacks;
  int32_t newton_iters;
  int32_t numeric_error;
  int32_t newton_max;
  int32_t max_iter;
  int32_t f3_steps;   // E steps in which the BF16 matrix-core kernel took items
  int32_t pad;
};

// Makes v ready at this point: an empty asm that takes v as an operand, so
// the load that produces v is issued and waited for before it.  Before a
// block's exit test (its problem is done) this keeps the loads the block
// needs next in the same memory round trip as the test's own load; the
// compiler would otherwise issue them after the test, one round trip later.
// Where several values must arrive together, the kernels put them in one such
// asm after a scheduling barrier (__builtin_amdgcn_sched_barrier(0)), so that
// every load is issued before any arithmetic waits on one of them.  The "s"
// forms are for wave-uniform values.
__device__ __forceinline__ void ready_s(int v) { asm volatile("" ::"s"(v)); }
__device__ __forceinline__ void ready_s(long long v) { asm volatile("" ::"s"(v)); }
__device__ __forceinline__ void ready_s(double v) { asm volatile("" ::"s"(v)); }
__device__ __forceinline__ void ready_s(const void *v) { asm volatile("" ::"s"(v)); }
__device__ __forceinline__ void ready_v(double v) { asm volatile("" ::"v"(v)); }

// gamma = (2 pi sigma^2)^{3/2} / V: the outlier term of the posterior's
// denominator relative to the component normaliser (Eq. 9)
__device__ inline double gamma_of(const DevState *s) {
  return pow(6.283185307179586477 * s->sigma2, 1.5) / s->V;
}

// Symmetric 3x3 eigen-decomposition by cyclic Jacobi rotations (FP64).
// On return a holds the eigenvalues on its diagonal and v the eigenvectors as
// columns.
__device__ inline void jacobi3(double a[3][3], double v[3][3]) {
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) v[r][c] = r == c ? 1.0 : 0.0;
  const int P[3] = {0, 0, 1};
  const int Q[3] = {1, 2, 2};
  for (int sweep = 0; sweep < 32; ++sweep) {
    const double off = a[0][1] * a[0][1] + a[0][2] * a[0][2] + a[1][2] * a[1][2];
    const double dia = a[0][0] * a[0][0] + a[1][1] * a[1][1] + a[2][2] * a[2][2];
    if (off == 0.0 || off <= 1e-36 * dia) break;
    for (int e = 0; e < 3; ++e) {
      const int p = P[e], q = Q[e];
      const double apq = a[p][q];
      if (apq == 0.0) continue;
      const double theta = (a[q][q] - a[p][p]) / (2.0 * apq);
      double t;
      if (fabs(theta) > 1e150)
        t = 0.5 / theta;
      else
        t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
      const double c = 1.0 / sqrt(t * t + 1.0);
      const double s = t * c;
      a[p][p] -= t * apq;
      a[q][q] += t * apq;
      a[p][q] = a[q][p] = 0.0;
      const int r = 3 - p - q;
      const double arp = a[r][p], arq = a[r][q];
      a[r][p] = a[p][r] = c * arp - s * arq;
      a[r][q] = a[q][r] = s * arp + c * arq;
      for (int k = 0; k < 3; ++k) {
        const double vkp = v[k][p], vkq = v[k][q];
        v[k][p] = c * vkp - s * vkq;
        v[k][q] = s * vkp + c * vkq;
      }
    }
  }
}

// ---------------------------------------------------------------- launchers
// All launchers enqueue on `st` and return the hipError_t of the launch.

// Normals: k nearest neighbours over the Hilbert-sorted copy Ys (x, y, z,
// original index bits; perm[i] = original index of Ys[i]) + PCA + alpha,
// written in the original order of Y.
size_t knn_workspace_bytes(int64_t M, int k);
hipError_t launch_normals(const float *Y, int64_t M, const float4 *Ys, const uint32_t *perm,
                          int k, double alpha_max, double lambda, float *normals, float *kappa,
                          float *alpha, void *work, size_t work_bytes, hipStream_t st);

// Bounding box and first/second moments of a cloud, optionally after the
// state's pose: out[0..2]=sum x', out[3]=sum |x'|^2, out[4..6]=min, out[7..9]=max.
hipError_t launch_moments(const float *P, int64_t n, const DevState *pose, double *partials,
                          int nblk, double *out, hipStream_t st);
int moments_blocks(int64_t n);

// Working volume, sigma^2 floor and (optionally) the initial sigma^2 from the
// moments of Y and of X at the initial pose.
hipError_t launch_init_state(DevState *s, const double *ymom, const double *xmom, int64_t M,
                             int64_t N, int v_auto, int s2_auto, hipStream_t st);

// Points sorted by their index along a Hilbert curve (box = moments of the
// cloud): writes the permuted cloud to out3 (x, y, z) and/or out4 (x, y, z,
// original index bits), and the permutation (sorted position -> original
// index) to perm; any of them may be null.
size_t curve_order_workspace_bytes(int64_t n);
hipError_t launch_curve_order(const float *P, int64_t n, const double *box, void *work,
                              size_t work_bytes, float *out3, float4 *out4, uint32_t *perm,
                              hipStream_t st);

// Target records.
// Record i describes target perm[i] (perm may be null); rec[M] is a sentinel
// whose exponent is -inf (rec holds M + 1 records); boxes gets one TBox per
// tile of kCullTile records.  Priors: pi null => 1/M; else pi[m], divided by
// *pi_sum when pi_sum (device) is not null.
// ftab (may be null): the accumulation features of every tile split into
// BF16 high and low parts for the matrix-core pair kernel (f3_table_bytes),
// and the largest alpha of each tile in its box's `pad`.
hipError_t launch_prep_targets(const float *Y, const float *normals, const float *alpha,
                               const float *pi, const double *pi_sum, const uint32_t *perm,
                               int64_t M, int exact, TRec *rec, TPt *pts, TBox *boxes,
                               void *ftab, hipStream_t st);
size_t f3_table_bytes(int64_t tiles);

// Confidence filtering (confidence.hip).  phi of depth-sensor points from the
// error model coef[0] + coef[1] z + coef[2] z^2; truncation to phi >= threshold
// (order kept; *count on the device); the target sums pi_sum and pic of a
// state (phi null => 1); a float gather dst[i] = src[perm[i]].
hipError_t launch_depth_confidence(const float *P, int64_t n, const double coef[3], double e_min,
                                   float *phi, hipStream_t st);
size_t select_workspace_bytes(int64_t n);
hipError_t launch_select_confident(const float *P, const float *phi, int64_t n, double threshold,
                                   void *work, size_t work_bytes, float *Pout, float *phiout,
                                   uint32_t *count, hipStream_t st);
int prior_blocks(int64_t M);
hipError_t launch_prior_sums(const float *phi, const float *alpha, int64_t M, int exact,
                             double *partials, DevState *s, hipStream_t st);
hipError_t launch_gather_f32(const float *src, const uint32_t *perm, int64_t n, float *dst,
                             hipStream_t st);

// E step: fused exponent + accumulation (over live target tiles in balanced
// work items, or over target chunks), then per-source finalisation + lift to
// the 86 statistics, then the deterministic reduction.
constexpr int kBackendScalar = 0;  // target records via the scalar cache (default)
constexpr int kBackendLds = 1;     // target records staged in LDS
constexpr int kBackendMfma = 2;    // FP64 matrix-core accumulation
constexpr int kPairS = 2;          // sources per thread in the LDS back end

// One registration problem of a batch, as the kernels see it (a table in
// device memory; the single-pair calls are batches of one).
struct Slot {
  const float *X;   // sources, N x 3 (Hilbert order when culled)
  const float *w;   // per-source weights, or null (then phi, else w0 of the state)
  const float *phi; // per-source confidences (order of X): w_n = 1 - (1 - w0) phi_n
  int64_t x_off;    // first source in the batch numbering (colS, colstats)
  int64_t y_off;    // first target in the packed positions; records start at y_off + slot
  int64_t list_off; // live-tile lists of the problem: ngroups x ntiles ints
  int32_t N, M;
  int32_t g_off, ngroups;            // source groups of kGroup (kernel-side constant)
  int32_t t_off, ntiles;             // target tiles of kCullTile
  int32_t item_off, item_cap, target;  // work items (scalar back end)
  int32_t fin_off, nfin;             // finalisation blocks
  int32_t pad;
};

// Host-side plan of one E step over a batch, with the tables the kernels
// index: the problem of every source group, work item and finalisation block.
struct BatchPlan {
  int backend = 0;
  int cull = 0;        // drop target tiles whose exponentials are all exact zeros
  int f3 = 0;          // E steps may run the BF16 matrix-core pair kernel (needs cull)
  int npairs = 0;
  int64_t groups = 0, tiles = 0, items = 0, fins = 0, list_ints = 0;
  int64_t sources = 0, targets = 0;
  std::vector<Slot> slots;
  std::vector<int> grp_slot, item_slot, fin_slot;
  // LDS and MFMA back ends (one problem): target chunks
  int nsplit = 0;
  int64_t mchunk = 0;
  int nsrc_blocks = 0;
};

// Device copies of the tables (one buffer, see batch_tables_*).
struct BatchDev {
  const Slot *slots;
  const int *grp_slot, *item_slot, *fin_slot;
};

// Written on the device by each E step of the scalar back end, per problem.
struct alignas(16) CullHdr {
  int items;           // work items of the problem
  int tiles_per_item;
  int uniform;         // items per group if every group has as many, else 0
  int split;           // 1: the 4 waves of a block share each tile of its item
};

// Plans a batch of sizes N[p], M[p]: work items about target_items in all,
// shared in proportion to M N.  The caller sets slots[p].X and .w.
BatchPlan batch_plan(int npairs, const int64_t *N, const int64_t *M, int backend, int cull,
                     int target_items);
size_t batch_tables_bytes(const BatchPlan &pl);
// Packs the tables for one host-to-device copy and returns the device view of
// a buffer at `dev` holding that copy.
void batch_tables_pack(const BatchPlan &pl, std::vector<char> &host);
BatchDev batch_tables_view(const BatchPlan &pl, const void *dev);

size_t estep_partial_bytes(const BatchPlan &pl);
// Device workspace of the work-item plan, and the per-problem counters of
// evaluated pairs inside it (scalar back end; null otherwise).
size_t estep_plan_bytes(const BatchPlan &pl);
unsigned long long *estep_plan_counter(const BatchPlan &pl, void *plan_ws);
// Item offsets per source group inside the plan workspace (scalar back end;
// null otherwise): the finalisation finds each source's item partials there.
const int *estep_plan_offsets(const BatchPlan &pl, const void *plan_ws);

// The work-item plan of the scalar back end (no-op for the others), then the
// pair kernel, then the per-source finalisation into stat-major block rows
// (problem p: rows at kStats * fin_off, nfin per row).
// With pl.f3 each work item runs on the BF16 matrix-core pair kernel if its
// exponent error bound holds at the current sigma^2 for the item's source
// group and tiles, else on the FP64 one; both kernels are launched and each
// skips the other's items.  ftab and boxes: as launch_prep_targets wrote
// them.  The counters (estep_plan_counter) hold, per problem, the pairs
// evaluated and then, at npairs + p, those of the BF16 kernel.
hipError_t launch_estep_plan(const BatchPlan &pl, const BatchDev &bd, const TBox *boxes,
                             DevState *s, void *plan_ws, hipStream_t st);
hipError_t launch_estep_pairs(const BatchPlan &pl, const BatchDev &bd, const TRec *rec,
                              const TPt *pts, const TBox *boxes, const void *ftab, DevState *s,
                              void *plan_ws, double *partial, hipStream_t st);
hipError_t launch_finalize(const BatchPlan &pl, const BatchDev &bd, const DevState *s,
                           const void *plan_ws, const double *partial, double *blockstats,
                           double *colS, double *colstats, hipStream_t st);
hipError_t launch_dump_P(const float *X, int64_t N, const TRec *rec, int64_t M, const float *w,
                         const DevState *s, const double *colS, float *P, hipStream_t st);

// Reduce the block statistics and run the M step of every problem.  mode 0:
// derive only (gradient, Hessian, next pose into the *_next fields); mode 1:
// EM update of the state (pose, sigma2, iteration, convergence).  nll_trace:
// null or trace_stride doubles per problem.  evcounts (may be null): pairs the
// pair kernels evaluated, added to s[p].evaluated_pairs, and at npairs + p
// those of the BF16 kernel (a nonzero count adds one to s[p].f3_steps);
// both are cleared for the next E step.
hipError_t launch_reduce_mstep(const BatchPlan &pl, const BatchDev &bd, double *blockstats,
                               DevState *s, double *nll_trace, int trace_stride,
                               unsigned long long *evcounts, int mode, hipStream_t st);

// ---------------------------------------------------- pose proposal (f2)
// Encoder parameters (flat float32, see proposal.hip) and the most points
// per cloud the encoder takes.
constexpr int kPropParams = 108425;
constexpr int kPropMaxPoints = 4096;
struct PropPair {
  const float *X, *Y;
  int64_t N, M;
};
// Workspace of a forward (train = 0) or training step (train = 1).
size_t prop_workspace_bytes(int npairs, int train);
// Encoder inputs: P sampled points of each cloud, the source rotated by
// Q[9 b ..] (Q may be null), each centred and expressed in its principal-axis
// frame, divided by the target's RMS radius; norm[kPropNorm b ..] =
// (mu_X, mu_Y, s, F_X, F_Y) with the frames row-major (columns = axes).
constexpr int kPropNorm = 25;
hipError_t launch_prop_inputs(const PropPair *pairs, int npairs, const double *Q, int P, float *Xn,
                              float *Yn, double *norm, hipStream_t st);
// Predicted poses (R row-major, t; world units), pose[12 b ..].
hipError_t launch_prop_forward(const float *theta, int npairs, int P, const float *Xn,
                               const float *Yn, const double *norm, double *pose, void *ws,
                               hipStream_t st);
// One Adam step on the mean loss of the batch: pair b of the batch is the
// inputs of pair idx[b] (idx null: b); label[12 b ..] its pose (R row-major,
// t; world units, source onto target); loss[b] per pair; argmax (2 npairs x
// 256, may be null) the pooled points; grad_out (may be null) the gradient
// that was applied.
hipError_t launch_prop_train(float *theta, float *m, float *v, int step, double lr, int npairs,
                             int P, const float *Xn, const float *Yn, const double *norm,
                             const int *idx, const double *label, double *loss, int *argmax,
                             float *grad_out, void *ws, hipStream_t st);

}  // namespace lsg
