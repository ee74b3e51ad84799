// Host side of liblsgcpd: argument validation, context workspace and the
// launch sequence of each public call (include/lsgcpd.h).
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "lsgcpd.h"
#include "lsgcpd_internal.h"

#define LSG_API extern "C" __attribute__((visibility("default")))

using lsg::DevState;

namespace {

constexpr int64_t kMaxPoints = (int64_t)1 << 27;

// Device memory of lsgcpd_estep_noalloc: one array per GPU, mapped once per
// device when the first context on it is created, kept until the process
// ends.  Host code never passes the array's name to a kernel or a copy (on
// the host it is a stand-in, not a device address): it uses the address that
// hipGetSymbolAddress returned for the device.  Every point count up to
// kNoAllocMaxPoints fits with kNoAllocItems work items (the largest layout,
// M = N = 65,536, takes about 31 MiB).
constexpr size_t kScratchBytes = (size_t)36 << 20;
constexpr int64_t kNoAllocMaxPoints = 65536;
constexpr int kNoAllocItems = 1024;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
std::mutex scratch_mutex;
void *scratch_ptr[kMaxDevices];  // device address of `scratch` on each device

// Maps the scratch array of the current device (once per device).
hipError_t map_scratch(int device, void **out) {
  std::lock_guard<std::mutex> lock(scratch_mutex);
  if (device < 0 || device >= kMaxDevices) {
    *out = nullptr;
    return hipSuccess;
  }
  if (!scratch_ptr[device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    scratch_ptr[device] = p;
  }
  *out = scratch_ptr[device];
  return hipSuccess;
}
constexpr int kMaxBatch = 1 << 16;
// The set-up of a batch (sorting, neighbour search and records of every
// cloud: a few small kernels per cloud) runs on this many streams at once.
constexpr int kSetupLanes = 4;
// A single pair with at most this many source-target pairs is registered
// without culling: its E step is too small to fill the GPU either way, and
// the two plan kernels per iteration (the group boxes and live-tile lists,
// then the items) cost more than the exact zeros they skip.  The dense plan
// does not change between iterations and is laid out once.
constexpr int64_t kDenseAutoPairs = (int64_t)1 << 22;

struct Buf {
  void *p = nullptr;
  size_t cap = 0;
};

}  // namespace

struct lsgcpd_ctx {
  int device = 0;
  void *scratch = nullptr;  // the device's static scratch array (lsgcpd_estep_noalloc)
  std::string err;
  Buf knn, rec, pts, boxes, ftab, ptab, pws, pbatch, pin, plan, partial, blockstats, colS, mom_part, mom, nrm, kap, alp,
      trace, order, xperm, yperm, ys4, tables, states;
  // confidence filtering: kept points and confidences of X and Y, selection
  // workspace, sorted source confidences, source permutation, prior sums
  Buf cfx, cfy, cfwork, xphi, xidx, prior;
  // set-up lanes 1 .. kSetupLanes - 1 of a batch: a stream each and their own
  // copies of the set-up scratch (lane 0 is the caller's stream with the
  // buffers above)
  struct LaneBufs {
    Buf order, knn, mom_part, mom, prior, xidx;
  };
  LaneBufs lane[kSetupLanes - 1];
  hipStream_t lstream[kSetupLanes - 1] = {};
  hipEvent_t lfork = nullptr;
  hipEvent_t ljoin[kSetupLanes - 1] = {};
  uint32_t *hcount = nullptr;  // pinned: kept point counts
  // work-item targets chosen by lsgcpd_autotune, per size class
  // (floor(log2(sum of M N))); forced_items > 0 overrides while tuning
  std::map<int, int> tuned_items;
  int forced_items = 0;
  // the recorded EM loop (LSGCPD_GRAPH), the stream it is recorded and
  // replayed on, and what it was recorded for
  hipStream_t gstream = nullptr;
  hipEvent_t gev[2] = {nullptr, nullptr};
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  std::vector<int64_t> gsig;
  DevState *dstate = nullptr;  // device states (ctx->states), one per problem of a batch
  DevState *hstate = nullptr;  // pinned host staging for hcap states
  size_t hcap = 0;
  std::vector<char> htables;   // host copy of the batch tables
  char *htab_pinned = nullptr; // pinned staging of that copy (an asynchronous upload)
  size_t htab_cap = 0;
  double *htr_pinned = nullptr;  // pinned copy of the NLL traces (read back with the states)
  size_t htr_cap = 0;
  std::vector<double> htrace;
  // E-step timing: 4 events per E step (start, before and after the pair
  // kernel, end)
  bool prof = false;
  std::vector<hipEvent_t> events;
  int ev_used = 0;
  int64_t prof_pairs_pending = 0;
  lsgcpd_profile totals = {0, 0, 0.0, 0.0, 0};
  std::vector<double> launch_pair_us, launch_estep_us;  // per timed E step, in order
};

namespace {

lsgcpd_status fail(lsgcpd_ctx *c, lsgcpd_status s, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  c->err = buf;
  return s;
}

#define HIPCHK(call)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail(ctx, LSGCPD_E_HIP, "%s failed: %s", #call, hipGetErrorString(e_));        \
  } while (0)

lsgcpd_status ensure(lsgcpd_ctx *ctx, Buf &b, size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (b.cap >= bytes) return LSGCPD_OK;
  if (b.p) {
    hipError_t e = hipFree(b.p);
    b.p = nullptr;
    b.cap = 0;
    if (e != hipSuccess) return fail(ctx, LSGCPD_E_HIP, "hipFree: %s", hipGetErrorString(e));
  }
  hipError_t e = hipMalloc(&b.p, bytes);
  if (e != hipSuccess) {
    b.p = nullptr;
    (void)hipGetLastError();
    return fail(ctx, LSGCPD_E_NOMEM, "workspace allocation of %zu bytes failed: %s", bytes,
                hipGetErrorString(e));
  }
  b.cap = bytes;
  return LSGCPD_OK;
}

#define RETURN_IF(x)                \
  do {                              \
    lsgcpd_status s_ = (x);         \
    if (s_ != LSGCPD_OK) return s_; \
  } while (0)

#define ENSURE(buf, bytes)                                     \
  do {                                                         \
    lsgcpd_status s_ = ensure(ctx, ctx->buf, (size_t)(bytes)); \
    if (s_ != LSGCPD_OK) return s_;                            \
  } while (0)

bool finite_pos(double v) { return isfinite(v) && v > 0.0; }

constexpr uint32_t kKnownFlags = LSGCPD_EXACT_NORMALIZER | LSGCPD_PAIRS_LDS | LSGCPD_PAIRS_MFMA |
                                 LSGCPD_DENSE | LSGCPD_GRAPH | LSGCPD_BF16_CROSS;

// About this many work items per E step for the scalar back end, by the
// number of pairs of the E step (whole registrations measured on MI355X: 1024
// was fastest at 6.4e7 pairs, 4096 and 8192 tie at 4e8, 8192 at 2.5e9 and
// 5e9; the thresholds sit between those sizes); LSGCPD_WORK_ITEMS overrides
// it for tuning sweeps.
int work_items(uint64_t pairs) {
  const char *e = getenv("LSGCPD_WORK_ITEMS");
  const int v = e ? atoi(e) : 0;
  if (v >= 64 && v <= (1 << 20)) return v;
  return pairs <= 160000000ull ? 1024 : pairs <= 1600000000ull ? 4096 : 8192;
}

int size_class(int npairs, const int64_t *N, const int64_t *M) {
  uint64_t mn = 1;
  for (int i = 0; i < npairs; ++i) mn += (uint64_t)N[i] * (uint64_t)M[i];
  int c = 0;
  while (mn >>= 1) ++c;
  return c;
}

// Work-item target of an E step over these sizes: the one lsgcpd_autotune
// measured fastest for their size class, else work_items(sum of M N).
int items_for(const lsgcpd_ctx *ctx, int npairs, const int64_t *N, const int64_t *M) {
  if (ctx->forced_items > 0) return ctx->forced_items;
  auto it = ctx->tuned_items.find(size_class(npairs, N, M));
  if (it != ctx->tuned_items.end()) return it->second;
  uint64_t mn = 0;
  for (int i = 0; i < npairs; ++i) mn += (uint64_t)N[i] * (uint64_t)M[i];
  return work_items(mn);
}

int backend_of(uint32_t flags) {
  if (flags & LSGCPD_PAIRS_MFMA) return lsg::kBackendMfma;
  if (flags & LSGCPD_PAIRS_LDS) return lsg::kBackendLds;
  return lsg::kBackendScalar;
}

lsgcpd_status check_pose(lsgcpd_ctx *ctx, const lsgcpd_pose *g) {
  for (int i = 0; i < 9; ++i)
    if (!isfinite(g->R[i])) return fail(ctx, LSGCPD_E_INVALID, "pose R is not finite");
  for (int i = 0; i < 3; ++i)
    if (!isfinite(g->t[i])) return fail(ctx, LSGCPD_E_INVALID, "pose t is not finite");
  double dev = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += g->R[3 * k + i] * g->R[3 * k + j];
      dev = fmax(dev, fabs(s - (i == j ? 1.0 : 0.0)));
    }
  const double det = g->R[0] * (g->R[4] * g->R[8] - g->R[5] * g->R[7]) -
                     g->R[1] * (g->R[3] * g->R[8] - g->R[5] * g->R[6]) +
                     g->R[2] * (g->R[3] * g->R[7] - g->R[4] * g->R[6]);
  if (dev > 1e-6 || det <= 0.0)
    return fail(ctx, LSGCPD_E_INVALID, "pose R is not a rotation (|R^T R - I| = %g, det = %g)",
                dev, det);
  return LSGCPD_OK;
}

// Checks shared by the registration calls.
lsgcpd_status check_params(lsgcpd_ctx *ctx, const lsgcpd_params *p) {
  if (p->k < 1 || p->k > 32)
    return fail(ctx, LSGCPD_E_INVALID, "k = %d must satisfy 1 <= k <= min(M, 32)", p->k);
  if (!(p->alpha_max >= 0.0) || !isfinite(p->alpha_max))
    return fail(ctx, LSGCPD_E_INVALID, "alpha_max must be finite and >= 0");
  if (!finite_pos(p->lambda)) return fail(ctx, LSGCPD_E_INVALID, "lambda must be finite and > 0");
  if (!(p->eta < 1.0) || !isfinite(p->eta))
    return fail(ctx, LSGCPD_E_INVALID, "eta must be finite and < 1");
  if (!(p->eta > 0.0) && !(p->w0 > 0.0 && p->w0 < 1.0))
    return fail(ctx, LSGCPD_E_INVALID, "w0 must lie in (0, 1)");
  if (!isfinite(p->V) || !isfinite(p->tol) || !isfinite(p->sigma2_init))
    return fail(ctx, LSGCPD_E_INVALID, "V, tol and sigma2_init must be finite");
  if (p->max_iter < 0 || p->max_iter > 100000)
    return fail(ctx, LSGCPD_E_INVALID, "max_iter = %d out of range", p->max_iter);
  if (p->newton_max < 1 || p->newton_max > 1000)
    return fail(ctx, LSGCPD_E_INVALID, "newton_max = %d out of range", p->newton_max);
  if (p->flags & ~kKnownFlags) return fail(ctx, LSGCPD_E_INVALID, "unknown flags 0x%x", p->flags);
  if ((p->flags & LSGCPD_PAIRS_LDS) && (p->flags & LSGCPD_PAIRS_MFMA))
    return fail(ctx, LSGCPD_E_INVALID, "LSGCPD_PAIRS_LDS and LSGCPD_PAIRS_MFMA exclude each other");
  if ((p->flags & LSGCPD_BF16_CROSS) &&
      (p->flags & (LSGCPD_PAIRS_LDS | LSGCPD_PAIRS_MFMA | LSGCPD_DENSE)))
    return fail(ctx, LSGCPD_E_INVALID,
                "LSGCPD_BF16_CROSS runs on the culled default plan (no LDS, MFMA or DENSE flag)");
  return LSGCPD_OK;
}

lsgcpd_status set_device(lsgcpd_ctx *ctx) {
  HIPCHK(hipSetDevice(ctx->device));
  return LSGCPD_OK;
}

void fill_state(DevState *s, const lsgcpd_pose *g, double sigma2, double V, double w0,
                double eta, double tol, int newton_max, int max_iter) {
  memset(s, 0, sizeof(DevState));
  if (g) {
    memcpy(s->R, g->R, sizeof s->R);
    memcpy(s->t, g->t, sizeof s->t);
  } else {
    s->R[0] = s->R[4] = s->R[8] = 1.0;
  }
  s->sigma2 = sigma2;
  s->V = V;
  s->w0 = w0;
  s->eta = eta > 0.0 ? eta : 0.0;
  s->pi_sum = 1.0;
  s->pic = 1.0;
  s->tol = tol;
  s->newton_max = newton_max;
  s->max_iter = max_iter;
}

// Device and pinned host states for n problems.
lsgcpd_status ensure_states(lsgcpd_ctx *ctx, int n) {
  ENSURE(states, (size_t)n * sizeof(DevState));
  ctx->dstate = (DevState *)ctx->states.p;
  if (ctx->hcap < (size_t)n) {
    if (ctx->hstate) (void)hipHostFree(ctx->hstate);
    ctx->hstate = nullptr;
    ctx->hcap = 0;
    if (hipHostMalloc((void **)&ctx->hstate, (size_t)n * sizeof(DevState), hipHostMallocDefault) !=
        hipSuccess) {
      ctx->hstate = nullptr;
      (void)hipGetLastError();
      return fail(ctx, LSGCPD_E_NOMEM, "pinned host staging for %d states failed", n);
    }
    ctx->hcap = (size_t)n;
  }
  return LSGCPD_OK;
}

// The stream and set-up scratch of lane q (0: the caller's stream st).
struct Lane {
  hipStream_t st;
  Buf *order, *knn, *mom_part, *mom, *prior, *xidx;
};

Lane lane_of(lsgcpd_ctx *ctx, int q, hipStream_t st) {
  if (q == 0) return {st, &ctx->order, &ctx->knn, &ctx->mom_part, &ctx->mom, &ctx->prior, &ctx->xidx};
  lsgcpd_ctx::LaneBufs &b = ctx->lane[q - 1];
  return {ctx->lstream[q - 1], &b.order, &b.knn, &b.mom_part, &b.mom, &b.prior, &b.xidx};
}

// Device memory read and written by the kernels of an E step: the context's
// workspace, or regions of the library's static scratch array.  timed: record
// the context's timing events around the E-step kernels.
struct EstepMem {
  DevState *state;  // one per problem
  lsg::TRec *rec;
  lsg::TPt *pts;
  lsg::TBox *boxes;
  void *ftab;  // BF16 feature tables (null unless the plan may use them)
  void *plan;
  double *partial;
  double *blockstats;
  bool timed;
};

// The context's workspace (valid until the next ensure_* call).
EstepMem ctx_mem(lsgcpd_ctx *ctx) {
  return {ctx->dstate,
          (lsg::TRec *)ctx->rec.p,
          (lsg::TPt *)ctx->pts.p,
          (lsg::TBox *)ctx->boxes.p,
          ctx->ftab.p,
          ctx->plan.p,
          (double *)ctx->partial.p,
          (double *)ctx->blockstats.p,
          ctx->prof};
}

// Streams and events of lanes 1 .. n - 1 (created once, default priority).
lsgcpd_status ensure_lanes(lsgcpd_ctx *ctx, int n) {
  if (n > 1 && !ctx->lfork) HIPCHK(hipEventCreateWithFlags(&ctx->lfork, hipEventDisableTiming));
  for (int q = 1; q < n; ++q) {
    if (!ctx->lstream[q - 1])
      HIPCHK(hipStreamCreateWithFlags(&ctx->lstream[q - 1], hipStreamNonBlocking));
    if (!ctx->ljoin[q - 1])
      HIPCHK(hipEventCreateWithFlags(&ctx->ljoin[q - 1], hipEventDisableTiming));
  }
  return LSGCPD_OK;
}

// Lanes 1 .. n - 1 start after the work queued on st so far ...
lsgcpd_status fork_lanes(lsgcpd_ctx *ctx, int n, hipStream_t st) {
  if (n <= 1) return LSGCPD_OK;
  HIPCHK(hipEventRecord(ctx->lfork, st));
  for (int q = 1; q < n; ++q) HIPCHK(hipStreamWaitEvent(ctx->lstream[q - 1], ctx->lfork, 0));
  return LSGCPD_OK;
}

// ... and st continues after all of their work.
lsgcpd_status join_lanes(lsgcpd_ctx *ctx, int n, hipStream_t st) {
  for (int q = 1; q < n; ++q) {
    HIPCHK(hipEventRecord(ctx->ljoin[q - 1], ctx->lstream[q - 1]));
    HIPCHK(hipStreamWaitEvent(st, ctx->ljoin[q - 1], 0));
  }
  return LSGCPD_OK;
}

// Problem p of a batch: target records (record i of the problem describes its
// target yperm[i], or target i if yperm is null) and their tile boxes, then
// moments of Y, X at the problem's pose, then init_state.
// Target records, working volume, sigma^2 floor and initial sigma^2 of
// problem p.  Priors: pi (raw priors) or phi (target confidences, normalised
// on the device: Sec. 3.3), else uniform; with eta > 0 the state's w0 becomes
// w_max (Sec. 3.2).
lsgcpd_status setup_problem(lsgcpd_ctx *ctx, const Lane &ln, const EstepMem &mem,
                            const lsg::BatchPlan &pl, int p,
                            const float *Y, const float *normals, const float *alpha,
                            const float *pi, const float *phi, double eta,
                            const uint32_t *yperm, uint32_t flags, int v_auto, int s2_auto) {
  const hipStream_t st = ln.st;
  const lsg::Slot &sl = pl.slots[p];
  const int exact = (flags & LSGCPD_EXACT_NORMALIZER) ? 1 : 0;
  if (phi || eta > 0.0)
    HIPCHK(lsg::launch_prior_sums(phi, alpha, sl.M, exact, (double *)ln.prior->p,
                                  mem.state + p, st));
  HIPCHK(lsg::launch_prep_targets(Y, normals, alpha, phi ? phi : pi,
                                  phi ? &(mem.state + p)->pi_sum : nullptr, yperm, sl.M,
                                  exact,
                                  mem.rec + sl.y_off + p, mem.pts + sl.y_off,
                                  mem.boxes + sl.t_off,
                                  pl.f3 ? (char *)mem.ftab + lsg::f3_table_bytes(sl.t_off)
                                        : nullptr,
                                  st));
  double *ymom = (double *)ln.mom->p;
  double *xmom = ymom + 16;
  HIPCHK(lsg::launch_moments(Y, sl.M, nullptr, (double *)ln.mom_part->p,
                             lsg::moments_blocks(sl.M), ymom, st));
  if (s2_auto)
    HIPCHK(lsg::launch_moments(sl.X, sl.N, mem.state + p, (double *)ln.mom_part->p,
                               lsg::moments_blocks(sl.N), xmom, st));
  HIPCHK(lsg::launch_init_state(mem.state + p, ymom, xmom, sl.M, sl.N, v_auto, s2_auto, st));
  return LSGCPD_OK;
}

// Y (M points) in Hilbert order into ys4 + off (x, y, z, index within Y) and
// yperm + off.
lsgcpd_status sort_targets(lsgcpd_ctx *ctx, const Lane &ln, const float *Y, int64_t M,
                           int64_t off) {
  const hipStream_t st = ln.st;
  const int nb = lsg::moments_blocks(M);
  double *box = (double *)ln.mom->p + 32;
  HIPCHK(lsg::launch_moments(Y, M, nullptr, (double *)ln.mom_part->p, nb, box, st));
  HIPCHK(lsg::launch_curve_order(Y, M, box, ln.order->p, ln.order->cap, nullptr,
                                 (float4 *)ctx->ys4.p + off, (uint32_t *)ctx->yperm.p + off, st));
  return LSGCPD_OK;
}

lsgcpd_status normals_sorted(lsgcpd_ctx *ctx, const Lane &ln, const float *Y, int64_t M,
                             int64_t off, int k, double alpha_max, double lambda, float *normals,
                             float *kappa, float *alpha) {
  HIPCHK(lsg::launch_normals(Y, M, (const float4 *)ctx->ys4.p + off,
                             (const uint32_t *)ctx->yperm.p + off, k, alpha_max, lambda, normals,
                             kappa, alpha, ln.knn->p, ln.knn->cap, ln.st));
  return LSGCPD_OK;
}

// Workspace of the Hilbert-order sorts and moments of the npairs clouds of N[i]
// sources (N may be null) and M[i] targets, of the neighbour search (k
// neighbours) over each target cloud, and the sorted copies of `mtot`
// targets.  The sort and search workspaces are maxima over the clouds, not
// the workspace of the largest cloud: the number of target splits of the
// search falls as M grows, and so may the sort's scratch.  Each of the first
// `lanes` set-up lanes gets its own scratch.
lsgcpd_status ensure_geometry(lsgcpd_ctx *ctx, int npairs, const int64_t *N, const int64_t *M,
                              int64_t mtot, int k, int lanes) {
  size_t ob = 0, kb = 0;
  int64_t nmax = 1;
  for (int i = 0; i < npairs; ++i) {
    const int64_t n = N ? N[i] : 0;
    const size_t a = lsg::curve_order_workspace_bytes(M[i]);
    const size_t b = n > 0 ? lsg::curve_order_workspace_bytes(n) : 0;
    const size_t c = lsg::knn_workspace_bytes(M[i], k);
    ob = a > ob ? a : ob;
    ob = b > ob ? b : ob;
    kb = c > kb ? c : kb;
    nmax = M[i] > nmax ? M[i] : nmax;
    nmax = n > nmax ? n : nmax;
  }
  ENSURE(yperm, (size_t)mtot * sizeof(uint32_t));
  ENSURE(ys4, (size_t)mtot * sizeof(float4));
  for (int q = 0; q < lanes; ++q) {
    const Lane ln = lane_of(ctx, q, nullptr);
    RETURN_IF(ensure(ctx, *ln.order, ob));
    RETURN_IF(ensure(ctx, *ln.mom_part, (size_t)lsg::moments_blocks(nmax) * 10 * sizeof(double)));
    RETURN_IF(ensure(ctx, *ln.mom, 48 * sizeof(double)));
    RETURN_IF(ensure(ctx, *ln.knn, kb));
    RETURN_IF(ensure(ctx, *ln.prior, (size_t)2 * lsg::prior_blocks(nmax) * sizeof(double)));
  }
  return ensure_lanes(ctx, lanes);
}

// Makes room for `steps` more timed E steps (no-op unless profiling).
lsgcpd_status prof_reserve(lsgcpd_ctx *ctx, int steps) {
  if (!ctx->prof) return LSGCPD_OK;
  const size_t need = (size_t)(ctx->ev_used + 4 * steps);
  while (ctx->events.size() < need) {
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    ctx->events.push_back(e);
  }
  return LSGCPD_OK;
}

lsgcpd_status prof_record(lsgcpd_ctx *ctx, hipStream_t st) {
  if (!ctx->prof || ctx->ev_used >= (int)ctx->events.size()) return LSGCPD_OK;
  HIPCHK(hipEventRecord(ctx->events[ctx->ev_used++], st));
  return LSGCPD_OK;
}

// After the stream has been synchronised: fold the recorded events and the
// pairs the pair kernel evaluated into the totals.
lsgcpd_status prof_collect(lsgcpd_ctx *ctx, int64_t evaluated) {
  if (!ctx->prof) return LSGCPD_OK;
  ctx->totals.evaluated_pairs += evaluated;
  for (int i = 0; i + 4 <= ctx->ev_used; i += 4) {
    float a = 0.f, b = 0.f;
    HIPCHK(hipEventElapsedTime(&a, ctx->events[i + 1], ctx->events[i + 2]));
    HIPCHK(hipEventElapsedTime(&b, ctx->events[i], ctx->events[i + 3]));
    ctx->totals.pair_kernel_ms += a;
    ctx->totals.estep_ms += b;
    ctx->launch_pair_us.push_back(1e3 * a);
    ctx->launch_estep_us.push_back(1e3 * b);
    ctx->totals.launches += 1;
  }
  ctx->totals.pairs += ctx->prof_pairs_pending;
  ctx->prof_pairs_pending = 0;
  ctx->ev_used = 0;
  return LSGCPD_OK;
}

// One E step (plan, accumulation, finalisation) + reduction/M step in
// `mode`, for every problem of the batch.  first: the first E step of the
// call (a dense plan is laid out only then; a culled one every E step).
lsgcpd_status run_estep(lsgcpd_ctx *ctx, const lsg::BatchPlan &pl, const lsg::BatchDev &bd,
                        const EstepMem &mem, double *colS, double *colstats, double *trace,
                        int trace_stride, int mode, hipStream_t st, bool first = true) {
  lsgcpd_status s = LSGCPD_OK;
  if (mem.timed && (s = prof_record(ctx, st)) != LSGCPD_OK) return s;
  if (first || pl.cull) HIPCHK(lsg::launch_estep_plan(pl, bd, mem.boxes, mem.state, mem.plan, st));
  if (mem.timed && (s = prof_record(ctx, st)) != LSGCPD_OK) return s;
  HIPCHK(lsg::launch_estep_pairs(pl, bd, mem.rec, mem.pts, mem.boxes, mem.ftab, mem.state,
                                 mem.plan, mem.partial, st));
  if (mem.timed && (s = prof_record(ctx, st)) != LSGCPD_OK) return s;
  HIPCHK(lsg::launch_finalize(pl, bd, mem.state, mem.plan, mem.partial, mem.blockstats, colS,
                              colstats, st));
  if (mem.timed && (s = prof_record(ctx, st)) != LSGCPD_OK) return s;
  if (mem.timed)
    for (const lsg::Slot &sl : pl.slots) ctx->prof_pairs_pending += (int64_t)sl.M * sl.N;
  HIPCHK(lsg::launch_reduce_mstep(pl, bd, mem.blockstats, mem.state, trace, trace_stride,
                                  lsg::estep_plan_counter(pl, mem.plan), mode, st));
  return LSGCPD_OK;
}

// max_iter EM iterations of every problem, launched one by one, or (graph)
// replayed from a recording of all of them.  Every kernel of the loop takes
// only context buffers and the plan's sizes as arguments (the problems'
// clouds are reached through the tables uploaded before), so a recording
// stays valid while the sizes, parameters and buffers it was made with do.
// It is made and replayed on a stream of the context, ordered after `st`
// and before the rest of `st` by events.
lsgcpd_status run_em(lsgcpd_ctx *ctx, const lsg::BatchPlan &pl, const lsg::BatchDev &bd,
                     int max_iter, int stride, bool graph, hipStream_t st) {
  if (!graph || ctx->prof || max_iter < 1) {
    for (int it = 0; it < max_iter; ++it)
      RETURN_IF(run_estep(ctx, pl, bd, ctx_mem(ctx), nullptr, nullptr, (double *)ctx->trace.p,
                                stride, 1, st, it == 0));
    return LSGCPD_OK;
  }
  if (!ctx->gstream) {
    HIPCHK(hipStreamCreateWithFlags(&ctx->gstream, hipStreamNonBlocking));
    for (hipEvent_t &e : ctx->gev) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }
  std::vector<int64_t> sig = {pl.npairs, pl.backend, pl.cull, pl.groups, pl.tiles, pl.items,
                              pl.fins, pl.list_ints, max_iter, stride};
  for (const lsg::Slot &sl : pl.slots) {
    sig.push_back(sl.N);
    sig.push_back(sl.M);
  }
  for (const Buf *b : {&ctx->plan, &ctx->partial, &ctx->blockstats, &ctx->rec, &ctx->pts,
                       &ctx->boxes, &ctx->states, &ctx->trace, &ctx->tables})
    sig.push_back((int64_t)(intptr_t)b->p);
  hipStream_t gs = ctx->gstream;
  HIPCHK(hipEventRecord(ctx->gev[0], st));
  HIPCHK(hipStreamWaitEvent(gs, ctx->gev[0], 0));
  if (!ctx->gexec || sig != ctx->gsig) {
    if (ctx->gexec) (void)hipGraphExecDestroy(ctx->gexec);
    if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
    ctx->gexec = nullptr;
    ctx->graph = nullptr;
    ctx->gsig.clear();
    HIPCHK(hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal));
    lsgcpd_status s = LSGCPD_OK;
    for (int it = 0; it < max_iter && s == LSGCPD_OK; ++it)
      s = run_estep(ctx, pl, bd, ctx_mem(ctx), nullptr, nullptr, (double *)ctx->trace.p,
                    stride, 1, gs, it == 0);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(gs, &g);
    if (s != LSGCPD_OK || e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return s != LSGCPD_OK ? s
                            : fail(ctx, LSGCPD_E_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    }
    ctx->graph = g;
    HIPCHK(hipGraphInstantiate(&ctx->gexec, g, nullptr, nullptr, 0));
    ctx->gsig = sig;
  }
  HIPCHK(hipGraphLaunch(ctx->gexec, gs));
  HIPCHK(hipEventRecord(ctx->gev[1], gs));
  HIPCHK(hipStreamWaitEvent(st, ctx->gev[1], 0));
  return LSGCPD_OK;
}

// E-step workspace and the tables of the plan (uploaded on `st`).
lsgcpd_status ensure_estep(lsgcpd_ctx *ctx, const lsg::BatchPlan &pl) {
  ENSURE(plan, lsg::estep_plan_bytes(pl));
  ENSURE(partial, lsg::estep_partial_bytes(pl));
  ENSURE(blockstats, (size_t)pl.fins * lsg::kStats * sizeof(double));
  ENSURE(tables, lsg::batch_tables_bytes(pl));
  ENSURE(rec, (size_t)(pl.targets + pl.npairs) * sizeof(lsg::TRec));  // + a sentinel each
  ENSURE(pts, (size_t)pl.targets * sizeof(lsg::TPt));
  ENSURE(boxes, (size_t)pl.tiles * sizeof(lsg::TBox));
  if (pl.f3) ENSURE(ftab, lsg::f3_table_bytes(pl.tiles));
  ENSURE(mom, 48 * sizeof(double));
  int64_t nmax = 1;
  for (const lsg::Slot &sl : pl.slots) {
    nmax = sl.N > nmax ? sl.N : nmax;
    nmax = sl.M > nmax ? sl.M : nmax;
  }
  ENSURE(mom_part, (size_t)lsg::moments_blocks(nmax) * 10 * sizeof(double));
  return LSGCPD_OK;
}

lsgcpd_status upload_tables(lsgcpd_ctx *ctx, const lsg::BatchPlan &pl, hipStream_t st,
                            lsg::BatchDev *bd) {
  lsg::batch_tables_pack(pl, ctx->htables);
  const size_t n = ctx->htables.size();
  if (ctx->htab_cap < n) {
    // the previous upload from the staging buffer has completed: every call
    // synchronises its stream before returning
    if (ctx->htab_pinned) (void)hipHostFree(ctx->htab_pinned);
    ctx->htab_pinned = nullptr;
    ctx->htab_cap = 0;
    if (hipHostMalloc((void **)&ctx->htab_pinned, n, hipHostMallocDefault) != hipSuccess) {
      ctx->htab_pinned = nullptr;
      (void)hipGetLastError();
      return fail(ctx, LSGCPD_E_NOMEM, "pinned staging of %zu bytes failed", n);
    }
    ctx->htab_cap = n;
  }
  memcpy(ctx->htab_pinned, ctx->htables.data(), n);
  HIPCHK(hipMemcpyAsync(ctx->tables.p, ctx->htab_pinned, n, hipMemcpyHostToDevice, st));
  *bd = lsg::batch_tables_view(pl, ctx->tables.p);
  return LSGCPD_OK;
}

// Target geometry of pair i (Hilbert order of Y, neighbours, normals) and,
// with culling, its sources in Hilbert order (their confidences carried
// along), on lane ln.  With culling the target records follow the Hilbert
// order of Y and the sources are put in Hilbert order too, so that a source
// group's and a target tile's points are neighbours.  Every statistic is a
// sum over all sources and all targets, so the order changes only the
// rounding of the sums.
lsgcpd_status pair_geometry(lsgcpd_ctx *ctx, const Lane &ln, lsg::BatchPlan &pl, int i,
                            const float *X, const float *Y, const float *phx,
                            const lsgcpd_params *p, float *nrm, float *kap, float *alp) {
  lsg::Slot &sl = pl.slots[i];
  const int64_t yo = sl.y_off, M = sl.M, N = sl.N;
  RETURN_IF(sort_targets(ctx, ln, Y, M, yo));
  RETURN_IF(normals_sorted(ctx, ln, Y, M, yo, p->k, p->alpha_max, p->lambda, nrm + 3 * yo,
                           kap + yo, alp + yo));
  sl.X = X;
  sl.w = nullptr;
  sl.phi = phx;
  if (pl.cull && N > 256) {
    const hipStream_t st = ln.st;
    float *xs = (float *)ctx->xperm.p + 3 * sl.x_off;
    double *xbox = (double *)ln.mom->p + 32;
    uint32_t *xi = phx ? (uint32_t *)ln.xidx->p : nullptr;
    HIPCHK(lsg::launch_moments(X, N, nullptr, (double *)ln.mom_part->p, lsg::moments_blocks(N),
                               xbox, st));
    HIPCHK(lsg::launch_curve_order(X, N, xbox, ln.order->p, ln.order->cap, xs, nullptr, xi, st));
    sl.X = xs;
    if (phx) {  // confidences follow their points
      float *ps = (float *)ctx->xphi.p + sl.x_off;
      HIPCHK(lsg::launch_gather_f32(phx, xi, N, ps, st));
      sl.phi = ps;
    }
  }
  return LSGCPD_OK;
}

// Registration of npairs problems that share the parameters: the E steps and
// M steps of all problems run in the same launches.
// phi_x / phi_y: null, or per-pair source / target confidences (entries may
// be null) for confidence filtering (Sec. 3.3).
lsgcpd_status register_problems(lsgcpd_ctx *ctx, int npairs, const float *const *X,
                                const int64_t *N, const float *const *Y, const int64_t *M,
                                const float *const *phi_x, const float *const *phi_y,
                                const lsgcpd_params *p, const lsgcpd_pose *init,
                                lsgcpd_pose *out, lsgcpd_report *reports, double *nll_trace,
                                hipStream_t st) {
  const int backend = backend_of(p->flags);
  if (npairs > 1 && backend != lsg::kBackendScalar)
    return fail(ctx, LSGCPD_E_UNSUPPORTED, "batches use the default pair kernel only");
  const bool small = npairs == 1 && backend == lsg::kBackendScalar &&
                     !(p->flags & LSGCPD_BF16_CROSS) && N[0] * M[0] <= kDenseAutoPairs;
  lsg::BatchPlan pl =
      lsg::batch_plan(npairs, N, M, backend, (p->flags & LSGCPD_DENSE) || small ? 0 : 1,
                      items_for(ctx, npairs, N, M));
  pl.f3 = (p->flags & LSGCPD_BF16_CROSS) && pl.cull ? 1 : 0;
  const int lanes = npairs < kSetupLanes ? npairs : kSetupLanes;
  RETURN_IF(ensure_geometry(ctx, npairs, N, M, pl.targets, p->k, lanes));
  ENSURE(nrm, (size_t)pl.targets * 3 * sizeof(float));
  ENSURE(kap, (size_t)pl.targets * sizeof(float));
  ENSURE(alp, (size_t)pl.targets * sizeof(float));
  const int stride = p->max_iter > 0 ? p->max_iter : 1;
  ENSURE(trace, (size_t)npairs * stride * sizeof(double));
  if (pl.cull) ENSURE(xperm, (size_t)pl.sources * 3 * sizeof(float));
  bool any_phi_x = false;
  int64_t nmax = 1;
  for (int i = 0; i < npairs; ++i) {
    any_phi_x = any_phi_x || (phi_x && phi_x[i]);
    nmax = N[i] > nmax ? N[i] : nmax;
  }
  if (any_phi_x && pl.cull) {
    ENSURE(xphi, (size_t)pl.sources * sizeof(float));
    for (int q = 0; q < lanes; ++q)
      RETURN_IF(ensure(ctx, *lane_of(ctx, q, st).xidx, (size_t)nmax * sizeof(uint32_t)));
  }
  RETURN_IF(ensure_states(ctx, npairs));
  lsg::BatchDev bd;
  RETURN_IF(ensure_estep(ctx, pl));

  float *nrm = (float *)ctx->nrm.p, *kap = (float *)ctx->kap.p, *alp = (float *)ctx->alp.p;
  // The set-up kernels of a cloud are small and those of different pairs are
  // independent: pair i is set up on lane i % lanes, and the lanes overlap.
  lsgcpd_status status = fork_lanes(ctx, lanes, st);
  for (int i = 0; status == LSGCPD_OK && i < npairs; ++i)
    status = pair_geometry(ctx, lane_of(ctx, i % lanes, st), pl, i, X[i], Y[i],
                           phi_x ? phi_x[i] : nullptr, p, nrm, kap, alp);
  {
    const lsgcpd_status js = join_lanes(ctx, lanes, st);
    if (status == LSGCPD_OK) status = js;
  }
  RETURN_IF(status);
  RETURN_IF(upload_tables(ctx, pl, st, &bd));
  const int s2_auto = p->sigma2_init > 0.0 ? 0 : 1;
  for (int i = 0; i < npairs; ++i)
    fill_state(ctx->hstate + i, init ? init + i : nullptr, s2_auto ? 1.0 : p->sigma2_init,
               p->V > 0.0 ? p->V : 0.0, p->w0, p->eta, p->tol, p->newton_max, p->max_iter);
  HIPCHK(hipMemcpyAsync(ctx->dstate, ctx->hstate, (size_t)npairs * sizeof(DevState),
                        hipMemcpyHostToDevice, st));
  status = fork_lanes(ctx, lanes, st);
  for (int i = 0; status == LSGCPD_OK && i < npairs; ++i) {
    const int64_t yo = pl.slots[i].y_off;
    status = setup_problem(ctx, lane_of(ctx, i % lanes, st), ctx_mem(ctx), pl, i, Y[i],
                           nrm + 3 * yo, alp + yo, nullptr, phi_y ? phi_y[i] : nullptr, p->eta,
                           pl.cull ? (const uint32_t *)ctx->yperm.p + yo : nullptr, p->flags,
                           p->V > 0.0 ? 0 : 1, s2_auto);
  }
  {
    const lsgcpd_status js = join_lanes(ctx, lanes, st);
    if (status == LSGCPD_OK) status = js;
  }
  RETURN_IF(status);
  RETURN_IF(prof_reserve(ctx, p->max_iter));
  RETURN_IF(run_em(ctx, pl, bd, p->max_iter, stride, (p->flags & LSGCPD_GRAPH) != 0, st));
  const size_t ntr = (size_t)npairs * stride;
  if (ctx->htr_cap < ntr) {
    if (ctx->htr_pinned) (void)hipHostFree(ctx->htr_pinned);
    ctx->htr_pinned = nullptr;
    ctx->htr_cap = 0;
    if (hipHostMalloc((void **)&ctx->htr_pinned, ntr * sizeof(double), hipHostMallocDefault) !=
        hipSuccess) {
      ctx->htr_pinned = nullptr;
      (void)hipGetLastError();
      return fail(ctx, LSGCPD_E_NOMEM, "pinned trace of %zu doubles failed", ntr);
    }
    ctx->htr_cap = ntr;
  }
  HIPCHK(hipMemcpyAsync(ctx->hstate, ctx->dstate, (size_t)npairs * sizeof(DevState),
                        hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(ctx->htr_pinned, ctx->trace.p, ntr * sizeof(double),
                        hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  ctx->htrace.assign(ctx->htr_pinned, ctx->htr_pinned + ntr);
  int64_t evaluated = 0;
  for (int i = 0; i < npairs; ++i) {
    const DevState &s = ctx->hstate[i];
    evaluated += backend == lsg::kBackendScalar ? s.evaluated_pairs
                                                : M[i] * N[i] * (s.iter + s.converged);
  }
  RETURN_IF(prof_collect(ctx, evaluated));
  status = LSGCPD_OK;
  for (int i = 0; i < npairs; ++i) {
    const DevState &s = ctx->hstate[i];
    const int filled = s.iter + s.converged;
    const double *tr = ctx->htrace.data() + (size_t)i * stride;
    memcpy(out[i].R, s.R, sizeof out[i].R);
    memcpy(out[i].t, s.t, sizeof out[i].t);
    if (reports) {
      lsgcpd_report &r = reports[i];
      r.iters = s.iter;
      r.converged = s.converged;
      r.gn_fallbacks = s.gn_fallbacks;
      r.sigma2 = s.sigma2;
      r.V = s.V;
      r.nll_last = s.nll;
      r.nll_first = p->max_iter > 0 && filled > 0 ? tr[0] : s.nll;
      r.w0 = s.w0;
      r.n_used = N[i];
      r.m_used = M[i];
      r.bf16_steps = s.f3_steps;
      r.pad = 0;
    }
    if (i == 0 && nll_trace && p->max_iter > 0)
      memcpy(nll_trace, tr, (size_t)filled * sizeof(double));
    if (status == LSGCPD_OK && s.numeric_error)
      status = fail(ctx, LSGCPD_E_NUMERIC, "EM produced a non-finite pose or sigma^2 (pair %d)", i);
    if (status == LSGCPD_OK && !finite_pos(s.sigma2))
      status = fail(ctx, LSGCPD_E_NUMERIC, "sigma^2 is not finite (pair %d)", i);
  }
  return status;
}

// Argument checks of the E-step calls.
lsgcpd_status check_estep_args(lsgcpd_ctx *ctx, const float *X, int64_t N, const float *Y,
                               const float *normals, const float *alpha, int64_t M,
                               const float *w, double w0, double V, const lsgcpd_pose *g,
                               double sigma2, uint32_t flags, const lsgcpd_estep_out *out) {
  if (!X || !Y || !normals || !alpha || !g || !out)
    return fail(ctx, LSGCPD_E_INVALID, "NULL required argument");
  if (N < 1 || M < 1 || N > kMaxPoints || M > kMaxPoints)
    return fail(ctx, LSGCPD_E_INVALID, "M = %lld, N = %lld out of range", (long long)M,
                (long long)N);
  if (!w && !(w0 > 0.0 && w0 < 1.0)) return fail(ctx, LSGCPD_E_INVALID, "w0 must lie in (0, 1)");
  if (!finite_pos(sigma2)) return fail(ctx, LSGCPD_E_INVALID, "sigma2 must be finite and > 0");
  if (!isfinite(V)) return fail(ctx, LSGCPD_E_INVALID, "V must be finite");
  if (flags & ~kKnownFlags) return fail(ctx, LSGCPD_E_INVALID, "unknown flags 0x%x", flags);
  if ((flags & LSGCPD_PAIRS_LDS) && (flags & LSGCPD_PAIRS_MFMA))
    return fail(ctx, LSGCPD_E_INVALID, "LSGCPD_PAIRS_LDS and LSGCPD_PAIRS_MFMA exclude each other");
  if ((flags & LSGCPD_BF16_CROSS) &&
      (flags & (LSGCPD_PAIRS_LDS | LSGCPD_PAIRS_MFMA | LSGCPD_DENSE)))
    return fail(ctx, LSGCPD_E_INVALID,
                "LSGCPD_BF16_CROSS runs on the culled default plan (no LDS, MFMA or DENSE flag)");
  return check_pose(ctx, g);
}

// Host outputs of an E step from the state read back after it.
lsgcpd_status estep_results(lsgcpd_ctx *ctx, const DevState &s, lsgcpd_estep_out *out) {
  out->sigma2 = s.sigma2;
  out->gamma = s.gamma;
  out->V = s.V;
  out->sumP = s.stats[9];
  out->outlier_mass = s.stats[84];
  out->nll = s.nll;
  out->pd = s.pd;
  memcpy(out->stats, s.stats, sizeof out->stats);
  memcpy(out->grad, s.grad, sizeof out->grad);
  memcpy(out->hess, s.hess, sizeof out->hess);
  memcpy(out->pose_next.R, s.R_next, sizeof s.R_next);
  memcpy(out->pose_next.t, s.t_next, sizeof s.t_next);
  out->sigma2_next = s.sigma2_next;
  out->newton_iters = s.newton_iters;
  out->gn_fallbacks = s.gn_fallbacks;
  out->bf16_cross = s.f3_steps;
  out->pad = 0;
  if (s.numeric_error) return fail(ctx, LSGCPD_E_NUMERIC, "M step produced a non-finite result");
  return LSGCPD_OK;
}

}  // namespace


LSG_API int lsgcpd_abi_version(void) { return LSGCPD_ABI_VERSION; }

LSG_API const char *lsgcpd_status_string(lsgcpd_status s) {
  switch (s) {
    case LSGCPD_OK: return "LSGCPD_OK";
    case LSGCPD_E_INVALID: return "LSGCPD_E_INVALID";
    case LSGCPD_E_HIP: return "LSGCPD_E_HIP";
    case LSGCPD_E_NOMEM: return "LSGCPD_E_NOMEM";
    case LSGCPD_E_NUMERIC: return "LSGCPD_E_NUMERIC";
    case LSGCPD_E_UNSUPPORTED: return "LSGCPD_E_UNSUPPORTED";
  }
  return "unknown status";
}

LSG_API lsgcpd_status lsgcpd_ctx_create(int device, lsgcpd_ctx **out) {
  if (!out) return LSGCPD_E_INVALID;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) {
    (void)hipGetLastError();
    return LSGCPD_E_HIP;
  }
  lsgcpd_ctx *c = new lsgcpd_ctx();
  c->device = device;
  if (hipSetDevice(device) != hipSuccess || map_scratch(device, &c->scratch) != hipSuccess) {
    (void)hipGetLastError();
    delete c;
    return LSGCPD_E_HIP;
  }
  *out = c;
  return LSGCPD_OK;
}

LSG_API void lsgcpd_ctx_destroy(lsgcpd_ctx *c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  Buf *bufs[] = {&c->knn,   &c->rec,   &c->pts,        &c->boxes, &c->ftab, &c->ptab, &c->pws,
                 &c->pbatch, &c->pin, &c->plan,  &c->partial,
                 &c->blockstats, &c->colS, &c->mom_part, &c->mom, &c->nrm,  &c->kap,
                 &c->alp,   &c->trace, &c->order,      &c->xperm, &c->yperm, &c->ys4,
                 &c->tables, &c->states, &c->cfx, &c->cfy, &c->cfwork, &c->xphi,
                 &c->xidx,  &c->prior};
  for (Buf *b : bufs)
    if (b->p) (void)hipFree(b->p);
  for (lsgcpd_ctx::LaneBufs &l : c->lane)
    for (Buf *b : {&l.order, &l.knn, &l.mom_part, &l.mom, &l.prior, &l.xidx})
      if (b->p) (void)hipFree(b->p);
  for (hipStream_t s : c->lstream)
    if (s) (void)hipStreamDestroy(s);
  for (hipEvent_t e : c->ljoin)
    if (e) (void)hipEventDestroy(e);
  if (c->lfork) (void)hipEventDestroy(c->lfork);
  for (hipEvent_t e : c->events) (void)hipEventDestroy(e);
  if (c->hstate) (void)hipHostFree(c->hstate);
  if (c->hcount) (void)hipHostFree(c->hcount);
  if (c->htab_pinned) (void)hipHostFree(c->htab_pinned);
  if (c->htr_pinned) (void)hipHostFree(c->htr_pinned);
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  for (hipEvent_t e : c->gev)
    if (e) (void)hipEventDestroy(e);
  if (c->gstream) (void)hipStreamDestroy(c->gstream);
  delete c;
}

LSG_API const char *lsgcpd_last_error(const lsgcpd_ctx *c) { return c ? c->err.c_str() : ""; }

LSG_API void lsgcpd_params_default(lsgcpd_params *p) {
  if (!p) return;
  p->k = 10;
  p->alpha_max = 30.0;
  p->lambda = 0.2;
  p->w0 = 0.1;
  p->V = 0.0;
  p->max_iter = 50;
  p->tol = 0.0;
  p->sigma2_init = 0.0;
  p->newton_max = 20;
  p->flags = 0;
  p->eta = 0.0;
}

LSG_API lsgcpd_status lsgcpd_normals(lsgcpd_ctx *ctx, const float *Y, int64_t M, int32_t k,
                                     double alpha_max, double lambda, float *normals,
                                     float *kappa, float *alpha, lsgcpd_stream stream) {
  if (!ctx) return LSGCPD_E_INVALID;
  if (!Y || !normals || !alpha) return fail(ctx, LSGCPD_E_INVALID, "NULL array argument");
  if (M < 1 || M > kMaxPoints) return fail(ctx, LSGCPD_E_INVALID, "M = %lld out of range", (long long)M);
  if (k < 1 || k > 32 || k > M)
    return fail(ctx, LSGCPD_E_INVALID, "k = %d must satisfy 1 <= k <= min(M, 32)", k);
  if (!(alpha_max >= 0.0) || !isfinite(alpha_max))
    return fail(ctx, LSGCPD_E_INVALID, "alpha_max must be finite and >= 0");
  if (!finite_pos(lambda)) return fail(ctx, LSGCPD_E_INVALID, "lambda must be finite and > 0");
  RETURN_IF(set_device(ctx));
  hipStream_t st = (hipStream_t)stream;
  RETURN_IF(ensure_geometry(ctx, 1, nullptr, &M, M, k, 1));
  const Lane ln = lane_of(ctx, 0, st);
  RETURN_IF(sort_targets(ctx, ln, Y, M, 0));
  return normals_sorted(ctx, ln, Y, M, 0, k, alpha_max, lambda, normals, kappa, alpha);
}

LSG_API lsgcpd_status lsgcpd_estep(lsgcpd_ctx *ctx, const float *X, int64_t N, const float *Y,
                                   const float *normals, const float *alpha, int64_t M,
                                   const float *pi, const float *w, double w0, double V,
                                   const lsgcpd_pose *g, double sigma2, uint32_t flags,
                                   lsgcpd_estep_out *out, float *P, double *colstats,
                                   lsgcpd_stream stream) {
  if (!ctx) return LSGCPD_E_INVALID;
  RETURN_IF(check_estep_args(ctx, X, N, Y, normals, alpha, M, w, w0, V, g, sigma2, flags, out));
  RETURN_IF(set_device(ctx));
  hipStream_t st = (hipStream_t)stream;
  lsg::BatchPlan pl =
      lsg::batch_plan(1, &N, &M, backend_of(flags), (flags & LSGCPD_DENSE) ? 0 : 1,
                      items_for(ctx, 1, &N, &M));
  pl.f3 = (flags & LSGCPD_BF16_CROSS) && pl.cull ? 1 : 0;
  pl.slots[0].X = X;
  pl.slots[0].w = w;
  RETURN_IF(ensure_states(ctx, 1));
  RETURN_IF(ensure_estep(ctx, pl));
  ENSURE(colS, (size_t)N * sizeof(double));
  lsg::BatchDev bd;
  RETURN_IF(upload_tables(ctx, pl, st, &bd));
  fill_state(ctx->hstate, g, sigma2, V > 0.0 ? V : 0.0, w ? 0.5 : w0, 0.0, 0.0, 20, 1);
  HIPCHK(hipMemcpyAsync(ctx->dstate, ctx->hstate, sizeof(DevState), hipMemcpyHostToDevice, st));
  const EstepMem mem = ctx_mem(ctx);
  RETURN_IF(setup_problem(ctx, lane_of(ctx, 0, st), mem, pl, 0, Y, normals, alpha, pi, nullptr,
                          0.0, nullptr, flags, V > 0.0 ? 0 : 1, 0));
  RETURN_IF(prof_reserve(ctx, 1));
  RETURN_IF(run_estep(ctx, pl, bd, mem, (double *)ctx->colS.p, colstats, nullptr, 1, 0, st));
  if (P)
    HIPCHK(lsg::launch_dump_P(X, N, mem.rec, M, w, mem.state, (const double *)ctx->colS.p, P, st));
  HIPCHK(hipMemcpyAsync(ctx->hstate, ctx->dstate, sizeof(DevState), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  RETURN_IF(prof_collect(
      ctx, pl.backend == lsg::kBackendScalar ? ctx->hstate->evaluated_pairs : M * N));
  return estep_results(ctx, *ctx->hstate, out);
}

LSG_API lsgcpd_status lsgcpd_estep_noalloc(lsgcpd_ctx *ctx, const float *X, int64_t N,
                                           const float *Y, const float *normals,
                                           const float *alpha, int64_t M, const float *pi,
                                           const float *w, double w0, double V,
                                           const lsgcpd_pose *g, double sigma2, uint32_t flags,
                                           lsgcpd_estep_out *out, float *P, double *colstats,
                                           lsgcpd_stream stream) {
  if (!ctx) return LSGCPD_E_INVALID;
  RETURN_IF(check_estep_args(ctx, X, N, Y, normals, alpha, M, w, w0, V, g, sigma2, flags, out));
  if (flags & (LSGCPD_PAIRS_LDS | LSGCPD_PAIRS_MFMA))
    return fail(ctx, LSGCPD_E_UNSUPPORTED,
                "lsgcpd_estep_noalloc runs the default pair kernel only (no LDS or MFMA flag)");
  if (N > kNoAllocMaxPoints || M > kNoAllocMaxPoints)
    return fail(ctx, LSGCPD_E_UNSUPPORTED,
                "lsgcpd_estep_noalloc takes at most %lld points per cloud (M = %lld, N = %lld)",
                (long long)kNoAllocMaxPoints, (long long)M, (long long)N);
  char *base = (char *)ctx->scratch;
  if (!base) return fail(ctx, LSGCPD_E_HIP, "the static scratch array of the device is not mapped");
  RETURN_IF(set_device(ctx));
  hipStream_t st = (hipStream_t)stream;
  lsg::BatchPlan pl = lsg::batch_plan(1, &N, &M, lsg::kBackendScalar,
                                      (flags & LSGCPD_DENSE) ? 0 : 1, kNoAllocItems);
  pl.f3 = (flags & LSGCPD_BF16_CROSS) && pl.cull ? 1 : 0;
  pl.slots[0].X = X;
  pl.slots[0].w = w;
  // The scratch array, carved in call order (256-byte aligned regions).
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char *q = base + off;
    off += (bytes + 255) / 256 * 256;
    return (void *)q;
  };
  std::vector<char> tables;  // host copy of the plan's tables (a few KB)
  lsg::batch_tables_pack(pl, tables);
  EstepMem mem;
  mem.state = (DevState *)take(sizeof(DevState));
  void *dtab = take(tables.size());
  mem.rec = (lsg::TRec *)take((size_t)(M + 1) * sizeof(lsg::TRec));
  mem.pts = (lsg::TPt *)take((size_t)M * sizeof(lsg::TPt));
  mem.boxes = (lsg::TBox *)take((size_t)pl.tiles * sizeof(lsg::TBox));
  mem.ftab = pl.f3 ? take(lsg::f3_table_bytes(pl.tiles)) : nullptr;
  mem.plan = take(lsg::estep_plan_bytes(pl));
  mem.partial = (double *)take(lsg::estep_partial_bytes(pl));
  mem.blockstats = (double *)take((size_t)pl.fins * lsg::kStats * sizeof(double));
  mem.timed = false;
  double *colS = (double *)take((size_t)N * sizeof(double));
  Buf mom, mom_part;
  mom.cap = 48 * sizeof(double);
  mom.p = take(mom.cap);
  mom_part.cap = (size_t)lsg::moments_blocks(M > N ? M : N) * 10 * sizeof(double);
  mom_part.p = take(mom_part.cap);
  if (off > kScratchBytes)
    return fail(ctx, LSGCPD_E_UNSUPPORTED,
                "M = %lld, N = %lld need %zu bytes of scratch; lsgcpd_estep_noalloc has %zu",
                (long long)M, (long long)N, off, kScratchBytes);
  // pageable host sources: both copies complete before the synchronisation below
  HIPCHK(hipMemcpyAsync(dtab, tables.data(), tables.size(), hipMemcpyHostToDevice, st));
  const lsg::BatchDev bd = lsg::batch_tables_view(pl, dtab);
  DevState hs;
  fill_state(&hs, g, sigma2, V > 0.0 ? V : 0.0, w ? 0.5 : w0, 0.0, 0.0, 20, 1);
  HIPCHK(hipMemcpyAsync(mem.state, &hs, sizeof(DevState), hipMemcpyHostToDevice, st));
  const Lane ln = {st, nullptr, nullptr, &mom_part, &mom, nullptr, nullptr};
  RETURN_IF(setup_problem(ctx, ln, mem, pl, 0, Y, normals, alpha, pi, nullptr, 0.0, nullptr,
                          flags, V > 0.0 ? 0 : 1, 0));
  RETURN_IF(run_estep(ctx, pl, bd, mem, colS, colstats, nullptr, 1, 0, st));
  if (P) HIPCHK(lsg::launch_dump_P(X, N, mem.rec, M, w, mem.state, colS, P, st));
  HIPCHK(hipMemcpyAsync(&hs, mem.state, sizeof(DevState), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return estep_results(ctx, hs, out);
}

LSG_API lsgcpd_status lsgcpd_register(lsgcpd_ctx *ctx, const float *X, int64_t N, const float *Y,
                                      int64_t M, const lsgcpd_params *p, const lsgcpd_pose *init,
                                      lsgcpd_pose *out, lsgcpd_report *report, double *nll_trace,
                                      lsgcpd_stream stream) {
  if (!ctx) return LSGCPD_E_INVALID;
  if (!X || !Y || !p || !out) return fail(ctx, LSGCPD_E_INVALID, "NULL required argument");
  if (N < 1 || M < 1 || N > kMaxPoints || M > kMaxPoints)
    return fail(ctx, LSGCPD_E_INVALID, "M = %lld, N = %lld out of range", (long long)M,
                (long long)N);
  if (p->k > M)
    return fail(ctx, LSGCPD_E_INVALID, "k = %d must satisfy 1 <= k <= min(M, 32)", p->k);
  RETURN_IF(check_params(ctx, p));
  if (init) RETURN_IF(check_pose(ctx, init));
  RETURN_IF(set_device(ctx));
  return register_problems(ctx, 1, &X, &N, &Y, &M, nullptr, nullptr, p, init, out, report,
                           nll_trace, (hipStream_t)stream);
}

LSG_API lsgcpd_status lsgcpd_register_batch(lsgcpd_ctx *ctx, int32_t npairs,
                                            const float *const *X, const int64_t *N,
                                            const float *const *Y, const int64_t *M,
                                            const lsgcpd_params *p, const lsgcpd_pose *init,
                                            lsgcpd_pose *out, lsgcpd_report *reports,
                                            lsgcpd_stream stream) {
  if (!ctx) return LSGCPD_E_INVALID;
  if (!X || !N || !Y || !M || !p || !out)
    return fail(ctx, LSGCPD_E_INVALID, "NULL required argument");
  if (npairs < 1 || npairs > kMaxBatch)
    return fail(ctx, LSGCPD_E_INVALID, "npairs = %d out of range", npairs);
  RETURN_IF(check_params(ctx, p));
  int64_t total = 0;
  for (int i = 0; i < npairs; ++i) {
    if (!X[i] || !Y[i]) return fail(ctx, LSGCPD_E_INVALID, "NULL cloud of pair %d", i);
    if (N[i] < 1 || M[i] < 1 || N[i] > kMaxPoints || M[i] > kMaxPoints)
      return fail(ctx, LSGCPD_E_INVALID, "pair %d: M = %lld, N = %lld out of range", i,
                  (long long)M[i], (long long)N[i]);
    if (p->k > M[i])
      return fail(ctx, LSGCPD_E_INVALID, "pair %d: k = %d exceeds M = %lld", i, p->k,
                  (long long)M[i]);
    if (init) RETURN_IF(check_pose(ctx, init + i));
    total += N[i] + M[i];
  }
  if (total > kMaxPoints) return fail(ctx, LSGCPD_E_INVALID, "batch holds more than 2^27 points");
  RETURN_IF(set_device(ctx));
  return register_problems(ctx, npairs, X, N, Y, M, nullptr, nullptr, p, init, out, reports,
                           nullptr, (hipStream_t)stream);
}

LSG_API lsgcpd_status lsgcpd_depth_confidence(lsgcpd_ctx *ctx, const float *P, int64_t n,
                                              const double *coef, double e_min, float *phi,
                                              lsgcpd_stream stream) {
  if (!ctx) return LSGCPD_E_INVALID;
  if (!P || !coef || !phi) return fail(ctx, LSGCPD_E_INVALID, "NULL required argument");
  if (n < 1 || n > kMaxPoints) return fail(ctx, LSGCPD_E_INVALID, "n = %lld out of range", (long long)n);
  if (!finite_pos(e_min)) return fail(ctx, LSGCPD_E_INVALID, "e_min must be finite and > 0");
  for (int i = 0; i < 3; ++i)
    if (!isfinite(coef[i])) return fail(ctx, LSGCPD_E_INVALID, "error model coefficients must be finite");
  RETURN_IF(set_device(ctx));
  HIPCHK(lsg::launch_depth_confidence(P, n, coef, e_min, phi, (hipStream_t)stream));
  return LSGCPD_OK;
}

LSG_API lsgcpd_status lsgcpd_register_cf(lsgcpd_ctx *ctx, const float *X, const float *phi_x,
                                         int64_t N, const float *Y, const float *phi_y, int64_t M,
                                         double threshold, const lsgcpd_params *p,
                                         const lsgcpd_pose *init, lsgcpd_pose *out,
                                         lsgcpd_report *report, double *nll_trace,
                                         lsgcpd_stream stream) {
  if (!ctx) return LSGCPD_E_INVALID;
  if (!X || !Y || !p || !out) return fail(ctx, LSGCPD_E_INVALID, "NULL required argument");
  if (N < 1 || M < 1 || N > kMaxPoints || M > kMaxPoints)
    return fail(ctx, LSGCPD_E_INVALID, "M = %lld, N = %lld out of range", (long long)M,
                (long long)N);
  if (!isfinite(threshold)) return fail(ctx, LSGCPD_E_INVALID, "threshold must be finite");
  RETURN_IF(check_params(ctx, p));
  if (init) RETURN_IF(check_pose(ctx, init));
  RETURN_IF(set_device(ctx));
  hipStream_t st = (hipStream_t)stream;
  const float *Xu = X, *Yu = Y, *px = phi_x, *py = phi_y;
  int64_t Nu = N, Mu = M;
  if (threshold > 0.0 && (phi_x || phi_y)) {
    // Sec. 3.3: drop the points whose confidence is below the threshold
    if (!ctx->hcount && hipHostMalloc((void **)&ctx->hcount, 2 * sizeof(uint32_t),
                                      hipHostMallocDefault) != hipSuccess) {
      ctx->hcount = nullptr;
      (void)hipGetLastError();
      return fail(ctx, LSGCPD_E_NOMEM, "pinned count allocation failed");
    }
    const size_t wx = lsg::select_workspace_bytes(N), wy = lsg::select_workspace_bytes(M);
    ENSURE(cfwork, (wx > wy ? wx : wy) + 256);
    uint32_t *dcount = (uint32_t *)((char *)ctx->cfwork.p + ctx->cfwork.cap - 256);
    const size_t wbytes = ctx->cfwork.cap - 256;
    if (phi_x) {
      ENSURE(cfx, (size_t)N * 4 * sizeof(float));
      float *xs = (float *)ctx->cfx.p;
      HIPCHK(lsg::launch_select_confident(X, phi_x, N, threshold, ctx->cfwork.p, wbytes, xs,
                                          xs + 3 * N, dcount, st));
      HIPCHK(hipMemcpyAsync(ctx->hcount, dcount, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    }
    if (phi_y) {
      ENSURE(cfy, (size_t)M * 4 * sizeof(float));
      float *ys = (float *)ctx->cfy.p;
      HIPCHK(lsg::launch_select_confident(Y, phi_y, M, threshold, ctx->cfwork.p, wbytes, ys,
                                          ys + 3 * M, dcount + 1, st));
      HIPCHK(hipMemcpyAsync(ctx->hcount + 1, dcount + 1, sizeof(uint32_t),
                            hipMemcpyDeviceToHost, st));
    }
    HIPCHK(hipStreamSynchronize(st));
    if (phi_x) {
      Nu = ctx->hcount[0];
      Xu = (const float *)ctx->cfx.p;
      px = Xu + 3 * N;
    }
    if (phi_y) {
      Mu = ctx->hcount[1];
      Yu = (const float *)ctx->cfy.p;
      py = Yu + 3 * M;
    }
    if (Nu < 1 || Mu < 1)
      return fail(ctx, LSGCPD_E_INVALID, "no point of %s has confidence >= %g",
                  Nu < 1 ? "X" : "Y", threshold);
  }
  if (p->k > Mu)
    return fail(ctx, LSGCPD_E_INVALID, "k = %d exceeds the %lld target points kept", p->k,
                (long long)Mu);
  return register_problems(ctx, 1, &Xu, &Nu, &Yu, &Mu, &px, &py, p, init, out, report,
                           nll_trace, st);
}

LSG_API lsgcpd_status lsgcpd_autotune(lsgcpd_ctx *ctx, const float *X, int64_t N,
                                      const float *Y, int64_t M, const lsgcpd_params *p,
                                      int32_t *items_out, lsgcpd_stream stream) {
  if (!ctx) return LSGCPD_E_INVALID;
  if (!X || !Y || !p) return fail(ctx, LSGCPD_E_INVALID, "NULL required argument");
  if (N < 1 || M < 1 || N > kMaxPoints || M > kMaxPoints)
    return fail(ctx, LSGCPD_E_INVALID, "M = %lld, N = %lld out of range", (long long)M,
                (long long)N);
  if (p->k > M)
    return fail(ctx, LSGCPD_E_INVALID, "k = %d must satisfy 1 <= k <= min(M, 32)", p->k);
  RETURN_IF(check_params(ctx, p));
  RETURN_IF(set_device(ctx));
  hipStream_t st = (hipStream_t)stream;
  static const int kCandidates[] = {1024, 2048, 4096, 8192, 16384, 32768};
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(ctx, LSGCPD_E_HIP, "hipEventCreate failed");
  }
  const bool prof = ctx->prof;
  ctx->prof = false;
  lsgcpd_status status = LSGCPD_OK;
  int best = 0;
  float best_ms = 0.f;
  for (int c : kCandidates) {
    ctx->forced_items = c;
    float ms = 0.f;
    for (int rep = 0; rep < 2 && status == LSGCPD_OK; ++rep) {  // the first warms up
      lsgcpd_pose out;
      float t = 0.f;
      if (hipEventRecord(e0, st) != hipSuccess) status = fail(ctx, LSGCPD_E_HIP, "hipEventRecord failed");
      if (status == LSGCPD_OK)
        status = register_problems(ctx, 1, &X, &N, &Y, &M, nullptr, nullptr, p, nullptr, &out,
                                   nullptr, nullptr, st);
      if (status == LSGCPD_OK && (hipEventRecord(e1, st) != hipSuccess ||
                                  hipEventSynchronize(e1) != hipSuccess ||
                                  hipEventElapsedTime(&t, e0, e1) != hipSuccess))
        status = fail(ctx, LSGCPD_E_HIP, "event timing failed");
      ms = t;
    }
    if (status != LSGCPD_OK) break;
    if (best == 0 || ms < best_ms) {
      best = c;
      best_ms = ms;
    }
  }
  ctx->forced_items = 0;
  ctx->prof = prof;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (status != LSGCPD_OK) return status;
  ctx->tuned_items[size_class(1, &N, &M)] = best;
  if (items_out) *items_out = best;
  return LSGCPD_OK;
}

LSG_API lsgcpd_status lsgcpd_profile_enable(lsgcpd_ctx *ctx, int on) {
  if (!ctx) return LSGCPD_E_INVALID;
  ctx->prof = on != 0;
  ctx->ev_used = 0;
  ctx->prof_pairs_pending = 0;
  return LSGCPD_OK;
}

LSG_API lsgcpd_status lsgcpd_profile_read(lsgcpd_ctx *ctx, lsgcpd_profile *out, int reset) {
  if (!ctx) return LSGCPD_E_INVALID;
  if (out) *out = ctx->totals;
  if (reset) {
    ctx->totals = lsgcpd_profile{0, 0, 0.0, 0.0, 0};
    ctx->launch_pair_us.clear();
    ctx->launch_estep_us.clear();
  }
  return LSGCPD_OK;
}

LSG_API lsgcpd_status lsgcpd_profile_launches(lsgcpd_ctx *ctx, double *pair_us, double *estep_us,
                                              int64_t cap, int64_t *count) {
  if (!ctx) return LSGCPD_E_INVALID;
  if (cap < 0 || (cap > 0 && (!pair_us || !estep_us)))
    return fail(ctx, LSGCPD_E_INVALID, "NULL output arrays");
  const int64_t n = (int64_t)ctx->launch_pair_us.size();
  const int64_t k = n < cap ? n : cap;
  for (int64_t i = 0; i < k; ++i) {
    pair_us[i] = ctx->launch_pair_us[i];
    estep_us[i] = ctx->launch_estep_us[i];
  }
  if (count) *count = n;
  return LSGCPD_OK;
}

// ---------------------------------------------------- pose proposal (f2)

namespace {

lsgcpd_status check_prop(lsgcpd_ctx *ctx, int npairs, int P) {
  if (npairs < 1 || npairs > kMaxBatch)
    return fail(ctx, LSGCPD_E_INVALID, "npairs = %d out of range", npairs);
  if (P < 1 || P > lsg::kPropMaxPoints)
    return fail(ctx, LSGCPD_E_INVALID, "P = %d must lie in [1, %d]", P, lsg::kPropMaxPoints);
  return LSGCPD_OK;
}

}  // namespace

LSG_API lsgcpd_status lsgcpd_proposal_inputs(lsgcpd_ctx *ctx, int32_t npairs,
                                             const float *const *X, const int64_t *N,
                                             const float *const *Y, const int64_t *M,
                                             const double *Q, int32_t P, float *Xn, float *Yn,
                                             double *norm, lsgcpd_stream stream) {
  if (!ctx) return LSGCPD_E_INVALID;
  if (!X || !N || !Y || !M || !Xn || !Yn || !norm)
    return fail(ctx, LSGCPD_E_INVALID, "NULL required argument");
  RETURN_IF(check_prop(ctx, npairs, P));
  std::vector<lsg::PropPair> pairs((size_t)npairs);
  for (int i = 0; i < npairs; ++i) {
    if (!X[i] || !Y[i]) return fail(ctx, LSGCPD_E_INVALID, "pair %d: NULL cloud", i);
    if (N[i] < 1 || M[i] < 1 || N[i] > kMaxPoints || M[i] > kMaxPoints)
      return fail(ctx, LSGCPD_E_INVALID, "pair %d: M = %lld, N = %lld out of range", i,
                  (long long)M[i], (long long)N[i]);
    pairs[i] = {X[i], Y[i], N[i], M[i]};
  }
  RETURN_IF(set_device(ctx));
  hipStream_t st = (hipStream_t)stream;
  const size_t pb = pairs.size() * sizeof(lsg::PropPair), qb = Q ? (size_t)npairs * 9 * 8 : 0;
  ENSURE(ptab, pb + qb);
  // pageable sources: the call synchronises the stream before returning
  HIPCHK(hipMemcpyAsync(ctx->ptab.p, pairs.data(), pb, hipMemcpyHostToDevice, st));
  double *dq = nullptr;
  if (Q) {
    dq = (double *)((char *)ctx->ptab.p + pb);
    HIPCHK(hipMemcpyAsync(dq, Q, qb, hipMemcpyHostToDevice, st));
  }
  HIPCHK(lsg::launch_prop_inputs((const lsg::PropPair *)ctx->ptab.p, npairs, dq, P, Xn, Yn, norm,
                                 st));
  HIPCHK(hipStreamSynchronize(st));
  return LSGCPD_OK;
}

LSG_API lsgcpd_status lsgcpd_proposal_forward(lsgcpd_ctx *ctx, const float *theta, int32_t npairs,
                                              int32_t P, const float *Xn, const float *Yn,
                                              const double *norm, double *pose,
                                              lsgcpd_stream stream) {
  if (!ctx) return LSGCPD_E_INVALID;
  if (!theta || !Xn || !Yn || !norm || !pose)
    return fail(ctx, LSGCPD_E_INVALID, "NULL required argument");
  RETURN_IF(check_prop(ctx, npairs, P));
  RETURN_IF(set_device(ctx));
  ENSURE(pws, lsg::prop_workspace_bytes(npairs, 0));
  HIPCHK(lsg::launch_prop_forward(theta, npairs, P, Xn, Yn, norm, pose, ctx->pws.p,
                                  (hipStream_t)stream));
  return LSGCPD_OK;
}

LSG_API lsgcpd_status lsgcpd_proposal_train_step(lsgcpd_ctx *ctx, float *theta, float *m, float *v,
                                                 int32_t step, double lr, int32_t npairs,
                                                 int32_t P, const float *Xn, const float *Yn,
                                                 const double *norm, int32_t nstored,
                                                 const int32_t *index, const double *label,
                                                 double *loss, int32_t *argmax, float *grad,
                                                 lsgcpd_stream stream) {
  if (!ctx) return LSGCPD_E_INVALID;
  if (!theta || !m || !v || !Xn || !Yn || !norm || !label || !loss)
    return fail(ctx, LSGCPD_E_INVALID, "NULL required argument");
  RETURN_IF(check_prop(ctx, npairs, P));
  if (step < 1) return fail(ctx, LSGCPD_E_INVALID, "step = %d must be >= 1", step);
  if (!finite_pos(lr)) return fail(ctx, LSGCPD_E_INVALID, "lr must be finite and > 0");
  if (index) {
    for (int b = 0; b < npairs; ++b)
      if (index[b] < 0 || index[b] >= nstored)
        return fail(ctx, LSGCPD_E_INVALID, "index[%d] = %d not in [0, %d)", b, index[b], nstored);
  } else if (nstored < npairs) {
    return fail(ctx, LSGCPD_E_INVALID, "nstored = %d < npairs = %d", nstored, npairs);
  }
  RETURN_IF(set_device(ctx));
  hipStream_t st = (hipStream_t)stream;
  ENSURE(pws, lsg::prop_workspace_bytes(npairs, 1));
  // the batch description (host) in one device buffer: labels, indices
  const size_t lb = (size_t)npairs * 12 * 8, ib = index ? (size_t)npairs * 4 : 0;
  ENSURE(pbatch, lb + ib);
  char *base = (char *)ctx->pbatch.p;
  HIPCHK(hipMemcpyAsync(base, label, lb, hipMemcpyHostToDevice, st));
  if (index) HIPCHK(hipMemcpyAsync(base + lb, index, ib, hipMemcpyHostToDevice, st));
  HIPCHK(lsg::launch_prop_train(theta, m, v, step, lr, npairs, P, Xn, Yn, norm,
                                index ? (const int *)(base + lb) : nullptr, (const double *)base,
                                loss, argmax, grad, ctx->pws.p, st));
  // pageable sources: the call synchronises the stream before returning
  HIPCHK(hipStreamSynchronize(st));
  return LSGCPD_OK;
}

namespace {

// The 24 rotations of the cube (signed permutation matrices of determinant
// +1), row-major: the multi-start set of lsgcpd_register_proposed.
void cube_rotations(double (*G)[9]) {
  static const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
  int n = 0;
  for (const auto &pm : perm)
    for (int s = 0; s < 8; ++s) {
      double R[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
      for (int r = 0; r < 3; ++r) R[3 * r + pm[r]] = (s >> r) & 1 ? -1.0 : 1.0;
      const double det = R[0] * (R[4] * R[8] - R[5] * R[7]) - R[1] * (R[3] * R[8] - R[5] * R[6]) +
                         R[2] * (R[3] * R[7] - R[4] * R[6]);
      if (det > 0.0) memcpy(G[n++], R, sizeof R);
    }
}

}  // namespace

LSG_API lsgcpd_status lsgcpd_register_proposed(lsgcpd_ctx *ctx, int32_t npairs,
                                               const float *const *X, const int64_t *N,
                                               const float *const *Y, const int64_t *M,
                                               const lsgcpd_params *p, const float *theta,
                                               int32_t P, double accept, lsgcpd_pose *out,
                                               lsgcpd_report *reports, int32_t *fallback,
                                               lsgcpd_stream stream) {
  if (!ctx) return LSGCPD_E_INVALID;
  if (!X || !N || !Y || !M || !p || !theta || !out)
    return fail(ctx, LSGCPD_E_INVALID, "NULL required argument");
  RETURN_IF(check_prop(ctx, npairs, P));
  if (!(accept > 0.0) || !isfinite(accept))
    return fail(ctx, LSGCPD_E_INVALID, "accept must be finite and > 0");
  RETURN_IF(check_params(ctx, p));
  for (int i = 0; i < npairs; ++i) {
    if (!X[i] || !Y[i]) return fail(ctx, LSGCPD_E_INVALID, "pair %d: NULL cloud", i);
    if (N[i] < 1 || M[i] < 1 || N[i] > kMaxPoints || M[i] > kMaxPoints || p->k > M[i])
      return fail(ctx, LSGCPD_E_INVALID, "pair %d: M = %lld, N = %lld out of range", i,
                  (long long)M[i], (long long)N[i]);
  }
  RETURN_IF(set_device(ctx));
  hipStream_t st = (hipStream_t)stream;
  // 1. proposals
  constexpr int NS = lsg::kPropNorm;
  const size_t ni = (size_t)npairs * P * 3;
  ENSURE(pin, ni * 2 * sizeof(float) + (size_t)npairs * (NS + 12) * sizeof(double));
  float *Xn = (float *)ctx->pin.p, *Yn = Xn + ni;
  double *norm = (double *)(Yn + ni), *pose = norm + (size_t)npairs * NS;
  RETURN_IF(lsgcpd_proposal_inputs(ctx, npairs, X, N, Y, M, nullptr, P, Xn, Yn, norm, stream));
  RETURN_IF(lsgcpd_proposal_forward(ctx, theta, npairs, P, Xn, Yn, norm, pose, stream));
  std::vector<double> hp((size_t)npairs * (NS + 12));
  HIPCHK(hipMemcpyAsync(hp.data(), norm, hp.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  std::vector<lsgcpd_pose> init((size_t)npairs);
  for (int i = 0; i < npairs; ++i) {
    const double *q = hp.data() + (size_t)npairs * NS + 12 * (size_t)i;
    memcpy(init[i].R, q, sizeof init[i].R);
    memcpy(init[i].t, q + 9, sizeof init[i].t);
  }
  // 2. EM from the proposals, all pairs in one batch
  std::vector<lsgcpd_report> rep((size_t)npairs);
  {
    // a pair whose EM ends on a non-finite state is simply not accepted
    const lsgcpd_status s = register_problems(ctx, npairs, X, N, Y, M, nullptr, nullptr, p,
                                              init.data(), out, rep.data(), nullptr, st);
    if (s != LSGCPD_OK && s != LSGCPD_E_NUMERIC) return s;
  }
  // 3. acceptance: final sigma against the RMS radius of the target's samples
  auto accepted = [&](int i) {
    return isfinite(rep[i].sigma2) && sqrt(rep[i].sigma2) <= accept * hp[(size_t)NS * i + 6];
  };
  std::vector<int> rej;
  for (int i = 0; i < npairs; ++i) {
    if (fallback) fallback[i] = accepted(i) ? 0 : 1;
    if (!accepted(i)) rej.push_back(i);
  }
  // 4. starts in the pair's principal-axis frames, R = F_Y G F_X^T with G
  // first the 4 sign changes of the axes, then the other 20 rotations of the
  // cube (axis permutations), t aligning the sampled centroids; batches of
  // kFallbackPairs pairs (their live-tile lists stay within the culled
  // plan's limit).  The run with the lowest final NLL of Eq. 4 is kept, the
  // proposal's own run included; a pair accepted after the sign changes
  // does not take the other 20.
  constexpr size_t kFallbackPairs = 32;
  double G[24][9];
  cube_rotations(G);
  for (int stage = 0; stage < 2 && !rej.empty(); ++stage) {
    std::vector<int> ks;
    for (int k = 0; k < 24; ++k) {
      const bool diag = G[k][1] == 0.0 && G[k][2] == 0.0 && G[k][5] == 0.0;
      if (diag == (stage == 0)) ks.push_back(k);
    }
    const size_t nk = ks.size();
    for (size_t r0 = 0; r0 < rej.size(); r0 += kFallbackPairs) {
      const size_t nr = rej.size() - r0 < kFallbackPairs ? rej.size() - r0 : kFallbackPairs;
      const size_t nb = nr * nk;
      std::vector<const float *> xs(nb), ys(nb);
      std::vector<int64_t> ns(nb), ms(nb);
      std::vector<lsgcpd_pose> st0(nb), so(nb);
      std::vector<lsgcpd_report> sr(nb);
      for (size_t r = 0; r < nr; ++r) {
        const int i = rej[r0 + r];
        const double *nm = hp.data() + (size_t)NS * i, *FX = nm + 7, *FY = nm + 16;
        for (size_t kk = 0; kk < nk; ++kk) {
          const double *g = G[ks[kk]];
          const size_t j = r * nk + kk;
          xs[j] = X[i];
          ys[j] = Y[i];
          ns[j] = N[i];
          ms[j] = M[i];
          double T[9];
          for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
              T[3 * a + b] = FY[3 * a] * g[b] + FY[3 * a + 1] * g[3 + b] + FY[3 * a + 2] * g[6 + b];
          for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
              st0[j].R[3 * a + b] =
                  T[3 * a] * FX[3 * b] + T[3 * a + 1] * FX[3 * b + 1] + T[3 * a + 2] * FX[3 * b + 2];
          for (int a = 0; a < 3; ++a)
            st0[j].t[a] = nm[3 + a] - (st0[j].R[3 * a] * nm[0] + st0[j].R[3 * a + 1] * nm[1] +
                                       st0[j].R[3 * a + 2] * nm[2]);
        }
      }
      const lsgcpd_status s = register_problems(ctx, (int)nb, xs.data(), ns.data(), ys.data(),
                                                ms.data(), nullptr, nullptr, p, st0.data(),
                                                so.data(), sr.data(), nullptr, st);
      if (s != LSGCPD_OK && s != LSGCPD_E_NUMERIC) return s;
      for (size_t r = 0; r < nr; ++r) {
        const int i = rej[r0 + r];
        for (size_t kk = 0; kk < nk; ++kk) {
          const size_t j = r * nk + kk;
          if (isfinite(sr[j].nll_last) && !(sr[j].nll_last >= rep[i].nll_last)) {
            out[i] = so[j];
            rep[i] = sr[j];
          }
        }
      }
    }
    std::vector<int> still;
    for (int i : rej)
      if (!accepted(i)) still.push_back(i);
    rej.swap(still);
  }
  if (reports) memcpy(reports, rep.data(), rep.size() * sizeof(lsgcpd_report));
  return LSGCPD_OK;
}
