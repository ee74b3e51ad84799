// Host side of liblsgcpd: argument validation, context workspace and the
// launch sequence of each public call (include/lsgcpd.h).
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <string>
#include <vector>

#include "lsgcpd.h"
#include "lsgcpd_internal.h"

#define LSG_API extern "C" __attribute__((visibility("default")))

using lsg::DevState;

namespace {

constexpr int64_t kMaxPoints = (int64_t)1 << 27;

struct Buf {
  void *p = nullptr;
  size_t cap = 0;
};

}  // namespace

struct lsgcpd_ctx {
  int device = 0;
  std::string err;
  Buf knn, rec, pts, boxes, plan, partial, blockstats, colS, mom_part, mom, nrm, kap, alp,
      trace, order, xperm, yperm, ys4;
  DevState *dstate = nullptr;  // device
  DevState *hstate = nullptr;  // pinned host staging
  // E-step timing: 4 events per E step (start, before and after the pair
  // kernel, end)
  bool prof = false;
  std::vector<hipEvent_t> events;
  int ev_used = 0;
  int64_t prof_pairs_pending = 0;
  lsgcpd_profile totals = {0, 0, 0.0, 0.0, 0};
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

#define ENSURE(buf, bytes)                                     \
  do {                                                         \
    lsgcpd_status s_ = ensure(ctx, ctx->buf, (size_t)(bytes)); \
    if (s_ != LSGCPD_OK) return s_;                            \
  } while (0)

bool finite_pos(double v) { return isfinite(v) && v > 0.0; }

constexpr uint32_t kKnownFlags =
    LSGCPD_EXACT_NORMALIZER | LSGCPD_PAIRS_LDS | LSGCPD_PAIRS_MFMA | LSGCPD_DENSE;

// About this many work items per E step for the scalar back end (the
// fastest measured on MI355X for the 20k x 20k and 100k x 50k workloads);
// LSGCPD_WORK_ITEMS overrides it for tuning sweeps.
int work_items() {
  const char *e = getenv("LSGCPD_WORK_ITEMS");
  const int v = e ? atoi(e) : 0;
  return v >= 64 && v <= (1 << 20) ? v : 8192;
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

lsgcpd_status set_device(lsgcpd_ctx *ctx) {
  HIPCHK(hipSetDevice(ctx->device));
  return LSGCPD_OK;
}

void fill_state(DevState *s, const lsgcpd_pose *g, double sigma2, double V, double w0,
                double tol, int newton_max, int max_iter) {
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
  s->tol = tol;
  s->newton_max = newton_max;
  s->max_iter = max_iter;
}

// Target records (record i describes target yperm[i], or target i if yperm is
// null) and their tile boxes + moments of Y, X at the state's pose + init_state.
lsgcpd_status setup(lsgcpd_ctx *ctx, const float *X, int64_t N, const float *Y,
                    const float *normals, const float *alpha, const float *pi,
                    const uint32_t *yperm, int64_t M, uint32_t flags, int v_auto, int s2_auto,
                    hipStream_t st) {
  ENSURE(rec, (size_t)(M + 1) * sizeof(lsg::TRec));  // + sentinel
  ENSURE(pts, (size_t)M * sizeof(lsg::TPt));
  ENSURE(boxes, (size_t)((M + lsg::kCullTile - 1) / lsg::kCullTile) * sizeof(lsg::TBox));
  const int nb = lsg::moments_blocks(N > M ? N : M);
  ENSURE(mom_part, (size_t)nb * 10 * sizeof(double));
  ENSURE(mom, 48 * sizeof(double));
  HIPCHK(hipMemcpyAsync(ctx->dstate, ctx->hstate, sizeof(DevState), hipMemcpyHostToDevice, st));
  HIPCHK(lsg::launch_prep_targets(Y, normals, alpha, pi, yperm, M,
                                  (flags & LSGCPD_EXACT_NORMALIZER) ? 1 : 0,
                                  (lsg::TRec *)ctx->rec.p, (lsg::TPt *)ctx->pts.p,
                                  (lsg::TBox *)ctx->boxes.p, st));
  double *ymom = (double *)ctx->mom.p;
  double *xmom = ymom + 16;
  HIPCHK(lsg::launch_moments(Y, M, nullptr, (double *)ctx->mom_part.p, lsg::moments_blocks(M),
                             ymom, st));
  if (s2_auto)
    HIPCHK(lsg::launch_moments(X, N, ctx->dstate, (double *)ctx->mom_part.p,
                               lsg::moments_blocks(N), xmom, st));
  HIPCHK(lsg::launch_init_state(ctx->dstate, ymom, xmom, M, N, v_auto, s2_auto, st));
  return LSGCPD_OK;
}

// Y in Morton order: ctx->ys4 (x, y, z, original index) and ctx->yperm.
lsgcpd_status sort_targets(lsgcpd_ctx *ctx, const float *Y, int64_t M, hipStream_t st) {
  const int nb = lsg::moments_blocks(M);
  ENSURE(mom_part, (size_t)nb * 10 * sizeof(double));
  ENSURE(mom, 48 * sizeof(double));
  ENSURE(order, lsg::morton_workspace_bytes(M));
  ENSURE(yperm, (size_t)M * sizeof(uint32_t));
  ENSURE(ys4, (size_t)M * sizeof(float4));
  double *box = (double *)ctx->mom.p + 32;
  HIPCHK(lsg::launch_moments(Y, M, nullptr, (double *)ctx->mom_part.p, nb, box, st));
  HIPCHK(lsg::launch_morton_order(Y, M, box, ctx->order.p, ctx->order.cap, nullptr,
                                  (float4 *)ctx->ys4.p, (uint32_t *)ctx->yperm.p, st));
  return LSGCPD_OK;
}

lsgcpd_status normals_sorted(lsgcpd_ctx *ctx, const float *Y, int64_t M, int k, double alpha_max,
                             double lambda, float *normals, float *kappa, float *alpha,
                             hipStream_t st) {
  ENSURE(knn, lsg::knn_workspace_bytes(M, k));
  HIPCHK(lsg::launch_normals(Y, M, (const float4 *)ctx->ys4.p, (const uint32_t *)ctx->yperm.p, k,
                             alpha_max, lambda, normals, kappa, alpha, ctx->knn.p, st));
  return LSGCPD_OK;
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
    ctx->totals.launches += 1;
  }
  ctx->totals.pairs += ctx->prof_pairs_pending;
  ctx->prof_pairs_pending = 0;
  ctx->ev_used = 0;
  return LSGCPD_OK;
}

// One E step (accumulation, finalisation) + reduction/M step in `mode`.
lsgcpd_status run_estep(lsgcpd_ctx *ctx, const lsg::EstepPlan &pl, const float *X, int64_t N,
                        int64_t M, const float *w, double *colstats, double *trace, int mode,
                        hipStream_t st) {
  lsgcpd_status s = prof_record(ctx, st);
  if (s != LSGCPD_OK) return s;
  HIPCHK(lsg::launch_estep_plan(pl, X, N, (const lsg::TBox *)ctx->boxes.p, ctx->dstate,
                                ctx->plan.p, st));
  if ((s = prof_record(ctx, st)) != LSGCPD_OK) return s;
  HIPCHK(lsg::launch_estep_pairs(pl, X, N, (const lsg::TRec *)ctx->rec.p,
                                 (const lsg::TPt *)ctx->pts.p, M, ctx->dstate, ctx->plan.p,
                                 (double *)ctx->partial.p, st));
  if ((s = prof_record(ctx, st)) != LSGCPD_OK) return s;
  HIPCHK(lsg::launch_finalize(pl, X, N, w, ctx->dstate, ctx->plan.p,
                              (const double *)ctx->partial.p, (double *)ctx->blockstats.p,
                              (double *)ctx->colS.p, colstats, st));
  if ((s = prof_record(ctx, st)) != LSGCPD_OK) return s;
  if (ctx->prof) ctx->prof_pairs_pending += M * N;
  HIPCHK(lsg::launch_reduce_mstep((double *)ctx->blockstats.p, pl.nfin_blocks, N, ctx->dstate,
                                  trace, lsg::estep_plan_counter(pl, ctx->plan.p), mode, st));
  return LSGCPD_OK;
}

lsgcpd_status ensure_estep(lsgcpd_ctx *ctx, const lsg::EstepPlan &pl, int64_t N) {
  ENSURE(plan, lsg::estep_plan_bytes(pl));
  ENSURE(partial, lsg::estep_partial_bytes(pl, N));
  ENSURE(blockstats, (size_t)pl.nfin_blocks * lsg::kStats * sizeof(double));
  ENSURE(colS, (size_t)N * sizeof(double));
  return LSGCPD_OK;
}

}  // namespace

#define RETURN_IF(x)                \
  do {                              \
    lsgcpd_status s_ = (x);         \
    if (s_ != LSGCPD_OK) return s_; \
  } while (0)

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
  if (hipSetDevice(device) != hipSuccess ||
      hipMalloc((void **)&c->dstate, sizeof(DevState)) != hipSuccess ||
      hipHostMalloc((void **)&c->hstate, sizeof(DevState), hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    if (c->dstate) (void)hipFree(c->dstate);
    delete c;
    return LSGCPD_E_HIP;
  }
  *out = c;
  return LSGCPD_OK;
}

LSG_API void lsgcpd_ctx_destroy(lsgcpd_ctx *c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  Buf *bufs[] = {&c->knn,  &c->rec,      &c->pts, &c->boxes, &c->plan,  &c->partial,
                 &c->blockstats, &c->colS, &c->mom_part, &c->mom, &c->nrm, &c->kap,
                 &c->alp,  &c->trace,    &c->order, &c->xperm, &c->yperm, &c->ys4};
  for (Buf *b : bufs)
    if (b->p) (void)hipFree(b->p);
  for (hipEvent_t e : c->events) (void)hipEventDestroy(e);
  if (c->dstate) (void)hipFree(c->dstate);
  if (c->hstate) (void)hipHostFree(c->hstate);
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
  RETURN_IF(sort_targets(ctx, Y, M, st));
  return normals_sorted(ctx, Y, M, k, alpha_max, lambda, normals, kappa, alpha, st);
}

LSG_API lsgcpd_status lsgcpd_estep(lsgcpd_ctx *ctx, const float *X, int64_t N, const float *Y,
                                   const float *normals, const float *alpha, int64_t M,
                                   const float *pi, const float *w, double w0, double V,
                                   const lsgcpd_pose *g, double sigma2, uint32_t flags,
                                   lsgcpd_estep_out *out, float *P, double *colstats,
                                   lsgcpd_stream stream) {
  if (!ctx) return LSGCPD_E_INVALID;
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
  RETURN_IF(check_pose(ctx, g));
  RETURN_IF(set_device(ctx));
  hipStream_t st = (hipStream_t)stream;
  const lsg::EstepPlan pl =
      lsg::estep_plan(N, M, backend_of(flags), (flags & LSGCPD_DENSE) ? 0 : 1, work_items());
  RETURN_IF(ensure_estep(ctx, pl, N));
  fill_state(ctx->hstate, g, sigma2, V > 0.0 ? V : 0.0, w ? 0.5 : w0, 0.0, 20, 1);
  RETURN_IF(
      setup(ctx, X, N, Y, normals, alpha, pi, nullptr, M, flags, V > 0.0 ? 0 : 1, 0, st));
  RETURN_IF(prof_reserve(ctx, 1));
  RETURN_IF(run_estep(ctx, pl, X, N, M, w, colstats, nullptr, 0, st));
  if (P)
    HIPCHK(lsg::launch_dump_P(X, N, (const lsg::TRec *)ctx->rec.p, M, w, ctx->dstate,
                              (const double *)ctx->colS.p, P, st));
  HIPCHK(hipMemcpyAsync(ctx->hstate, ctx->dstate, sizeof(DevState), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  RETURN_IF(prof_collect(
      ctx, pl.backend == lsg::kBackendScalar ? ctx->hstate->evaluated_pairs : M * N));
  const DevState &s = *ctx->hstate;
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
  if (s.numeric_error) return fail(ctx, LSGCPD_E_NUMERIC, "M step produced a non-finite result");
  return LSGCPD_OK;
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
  if (p->k < 1 || p->k > 32 || p->k > M)
    return fail(ctx, LSGCPD_E_INVALID, "k = %d must satisfy 1 <= k <= min(M, 32)", p->k);
  if (!(p->alpha_max >= 0.0) || !isfinite(p->alpha_max))
    return fail(ctx, LSGCPD_E_INVALID, "alpha_max must be finite and >= 0");
  if (!finite_pos(p->lambda)) return fail(ctx, LSGCPD_E_INVALID, "lambda must be finite and > 0");
  if (!(p->w0 > 0.0 && p->w0 < 1.0)) return fail(ctx, LSGCPD_E_INVALID, "w0 must lie in (0, 1)");
  if (!isfinite(p->V) || !isfinite(p->tol) || !isfinite(p->sigma2_init))
    return fail(ctx, LSGCPD_E_INVALID, "V, tol and sigma2_init must be finite");
  if (p->max_iter < 0 || p->max_iter > 100000)
    return fail(ctx, LSGCPD_E_INVALID, "max_iter = %d out of range", p->max_iter);
  if (p->newton_max < 1 || p->newton_max > 1000)
    return fail(ctx, LSGCPD_E_INVALID, "newton_max = %d out of range", p->newton_max);
  if (p->flags & ~kKnownFlags) return fail(ctx, LSGCPD_E_INVALID, "unknown flags 0x%x", p->flags);
  if ((p->flags & LSGCPD_PAIRS_LDS) && (p->flags & LSGCPD_PAIRS_MFMA))
    return fail(ctx, LSGCPD_E_INVALID, "LSGCPD_PAIRS_LDS and LSGCPD_PAIRS_MFMA exclude each other");
  if (init) RETURN_IF(check_pose(ctx, init));
  RETURN_IF(set_device(ctx));
  hipStream_t st = (hipStream_t)stream;

  // target geometry: neighbours over Y in Morton order (the sort workspace is
  // sized for both clouds up front, so it is not reallocated while in use)
  ENSURE(order, lsg::morton_workspace_bytes(N > M ? N : M));
  ENSURE(mom_part, (size_t)lsg::moments_blocks(N > M ? N : M) * 10 * sizeof(double));
  ENSURE(nrm, (size_t)M * 3 * sizeof(float));
  ENSURE(kap, (size_t)M * sizeof(float));
  ENSURE(alp, (size_t)M * sizeof(float));
  RETURN_IF(sort_targets(ctx, Y, M, st));
  RETURN_IF(normals_sorted(ctx, Y, M, p->k, p->alpha_max, p->lambda, (float *)ctx->nrm.p,
                           (float *)ctx->kap.p, (float *)ctx->alp.p, st));

  const lsg::EstepPlan pl =
      lsg::estep_plan(N, M, backend_of(p->flags), (p->flags & LSGCPD_DENSE) ? 0 : 1, work_items());
  RETURN_IF(ensure_estep(ctx, pl, N));
  // With culling the target records follow the Morton order of Y and the
  // sources are put in Morton order too, so that a source group's and a target
  // tile's points are neighbours.  Every statistic is a sum over all sources
  // and all targets, so the order changes only the rounding of the sums.
  const uint32_t *yperm = nullptr;
  if (pl.backend == lsg::kBackendScalar && pl.cull && N > 256) {
    ENSURE(xperm, (size_t)N * 3 * sizeof(float));
    double *xbox = (double *)ctx->mom.p + 32;
    HIPCHK(lsg::launch_moments(X, N, nullptr, (double *)ctx->mom_part.p, lsg::moments_blocks(N),
                               xbox, st));
    HIPCHK(lsg::launch_morton_order(X, N, xbox, ctx->order.p, ctx->order.cap,
                                    (float *)ctx->xperm.p, nullptr, nullptr, st));
    X = (const float *)ctx->xperm.p;
    yperm = (const uint32_t *)ctx->yperm.p;
  }
  ENSURE(trace, (size_t)(p->max_iter > 0 ? p->max_iter : 1) * sizeof(double));
  const int s2_auto = p->sigma2_init > 0.0 ? 0 : 1;
  fill_state(ctx->hstate, init, s2_auto ? 1.0 : p->sigma2_init, p->V > 0.0 ? p->V : 0.0, p->w0,
             p->tol, p->newton_max, p->max_iter);
  RETURN_IF(setup(ctx, X, N, Y, (const float *)ctx->nrm.p, (const float *)ctx->alp.p, nullptr,
                  yperm, M, p->flags, p->V > 0.0 ? 0 : 1, s2_auto, st));
  RETURN_IF(prof_reserve(ctx, p->max_iter));
  for (int it = 0; it < p->max_iter; ++it)
    RETURN_IF(run_estep(ctx, pl, X, N, M, nullptr, nullptr, (double *)ctx->trace.p, 1, st));
  HIPCHK(hipMemcpyAsync(ctx->hstate, ctx->dstate, sizeof(DevState), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  RETURN_IF(prof_collect(ctx, pl.backend == lsg::kBackendScalar
                                  ? ctx->hstate->evaluated_pairs
                                  : M * N * (ctx->hstate->iter + ctx->hstate->converged)));
  double first = ctx->hstate->nll;
  if (p->max_iter > 0 && ctx->hstate->iter + ctx->hstate->converged > 0) {
    HIPCHK(hipMemcpy(&first, ctx->trace.p, sizeof(double), hipMemcpyDeviceToHost));
    const int filled = ctx->hstate->iter + ctx->hstate->converged;
    if (nll_trace)
      HIPCHK(hipMemcpy(nll_trace, ctx->trace.p, (size_t)filled * sizeof(double),
                       hipMemcpyDeviceToHost));
  }
  const DevState &s = *ctx->hstate;
  memcpy(out->R, s.R, sizeof out->R);
  memcpy(out->t, s.t, sizeof out->t);
  if (report) {
    report->iters = s.iter;
    report->converged = s.converged;
    report->gn_fallbacks = s.gn_fallbacks;
    report->sigma2 = s.sigma2;
    report->V = s.V;
    report->nll_last = s.nll;
    report->nll_first = first;
  }
  if (s.numeric_error) return fail(ctx, LSGCPD_E_NUMERIC, "EM produced a non-finite pose or sigma^2");
  if (!finite_pos(s.sigma2)) return fail(ctx, LSGCPD_E_NUMERIC, "sigma^2 is not finite");
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
  if (reset) ctx->totals = lsgcpd_profile{0, 0, 0.0, 0.0, 0};
  return LSGCPD_OK;
}
