// The LSG-CPD E step on gfx950 (Sec. 3.1 Eq. 5, Sec. 3.4 Eq. 9-10).
//
// For every (target m, source n) pair the kernels evaluate
//   K_mn / rho_n = 2^( l_m - d_mn * log2(e) / (2 sigma^2) ),
//   d_mn = |r|^2 + (a_m . r)^2,  r = g(x_n) - y_m,  a_m = sqrt(alpha_m) n_m,
// which is the Mahalanobis form of Eq. 2 times sigma^2, and accumulate, for each
// source, the unnormalised sums  T_n[c] = sum_m (K_mn / rho_n) f_m[c]  of the 11
// target features f_m = [1, alpha n n^T, M_m y_m, y_m^T M_m y_m].  The
// posterior normaliser of Eq. 9 is per source (a column of P), so one pass over
// the pairs suffices: P_mn = rho_n e_mn / (rho_n T_n[0] + gamma), and every
// P-weighted sum is rho_n T_n[c] / (rho_n T_n[0] + gamma).  The M x N posterior
// is never stored.
//
// Precision: g(x_n) is formed in FP64 and split into float32 hi + lo; the
// residual is (hi - y) + lo, so its error is a few ulp of |r| rather than of
// |g(x)|.  Residual, exponent and exp2 are float32; the products e * f_m and
// all sums are FP64 (features are exact FP64 functions of the float32 inputs).
//
// Two accumulation back ends with identical arithmetic up to summation order:
//  * estep_mfma: V_MFMA_F64_16X16X4 -- a wave multiplies the 16(sources) x 4
//    (targets) block of exponentials by the 4 x 16 block of target features,
//    so the FP64 accumulation runs on the matrix cores while the vector ALU
//    computes the next exponentials.
//  * estep_valu: plain FP64 FMAs on the vector ALU.
// Both stream targets through LDS in tiles and keep source points in
// registers.  Target chunks (split-M) give enough blocks for small N; the
// per-chunk partial sums are combined in a fixed order by estep_finalize.
#include <math.h>

#include "lsgcpd_internal.h"

namespace lsg {

namespace {

constexpr double kLog2e = 1.4426950408889634074;
constexpr double kTwoPi = 6.283185307179586477;
constexpr int kBlock = 256;
constexpr int kTile = 128;           // targets per LDS tile
constexpr int kValuS = 2;            // sources per thread in estep_valu

__device__ __forceinline__ double gamma_of(const DevState *s) {
  return pow(kTwoPi * s->sigma2, 1.5) / s->V;
}

// Transformed source point split into hi + lo float32 parts.
struct Src {
  float h0, h1, h2, l0, l1, l2;
};

__device__ __forceinline__ Src load_src(const float *__restrict__ X, int n, int N,
                                        const double *R, const double *t) {
  Src o;
  double x = 0.0, y = 0.0, z = 0.0;
  if (n < N) {
    x = X[3 * n];
    y = X[3 * n + 1];
    z = X[3 * n + 2];
  }
  const double p0 = fma(R[0], x, fma(R[1], y, fma(R[2], z, t[0])));
  const double p1 = fma(R[3], x, fma(R[4], y, fma(R[5], z, t[1])));
  const double p2 = fma(R[6], x, fma(R[7], y, fma(R[8], z, t[2])));
  o.h0 = (float)p0;
  o.h1 = (float)p1;
  o.h2 = (float)p2;
  o.l0 = (float)(p0 - (double)o.h0);
  o.l1 = (float)(p1 - (double)o.h1);
  o.l2 = (float)(p2 - (double)o.h2);
  return o;
}

// e = K_mn / rho_n for one pair.  g0 = (y, l), g1 = (a, 0).  Every operation is
// written out so that the P-dump kernel reproduces the same float32 value.
__device__ __forceinline__ float pair_exp(const Src &x, const float4 g0, const float4 g1,
                                          float negc) {
  const float r0 = (x.h0 - g0.x) + x.l0;
  const float r1 = (x.h1 - g0.y) + x.l1;
  const float r2 = (x.h2 - g0.z) + x.l2;
  const float q = __builtin_fmaf(r2, r2, __builtin_fmaf(r1, r1, r0 * r0));
  const float p = __builtin_fmaf(g1.z, r2, __builtin_fmaf(g1.y, r1, g1.x * r0));
  const float d = __builtin_fmaf(p, p, q);
  return __builtin_amdgcn_exp2f(__builtin_fmaf(d, negc, g0.w));
}

__device__ __forceinline__ float neg_c_of(const DevState *s) {
  return (float)(-kLog2e / (2.0 * s->sigma2));
}

// Cooperative load of one tile of target records into LDS; slots past the end
// get l = -inf (e = 0) and zero features.
template <int NF>
__device__ __forceinline__ void load_tile(const float4 *__restrict__ geo,
                                          const double *__restrict__ feat, int64_t mt, int cnt,
                                          float4 *sg, double *sf) {
  for (int i = threadIdx.x; i < 2 * kTile; i += kBlock) {
    const int j = i >> 1;
    float4 v;
    if (j < cnt)
      v = geo[2 * (mt + j) + (i & 1)];
    else
      v = (i & 1) ? make_float4(0.f, 0.f, 0.f, 0.f) : make_float4(0.f, 0.f, 0.f, -INFINITY);
    sg[i] = v;
  }
  for (int i = threadIdx.x; i < NF * kTile; i += kBlock) {
    const int j = i / NF;
    const int c = i - j * NF;
    sf[i] = j < cnt ? feat[(mt + j) * kFeat + c] : 0.0;
  }
}

// ---------------------------------------------------------------- VALU path
template <int S>
__global__ __launch_bounds__(kBlock) void estep_valu(const float *__restrict__ X, int N,
                                                     const float4 *__restrict__ geo,
                                                     const double *__restrict__ feat, int64_t M,
                                                     const DevState *__restrict__ st,
                                                     int64_t mchunk, int nsplit,
                                                     double *__restrict__ partial) {
  if (st->done) return;
  const int split = blockIdx.x % nsplit;
  const int sb = blockIdx.x / nsplit;
  const int64_t m0 = (int64_t)split * mchunk;
  const int64_t m1 = m0 + mchunk < M ? m0 + mchunk : M;
  double R[9], t[3];
  for (int i = 0; i < 9; ++i) R[i] = st->R[i];
  for (int i = 0; i < 3; ++i) t[i] = st->t[i];
  const float negc = neg_c_of(st);
  Src x[S];
  int nidx[S];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    nidx[s] = sb * kBlock * S + s * kBlock + threadIdx.x;
    x[s] = load_src(X, nidx[s], N, R, t);
  }
  double acc[S][kFeatUsed];
#pragma unroll
  for (int s = 0; s < S; ++s)
#pragma unroll
    for (int c = 0; c < kFeatUsed; ++c) acc[s][c] = 0.0;
  __shared__ float4 sg[2 * kTile];
  __shared__ double sf[kFeatUsed * kTile];
  for (int64_t mt = m0; mt < m1; mt += kTile) {
    const int cnt = (int)(m1 - mt < kTile ? m1 - mt : kTile);
    __syncthreads();
    load_tile<kFeatUsed>(geo, feat, mt, cnt, sg, sf);
    __syncthreads();
    for (int j = 0; j < cnt; ++j) {
      const float4 g0 = sg[2 * j];
      const float4 g1 = sg[2 * j + 1];
      double f[kFeatUsed];
#pragma unroll
      for (int c = 1; c < kFeatUsed; ++c) f[c] = sf[kFeatUsed * j + c];
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const double e = (double)pair_exp(x[s], g0, g1, negc);
        acc[s][0] += e;
#pragma unroll
        for (int c = 1; c < kFeatUsed; ++c) acc[s][c] = fma(e, f[c], acc[s][c]);
      }
    }
  }
#pragma unroll
  for (int s = 0; s < S; ++s) {
    if (nidx[s] < N) {
#pragma unroll
      for (int c = 0; c < kFeatUsed; ++c)
        partial[((size_t)split * kFeatUsed + c) * N + nidx[s]] = acc[s][c];
    }
  }
}

// ---------------------------------------------------------------- MFMA path
// Wave layout: lane l, r = l % 16 (row in a 16-source group), kq = l / 16
// (target slot).  Each wave owns 64 sources (4 groups of 16).  Per step of 4
// targets, lane l computes e(source 16j + r, target 4s + kq) for j = 0..3 --
// exactly the A operand (16 x 4) element it must supply -- and reads feature r
// of target 4s + kq as its B operand (4 x 16) element.
typedef double d4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(kBlock) void estep_mfma(const float *__restrict__ X, int N,
                                                    const float4 *__restrict__ geo,
                                                    const double *__restrict__ feat, int64_t M,
                                                    const DevState *__restrict__ st,
                                                    int64_t mchunk, int nsplit,
                                                    double *__restrict__ partial) {
  if (st->done) return;
  const int split = blockIdx.x % nsplit;
  const int sb = blockIdx.x / nsplit;
  const int64_t m0 = (int64_t)split * mchunk;
  const int64_t m1 = m0 + mchunk < M ? m0 + mchunk : M;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int r = lane & 15;
  const int kq = lane >> 4;
  const int wbase = sb * kBlock + wave * 64;
  double R[9], t[3];
  for (int i = 0; i < 9; ++i) R[i] = st->R[i];
  for (int i = 0; i < 3; ++i) t[i] = st->t[i];
  const float negc = neg_c_of(st);
  Src x[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) x[j] = load_src(X, wbase + 16 * j + r, N, R, t);
  d4 acc[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) acc[j] = (d4){0.0, 0.0, 0.0, 0.0};
  __shared__ float4 sg[2 * kTile];
  __shared__ double sf[kFeat * kTile];
  for (int64_t mt = m0; mt < m1; mt += kTile) {
    const int cnt = (int)(m1 - mt < kTile ? m1 - mt : kTile);
    __syncthreads();
    load_tile<kFeat>(geo, feat, mt, cnt, sg, sf);
    __syncthreads();
    const int steps = (cnt + 3) >> 2;
    for (int s = 0; s < steps; ++s) {
      const int jt = 4 * s + kq;
      const float4 g0 = sg[2 * jt];
      const float4 g1 = sg[2 * jt + 1];
      const double b = sf[kFeat * jt + r];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const double a = (double)pair_exp(x[j], g0, g1, negc);
        acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[j], 0, 0, 0);
      }
    }
  }
  // lane holds rows kq + 4q (q = 0..3) of each 16 x 16 block, column r
  if (r < kFeatUsed) {
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int n = wbase + 16 * j + kq + 4 * q;
        if (n < N) partial[((size_t)split * kFeatUsed + r) * N + n] = acc[j][q];
      }
  }
}

// ------------------------------------------------------------- finalisation
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__global__ __launch_bounds__(kBlock) void estep_finalize(
    const float *__restrict__ X, int N, const float *__restrict__ w,
    const DevState *__restrict__ st, const double *__restrict__ partial, int nsplit,
    double *__restrict__ blockstats, double *__restrict__ colS, double *__restrict__ colstats) {
  if (st->done) return;
  const int n = blockIdx.x * kBlock + threadIdx.x;
  double p = 0.0, W[6] = {0, 0, 0, 0, 0, 0}, B[3] = {0, 0, 0}, C = 0.0, lg = 0.0, outl = 0.0,
         logw = 0.0;
  double xt[4] = {0.0, 0.0, 0.0, 0.0};
  if (n < N) {
    double T[kFeatUsed];
#pragma unroll
    for (int c = 0; c < kFeatUsed; ++c) T[c] = 0.0;
    for (int sp = 0; sp < nsplit; ++sp)
#pragma unroll
      for (int c = 0; c < kFeatUsed; ++c) T[c] += partial[((size_t)sp * kFeatUsed + c) * N + n];
    const double wn = w ? (double)w[n] : st->w0;
    const double rho = (1.0 - wn) / wn;
    const double gam = gamma_of(st);
    const double den = rho * T[0];
    const double inv = 1.0 / (den + gam);
    const double sc = rho * inv;
    p = den * inv;
#pragma unroll
    for (int i = 0; i < 6; ++i) W[i] = sc * T[1 + i];
#pragma unroll
    for (int i = 0; i < 3; ++i) B[i] = sc * T[7 + i];
    C = sc * T[10];
    lg = log(den + gam);
    outl = gam * inv;
    logw = log(wn);
    colS[n] = T[0];
    if (colstats) {
      double *cs = colstats + (size_t)n * kColStats;
      cs[0] = T[0];
      cs[1] = den;
      cs[2] = p;
      for (int i = 0; i < 6; ++i) cs[3 + i] = W[i];
      for (int i = 0; i < 3; ++i) cs[9 + i] = B[i];
      cs[12] = C;
      cs[13] = lg;
      cs[14] = outl;
      cs[15] = 0.0;
    }
    xt[0] = (double)X[3 * n];
    xt[1] = (double)X[3 * n + 1];
    xt[2] = (double)X[3 * n + 2];
    xt[3] = 1.0;
  }
  double xx[10];
  {
    int o = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = i; j < 4; ++j) xx[o++] = xt[i] * xt[j];
  }
  // statistic i of this source (layout documented with the public header)
  auto value = [&](int i) -> double {
    if (i < 10) return p * xx[i];
    if (i < 70) return W[(i - 10) / 10] * xx[(i - 10) % 10];
    if (i < 82) return B[(i - 70) / 4] * xt[(i - 70) % 4];
    if (i == 82) return C;
    if (i == 83) return lg;
    if (i == 84) return outl;
    return logw;
  };
  __shared__ double red[kBlock / 64][kStats];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < kStats; ++i) {
    const double s = wave_sum(value(i));
    if (lane == 0) red[wave][i] = s;
  }
  __syncthreads();
  if (threadIdx.x < kStats) {
    double s = 0.0;
    for (int wv = 0; wv < kBlock / 64; ++wv) s += red[wv][threadIdx.x];
    blockstats[(size_t)blockIdx.x * kStats + threadIdx.x] = s;
  }
}

// Test aid: writes P (M x N, float32) from the same per-pair exponent.
__global__ void dump_P(const float *__restrict__ X, int N, const float4 *__restrict__ geo,
                       int64_t M, const float *__restrict__ w, const DevState *__restrict__ st,
                       const double *__restrict__ colS, float *__restrict__ P) {
  double R[9], t[3];
  for (int i = 0; i < 9; ++i) R[i] = st->R[i];
  for (int i = 0; i < 3; ++i) t[i] = st->t[i];
  const float negc = neg_c_of(st);
  const double gam = gamma_of(st);
  const int64_t total = M * (int64_t)N;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t m = idx / N;
    const int n = (int)(idx - m * N);
    const Src x = load_src(X, n, N, R, t);
    const float e = pair_exp(x, geo[2 * m], geo[2 * m + 1], negc);
    const double wn = w ? (double)w[n] : st->w0;
    const double rho = (1.0 - wn) / wn;
    P[idx] = (float)(rho * (double)e / (rho * colS[n] + gam));
  }
}

// ----------------------------------------------------------- target records
__global__ void prep_targets(const float *__restrict__ Y, const float *__restrict__ nrm,
                             const float *__restrict__ alpha, const float *__restrict__ pi,
                             int64_t M, int exact, float4 *__restrict__ geo,
                             double *__restrict__ feat) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M) return;
  const double y0 = Y[3 * m], y1 = Y[3 * m + 1], y2 = Y[3 * m + 2];
  const double n0 = nrm[3 * m], n1 = nrm[3 * m + 1], n2 = nrm[3 * m + 2];
  const double al = alpha[m];
  const double pm = pi ? (double)pi[m] : 1.0 / (double)M;
  double l = log2(pm);
  if (exact) l += 0.5 * log2(1.0 + al);
  const double sa = sqrt(al);
  geo[2 * m] = make_float4((float)y0, (float)y1, (float)y2, (float)l);
  geo[2 * m + 1] = make_float4((float)(sa * n0), (float)(sa * n1), (float)(sa * n2), 0.f);
  const double s = y0 * n0 + y1 * n1 + y2 * n2;
  double *f = feat + m * kFeat;
  f[0] = 1.0;
  f[1] = al * n0 * n0;
  f[2] = al * n0 * n1;
  f[3] = al * n0 * n2;
  f[4] = al * n1 * n1;
  f[5] = al * n1 * n2;
  f[6] = al * n2 * n2;
  f[7] = y0 + al * s * n0;
  f[8] = y1 + al * s * n1;
  f[9] = y2 + al * s * n2;
  f[10] = y0 * y0 + y1 * y1 + y2 * y2 + al * s * s;
  for (int c = kFeatUsed; c < kFeat; ++c) f[c] = 0.0;
}

// ---------------------------------------------------------------- moments
__global__ __launch_bounds__(256) void moments_partial(const float *__restrict__ P, int n,
                                                       const DevState *__restrict__ pose,
                                                       double *__restrict__ part) {
  double R[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1}, t[3] = {0, 0, 0};
  if (pose) {
    for (int i = 0; i < 9; ++i) R[i] = pose->R[i];
    for (int i = 0; i < 3; ++i) t[i] = pose->t[i];
  }
  double v[10] = {0, 0, 0, 0, INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const double x = P[3 * i], y = P[3 * i + 1], z = P[3 * i + 2];
    const double p0 = fma(R[0], x, fma(R[1], y, fma(R[2], z, t[0])));
    const double p1 = fma(R[3], x, fma(R[4], y, fma(R[5], z, t[1])));
    const double p2 = fma(R[6], x, fma(R[7], y, fma(R[8], z, t[2])));
    v[0] += p0;
    v[1] += p1;
    v[2] += p2;
    v[3] += p0 * p0 + p1 * p1 + p2 * p2;
    v[4] = fmin(v[4], p0);
    v[5] = fmin(v[5], p1);
    v[6] = fmin(v[6], p2);
    v[7] = fmax(v[7], p0);
    v[8] = fmax(v[8], p1);
    v[9] = fmax(v[9], p2);
  }
  __shared__ double red[4][10];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 10; ++k) {
    double a = v[k];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double b = __shfl_xor(a, o, 64);
      a = k < 4 ? a + b : (k < 7 ? fmin(a, b) : fmax(a, b));
    }
    if (lane == 0) red[wave][k] = a;
  }
  __syncthreads();
  if (threadIdx.x < 10) {
    const int k = threadIdx.x;
    double a = red[0][k];
    for (int wv = 1; wv < 4; ++wv) {
      const double b = red[wv][k];
      a = k < 4 ? a + b : (k < 7 ? fmin(a, b) : fmax(a, b));
    }
    part[blockIdx.x * 10 + k] = a;
  }
}

__global__ void moments_final(const double *__restrict__ part, int nblk, double *__restrict__ out) {
  const int k = threadIdx.x;
  if (k >= 10) return;
  double a = part[k];
  for (int b = 1; b < nblk; ++b) {
    const double c = part[b * 10 + k];
    a = k < 4 ? a + c : (k < 7 ? fmin(a, c) : fmax(a, c));
  }
  out[k] = a;
}

}  // namespace

// ----------------------------------------------------------------- launchers

EstepPlan estep_plan(int64_t N, int64_t M, int mfma) {
  EstepPlan pl;
  pl.mfma = mfma;
  const int64_t per_block = mfma ? kBlock : (int64_t)kBlock * kValuS;
  pl.nsrc_blocks = (int)((N + per_block - 1) / per_block);
  // enough blocks to fill 256 CUs several times; chunks of >= 2 tiles
  const int64_t want = 2048;
  int64_t ns = (want + pl.nsrc_blocks - 1) / pl.nsrc_blocks;
  const int64_t maxs = (M + 2 * kTile - 1) / (2 * kTile);
  if (ns > maxs) ns = maxs;
  if (ns > 64) ns = 64;
  if (ns < 1) ns = 1;
  int64_t chunk = (M + ns - 1) / ns;
  chunk = (chunk + kTile - 1) / kTile * kTile;
  ns = (M + chunk - 1) / chunk;
  pl.nsplit = (int)ns;
  pl.mchunk = chunk;
  pl.nfin_blocks = (int)((N + kBlock - 1) / kBlock);
  return pl;
}

size_t estep_partial_bytes(const EstepPlan &pl, int64_t N) {
  return (size_t)pl.nsplit * kFeatUsed * (size_t)N * sizeof(double);
}

hipError_t launch_estep(const EstepPlan &pl, const float *X, int64_t N, const float4 *geo,
                        const double *feat, int64_t M, const DevState *s, double *partial,
                        hipStream_t st) {
  dim3 grid((unsigned)(pl.nsrc_blocks * pl.nsplit));
  if (pl.mfma)
    hipLaunchKernelGGL(estep_mfma, grid, dim3(kBlock), 0, st, X, (int)N, geo, feat, M, s,
                       pl.mchunk, pl.nsplit, partial);
  else
    hipLaunchKernelGGL(estep_valu<kValuS>, grid, dim3(kBlock), 0, st, X, (int)N, geo, feat, M,
                       s, pl.mchunk, pl.nsplit, partial);
  return hipGetLastError();
}

hipError_t launch_finalize(const EstepPlan &pl, const float *X, int64_t N, const float *w,
                           const DevState *s, const double *partial, double *blockstats,
                           double *colS, double *colstats, hipStream_t st) {
  hipLaunchKernelGGL(estep_finalize, dim3((unsigned)pl.nfin_blocks), dim3(kBlock), 0, st, X,
                     (int)N, w, s, partial, pl.nsplit, blockstats, colS, colstats);
  return hipGetLastError();
}

hipError_t launch_dump_P(const float *X, int64_t N, const float4 *geo, int64_t M, const float *w,
                         const DevState *s, const double *colS, float *P, hipStream_t st) {
  const int64_t total = M * N;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(dump_P, dim3((unsigned)blocks), dim3(256), 0, st, X, (int)N, geo, M, w, s,
                     colS, P);
  return hipGetLastError();
}

hipError_t launch_prep_targets(const float *Y, const float *normals, const float *alpha,
                               const float *pi, int64_t M, int exact, float4 *geo, double *feat,
                               hipStream_t st) {
  hipLaunchKernelGGL(prep_targets, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, st, Y,
                     normals, alpha, pi, M, exact, geo, feat);
  return hipGetLastError();
}

int moments_blocks(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 512) b = 512;
  if (b < 1) b = 1;
  return (int)b;
}

hipError_t launch_moments(const float *P, int64_t n, const DevState *pose, double *partials,
                          int nblk, double *out, hipStream_t st) {
  hipLaunchKernelGGL(moments_partial, dim3((unsigned)nblk), dim3(256), 0, st, P, (int)n, pose,
                     partials);
  hipLaunchKernelGGL(moments_final, dim3(1), dim3(64), 0, st, partials, nblk, out);
  return hipGetLastError();
}

}  // namespace lsg
