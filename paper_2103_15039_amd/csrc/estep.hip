// The LSG-CPD E step on gfx950 (Sec. 3.1 Eq. 5, Sec. 3.4 Eq. 9-10).
//
// For every (target m, source n) pair the kernels evaluate
//   e_mn = K_mn / rho_n = 2^( l_m - c d_mn ),   c = log2(e) / (2 sigma^2),
//   d_mn = |r|^2 + (a_m . r)^2,  r = g(x_n) - y_m,  a_m = sqrt(alpha_m) n_m,
// i.e. sigma^2 times the Mahalanobis form of Eq. 2, and accumulate for each
// source the unnormalised sums  T_n[c] = sum_m e_mn f_m[c]  of 11 target
// features f_m = [1, alpha n n^T, M_m y_m, y_m^T M_m y_m]  (M_m = I + alpha n n^T).
// The normaliser of Eq. 9 is per source (a column of P), so one pass over the
// pairs suffices: P_mn = rho_n e_mn / (rho_n T_n[0] + gamma), and every
// P-weighted sum is rho_n T_n[c] / (rho_n T_n[0] + gamma).  The M x N posterior
// is never stored.
//
// Arithmetic per pair (gfx950 runs FP64 FMA at the FP32 rate, and packed FP32
// is not used): with the source pre-scaled, s_n = sqrt(c) g(x_n),
//   r = s_n - sqrt(c) y_m          3 FP64 FMA
//   q = l_m - |r|^2                 3 FP64 FMA
//   p = a_m . r                     3 FP64
//   z = q - p^2                     1 FP64 FMA   (= l_m - c d_mn)
//   e = exp2((float) z)             cvt + v_exp_f32 + cvt
//   T += e f_m                      11 FP64 add/FMA
// so residual and exponent are FP64 and only the exponential is float32
// (relative error of e about 2e-6 over the range that matters); features are
// exact FP64 functions of the float32 inputs and all sums are FP64.
//
// Back ends (same pair arithmetic, different data movement):
//  * estep_pairs_scalar<S> (default): all lanes of a wave take the same target
//    at the same time, so the target record is wave-uniform and is read
//    through the scalar data cache straight into SGPR operands; each lane keeps
//    S sources in registers.
//  * estep_pairs_lds<S>: the block stages tiles of target records in LDS and
//    every wave reads them back with broadcast LDS loads.
//  * estep_mfma: V_MFMA_F64_16X16X4 multiplies 16 (sources) x 4 (targets)
//    exponentials by 4 x 16 features.  On gfx950 matrix and vector
//    instructions of a SIMD do not execute concurrently and the FP64 matrix
//    rate equals the FP64 vector rate, so this is kept only for comparison.
// Target chunks (split-M) give enough blocks for small N; the per-chunk
// partial sums are combined in a fixed order by estep_finalize, so results are
// bitwise reproducible.
#include <math.h>

#include "lsgcpd_internal.h"

namespace lsg {

namespace {

constexpr double kLog2e = 1.4426950408889634074;
constexpr double kTwoPi = 6.283185307179586477;
constexpr int kBlock = 256;
constexpr int kTile = 64;            // targets per LDS tile (LDS back end)

__device__ __forceinline__ double gamma_of(const DevState *s) {
  return pow(kTwoPi * s->sigma2, 1.5) / s->V;
}

// sqrt(c) with c = log2(e) / (2 sigma^2)
__device__ __forceinline__ double sqrt_c_of(const DevState *s) {
  return sqrt(kLog2e / (2.0 * s->sigma2));
}

struct Src {
  double x0, x1, x2;  // sqrt(c) * g(x_n)
};

__device__ __forceinline__ Src load_src(const float *__restrict__ X, int n, int N,
                                        const double *R, const double *t, double sc) {
  double x = 0.0, y = 0.0, z = 0.0;
  if (n < N) {
    x = X[3 * n];
    y = X[3 * n + 1];
    z = X[3 * n + 2];
  }
  Src o;
  o.x0 = sc * fma(R[0], x, fma(R[1], y, fma(R[2], z, t[0])));
  o.x1 = sc * fma(R[3], x, fma(R[4], y, fma(R[5], z, t[1])));
  o.x2 = sc * fma(R[6], x, fma(R[7], y, fma(R[8], z, t[2])));
  return o;
}

// e = K_mn / rho_n of one pair; negsc = -sqrt(c).  Every operation is written
// out so that every kernel (and the P dump) produces the same value.
__device__ __forceinline__ double pair_exp(const Src &s, double y0, double y1, double y2,
                                           double a0, double a1, double a2, double l,
                                           double negsc) {
  const double r0 = fma(negsc, y0, s.x0);
  const double r1 = fma(negsc, y1, s.x1);
  const double r2 = fma(negsc, y2, s.x2);
  double q = fma(-r0, r0, l);
  q = fma(-r1, r1, q);
  q = fma(-r2, r2, q);
  double p = a0 * r0;
  p = fma(a1, r1, p);
  p = fma(a2, r2, p);
  const double z = fma(-p, p, q);
  return (double)__builtin_amdgcn_exp2f((float)z);
}

__device__ __forceinline__ double rec_exp(const Src &s, const TRec &t, double negsc) {
  return pair_exp(s, t.y[0], t.y[1], t.y[2], t.a[0], t.a[1], t.a[2], t.l, negsc);
}

template <int S>
__device__ __forceinline__ void accumulate(const Src (&x)[S], const TRec &t, double negsc,
                                           double (&acc)[S][kFeatUsed]) {
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const double e = rec_exp(x[s], t, negsc);
    acc[s][0] += e;
#pragma unroll
    for (int c = 1; c < kFeatUsed; ++c) acc[s][c] = fma(e, t.f[c - 1], acc[s][c]);
  }
}

// ------------------------------------------------------- pair kernel (VALU)
// Scalar-cache back end.  The block's four waves form 4/Q source groups of Q
// waves; a group owns 64*S sources (S per lane) and its Q waves split the
// block's target chunk into Q parts.  Waves of different groups read the same
// records at about the same time (scalar-cache reuse 4/Q); the Q partial sums
// of a group are added through LDS in a fixed order, so a block writes one
// partial per source (Q times fewer partials than one per wave).
template <int S, int Q>
__global__ __launch_bounds__(kBlock) void estep_pairs_scalar(const float *__restrict__ X, int N,
                                                             const TRec *__restrict__ rec,
                                                             int64_t M,
                                                             const DevState *__restrict__ st,
                                                             int64_t mchunk, int nsplit,
                                                             double *__restrict__ partial) {
  if (st->done) return;
  constexpr int G = 4 / Q;  // source groups per block
  const int split = blockIdx.x % nsplit;
  const int sb = blockIdx.x / nsplit;
  // the wave index is wave-uniform; readfirstlane tells the compiler so, which
  // keeps the target loop counter (and so the record loads) scalar
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int grp = wave % G, part = wave / G;
  const int64_t m0 = (int64_t)split * mchunk;
  const int64_t m1 = m0 + mchunk < M ? m0 + mchunk : M;
  const int64_t qc = (m1 - m0 + Q - 1) / Q;
  const int64_t w0 = m0 + part * qc < m1 ? m0 + part * qc : m1;
  const int64_t w1 = w0 + qc < m1 ? w0 + qc : m1;
  double R[9], t[3];
  for (int i = 0; i < 9; ++i) R[i] = st->R[i];
  for (int i = 0; i < 3; ++i) t[i] = st->t[i];
  const double sc = sqrt_c_of(st);
  const double negsc = -sc;
  Src x[S];
  int nidx[S];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    nidx[s] = (sb * G + grp) * 64 * S + s * 64 + lane;
    x[s] = load_src(X, nidx[s], N, R, t, sc);
  }
  double acc[S][kFeatUsed];
#pragma unroll
  for (int s = 0; s < S; ++s)
#pragma unroll
    for (int c = 0; c < kFeatUsed; ++c) acc[s][c] = 0.0;
  for (int64_t m = w0; m < w1; ++m) accumulate<S>(x, rec[m], negsc, acc);
  if constexpr (Q == 1) {
#pragma unroll
    for (int s = 0; s < S; ++s) {
      if (nidx[s] < N) {
#pragma unroll
        for (int c = 0; c < kFeatUsed; ++c)
          partial[((size_t)split * kFeatUsed + c) * N + nidx[s]] = acc[s][c];
      }
    }
  } else {
    __shared__ double red[4 - G][kFeatUsed][64];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      if (part > 0)
#pragma unroll
        for (int c = 0; c < kFeatUsed; ++c) red[wave - G][c][lane] = acc[s][c];
      __syncthreads();
      if (part == 0 && nidx[s] < N) {
#pragma unroll
        for (int c = 0; c < kFeatUsed; ++c) {
          double v = acc[s][c];
#pragma unroll
          for (int p = 1; p < Q; ++p) v += red[p * G + grp - G][c][lane];
          partial[((size_t)split * kFeatUsed + c) * N + nidx[s]] = v;
        }
      }
      __syncthreads();
    }
  }
}

// LDS back end: the block stages tiles of target records in LDS and every
// wave reads them back with broadcast loads; a block owns 256*S sources.
template <int S>
__global__ __launch_bounds__(kBlock) void estep_pairs_lds(const float *__restrict__ X, int N,
                                                          const TRec *__restrict__ rec, int64_t M,
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
  const double sc = sqrt_c_of(st);
  const double negsc = -sc;
  Src x[S];
  int nidx[S];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    nidx[s] = sb * kBlock * S + s * kBlock + threadIdx.x;
    x[s] = load_src(X, nidx[s], N, R, t, sc);
  }
  double acc[S][kFeatUsed];
#pragma unroll
  for (int s = 0; s < S; ++s)
#pragma unroll
    for (int c = 0; c < kFeatUsed; ++c) acc[s][c] = 0.0;
  __shared__ TRec tile[kTile];
  for (int64_t mt = m0; mt < m1; mt += kTile) {
    const int cnt = (int)(m1 - mt < kTile ? m1 - mt : kTile);
    __syncthreads();
    const double *src = (const double *)(rec + mt);
    double *dst = (double *)tile;
    for (int i = threadIdx.x; i < cnt * kRecDoubles; i += kBlock) dst[i] = src[i];
    __syncthreads();
    for (int j = 0; j < cnt; ++j) accumulate<S>(x, tile[j], negsc, acc);
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

// ------------------------------------------------------- pair kernel (MFMA)
// Wave layout: lane l, r = l % 16 (row in a 16-source group), kq = l / 16
// (target slot).  Each wave owns 64 sources (4 groups of 16).  Per step of 4
// targets, lane l computes e(source 16j + r, target 4s + kq) for j = 0..3 --
// the A operand (16 x 4) element it supplies -- and feature r of target
// 4s + kq is its B operand (4 x 16) element.
typedef double d4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(kBlock) void estep_mfma(const float *__restrict__ X, int N,
                                                    const TRec *__restrict__ rec, int64_t M,
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
  const double sc = sqrt_c_of(st);
  const double negsc = -sc;
  Src x[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) x[j] = load_src(X, wbase + 16 * j + r, N, R, t, sc);
  d4 acc[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) acc[j] = (d4){0.0, 0.0, 0.0, 0.0};
  for (int64_t mt = m0; mt < m1; mt += 4) {
    const int64_t m = mt + kq;
    const bool ok = m < m1;
    const TRec &tr = rec[ok ? m : m0];
    const double b = !ok ? 0.0 : (r == 0 ? 1.0 : (r < kFeatUsed ? tr.f[r - 1] : 0.0));
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const double a = ok ? rec_exp(x[j], tr, negsc) : 0.0;
      acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[j], 0, 0, 0);
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

constexpr int kFinBlock = 64;

__global__ __launch_bounds__(kFinBlock) void estep_finalize(
    const float *__restrict__ X, int N, const float *__restrict__ w,
    const DevState *__restrict__ st, const double *__restrict__ partial, int nsplit,
    double *__restrict__ blockstats, double *__restrict__ colS, double *__restrict__ colstats) {
  if (st->done) return;
  const int n = blockIdx.x * kFinBlock + threadIdx.x;
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
  // statistic i of this source (layout documented with the public header),
  // written to LDS and summed over the block's sources in a fixed order
  __shared__ double red[kStats][kFinBlock + 1];
  const int l = threadIdx.x;
#pragma unroll
  for (int i = 0; i < 10; ++i) red[i][l] = p * xx[i];
#pragma unroll
  for (int ab = 0; ab < 6; ++ab)
#pragma unroll
    for (int i = 0; i < 10; ++i) red[10 + 10 * ab + i][l] = W[ab] * xx[i];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int j = 0; j < 4; ++j) red[70 + 4 * a + j][l] = B[a] * xt[j];
  red[82][l] = C;
  red[83][l] = lg;
  red[84][l] = outl;
  red[85][l] = logw;
  __syncthreads();
  for (int i = l; i < kStats; i += kFinBlock) {
    double s = 0.0;
    for (int k = 0; k < kFinBlock; ++k) s += red[i][k];
    blockstats[(size_t)i * gridDim.x + blockIdx.x] = s;  // stat-major
  }
}

// Test aid: writes P (M x N, float32) from the same per-pair exponent.
__global__ void dump_P(const float *__restrict__ X, int N, const TRec *__restrict__ rec,
                       int64_t M, const float *__restrict__ w, const DevState *__restrict__ st,
                       const double *__restrict__ colS, float *__restrict__ P) {
  double R[9], t[3];
  for (int i = 0; i < 9; ++i) R[i] = st->R[i];
  for (int i = 0; i < 3; ++i) t[i] = st->t[i];
  const double sc = sqrt_c_of(st);
  const double gam = gamma_of(st);
  const int64_t total = M * (int64_t)N;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t m = idx / N;
    const int n = (int)(idx - m * N);
    const Src x = load_src(X, n, N, R, t, sc);
    const double e = rec_exp(x, rec[m], -sc);
    const double wn = w ? (double)w[n] : st->w0;
    const double rho = (1.0 - wn) / wn;
    P[idx] = (float)(rho * e / (rho * colS[n] + gam));
  }
}

// ----------------------------------------------------------- target records
__global__ void prep_targets(const float *__restrict__ Y, const float *__restrict__ nrm,
                             const float *__restrict__ alpha, const float *__restrict__ pi,
                             int64_t M, int exact, TRec *__restrict__ rec) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M) return;
  const double y0 = Y[3 * m], y1 = Y[3 * m + 1], y2 = Y[3 * m + 2];
  const double n0 = nrm[3 * m], n1 = nrm[3 * m + 1], n2 = nrm[3 * m + 2];
  const double al = alpha[m];
  const double pm = pi ? (double)pi[m] : 1.0 / (double)M;
  double l = log2(pm);
  if (exact) l += 0.5 * log2(1.0 + al);
  const double sa = sqrt(al);
  const double s = y0 * n0 + y1 * n1 + y2 * n2;
  TRec r;
  r.y[0] = y0;
  r.y[1] = y1;
  r.y[2] = y2;
  r.a[0] = sa * n0;
  r.a[1] = sa * n1;
  r.a[2] = sa * n2;
  r.l = l;
  r.f[0] = al * n0 * n0;
  r.f[1] = al * n0 * n1;
  r.f[2] = al * n0 * n2;
  r.f[3] = al * n1 * n1;
  r.f[4] = al * n1 * n2;
  r.f[5] = al * n2 * n2;
  r.f[6] = y0 + al * s * n0;
  r.f[7] = y1 + al * s * n1;
  r.f[8] = y2 + al * s * n2;
  r.f[9] = y0 * y0 + y1 * y1 + y2 * y2 + al * s * s;
  r.pad = 0.0;
  rec[m] = r;
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

EstepPlan estep_plan(int64_t N, int64_t M, int backend, int srcs_per_lane, int parts) {
  EstepPlan pl;
  pl.backend = backend;
  pl.srcs_per_lane = backend == kBackendScalar && srcs_per_lane == 4 ? 4 : kPairS;
  pl.parts = parts == 1 || parts == 4 ? parts : 2;
  // sources per block: the scalar back end has 4/Q groups of 64*S sources,
  // the LDS back end gives every thread its own S, MFMA 64 per wave
  const int64_t per_block = backend == kBackendScalar
                                ? (int64_t)(4 / pl.parts) * 64 * pl.srcs_per_lane
                            : backend == kBackendLds ? (int64_t)kBlock * pl.srcs_per_lane
                                                     : (int64_t)kBlock;
  pl.nsrc_blocks = (int)((N + per_block - 1) / per_block);
  // about 1024 blocks (4096 waves) fill the 256 CUs; every split adds one
  // FP64 partial per source and feature, so no more splits than that
  const int64_t want = 1024;
  int64_t ns = (want + pl.nsrc_blocks - 1) / pl.nsrc_blocks;
  const int64_t maxs = (M + 127) / 128;
  if (ns > maxs) ns = maxs;
  if (ns > 64) ns = 64;
  if (ns < 1) ns = 1;
  int64_t chunk = (M + ns - 1) / ns;
  chunk = (chunk + 3) / 4 * 4;
  ns = (M + chunk - 1) / chunk;
  pl.nsplit = (int)ns;
  pl.mchunk = chunk;
  pl.nfin_blocks = (int)((N + kFinBlock - 1) / kFinBlock);
  return pl;
}

size_t estep_partial_bytes(const EstepPlan &pl, int64_t N) {
  return (size_t)pl.nsplit * kFeatUsed * (size_t)N * sizeof(double);
}

hipError_t launch_estep(const EstepPlan &pl, const float *X, int64_t N, const TRec *rec,
                        int64_t M, const DevState *s, double *partial, hipStream_t st) {
  dim3 grid((unsigned)(pl.nsrc_blocks * pl.nsplit));
  if (pl.backend == kBackendMfma)
    hipLaunchKernelGGL(estep_mfma, grid, dim3(kBlock), 0, st, X, (int)N, rec, M, s, pl.mchunk,
                       pl.nsplit, partial);
  else if (pl.backend == kBackendLds)
    hipLaunchKernelGGL(estep_pairs_lds<kPairS>, grid, dim3(kBlock), 0, st, X, (int)N, rec, M, s,
                       pl.mchunk, pl.nsplit, partial);
  else {
#define LSG_PAIRS(S_, Q_)                                                                  \
  hipLaunchKernelGGL((estep_pairs_scalar<S_, Q_>), grid, dim3(kBlock), 0, st, X, (int)N, rec, \
                     M, s, pl.mchunk, pl.nsplit, partial)
    if (pl.srcs_per_lane == 4) {
      if (pl.parts == 1) LSG_PAIRS(4, 1);
      else if (pl.parts == 2) LSG_PAIRS(4, 2);
      else LSG_PAIRS(4, 4);
    } else {
      if (pl.parts == 1) LSG_PAIRS(2, 1);
      else if (pl.parts == 2) LSG_PAIRS(2, 2);
      else LSG_PAIRS(2, 4);
    }
#undef LSG_PAIRS
  }
  return hipGetLastError();
}

hipError_t launch_finalize(const EstepPlan &pl, const float *X, int64_t N, const float *w,
                           const DevState *s, const double *partial, double *blockstats,
                           double *colS, double *colstats, hipStream_t st) {
  hipLaunchKernelGGL(estep_finalize, dim3((unsigned)pl.nfin_blocks), dim3(kFinBlock), 0, st, X,
                     (int)N, w, s, partial, pl.nsplit, blockstats, colS, colstats);
  return hipGetLastError();
}

hipError_t launch_dump_P(const float *X, int64_t N, const TRec *rec, int64_t M, const float *w,
                         const DevState *s, const double *colS, float *P, hipStream_t st) {
  const int64_t total = M * N;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(dump_P, dim3((unsigned)blocks), dim3(256), 0, st, X, (int)N, rec, M, w, s,
                     colS, P);
  return hipGetLastError();
}

hipError_t launch_prep_targets(const float *Y, const float *normals, const float *alpha,
                               const float *pi, int64_t M, int exact, TRec *rec,
                               hipStream_t st) {
  hipLaunchKernelGGL(prep_targets, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, st, Y,
                     normals, alpha, pi, M, exact, rec);
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
