// Learned initial-pose proposal: a point-set encoder that predicts the rigid
// motion between two clouds, so that LSG-CPD starts inside its basin of
// convergence (the method, like every local registration, needs a good
// start: Sec. 1 and Sec. 5).
//
// Model (one flat float32 parameter vector, W row-major [out][in], then b):
//   per point  3 -> 64 -> 128 -> 256, ReLU after each layer, max-pool over
//              the cloud's points;
//   per pair   [source 256 | target 256] -> 128 (ReLU) -> 9:
//              two 3-vectors -> rotation by Gram-Schmidt (6-D rotation
//              representation), and a translation in normalised units.
// Inputs: P points of each cloud at indices floor((2k + 1) N / (2P)), the
// source optionally rotated by Q, each cloud centred on its sampled mean and
// both divided by the RMS radius s of the sampled target.
//
// Kernels (all FP32 except the Gram-Schmidt step and the pose, FP64):
//  * prop_inputs      one block per pair: sampling, centring, scale;
//  * prop_prepare     transposed copies of W2 and W3 (MFMA B operands read
//                     16 consecutive output channels per lane group);
//  * prop_encode      one block per (cloud, 64 points): layer 1 on the VALU,
//                     layers 2 and 3 as V_MFMA_F32_16X16X4F32 products (16
//                     points per wave), ReLU and the max-pool fused into the
//                     last product's epilogue; the pooled value and its point
//                     travel as one 64-bit key (value bits, then the complement
//                     of the point index) so that a single atomicMax keeps the
//                     largest value and, on ties, the lowest point -- no
//                     P x 256 activation ever reaches memory;
//  * prop_head        one block per pair: 512 -> 128 -> 9, Gram-Schmidt, pose;
//  * prop_head_train  the same, the loss (least squares of the 9 outputs
//                     against the label's first two rotation columns and its
//                     translation, in the frames) and its gradient back to
//                     the pooled features;
//  * prop_encode_back one block per cloud: the gradient reaches only the
//                     argmax point of each live channel, so the per-point
//                     layers are recomputed and differentiated at those
//                     (at most 256) points only;
//  * prop_grad_sum    fixed-order sums of the per-cloud and per-pair parts
//                     (deterministic, no atomics);
//  * prop_adam        Adam with bias correction.
#include <math.h>

#include "lsgcpd_internal.h"

namespace lsg {

namespace {

constexpr int oW1 = 0, oB1 = oW1 + 64 * 3, oW2 = oB1 + 64, oB2 = oW2 + 128 * 64, oW3 = oB2 + 128,
              oB3 = oW3 + 256 * 128, oW4 = oB3 + 256, oB4 = oW4 + 128 * 512, oW5 = oB4 + 128,
              oB5 = oW5 + 9 * 128, kNP = oB5 + 9;
static_assert(kNP == kPropParams, "parameter layout");
// the encoder's parameters W1 .. b3 come first: their per-cloud gradients
constexpr int kEncParams = oW4;
constexpr int kChunk = 64;       // points per encoder block (16 per wave)
constexpr int kBackPts = 32;     // argmax points per round of the backward

typedef float f32x4 __attribute__((ext_vector_type(4)));

// Fixed-order sum over a block of 256 threads (4 waves).
__device__ double block_sum(double v, double *red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  return ((red[0] + red[1]) + red[2]) + red[3];
}

__device__ __forceinline__ int64_t sample_index(int k, int64_t n, int P) {
  return ((2 * (int64_t)k + 1) * n) / (2 * (int64_t)P);
}

// Point p of cloud c (pair c >> 1; source if c is even): the inputs of pair
// idx[b] (idx null: pair b).
__device__ __forceinline__ void load_point(const float *__restrict__ Xn,
                                           const float *__restrict__ Yn, int P,
                                           const int *__restrict__ idx, int cloud, int p,
                                           float &x0, float &x1, float &x2) {
  const int b = cloud >> 1;
  const int base = idx ? idx[b] : b;
  const float *q = ((cloud & 1) ? Yn : Xn) + ((size_t)base * P + p) * 3;
  x0 = q[0];
  x1 = q[1];
  x2 = q[2];
}

// Principal-axis frame of a cloud from its covariance (00 01 02 11 12 22,
// about the mean): eigenvectors in decreasing order of eigenvalue, as the
// columns of F (row-major 3x3); the identity for a zero covariance.  Signs
// are set afterwards from the third moments (sign_frame).
__device__ void eigen_frame(const double (&cv)[6], double (&F)[9]) {
  if (cv[0] == 0.0 && cv[1] == 0.0 && cv[2] == 0.0 && cv[3] == 0.0 && cv[4] == 0.0 &&
      cv[5] == 0.0) {
    for (int i = 0; i < 9; ++i) F[i] = i % 4 == 0 ? 1.0 : 0.0;
    return;
  }
  double a[3][3] = {{cv[0], cv[1], cv[2]}, {cv[1], cv[3], cv[4]}, {cv[2], cv[4], cv[5]}};
  double v[3][3];
  jacobi3(a, v);
  int o[3] = {0, 1, 2};  // decreasing eigenvalues
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2 - i; ++j)
      if (a[o[j]][o[j]] < a[o[j + 1]][o[j + 1]]) {
        const int t = o[j];
        o[j] = o[j + 1];
        o[j + 1] = t;
      }
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) F[3 * r + c] = v[r][o[c]];
}

// Signs of e0 and e1 from their third moments m3 (if one is exactly 0: the
// largest component positive), then e2 = e0 x e1.
__device__ void sign_frame(double (&F)[9], const double *m3) {
  for (int c = 0; c < 2; ++c) {
    int big = 0;
    for (int r = 1; r < 3; ++r)
      if (fabs(F[3 * r + c]) > fabs(F[3 * big + c])) big = r;
    if (m3[c] < 0.0 || (m3[c] == 0.0 && F[3 * big + c] < 0.0))
      for (int r = 0; r < 3; ++r) F[3 * r + c] = -F[3 * r + c];
  }
  F[2] = F[3] * F[7] - F[6] * F[4];
  F[5] = F[6] * F[1] - F[0] * F[7];
  F[8] = F[0] * F[4] - F[3] * F[1];
}

// One block per pair: samples, means, target scale, the two frames, inputs.
__global__ __launch_bounds__(256) void prop_inputs(const PropPair *__restrict__ pairs,
                                                   const double *__restrict__ Q, int P,
                                                   float *__restrict__ Xn, float *__restrict__ Yn,
                                                   double *__restrict__ norm) {
  const int b = blockIdx.x;
  const PropPair pr = pairs[b];
  double q[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
  if (Q)
    for (int i = 0; i < 9; ++i) q[i] = Q[9 * b + i];
  __shared__ double red[4];
  auto xpt = [&](int k, double (&x)[3]) {
    const int64_t ix = sample_index(k, pr.N, P);
    const double x0 = pr.X[3 * ix], x1 = pr.X[3 * ix + 1], x2 = pr.X[3 * ix + 2];
    for (int a = 0; a < 3; ++a) x[a] = q[3 * a] * x0 + q[3 * a + 1] * x1 + q[3 * a + 2] * x2;
  };
  auto ypt = [&](int k, double (&y)[3]) {
    const int64_t iy = sample_index(k, pr.M, P);
    for (int a = 0; a < 3; ++a) y[a] = (double)pr.Y[3 * iy + a];
  };
  double sx[3] = {0, 0, 0}, sy[3] = {0, 0, 0};
  for (int k = threadIdx.x; k < P; k += 256) {
    double x[3], y[3];
    xpt(k, x);
    ypt(k, y);
    for (int a = 0; a < 3; ++a) {
      sx[a] += x[a];
      sy[a] += y[a];
    }
  }
  double mx[3], my[3];
  for (int a = 0; a < 3; ++a) {
    mx[a] = block_sum(sx[a], red) / P;
    my[a] = block_sum(sy[a], red) / P;
  }
  // covariances about the means
  double cx[6] = {0, 0, 0, 0, 0, 0}, cy[6] = {0, 0, 0, 0, 0, 0};
  for (int k = threadIdx.x; k < P; k += 256) {
    double x[3], y[3];
    xpt(k, x);
    ypt(k, y);
    for (int a = 0; a < 3; ++a) {
      x[a] -= mx[a];
      y[a] -= my[a];
    }
    int o = 0;
    for (int i = 0; i < 3; ++i)
      for (int j = i; j < 3; ++j, ++o) {
        cx[o] += x[i] * x[j];
        cy[o] += y[i] * y[j];
      }
  }
  for (int o = 0; o < 6; ++o) {
    cx[o] = block_sum(cx[o], red) / P;
    cy[o] = block_sum(cy[o], red) / P;
  }
  double s = sqrt(cy[0] + cy[3] + cy[5]);
  if (!(s > 0.0)) s = 1.0;  // the target's samples are one point
  double FX[9], FY[9];
  eigen_frame(cx, FX);
  eigen_frame(cy, FY);
  // third moments along e0 and e1 of each cloud
  double m3[4] = {0, 0, 0, 0};
  for (int k = threadIdx.x; k < P; k += 256) {
    double x[3], y[3];
    xpt(k, x);
    ypt(k, y);
    for (int c = 0; c < 2; ++c) {
      double u = 0.0, w = 0.0;
      for (int a = 0; a < 3; ++a) {
        u += (x[a] - mx[a]) * FX[3 * a + c];
        w += (y[a] - my[a]) * FY[3 * a + c];
      }
      m3[c] += u * u * u;
      m3[2 + c] += w * w * w;
    }
  }
  for (int c = 0; c < 4; ++c) m3[c] = block_sum(m3[c], red);
  sign_frame(FX, m3);
  sign_frame(FY, m3 + 2);
  float *xo = Xn + (size_t)b * P * 3, *yo = Yn + (size_t)b * P * 3;
  for (int k = threadIdx.x; k < P; k += 256) {
    double x[3], y[3];
    xpt(k, x);
    ypt(k, y);
    for (int c = 0; c < 3; ++c) {
      double u = 0.0, w = 0.0;
      for (int a = 0; a < 3; ++a) {
        u += (x[a] - mx[a]) * FX[3 * a + c];
        w += (y[a] - my[a]) * FY[3 * a + c];
      }
      xo[3 * k + c] = (float)(u / s);
      yo[3 * k + c] = (float)(w / s);
    }
  }
  if (threadIdx.x == 0) {
    double *nm = norm + kPropNorm * b;
    for (int a = 0; a < 3; ++a) {
      nm[a] = mx[a];
      nm[3 + a] = my[a];
    }
    nm[6] = s;
    for (int i = 0; i < 9; ++i) {
      nm[7 + i] = FX[i];
      nm[16 + i] = FY[i];
    }
  }
}

// wt = [W2^T (64 x 128) | W3^T (128 x 256)]
__global__ void prop_prepare(const float *__restrict__ th, float *__restrict__ wt,
                             unsigned long long *__restrict__ pool, int npool) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < 128 * 64) {
    const int o = i / 64, k = i % 64;
    wt[k * 128 + o] = th[oW2 + i];
  }
  if (i < 256 * 128) {
    const int o = i / 128, k = i % 128;
    wt[64 * 128 + k * 256 + o] = th[oW3 + i];
  }
  if (i < npool) pool[i] = 0ull;  // empty keys for the max-pool
}

// Grid (chunks of 64 points, clouds); cloud c: pair c >> 1, source (even) or
// target (odd).  Lane l of a wave: row l & 15 (a point for the A operands, an
// output channel for B and the results), group l >> 4.
__global__ __launch_bounds__(256) void prop_encode(const float *__restrict__ th,
                                                   const float *__restrict__ wt,
                                                   const float *__restrict__ Xn,
                                                   const float *__restrict__ Yn, int P,
                                                   const int *__restrict__ idx,
                                                   unsigned long long *__restrict__ pool) {
  const int cloud = blockIdx.y;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lr = lane & 15, lg = lane >> 4;
  const int p0 = blockIdx.x * kChunk + wave * 16;
  const int pa = p0 + lr;
  float x0 = 0.f, x1 = 0.f, x2 = 0.f;
  if (pa < P) load_point(Xn, Yn, P, idx, cloud, pa, x0, x1, x2);
  const float *W2T = wt, *W3T = wt + 64 * 128;
  __shared__ float h2s[4][16][129];
  __shared__ unsigned long long best[4][256];
  // layer 1 in the A layout of layer 2: h1[pa][4 s + lg]
  float a1[16];
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    const int c = 4 * s + lg;
    const float v = fmaf(th[oW1 + 3 * c], x0,
                         fmaf(th[oW1 + 3 * c + 1], x1, fmaf(th[oW1 + 3 * c + 2], x2, th[oB1 + c])));
    a1[s] = fmaxf(v, 0.f);
  }
  // layer 2: 8 blocks of 16 output channels; result h2[p0 + 4 lg + i][16 j + lr]
#pragma unroll 2
  for (int j = 0; j < 8; ++j) {
    f32x4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < 16; ++s)
      c = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[s], W2T[(4 * s + lg) * 128 + 16 * j + lr], c, 0, 0,
                                               0);
    const float bias = th[oB2 + 16 * j + lr];
#pragma unroll
    for (int i = 0; i < 4; ++i) h2s[wave][4 * lg + i][16 * j + lr] = fmaxf(c[i] + bias, 0.f);
  }
  __builtin_amdgcn_wave_barrier();
  // A operand of layer 3: h2[p0 + lr][4 s + lg]
  float a2[32];
#pragma unroll
  for (int s = 0; s < 32; ++s) a2[s] = h2s[wave][lr][4 * s + lg];
  // layer 3 + ReLU + max over the wave's 16 points
  for (int j = 0; j < 16; ++j) {
    f32x4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < 32; ++s)
      c = __builtin_amdgcn_mfma_f32_16x16x4f32(a2[s], W3T[(4 * s + lg) * 256 + 16 * j + lr], c, 0, 0,
                                               0);
    const float bias = th[oB3 + 16 * j + lr];
    unsigned long long key = 0ull;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int p = p0 + 4 * lg + i;
      if (p < P) {
        const float v = fmaxf(c[i] + bias, 0.f);
        const unsigned long long k =
            ((unsigned long long)__float_as_uint(v) << 32) | (unsigned long long)(0xFFFFFFFFu - (unsigned)p);
        key = k > key ? k : key;
      }
    }
    unsigned long long o = __shfl_xor(key, 16, 64);
    key = o > key ? o : key;
    o = __shfl_xor(key, 32, 64);
    key = o > key ? o : key;
    if (lg == 0) best[wave][16 * j + lr] = key;
  }
  __syncthreads();
  const int ch = threadIdx.x;
  unsigned long long k = best[0][ch];
  for (int w = 1; w < 4; ++w) k = best[w][ch] > k ? best[w][ch] : k;
  if (k) atomicMax(pool + (size_t)cloud * 256 + ch, k);
}

__device__ __forceinline__ float pooled_value(unsigned long long key) {
  return __uint_as_float((unsigned)(key >> 32));
}
__device__ __forceinline__ int pooled_point(unsigned long long key) {
  return (int)(0xFFFFFFFFu - (unsigned)(key & 0xFFFFFFFFull));
}

// Shared head forward of one pair (128 threads): z, h4 and o into LDS.
__device__ void head_forward(const float *__restrict__ th, const unsigned long long *pool, int b,
                             float *zs, float *h4s, float *os) {
  const int t = threadIdx.x;
  for (int i = t; i < 512; i += 128) zs[i] = pooled_value(pool[(size_t)(2 * b + (i >> 8)) * 256 + (i & 255)]);
  __syncthreads();
  float a = th[oB4 + t];
  const float *w = th + oW4 + (size_t)t * 512;
  for (int i = 0; i < 512; ++i) a = fmaf(w[i], zs[i], a);
  h4s[t] = fmaxf(a, 0.f);
  __syncthreads();
  if (t < 9) {
    float o = th[oB5 + t];
    const float *w5 = th + oW5 + t * 128;
    for (int i = 0; i < 128; ++i) o = fmaf(w5[i], h4s[i], o);
    os[t] = o;
  }
  __syncthreads();
}

__device__ void gram_schmidt(const double *a1, const double *a2, double *b1, double *b2, double *b3,
                             double &n1, double &n2, double &c) {
  n1 = sqrt(a1[0] * a1[0] + a1[1] * a1[1] + a1[2] * a1[2]);
  for (int i = 0; i < 3; ++i) b1[i] = a1[i] / n1;
  c = b1[0] * a2[0] + b1[1] * a2[1] + b1[2] * a2[2];
  double u[3];
  for (int i = 0; i < 3; ++i) u[i] = a2[i] - c * b1[i];
  n2 = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  for (int i = 0; i < 3; ++i) b2[i] = u[i] / n2;
  b3[0] = b1[1] * b2[2] - b1[2] * b2[1];
  b3[1] = b1[2] * b2[0] - b1[0] * b2[2];
  b3[2] = b1[0] * b2[1] - b1[1] * b2[0];
}

// Inference: pose[b] = (R row-major, t) in world units.
__global__ __launch_bounds__(128) void prop_head(const float *__restrict__ th,
                                                 const unsigned long long *__restrict__ pool,
                                                 const double *__restrict__ norm,
                                                 double *__restrict__ pose) {
  const int b = blockIdx.x;
  __shared__ float zs[512], h4s[128], os[9];
  head_forward(th, pool, b, zs, h4s, os);
  if (threadIdx.x == 0) {
    double a1[3] = {os[0], os[1], os[2]}, a2[3] = {os[3], os[4], os[5]};
    double b1[3], b2[3], b3[3], n1, n2, c;
    gram_schmidt(a1, a2, b1, b2, b3, n1, n2, c);
    const double *nm = norm + kPropNorm * b, *FX = nm + 7, *FY = nm + 16;
    const double Rc[9] = {b1[0], b2[0], b3[0], b1[1], b2[1], b3[1], b1[2], b2[2], b3[2]};
    // R = F_Y R_c F_X^T, t = mu_Y + s F_Y t^ - R mu_X
    double T[9], R[9];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        T[3 * i + j] = FY[3 * i] * Rc[j] + FY[3 * i + 1] * Rc[3 + j] + FY[3 * i + 2] * Rc[6 + j];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        R[3 * i + j] = T[3 * i] * FX[3 * j] + T[3 * i + 1] * FX[3 * j + 1] + T[3 * i + 2] * FX[3 * j + 2];
    double *out = pose + 12 * b;
    for (int i = 0; i < 9; ++i) out[i] = R[i];
    for (int r = 0; r < 3; ++r)
      out[9 + r] = nm[3 + r] +
                   nm[6] * (FY[3 * r] * os[6] + FY[3 * r + 1] * os[7] + FY[3 * r + 2] * os[8]) -
                   (R[3 * r] * nm[0] + R[3 * r + 1] * nm[1] + R[3 * r + 2] * nm[2]);
  }
}

// Training: per pair the loss, and what the gradient sums need: z (512),
// h4 (128), the head-output gradient go (9), ga4 = dL/d(pre-ReLU of h4)
// (128) and gz = dL/dz (512).  label[b]: (R row-major, t) mapping the
// (rotated) source onto the target, in world units.
__global__ __launch_bounds__(128) void prop_head_train(
    const float *__restrict__ th, const unsigned long long *__restrict__ pool,
    const double *__restrict__ norm, const int *__restrict__ idx,
    const double *__restrict__ label, int B, double *__restrict__ loss, float *__restrict__ zo, float *__restrict__ h4o,
    float *__restrict__ goo, float *__restrict__ ga4o, float *__restrict__ gzo) {
  const int b = blockIdx.x, t = threadIdx.x;
  __shared__ float zs[512], h4s[128], os[9], gos[9], ga4s[128];
  head_forward(th, pool, b, zs, h4s, os);
  if (t == 0) {
    const double *nm = norm + kPropNorm * (idx ? idx[b] : b), *lb = label + 12 * b;
    const double *FX = nm + 7, *FY = nm + 16;
    // label in the frames: R_l = F_Y^T R F_X, t_l = F_Y^T (R mu_X + t - mu_Y) / s
    double T[9], Rl[9], tl[3], d[3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        T[3 * i + j] = FY[i] * lb[j] + FY[3 + i] * lb[3 + j] + FY[6 + i] * lb[6 + j];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        Rl[3 * i + j] = T[3 * i] * FX[j] + T[3 * i + 1] * FX[3 + j] + T[3 * i + 2] * FX[6 + j];
    for (int r = 0; r < 3; ++r)
      d[r] = lb[3 * r] * nm[0] + lb[3 * r + 1] * nm[1] + lb[3 * r + 2] * nm[2] + lb[9 + r] - nm[3 + r];
    for (int i = 0; i < 3; ++i) tl[i] = (FY[i] * d[0] + FY[3 + i] * d[1] + FY[6 + i] * d[2]) / nm[6];
    // least squares on the outputs: R_l's first two columns, then t_l
    const double tgt[9] = {Rl[0], Rl[3], Rl[6], Rl[1], Rl[4], Rl[7], tl[0], tl[1], tl[2]};
    double L = 0.0;
    for (int q = 0; q < 9; ++q) {
      const double e = (double)os[q] - tgt[q];
      L += e * e;
      gos[q] = (float)(2.0 * e / B);
    }
    loss[b] = L;
  }
  __syncthreads();
  {
    float gh = 0.f;
    for (int q = 0; q < 9; ++q) gh = fmaf(th[oW5 + q * 128 + t], gos[q], gh);
    ga4s[t] = h4s[t] > 0.f ? gh : 0.f;
  }
  __syncthreads();
  for (int i = t; i < 512; i += 128) {
    float gz = 0.f;
    for (int u = 0; u < 128; ++u) gz = fmaf(th[oW4 + (size_t)u * 512 + i], ga4s[u], gz);
    gzo[(size_t)b * 512 + i] = gz;
    zo[(size_t)b * 512 + i] = zs[i];
  }
  h4o[(size_t)b * 128 + t] = h4s[t];
  ga4o[(size_t)b * 128 + t] = ga4s[t];
  if (t < 9) goo[b * 9 + t] = gos[t];
}

// Gradient of one cloud's encoder parameters (W1 .. b3, kEncParams values)
// into part[cloud].  Thread k first owns channel k: its pooled point p_k and
// the gradient g_k of its pooled value (0 if the channel is inactive).  The
// distinct pooled points, in increasing order, are processed kBackPts at a
// time: their layer-1 and layer-2 activations are recomputed, the gradient
// of layer 2's output is the sum of g_k W3[k] over the channels pooled
// there (in channel order), and the parameter gradients are sums over the
// points (in point order), so the result is deterministic.
__global__ __launch_bounds__(256) void prop_encode_back(
    const float *__restrict__ th, const float *__restrict__ Xn, const float *__restrict__ Yn, int P,
    const int *__restrict__ idx, const unsigned long long *__restrict__ pool,
    const float *__restrict__ gz,
    float *__restrict__ part) {
  const int cloud = blockIdx.x, k = threadIdx.x;
  float *gp = part + (size_t)cloud * kEncParams;
  __shared__ int slot[kPropMaxPoints];  // per point: -1, or its distinct index
  const unsigned long long key = pool[(size_t)cloud * 256 + k];
  const float fk = pooled_value(key);
  const bool live = fk > 0.f;
  const int pk = live ? pooled_point(key) : -1;
  const float gk = live ? gz[(size_t)(cloud >> 1) * 512 + (cloud & 1) * 256 + k] : 0.f;
  gp[oB3 + k] = gk;
  for (int p = k; p < P; p += 256) slot[p] = -1;
  __syncthreads();
  if (live) slot[pk] = 0;  // mark (same value from every writer)
  __syncthreads();
  // distinct points in increasing order: a block-wide exclusive scan of the marks
  __shared__ int scan[256];
  __shared__ int total;
  int run = 0;
  for (int p0 = 0; p0 < P; p0 += 256) {
    const int p = p0 + k;
    const int v = p < P && slot[p] == 0 ? 1 : 0;
    scan[k] = v;
    __syncthreads();
    for (int d = 1; d < 256; d <<= 1) {
      const int add = k >= d ? scan[k - d] : 0;
      __syncthreads();
      scan[k] += add;
      __syncthreads();
    }
    if (v) slot[p] = run + scan[k] - 1;
    run += scan[255];
    __syncthreads();
  }
  if (k == 0) total = run;
  __syncthreads();
  const int D = total;
  const int sk = live ? slot[pk] : -1;
  // channels of each distinct point in channel order: k's position among
  // the live channels < k with the same point
  __shared__ int kslot[256];
  __shared__ float kg[256];
  kslot[k] = sk;
  kg[k] = gk;
  __syncthreads();
  // per-thread parameter accumulators: W2 entries k + 256 r (j = e / 64,
  // i = e % 64), b2 (k < 128), W1 and b1 (k < 192 / k < 64)
  float aW2[32];
#pragma unroll
  for (int r = 0; r < 32; ++r) aW2[r] = 0.f;
  float ab2 = 0.f, aW1 = 0.f, ab1 = 0.f;
  __shared__ float H1[kBackPts][64], H2[kBackPts][128], G2[kBackPts][128], G1[kBackPts][64];
  __shared__ float XP[kBackPts][3];
  __shared__ int dpt[kBackPts];
  for (int d0 = 0; d0 < D; d0 += kBackPts) {
    const int nd = D - d0 < kBackPts ? D - d0 : kBackPts;
    // the points of this round
    for (int p = k; p < P; p += 256) {
      const int s = slot[p];
      if (s >= d0 && s < d0 + nd) dpt[s - d0] = p;
    }
    __syncthreads();
    if (k < kBackPts) {
      float x0 = 0.f, x1 = 0.f, x2 = 0.f;
      if (k < nd) load_point(Xn, Yn, P, idx, cloud, dpt[k], x0, x1, x2);
      XP[k][0] = x0;
      XP[k][1] = x1;
      XP[k][2] = x2;
    }
    __syncthreads();
    for (int e = k; e < kBackPts * 64; e += 256) {
      const int d = e / 64, c = e % 64;
      const float v = fmaf(th[oW1 + 3 * c], XP[d][0],
                           fmaf(th[oW1 + 3 * c + 1], XP[d][1], fmaf(th[oW1 + 3 * c + 2], XP[d][2], th[oB1 + c])));
      H1[d][c] = fmaxf(v, 0.f);
    }
    __syncthreads();
    for (int e = k; e < kBackPts * 128; e += 256) {
      const int d = e / 128, j = e % 128;
      float v = th[oB2 + j];
      const float *w = th + oW2 + j * 64;
      for (int i = 0; i < 64; ++i) v = fmaf(w[i], H1[d][i], v);
      H2[d][j] = fmaxf(v, 0.f);
    }
    __syncthreads();
    // gradient at layer 2's output, through its ReLU
    for (int e = k; e < kBackPts * 128; e += 256) {
      const int d = e / 128, j = e % 128;
      float g = 0.f;
      if (d < nd)
        for (int c = 0; c < 256; ++c)
          if (kslot[c] == d0 + d) g = fmaf(kg[c], th[oW3 + c * 128 + j], g);
      G2[d][j] = H2[d][j] > 0.f ? g : 0.f;
    }
    // W3 rows of the channels pooled at this round's points
    if (sk >= d0 && sk < d0 + nd)
      for (int j = 0; j < 128; ++j) gp[oW3 + k * 128 + j] = gk * H2[sk - d0][j];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 32; ++r) {
      const int e = k + 256 * r, j = e / 64, i = e % 64;
      float s = aW2[r];
      for (int d = 0; d < nd; ++d) s = fmaf(G2[d][j], H1[d][i], s);
      aW2[r] = s;
    }
    if (k < 128)
      for (int d = 0; d < nd; ++d) ab2 += G2[d][k];
    // gradient at layer 1's output, through its ReLU
    for (int e = k; e < kBackPts * 64; e += 256) {
      const int d = e / 64, i = e % 64;
      float g = 0.f;
      for (int j = 0; j < 128; ++j) g = fmaf(G2[d][j], th[oW2 + j * 64 + i], g);
      G1[d][i] = H1[d][i] > 0.f ? g : 0.f;
    }
    __syncthreads();
    if (k < 192) {
      const int i = k / 3, a = k % 3;
      for (int d = 0; d < nd; ++d) aW1 = fmaf(G1[d][i], XP[d][a], aW1);
    }
    if (k < 64)
      for (int d = 0; d < nd; ++d) ab1 += G1[d][k];
    __syncthreads();
  }
  if (!live || sk < 0)
    for (int j = 0; j < 128; ++j) gp[oW3 + k * 128 + j] = 0.f;
#pragma unroll
  for (int r = 0; r < 32; ++r) gp[oW2 + k + 256 * r] = aW2[r];
  if (k < 128) gp[oB2 + k] = ab2;
  if (k < 192) gp[oW1 + k] = aW1;
  if (k < 64) gp[oB1 + k] = ab1;
}

// grad[e] for every parameter: encoder entries summed over the clouds, head
// entries over the pairs, each in increasing order.
__global__ void prop_grad_sum(const float *__restrict__ part, int nclouds,
                              const float *__restrict__ z, const float *__restrict__ h4,
                              const float *__restrict__ go, const float *__restrict__ ga4, int B,
                              float *__restrict__ grad) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= kNP) return;
  float s = 0.f;
  if (e < kEncParams) {
    for (int c = 0; c < nclouds; ++c) s += part[(size_t)c * kEncParams + e];
  } else if (e < oB4) {
    const int u = (e - oW4) / 512, i = (e - oW4) % 512;
    for (int b = 0; b < B; ++b) s = fmaf(ga4[(size_t)b * 128 + u], z[(size_t)b * 512 + i], s);
  } else if (e < oW5) {
    const int u = e - oB4;
    for (int b = 0; b < B; ++b) s += ga4[(size_t)b * 128 + u];
  } else if (e < oB5) {
    const int q = (e - oW5) / 128, u = (e - oW5) % 128;
    for (int b = 0; b < B; ++b) s = fmaf(go[b * 9 + q], h4[(size_t)b * 128 + u], s);
  } else {
    const int q = e - oB5;
    for (int b = 0; b < B; ++b) s += go[b * 9 + q];
  }
  grad[e] = s;
}

// Pooled point of every (cloud, channel) (test aid).
__global__ void prop_argmax(const unsigned long long *__restrict__ pool, int *__restrict__ out) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  out[i] = pooled_point(pool[i]);
}

__global__ void prop_adam(float *__restrict__ th, float *__restrict__ m, float *__restrict__ v,
                          const float *__restrict__ grad, float lr, float c1, float c2) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= kNP) return;
  const float g = grad[e];
  const float mm = 0.9f * m[e] + 0.1f * g;
  const float vv = 0.999f * v[e] + 0.001f * g * g;
  m[e] = mm;
  v[e] = vv;
  th[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + 1e-8f);
}

}  // namespace

size_t prop_workspace_bytes(int npairs, int train) {
  size_t b = 0;
  auto add = [&b](size_t n) { b += (n + 255) / 256 * 256; };
  add((size_t)(64 * 128 + 128 * 256) * sizeof(float));          // transposed W2, W3
  add((size_t)2 * npairs * 256 * sizeof(unsigned long long));    // pooled keys
  if (train) {
    add((size_t)npairs * (512 + 128 + 9 + 128 + 512) * sizeof(float));
    add((size_t)2 * npairs * kEncParams * sizeof(float));        // per-cloud parts
    add((size_t)kNP * sizeof(float));                            // gradient
  }
  return b;
}

namespace {
struct PropWs {
  float *wt;
  unsigned long long *pool;
  float *z, *h4, *go, *ga4, *gz, *part, *grad;
};
PropWs prop_ws(void *ws, int npairs, int train) {
  char *p = (char *)ws;
  auto take = [&p](size_t n) {
    char *q = p;
    p += (n + 255) / 256 * 256;
    return (void *)q;
  };
  PropWs w = {};
  w.wt = (float *)take((size_t)(64 * 128 + 128 * 256) * sizeof(float));
  w.pool = (unsigned long long *)take((size_t)2 * npairs * 256 * sizeof(unsigned long long));
  if (train) {
    float *f = (float *)take((size_t)npairs * (512 + 128 + 9 + 128 + 512) * sizeof(float));
    w.z = f;
    w.h4 = f + (size_t)npairs * 512;
    w.go = w.h4 + (size_t)npairs * 128;
    w.ga4 = w.go + (size_t)npairs * 9;
    w.gz = w.ga4 + (size_t)npairs * 128;
    w.part = (float *)take((size_t)2 * npairs * kEncParams * sizeof(float));
    w.grad = (float *)take((size_t)kNP * sizeof(float));
  }
  return w;
}

void encode_launch(const float *theta, const PropWs &w, int npairs, int P, const float *Xn,
                   const float *Yn, const int *idx, hipStream_t st) {
  const int n = 256 * 128;
  const int npool = 2 * npairs * 256;
  const int m = n > npool ? n : npool;
  hipLaunchKernelGGL(prop_prepare, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, theta, w.wt,
                     w.pool, npool);
  hipLaunchKernelGGL(prop_encode, dim3((unsigned)((P + kChunk - 1) / kChunk), (unsigned)(2 * npairs)),
                     dim3(256), 0, st, theta, w.wt, Xn, Yn, P, idx, w.pool);
}
}  // namespace

hipError_t launch_prop_inputs(const PropPair *pairs, int npairs, const double *Q, int P, float *Xn,
                              float *Yn, double *norm, hipStream_t st) {
  hipLaunchKernelGGL(prop_inputs, dim3((unsigned)npairs), dim3(256), 0, st, pairs, Q, P, Xn, Yn, norm);
  return hipGetLastError();
}

hipError_t launch_prop_forward(const float *theta, int npairs, int P, const float *Xn,
                               const float *Yn, const double *norm, double *pose, void *ws,
                               hipStream_t st) {
  const PropWs w = prop_ws(ws, npairs, 0);
  encode_launch(theta, w, npairs, P, Xn, Yn, nullptr, st);
  hipLaunchKernelGGL(prop_head, dim3((unsigned)npairs), dim3(128), 0, st, theta, w.pool, norm, pose);
  return hipGetLastError();
}

hipError_t launch_prop_train(float *theta, float *m, float *v, int step, double lr, int npairs,
                             int P, const float *Xn, const float *Yn, const double *norm,
                             const int *idx, const double *label, double *loss, int *argmax,
                             float *grad_out, void *ws, hipStream_t st) {
  const PropWs w = prop_ws(ws, npairs, 1);
  encode_launch(theta, w, npairs, P, Xn, Yn, idx, st);
  hipLaunchKernelGGL(prop_head_train, dim3((unsigned)npairs), dim3(128), 0, st, theta, w.pool, norm,
                     idx, label, npairs, loss, w.z, w.h4, w.go, w.ga4, w.gz);
  hipLaunchKernelGGL(prop_encode_back, dim3((unsigned)(2 * npairs)), dim3(256), 0, st, theta, Xn, Yn,
                     P, idx, w.pool, w.gz, w.part);
  hipLaunchKernelGGL(prop_grad_sum, dim3((unsigned)((kNP + 255) / 256)), dim3(256), 0, st, w.part,
                     2 * npairs, w.z, w.h4, w.go, w.ga4, npairs, grad_out ? grad_out : w.grad);
  if (argmax)
    hipLaunchKernelGGL(prop_argmax, dim3((unsigned)(2 * npairs)), dim3(256), 0, st, w.pool, argmax);
  const double c1 = 1.0 - pow(0.9, step), c2 = 1.0 - pow(0.999, step);
  hipLaunchKernelGGL(prop_adam, dim3((unsigned)((kNP + 255) / 256)), dim3(256), 0, st, theta, m, v,
                     grad_out ? grad_out : w.grad, (float)lr, (float)c1, (float)c2);
  return hipGetLastError();
}

}  // namespace lsg
