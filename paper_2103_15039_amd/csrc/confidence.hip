// Confidence filtering (Sec. 3.3) and the outlier weight from the outlier
// ratio (Sec. 3.2):
//   * the measurement confidence of depth-sensor points, phi = e_min / e(z)
//     for the error model e(z) = c0 + c1 z + c2 z^2 of the depth z (points
//     whose modelled error is at most e_min get phi = 1);
//   * truncation: the points with phi >= threshold, in their original order;
//   * the target sums behind the priors pi(m) = phi(y_m) / sum phi and behind
//     w_max: sum_m phi_m and sum_m pi(m) c_m (2 pi sigma^2)^{3/2}, the bound
//     c_m of the component density of Eq. 2 without its sigma^2 factor.
#include <rocprim/device/device_select.hpp>
#include <rocprim/iterator/counting_iterator.hpp>

#include "lsgcpd_internal.h"

namespace lsg {

namespace {

__global__ void depth_confidence(const float *__restrict__ P, int64_t n, double c0, double c1,
                                 double c2, double e_min, float *__restrict__ phi) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double z = (double)P[3 * i + 2];
  const double e = c0 + c1 * z + c2 * (z * z);
  phi[i] = e <= e_min ? 1.0f : (float)(e_min / e);
}

__global__ void confident_flags(const float *__restrict__ phi, int64_t n, double threshold,
                                unsigned char *__restrict__ flags) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) flags[i] = (double)phi[i] >= threshold ? 1 : 0;
}

// Points and confidences of the selected indices; `count` (device) bounds
// the output.
__global__ void gather_selected(const float *__restrict__ P, const float *__restrict__ phi,
                                const uint32_t *__restrict__ idx,
                                const uint32_t *__restrict__ count, int64_t n,
                                float *__restrict__ Pout, float *__restrict__ phiout) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || i >= (int64_t)*count) return;
  const int64_t j = idx[i];
  Pout[3 * i] = P[3 * j];
  Pout[3 * i + 1] = P[3 * j + 1];
  Pout[3 * i + 2] = P[3 * j + 2];
  phiout[i] = phi[j];
}

__global__ void gather_f32(const float *__restrict__ src, const uint32_t *__restrict__ perm,
                           int64_t n, float *__restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[perm[i]];
}

constexpr int kPriorBlock = 256;

// Block partials of (sum phi_m, sum phi_m chat_m), chat_m = sqrt(1 + alpha_m)
// with the exact normaliser, else 1; phi null => phi_m = 1.
__global__ __launch_bounds__(kPriorBlock) void prior_partial(const float *__restrict__ phi,
                                                            const float *__restrict__ alpha,
                                                            int64_t M, int exact,
                                                            double *__restrict__ part) {
  double s0 = 0.0, s1 = 0.0;
  for (int64_t m = (int64_t)blockIdx.x * kPriorBlock + threadIdx.x; m < M;
       m += (int64_t)gridDim.x * kPriorBlock) {
    const double f = phi ? (double)phi[m] : 1.0;
    const double c = exact ? sqrt(1.0 + (double)alpha[m]) : 1.0;
    s0 += f;
    s1 += f * c;
  }
  __shared__ double r0[kPriorBlock], r1[kPriorBlock];
  r0[threadIdx.x] = s0;
  r1[threadIdx.x] = s1;
  __syncthreads();
  for (int h = kPriorBlock / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      r0[threadIdx.x] += r0[threadIdx.x + h];
      r1[threadIdx.x] += r1[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = r0[0];
    part[2 * blockIdx.x + 1] = r1[0];
  }
}

__global__ __launch_bounds__(kPriorBlock) void prior_final(const double *__restrict__ part,
                                                          int nblk, DevState *__restrict__ s) {
  __shared__ double r0[kPriorBlock], r1[kPriorBlock];
  double s0 = 0.0, s1 = 0.0;
  for (int b = threadIdx.x; b < nblk; b += kPriorBlock) {
    s0 += part[2 * b];
    s1 += part[2 * b + 1];
  }
  r0[threadIdx.x] = s0;
  r1[threadIdx.x] = s1;
  __syncthreads();
  for (int h = kPriorBlock / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      r0[threadIdx.x] += r0[threadIdx.x + h];
      r1[threadIdx.x] += r1[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    s->pi_sum = r0[0];
    s->pic = r1[0] / r0[0];
  }
}

inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

hipError_t launch_depth_confidence(const float *P, int64_t n, const double coef[3], double e_min,
                                   float *phi, hipStream_t st) {
  hipLaunchKernelGGL(depth_confidence, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, P, n,
                     coef[0], coef[1], coef[2], e_min, phi);
  return hipGetLastError();
}

size_t select_workspace_bytes(int64_t n) {
  size_t tmp = 0;
  uint32_t *nul = nullptr;
  unsigned char *fl = nullptr;
  if (rocprim::select(nullptr, tmp, rocprim::counting_iterator<uint32_t>(0), fl, nul, nul,
                      (size_t)n) != hipSuccess)
    tmp = 0;
  // flags + indices + count + select scratch
  return align256((size_t)n) + align256((size_t)n * sizeof(uint32_t)) + 256 + tmp + 256;
}

hipError_t launch_select_confident(const float *P, const float *phi, int64_t n, double threshold,
                                   void *work, size_t work_bytes, float *Pout, float *phiout,
                                   uint32_t *count, hipStream_t st) {
  if (work_bytes < select_workspace_bytes(n)) return hipErrorInvalidValue;
  char *w = (char *)work;
  unsigned char *flags = (unsigned char *)w;
  uint32_t *idx = (uint32_t *)(w + align256((size_t)n));
  char *tmp = (char *)idx + align256((size_t)n * sizeof(uint32_t));
  size_t tmp_bytes = work_bytes - (size_t)(tmp - w);
  const unsigned blocks = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(confident_flags, dim3(blocks), dim3(256), 0, st, phi, n, threshold, flags);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = rocprim::select(tmp, tmp_bytes, rocprim::counting_iterator<uint32_t>(0), flags, idx, count,
                      (size_t)n, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(gather_selected, dim3(blocks), dim3(256), 0, st, P, phi, idx, count, n, Pout,
                     phiout);
  return hipGetLastError();
}

hipError_t launch_gather_f32(const float *src, const uint32_t *perm, int64_t n, float *dst,
                             hipStream_t st) {
  hipLaunchKernelGGL(gather_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, perm, n,
                     dst);
  return hipGetLastError();
}

int prior_blocks(int64_t M) {
  int64_t b = (M + kPriorBlock - 1) / kPriorBlock;
  if (b > 256) b = 256;
  if (b < 1) b = 1;
  return (int)b;
}

hipError_t launch_prior_sums(const float *phi, const float *alpha, int64_t M, int exact,
                             double *partials, DevState *s, hipStream_t st) {
  const int nb = prior_blocks(M);
  hipLaunchKernelGGL(prior_partial, dim3((unsigned)nb), dim3(kPriorBlock), 0, st, phi, alpha, M,
                     exact, partials);
  hipLaunchKernelGGL(prior_final, dim3(1), dim3(kPriorBlock), 0, st, partials, nb, s);
  return hipGetLastError();
}

}  // namespace lsg
