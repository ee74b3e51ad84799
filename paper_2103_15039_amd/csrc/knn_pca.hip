// Target geometry on the GPU (Sec. 3.1 and Eq. 3 of LSG-CPD): brute-force k
// nearest neighbours, FP64 3x3 PCA of each neighbourhood, surface variation
// kappa and the penalty alpha.
//
// Pass 1 (knn_partial): the target range is split into `nsplit` chunks; block
// (qb, split) streams its chunk through LDS in tiles and every thread keeps the
// k best (distance, index) pairs of one query in registers.  Distances are
// float32 ((dx*dx + dy*dy) + dz*dz), no contraction, so that the neighbour set
// is decided exactly as the float32 definition says; pairs are ordered by the
// 64-bit key (distance bits, index), i.e. by distance with ties to the lower
// index.  Before the scan each query takes, as an upper bound tau0 of its k-th
// distance, the k-th smallest distance to its 2k+1 index neighbours; only keys
// <= (tau0, any index) can belong to the answer, so the list starts filled
// with (tau0, +inf) sentinels.  On clouds stored in scan or image order (index
// neighbours are spatial neighbours) this removes almost all list updates;
// the result is exact for any order.
// Pass 2 (knn_merge_pca): one thread per query merges the nsplit partial
// lists, forms the neighbourhood covariance about its mean in FP64 and
// diagonalises it by cyclic Jacobi rotations.
#include <math.h>

#include "lsgcpd_internal.h"

namespace lsg {

namespace {

constexpr int kKnnBlock = 256;
constexpr int kKnnTile = 256;
constexpr uint32_t kNoIndex = 0xffffffffu;

__device__ __forceinline__ float dist2_f32(float ax, float ay, float az, float bx, float by,
                                           float bz) {
#pragma clang fp contract(off)
  const float dx = ax - bx;
  const float dy = ay - by;
  const float dz = az - bz;
  return (dx * dx + dy * dy) + dz * dz;
}

__device__ __forceinline__ uint64_t make_key(float d, uint32_t i) {
  return ((uint64_t)__float_as_uint(d) << 32) | (uint64_t)i;
}
__device__ __forceinline__ float key_dist(uint64_t k) { return __uint_as_float((uint32_t)(k >> 32)); }
__device__ __forceinline__ uint32_t key_index(uint64_t k) { return (uint32_t)k; }

// The KM smallest keys seen so far, sorted, in registers (all indices are
// compile-time constants, so nothing spills).  The caller uses the first
// k <= KM entries; `worst` is the k-th key, the bound a new key must beat.
template <int KM>
struct TopK {
  uint64_t key[KM];
  uint64_t worst;
  int k;

  __device__ __forceinline__ void init(int k_, uint64_t fill) {
    k = k_;
#pragma unroll
    for (int j = 0; j < KM; ++j) key[j] = fill;
    worst = fill;
  }

  // one bubbling pass: the new key moves past every smaller key
  __device__ __forceinline__ void insert(uint64_t kn) {
    uint64_t c = kn;
#pragma unroll
    for (int j = 0; j < KM; ++j) {
      const uint64_t o = key[j];
      const bool lt = c < o;
      key[j] = lt ? c : o;
      c = lt ? o : c;
    }
    uint64_t w = key[0];
#pragma unroll
    for (int j = 1; j < KM; ++j) w = (j == k - 1) ? key[j] : w;
    worst = w;
  }

  __device__ __forceinline__ void offer(uint64_t kn) {
    if (kn < worst) insert(kn);
  }
};

// tau0: k-th smallest distance from query q to its 2k+1 index neighbours.
template <int KM>
__device__ float index_window_bound(const float *__restrict__ Y, int M, int k, int q, float qx,
                                    float qy, float qz) {
  TopK<KM> t;
  t.init(k, ~(uint64_t)0);
  int lo = q - k, hi = q + k;
  if (lo < 0) {
    hi -= lo;
    lo = 0;
  }
  if (hi > M - 1) {
    lo -= hi - (M - 1);
    hi = M - 1;
    if (lo < 0) lo = 0;
  }
  for (int j = lo; j <= hi; ++j)
    t.offer(make_key(dist2_f32(qx, qy, qz, Y[3 * j], Y[3 * j + 1], Y[3 * j + 2]), (uint32_t)j));
  return key_dist(t.worst);
}

template <int KM>
__global__ __launch_bounds__(kKnnBlock) void knn_partial(const float *__restrict__ Y, int M,
                                                         int k, int chunk,
                                                         uint64_t *__restrict__ out) {
  const int split = blockIdx.y;
  const int q = blockIdx.x * kKnnBlock + threadIdx.x;
  const int j0 = split * chunk;
  const int j1 = min(M, j0 + chunk);
  float qx = 0.f, qy = 0.f, qz = 0.f;
  float tau = 0.f;
  if (q < M) {
    qx = Y[3 * q];
    qy = Y[3 * q + 1];
    qz = Y[3 * q + 2];
    tau = index_window_bound<KM>(Y, M, k, q, qx, qy, qz);
  }
  __shared__ float4 tile[kKnnTile];
  TopK<KM> top;
  top.init(k, make_key(tau, kNoIndex));
  for (int jt = j0; jt < j1; jt += kKnnTile) {
    const int cnt = min(kKnnTile, j1 - jt);
    if (threadIdx.x < cnt) {
      const int j = jt + threadIdx.x;
      tile[threadIdx.x] = make_float4(Y[3 * j], Y[3 * j + 1], Y[3 * j + 2], 0.f);
    }
    __syncthreads();
    for (int jj = 0; jj < cnt; ++jj) {
      const float4 p = tile[jj];
      const float d = dist2_f32(qx, qy, qz, p.x, p.y, p.z);
      // cheap float test first; the exact key order decides inside
      if (d <= key_dist(top.worst)) top.offer(make_key(d, (uint32_t)(jt + jj)));
    }
    __syncthreads();
  }
  if (q < M) {
#pragma unroll
    for (int j = 0; j < KM; ++j)
      if (j < k) out[((size_t)split * k + j) * M + q] = top.key[j];
  }
}

// Symmetric 3x3 eigen-decomposition by cyclic Jacobi rotations (FP64).
// On return a holds the eigenvalues on its diagonal and v the eigenvectors as
// columns.
__device__ void jacobi3(double a[3][3], double v[3][3]) {
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

template <int KM>
__global__ __launch_bounds__(256) void knn_merge_pca(const float *__restrict__ Y, int M, int k,
                                                     int nsplit,
                                                     const uint64_t *__restrict__ keys,
                                                     double alpha_max, double lambda,
                                                     float *__restrict__ normals,
                                                     float *__restrict__ kappa,
                                                     float *__restrict__ alpha) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= M) return;
  TopK<KM> top;
  top.init(k, ~(uint64_t)0);
  for (int s = 0; s < nsplit; ++s)
    for (int j = 0; j < k; ++j) {
      const uint64_t kk = keys[((size_t)s * k + j) * M + q];
      if (key_index(kk) < (uint32_t)M) top.offer(kk);
    }
  // every slot holds a valid index unless the inputs were not finite; such
  // slots fall back to the query point itself
  int idx[KM];
#pragma unroll
  for (int j = 0; j < KM; ++j) {
    const uint32_t i = key_index(top.key[j]);
    idx[j] = i < (uint32_t)M ? (int)i : q;
  }
  double mx = 0.0, my = 0.0, mz = 0.0;
#pragma unroll
  for (int j = 0; j < KM; ++j) {
    if (j < k) {
      mx += (double)Y[3 * idx[j]];
      my += (double)Y[3 * idx[j] + 1];
      mz += (double)Y[3 * idx[j] + 2];
    }
  }
  const double invk = 1.0 / (double)k;
  mx *= invk;
  my *= invk;
  mz *= invk;
  double c00 = 0, c01 = 0, c02 = 0, c11 = 0, c12 = 0, c22 = 0;
#pragma unroll
  for (int j = 0; j < KM; ++j) {
    if (j < k) {
      const double dx = (double)Y[3 * idx[j]] - mx;
      const double dy = (double)Y[3 * idx[j] + 1] - my;
      const double dz = (double)Y[3 * idx[j] + 2] - mz;
      c00 += dx * dx;
      c01 += dx * dy;
      c02 += dx * dz;
      c11 += dy * dy;
      c12 += dy * dz;
      c22 += dz * dz;
    }
  }
  double a[3][3] = {{c00 * invk, c01 * invk, c02 * invk},
                    {c01 * invk, c11 * invk, c12 * invk},
                    {c02 * invk, c12 * invk, c22 * invk}};
  const double tr = a[0][0] + a[1][1] + a[2][2];
  double nx = 0.0, ny = 0.0, nz = 1.0, kap = 1.0 / 3.0;
  if (tr > 0.0) {
    double v[3][3];
    jacobi3(a, v);
    int imin = 0;
    if (a[1][1] < a[imin][imin]) imin = 1;
    if (a[2][2] < a[imin][imin]) imin = 2;
    nx = v[0][imin];
    ny = v[1][imin];
    nz = v[2][imin];
    const double nn = sqrt(nx * nx + ny * ny + nz * nz);
    nx /= nn;
    ny /= nn;
    nz /= nn;
    kap = fmin(fmax(a[imin][imin] / tr, 0.0), 1.0 / 3.0);
  }
  double al;
  if (kap <= 0.0) {
    al = alpha_max;
  } else {
    const double u = exp(lambda * (3.0 - 1.0 / kap));
    al = fmax((1.0 - u) / (1.0 + u) * alpha_max, 0.0);
  }
  normals[3 * q] = (float)nx;
  normals[3 * q + 1] = (float)ny;
  normals[3 * q + 2] = (float)nz;
  if (kappa) kappa[q] = (float)kap;
  alpha[q] = (float)al;
}

}  // namespace

int knn_choose_splits(int64_t M) {
  const int64_t qb = (M + kKnnBlock - 1) / kKnnBlock;
  int64_t ns = (1536 + qb - 1) / qb;
  const int64_t cap = M / 512 > 1 ? M / 512 : 1;
  if (ns > cap) ns = cap;
  if (ns > 64) ns = 64;
  if (ns < 1) ns = 1;
  return (int)ns;
}

size_t knn_workspace_bytes(int64_t M, int nsplit) {
  return (size_t)nsplit * 32 * (size_t)M * sizeof(uint64_t);
}

hipError_t launch_normals(const float *Y, int64_t M, int k, double alpha_max, double lambda,
                          float *normals, float *kappa, float *alpha, void *work, int nsplit,
                          hipStream_t st) {
  const int Mi = (int)M;
  const int chunk = (int)((M + nsplit - 1) / nsplit);
  uint64_t *keys = (uint64_t *)work;
  dim3 g1((unsigned)((M + kKnnBlock - 1) / kKnnBlock), (unsigned)nsplit);
  dim3 g2((unsigned)((M + 255) / 256));
#define LSG_KNN(KM_)                                                                         \
  do {                                                                                       \
    hipLaunchKernelGGL(knn_partial<KM_>, g1, dim3(kKnnBlock), 0, st, Y, Mi, k, chunk, keys); \
    hipLaunchKernelGGL(knn_merge_pca<KM_>, g2, dim3(256), 0, st, Y, Mi, k, nsplit, keys,     \
                       alpha_max, lambda, normals, kappa, alpha);                            \
  } while (0)
  if (k <= 8) LSG_KNN(8);
  else if (k <= 16) LSG_KNN(16);
  else if (k <= 20) LSG_KNN(20);
  else LSG_KNN(32);
#undef LSG_KNN
  return hipGetLastError();
}

}  // namespace lsg
