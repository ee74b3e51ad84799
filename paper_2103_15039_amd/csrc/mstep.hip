// The LSG-CPD M step on gfx950 (Sec. 3.5, Eq. 11-13): deterministic reduction
// of the per-block statistics, then Newton's method on SE(3) in FP64.
//
// With the 86 statistics of one E step the objective of Eq. 6 in g is, up to
// constants, D(G) / (2 sigma^2) with
//   D(G) = vec(G)^T H vec(G) - 2 b^T vec(G) + c,   G = [R | t] (3 x 4),
// H[4a+i][4b+j] = delta_ab S0[i][j] + S1[ab][i][j], b = vec(S2), c = S3,
// an exact quadratic in the 12 entries of G.  Newton steps are taken on the
// group: G <- G exp(xi^), xi = -Hs^{-1} grad, where grad and the symmetrised
// Hessian Hs are the right derivatives of Eq. 11-12 (divided, as printed, by
// sigma^2).  If Hs is not positive definite the Gauss-Newton part is used
// through its minimum-norm least-squares solution;
// steps are halved until D does not grow beyond a rounding allowance (the
// change of D is evaluated as the exact difference of the quadratic).  After
// the pose, sigma^2 = D(G_new) / (3 N_P) (Sec. 3.5, last paragraph).
// reduce_stats sums the block statistics with one block per statistic and
// problem; reduce_mstep runs the Newton iteration of each problem of a batch
// in one block, whose threads share the 12 x 12 products and the entries of
// the gradient and Hessian while thread 0 does the 6 x 6 Cholesky solve and
// the exponential map.
#include <math.h>

#include "lsgcpd_internal.h"

namespace lsg {

namespace {

constexpr double kTwoPi = 6.283185307179586477;

// SE(3) exponential of the twist xi = (omega, v): Rodrigues rotation and the
// left Jacobian of SO(3) for the translation.
__device__ void se3_exp(const double xi[6], double Rx[3][3], double tx[3]) {
  const double w0 = xi[0], w1 = xi[1], w2 = xi[2];
  const double th2 = w0 * w0 + w1 * w1 + w2 * w2;
  const double th = sqrt(th2);
  double A, B, C;
  if (th < 1e-6) {
    A = 1.0 - th2 / 6.0;
    B = 0.5 - th2 / 24.0;
    C = 1.0 / 6.0 - th2 / 120.0;
  } else {
    double sn, cs;
    sincos(th, &sn, &cs);
    const double it = 1.0 / th, it2 = it * it;
    A = sn * it;
    B = (1.0 - cs) * it2;
    C = (th - sn) * (it2 * it);
  }
  const double W[3][3] = {{0.0, -w2, w1}, {w2, 0.0, -w0}, {-w1, w0, 0.0}};
  double W2[3][3];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += W[r][k] * W[k][c];
      W2[r][c] = s;
    }
  double Vm[3][3];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      const double I = r == c ? 1.0 : 0.0;
      Rx[r][c] = I + A * W[r][c] + B * W2[r][c];
      Vm[r][c] = I + B * W[r][c] + C * W2[r][c];
    }
  for (int r = 0; r < 3; ++r) tx[r] = Vm[r][0] * xi[3] + Vm[r][1] * xi[4] + Vm[r][2] * xi[5];
}

// g_out = vec(G exp(xi^)) for g = vec(G), G = [R | t] (3 x 4 row-major)
__device__ void compose(const double *g, const double xi[6], double *gout) {
  double Rx[3][3], tx[3];
  se3_exp(xi, Rx, tx);
  for (int a = 0; a < 3; ++a) {
    const double *G = g + 4 * a;
    for (int c = 0; c < 3; ++c) gout[4 * a + c] = G[0] * Rx[0][c] + G[1] * Rx[1][c] + G[2] * Rx[2][c];
    gout[4 * a + 3] = G[0] * tx[0] + G[1] * tx[1] + G[2] * tx[2] + G[3];
  }
}

// Cholesky solve of the 6x6 system A x = -g; false if A is not positive
// definite.  One reciprocal per column: the divisions are the long-latency
// steps of this serial code.
__device__ bool chol_solve6(const double A[6][6], const double g[6], double x[6]) {
  double L[6][6], inv[6];
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) L[i][j] = 0.0;
  for (int j = 0; j < 6; ++j) {
    double d = A[j][j];
    for (int k = 0; k < j; ++k) d -= L[j][k] * L[j][k];
    if (!(d > 0.0)) return false;
    L[j][j] = sqrt(d);
    inv[j] = 1.0 / L[j][j];
    for (int i = j + 1; i < 6; ++i) {
      double s = A[i][j];
      for (int k = 0; k < j; ++k) s -= L[i][k] * L[j][k];
      L[i][j] = s * inv[j];
    }
  }
  double y[6];
  for (int i = 0; i < 6; ++i) {
    double s = -g[i];
    for (int k = 0; k < i; ++k) s -= L[i][k] * y[k];
    y[i] = s * inv[i];
  }
  for (int i = 5; i >= 0; --i) {
    double s = y[i];
    for (int k = i + 1; k < 6; ++k) s -= L[k][i] * x[k];
    x[i] = s * inv[i];
  }
  return true;
}

// Minimum-norm least-squares solution of A x = -g for the symmetric 6x6
// Gauss-Newton matrix A (singular for degenerate inputs such as a single
// source point, whose rotations about itself are free): eigen-decomposition by cyclic Jacobi rotations, then
//   x = -sum_i (v_i . g / lambda_i) v_i  over |lambda_i| > 6 eps max|lambda|,
// the pseudo-inverse a singular-value solve with that cutoff gives (for a
// symmetric matrix the singular values are the |lambda_i|).  False if A is 0.
__device__ bool pinv_solve6(const double Ain[6][6], const double g[6], double x[6]) {
  double a[6][6], v[6][6];
  for (int r = 0; r < 6; ++r)
    for (int c = 0; c < 6; ++c) {
      a[r][c] = Ain[r][c];
      v[r][c] = r == c ? 1.0 : 0.0;
    }
  for (int sweep = 0; sweep < 50; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (int r = 0; r < 6; ++r) {
      dia += a[r][r] * a[r][r];
      for (int c = r + 1; c < 6; ++c) off += a[r][c] * a[r][c];
    }
    if (off == 0.0 || off <= 1e-36 * dia) break;
    for (int p = 0; p < 5; ++p)
      for (int q = p + 1; q < 6; ++q) {
        const double apq = a[p][q];
        if (apq == 0.0) continue;
        const double theta = (a[q][q] - a[p][p]) / (2.0 * apq);
        const double t = fabs(theta) > 1e150
                             ? 0.5 / theta
                             : (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0);
        const double sn = t * c;
        for (int k = 0; k < 6; ++k) {  // columns p, q
          const double akp = a[k][p], akq = a[k][q];
          a[k][p] = c * akp - sn * akq;
          a[k][q] = sn * akp + c * akq;
        }
        for (int k = 0; k < 6; ++k) {  // rows p, q
          const double apk = a[p][k], aqk = a[q][k];
          a[p][k] = c * apk - sn * aqk;
          a[q][k] = sn * apk + c * aqk;
        }
        a[p][q] = a[q][p] = 0.0;
        for (int k = 0; k < 6; ++k) {
          const double vkp = v[k][p], vkq = v[k][q];
          v[k][p] = c * vkp - sn * vkq;
          v[k][q] = sn * vkp + c * vkq;
        }
      }
  }
  double mx = 0.0;
  for (int i = 0; i < 6; ++i) mx = fmax(mx, fabs(a[i][i]));
  if (!(mx > 0.0) || !isfinite(mx)) return false;
  const double cut = 6.0 * 2.220446049250313e-16 * mx;
  for (int i = 0; i < 6; ++i) x[i] = 0.0;
  for (int j = 0; j < 6; ++j) {
    const double lam = a[j][j];
    if (!(fabs(lam) > cut)) continue;
    double d = 0.0;
    for (int k = 0; k < 6; ++k) d += v[k][j] * g[k];
    const double f = -d / lam;
    for (int k = 0; k < 6; ++k) x[k] += f * v[k][j];
  }
  return true;
}

// Shared state of the block-parallel M step.
struct MSh {
  double H[12][12];   // H[4a+i][4b+j] = delta_ab S0[i][j] + S1[ab][i][j]
  double b[12];       // vec(S2)
  double c;           // S3
  double g[12];       // vec(G), the current pose
  double gn[12];      // trial pose
  double J[6][12];    // vec(G E_i) of the six generators
  double HJ[6][12];
  double Hg[12];
  double GN[6][6];
  double Q[3][3], w[3];   // R^T (H g - b), split as the second-order term uses it
  double Hs[6][6], Hgn[6][6], grad[6];
  double xi[6];
  double cur, val, step;
  int go;             // 1 while Newton continues
  int accept;
};

__device__ __forceinline__ int pair_index(int a, int b) {
  const int lo = a < b ? a : b, hi = a < b ? b : a;  // (00 01 02 11 12 22)
  return lo == 0 ? hi : (lo == 1 ? 2 + hi : 5);
}

// upper-triangle position of (i, j) in the 4x4 packing (00 01 02 03 11 12 13 22 23 33)
__device__ __forceinline__ int tri4(int i, int j) {
  const int lo = i < j ? i : j, hi = i < j ? j : i;
  const int base[4] = {0, 4, 7, 9};
  return base[lo] + hi - lo;
}

// D(vec) = v^T H v - 2 b^T v + c with the block's threads: rows in parallel.
__device__ double block_quad(MSh &m, const double *v, double *rowbuf) {
  const int tid = threadIdx.x;
  if (tid < 12) {
    double s = 0.0;
    for (int k = 0; k < 12; ++k) s = fma(m.H[tid][k], v[k], s);
    rowbuf[tid] = v[tid] * (s - 2.0 * m.b[tid]);
  }
  __syncthreads();
  double tot = m.c;
  for (int r = 0; r < 12; ++r) tot += rowbuf[r];
  __syncthreads();
  return tot;
}

// Problems with at most this many finalisation blocks (64 sources each) are
// summed by reduce_mstep itself: for them a kernel of its own costs more in
// launch latency than the sums.
constexpr int kFewBlocks = 64;

// Sum of row i of a problem's stat-major block statistics (one block per
// statistic and problem, so that the reads are spread over many CUs): thread
// t adds the partials t, t + 256, ... in order, then a fixed tree adds the
// threads.  The result does not depend on timing.
__global__ __launch_bounds__(256) void reduce_stats(const Slot *__restrict__ slots,
                                                     const double *__restrict__ blockstats,
                                                     DevState *__restrict__ states) {
  const int p = blockIdx.x / kStats, i = blockIdx.x % kStats, tid = threadIdx.x;
  DevState *s = states + p;
  const int nblk = slots[p].nfin;
  if (s->done || nblk <= kFewBlocks) return;  // reduce_mstep sums those itself
  const double *row = blockstats + (size_t)kStats * slots[p].fin_off + (size_t)i * nblk;
  double a = 0.0;
  for (int c0 = 0; c0 < nblk; c0 += 8 * 256) {
    double v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int b = c0 + k * 256 + tid;
      v[k] = b < nblk ? row[b] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) a += v[k];
  }
  __shared__ double r[256];
  r[tid] = a;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o) r[tid] += r[tid + o];
    __syncthreads();
  }
  if (tid == 0) s->stats[i] = r[0];
}

// The M step from the 86 statistics in s->stats.
__global__ __launch_bounds__(256) void reduce_mstep(const Slot *__restrict__ slots,
                                                    const double *__restrict__ blockstats,
                                                    DevState *__restrict__ states,
                                                    double *__restrict__ traces, int trace_stride,
                                                    const unsigned long long *__restrict__ evcounts,
                                                    int mode) {
  const int pidx = blockIdx.x;
  DevState *s = states + pidx;
  const int tid = threadIdx.x;
  // every value of the state this kernel reads, loaded together (the done
  // flag included) before the first write to the state, which would order
  // later loads after it: one round trip instead of a chain of them
  const int done = s->done;
  const int N = slots[pidx].N, nfin = slots[pidx].nfin, fin_off = slots[pidx].fin_off;
  const double sigma2 = s->sigma2, V = s->V, tol = s->tol, nll_prev = s->nll_prev;
  const double sigma2_floor = s->sigma2_floor;
  const int it0 = s->iter, newton_max = s->newton_max;
  double stat = 0.0;
  if (tid < kStats) {
    if (nfin <= kFewBlocks) {
      // the block partials of statistic tid, in order, the loads of 8 in flight
      const double *row = blockstats + (size_t)kStats * fin_off + (size_t)tid * nfin;
      for (int b0 = 0; b0 < nfin; b0 += 8) {
        double v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = b0 + k < nfin ? row[b0 + k] : 0.0;
#pragma unroll
        for (int k = 0; k < 8; ++k) stat += v[k];
      }
    } else {
      stat = s->stats[tid];
    }
  }
  double g0 = 0.0;
  if (tid < 12) {
    const int a = tid >> 2, j = tid & 3;
    g0 = j < 3 ? s->R[3 * a + j] : s->t[a];
  }
  const unsigned long long evc = evcounts && tid == 0 ? evcounts[pidx] : 0ull;
  if (done) return;
  double *trace = traces ? traces + (size_t)pidx * trace_stride : nullptr;
  if (evcounts && tid == 0) s->evaluated_pairs += (int64_t)evc;
  __shared__ double S[kStats];
  __shared__ MSh m;
  __shared__ double rowbuf[12];
  if (tid < kStats) {
    S[tid] = stat;
    if (nfin <= kFewBlocks) s->stats[tid] = stat;
  }
  __syncthreads();
  // the quadratic and the pose
  for (int e = tid; e < 144; e += blockDim.x) {
    const int r = e / 12, cc = e % 12;
    const int a = r >> 2, i = r & 3, bb = cc >> 2, k = cc & 3;
    double v = S[10 + 10 * pair_index(a, bb) + tri4(i, k)];
    if (a == bb) v += S[tri4(i, k)];
    m.H[r][cc] = v;
  }
  if (tid < 12) {
    m.b[tid] = S[70 + tid];
    m.g[tid] = g0;
  }
  if (tid == 0) m.c = S[82];
  __syncthreads();

  const double inv_s2 = 1.0 / sigma2;
  const double Np = S[9];
  const double nll = -(S[85] + S[83] - 1.5 * (double)N * log(kTwoPi * sigma2));
  double cur = block_quad(m, m.g, rowbuf);
  if (tid == 0) {
    s->gamma = pow(kTwoPi * sigma2, 1.5) / V;
    s->nll = nll;
    s->pd = cur;
    m.cur = cur;
    m.go = Np > 0.0 ? 1 : 0;
    if (mode == 1) {
      const int it = it0;
      if (trace) trace[it] = nll;
      if (tol > 0.0 && it > 0 && fabs(nll - nll_prev) <= tol * fabs(nll)) {
        s->done = 1;
        s->converged = 1;
        m.go = -1;
      } else {
        s->nll_prev = nll;
      }
    }
    if (mode == 0 && Np <= 0.0) {
      for (int i = 0; i < 6; ++i) s->grad[i] = 0.0;
      for (int i = 0; i < 36; ++i) s->hess[i] = 0.0;
    }
  }
  __syncthreads();
  if (m.go < 0) return;  // EM stopped by the tolerance (uniform)

  int iters = 0, gnf = 0;
  for (int itn = 0; itn < newton_max && m.go == 1; ++itn) {
    ++iters;
    // generators J_i = vec(G E_i): rotation i -> [R [e_i]x | 0], translation i -> [0 | R e_i]
    if (tid < 72) {
      const int i = tid / 12, r = tid % 12, a = r >> 2, c = r & 3;
      double v = 0.0;
      if (i < 3) {
        const int u = (i + 1) % 3, w = (i + 2) % 3;  // [e_i]x: (w, u) = 1, (u, w) = -1
        if (c == u) v = m.g[4 * a + w];
        else if (c == w) v = -m.g[4 * a + u];
      } else if (c == 3) {
        v = m.g[4 * a + (i - 3)];
      }
      m.J[i][r] = v;
    }
    __syncthreads();
    if (tid < 72) {
      const int i = tid / 12, r = tid % 12;
      double acc = 0.0;
      for (int k = 0; k < 12; ++k) acc = fma(m.H[r][k], m.J[i][k], acc);
      m.HJ[i][r] = acc;
    } else if (tid >= 96 && tid < 108) {
      const int r = tid - 96;
      double acc = 0.0;
      for (int k = 0; k < 12; ++k) acc = fma(m.H[r][k], m.g[k], acc);
      m.Hg[r] = acc;
    }
    __syncthreads();
    if (tid < 36) {
      const int i = tid / 6, j = tid % 6;
      double acc = 0.0;
      for (int r = 0; r < 12; ++r) acc = fma(m.J[i][r], m.HJ[j][r], acc);
      m.GN[i][j] = acc;
    } else if (tid >= 64 && tid < 76) {
      // V = H g - b;  Q = R^T V[:, 0:3],  w = R^T V[:, 3]
      const int e = tid - 64;
      if (e < 9) {
        const int l = e / 3, k = e % 3;
        m.Q[l][k] = m.g[l] * (m.Hg[k] - m.b[k]) + m.g[4 + l] * (m.Hg[4 + k] - m.b[4 + k]) +
                    m.g[8 + l] * (m.Hg[8 + k] - m.b[8 + k]);
      } else {
        const int l = e - 9;
        m.w[l] = m.g[l] * (m.Hg[3] - m.b[3]) + m.g[4 + l] * (m.Hg[7] - m.b[7]) +
                 m.g[8 + l] * (m.Hg[11] - m.b[11]);
      }
    }
    __syncthreads();
    // gradient and symmetrised Hessian, one entry per thread.  Second-order
    // term 2 <V, G (E_i E_j + E_j E_i)/2>: rot-rot Q_ij + Q_ji - 2 delta_ij tr Q,
    // rot i / trans j  w . (e_i x e_j)
    if (tid < 36) {
      const int i = tid / 6, j = tid % 6;
      double t2 = 0.0;
      if (i < 3 && j < 3) {
        const double trQ = m.Q[0][0] + m.Q[1][1] + m.Q[2][2];
        t2 = m.Q[i][j] + m.Q[j][i] - (i == j ? 2.0 * trQ : 0.0);
      } else if ((i < 3) != (j < 3)) {
        const int ir = i < 3 ? i : j, jt = (i < 3 ? j : i) - 3;
        if (ir != jt) {
          const int k = 3 - ir - jt;
          t2 = ((jt - ir + 3) % 3 == 1 ? 1.0 : -1.0) * m.w[k];
        }
      }
      const double gn = 0.5 * (m.GN[i][j] + m.GN[j][i]);
      m.Hgn[i][j] = 2.0 * gn * inv_s2;
      m.Hs[i][j] = (2.0 * gn + t2) * inv_s2;
    } else if (tid >= 64 && tid < 70) {
      const int i = tid - 64;
      m.grad[i] = i < 3 ? 2.0 * (m.Q[(i + 2) % 3][(i + 1) % 3] - m.Q[(i + 1) % 3][(i + 2) % 3]) *
                              inv_s2
                        : 2.0 * m.w[i - 3] * inv_s2;
    }
    __syncthreads();
    if (tid == 0) {
      if (itn == 0 && mode == 0) {
        for (int i = 0; i < 6; ++i) s->grad[i] = m.grad[i];
        for (int i = 0; i < 6; ++i)
          for (int j = 0; j < 6; ++j) s->hess[6 * i + j] = m.Hs[i][j];
      }
      double xi[6];
      bool ok = chol_solve6(m.Hs, m.grad, xi);
      if (!ok) {
        ++gnf;
        // least squares, as a singular Gauss-Newton matrix (degenerate
        // inputs) can pass a Cholesky factorisation by rounding alone
        ok = pinv_solve6(m.Hgn, m.grad, xi);
      }
      for (int i = 0; i < 6; ++i) m.xi[i] = ok ? xi[i] : 0.0;
      m.go = ok ? 1 : 0;
      m.step = 1.0;
      m.accept = 0;
    }
    __syncthreads();
    if (m.go != 1) break;
    // halve the step until D does not grow beyond a rounding allowance.  The
    // change of D is computed as  dD = d^T (2 (H g - b) + H d),  d = g' - g,
    // which is exact for the quadratic and free of the cancellation between
    // the large terms of D itself
    for (int h = 0; h < 31; ++h) {
      if (tid == 0) {
        double xs[6];
        for (int i = 0; i < 6; ++i) xs[i] = m.step * m.xi[i];
        compose(m.g, xs, m.gn);
      }
      __syncthreads();
      if (tid < 12) {
        double hd = 0.0;
        for (int k = 0; k < 12; ++k) hd = fma(m.H[tid][k], m.gn[k] - m.g[k], hd);
        rowbuf[tid] = (m.gn[tid] - m.g[tid]) * (2.0 * (m.Hg[tid] - m.b[tid]) + hd);
      }
      __syncthreads();
      if (tid == 0) {
        double dD = 0.0;
        for (int r = 0; r < 12; ++r) dD += rowbuf[r];
        if (dD <= 1e-12 * fabs(m.cur)) {
          m.accept = 1;
          m.val = m.cur + dD;
        } else {
          m.step *= 0.5;
        }
      }
      __syncthreads();
      if (m.accept) break;
    }
    if (tid == 0) {
      if (!m.accept) {
        m.go = 0;
      } else {
        double mxs = 0.0;
        for (int i = 0; i < 6; ++i) mxs = fmax(mxs, fabs(m.step * m.xi[i]));
        for (int r = 0; r < 12; ++r) m.g[r] = m.gn[r];
        m.cur = m.val;
        if (mxs < 1e-12) m.go = 0;
      }
    }
    __syncthreads();
  }
  if (tid != 0) return;
  cur = m.cur;
  const double s2n = Np > 0.0 ? fmax(cur / (3.0 * Np), sigma2_floor) : sigma2;
  bool finite = isfinite(s2n);
  for (int r = 0; r < 12; ++r) finite = finite && isfinite(m.g[r]);
  s->newton_iters = iters;
  s->gn_fallbacks += gnf;
  for (int a = 0; a < 3; ++a) {
    for (int c = 0; c < 3; ++c) s->R_next[3 * a + c] = m.g[4 * a + c];
    s->t_next[a] = m.g[4 * a + 3];
  }
  s->sigma2_next = s2n;
  if (mode == 1) {
    if (!finite) {
      s->numeric_error = 1;
      s->done = 1;
      return;
    }
    for (int a = 0; a < 3; ++a) {
      for (int c = 0; c < 3; ++c) s->R[3 * a + c] = m.g[4 * a + c];
      s->t[a] = m.g[4 * a + 3];
    }
    s->sigma2 = s2n;
    s->iter += 1;
  } else if (!finite) {
    s->numeric_error = 1;
  }
}

// Completes the state after the moments of Y (and X at the initial pose):
// working volume (box edges floored at 1e-3 of the diagonal), sigma^2 floor,
// and the initial sigma^2 if requested.
__global__ void init_state(DevState *__restrict__ s, const double *__restrict__ ymom,
                           const double *__restrict__ xmom, int64_t M, int64_t N, int v_auto,
                           int s2_auto) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double e[3];
  for (int i = 0; i < 3; ++i) e[i] = ymom[7 + i] - ymom[4 + i];
  const double diag = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
  if (v_auto) {
    if (diag == 0.0) {
      s->V = 1.0;
    } else {
      double V = 1.0;
      for (int i = 0; i < 3; ++i) V *= fmax(e[i], 1e-3 * diag);
      s->V = V;
    }
  }
  s->sigma2_floor = 1e-12 * diag * diag;
  if (s2_auto) {
    // sum_mn |x'_n - y_m|^2 = M sum|x'|^2 + N sum|y|^2 - 2 (sum x') . (sum y)
    const double dot = xmom[0] * ymom[0] + xmom[1] * ymom[1] + xmom[2] * ymom[2];
    const double tot = (double)M * xmom[3] + (double)N * ymom[3] - 2.0 * dot;
    s->sigma2 = tot / (3.0 * (double)M * (double)N);
  }
  if (s->eta > 0.0) {
    // Sec. 3.2: w_max = eta V S / ((1 - eta) + eta V S), S = sum_m pi(m) c_m
    // with the component bound c_m at the initial sigma^2
    const double a = s->eta * s->V * s->pic * pow(kTwoPi * s->sigma2, -1.5);
    s->w0 = a / ((1.0 - s->eta) + a);
  }
}

}  // namespace

hipError_t launch_reduce_mstep(const BatchPlan &pl, const BatchDev &bd, double *blockstats,
                               DevState *s, double *nll_trace, int trace_stride,
                               const unsigned long long *evcounts, int mode, hipStream_t st) {
  bool many = false;
  for (const Slot &sl : pl.slots) many = many || sl.nfin > kFewBlocks;
  if (many)
    hipLaunchKernelGGL(reduce_stats, dim3((unsigned)(kStats * pl.npairs)), dim3(256), 0, st,
                       bd.slots, blockstats, s);
  hipLaunchKernelGGL(reduce_mstep, dim3((unsigned)pl.npairs), dim3(256), 0, st, bd.slots,
                     (const double *)blockstats, s,
                     nll_trace, trace_stride, evcounts, mode);
  return hipGetLastError();
}

hipError_t launch_init_state(DevState *s, const double *ymom, const double *xmom, int64_t M,
                             int64_t N, int v_auto, int s2_auto, hipStream_t st) {
  hipLaunchKernelGGL(init_state, dim3(1), dim3(64), 0, st, s, ymom, xmom, M, N, v_auto, s2_auto);
  return hipGetLastError();
}

}  // namespace lsg
