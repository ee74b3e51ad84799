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
// sigma^2).  If Hs is not positive definite the Gauss-Newton part is used;
// steps are halved until D does not grow beyond a rounding allowance.  After
// the pose, sigma^2 = D(G_new) / (3 N_P) (Sec. 3.5, last paragraph).
// The solve is a few thousand FP64 operations; one thread does it.
#include <math.h>

#include "lsgcpd_internal.h"

namespace lsg {

namespace {

constexpr double kTwoPi = 6.283185307179586477;

struct Quad {
  double H[12][12];
  double b[12];
  double c;
};

__device__ void build_quad(const double *S, Quad &q) {
  // upper-triangle order (00 01 02 03 11 12 13 22 23 33)
  double S0[4][4], S1[6][4][4];
  auto unpack = [](const double *u, double M4[4][4]) {
    int o = 0;
    for (int i = 0; i < 4; ++i)
      for (int j = i; j < 4; ++j) {
        M4[i][j] = u[o];
        M4[j][i] = u[o];
        ++o;
      }
  };
  unpack(S, S0);
  for (int ab = 0; ab < 6; ++ab) unpack(S + 10 + 10 * ab, S1[ab]);
  const int pair[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
  for (int a = 0; a < 3; ++a)
    for (int bb = 0; bb < 3; ++bb)
      for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j)
          q.H[4 * a + i][4 * bb + j] = (a == bb ? S0[i][j] : 0.0) + S1[pair[a][bb]][i][j];
  for (int i = 0; i < 12; ++i) q.b[i] = S[70 + i];
  q.c = S[82];
}

__device__ double quad_eval(const Quad &q, const double G[4][4]) {
  double g[12];
  for (int a = 0; a < 3; ++a)
    for (int j = 0; j < 4; ++j) g[4 * a + j] = G[a][j];
  double s = q.c;
  for (int r = 0; r < 12; ++r) {
    double hr = 0.0;
    for (int c = 0; c < 12; ++c) hr = fma(q.H[r][c], g[c], hr);
    s = fma(g[r], hr - 2.0 * q.b[r], s);
  }
  return s;
}

// se(3) basis: E_0..E_2 rotations about x, y, z; E_3..E_5 translations.
__device__ void basis(int i, double E[4][4]) {
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) E[r][c] = 0.0;
  if (i < 3) {
    const int a = (i + 1) % 3, b = (i + 2) % 3;  // [e_i]_x: E[b][a] = 1, E[a][b] = -1
    E[b][a] = 1.0;
    E[a][b] = -1.0;
  } else {
    E[i - 3][3] = 1.0;
  }
}

__device__ void mat4_mul(const double A[4][4], const double B[4][4], double C[4][4]) {
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) {
      double s = 0.0;
      for (int k = 0; k < 4; ++k) s = fma(A[r][k], B[k][c], s);
      C[r][c] = s;
    }
}

// exp of the twist xi = (omega, v): Rodrigues rotation and left Jacobian.
__device__ void se3_exp(const double xi[6], double T[4][4]) {
  const double w0 = xi[0], w1 = xi[1], w2 = xi[2];
  const double th2 = w0 * w0 + w1 * w1 + w2 * w2;
  const double th = sqrt(th2);
  double A, B, C;
  if (th < 1e-6) {
    A = 1.0 - th2 / 6.0;
    B = 0.5 - th2 / 24.0;
    C = 1.0 / 6.0 - th2 / 120.0;
  } else {
    A = sin(th) / th;
    B = (1.0 - cos(th)) / th2;
    C = (th - sin(th)) / (th2 * th);
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
      T[r][c] = I + A * W[r][c] + B * W2[r][c];
      Vm[r][c] = I + B * W[r][c] + C * W2[r][c];
    }
  for (int r = 0; r < 3; ++r) T[r][3] = Vm[r][0] * xi[3] + Vm[r][1] * xi[4] + Vm[r][2] * xi[5];
  T[3][0] = T[3][1] = T[3][2] = 0.0;
  T[3][3] = 1.0;
}

// Cholesky solve of the 6x6 system A x = -g; false if A is not positive definite.
__device__ bool chol_solve6(const double A[6][6], const double g[6], double x[6]) {
  double L[6][6];
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) L[i][j] = 0.0;
  for (int j = 0; j < 6; ++j) {
    double d = A[j][j];
    for (int k = 0; k < j; ++k) d -= L[j][k] * L[j][k];
    if (!(d > 0.0)) return false;
    L[j][j] = sqrt(d);
    for (int i = j + 1; i < 6; ++i) {
      double s = A[i][j];
      for (int k = 0; k < j; ++k) s -= L[i][k] * L[j][k];
      L[i][j] = s / L[j][j];
    }
  }
  double y[6];
  for (int i = 0; i < 6; ++i) {
    double s = -g[i];
    for (int k = 0; k < i; ++k) s -= L[i][k] * y[k];
    y[i] = s / L[i][i];
  }
  for (int i = 5; i >= 0; --i) {
    double s = y[i];
    for (int k = i + 1; k < 6; ++k) s -= L[k][i] * x[k];
    x[i] = s / L[i][i];
  }
  return true;
}

// Gradient (Eq. 11) and symmetrised Hessian (Eq. 12) at G, and the
// Gauss-Newton part of the Hessian, all divided by sigma^2.
__device__ void derivatives(const Quad &q, const double G[4][4], double inv_s2, double grad[6],
                            double Hs[6][6], double Hgn[6][6]) {
  double g[12];
  for (int a = 0; a < 3; ++a)
    for (int j = 0; j < 4; ++j) g[4 * a + j] = G[a][j];
  double v[12];
  for (int r = 0; r < 12; ++r) {
    double s = -q.b[r];
    for (int c = 0; c < 12; ++c) s = fma(q.H[r][c], g[c], s);
    v[r] = s;
  }
  double J[6][12], HJ[6][12];
  for (int i = 0; i < 6; ++i) {
    double E[4][4], GE[4][4];
    basis(i, E);
    mat4_mul(G, E, GE);
    for (int a = 0; a < 3; ++a)
      for (int j = 0; j < 4; ++j) J[i][4 * a + j] = GE[a][j];
  }
  for (int i = 0; i < 6; ++i)
    for (int r = 0; r < 12; ++r) {
      double s = 0.0;
      for (int c = 0; c < 12; ++c) s = fma(q.H[r][c], J[i][c], s);
      HJ[i][r] = s;
    }
  for (int i = 0; i < 6; ++i) {
    double s = 0.0;
    for (int r = 0; r < 12; ++r) s = fma(v[r], J[i][r], s);
    grad[i] = 2.0 * s * inv_s2;
  }
  for (int i = 0; i < 6; ++i)
    for (int j = i; j < 6; ++j) {
      double s = 0.0;
      for (int r = 0; r < 12; ++r) s = fma(J[i][r], HJ[j][r], s);
      double Ei[4][4], Ej[4][4], EiEj[4][4], EjEi[4][4], K[4][4], GK[4][4];
      basis(i, Ei);
      basis(j, Ej);
      mat4_mul(Ei, Ej, EiEj);
      mat4_mul(Ej, Ei, EjEi);
      for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) K[r][c] = 0.5 * (EiEj[r][c] + EjEi[r][c]);
      mat4_mul(G, K, GK);
      double t2 = 0.0;
      for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 4; ++c) t2 = fma(v[4 * a + c], GK[a][c], t2);
      Hgn[i][j] = Hgn[j][i] = 2.0 * s * inv_s2;
      Hs[i][j] = Hs[j][i] = 2.0 * (s + t2) * inv_s2;
    }
}

__global__ __launch_bounds__(256) void reduce_mstep(const double *__restrict__ blockstats, int nblk,
                                                    int N, DevState *__restrict__ s,
                                                    double *__restrict__ trace, int mode) {
  if (s->done) return;
  __shared__ double S[kStats];
  for (int i = threadIdx.x; i < kStats; i += blockDim.x) {
    double a = 0.0;
    for (int b = 0; b < nblk; ++b) a += blockstats[(size_t)b * kStats + i];
    S[i] = a;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;

  const double sigma2 = s->sigma2;
  const double gam = pow(kTwoPi * sigma2, 1.5) / s->V;
  const double Np = S[9];
  const double nll = -(S[85] + S[83] - 1.5 * (double)N * log(kTwoPi * sigma2));
  for (int i = 0; i < kStats; ++i) s->stats[i] = S[i];
  s->gamma = gam;
  s->nll = nll;

  Quad q;
  build_quad(S, q);
  double G[4][4];
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) G[r][c] = s->R[3 * r + c];
    G[r][3] = s->t[r];
  }
  G[3][0] = G[3][1] = G[3][2] = 0.0;
  G[3][3] = 1.0;
  double cur = quad_eval(q, G);
  s->pd = cur;

  if (mode == 1) {
    const int it = s->iter;
    if (trace) trace[it] = nll;
    if (s->tol > 0.0 && it > 0 && fabs(nll - s->nll_prev) <= s->tol * fabs(nll)) {
      s->done = 1;
      s->converged = 1;
      return;
    }
    s->nll_prev = nll;
  }

  const double inv_s2 = 1.0 / sigma2;
  int iters = 0, gnf = 0;
  double grad[6], Hs[6][6], Hgn[6][6];
  if (Np > 0.0) {
    for (int itn = 0; itn < s->newton_max; ++itn) {
      ++iters;
      derivatives(q, G, inv_s2, grad, Hs, Hgn);
      if (itn == 0 && mode == 0) {
        for (int i = 0; i < 6; ++i) s->grad[i] = grad[i];
        for (int i = 0; i < 6; ++i)
          for (int j = 0; j < 6; ++j) s->hess[6 * i + j] = Hs[i][j];
      }
      double xi[6];
      if (!chol_solve6(Hs, grad, xi)) {
        ++gnf;
        if (!chol_solve6(Hgn, grad, xi)) {
          double mx = 0.0;
          for (int i = 0; i < 6; ++i) mx = fmax(mx, Hgn[i][i]);
          for (int i = 0; i < 6; ++i) Hgn[i][i] += 1e-10 * mx + 1e-300;
          if (!chol_solve6(Hgn, grad, xi)) break;
        }
      }
      double step = 1.0;
      bool ok = false;
      double Gn[4][4], val = cur;
      for (int h = 0; h < 31; ++h) {
        double xs[6], T[4][4];
        for (int i = 0; i < 6; ++i) xs[i] = step * xi[i];
        se3_exp(xs, T);
        mat4_mul(G, T, Gn);
        val = quad_eval(q, Gn);
        if (val <= cur + 1e-12 * fabs(cur)) {
          ok = true;
          break;
        }
        step *= 0.5;
      }
      if (!ok) break;
      for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) G[r][c] = Gn[r][c];
      cur = val;
      double mxs = 0.0;
      for (int i = 0; i < 6; ++i) mxs = fmax(mxs, fabs(step * xi[i]));
      if (mxs < 1e-12) break;
    }
  } else if (mode == 0) {
    for (int i = 0; i < 6; ++i) s->grad[i] = 0.0;
    for (int i = 0; i < 36; ++i) s->hess[i] = 0.0;
  }
  double s2n = Np > 0.0 ? fmax(cur / (3.0 * Np), s->sigma2_floor) : sigma2;
  bool finite = isfinite(s2n);
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 4; ++c) finite = finite && isfinite(G[r][c]);
  s->newton_iters = iters;
  s->gn_fallbacks += gnf;
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) s->R_next[3 * r + c] = G[r][c];
    s->t_next[r] = G[r][3];
  }
  s->sigma2_next = s2n;
  if (mode == 1) {
    if (!finite) {
      s->numeric_error = 1;
      s->done = 1;
      return;
    }
    for (int r = 0; r < 3; ++r) {
      for (int c = 0; c < 3; ++c) s->R[3 * r + c] = G[r][c];
      s->t[r] = G[r][3];
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
}

}  // namespace

hipError_t launch_reduce_mstep(double *blockstats, int nblk, int64_t N, DevState *s,
                               double *nll_trace, int mode, hipStream_t st) {
  hipLaunchKernelGGL(reduce_mstep, dim3(1), dim3(256), 0, st, blockstats, nblk, (int)N, s,
                     nll_trace, mode);
  return hipGetLastError();
}

hipError_t launch_init_state(DevState *s, const double *ymom, const double *xmom, int64_t M,
                             int64_t N, int v_auto, int s2_auto, hipStream_t st) {
  hipLaunchKernelGGL(init_state, dim3(1), dim3(64), 0, st, s, ymom, xmom, M, N, v_auto, s2_auto);
  return hipGetLastError();
}

}  // namespace lsg
