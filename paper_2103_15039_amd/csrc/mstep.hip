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
// The finalisation turns each source's summed exponentials into its
// posterior weights (Eq. 9) and its terms of the 86 statistics, one block per
// 64 sources; reduce_stats (one block per statistic and problem) and
// reduce_mstep sum the block statistics in a fixed order and run the M step
// of each problem.
// The M step (mstep_wave) runs the Newton iteration of a problem on one
// wave, whose lanes share the 12 x 12 products and the entries of the
// gradient and Hessian, and each of which then takes the 6 x 6 LDL^T solve
// and the exponential map itself.
#include <math.h>

#include "lsgcpd_internal.h"

namespace lsg {

namespace {

constexpr double kTwoPi = 6.283185307179586477;

// SE(3) exponential of the twist xi = (omega, v): Rodrigues rotation and the
// left Jacobian of SO(3) for the translation,
//   A = sin(th)/th,  B = (1 - cos th)/th^2,  C = (th - sin th)/th^3.
// For th < 1/4 (every Newton step but the first few of a registration) the
// three are their Taylor series in th^2 to the th^10 term; the first omitted
// term is below 1e-17 of each, under half an FP64 ulp.
__device__ __forceinline__ void se3_exp(const double xi[6], double Rx[3][3], double tx[3]) {
  const double w0 = xi[0], w1 = xi[1], w2 = xi[2];
  const double th2 = w0 * w0 + w1 * w1 + w2 * w2;
  double A, B, C;
  if (th2 < 0.0625) {
    // sum_k (-th^2)^k / (2k+1)!, / (2k+2)!, / (2k+3)!  for k = 0..5
    A = 1.0 + th2 * (-1.0 / 6 + th2 * (1.0 / 120 + th2 * (-1.0 / 5040 + th2 * (1.0 / 362880 +
        th2 * (-1.0 / 39916800)))));
    B = 0.5 + th2 * (-1.0 / 24 + th2 * (1.0 / 720 + th2 * (-1.0 / 40320 + th2 * (1.0 / 3628800 +
        th2 * (-1.0 / 479001600)))));
    C = 1.0 / 6 + th2 * (-1.0 / 120 + th2 * (1.0 / 5040 + th2 * (-1.0 / 362880 +
        th2 * (1.0 / 39916800 + th2 * (-1.0 / 6227020800.0)))));
  } else {
    const double th = sqrt(th2);
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
__device__ __forceinline__ void compose(const double *g, const double xi[6], double *gout) {
  double Rx[3][3], tx[3];
  se3_exp(xi, Rx, tx);
  for (int a = 0; a < 3; ++a) {
    const double *G = g + 4 * a;
    for (int c = 0; c < 3; ++c) gout[4 * a + c] = G[0] * Rx[0][c] + G[1] * Rx[1][c] + G[2] * Rx[2][c];
    gout[4 * a + 3] = G[0] * tx[0] + G[1] * tx[1] + G[2] * tx[2] + G[3];
  }
}

// 1/d from the hardware's reciprocal estimate and two Newton steps, each of
// which squares the relative error.
__device__ __forceinline__ double recip(double d) {
  double r = __builtin_amdgcn_rcp(d);
  r = fma(r, fma(-d, r, 1.0), r);
  return fma(r, fma(-d, r, 1.0), r);
}

// Solve of the 6x6 system A x = -g by the factorisation A = L D L^T (unit
// lower L, diagonal D > 0), computed in place in the lower triangle of A
// (the upper one is not read); false if a pivot is not positive, i.e. A is
// not positive definite.  One reciprocal per column and no square roots:
// the long-latency steps of this serial code.
__device__ __forceinline__ bool chol_solve6(double A[6][6], const double g[6], double x[6]) {
  double inv[6];
  for (int j = 0; j < 6; ++j) {
    double d = A[j][j];
    for (int k = 0; k < j; ++k) d -= A[j][k] * A[j][k] * A[k][k];
    if (!(d > 0.0)) return false;
    A[j][j] = d;
    inv[j] = recip(d);
    for (int i = j + 1; i < 6; ++i) {
      double s = A[i][j];
      for (int k = 0; k < j; ++k) s -= A[i][k] * A[j][k] * A[k][k];
      A[i][j] = s * inv[j];
    }
  }
  double y[6];
  for (int i = 0; i < 6; ++i) {
    double s = -g[i];
    for (int k = 0; k < i; ++k) s -= A[i][k] * y[k];
    y[i] = s;
  }
  for (int i = 5; i >= 0; --i) {
    double s = y[i] * inv[i];
    for (int k = i + 1; k < 6; ++k) s -= A[k][i] * x[k];
    x[i] = s;
  }
  return true;
}

// Minimum-norm least-squares solution of A x = -g for the symmetric 6x6
// Gauss-Newton matrix A (singular for degenerate inputs such as a single
// source point, whose rotations about itself are free): eigen-decomposition by cyclic Jacobi rotations, then
//   x = -sum_i (v_i . g / lambda_i) v_i  over |lambda_i| > 6 eps max|lambda|,
// the pseudo-inverse a singular-value solve with that cutoff gives (for a
// symmetric matrix the singular values are the |lambda_i|).  ok = 0 if A is
// 0.  Kept out of line (only degenerate inputs reach it), with the result
// returned by value so that the caller's arrays stay in registers.
struct Sol6 {
  double x[6];
  int ok;
};
__device__ __noinline__ Sol6 pinv_solve6(const double (*Ain)[6], const double *g) {
  Sol6 res;
  double *x = res.x;
  res.ok = 0;
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
  if (!(mx > 0.0) || !isfinite(mx)) return res;
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
  res.ok = 1;
  return res;
}

// LDS of the wave-parallel M step.
struct MSh {
  double H[12][12];   // H[4a+i][4b+j] = delta_ab S0[i][j] + S1[ab][i][j]
  double b[12];       // vec(S2)
  double g[12];       // vec(G), the current pose
  double HJ[6][12];   // H vec(G E_j) of the six generators
  double Hg[12];
  double GN[6][6];
  double Q[3][3], w[3];   // R^T (H g - b), split as the second-order term uses it
  double Hs[6][6], Hgn[6][6], grad[6];
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

// ------------------------------------------------------------- finalisation
// ITEMS: partials per work item ([item][feature][kGroup]; the items of
// source group g of problem p are its items off[g_off + p + g] ..
// off[g_off + p + g + 1] - 1), summed by 4 waves per block (wave q takes items
// q, q + 4, ...; the 4 sums are added in a fixed order); otherwise per target
// chunk ([chunk][feature][N], one problem), one wave per block.  Block b
// belongs to problem fin_slot[b]; its statistics go to the problem's
// stat-major rows (row i of problem p: blockstats[kStats fin_off + i nfin ..]).
static_assert(kGroup % kFinBlock == 0, "a finalisation block lies in one source group");

template <bool ITEMS>
__device__ void finalize_block(const Slot &sl, int ps, const DevState *__restrict__ st,
                               int single, const double *__restrict__ partial, int nsplit,
                               const int *__restrict__ offs, double *__restrict__ blockstats,
                               double *__restrict__ colS, double *__restrict__ colstats) {
  // One problem (single): every offset of its slot is 0, so the item range
  // of the block's source group loads with the done flag and the slot.  (A
  // block lies in one group; the group's item count has an entry for every
  // block of the problem.)
  const int done = st->done;
  const int N = sl.N, nfin = sl.nfin;
  const float *X = sl.X;
  const float *w = sl.w;
  const float *phi = sl.phi;
  const int64_t x_off = sl.x_off;
  int fin_off = 0, i0 = 0, i1 = 0;
  if (single) {
    if (ITEMS) {
      const int g = blockIdx.x * kFinBlock / kGroup;
      i0 = offs[g];
      i1 = offs[g + 1];
    }
  } else {
    fin_off = sl.fin_off;
    if (ITEMS) {
      const int g = (blockIdx.x - fin_off) * kFinBlock / kGroup;
      const int *off = offs + sl.g_off + ps;
      i0 = sl.item_off + off[g];
      i1 = sl.item_off + off[g + 1];
    }
  }
  // every load above is issued before any arithmetic on its value
  __builtin_amdgcn_sched_barrier(0);
  asm volatile("" ::"s"(done), "s"(N), "s"(nfin), "s"(X), "s"(fin_off), "s"(i0), "s"(i1));
  if (done) return;
  const int fb = blockIdx.x - fin_off;
  const int l = threadIdx.x & (kFinBlock - 1);
  const int part = threadIdx.x / kFinBlock;  // 0 without ITEMS
  const int n = fb * kFinBlock + l;
  // the source's coordinates, with the partial sums (index clamped to the
  // cloud, N >= 1)
  const int nc = n < N ? n : N - 1;
  const float fx = X[3 * nc], fy = X[3 * nc + 1], fz = X[3 * nc + 2];
  double p = 0.0, W[6] = {0, 0, 0, 0, 0, 0}, B[3] = {0, 0, 0}, C = 0.0, lg = 0.0, outl = 0.0,
         logw = 0.0;
  double xt[4] = {0.0, 0.0, 0.0, 0.0};
  double T[kFeatUsed];
#pragma unroll
  for (int c = 0; c < kFeatUsed; ++c) T[c] = 0.0;
  if (ITEMS) {
    if (n < N) {
      // this wave's items in increasing order, the loads of 4 issued together
      const int j = n % kGroup;
      int it = i0 + part;
      for (; it + 12 < i1; it += 16) {
        double v[4][kFeatUsed];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int c = 0; c < kFeatUsed; ++c)
            v[u][c] = partial[((size_t)(it + 4 * u) * kFeatUsed + c) * kGroup + j];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int c = 0; c < kFeatUsed; ++c) T[c] += v[u][c];
      }
      for (; it < i1; it += 4)
#pragma unroll
        for (int c = 0; c < kFeatUsed; ++c)
          T[c] += partial[((size_t)it * kFeatUsed + c) * kGroup + j];
    }
    __shared__ double tr[3][kFeatUsed][kFinBlock];
    if (part > 0)
#pragma unroll
      for (int c = 0; c < kFeatUsed; ++c) tr[part - 1][c][l] = T[c];
    __syncthreads();
    if (part == 0)
#pragma unroll
      for (int c = 0; c < kFeatUsed; ++c) T[c] = ((T[c] + tr[0][c][l]) + tr[1][c][l]) + tr[2][c][l];
  } else if (n < N) {
    for (int sp = 0; sp < nsplit; ++sp)
#pragma unroll
      for (int c = 0; c < kFeatUsed; ++c) T[c] += partial[((size_t)sp * kFeatUsed + c) * N + n];
  }
  if (part == 0 && n < N) {
    // Sec. 3.3: w_n = 1 - (1 - w0) phi(x_n) under confidence filtering
    const double wn = w ? (double)w[n] : phi ? 1.0 - (1.0 - st->w0) * (double)phi[n] : st->w0;
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
    if (colS) colS[x_off + n] = T[0];
    if (colstats) {
      double *cs = colstats + (size_t)(x_off + n) * kColStats;
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
    xt[0] = (double)fx;
    xt[1] = (double)fy;
    xt[2] = (double)fz;
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
  if (part == 0) {
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
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kStats; i += blockDim.x) {
    double s = 0.0;
    for (int k = 0; k < kFinBlock; ++k) s += red[i][k];
    blockstats[(size_t)kStats * fin_off + (size_t)i * nfin + fb] = s;  // stat-major
  }
}

// single: the batch is one problem (p = 0 without a table lookup).
template <bool ITEMS>
__global__ __launch_bounds__(4 * kFinBlock) void estep_finalize(
    int single, const Slot *__restrict__ slots, const int *__restrict__ fin_slot,
    const DevState *__restrict__ states, const int *__restrict__ offs,
    const double *__restrict__ partial, int nsplit, double *__restrict__ blockstats,
    double *__restrict__ colS, double *__restrict__ colstats) {
  const int ps = single ? 0 : fin_slot[blockIdx.x];
  finalize_block<ITEMS>(slots[ps], ps, states + ps, single, partial, nsplit, offs, blockstats,
                        colS, colstats);
}

// Problems with at most this many finalisation blocks (64 sources each) are
// summed by reduce_mstep itself: for them a kernel of its own costs more in
// launch latency than the sums.
constexpr int kFewBlocks = 64;

// Sum of row i of a problem's stat-major block statistics (one block per
// statistic and problem, so that the reads are spread over many CUs): thread
// t adds the partials t, t + 256, ... in order, then a fixed tree adds the
// threads.  The result does not depend on timing.
// nfin1: the block count of the batch's only problem (its rows then start at
// 0, and the first partials load with the done flag), 0 for a batch.
__global__ __launch_bounds__(256) void reduce_stats(int nfin1, const Slot *__restrict__ slots,
                                                     const double *__restrict__ blockstats,
                                                     DevState *__restrict__ states) {
  const int p = blockIdx.x / kStats, i = blockIdx.x % kStats, tid = threadIdx.x;
  DevState *s = states + p;
  const int done = s->done;
  const int nblk = nfin1 ? nfin1 : slots[p].nfin;
  const double *row =
      blockstats + (nfin1 ? (size_t)0 : (size_t)kStats * slots[p].fin_off) + (size_t)i * nblk;
  double v[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int b = k * 256 + tid;
    v[k] = b < nblk ? row[b] : 0.0;
  }
  ready_s(done);
#pragma unroll
  for (int k = 0; k < 8; ++k) ready_v(v[k]);
  if (done || nblk <= kFewBlocks) return;  // reduce_mstep sums those itself
  double a = 0.0;
  for (int c0 = 0;;) {
#pragma unroll
    for (int k = 0; k < 8; ++k) a += v[k];
    c0 += 8 * 256;
    if (c0 >= nblk) break;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int b = c0 + k * 256 + tid;
      v[k] = b < nblk ? row[b] : 0.0;
    }
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

// Values of the state the M step reads, loaded together at the start of
// reduce_mstep, before anything writes the state (only the M step does).
struct MIn {
  double g[12];  // vec(G) = rows of [R | t]
  double sigma2, V, tol, nll_prev, sigma2_floor;
  int iter, newton_max, N, f3_steps;
  int64_t evaluated_pairs;
  unsigned long long evc, f3c;  // this E step's evaluated pairs, of them BF16 (or 0)
};

__device__ __forceinline__ MIn load_min(const DevState *s, int N,
                                        const unsigned long long *evcounts, int pidx,
                                        int npairs) {
  MIn in;
  in.evaluated_pairs = s->evaluated_pairs;
  in.f3_steps = s->f3_steps;
  in.evc = evcounts ? evcounts[pidx] : 0ull;
  in.f3c = evcounts ? evcounts[npairs + pidx] : 0ull;
  for (int a = 0; a < 3; ++a) {
    for (int c = 0; c < 3; ++c) in.g[4 * a + c] = s->R[3 * a + c];
    in.g[4 * a + 3] = s->t[a];
  }
  in.sigma2 = s->sigma2;
  in.V = s->V;
  in.tol = s->tol;
  in.nll_prev = s->nll_prev;
  in.sigma2_floor = s->sigma2_floor;
  in.iter = s->iter;
  in.newton_max = s->newton_max;
  in.N = N;
  return in;
}

// Every value of `in` ready (loaded) at this point.
__device__ __forceinline__ void ready_min(const MIn &in) {
#pragma unroll
  for (int k = 0; k < 12; ++k) ready_s(in.g[k]);
  ready_s(in.sigma2);
  ready_s(in.V);
  ready_s(in.tol);
  ready_s(in.nll_prev);
  ready_s(in.sigma2_floor);
  ready_s(in.iter);
  ready_s(in.newton_max);
  ready_s(in.N);
  ready_s(in.f3_steps);
  ready_s((long long)in.evaluated_pairs);
  ready_s((long long)in.evc);
  ready_s((long long)in.f3c);
}

// Orders the LDS stores of one wave's lanes before the loads that follow.
// A wave's LDS operations are performed in order, so no wait is needed: the
// wavefront-scope fences only keep the compiler from moving memory
// operations across the point (a workgroup-scope fence would also wait for
// the wave's outstanding global stores).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// v of lane l - n within each row of 16 lanes (0 for l mod 16 < n): a DPP
// row shift (ctrl 0x110 + n) of both halves of the double
template <int CTRL>
__device__ __forceinline__ double row_shr(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, true);
  return __hiloint2double(hi, lo);
}

// Sum over lanes 0..15 (lanes 12..15 bring 0): running sums along the row,
// whose last lane then holds the total, read back as a wave-uniform value.
__device__ __forceinline__ double sum16(double v) {
  v += row_shr<0x111>(v);
  v += row_shr<0x112>(v);
  v += row_shr<0x114>(v);
  v += row_shr<0x118>(v);
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 15),
                          __builtin_amdgcn_readlane(__double2loint(v), 15));
}

// sum_k h_k v_k over the 12 entries as three independent chains (one per
// row of G) added at the end: a quarter of the dependent latency of one chain
__device__ __forceinline__ double dot12(const double (&h)[12], const double (&v)[12]) {
  double s[3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
    s[a] = fma(h[4 * a], v[4 * a], fma(h[4 * a + 1], v[4 * a + 1],
                                       fma(h[4 * a + 2], v[4 * a + 2], h[4 * a + 3] * v[4 * a + 3])));
  return (s[0] + s[1]) + s[2];
}

// v[lane] for lane < 12 (a selection, so that v stays in registers)
__device__ __forceinline__ double pick12(const double (&v)[12], int lane) {
  double r = 0.0;
#pragma unroll
  for (int k = 0; k < 12; ++k) r = lane == k ? v[k] : r;
  return r;
}

// The M step of problem pidx (of npairs), run by the 64 lanes of one wave
// from the 86 statistics in S (LDS, visible to the wave) and the state values
// in `in`.  The 12 x 12 products and the gradient and Hessian entries are
// spread over the lanes; every lane then solves the 6 x 6 system and takes
// the exponential map itself, so that the step and the trial pose need no
// exchange between lanes, and the change of D is a 12-lane sum.
__device__ void mstep_wave(int pidx, int npairs, const double *S, const MIn &in,
                           DevState *__restrict__ states, double *__restrict__ traces,
                           int trace_stride, const unsigned long long *__restrict__ evcounts,
                           int mode) {
  DevState *s = states + pidx;
  const int lane = threadIdx.x & 63;
  __shared__ MSh m;
  if (evcounts && lane == 0) {
    s->evaluated_pairs = in.evaluated_pairs + (int64_t)in.evc;
    if (in.f3c) s->f3_steps = in.f3_steps + 1;
  }
  s->stats[lane] = S[lane];
  if (lane < kStats - 64) s->stats[64 + lane] = S[64 + lane];
  // the quadratic and the pose
  for (int e = lane; e < 144; e += 64) {
    const int r = e / 12, cc = e % 12;
    const int a = r >> 2, i = r & 3, bb = cc >> 2, k = cc & 3;
    double v = S[10 + 10 * pair_index(a, bb) + tri4(i, k)];
    if (a == bb) v += S[tri4(i, k)];
    m.H[r][cc] = v;
  }
  if (lane < 12) {
    m.b[lane] = S[70 + lane];
    m.g[lane] = pick12(in.g, lane);
  }
  wave_sync();
  double g[12];
#pragma unroll
  for (int r = 0; r < 12; ++r) g[r] = in.g[r];
  // lane r < 12 keeps row r of H and b_r in registers for the whole M step
  double hrow[12], br = 0.0;
#pragma unroll
  for (int k = 0; k < 12; ++k) hrow[k] = lane < 12 ? m.H[lane][k] : 0.0;
  if (lane < 12) br = m.b[lane];
  // D(g) = sum_r g_r ((H g)_r - 2 b_r) + c
  double cur;
  {
    const double hg = dot12(hrow, g);
    cur = S[82] + sum16(lane < 12 ? pick12(g, lane) * (hg - 2.0 * br) : 0.0);
  }
  const double x2 = kTwoPi * in.sigma2;
  const double inv_s2 = 1.0 / in.sigma2;
  const double Np = S[9];
  const double nll = -(S[85] + S[83] - 1.5 * (double)in.N * log(x2));
  if (lane == 0) {
    s->gamma = x2 * sqrt(x2) / in.V;
    s->nll = nll;
    s->pd = cur;
  }
  if (mode == 1) {
    if (lane == 0 && traces) traces[(size_t)pidx * trace_stride + in.iter] = nll;
    if (in.tol > 0.0 && in.iter > 0 && fabs(nll - in.nll_prev) <= in.tol * fabs(nll)) {
      if (lane == 0) {
        s->done = 1;
        s->converged = 1;
      }
      return;  // EM stopped by the tolerance
    }
    if (lane == 0) s->nll_prev = nll;
  }
  if (mode == 0 && Np <= 0.0 && lane < 42) {
    if (lane < 36) s->hess[lane] = 0.0;
    else s->grad[lane - 36] = 0.0;
  }

  int iters = 0, gnf = 0;
  bool go = Np > 0.0;
  for (int itn = 0; itn < in.newton_max && go; ++itn) {
    ++iters;
    // H J_i and H g, lane r < 12 taking row r.  J_i = vec(G E_i): rotation
    // i -> [R [e_i]x | 0] (in row a: +g(a, w) at column u, -g(a, u) at column
    // w, (u, w) = (i+1, i+2) mod 3), translation i -> [0 | R e_i] (g(a, i)
    // at column 3)
    if (lane < 12) {
      m.Hg[lane] = dot12(hrow, g);
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const int u = (i + 1) % 3, w = (i + 2) % 3;
        double t[3];
#pragma unroll
        for (int a = 0; a < 3; ++a)
          t[a] = fma(hrow[4 * a + u], g[4 * a + w], -hrow[4 * a + w] * g[4 * a + u]);
        m.HJ[i][lane] = (t[0] + t[1]) + t[2];
      }
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        m.HJ[3 + i][lane] = fma(hrow[3], g[i], fma(hrow[7], g[4 + i], hrow[11] * g[8 + i]));
      }
    }
    wave_sync();
    // J_i^T H J_j, and Q = R^T V[:, 0:3], w = R^T V[:, 3] with V = H g - b
    if (lane < 36) {
      const int i = lane / 6, j = lane % 6;
      double t[3];
      if (i < 3) {
        const int u = (i + 1) % 3, w = (i + 2) % 3;
#pragma unroll
        for (int a = 0; a < 3; ++a)
          t[a] = fma(m.g[4 * a + w], m.HJ[j][4 * a + u], -m.g[4 * a + u] * m.HJ[j][4 * a + w]);
      } else {
#pragma unroll
        for (int a = 0; a < 3; ++a) t[a] = m.g[4 * a + i - 3] * m.HJ[j][4 * a + 3];
      }
      m.GN[i][j] = (t[0] + t[1]) + t[2];
    } else if (lane < 48) {
      const int e = lane - 36;
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
    wave_sync();
    // gradient and symmetrised Hessian, one entry per lane.  Second-order
    // term 2 <V, G (E_i E_j + E_j E_i)/2>: rot-rot Q_ij + Q_ji - 2 delta_ij tr Q,
    // rot i / trans j  w . (e_i x e_j)
    if (lane < 36) {
      const int i = lane / 6, j = lane % 6;
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
      const double hs = (2.0 * gn + t2) * inv_s2;
      m.Hgn[i][j] = 2.0 * gn * inv_s2;
      m.Hs[i][j] = hs;
      if (itn == 0 && mode == 0) s->hess[lane] = hs;
    } else if (lane < 42) {
      const int i = lane - 36;
      const double gr = i < 3 ? 2.0 * (m.Q[(i + 2) % 3][(i + 1) % 3] - m.Q[(i + 1) % 3][(i + 2) % 3]) *
                                    inv_s2
                              : 2.0 * m.w[i - 3] * inv_s2;
      m.grad[i] = gr;
      if (itn == 0 && mode == 0) s->grad[i] = gr;
    }
    wave_sync();
    // the Newton step, on every lane
    double xi[6];
    {
      double A[6][6], gr[6];
      for (int i = 0; i < 6; ++i) {
        gr[i] = m.grad[i];
        for (int j = 0; j <= i; ++j) A[i][j] = m.Hs[i][j];
      }
      if (!chol_solve6(A, gr, xi)) {
        ++gnf;
        // least squares, as a singular Gauss-Newton matrix (degenerate
        // inputs) can pass a Cholesky factorisation by rounding alone
        const Sol6 r = pinv_solve6(m.Hgn, m.grad);
        if (!r.ok) break;
        for (int i = 0; i < 6; ++i) xi[i] = r.x[i];
      }
    }
    // halve the step until D does not grow beyond a rounding allowance.  The
    // change of D is computed as  dD = d^T (2 (H g - b) + H d),  d = g' - g,
    // which is exact for the quadratic and free of the cancellation between
    // the large terms of D itself
    const double vr = lane < 12 ? 2.0 * (m.Hg[lane] - br) : 0.0;
    double step = 1.0, gn[12];
    bool accept = false;
    for (int h = 0; h < 31; ++h) {
      double xs[6];
      for (int i = 0; i < 6; ++i) xs[i] = step * xi[i];
      compose(g, xs, gn);
      double d[12];
#pragma unroll
      for (int r = 0; r < 12; ++r) d[r] = gn[r] - g[r];
      const double hd = dot12(hrow, d);
      const double dD = sum16(lane < 12 ? pick12(d, lane) * (vr + hd) : 0.0);
      if (dD <= 1e-12 * fabs(cur)) {
        accept = true;
        cur += dD;
        break;
      }
      step *= 0.5;
    }
    if (!accept) break;
    double mxs = 0.0;
    for (int i = 0; i < 6; ++i) mxs = fmax(mxs, fabs(step * xi[i]));
#pragma unroll
    for (int r = 0; r < 12; ++r) g[r] = gn[r];
    if (lane < 12) m.g[lane] = pick12(g, lane);
    wave_sync();
    if (mxs < 1e-12) go = false;
  }
  if (lane != 0) return;
  const double s2n = Np > 0.0 ? fmax(cur / (3.0 * Np), in.sigma2_floor) : in.sigma2;
  bool finite = isfinite(s2n);
  for (int r = 0; r < 12; ++r) finite = finite && isfinite(g[r]);
  s->newton_iters = iters;
  s->gn_fallbacks += gnf;
  for (int a = 0; a < 3; ++a) {
    for (int c = 0; c < 3; ++c) s->R_next[3 * a + c] = g[4 * a + c];
    s->t_next[a] = g[4 * a + 3];
  }
  s->sigma2_next = s2n;
  if (mode == 1) {
    if (!finite) {
      s->numeric_error = 1;
      s->done = 1;
      return;
    }
    for (int a = 0; a < 3; ++a) {
      for (int c = 0; c < 3; ++c) s->R[3 * a + c] = g[4 * a + c];
      s->t[a] = g[4 * a + 3];
    }
    s->sigma2 = s2n;
    s->iter += 1;
  } else if (!finite) {
    s->numeric_error = 1;
  }
}

// The M step from the block statistics: summed here for problems with few
// finalisation blocks, else by reduce_stats into s->stats.  ONE: the batch is
// one problem, of nfin1 blocks (its rows start at 0, so its first partials
// load with the done flag and the state).
template <bool ONE>
__global__ __launch_bounds__(256) void reduce_mstep(int nfin1, const Slot *__restrict__ slots,
                                                    const double *__restrict__ blockstats,
                                                    DevState *__restrict__ states,
                                                    double *__restrict__ traces, int trace_stride,
                                                    unsigned long long *__restrict__ evcounts,
                                                    int mode) {
  const int pidx = blockIdx.x, tid = threadIdx.x;
  const int npairs = ONE ? 1 : (int)gridDim.x;
  const DevState *st = states + pidx;
  const int done = st->done;
  const MIn in = load_min(st, slots[pidx].N, evcounts, pidx, npairs);
  const int nfin = ONE ? nfin1 : slots[pidx].nfin;
  const int fin_off = ONE ? 0 : slots[pidx].fin_off;
  // statistic tid: its first 32 block partials in order (few blocks), else
  // the sum reduce_stats left in the state
  const bool few = nfin <= kFewBlocks;
  const double *row = blockstats + (size_t)kStats * fin_off + (size_t)tid * nfin;
  double v[32];
#pragma unroll
  for (int k = 0; k < 32; ++k) v[k] = tid < kStats && few && k < nfin ? row[k] : 0.0;
  const double summed = tid < kStats && !few ? states[pidx].stats[tid] : 0.0;
  // every load above is issued before any arithmetic on its value
  __builtin_amdgcn_sched_barrier(0);
  ready_s(done);
  ready_min(in);
#pragma unroll
  for (int k = 0; k < 32; ++k) ready_v(v[k]);
  ready_v(summed);
  if (done) return;
  if (evcounts && tid == 0) {  // read: cleared for the next E step
    evcounts[pidx] = 0ull;
    evcounts[npairs + pidx] = 0ull;
  }
  double stat = summed;
  if (tid < kStats && few) {
    // the rest of the partials, the loads of 32 in flight
    for (int b0 = 0;;) {
#pragma unroll
      for (int k = 0; k < 32; ++k) stat += v[k];
      b0 += 32;
      if (b0 >= nfin) break;
#pragma unroll
      for (int k = 0; k < 32; ++k) v[k] = b0 + k < nfin ? row[b0 + k] : 0.0;
    }
  }
  __shared__ double S[kStats];
  if (tid < kStats) S[tid] = stat;
  __syncthreads();
  if (tid >= 64) return;
  mstep_wave(pidx, npairs, S, in, states, traces, trace_stride, evcounts, mode);
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
                               unsigned long long *evcounts, int mode, hipStream_t st) {
  bool many = false;
  for (const Slot &sl : pl.slots) many = many || sl.nfin > kFewBlocks;
  const int nfin1 = pl.npairs == 1 ? pl.slots[0].nfin : 0;
  if (many)
    hipLaunchKernelGGL(reduce_stats, dim3((unsigned)(kStats * pl.npairs)), dim3(256), 0, st,
                       nfin1, bd.slots, blockstats, s);
  if (nfin1)
    hipLaunchKernelGGL(reduce_mstep<true>, dim3(1), dim3(256), 0, st, nfin1, bd.slots,
                       (const double *)blockstats, s, nll_trace, trace_stride, evcounts, mode);
  else
    hipLaunchKernelGGL(reduce_mstep<false>, dim3((unsigned)pl.npairs), dim3(256), 0, st, 0,
                       bd.slots, (const double *)blockstats, s, nll_trace, trace_stride, evcounts,
                       mode);
  return hipGetLastError();
}

hipError_t launch_finalize(const BatchPlan &pl, const BatchDev &bd, const DevState *s,
                           const void *plan_ws, const double *partial, double *blockstats,
                           double *colS, double *colstats, hipStream_t st) {
  const int single = pl.npairs == 1 ? 1 : 0;
  if (pl.backend == kBackendScalar)
    hipLaunchKernelGGL(estep_finalize<true>, dim3((unsigned)pl.fins), dim3(4 * kFinBlock), 0, st,
                       single, bd.slots, bd.fin_slot, s, estep_plan_offsets(pl, plan_ws), partial,
                       0, blockstats, colS, colstats);
  else
    hipLaunchKernelGGL(estep_finalize<false>, dim3((unsigned)pl.fins), dim3(kFinBlock), 0, st,
                       single, bd.slots, bd.fin_slot, s, (const int *)nullptr, partial, pl.nsplit,
                       blockstats, colS, colstats);
  return hipGetLastError();
}

hipError_t launch_init_state(DevState *s, const double *ymom, const double *xmom, int64_t M,
                             int64_t N, int v_auto, int s2_auto, hipStream_t st) {
  hipLaunchKernelGGL(init_state, dim3(1), dim3(64), 0, st, s, ymom, xmom, M, N, v_auto, s2_auto);
  return hipGetLastError();
}

}  // namespace lsg
