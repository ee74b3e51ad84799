/*
 * Plain FP64 C version of the oracle's E step, for clouds too large for the
 * dense NumPy version (tens of thousands of points) and for timing the CPU
 * baseline.  TEST INFRASTRUCTURE ONLY: used by the test-suite and the
 * benchmark's CPU leg, never by the GPU library; it shares no code with it.
 *
 * For every source n it evaluates, over all components m, the posterior of
 * Eq. (5) in the form of Eq. (9) (LSG-CPD, Sec. 3.4):
 *   K_mn = (1 - w_n)/w_n * pi_m * exp(-d_mn / (2 sigma^2)) [* sqrt(1 + alpha_m)],
 *   d_mn = |g(x_n) - y_m|^2 + alpha_m (n_m . (g(x_n) - y_m))^2,
 *   P_mn = K_mn / (sum_m K_mn + gamma),  gamma = (2 pi sigma^2)^{3/2} / V,
 * first the column sum, then P_mn, and the per-source sums of the oracle's
 * Columns record (M_m = I + alpha_m n_m n_m^T):
 *   out[16 n + 0]      sum_m K_mn
 *   out[16 n + 1]      p_n = sum_m P_mn
 *   out[16 n + 2..10]  A_n = sum_m P_mn M_m            (3x3 row-major)
 *   out[16 n + 11..13] B_n = sum_m P_mn M_m y_m
 *   out[16 n + 14]     C_n = sum_m P_mn y_m^T M_m y_m
 *   out[16 n + 15]     c_n = sum_m P_mn d_mn
 * The loops are the definition written out; OpenMP splits the sources over
 * threads, nothing else is reordered.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int oracle_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Threads of the later calls (timing runs: all cores, or one). */
void oracle_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

static double dmah(const double *x, const float *y, const float *nrm, double a) {
  const double r0 = x[0] - (double)y[0], r1 = x[1] - (double)y[1], r2 = x[2] - (double)y[2];
  const double p = (double)nrm[0] * r0 + (double)nrm[1] * r1 + (double)nrm[2] * r2;
  return r0 * r0 + r1 * r1 + r2 * r2 + a * p * p;
}

void oracle_estep_columns(const float *X, int64_t N, const float *Y, const float *nrm,
                          const float *alpha, int64_t M, const double *pi, const double *w,
                          double w0, double V, const double *R, const double *t, double sigma2,
                          int exact, const int64_t *sources, int64_t S, double *out) {
  const double gamma = pow(2.0 * M_PI * sigma2, 1.5) / V;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t s = 0; s < S; ++s) {
    const int64_t n = sources ? sources[s] : s;
    const double xs[3] = {(double)X[3 * n], (double)X[3 * n + 1], (double)X[3 * n + 2]};
    double x[3];
    for (int i = 0; i < 3; ++i)
      x[i] = R[3 * i] * xs[0] + R[3 * i + 1] * xs[1] + R[3 * i + 2] * xs[2] + t[i];
    const double wn = w ? w[n] : w0;
    const double rho = (1.0 - wn) / wn;
    double ksum = 0.0;
    for (int64_t m = 0; m < M; ++m) {
      const double a = (double)alpha[m];
      double c = rho * (pi ? pi[m] : 1.0 / (double)M);
      if (exact) c *= sqrt(1.0 + a);
      ksum += c * exp(-dmah(x, Y + 3 * m, nrm + 3 * m, a) / (2.0 * sigma2));
    }
    double acc[16] = {0};
    acc[0] = ksum;
    for (int64_t m = 0; m < M; ++m) {
      const double a = (double)alpha[m];
      double c = rho * (pi ? pi[m] : 1.0 / (double)M);
      if (exact) c *= sqrt(1.0 + a);
      const double d = dmah(x, Y + 3 * m, nrm + 3 * m, a);
      const double P = c * exp(-d / (2.0 * sigma2)) / (ksum + gamma);
      const double nv[3] = {(double)nrm[3 * m], (double)nrm[3 * m + 1], (double)nrm[3 * m + 2]};
      const double yv[3] = {(double)Y[3 * m], (double)Y[3 * m + 1], (double)Y[3 * m + 2]};
      double Mm[3][3];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Mm[i][j] = (i == j ? 1.0 : 0.0) + a * nv[i] * nv[j];
      acc[1] += P;
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) acc[2 + 3 * i + j] += P * Mm[i][j];
      double My[3];
      for (int i = 0; i < 3; ++i) My[i] = Mm[i][0] * yv[0] + Mm[i][1] * yv[1] + Mm[i][2] * yv[2];
      for (int i = 0; i < 3; ++i) acc[11 + i] += P * My[i];
      acc[14] += P * (yv[0] * My[0] + yv[1] * My[1] + yv[2] * My[2]);
      acc[15] += P * d;
    }
    for (int i = 0; i < 16; ++i) out[16 * s + i] = acc[i];
  }
}

/* sum_mn |g(x_n) - y_m|^2, the numerator of the initial sigma^2 (double loop). */
double oracle_pair_sqdist_sum(const float *X, int64_t N, const float *Y, int64_t M,
                              const double *R, const double *t) {
  double tot = 0.0;
#pragma omp parallel for reduction(+ : tot) schedule(static)
  for (int64_t n = 0; n < N; ++n) {
    double x[3];
    for (int i = 0; i < 3; ++i)
      x[i] = R[3 * i] * X[3 * n] + R[3 * i + 1] * X[3 * n + 1] + R[3 * i + 2] * X[3 * n + 2] + t[i];
    double s = 0.0;
    for (int64_t m = 0; m < M; ++m) {
      const double d0 = x[0] - Y[3 * m], d1 = x[1] - Y[3 * m + 1], d2 = x[2] - Y[3 * m + 2];
      s += d0 * d0 + d1 * d1 + d2 * d2;
    }
    tot += s;
  }
  return tot;
}

/* k nearest targets of each query (itself included, ties to the lower index),
 * float32 distances ((dx*dx + dy*dy) + dz*dz) rounded per operation; build
 * with -ffp-contract=off.  Insertion into a list sorted by (distance, index). */
void oracle_knn(const float *Y, int64_t M, int k, const int64_t *queries, int64_t Q,
                int64_t *out) {
#pragma omp parallel for schedule(dynamic, 8)
  for (int64_t s = 0; s < Q; ++s) {
    const int64_t q = queries ? queries[s] : s;
    float bd[64];
    int64_t bi[64];
    int cnt = 0;
    for (int64_t j = 0; j < M; ++j) {
      const float dx = Y[3 * q] - Y[3 * j];
      const float dy = Y[3 * q + 1] - Y[3 * j + 1];
      const float dz = Y[3 * q + 2] - Y[3 * j + 2];
      const float dd = (dx * dx + dy * dy) + dz * dz;
      if (cnt == k && !(dd < bd[k - 1])) continue;
      int pos = cnt < k ? cnt : k - 1;
      while (pos > 0 && bd[pos - 1] > dd) {
        bd[pos] = bd[pos - 1];
        bi[pos] = bi[pos - 1];
        --pos;
      }
      bd[pos] = dd;
      bi[pos] = j;
      if (cnt < k) ++cnt;
    }
    for (int i = 0; i < k; ++i) out[s * k + i] = bi[i];
  }
}
