/* FP64 CPU oracle for the block Vecchia log-likelihood -- TEST INFRASTRUCTURE.
 *
 * Only the test-suite, the smoke check and the benchmark's CPU-baseline leg
 * load this library.  It shares no code with the HIP library.
 *
 * bvo_loglik   : per block, one factor of eq. (vecchia-vector) by its
 *                definition, log p(y_B | y_N) = log N(y_J; 0, K_J) -
 *                log N(y_N; 0, K_N) with J = N u B: each Gaussian log-density
 *                from its own dense Cholesky factorisation (Matern covariance,
 *                eq. (maternkernel), plus the nugget on same-index pairs).
 * bvo_grad     : per block, the gradient of log p(y_J) - log p(y_N) w.r.t.
 *                (sigma2, beta, nugget) by the textbook trace formula
 *                0.5 tr[(alpha alpha^T - K^-1) dK], alpha = K^-1 y, with K^-1 from an
 *                explicit triangular inverse.
 * bvo_simulate : draws from the block Vecchia density (data generation).
 * Blocks run in parallel (OpenMP); each writes its own slot, and the caller
 * sums the slots in block order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define BVO_LOG2PI 1.8378770664093454835606594728112

typedef struct {
  double sigma2, beta, nugget, nu;
  double aniso[3];
} bvo_theta;

static double rho_of(double x, double nu) {
  double e = exp(-x);
  if (nu == 0.5) return e;
  if (nu == 1.5) return (1.0 + x) * e;
  return (1.0 + x + x * x / 3.0) * e; /* nu == 2.5 */
}

/* d rho / d beta at x = h / beta */
static double drho_dbeta(double x, double beta, double nu) {
  double e = exp(-x), g;
  if (nu == 0.5) g = e;
  else if (nu == 1.5) g = x * e;
  else g = (x / 3.0) * (1.0 + x) * e;
  return (x / beta) * g;
}

static double hdist(const double* si, const double* sj, int d, const bvo_theta* th) {
  double acc = 0.0;
  for (int k = 0; k < d; ++k) {
    double t = (si[k] - sj[k]) / th->aniso[k];
    acc += t * t;
  }
  return sqrt(acc);
}

static double cov(const double* si, const double* sj, int d, const bvo_theta* th, int same) {
  double c = th->sigma2 * rho_of(hdist(si, sj, d, th) / th->beta, th->nu);
  if (same) c += th->nugget;
  return c;
}

/* Unblocked Cholesky, lower, row-major n x n; returns 0 or -1 if not PD. */
static int potrf(double* A, int n) {
  for (int j = 0; j < n; ++j) {
    double s = A[j * n + j];
    for (int k = 0; k < j; ++k) s -= A[j * n + k] * A[j * n + k];
    if (!(s > 0.0)) return -1;
    double ljj = sqrt(s);
    A[j * n + j] = ljj;
    for (int i = j + 1; i < n; ++i) {
      double t = A[i * n + j];
      for (int k = 0; k < j; ++k) t -= A[i * n + k] * A[j * n + k];
      A[i * n + j] = t / ljj;
    }
    for (int i = 0; i < j; ++i) A[i * n + j] = 0.0;
  }
  return 0;
}

/* Solve L X = B in place; L n x n lower (row-major), B n x c (row-major). */
static void trsm_lower(const double* L, int n, double* B, int c) {
  for (int i = 0; i < n; ++i) {
    for (int k = 0; k < i; ++k) {
      double lik = L[i * n + k];
      for (int q = 0; q < c; ++q) B[i * c + q] -= lik * B[k * c + q];
    }
    for (int q = 0; q < c; ++q) B[i * c + q] /= L[i * n + i];
  }
}

/* log N(y_S; 0, K_S) for the points S = idx[0..p): K_S = L L^T, w = L^-1 y_S,
 * value -p log(2 pi) / 2 - sum log L_jj - w^T w / 2.  NaN if K_S is not PD.
 * work: p * p + p doubles. */
static double logpdf(const double* locs, const double* y, int d, const int64_t* idx, int p,
                     const bvo_theta* th, double* work) {
  double* K = work;
  double* w = K + (size_t)p * p;
  for (int i = 0; i < p; ++i) {
    for (int j = 0; j < p; ++j) K[i * p + j] = cov(locs + idx[i] * d, locs + idx[j] * d, d, th, i == j);
    w[i] = y[idx[i]];
  }
  if (potrf(K, p)) return NAN;
  trsm_lower(K, p, w, 1);
  double q = 0.0, ld = 0.0;
  for (int i = 0; i < p; ++i) {
    q += w[i] * w[i];
    ld += log(K[i * p + i]);
  }
  return -0.5 * p * BVO_LOG2PI - ld - 0.5 * q;
}

/* One block term: log N(y_J) - log N(y_N), J = (neighbours, block points). */
static double block_loglik(const double* locs, const double* y, int d, int64_t b0, int64_t b1,
                           const int64_t* nn, int m, const bvo_theta* th, int64_t* J, double* work) {
  int l = (int)(b1 - b0);
  for (int k = 0; k < m; ++k) J[k] = nn[k];
  for (int k = 0; k < l; ++k) J[m + k] = b0 + k;
  double v = logpdf(locs, y, d, J, m + l, th, work);
  if (m > 0) v -= logpdf(locs, y, d, J, m, th, work);
  return v;
}

/* Gradient of log N(y_S; 0, K_S) w.r.t. (sigma2, beta, nugget), S = idx[0..p). */
static int logpdf_grad(const double* locs, const double* y, int d, const int64_t* idx, int p,
                       const bvo_theta* th, double* g, double* work) {
  double* K = work;               /* p x p -> L */
  double* Li = K + p * p;         /* p x p inverse of L */
  double* Ki = Li + p * p;        /* p x p */
  double* al = Ki + p * p;        /* p */
  for (int i = 0; i < p; ++i)
    for (int j = 0; j < p; ++j)
      K[i * p + j] = cov(locs + idx[i] * d, locs + idx[j] * d, d, th, i == j);
  if (potrf(K, p)) return -1;
  memset(Li, 0, sizeof(double) * p * p);
  for (int i = 0; i < p; ++i) Li[i * p + i] = 1.0;
  trsm_lower(K, p, Li, p);                      /* Li = L^-1 */
  for (int i = 0; i < p; ++i)                   /* K^-1 = L^-T L^-1 */
    for (int j = 0; j < p; ++j) {
      double s = 0.0;
      for (int k = (i > j ? i : j); k < p; ++k) s += Li[k * p + i] * Li[k * p + j];
      Ki[i * p + j] = s;
    }
  for (int i = 0; i < p; ++i) {
    double s = 0.0;
    for (int j = 0; j < p; ++j) s += Ki[i * p + j] * y[idx[j]];
    al[i] = s;
  }
  g[0] = g[1] = g[2] = 0.0;
  for (int i = 0; i < p; ++i)
    for (int j = 0; j < p; ++j) {
      double w = al[i] * al[j] - Ki[i * p + j];
      double x = hdist(locs + idx[i] * d, locs + idx[j] * d, d, th) / th->beta;
      g[0] += w * rho_of(x, th->nu);
      g[1] += w * th->sigma2 * drho_dbeta(x, th->beta, th->nu);
      if (i == j) g[2] += w;
    }
  g[0] *= 0.5; g[1] *= 0.5; g[2] *= 0.5;
  return 0;
}

static int max_block(const int64_t* block_ptr, int64_t bc, const int64_t* nbr_ptr, int* lmax, int* mmax) {
  int a = 0, b = 0;
  for (int64_t i = 0; i < bc; ++i) {
    int l = (int)(block_ptr[i + 1] - block_ptr[i]);
    int m = (int)(nbr_ptr[i + 1] - nbr_ptr[i]);
    if (l > a) a = l;
    if (m > b) b = m;
  }
  *lmax = a; *mmax = b;
  return 0;
}

/* Per-block log-likelihood terms.  Returns the number of non-PD blocks (their
 * terms are NaN). */
int64_t bvo_loglik_sel(const double* locs, const double* y, int64_t n, int32_t d,
                       const int64_t* block_ptr, int64_t bc, const int64_t* nbr_ptr, const int64_t* nbr_idx,
                       const double* theta7, const int64_t* sel, int64_t nsel, double* partial, int32_t nthreads) {
  (void)n;
  bvo_theta th = {theta7[0], theta7[1], theta7[2], theta7[3], {theta7[4], theta7[5], theta7[6]}};
  int lmax, mmax;
  max_block(block_ptr, bc, nbr_ptr, &lmax, &mmax);
  const int pmax = lmax + mmax;
  size_t wsz = (size_t)pmax * pmax + pmax + 8;
  int64_t bad = 0;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel reduction(+ : bad)
  {
    double* work = (double*)malloc(sizeof(double) * wsz);
    int64_t* J = (int64_t*)malloc(sizeof(int64_t) * (pmax + 1));
#pragma omp for schedule(dynamic, 16)
    for (int64_t q = 0; q < nsel; ++q) {
      int64_t i = sel ? sel[q] : q;
      int m = (int)(nbr_ptr[i + 1] - nbr_ptr[i]);
      double v = block_loglik(locs, y, d, block_ptr[i], block_ptr[i + 1], nbr_idx + nbr_ptr[i], m, &th, J, work);
      partial[q] = v;
      if (isnan(v)) bad += 1;
    }
    free(work);
    free(J);
  }
  return bad;
}

/* Per-block gradient rows gpartial[3*i + k], k = (sigma2, beta, nugget). */
int64_t bvo_grad_sel(const double* locs, const double* y, int64_t n, int32_t d,
                     const int64_t* block_ptr, int64_t bc, const int64_t* nbr_ptr, const int64_t* nbr_idx,
                     const double* theta7, const int64_t* sel, int64_t nsel, double* gpartial, int32_t nthreads) {
  (void)n;
  bvo_theta th = {theta7[0], theta7[1], theta7[2], theta7[3], {theta7[4], theta7[5], theta7[6]}};
  int lmax, mmax;
  max_block(block_ptr, bc, nbr_ptr, &lmax, &mmax);
  int pmax = lmax + mmax;
  size_t wsz = 3 * (size_t)pmax * pmax + pmax + 8;
  int64_t bad = 0;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel reduction(+ : bad)
  {
    double* work = (double*)malloc(sizeof(double) * wsz);
    int64_t* J = (int64_t*)malloc(sizeof(int64_t) * (pmax + 1));
#pragma omp for schedule(dynamic, 8)
    for (int64_t q = 0; q < nsel; ++q) {
      int64_t i = sel ? sel[q] : q;
      int m = (int)(nbr_ptr[i + 1] - nbr_ptr[i]);
      int l = (int)(block_ptr[i + 1] - block_ptr[i]);
      for (int k = 0; k < m; ++k) J[k] = nbr_idx[nbr_ptr[i] + k];
      for (int k = 0; k < l; ++k) J[m + k] = block_ptr[i] + k;
      double gj[3], gn[3] = {0.0, 0.0, 0.0};
      int e = logpdf_grad(locs, y, d, J, m + l, &th, gj, work);
      if (!e && m > 0) e = logpdf_grad(locs, y, d, J, m, &th, gn, work);
      for (int k = 0; k < 3; ++k) gpartial[3 * q + k] = e ? NAN : gj[k] - gn[k];
      if (e) bad += 1;
    }
    free(work);
    free(J);
  }
  return bad;
}

/* Whole-workload entry points (every block, in order). */
int64_t bvo_loglik(const double* locs, const double* y, int64_t n, int32_t d, const int64_t* block_ptr, int64_t bc,
                   const int64_t* nbr_ptr, const int64_t* nbr_idx, const double* theta7, double* partial,
                   int32_t nthreads) {
  return bvo_loglik_sel(locs, y, n, d, block_ptr, bc, nbr_ptr, nbr_idx, theta7, NULL, bc, partial, nthreads);
}
int64_t bvo_grad(const double* locs, const double* y, int64_t n, int32_t d, const int64_t* block_ptr, int64_t bc,
                 const int64_t* nbr_ptr, const int64_t* nbr_idx, const double* theta7, double* gpartial,
                 int32_t nthreads) {
  return bvo_grad_sel(locs, y, n, d, block_ptr, bc, nbr_ptr, nbr_idx, theta7, NULL, bc, gpartial, nthreads);
}

/* Sequential simulation from the block Vecchia density (eq. (vecchia-vector)),
 * blocks in order: y_B = mu + chol(S) z_B with mu = K_BN K_NN^-1 y_N and
 * S = K_BB - K_BN K_NN^-1 K_NB.  With blocks of size one and N(i) the nearest
 * earlier points this is the sequential (classic) Vecchia simulator.  Sequential
 * over blocks: each block reads values drawn for earlier blocks. */
int64_t bvo_simulate(const double* locs, int64_t n, int32_t d, const int64_t* block_ptr, int64_t bc,
                     const int64_t* nbr_ptr, const int64_t* nbr_idx, const double* theta7, const double* z,
                     double* y) {
  (void)n;
  bvo_theta th = {theta7[0], theta7[1], theta7[2], theta7[3], {theta7[4], theta7[5], theta7[6]}};
  int lmax, mmax;
  max_block(block_ptr, bc, nbr_ptr, &lmax, &mmax);
  double* work = (double*)malloc(sizeof(double) * ((size_t)lmax * lmax + (size_t)mmax * mmax +
                                                   (size_t)mmax * lmax + mmax + 2 * lmax + 8));
  int64_t bad = 0;
  for (int64_t i = 0; i < bc; ++i) {
    int64_t b0 = block_ptr[i], b1 = block_ptr[i + 1];
    int l = (int)(b1 - b0), m = (int)(nbr_ptr[i + 1] - nbr_ptr[i]);
    const int64_t* nn = nbr_idx + nbr_ptr[i];
    double* S = work;              /* l x l */
    double* Kn = S + l * l;        /* m x m */
    double* Kc = Kn + m * m;       /* m x l */
    double* yn = Kc + m * l;       /* m */
    double* mu = yn + m;           /* l */
    for (int a = 0; a < l; ++a)
      for (int b = 0; b < l; ++b) S[a * l + b] = cov(locs + (b0 + a) * d, locs + (b0 + b) * d, d, &th, a == b);
    for (int a = 0; a < l; ++a) mu[a] = 0.0;
    if (m > 0) {
      for (int a = 0; a < m; ++a) {
        for (int b = 0; b < m; ++b) Kn[a * m + b] = cov(locs + nn[a] * d, locs + nn[b] * d, d, &th, a == b);
        for (int b = 0; b < l; ++b) Kc[a * l + b] = cov(locs + nn[a] * d, locs + (b0 + b) * d, d, &th, 0);
        yn[a] = y[nn[a]];
      }
      if (potrf(Kn, m)) { bad++; continue; }
      trsm_lower(Kn, m, Kc, l);
      trsm_lower(Kn, m, yn, 1);
      for (int a = 0; a < l; ++a) {
        double s = 0.0;
        for (int k = 0; k < m; ++k) s += Kc[k * l + a] * yn[k];
        mu[a] = s;
        for (int b = 0; b < l; ++b) {
          double t = 0.0;
          for (int k = 0; k < m; ++k) t += Kc[k * l + a] * Kc[k * l + b];
          S[a * l + b] -= t;
        }
      }
    }
    if (potrf(S, l)) { bad++; continue; }
    for (int a = 0; a < l; ++a) {
      double s = mu[a];
      for (int k = 0; k <= a; ++k) s += S[a * l + k] * z[b0 + k];
      y[b0 + a] = s;
    }
  }
  free(work);
  return bad;
}
