/*
 * Plain float64 CPU oracle for the Gaussian-process fit / expected-improvement
 * scoring path.  TEST INFRASTRUCTURE ONLY: it is linked by the tests, the
 * smoke check and the benchmark's CPU-baseline leg, never by the product path,
 * and it shares no code with the HIP library.
 *
 * The paper (Sec. III-A) says each Bayesian-optimisation step trains a
 * surrogate on the evaluated configurations and lets an acquisition function
 * pick the next one; Sec. IV-D says the surrogate is a Gaussian process whose
 * training is cubic in the number of evaluations N.  It gives no formulas, so
 * this file writes out the textbook definitions:
 *
 *   kernels      squared-exponential with per-dimension lengthscales, and
 *                Matern-5/2 (Rasmussen & Williams 2006, eqs. 4.9 and 4.17);
 *   fit          K = k(X,X) + sn2 I, Cholesky K = L L^T, alpha = K^-1 ytilde,
 *                log marginal likelihood (R&W Alg. 2.1, eq. 2.30);
 *   posterior    mean k*^T alpha, variance k** - |L^-1 k*|^2 (R&W eqs. 2.25-26);
 *   acquisition  expected improvement for minimisation in closed form
 *                (Jones, Schonlau & Welch 1998, eq. 15);
 *   learned      an MLP ensemble (forward, mean-squared-error gradient, Adam as
 *   prescreen    in Kingma & Ba 2015, Alg. 1), with optional bfloat16 rounding
 *                emulation at the points where the device kernels round.
 *
 * Everything is unblocked loops in float64, in the order the definitions
 * state them.  Candidate scoring runs an OpenMP loop over candidates; each
 * candidate's arithmetic is the same serial code.  No BLAS, no LAPACK.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_NOT_PD 2
#define OR_INVALID 1

#define OR_SE 0
#define OR_MATERN52 1

static const double OR_PI = 3.14159265358979323846;

/* ---------------------------------------------------------------------- */
/* Covariance functions (R&W eq. 4.9 squared exponential with ARD, eq. 4.17 */
/* Matern nu=5/2 on the lengthscale-scaled distance).                      */
/* ---------------------------------------------------------------------- */
double oracle_kernel(int kernel, int d, const double* a, const double* b,
                     const double* ls, double sf2) {
  double r2 = 0.0;
  for (int k = 0; k < d; ++k) {
    double t = (a[k] - b[k]) / ls[k];
    r2 += t * t;
  }
  if (kernel == OR_SE) return sf2 * exp(-0.5 * r2);
  double r = sqrt(r2);
  double s5r = sqrt(5.0) * r;
  return sf2 * (1.0 + s5r + 5.0 * r2 / 3.0) * exp(-s5r);
}

/* K = k(X, X) + sn2 * I, full symmetric n x n, row-major. */
void oracle_gram(int kernel, int n, int d, const double* X, const double* ls,
                 double sf2, double sn2, double* K) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double v = oracle_kernel(kernel, d, X + (size_t)i * d, X + (size_t)j * d, ls, sf2);
      if (i == j) v += sn2;
      K[(size_t)i * n + j] = v;
    }
}

/* Cholesky-Banachiewicz, row by row, unblocked.  Writes the lower triangle of
 * L (upper set to zero).  Returns OR_NOT_PD with *bad = failing pivot when a
 * pivot is not strictly positive or not finite. */
int oracle_cholesky(int n, const double* K, double* L, int* bad) {
  memset(L, 0, sizeof(double) * (size_t)n * n);
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j <= i; ++j) {
      double s = K[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) s -= L[(size_t)i * n + k] * L[(size_t)j * n + k];
      if (i == j) {
        if (!(s > 0.0) || !isfinite(s)) {
          if (bad) *bad = i;
          return OR_NOT_PD;
        }
        L[(size_t)i * n + i] = sqrt(s);
      } else {
        L[(size_t)i * n + j] = s / L[(size_t)j * n + j];
      }
    }
  }
  if (bad) *bad = -1;
  return OR_OK;
}

/* Solve L z = b (forward substitution). */
void oracle_forward_sub(int n, const double* L, const double* b, double* z) {
  for (int i = 0; i < n; ++i) {
    double s = b[i];
    for (int k = 0; k < i; ++k) s -= L[(size_t)i * n + k] * z[k];
    z[i] = s / L[(size_t)i * n + i];
  }
}

/* Solve L^T x = z (back substitution). */
void oracle_back_sub(int n, const double* L, const double* z, double* x) {
  for (int i = n - 1; i >= 0; --i) {
    double s = z[i];
    for (int k = i + 1; k < n; ++k) s -= L[(size_t)k * n + i] * x[k];
    x[i] = s / L[(size_t)i * n + i];
  }
}

/*
 * Fit: normalise y, build K, factor, solve alpha, log marginal likelihood.
 *   stats[0] = mean of y          stats[1] = scale s_y (population std; 1 if 0
 *   stats[2] = f_best = min y                 or if normalize_y == 0)
 *   stats[3] = log marginal likelihood of ytilde
 *   stats[4] = log det K
 * L (n*n) and alpha (n) are outputs.  Returns OR_OK / OR_NOT_PD / OR_INVALID.
 */
int oracle_fit(int n, int d, const double* X, const double* y, int kernel,
               const double* ls, double sf2, double sn2, int normalize_y,
               double* L, double* alpha, double* stats, int* bad) {
  if (n <= 0 || d <= 0) return OR_INVALID;
  double mean = 0.0;
  for (int i = 0; i < n; ++i) mean += y[i];
  mean /= n;
  double var = 0.0;
  for (int i = 0; i < n; ++i) var += (y[i] - mean) * (y[i] - mean);
  var /= n;
  double sy = sqrt(var);
  if (!normalize_y || sy == 0.0) sy = 1.0;
  double fbest = y[0];
  for (int i = 1; i < n; ++i) if (y[i] < fbest) fbest = y[i];

  double* K = (double*)malloc(sizeof(double) * (size_t)n * n);
  double* yt = (double*)malloc(sizeof(double) * n);
  double* z = (double*)malloc(sizeof(double) * n);
  for (int i = 0; i < n; ++i) yt[i] = (y[i] - mean) / sy;
  oracle_gram(kernel, n, d, X, ls, sf2, sn2, K);
  int st = oracle_cholesky(n, K, L, bad);
  if (st == OR_OK) {
    oracle_forward_sub(n, L, yt, z);
    oracle_back_sub(n, L, z, alpha);
    double quad = 0.0, logdet = 0.0;
    for (int i = 0; i < n; ++i) quad += yt[i] * alpha[i];
    for (int i = 0; i < n; ++i) logdet += 2.0 * log(L[(size_t)i * n + i]);
    stats[3] = -0.5 * quad - 0.5 * logdet - 0.5 * n * log(2.0 * OR_PI);
    stats[4] = logdet;
  }
  stats[0] = mean;
  stats[1] = sy;
  stats[2] = fbest;
  free(K);
  free(yt);
  free(z);
  return st;
}

/*
 * Rank-one extension of a Cholesky factor: the re-training step of the
 * Bayesian-optimisation loop (Sec. III-A) when one evaluated configuration is
 * added and the hyperparameters stay fixed.  With K = L L^T and the bordered
 * matrix K' = [[K, k], [k^T, kappa]], the factor of K' with positive diagonal
 * is unique, and its last row follows from the block product:
 *   L' = [[L, 0], [l^T, delta]],   L l = k,   delta = sqrt(kappa - l^T l).
 * L is n x n (row-major, lower), Lout receives the (n+1) x (n+1) factor.
 * Returns OR_NOT_PD (bad = n) when kappa - l^T l is not positive.
 */
int oracle_chol_append(int n, const double* L, const double* k, double kappa, double* Lout,
                       int* bad) {
  const int n1 = n + 1;
  double* l = (double*)malloc(sizeof(double) * (n > 0 ? n : 1));
  oracle_forward_sub(n, L, k, l);
  double ll = 0.0;
  for (int j = 0; j < n; ++j) ll += l[j] * l[j];
  const double d2 = kappa - ll;
  if (!(d2 > 0.0) || !isfinite(d2)) {
    free(l);
    if (bad) *bad = n;
    return OR_NOT_PD;
  }
  memset(Lout, 0, sizeof(double) * (size_t)n1 * n1);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j <= i; ++j) Lout[(size_t)i * n1 + j] = L[(size_t)i * n + j];
  for (int j = 0; j < n; ++j) Lout[(size_t)n * n1 + j] = l[j];
  Lout[(size_t)n * n1 + n] = sqrt(d2);
  free(l);
  if (bad) *bad = -1;
  return OR_OK;
}

/*
 * Gradient of the log marginal likelihood with respect to the log
 * hyperparameters theta = (log l_1 .. log l_d, log sf2, log sn2), for the
 * hyperparameter fitting the surrogate's training performs (Sec. IV-D trains
 * a Gaussian process on each search's evaluations):
 *   dLML/dtheta_j = 1/2 tr((alpha alpha^T - K^-1) dK/dtheta_j)
 * (Rasmussen & Williams 2006, eq. 5.9), with ytilde held fixed, and
 *   dK_il/dlog l_k = [SE]       k_f(r) (x_ik - x_lk)^2 / l_k^2
 *                    [Matern52] sf2 (5/3) (1 + sqrt5 r) e^{-sqrt5 r} (x_ik - x_lk)^2 / l_k^2
 *   dK/dlog sf2 = K - sn2 I,      dK/dlog sn2 = sn2 I
 * (the chain rule through r = |(x_i - x_l) / l| of eqs. 4.9 and 4.17).
 * K^-1 is formed column by column from the Cholesky factor.  grad has d + 2
 * entries; *lml receives the log marginal likelihood.  Returns the fit's
 * status (OR_NOT_PD: no gradient).
 */
int oracle_lml_grad(int n, int d, const double* X, const double* y, int kernel, const double* ls,
                    double sf2, double sn2, int normalize_y, double* grad, double* lml) {
  double* L = (double*)malloc(sizeof(double) * (size_t)n * n);
  double* alpha = (double*)malloc(sizeof(double) * n);
  double stats[5];
  int bad = -1;
  int st = oracle_fit(n, d, X, y, kernel, ls, sf2, sn2, normalize_y, L, alpha, stats, &bad);
  if (st != OR_OK) {
    free(L);
    free(alpha);
    return st;
  }
  *lml = stats[3];
  double* Kinv = (double*)malloc(sizeof(double) * (size_t)n * n);
  double* e = (double*)malloc(sizeof(double) * n);
  double* z = (double*)malloc(sizeof(double) * n);
  double* col = (double*)malloc(sizeof(double) * n);
  for (int j = 0; j < n; ++j) {
    for (int i = 0; i < n; ++i) e[i] = i == j ? 1.0 : 0.0;
    oracle_forward_sub(n, L, e, z);
    oracle_back_sub(n, L, z, col);
    for (int i = 0; i < n; ++i) Kinv[(size_t)i * n + j] = col[i];
  }
  for (int j = 0; j < d + 2; ++j) grad[j] = 0.0;
  for (int i = 0; i < n; ++i)
    for (int l = 0; l < n; ++l) {
      const double w = alpha[i] * alpha[l] - Kinv[(size_t)i * n + l];
      const double* xi = X + (size_t)i * d;
      const double* xl = X + (size_t)l * d;
      double r2 = 0.0;
      for (int k = 0; k < d; ++k) {
        const double t = (xi[k] - xl[k]) / ls[k];
        r2 += t * t;
      }
      const double kf = oracle_kernel(kernel, d, xi, xl, ls, sf2);
      double dr;  /* dK/d(r^2 / 2) up to the sign: the factor of (x_ik - x_lk)^2 / l_k^2 */
      if (kernel == OR_SE) {
        dr = kf;
      } else {
        const double r = sqrt(r2);
        dr = sf2 * (5.0 / 3.0) * (1.0 + sqrt(5.0) * r) * exp(-sqrt(5.0) * r);
      }
      for (int k = 0; k < d; ++k) {
        const double t = (xi[k] - xl[k]) / ls[k];
        grad[k] += 0.5 * w * dr * t * t;
      }
      grad[d] += 0.5 * w * kf;
      if (i == l) grad[d + 1] += 0.5 * w * sn2;
    }
  free(L);
  free(alpha);
  free(Kinv);
  free(e);
  free(z);
  free(col);
  return OR_OK;
}

/* Expected improvement for minimisation (Jones et al. 1998):
 *   sigma > 0:  EI = (f - mu) Phi(z) + sigma phi(z),  z = (f - mu) / sigma
 *   sigma = 0:  EI = max(f - mu, 0)                                       */
double oracle_ei(double mu, double sigma, double fbest) {
  if (sigma > 0.0) {
    double imp = fbest - mu;
    double z = imp / sigma;
    double Phi = 0.5 * erfc(-z / sqrt(2.0));
    double phi = exp(-0.5 * z * z) / sqrt(2.0 * OR_PI);
    return imp * Phi + sigma * phi;
  }
  return fbest - mu > 0.0 ? fbest - mu : 0.0;
}

/*
 * Posterior and EI for m candidates Xc (m x d) given a fit.
 * Per candidate: k* = k(x*, X); mu_z = k*^T alpha; v = L^-1 k* by forward
 * substitution; var_z = max(sf2 - v^T v, 0); mu = ymean + s_y mu_z;
 * sigma = s_y sqrt(var_z); ei = EI(mu, sigma, f_best).
 * Any of mu, sigma, ei may be NULL.  nthreads <= 0 keeps the OpenMP default.
 */
void oracle_score(int n, int d, const double* X, int kernel, const double* ls,
                  double sf2, const double* L, const double* alpha,
                  const double* stats, int64_t m, const double* Xc, double* mu,
                  double* sigma, double* ei, int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
  const double ymean = stats[0], sy = stats[1], fbest = stats[2];
#pragma omp parallel
  {
    double* ks = (double*)malloc(sizeof(double) * n);
    double* v = (double*)malloc(sizeof(double) * n);
#pragma omp for schedule(static)
    for (int64_t j = 0; j < m; ++j) {
      const double* xs = Xc + (size_t)j * d;
      for (int i = 0; i < n; ++i) ks[i] = oracle_kernel(kernel, d, xs, X + (size_t)i * d, ls, sf2);
      double muz = 0.0;
      for (int i = 0; i < n; ++i) muz += ks[i] * alpha[i];
      oracle_forward_sub(n, L, ks, v);
      double vv = 0.0;
      for (int i = 0; i < n; ++i) vv += v[i] * v[i];
      double varz = sf2 - vv;
      if (varz < 0.0) varz = 0.0;
      double mj = ymean + sy * muz;
      double sj = sy * sqrt(varz);
      if (mu) mu[j] = mj;
      if (sigma) sigma[j] = sj;
      if (ei) ei[j] = oracle_ei(mj, sj, fbest);
    }
    free(ks);
    free(v);
  }
}

/*
 * Posterior mean and an upper bound of the standard deviation and of EI for
 * m candidates, from the fit alone (no triangular solve):
 *   mu as in oracle_score;
 *   conditioning on fewer observations never lowers the posterior variance
 *   of the latent function, and conditioning on the single noisy
 *   observation y_i gives  var_i = sf2 - k(x*, x_i)^2 / (sf2 + sn2);  the
 *   smallest of these (the observation with the largest covariance) bounds
 *   the full posterior variance from above:
 *     var_ub_z = max(sf2 - max_i k(x*, x_i)^2 / (sf2 + sn2), 0);
 *   sigma_ub = s_y sqrt(var_ub_z);
 *   EI grows with sigma (dEI/dsigma = phi(z) > 0), so
 *     ei_ub = EI(mu, sigma_ub, f_best) >= EI(mu, sigma, f_best).
 * Any output may be NULL.  nthreads <= 0 keeps the OpenMP default.
 */
void oracle_score_bound(int n, int d, const double* X, int kernel, const double* ls, double sf2,
                        double sn2, const double* alpha, const double* stats, int64_t m,
                        const double* Xc, double* mu, double* sigma_ub, double* ei_ub,
                        int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
  const double ymean = stats[0], sy = stats[1], fbest = stats[2];
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < m; ++j) {
    const double* xs = Xc + (size_t)j * d;
    double muz = 0.0, kmax = 0.0;
    for (int i = 0; i < n; ++i) {
      const double k = oracle_kernel(kernel, d, xs, X + (size_t)i * d, ls, sf2);
      muz += k * alpha[i];
      if (k > kmax) kmax = k;
    }
    double varz = sf2 - kmax * kmax / (sf2 + sn2);
    if (varz < 0.0) varz = 0.0;
    const double mj = ymean + sy * muz;
    const double sj = sy * sqrt(varz);
    if (mu) mu[j] = mj;
    if (sigma_ub) sigma_ub[j] = sj;
    if (ei_ub) ei_ub[j] = oracle_ei(mj, sj, fbest);
  }
}

int oracle_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Largest value; among exact ties the lowest index.  NaN never wins. */
int64_t oracle_argmax(int64_t m, const double* v) {
  int64_t best = -1;
  for (int64_t j = 0; j < m; ++j) {
    if (v[j] != v[j]) continue;
    if (best < 0 || v[j] > v[best]) best = j;
  }
  return best;
}

/* Top k by (-value, index) order: repeated selection of the next argmax among
 * the remaining entries (O(k m), written for clarity, not speed). */
void oracle_topk(int64_t m, const double* v, int64_t k, int64_t* idx) {
  unsigned char* taken = (unsigned char*)calloc((size_t)m, 1);
  for (int64_t t = 0; t < k && t < m; ++t) {
    int64_t best = -1;
    for (int64_t j = 0; j < m; ++j) {
      if (taken[j] || v[j] != v[j]) continue;
      if (best < 0 || v[j] > v[best]) best = j;
    }
    idx[t] = best;
    if (best >= 0) taken[best] = 1;
  }
  free(taken);
}

/* ---------------------------------------------------------------------- */
/* MLP ensemble: x -> GELU(W1 x + b1) -> GELU(W2 h1 + b2) -> w3 . h2 + b3   */
/* ---------------------------------------------------------------------- */
/* Parameter vector of one member, in this order:
 *   W1 (H x D, row-major), b1 (H), W2 (H x H, row-major), b2 (H), w3 (H), b3 (1)
 */
int64_t oracle_mlp_nparams(int D, int H) {
  return (int64_t)H * D + H + (int64_t)H * H + H + H + 1;
}

/* Round to float32 (nearest even), then to bfloat16 (nearest even). */
double oracle_bf16(double x) {
  float f = (float)x;
  uint32_t u;
  memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) {       /* inf / nan: truncate */
    if (u & 0x007fffffu) u |= 0x00400000u;
    u &= 0xffff0000u;
  } else {
    uint32_t lsb = (u >> 16) & 1u;
    u = (u + 0x7fffu + lsb) & 0xffff0000u;
  }
  memcpy(&f, &u, 4);
  return (double)f;
}

static double rnd(double x, int bf16) { return bf16 ? oracle_bf16(x) : x; }

/* Exact GELU u Phi(u) and its derivative Phi(u) + u phi(u). */
double oracle_gelu(double u) { return 0.5 * u * (1.0 + erf(u / sqrt(2.0))); }
double oracle_gelu_grad(double u) {
  return 0.5 * (1.0 + erf(u / sqrt(2.0))) + u * exp(-0.5 * u * u) / sqrt(2.0 * OR_PI);
}

/* Forward pass of one member for one sample; fills pre1, h1, pre2, h2 (H
 * each, h1/h2 after rounding when bf16 != 0) and returns the output. */
static double mlp_forward_one(int D, int H, const double* p, const double* x,
                              int bf16, double* pre1, double* h1, double* pre2,
                              double* h2) {
  const double* W1 = p;
  const double* b1 = W1 + (size_t)H * D;
  const double* W2 = b1 + H;
  const double* b2 = W2 + (size_t)H * H;
  const double* w3 = b2 + H;
  const double b3 = w3[H];
  for (int h = 0; h < H; ++h) {
    double s = 0.0;
    for (int k = 0; k < D; ++k) s += rnd(W1[(size_t)h * D + k], bf16) * rnd(x[k], bf16);
    pre1[h] = s + b1[h];
    h1[h] = rnd(oracle_gelu(pre1[h]), bf16);
  }
  for (int h = 0; h < H; ++h) {
    double s = 0.0;
    for (int k = 0; k < H; ++k) s += rnd(W2[(size_t)h * H + k], bf16) * h1[k];
    pre2[h] = s + b2[h];
    h2[h] = rnd(oracle_gelu(pre2[h]), bf16);
  }
  double o = 0.0;
  for (int h = 0; h < H; ++h) o += rnd(w3[h], bf16) * h2[h];
  return o + b3;
}

/* Outputs of E members on n samples: out[e*n + i]. */
void oracle_mlp_forward(int E, int D, int H, const double* params, int64_t n,
                        const double* X, int bf16, double* out, int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
  const int64_t P = oracle_mlp_nparams(D, H);
#pragma omp parallel
  {
    double* buf = (double*)malloc(sizeof(double) * 4 * H);
#pragma omp for schedule(static)
    for (int64_t t = 0; t < (int64_t)E * n; ++t) {
      int64_t e = t / n, i = t % n;
      out[t] = mlp_forward_one(D, H, params + e * P, X + i * D, bf16, buf, buf + H,
                               buf + 2 * H, buf + 3 * H);
    }
    free(buf);
  }
}

/*
 * Mean-squared-error loss (1/n) sum_i (out_i - yt_i)^2 of each member and its
 * gradient with respect to every parameter (same layout as the parameters).
 * With bf16 != 0 the backward pass rounds dpre2 and dpre1 where they feed a
 * matrix product (weight gradients of W2 / W1 and the W2^T product), matching
 * the device kernels; bias gradients use the unrounded values.
 */
void oracle_mlp_loss_grad(int E, int D, int H, const double* params, int n,
                          const double* X, const double* yt, int bf16,
                          double* grad, double* loss) {
  const int64_t P = oracle_mlp_nparams(D, H);
  double* pre1 = (double*)malloc(sizeof(double) * H);
  double* h1 = (double*)malloc(sizeof(double) * H);
  double* pre2 = (double*)malloc(sizeof(double) * H);
  double* h2 = (double*)malloc(sizeof(double) * H);
  double* dp2 = (double*)malloc(sizeof(double) * H);
  double* dh1 = (double*)malloc(sizeof(double) * H);
  double* dp1 = (double*)malloc(sizeof(double) * H);
  for (int e = 0; e < E; ++e) {
    const double* p = params + e * P;
    double* g = grad + e * P;
    memset(g, 0, sizeof(double) * P);
    const double* W2 = p + (size_t)H * D + H;
    const double* w3 = W2 + (size_t)H * H + H;
    double* gW1 = g;
    double* gb1 = gW1 + (size_t)H * D;
    double* gW2 = gb1 + H;
    double* gb2 = gW2 + (size_t)H * H;
    double* gw3 = gb2 + H;
    double* gb3 = gw3 + H;
    double L = 0.0;
    for (int i = 0; i < n; ++i) {
      const double* x = X + (size_t)i * D;
      double o = mlp_forward_one(D, H, p, x, bf16, pre1, h1, pre2, h2);
      double r = o - yt[i];
      L += r * r;
      double dout = 2.0 * r / n;
      *gb3 += dout;
      for (int h = 0; h < H; ++h) gw3[h] += dout * h2[h];
      for (int h = 0; h < H; ++h) {
        double dh2 = dout * rnd(w3[h], bf16);
        double d = dh2 * oracle_gelu_grad(pre2[h]);
        gb2[h] += d;
        dp2[h] = rnd(d, bf16);
      }
      for (int h = 0; h < H; ++h)
        for (int k = 0; k < H; ++k) gW2[(size_t)h * H + k] += dp2[h] * h1[k];
      for (int k = 0; k < H; ++k) {
        double s = 0.0;
        for (int h = 0; h < H; ++h) s += rnd(W2[(size_t)h * H + k], bf16) * dp2[h];
        dh1[k] = s;
      }
      for (int h = 0; h < H; ++h) {
        double d = dh1[h] * oracle_gelu_grad(pre1[h]);
        gb1[h] += d;
        dp1[h] = rnd(d, bf16);
      }
      for (int h = 0; h < H; ++h)
        for (int k = 0; k < D; ++k) gW1[(size_t)h * D + k] += dp1[h] * rnd(x[k], bf16);
    }
    loss[e] = L / n;
  }
  free(pre1); free(h1); free(pre2); free(h2); free(dp2); free(dh1); free(dp1);
}

/* One Adam step (Kingma & Ba 2015, Alg. 1) on P parameters; t is the 1-based
 * step number used for bias correction. */
void oracle_adam(int64_t P, double* w, double* m, double* v, const double* g,
                 int t, double lr, double beta1, double beta2, double eps) {
  double c1 = 1.0 - pow(beta1, t);
  double c2 = 1.0 - pow(beta2, t);
  for (int64_t i = 0; i < P; ++i) {
    m[i] = beta1 * m[i] + (1.0 - beta1) * g[i];
    v[i] = beta2 * v[i] + (1.0 - beta2) * g[i] * g[i];
    double mh = m[i] / c1;
    double vh = v[i] / c2;
    w[i] -= lr * mh / (sqrt(vh) + eps);
  }
}

/* Ensemble posterior and EI: mean and population standard deviation over the
 * E member outputs (out[e*n + i]), then EI(mu, sigma, fbest) per sample. */
void oracle_ens_ei(int E, int64_t n, const double* out, double fbest,
                   double* mu, double* sigma, double* ei) {
  for (int64_t i = 0; i < n; ++i) {
    double s = 0.0;
    for (int e = 0; e < E; ++e) s += out[(int64_t)e * n + i];
    double mean = s / E;
    double q = 0.0;
    for (int e = 0; e < E; ++e) {
      double t = out[(int64_t)e * n + i] - mean;
      q += t * t;
    }
    double sd = sqrt(q / E);
    if (mu) mu[i] = mean;
    if (sigma) sigma[i] = sd;
    if (ei) ei[i] = oracle_ei(mean, sd, fbest);
  }
}
