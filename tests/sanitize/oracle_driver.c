/* Exercises every function of the float64 oracle (oracle/gp_oracle.c) at
 * small sizes and at its edge cases, for a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_oracle_sanitize.py).  Exit status 0
 * when every call returned what its contract says; any out-of-bounds access,
 * leak or undefined operation is reported by the sanitizers. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

double oracle_kernel(int, int, const double*, const double*, const double*, double);
void oracle_gram(int, int, int, const double*, const double*, double, double, double*);
int oracle_cholesky(int, const double*, double*, int*);
void oracle_forward_sub(int, const double*, const double*, double*);
void oracle_back_sub(int, const double*, const double*, double*);
int oracle_fit(int, int, const double*, const double*, int, const double*, double, double, int,
               double*, double*, double*, int*);
int oracle_chol_append(int, const double*, const double*, double, double*, int*);
int oracle_lml_grad(int, int, const double*, const double*, int, const double*, double, double,
                    int, double*, double*);
double oracle_ei(double, double, double);
void oracle_score(int, int, const double*, int, const double*, double, const double*,
                  const double*, const double*, int64_t, const double*, double*, double*,
                  double*, int);
void oracle_score_bound(int, int, const double*, int, const double*, double, double,
                        const double*, const double*, int64_t, const double*, double*, double*,
                        double*, int);
int64_t oracle_argmax(int64_t, const double*);
void oracle_topk(int64_t, const double*, int64_t, int64_t*);
int64_t oracle_mlp_nparams(int, int);
double oracle_bf16(double);
double oracle_gelu(double);
double oracle_gelu_grad(double);
void oracle_mlp_forward(int, int, int, const double*, int64_t, const double*, int, double*, int);
void oracle_mlp_loss_grad(int, int, int, const double*, int, const double*, const double*, int,
                          double*, double*);
void oracle_adam(int64_t, double*, double*, double*, const double*, int, double, double, double,
                 double);
void oracle_ens_ei(int, int64_t, const double*, double, double*, double*, double*);

static int failures = 0;
#define CHECK(c)                                                 \
  do {                                                           \
    if (!(c)) {                                                  \
      fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      ++failures;                                                \
    }                                                            \
  } while (0)

static double u01(unsigned* s) {
  *s = *s * 1664525u + 1013904223u;
  return (*s >> 8) * (1.0 / 16777216.0);
}

int main(void) {
  unsigned seed = 12345u;
  for (int kind = 0; kind < 2; ++kind)
    for (int n = 1; n <= 9; n += 4) {
      const int d = 3;
      double* X = malloc(sizeof(double) * (n + 1) * d);
      double* y = malloc(sizeof(double) * (n + 1));
      for (int i = 0; i < (n + 1) * d; ++i) X[i] = u01(&seed);
      for (int i = 0; i <= n; ++i) y[i] = sin(3.0 * X[i * d]) + X[i * d + 1];
      const double ls[3] = {0.4, 0.7, 1.1};
      double* K = malloc(sizeof(double) * (n + 1) * (n + 1));
      double* L = malloc(sizeof(double) * (n + 1) * (n + 1));
      double* La = malloc(sizeof(double) * (n + 1) * (n + 1));
      double* a = malloc(sizeof(double) * (n + 1));
      double* z = malloc(sizeof(double) * (n + 1));
      double st[5];
      int bad = 0;
      oracle_gram(kind, n + 1, d, X, ls, 1.3, 1e-3, K);
      CHECK(oracle_cholesky(n + 1, K, L, &bad) == 0 && bad == -1);
      oracle_forward_sub(n + 1, L, y, z);
      oracle_back_sub(n + 1, L, z, a);
      CHECK(oracle_fit(n, d, X, y, kind, ls, 1.3, 1e-3, 1, L, a, st, &bad) == 0);
      CHECK(isfinite(st[3]) && isfinite(st[4]));
      /* the factor of the first n rows extended by row n */
      double* Kn = malloc(sizeof(double) * n * n);
      double* Ln = malloc(sizeof(double) * n * n);
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Kn[i * n + j] = K[i * (n + 1) + j];
      CHECK(oracle_cholesky(n, Kn, Ln, &bad) == 0);
      double* kcol = malloc(sizeof(double) * n);
      for (int j = 0; j < n; ++j) kcol[j] = K[n * (n + 1) + j];
      CHECK(oracle_chol_append(n, Ln, kcol, K[n * (n + 1) + n], La, &bad) == 0);
      CHECK(oracle_chol_append(n, Ln, kcol, -1.0, La, &bad) == 2 && bad == n);
      double g[5], lml = 0.0;
      CHECK(oracle_lml_grad(n, d, X, y, kind, ls, 1.3, 1e-3, 1, g, &lml) == 0 && isfinite(lml));
      CHECK(oracle_lml_grad(n, d, X, y, kind, ls, 1.3, 1e-3, 0, g, &lml) == 0);
      const int64_t m = 17;
      double* Xc = malloc(sizeof(double) * m * d);
      for (int i = 0; i < m * d; ++i) Xc[i] = u01(&seed);
      double *mu = malloc(sizeof(double) * m), *sg = malloc(sizeof(double) * m),
             *ei = malloc(sizeof(double) * m);
      oracle_fit(n, d, X, y, kind, ls, 1.3, 1e-3, 1, L, a, st, &bad);
      oracle_score(n, d, X, kind, ls, 1.3, L, a, st, m, Xc, mu, sg, ei, 2);
      oracle_score(n, d, X, kind, ls, 1.3, L, a, st, m, Xc, NULL, NULL, ei, 1);
      oracle_score_bound(n, d, X, kind, ls, 1.3, 1e-3, a, st, m, Xc, mu, sg, ei, 2);
      int64_t idx[5];
      CHECK(oracle_argmax(m, ei) >= 0);
      oracle_topk(m, ei, 5, idx);
      (void)oracle_kernel(kind, d, X, Xc, ls, 1.3);
      free(X); free(y); free(K); free(L); free(La); free(a); free(z); free(Kn); free(Ln);
      free(kcol); free(Xc); free(mu); free(sg); free(ei);
    }
  /* a singular matrix and a NaN pivot */
  {
    const double K2[4] = {1.0, 1.0, 1.0, 1.0};
    double L2[4];
    int bad = 0;
    CHECK(oracle_cholesky(2, K2, L2, &bad) == 2 && bad == 1);
    const double K3[4] = {NAN, 0.0, 0.0, 1.0};
    CHECK(oracle_cholesky(2, K3, L2, &bad) == 2 && bad == 0);
  }
  /* EI at its special cases; argmax with NaN and ties; empty top-k */
  CHECK(oracle_ei(0.0, 0.0, 1.0) == 1.0 && oracle_ei(2.0, 0.0, 1.0) == 0.0);
  {
    const double v[5] = {NAN, 1.0, 3.0, 3.0, -INFINITY};
    CHECK(oracle_argmax(5, v) == 2);
    int64_t idx[5];
    oracle_topk(5, v, 5, idx);
    oracle_topk(5, v, 0, idx);
    CHECK(oracle_argmax(0, v) == -1);
  }
  CHECK(oracle_bf16(1.0) == 1.0 && isnan(oracle_bf16(NAN)));
  CHECK(oracle_gelu(0.0) == 0.0 && isfinite(oracle_gelu_grad(-3.0)));
  /* a small ensemble: forward (both roundings), gradient, Adam, ensemble EI */
  {
    const int E = 2, D = 3, H = 4;
    const int64_t P = oracle_mlp_nparams(D, H);
    double* p = malloc(sizeof(double) * E * P);
    for (int64_t i = 0; i < E * P; ++i) p[i] = u01(&seed) - 0.5;
    const int n = 6;
    double Xm[18], yt[6];
    for (int i = 0; i < 18; ++i) Xm[i] = u01(&seed);
    for (int i = 0; i < 6; ++i) yt[i] = u01(&seed);
    double out[12], grad[2 * 64], loss[2];
    CHECK(P <= 64);
    oracle_mlp_forward(E, D, H, p, n, Xm, 0, out, 1);
    oracle_mlp_forward(E, D, H, p, n, Xm, 1, out, 2);
    oracle_mlp_loss_grad(E, D, H, p, n, Xm, yt, 0, grad, loss);
    oracle_mlp_loss_grad(E, D, H, p, n, Xm, yt, 1, grad, loss);
    double* mm = calloc(E * P, sizeof(double));
    double* vv = calloc(E * P, sizeof(double));
    oracle_adam(E * P, p, mm, vv, grad, 1, 1e-3, 0.9, 0.999, 1e-8);
    double mu[6], sg[6], ei[6];
    oracle_ens_ei(E, n, out, 0.3, mu, sg, ei);
    free(p); free(mm); free(vv);
  }
  if (failures) fprintf(stderr, "%d checks failed\n", failures);
  return failures ? 1 : 0;
}
