/* Runs the FP64 oracle (compiled into this program with AddressSanitizer and
 * UndefinedBehaviorSanitizer by tests/test_oracle_pins.py) through every
 * kernel, both admissibilities, distinct point sets, the double-layer data,
 * a swap-heavy bound, the Taylor basis and the Cauchy-like generators, and
 * checks each product against the dense one.
 * Any sanitizer report or a failed check ends the program with a nonzero
 * status.  Test infrastructure only. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_build(const double *x, int64_t nx, const double *y, int64_t ny, int same_xy, int d,
                 int kid, int leaf, int p, int adm, double tol, double tau, double eps_svd,
                 double f, double diag, int has_root, const double *root_lo, double root_side,
                 int max_depth, const double *data, void **out);
int oracle_matvec(void *hv, const double *Q, int64_t R64, double *Z);
int oracle_export(void *hv, int what, void *buf, int64_t *count);
void oracle_destroy(void *hv);
int oracle_build_basis(const double *x, int64_t nx, const double *y, int64_t ny, int same_xy,
                       int d, int kid, int leaf, int p, int adm, double tol, double tau,
                       double eps_svd, double f, double diag, int has_root,
                       const double *root_lo, double root_side, int max_depth,
                       const double *data, int basis, void **out);
void oracle_cauchy_like_dense(const double *x, int64_t nx, const double *y, int64_t ny,
                              const double *w, const double *v, int p, const double *Q,
                              int64_t R, double *Z);
int oracle_cauchy_like_matvec(void *hv, const double *w, const double *v, int p,
                              const double *Q, int64_t R, double *Z);
void oracle_dense_matvec(const double *x, int64_t nx, const double *y, int64_t ny, int d, int kid,
                         double diag, const double *data_x, const double *data_y, const double *Q,
                         int64_t R, double *Z);

static uint64_t rng = 88172645463325252ull;
static double urand(void) {
  rng ^= rng << 13;
  rng ^= rng >> 7;
  rng ^= rng << 17;
  return (double)(rng >> 11) * (1.0 / 9007199254740992.0);
}

static int run(const char *name, const double *x, int64_t nx, const double *y, int64_t ny, int d,
               int kid, int leaf, int p, int adm, double tol, double eps_svd, double f,
               double diag, const double *data, double bound) {
  const int same = y == NULL;
  const int R = 3;
  void *h = NULL;
  int rc = oracle_build(x, nx, same ? x : y, same ? nx : ny, same, d, kid, leaf, p, adm, tol,
                        adm ? 0.7 : 0.6, eps_svd, f, diag, 0, NULL, 0.0, 0, data, &h);
  if (rc != 0) {
    fprintf(stderr, "%s: build failed %d\n", name, rc);
    return 1;
  }
  const int64_t nq = same ? nx : ny;
  double *Q = malloc(sizeof(double) * nq * R), *Z = malloc(sizeof(double) * nx * R),
         *Zd = malloc(sizeof(double) * nx * R);
  for (int64_t a = 0; a < nq * R; a++) Q[a] = urand() - 0.5;
  rc = oracle_matvec(h, Q, R, Z);
  oracle_dense_matvec(x, nx, same ? x : y, nq, d, kid, diag, data, data, Q, R, Zd);
  double num = 0.0, den = 0.0;
  for (int64_t a = 0; a < nx * R; a++) {
    num += (Z[a] - Zd[a]) * (Z[a] - Zd[a]);
    den += Zd[a] * Zd[a];
  }
  for (int what = 1; what <= 19; what++) {  /* every export, sized then copied */
    int64_t n = 0;
    if (oracle_export(h, what, NULL, &n) != 0 || n <= 0) continue;
    void *buf = malloc(8 * (size_t)n);
    oracle_export(h, what, buf, &n);
    free(buf);
  }
  oracle_destroy(h);
  free(Q);
  free(Z);
  free(Zd);
  const double err = sqrt(num / (den > 0 ? den : 1.0));
  printf("%s: matvec rc %d, relative error %.2e\n", name, rc, err);
  return rc != 0 || !(err < bound);
}

int main(void) {
  int bad = 0;
  const int n1 = 500, n2 = 900, n3 = 2500, nc = 400, nd = 320;
  double *x1 = malloc(sizeof(double) * n1), *x2 = malloc(sizeof(double) * 2 * n2),
         *x3 = malloc(sizeof(double) * 3 * n3), *cx = malloc(sizeof(double) * nc),
         *cy = malloc(sizeof(double) * nc), *dp = malloc(sizeof(double) * 2 * nd),
         *dd = malloc(sizeof(double) * 3 * nd);
  for (int a = 0; a < n1; a++) x1[a] = urand();
  for (int a = 0; a < 2 * n2; a++) x2[a] = urand();
  for (int a = 0; a < 3 * n3; a++) x3[a] = a % 3 == 0 && a < 3 * n3 / 2 ? 0.3 + 0.02 * urand() : urand();
  for (int a = 0; a < nc; a++) {
    cx[a] = cos(M_PI * (2.0 * a + 1.0) / (2.0 * nc));
    cy[a] = cx[a] + 1e-3 * urand();
  }
  /* the ram-head curve of Sec. 6.4 with trapezoidal Nystrom data */
  for (int k = 0; k < nd; k++) {
    const double t = (double)k / nd, tp = 2.0 * M_PI, a = tp * t, b = 2.0 * tp * t;
    const double cb = cos(b), sb = sin(b);
    const double d1 = -2.0 * tp * sin(a);
    const double d2 = tp * cos(a) + 1.4 * 4.0 * cb * cb * cb * sb * 2.0 * tp;
    const double e1 = -2.0 * tp * tp * cos(a);
    const double e2 = -tp * tp * sin(a) + 1.4 * 4.0 * (2.0 * tp) * (2.0 * tp) *
                                              (cb * cb * cb * cb - 3.0 * cb * cb * sb * sb);
    dp[2 * k] = 2.0 * cos(a);
    dp[2 * k + 1] = 1.0 + sin(a) - 1.4 * cb * cb * cb * cb;
    dd[3 * k] = d2 / nd;
    dd[3 * k + 1] = -d1 / nd;
    dd[3 * k + 2] = (e1 * d2 - e2 * d1) / (4.0 * M_PI * (d1 * d1 + d2 * d2)) / nd - 0.5;
  }
  bad += run("1/r HSS 1D", x1, n1, NULL, 0, 1, 0, 16, 8, 0, 1e-9, 1e-9, 2.0, 0.0, NULL, 1e-6);
  bad += run("log r H2 2D", x2, n2, NULL, 0, 2, 1, 32, 6, 1, 1e-7, 0.0, 2.0, 0.0, NULL, 1e-5);
  bad += run("exp(-r) H2 2D", x2, n2, NULL, 0, 2, 2, 32, 6, 1, 1e-7, 0.0, 2.0, 1.0, NULL, 1e-5);
  bad += run("1/r H2 3D swaps", x3, n3, NULL, 0, 3, 0, 32, 4, 1, 1e-6, 0.0, 1.05, 0.0, NULL, 1e-4);
  bad += run("Cauchy HSS X != Y", cx, nc, cy, nc, 1, 3, 32, 12, 0, 1e-8, 1e-9, 2.0, 0.0, NULL,
             1e-5);
  bad += run("double layer HSS", dp, nd, NULL, 0, 2, 4, 40, 5, 0, 1e-8, 1e-9, 2.0, 0.0, dd, 1e-5);
  {  /* the Taylor basis (eqs. (2.4)-(2.5)) in place of interpolation */
    const int R = 2;
    double *Q = malloc(sizeof(double) * nc * R), *Z = malloc(sizeof(double) * nc * R),
           *Zd = malloc(sizeof(double) * nc * R);
    for (int a = 0; a < nc * R; a++) Q[a] = urand() - 0.5;
    void *h = NULL;
    int rc = oracle_build_basis(cx, nc, cy, nc, 0, 1, 3, 32, 12, 0, 1e-8, 0.6, 1e-9, 2.0, 0.0, 0,
                                NULL, 0.0, 0, NULL, 1, &h);
    if (rc == 0) rc = oracle_matvec(h, Q, R, Z);
    oracle_dense_matvec(cx, nc, cy, nc, 1, 3, 0.0, NULL, NULL, Q, R, Zd);
    double num = 0.0, den = 0.0;
    for (int a = 0; a < nc * R; a++) {
      num += (Z[a] - Zd[a]) * (Z[a] - Zd[a]);
      den += Zd[a] * Zd[a];
    }
    const double err = sqrt(num / (den > 0 ? den : 1.0));
    printf("Taylor-basis HSS: rc %d, relative error %.2e\n", rc, err);
    bad += rc != 0 || !(err < 1e-6);
    if (h) oracle_destroy(h);
    free(Q);
    free(Z);
    free(Zd);
  }
  {  /* Cauchy-like generators (eqs. (6.1)-(6.2)) over the Cauchy HSS */
    const int p = 2, R = 2;
    double *w = malloc(sizeof(double) * nc * p), *v = malloc(sizeof(double) * nc * p),
           *Q = malloc(sizeof(double) * nc * R), *Z = malloc(sizeof(double) * nc * R),
           *Zd = malloc(sizeof(double) * nc * R);
    for (int a = 0; a < nc * p; a++) {
      w[a] = urand();
      v[a] = urand();
    }
    for (int a = 0; a < nc * R; a++) Q[a] = urand() - 0.5;
    void *h = NULL;
    int rc = oracle_build(cx, nc, cy, nc, 0, 1, 3, 32, 12, 0, 1e-8, 0.6, 1e-9, 2.0, 0.0, 0, NULL,
                          0.0, 0, NULL, &h);
    if (rc == 0) rc = oracle_cauchy_like_matvec(h, w, v, p, Q, R, Z);
    oracle_cauchy_like_dense(cx, nc, cy, nc, w, v, p, Q, R, Zd);
    double num = 0.0, den = 0.0;
    for (int a = 0; a < nc * R; a++) {
      num += (Z[a] - Zd[a]) * (Z[a] - Zd[a]);
      den += Zd[a] * Zd[a];
    }
    const double err = sqrt(num / (den > 0 ? den : 1.0));
    printf("Cauchy-like HSS: rc %d, relative error %.2e\n", rc, err);
    bad += rc != 0 || !(err < 1e-6);
    if (h) oracle_destroy(h);
    free(w);
    free(v);
    free(Q);
    free(Z);
    free(Zd);
  }
  free(x1);
  free(x2);
  free(x3);
  free(cx);
  free(cy);
  free(dp);
  free(dd);
  printf(bad ? "FAILED\n" : "all cases clean\n");
  return bad ? 1 : 0;
}
