/* Drives the oracle's entry points on small inputs, for a build with AddressSanitizer
 * and UndefinedBehaviorSanitizer: every call must finish without a report and with
 * finite results.  The values themselves are checked by the oracle's Python tests. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

void orc_direct(int L, const double *d, const double *k, int N, const double *x, const double *y,
                const double *z, const int *lay, const double *q, int n_tgt, const int *tgt, double b, int what,
                double *phi_out);
void orc_fmm(int L, const double *d, const double *k, int p, int leaf_max, int max_depth, double qb, int N,
             const double *x, const double *y, const double *z, const int *lay, const double *q, int what,
             double *phi_out, int *info_out);
void orc_reaction_T(int L, const double *d, const double *k, int l, int a, int lp, int b, double dx, double dy,
                    double zt, double zs, int p, double qb, double *out);
void orc_reaction_T_mass(int L, const double *d, const double *k, int l, int a, int lp, int b, double dx,
                         double dy, double zt, double zs, int p, double qb, double *out);
void orc_translation(int kind, double k, const double *bv, int p, double *op_out);
void orc_densities(int L, const double *d, const double *k, double kr_re, double kr_im, int l, int lp,
                   double *out);

static unsigned long long rs = 88172645463325252ull;
static double urand(void) {  /* xorshift64, uniform on [0, 1) */
  rs ^= rs << 13;
  rs ^= rs >> 7;
  rs ^= rs << 17;
  return (double)(rs >> 11) * (1.0 / 9007199254740992.0);
}

static int finite_all(const double *v, int n) {
  for (int i = 0; i < n; i++)
    if (!isfinite(v[i])) return 0;
  return 1;
}

int main(void) {
  const int L = 2;
  const double d[2] = {0.0, -1.2}, k[3] = {0.8, 1.5, 2.0};
  const double zc[3] = {0.6, -0.6, -1.8};
  const int N = 240;
  double *x = malloc(sizeof(double) * N), *y = malloc(sizeof(double) * N), *z = malloc(sizeof(double) * N);
  double *q = malloc(sizeof(double) * 2 * N), *phi = malloc(sizeof(double) * 2 * N);
  int *lay = malloc(sizeof(int) * N), *tgt = malloc(sizeof(int) * N);
  for (int i = 0; i < N; i++) {
    int l = i % 3;
    x[i] = urand() - 0.5;
    y[i] = urand() - 0.5;
    z[i] = zc[l] + 0.9 * (urand() - 0.5);
    lay[i] = l;
    q[2 * i] = 2 * urand() - 1;
    q[2 * i + 1] = 2 * urand() - 1;
    tgt[i] = i;
  }
  int bad = 0;
  orc_direct(L, d, k, N, x, y, z, lay, q, 16, tgt, 0.5, 3, phi);
  bad += !finite_all(phi, 32);
  int info[L + 2];
  orc_fmm(L, d, k, 4, 20, 8, 0.5, N, x, y, z, lay, q, 3, phi, info);
  bad += !finite_all(phi, 2 * N);
  const int p = 6, NC = (p + 1) * (p + 1);
  double *T = malloc(sizeof(double) * 2 * NC * NC), *M = malloc(sizeof(double) * NC * NC);
  orc_reaction_T(L, d, k, 1, 0, 1, 1, 0.3, -0.2, 0.15, 0.25, p, 0.5, T);
  bad += !finite_all(T, 2 * NC * NC);
  orc_reaction_T_mass(L, d, k, 0, 0, 2, 1, 0.1, 0.0, 0.2, 0.1, p, 0.5, M);
  bad += !finite_all(M, NC * NC);
  const double bv[3] = {0.25, -0.25, 0.25};
  for (int kind = 0; kind < 2; kind++) {
    orc_translation(kind, 1.5, bv, p, T);
    bad += !finite_all(T, 2 * NC * NC);
  }
  double sig[8];
  orc_densities(L, d, k, 0.7, -0.1, 1, 2, sig);
  bad += !finite_all(sig, 8);
  free(x), free(y), free(z), free(q), free(phi), free(lay), free(tgt), free(T), free(M);
  printf("oracle run: %s\n", bad ? "non-finite results" : "ok");
  return bad ? 1 : 0;
}
