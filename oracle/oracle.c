/*
 * Layered-media Helmholtz FMM oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU implementation of what the layered-media FMM of
 * Wang, Zhang & Cai ("Fast multipole method for 3-D Helmholtz equation in
 * layered media", SISC 2019) computes.  Only the test suite, the package's
 * smoke() check and the cpu_baseline leg of bench.py may load it.  It shares
 * no code, table or constant generator with the HIP library: every special
 * function, quadrature rule, density solve, tree rule and translation operator
 * below is written here from the paper and the mathematics.
 *
 * Two levels of reference are provided:
 *   (1) orc_direct_*  -- the exact quantity: direct summation of the layered
 *       Green's function (free part in closed form, the reaction part by
 *       Sommerfeld quadrature), Section 3.4 eq. (totalinteraction).
 *   (2) orc_fmm       -- the paper's approximation: a plain FMM that follows
 *       Algorithm 1 for every reaction component and the classic FMM for every
 *       free-space component, truncated at order p, on the uniform octrees
 *       defined by the tree rule stated at orc_fmm.
 *
 * Conventions (Section 2.1): Y_n^m = Phat_n^m(cos t) e^{i m phi}, Phat without
 * the Condon-Shortley phase, Phat_n^{-m} = (-1)^m Phat_n^m.  Coefficient
 * arrays are indexed idx(n,m) = n*n + n + m, n = 0..p, |m| <= n.
 * The Phi normalization multiplies physical potentials by 4 pi/(i k_l)
 * (Section 3.4, the factor omitted after eq. (totalinteraction)).
 */
#define _GNU_SOURCE
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;
#define PI 3.14159265358979323846264338327950288
#define NGL 16
#define DMAX 8
#define LMAXL 16

static int idx(int n, int m) { return n * n + n + m; }
static int tidx(int n, int m) { return n * (n + 1) / 2 + m; }
static cplx ipow(int n) {
  int r = ((n % 4) + 4) % 4;
  return r == 0 ? 1.0 : r == 1 ? I : r == 2 ? -1.0 : -I;
}
static double msign(int m) { return (m & 1) ? -1.0 : 1.0; }

/* ------------------------------------------------------------------------- */
/* Special functions                                                          */
/* ------------------------------------------------------------------------- */

/* Spherical Bessel j_n(x), n = 0..nmax, real x >= 0: Miller's backward
 * recurrence f_{n-1} = (2n+1)/x f_n - f_{n+1}, normalised by the closed form of
 * j_0 or j_1 (whichever is larger in magnitude). */
void orc_sph_j(int nmax, double x, double *out) {
  if (x == 0.0) {
    out[0] = 1.0;
    for (int n = 1; n <= nmax; n++) out[n] = 0.0;
    return;
  }
  int top = (nmax > 1 ? nmax : 1);
  int N = top + (int)x + 40;
  double *f = (double *)malloc(sizeof(double) * (top + 1));
  double fn1 = 0.0, fn = 1.0;
  for (int n = N; n >= 1; n--) {
    double fm = (2.0 * n + 1.0) / x * fn - fn1;
    fn1 = fn;
    fn = fm; /* fn now holds f_{n-1}, fn1 holds f_n */
    if (n - 1 <= top) f[n - 1] = fn;
    if (n <= top) f[n] = fn1;
    if (fabs(fn) > 1e250) {
      fn *= 1e-250;
      fn1 *= 1e-250;
      for (int j = n - 1; j <= top; j++)
        if (j >= 0) f[j] *= 1e-250;
    }
  }
  double j0 = sin(x) / x, j1 = sin(x) / (x * x) - cos(x) / x;
  double sc = (fabs(j0) >= fabs(j1)) ? j0 / f[0] : j1 / f[1];
  for (int n = 0; n <= nmax; n++) out[n] = f[n] * sc;
  free(f);
}

/* Spherical Bessel y_n(x), x > 0, upward recurrence. */
void orc_sph_y(int nmax, double x, double *out) {
  out[0] = -cos(x) / x;
  if (nmax >= 1) out[1] = -cos(x) / (x * x) - sin(x) / x;
  for (int n = 1; n < nmax; n++) out[n + 1] = (2.0 * n + 1.0) / x * out[n] - out[n - 1];
}

/* Spherical Hankel h_n^(1)(x) = j_n + i y_n, x > 0. */
static void sph_h(int nmax, double x, cplx *out) {
  double *j = (double *)malloc(sizeof(double) * (nmax + 2));
  double *y = (double *)malloc(sizeof(double) * (nmax + 2));
  orc_sph_j(nmax, x, j);
  orc_sph_y(nmax, x, y);
  for (int n = 0; n <= nmax; n++) out[n] = j[n] + I * y[n];
  free(j);
  free(y);
}

/* Hankel's asymptotic expansion of J_nu(z) for large |z| (|arg z| < pi). */
static cplx hankel_asym_J(int nu, cplx z) {
  double mu = 4.0 * nu * nu;
  cplx P = 1.0, Q = 0.0, term = 1.0;
  for (int k = 1; k < 80; k++) {
    term *= (mu - (2.0 * k - 1.0) * (2.0 * k - 1.0)) / (8.0 * k * z);
    if (k & 1)
      Q += (((k - 1) / 2) & 1 ? -1.0 : 1.0) * term;
    else
      P += ((k / 2) & 1 ? -1.0 : 1.0) * term;
    if (cabs(term) < 1e-18) break;
  }
  cplx w = z - nu * PI / 2.0 - PI / 4.0;
  return csqrt(2.0 / (PI * z)) * (P * ccos(w) - Q * csin(w));
}

/* Cylindrical Bessel J_n(z), n = 0..nmax, complex z.  |z| <= 25 (or nmax large):
 * Miller's backward recurrence J_{n-1} = (2n/z) J_n - J_{n+1}, normalised with the
 * generating-function sum e^{+iz} = J_0 + 2 sum i^n J_n (Im z <= 0) or
 * e^{-iz} = J_0 + 2 sum (-i)^n J_n (Im z > 0).  |z| > 25: Hankel's expansion for
 * J_0, J_1 and forward recurrence (stable for n < |z|). */
void orc_bessel_J(int nmax, cplx z, cplx *out) {
  double az = cabs(z);
  if (az == 0.0) {
    out[0] = 1.0;
    for (int n = 1; n <= nmax; n++) out[n] = 0.0;
    return;
  }
  if (az < 1.0) { /* power series J_n(z) = sum_k (-1)^k (z/2)^{2k+n} / (k! (n+k)!) */
    cplx h = 0.5 * z, h2 = h * h, hn = 1.0;
    double nf = 1.0;
    for (int n = 0; n <= nmax; n++) {
      if (n > 0) {
        hn *= h;
        nf *= n;
      }
      cplx term = hn / nf, s = term;
      for (int kk = 1; kk < 40; kk++) {
        term *= -h2 / ((double)kk * (n + kk));
        s += term;
        if (cabs(term) < 1e-18 * cabs(s)) break;
      }
      out[n] = s;
    }
    return;
  }
  if (az > 25.0 && nmax <= az / 2.0) {
    out[0] = hankel_asym_J(0, z);
    if (nmax >= 1) out[1] = hankel_asym_J(1, z);
    for (int n = 1; n < nmax; n++) out[n + 1] = (2.0 * n) / z * out[n] - out[n - 1];
    return;
  }
  int top = nmax;
  int N = nmax + (int)az + 40;
  cplx w = (cimag(z) <= 0.0) ? I : -I;
  cplx *f = (cplx *)malloc(sizeof(cplx) * (top + 1));
  cplx fn1 = 0.0, fn = 1e-30; /* f_{N+1}, f_N */
  /* normalisation sum: J_0 + 2 sum_{n>=1} w^n J_n, accumulated downward */
  cplx wn; /* w^N, exact powers of +-i */
  {
    int r = N % 4;
    wn = (r == 0) ? 1.0 : (r == 1) ? w : (r == 2) ? -1.0 : -w;
  }
  cplx S = 2.0 * wn * fn;
  if (N <= top) f[N] = fn;
  for (int n = N; n >= 1; n--) {
    cplx fm = (2.0 * n) / z * fn - fn1;
    fn1 = fn;
    fn = fm; /* f_{n-1} */
    wn = wn / w;  /* w^{n-1} */
    if (n - 1 <= top) f[n - 1] = fn;
    S += (n - 1 == 0 ? 1.0 : 2.0) * wn * fn;
    if (cabs(fn) > 1e250) {
      fn *= 1e-250;
      fn1 *= 1e-250;
      S *= 1e-250;
      for (int j = n - 1; j <= top; j++)
        if (j >= 0) f[j] *= 1e-250;
    }
  }
  cplx target = (cimag(z) <= 0.0) ? cexp(I * z) : cexp(-I * z);
  cplx sc = target / S;
  for (int n = 0; n <= nmax; n++) out[n] = f[n] * sc;
  free(f);
}

/* sqrt(1 - z^2) with the branch of eq. (branch): cut on [-1,1],
 * sqrt(1-z^2) = -i sqrt(r1 r2) e^{i (t1+t2)/2}, z+1 = r1 e^{i t1}, z-1 = r2 e^{i t2}. */
cplx orc_branch_sqrt(cplx z) {
  double r1 = cabs(z + 1.0), t1 = carg(z + 1.0);
  double r2 = cabs(z - 1.0), t2 = carg(z - 1.0);
  return -I * sqrt(r1 * r2) * cexp(I * 0.5 * (t1 + t2));
}

/* Normalised associated Legendre Phat_n^m(x), 0 <= m <= n <= p, given x and
 * s = sqrt(1 - x^2) on the chosen branch (Section 2.2 recurrences, with
 * Phat_0^0 = 1/sqrt(4 pi)).  out[tidx(n,m)]. */
void orc_legendre(int p, cplx x, cplx s, cplx *out) {
  out[0] = 1.0 / sqrt(4.0 * PI);
  for (int m = 1; m <= p; m++)
    out[tidx(m, m)] = sqrt((2.0 * m + 1.0) / (2.0 * m)) * s * out[tidx(m - 1, m - 1)];
  for (int m = 0; m < p; m++) out[tidx(m + 1, m)] = sqrt(2.0 * m + 3.0) * x * out[tidx(m, m)];
  for (int m = 0; m <= p; m++)
    for (int n = m + 2; n <= p; n++) {
      double a = sqrt((2.0 * n - 1.0) * (2.0 * n + 1.0) / ((double)(n - m) * (n + m)));
      double b = sqrt((2.0 * n + 1.0) * (n - m - 1.0) * (n + m - 1.0) /
                      ((2.0 * n - 3.0) * (n + m) * (double)(n - m)));
      out[tidx(n, m)] = a * x * out[tidx(n - 1, m)] - b * out[tidx(n - 2, m)];
    }
}

/* Phat_n^m for any m (|m| <= n) from a table over m >= 0. */
static cplx phat(const cplx *tab, int n, int m) {
  return m >= 0 ? tab[tidx(n, m)] : msign(m) * tab[tidx(n, -m)];
}

/* Y_n^m at a real direction given by a cartesian vector (x,y,z). */
void orc_sph_harm(int p, double x, double y, double z, cplx *Y) {
  double r = sqrt(x * x + y * y + z * z);
  double ct = (r > 0.0) ? z / r : 1.0;
  double st = (r > 0.0) ? sqrt(x * x + y * y) / r : 0.0;
  double ph = atan2(y, x);
  int nt = (p + 1) * (p + 2) / 2;
  cplx *tab = (cplx *)malloc(sizeof(cplx) * nt);
  orc_legendre(p, ct, st, tab);
  for (int n = 0; n <= p; n++)
    for (int m = -n; m <= n; m++) Y[idx(n, m)] = phat(tab, n, m) * cexp(I * m * ph);
  free(tab);
}

/* ------------------------------------------------------------------------- */
/* Gauss-Legendre rule on [-1,1] (Newton on P_n)                              */
/* ------------------------------------------------------------------------- */
static double gl_x[NGL], gl_w[NGL];
static int gl_ready = 0;
static void gl_init(void) {
  if (gl_ready) return;
  int n = NGL;
  for (int i = 0; i < n; i++) {
    double x = cos(PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; it++) {
      double p0 = 1.0, p1 = x;
      for (int k = 2; k <= n; k++) {
        double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      double dp = n * (x * p1 - p0) / (x * x - 1.0);
      double dx = p1 / dp;
      x -= dx;
      if (fabs(dx) < 1e-16) break;
    }
    double p0 = 1.0, p1 = x;
    for (int k = 2; k <= n; k++) {
      double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    double dp = n * (x * p1 - p0) / (x * x - 1.0);
    gl_x[i] = x;
    gl_w[i] = 2.0 / ((1.0 - x * x) * dp * dp);
  }
  gl_ready = 1;
}
void orc_gauss_legendre(double *x, double *w) {
  gl_init();
  for (int i = 0; i < NGL; i++) {
    x[i] = gl_x[i];
    w[i] = gl_w[i];
  }
}

/* ------------------------------------------------------------------------- */
/* Layered medium: densities by the dense 2L x 2L interface system            */
/* ------------------------------------------------------------------------- */
typedef struct {
  int L;               /* number of interfaces; layers 0..L */
  double d[LMAXL];     /* interfaces, top to bottom, strictly decreasing */
  double k[LMAXL + 1]; /* wavenumbers, layer 0 = top (z > d_0) */
} stack_t;

static cplx kz_of(double k, cplx kr) { return csqrt(k * k - kr * kr); }

/* Complex Gaussian elimination with partial pivoting; A is n x n row-major,
 * B is n x nr.  Solution overwrites B. */
static void csolve(int n, cplx *A, int nr, cplx *B) {
  for (int c = 0; c < n; c++) {
    int piv = c;
    double best = cabs(A[c * n + c]);
    for (int r = c + 1; r < n; r++)
      if (cabs(A[r * n + c]) > best) {
        best = cabs(A[r * n + c]);
        piv = r;
      }
    if (piv != c) {
      for (int j = 0; j < n; j++) {
        cplx t = A[c * n + j];
        A[c * n + j] = A[piv * n + j];
        A[piv * n + j] = t;
      }
      for (int j = 0; j < nr; j++) {
        cplx t = B[c * nr + j];
        B[c * nr + j] = B[piv * nr + j];
        B[piv * nr + j] = t;
      }
    }
    for (int r = c + 1; r < n; r++) {
      cplx f = A[r * n + c] / A[c * n + c];
      if (f == 0.0) continue;
      for (int j = c; j < n; j++) A[r * n + j] -= f * A[c * n + j];
      for (int j = 0; j < nr; j++) B[r * nr + j] -= f * B[c * nr + j];
    }
  }
  for (int c = n - 1; c >= 0; c--) {
    for (int j = 0; j < nr; j++) {
      cplx s = B[c * nr + j];
      for (int k = c + 1; k < n; k++) s -= A[c * n + k] * B[k * nr + j];
      B[c * nr + j] = s / A[c * n + c];
    }
  }
}

/* Reaction densities sigma^{ab}_{l,lp}(k_rho) (Section 3.1, eqs. (greenfuncomponent)
 * and (totaldensity)).  In layer m the reaction field has the spectral form
 *   [U_m e^{i kz_m (z - d_m)} + D_m e^{i kz_m (d_{m-1} - z)}] / kz_m,
 * (no U in layer L, no D in layer 0); the source layer also carries the free wave
 * e^{i kz |z - z'|}/kz.  At every interface the field and k_m times its
 * z-derivative are continuous.  sigma^{a b}: a = 0 (up, U_l) or 1 (down, D_l);
 * b = 0 for unit excitation X_b = e^{i kz_lp (z' - d_lp)} (the source's wave
 * arriving at the bottom interface), b = 1 for unit X_t = e^{i kz_lp (d_{lp-1} - z')}.
 * Entries that do not exist are returned as 0. */
void orc_densities_c(const stack_t *st, cplx kr, int l, int lp, cplx sig[2][2]) {
  int L = st->L, n = 2 * L;
  cplx kz[LMAXL + 1], E[LMAXL + 1];
  for (int m = 0; m <= L; m++) kz[m] = kz_of(st->k[m], kr);
  for (int m = 1; m <= L - 1; m++) E[m] = cexp(I * kz[m] * (st->d[m - 1] - st->d[m]));
  cplx *A = (cplx *)calloc((size_t)n * n, sizeof(cplx));
  cplx B[2 * LMAXL * 2];
  memset(B, 0, sizeof(B));
  /* unknown columns: U_m -> m (m = 0..L-1); D_m -> L + m - 1 (m = 1..L) */
  for (int j = 0; j < L; j++) {
    int rv = 2 * j, rd = 2 * j + 1;
    /* layer j (above interface j) */
    A[rv * n + j] += 1.0 / kz[j];
    A[rd * n + j] += st->k[j];
    if (j >= 1) {
      A[rv * n + (L + j - 1)] += E[j] / kz[j];
      A[rd * n + (L + j - 1)] += -st->k[j] * E[j];
    }
    /* layer j+1 (below interface j), moved to the left-hand side with a minus */
    if (j + 1 <= L - 1) {
      A[rv * n + (j + 1)] -= E[j + 1] / kz[j + 1];
      A[rd * n + (j + 1)] -= st->k[j + 1] * E[j + 1];
    }
    A[rv * n + (L + j)] -= 1.0 / kz[j + 1];
    A[rd * n + (L + j)] -= -st->k[j + 1];
  }
  /* right-hand sides: column 0 -> X_b = 1, column 1 -> X_t = 1 */
  if (lp <= L - 1) { /* free wave at interface lp, source layer above it */
    B[(2 * lp) * 2 + 0] += -1.0 / kz[lp];
    B[(2 * lp + 1) * 2 + 0] += st->k[lp];
  }
  if (lp >= 1) { /* free wave at interface lp-1, source layer below it */
    B[(2 * (lp - 1)) * 2 + 1] += 1.0 / kz[lp];
    B[(2 * (lp - 1) + 1) * 2 + 1] += st->k[lp];
  }
  csolve(n, A, 2, B);
  for (int b = 0; b < 2; b++) {
    int exists_b = (b == 0) ? (lp <= L - 1) : (lp >= 1);
    sig[0][b] = (exists_b && l <= L - 1) ? B[l * 2 + b] : 0.0;
    sig[1][b] = (exists_b && l >= 1) ? B[(L + l - 1) * 2 + b] : 0.0;
  }
  free(A);
}

static void make_stack(stack_t *st, int L, const double *d, const double *k) {
  st->L = L;
  for (int i = 0; i < L; i++) st->d[i] = d[i];
  for (int i = 0; i <= L; i++) st->k[i] = k[i];
}

/* ctypes entry: sig_out[4] = (up,up), (up,down), (down,up), (down,down) as re/im pairs */
void orc_densities(int L, const double *d, const double *k, double kr_re, double kr_im, int l, int lp,
                   double *sig_out) {
  stack_t st;
  make_stack(&st, L, d, k);
  cplx sig[2][2];
  orc_densities_c(&st, kr_re + I * kr_im, l, lp, sig);
  for (int a = 0; a < 2; a++)
    for (int b = 0; b < 2; b++) {
      sig_out[2 * (2 * a + b)] = creal(sig[a][b]);
      sig_out[2 * (2 * a + b) + 1] = cimag(sig[a][b]);
    }
}

/* Height of a point in layer l above the bottom interface (a = 0) or below the
 * top interface (a = 1); the distances in the exponentials of eq. (mekernel). */
static double h_up(const stack_t *st, int l, double z) { return z - st->d[l]; }
static double h_dn(const stack_t *st, int l, double z) { return st->d[l - 1] - z; }
static double hdist(const stack_t *st, int l, int a, double z) {
  return a == 0 ? h_up(st, l, z) : h_dn(st, l, z);
}
static int has_dir(const stack_t *st, int l, int a) { return a == 0 ? (l <= st->L - 1) : (l >= 1); }

/* ------------------------------------------------------------------------- */
/* Sommerfeld contour and quadrature rule (Section 3.5 contour Gamma1 u Gamma2) */
/* ------------------------------------------------------------------------- */
typedef struct {
  int n;
  cplx *kr, *w;
} qrule_t;

/* smallest x > N with x - N ln(x/N) - N >= c  (decay of t^N e^{-t dz} below e^{-c}
 * of its peak, in the variable x = t dz) */
static double decay_len(int N, double c) {
  if (N <= 0) return c;
  double lo = N, hi = N + c + 10.0 * N + 10.0;
  for (int it = 0; it < 200; it++) {
    double mid = 0.5 * (lo + hi);
    double v = mid - N * log(mid / N) - N;
    if (v >= c) hi = mid; else lo = mid;
  }
  return hi;
}

/* Nodes and weights (dk_rho included) on Gamma1: k_rho = -i s, s in [0,b]
 * (2 panels) and Gamma2: k_rho = t - i b: near part [0, T0] in panels of 0.5,
 * far part up to T0 + U/dz in panels of length min(4/dz, 4/rho, 4).  dz is the
 * smallest vertical decay distance of the integrand, rho the largest radial
 * argument of the Bessel factor, npow the power growth of the integrand. */
static qrule_t make_rule(double b, double kmax, double dz, double rho, int npow) {
  gl_init();
  double T0 = 0.5 * ceil(2.0 * (kmax + 2.0));
  double U = decay_len(npow, 41.5);
  double tfar = U / dz;
  double P = 4.0 / dz;
  if (rho > 0.0 && 4.0 / rho < P) P = 4.0 / rho;
  if (P > 4.0) P = 4.0;
  int nfar = (int)ceil(tfar / P);
  int nnear = (int)llround(T0 / 0.5);
  int np = 2 + nnear + nfar;
  qrule_t q;
  q.n = np * NGL;
  q.kr = (cplx *)malloc(sizeof(cplx) * q.n);
  q.w = (cplx *)malloc(sizeof(cplx) * q.n);
  int c = 0;
  for (int pnl = 0; pnl < 2; pnl++) {
    double s0 = b * pnl / 2.0, s1 = b * (pnl + 1) / 2.0, mid = 0.5 * (s0 + s1), hw = 0.5 * (s1 - s0);
    for (int g = 0; g < NGL; g++) {
      q.kr[c] = -I * (mid + hw * gl_x[g]);
      q.w[c] = -I * hw * gl_w[g];
      c++;
    }
  }
  for (int pnl = 0; pnl < nnear; pnl++) {
    double t0 = 0.5 * pnl, mid = t0 + 0.25, hw = 0.25;
    for (int g = 0; g < NGL; g++) {
      q.kr[c] = (mid + hw * gl_x[g]) - I * b;
      q.w[c] = hw * gl_w[g];
      c++;
    }
  }
  double plen = tfar / nfar;
  for (int pnl = 0; pnl < nfar; pnl++) {
    double t0 = T0 + plen * pnl, mid = t0 + 0.5 * plen, hw = 0.5 * plen;
    for (int g = 0; g < NGL; g++) {
      q.kr[c] = (mid + hw * gl_x[g]) - I * b;
      q.w[c] = hw * gl_w[g];
      c++;
    }
  }
  return q;
}
static void free_rule(qrule_t *q) {
  free(q->kr);
  free(q->w);
}

static double stack_kmax(const stack_t *st) {
  double km = 0;
  for (int i = 0; i <= st->L; i++)
    if (st->k[i] > km) km = st->k[i];
  return km;
}

/* Quadrature check: (1/k) int_Gamma k_rho J_0(k_rho rho) e^{i kz dz}/kz dk_rho,
 * which the Sommerfeld identity (eq. (sommerfeldid)) makes equal to
 * h_0(k sqrt(rho^2 + dz^2)). */
void orc_sommerfeld_h0(double k, double rho, double dz, double b, double scale, double *out) {
  qrule_t q = make_rule(b, k, dz / scale, rho * scale, 0);
  cplx s = 0;
  cplx J[2];
  for (int i = 0; i < q.n; i++) {
    cplx kr = q.kr[i], kz = kz_of(k, kr);
    orc_bessel_J(0, kr * rho, J);
    s += q.w[i] * kr * J[0] * cexp(I * kz * dz) / kz;
  }
  s /= k;
  out[0] = creal(s);
  out[1] = cimag(s);
  out[2] = q.n;
  free_rule(&q);
}

/* ------------------------------------------------------------------------- */
/* Direct summation of the layered Green's function (the exact quantity)      */
/* ------------------------------------------------------------------------- */
static cplx h0(double x) { return cexp(I * x) / (I * x); }

/* Per (target layer, source layer) quadrature table: nodes, weights and the
 * four densities at each node. */
typedef struct {
  qrule_t q;
  cplx *sig; /* [node][a][b] */
  cplx *kzt, *kzs;
} lptab_t;

static void build_lptab(lptab_t *t, const stack_t *st, int l, int lp, double dzmin, double rhomax, int npow,
                        double b) {
  t->q = make_rule(b, stack_kmax(st), dzmin, rhomax, npow);
  int n = t->q.n;
  t->sig = (cplx *)malloc(sizeof(cplx) * 4 * n);
  t->kzt = (cplx *)malloc(sizeof(cplx) * n);
  t->kzs = (cplx *)malloc(sizeof(cplx) * n);
  for (int i = 0; i < n; i++) {
    cplx s[2][2];
    orc_densities_c(st, t->q.kr[i], l, lp, s);
    for (int a = 0; a < 2; a++)
      for (int bb = 0; bb < 2; bb++) t->sig[4 * i + 2 * a + bb] = s[a][bb];
    t->kzt[i] = kz_of(st->k[l], t->q.kr[i]);
    t->kzs[i] = kz_of(st->k[lp], t->q.kr[i]);
  }
}
static void free_lptab(lptab_t *t) {
  free_rule(&t->q);
  free(t->sig);
  free(t->kzt);
  free(t->kzs);
}

/* Reaction kernel in the Phi normalisation for target (x,y,z) in layer l and
 * source (x',y',z') in layer lp, summed over the existing (a,b) components:
 *   G = (1/k_l) int k_rho J0(k_rho rho) sum_ab e^{i kz_l h_a(z) + i kz_lp h_b(z')}
 *       sigma^{ab}(k_rho)/kz_l dk_rho . */
static cplx reaction_pair(const stack_t *st, const lptab_t *t, int l, int lp, double rho, double z, double zp) {
  double ht[2], hs[2];
  int ea[2], eb[2];
  for (int a = 0; a < 2; a++) {
    ea[a] = has_dir(st, l, a);
    ht[a] = ea[a] ? hdist(st, l, a, z) : 0.0;
    eb[a] = has_dir(st, lp, a);
    hs[a] = eb[a] ? hdist(st, lp, a, zp) : 0.0;
  }
  cplx s = 0;
  cplx J[2];
  for (int i = 0; i < t->q.n; i++) {
    cplx kr = t->q.kr[i], kzt = t->kzt[i], kzs = t->kzs[i];
    cplx acc = 0;
    for (int a = 0; a < 2; a++) {
      if (!ea[a]) continue;
      cplx et = cexp(I * kzt * ht[a]);
      for (int b = 0; b < 2; b++) {
        if (!eb[b]) continue;
        acc += et * cexp(I * kzs * hs[b]) * t->sig[4 * i + 2 * a + b];
      }
    }
    orc_bessel_J(0, kr * rho, J);
    s += t->q.w[i] * kr * J[0] * acc / kzt;
  }
  return s / st->k[l];
}

/* Smallest decay distance among the present (a,b) terms over sets of target
 * and source heights: min_a min h_t^a + min_b min h_s^b. */
static double min_h(const stack_t *st, int l, int n, const double *z, const int *lay, const int *sel, int nsel) {
  double best = INFINITY;
  for (int a = 0; a < 2; a++) {
    if (!has_dir(st, l, a)) continue;
    for (int ii = 0; ii < (sel ? nsel : n); ii++) {
      int i = sel ? sel[ii] : ii;
      if (lay[i] != l) continue;
      double h = hdist(st, l, a, z[i]);
      if (h < best) best = h;
    }
  }
  return best;
}

/* Potentials Phi_l(r_i) for the listed targets (eq. (totalinteraction)), by direct
 * summation over all N sources.  phi_out: 2*n_tgt doubles (re, im).
 * what: 1 = free part only, 2 = reaction part only, 3 = both. */
void orc_direct(int L, const double *d, const double *k, int N, const double *x, const double *y,
                const double *z, const int *lay, const double *q, int n_tgt, const int *tgt, double b, int what,
                double *phi_out) {
  gl_init();
  stack_t st;
  make_stack(&st, L, d, k);
  double xlo = INFINITY, xhi = -INFINITY, ylo = INFINITY, yhi = -INFINITY;
  for (int i = 0; i < N; i++) {
    if (x[i] < xlo) xlo = x[i];
    if (x[i] > xhi) xhi = x[i];
    if (y[i] < ylo) ylo = y[i];
    if (y[i] > yhi) yhi = y[i];
  }
  double rhomax = sqrt((xhi - xlo) * (xhi - xlo) + (yhi - ylo) * (yhi - ylo));
  lptab_t tabs[LMAXL + 1][LMAXL + 1];
  int have[LMAXL + 1][LMAXL + 1];
  memset(have, 0, sizeof(have));
  if (what & 2) {
    for (int l = 0; l <= L; l++) {
      double ht = min_h(&st, l, n_tgt, z, lay, tgt, n_tgt);
      if (!isfinite(ht)) continue;
      for (int lp = 0; lp <= L; lp++) {
        double hs = min_h(&st, lp, N, z, lay, NULL, 0);
        if (!isfinite(hs)) continue;
        build_lptab(&tabs[l][lp], &st, l, lp, ht + hs, rhomax, 0, b);
        have[l][lp] = 1;
      }
    }
  }
  for (int tt = 0; tt < n_tgt; tt++) {
    int i = tgt[tt], l = lay[i];
    double sre = 0.0, sim = 0.0;
#pragma omp parallel for reduction(+ : sre, sim) schedule(dynamic, 64)
    for (int j = 0; j < N; j++) {
      cplx qj = q[2 * j] + I * q[2 * j + 1];
      cplx v = 0;
      double dx = x[i] - x[j], dy = y[i] - y[j], dzz = z[i] - z[j];
      if ((what & 1) && lay[j] == l && j != i) {
        double r = sqrt(dx * dx + dy * dy + dzz * dzz);
        if (r > 0.0) v += qj * h0(k[l] * r);
      }
      if ((what & 2) && have[l][lay[j]]) {
        double rho = sqrt(dx * dx + dy * dy);
        v += qj * reaction_pair(&st, &tabs[l][lay[j]], l, lay[j], rho, z[i], z[j]);
      }
      sre += creal(v);
      sim += cimag(v);
    }
    phi_out[2 * tt] = sre;
    phi_out[2 * tt + 1] = sim;
  }
  for (int l = 0; l <= L; l++)
    for (int lp = 0; lp <= L; lp++)
      if (have[l][lp]) free_lptab(&tabs[l][lp]);
}

/* Spectral Green's function of the stack at one k_rho, for checks of the
 * densities (reciprocity, equal wavenumbers, layer merge):
 *   g(z,z') = sum_ab e^{i kz_l h_a(z) + i kz_lp h_b(z')} sigma^{ab}/kz_l
 *             [+ e^{i kz_l |z - z'|}/kz_l if l == lp and with_free]. */
void orc_spectral_g(int L, const double *d, const double *k, double kr_re, double kr_im, int l, double z, int lp,
                    double zp, int with_free, double *out) {
  stack_t st;
  make_stack(&st, L, d, k);
  cplx kr = kr_re + I * kr_im;
  cplx sig[2][2];
  orc_densities_c(&st, kr, l, lp, sig);
  cplx kzt = kz_of(k[l], kr), kzs = kz_of(k[lp], kr);
  cplx g = 0;
  for (int a = 0; a < 2; a++) {
    if (!has_dir(&st, l, a)) continue;
    for (int bb = 0; bb < 2; bb++) {
      if (!has_dir(&st, lp, bb)) continue;
      g += cexp(I * kzt * hdist(&st, l, a, z) + I * kzs * hdist(&st, lp, bb, zp)) * sig[a][bb] / kzt;
    }
  }
  if (with_free && l == lp) g += cexp(I * kzt * fabs(z - zp)) / kzt;
  out[0] = creal(g);
  out[1] = cimag(g);
}

/* ------------------------------------------------------------------------- */
/* Wigner 3j, Gaunt coefficients and free-space translation operators         */
/* ------------------------------------------------------------------------- */
static long double lfact(int n) {
  int sg;
  return lgammal_r((long double)n + 1.0L, &sg);
}

/* Racah's formula for the Wigner 3j symbol. */
double orc_wigner3j(int j1, int j2, int j3, int m1, int m2, int m3) {
  if (m1 + m2 + m3 != 0) return 0.0;
  if (abs(m1) > j1 || abs(m2) > j2 || abs(m3) > j3) return 0.0;
  if (j3 < abs(j1 - j2) || j3 > j1 + j2) return 0.0;
  long double lpre = 0.5L * (lfact(j1 + j2 - j3) + lfact(j1 - j2 + j3) + lfact(-j1 + j2 + j3) -
                             lfact(j1 + j2 + j3 + 1) + lfact(j1 + m1) + lfact(j1 - m1) + lfact(j2 + m2) +
                             lfact(j2 - m2) + lfact(j3 + m3) + lfact(j3 - m3));
  int tmin = 0, tmax = j1 + j2 - j3;
  if (j2 - j3 - m1 > tmin) tmin = j2 - j3 - m1;
  if (j1 - j3 + m2 > tmin) tmin = j1 - j3 + m2;
  if (j1 - m1 < tmax) tmax = j1 - m1;
  if (j2 + m2 < tmax) tmax = j2 + m2;
  long double s = 0.0L;
  for (int t = tmin; t <= tmax; t++) {
    long double lt = lfact(t) + lfact(j3 - j2 + t + m1) + lfact(j3 - j1 + t - m2) + lfact(j1 + j2 - j3 - t) +
                     lfact(j1 - t - m1) + lfact(j2 - t + m2);
    long double term = expl(lpre - lt);
    s += (t & 1) ? -term : term;
  }
  int ph = j1 - j2 - m3;
  return (double)(((ph % 2) != 0) ? -s : s);
}

/* G(a,al; c,ga; e) = int Y_a^al Y_c^ga conj(Y_e^{al+ga}) dOmega
 *   = (-1)^{al+ga} sqrt((2a+1)(2c+1)(2e+1)/(4 pi)) (a c e;0 0 0)(a c e; al ga -al-ga),
 * the Gaunt coefficient of Section 2.1. */
double orc_gaunt(int a, int al, int c, int ga, int e) {
  double w0 = orc_wigner3j(a, c, e, 0, 0, 0);
  if (w0 == 0.0) return 0.0;
  double w1 = orc_wigner3j(a, c, e, al, ga, -al - ga);
  return msign(al + ga) * sqrt((2.0 * a + 1.0) * (2.0 * c + 1.0) * (2.0 * e + 1.0) / (4.0 * PI)) * w0 * w1;
}

/* Translation operator of the addition theorems (Section 2.1):
 *   new_{nm} = sum_{nu mu} Op[idx(n,m)][idx(nu,mu)] old_{nu mu},
 *   Op = 4 pi i^{n-nu} sum_q i^q z_q(k|b|) conj(Y_q^{m-mu}(b^)) G(nu,mu; q,m-mu; n),
 * z = j_q (kind 0: expansion-centre shifts, M2M with b = P - c, L2L with b = c - P)
 * or h_q (kind 1: M2L with b = c_t - c_s). */
void orc_translation(int kind, double k, const double *bv, int p, double *op_out) {
  int NC = (p + 1) * (p + 1);
  int Q = 2 * p;
  double bb = sqrt(bv[0] * bv[0] + bv[1] * bv[1] + bv[2] * bv[2]);
  cplx *zq = (cplx *)malloc(sizeof(cplx) * (Q + 1));
  if (kind == 0) {
    double *jj = (double *)malloc(sizeof(double) * (Q + 2));
    orc_sph_j(Q, k * bb, jj);
    for (int qq = 0; qq <= Q; qq++) zq[qq] = jj[qq];
    free(jj);
  } else {
    sph_h(Q, k * bb, zq);
  }
  int NQ = (Q + 1) * (Q + 1);
  cplx *Yq = (cplx *)malloc(sizeof(cplx) * NQ);
  orc_sph_harm(Q, bv[0], bv[1], bv[2], Yq);
  for (int n = 0; n <= p; n++)
    for (int m = -n; m <= n; m++)
      for (int nu = 0; nu <= p; nu++)
        for (int mu = -nu; mu <= nu; mu++) {
          int s = m - mu;
          cplx acc = 0;
          for (int qq = abs(n - nu); qq <= n + nu; qq++) {
            if (((n + nu + qq) & 1) || abs(s) > qq) continue;
            double g = orc_gaunt(nu, mu, qq, s, n);
            if (g == 0.0) continue;
            acc += ipow(qq) * zq[qq] * conj(Yq[idx(qq, s)]) * g;
          }
          cplx v = 4.0 * PI * ipow(n - nu) * acc;
          op_out[2 * ((size_t)idx(n, m) * NC + idx(nu, mu))] = creal(v);
          op_out[2 * ((size_t)idx(n, m) * NC + idx(nu, mu)) + 1] = cimag(v);
        }
  free(zq);
  free(Yq);
}

/* Multipole (M) or local (L) coefficients of a unit point source at offset rv
 * from the expansion centre (eq. (melecoeffree)):
 *   kind 0: M_nm = 4 pi j_n(k r) conj(Y_n^m(r^))   kind 1: L_nm = 4 pi h_n(k r) conj(Y_n^m(r^)) */
void orc_point_expansion(int kind, double k, const double *rv, int p, double *out) {
  int NC = (p + 1) * (p + 1);
  double r = sqrt(rv[0] * rv[0] + rv[1] * rv[1] + rv[2] * rv[2]);
  cplx *zn = (cplx *)malloc(sizeof(cplx) * (p + 2));
  if (kind == 0) {
    double *jj = (double *)malloc(sizeof(double) * (p + 2));
    orc_sph_j(p, k * r, jj);
    for (int n = 0; n <= p; n++) zn[n] = jj[n];
    free(jj);
  } else {
    sph_h(p, k * r, zn);
  }
  cplx *Y = (cplx *)malloc(sizeof(cplx) * NC);
  orc_sph_harm(p, rv[0], rv[1], rv[2], Y);
  for (int n = 0; n <= p; n++)
    for (int m = -n; m <= n; m++) {
      cplx v = 4.0 * PI * zn[n] * conj(Y[idx(n, m)]);
      out[2 * idx(n, m)] = creal(v);
      out[2 * idx(n, m) + 1] = cimag(v);
    }
  free(zn);
  free(Y);
}

/* Evaluate an expansion at offset rv from its centre: kind 0 (multipole) sum
 * M_nm h_n(k r) Y_n^m(r^); kind 1 (local) sum L_nm j_n(k r) Y_n^m(r^). */
void orc_eval_expansion(int kind, double k, const double *coef, const double *rv, int p, double *out) {
  int NC = (p + 1) * (p + 1);
  double r = sqrt(rv[0] * rv[0] + rv[1] * rv[1] + rv[2] * rv[2]);
  cplx *zn = (cplx *)malloc(sizeof(cplx) * (p + 2));
  if (kind == 1) {
    double *jj = (double *)malloc(sizeof(double) * (p + 2));
    orc_sph_j(p, k * r, jj);
    for (int n = 0; n <= p; n++) zn[n] = jj[n];
    free(jj);
  } else {
    sph_h(p, k * r, zn);
  }
  cplx *Y = (cplx *)malloc(sizeof(cplx) * NC);
  orc_sph_harm(p, rv[0], rv[1], rv[2], Y);
  cplx s = 0;
  for (int n = 0; n <= p; n++)
    for (int m = -n; m <= n; m++) s += (coef[2 * idx(n, m)] + I * coef[2 * idx(n, m) + 1]) * zn[n] * Y[idx(n, m)];
  out[0] = creal(s);
  out[1] = cimag(s);
  free(zn);
  free(Y);
}

/* ------------------------------------------------------------------------- */
/* Reaction-component expansions in the polarisation frame                    */
/* ------------------------------------------------------------------------- */
/* All reaction work is done in a frame where the interface of the component is
 * z = 0, targets sit at height ht > 0 above it and the equivalent polarisation
 * sources (eq. (eqpolarizedsource)) at depth hs > 0 below it; for a target
 * direction a = down the frame is mirrored in z.  The kernel there is
 *   G(r, r_s) = (1/k_t) int k_rho J0(k_rho rho) e^{i kz_t ht + i kz_s hs} sigma/kz_t dk_rho
 * with kz_t for the target layer, kz_s for the source layer (eqs.
 * (zexponentialimage), (generalcomponentsimag), in the Phi normalisation). */

/* Reaction M2L operator (eqs. (metoleimage1), (metoleimage2), (me2lesimplified))
 * between a target centre at height zt > 0 and a source centre at depth zs > 0,
 * lateral offset (dx, dy) = target minus source:
 *   T_{nm,n'm'} = (4 pi / k_t) i^n (-i)^{n'} i^q e^{i q phi}
 *       int k_rho J_q(k_rho rho) e^{i kz_t zt + i kz_s zs} sigma/kz_t
 *           Phat_n^m(kz_t/k_t) Phat_{n'}^{m'}(kz_s/k_s) dk_rho,   q = m' - m.
 * op_out[idx(n,m)][idx(n',m')]. */
static void reaction_T(const stack_t *st, int l, int a, int lp, int b, double dx, double dy, double zt, double zs,
                       int p, double qb, cplx *T) {
  int NC = (p + 1) * (p + 1), NT = (p + 1) * (p + 2) / 2, Q = 2 * p;
  double rho = sqrt(dx * dx + dy * dy), phi = atan2(dy, dx);
  double kt = st->k[l], ks = st->k[lp];
  qrule_t qr = make_rule(qb, stack_kmax(st), zt + zs, rho, 2 * p + 1);
  cplx *I_ = (cplx *)calloc((size_t)NC * NC, sizeof(cplx));
  cplx *Pt = (cplx *)malloc(sizeof(cplx) * NT), *Ps = (cplx *)malloc(sizeof(cplx) * NT);
  cplx *J = (cplx *)malloc(sizeof(cplx) * (Q + 1));
  for (int i = 0; i < qr.n; i++) {
    cplx kr = qr.kr[i];
    cplx kzt = kz_of(kt, kr), kzs = kz_of(ks, kr);
    cplx sig[2][2];
    orc_densities_c(st, kr, l, lp, sig);
    cplx f = qr.w[i] * kr * cexp(I * kzt * zt + I * kzs * zs) * sig[a][b] / kzt;
    orc_bessel_J(Q, kr * rho, J);
    orc_legendre(p, kzt / kt, orc_branch_sqrt(kzt / kt), Pt);
    orc_legendre(p, kzs / ks, orc_branch_sqrt(kzs / ks), Ps);
    for (int n = 0; n <= p; n++)
      for (int m = -n; m <= n; m++) {
        cplx pt = phat(Pt, n, m) * f;
        for (int n2 = 0; n2 <= p; n2++)
          for (int m2 = -n2; m2 <= n2; m2++) {
            int qq = m2 - m;
            cplx Jq = qq >= 0 ? J[qq] : msign(qq) * J[-qq];
            I_[(size_t)idx(n, m) * NC + idx(n2, m2)] += pt * phat(Ps, n2, m2) * Jq;
          }
      }
  }
  for (int n = 0; n <= p; n++)
    for (int m = -n; m <= n; m++)
      for (int n2 = 0; n2 <= p; n2++)
        for (int m2 = -n2; m2 <= n2; m2++) {
          int qq = m2 - m;
          /* i^n (-i)^{n'} = i^n i^{-n'} */
          cplx c = (4.0 * PI / kt) * ipow(n) * ipow(-n2) * ipow(qq) * cexp(I * (double)qq * phi);
          T[(size_t)idx(n, m) * NC + idx(n2, m2)] = c * I_[(size_t)idx(n, m) * NC + idx(n2, m2)];
        }
  free(I_);
  free(Pt);
  free(Ps);
  free(J);
  free_rule(&qr);
}

/* Rounding scale of reaction_T: the same quadrature with every term replaced by
 * its modulus, sum_i |w_i k_rho J_q e^{...} sigma/kz_t Phat Phat| times the
 * prefactor modulus.  Differences between two correct quadratures of the
 * oscillatory integrals (Section 3.5) are bounded by a small multiple of
 * eps times this mass. */
void orc_reaction_T_mass(int L, const double *d, const double *k, int l, int a, int lp, int b, double dx, double dy,
                         double zt, double zs, int p, double qb, double *out) {
  stack_t st;
  make_stack(&st, L, d, k);
  int NC = (p + 1) * (p + 1), NT = (p + 1) * (p + 2) / 2, Q = 2 * p;
  double rho = sqrt(dx * dx + dy * dy);
  double kt = st.k[l], ks = st.k[lp];
  qrule_t qr = make_rule(qb, stack_kmax(&st), zt + zs, rho, 2 * p + 1);
  double *mass = (double *)calloc((size_t)NC * NC, sizeof(double));
  cplx *Pt = (cplx *)malloc(sizeof(cplx) * NT), *Ps = (cplx *)malloc(sizeof(cplx) * NT);
  cplx *J = (cplx *)malloc(sizeof(cplx) * (Q + 1));
  for (int i = 0; i < qr.n; i++) {
    cplx kr = qr.kr[i], kzt = kz_of(kt, kr), kzs = kz_of(ks, kr);
    cplx sig[2][2];
    orc_densities_c(&st, kr, l, lp, sig);
    double f = cabs(qr.w[i] * kr * cexp(I * kzt * zt + I * kzs * zs) * sig[a][b] / kzt);
    orc_bessel_J(Q, kr * rho, J);
    orc_legendre(p, kzt / kt, orc_branch_sqrt(kzt / kt), Pt);
    orc_legendre(p, kzs / ks, orc_branch_sqrt(kzs / ks), Ps);
    for (int n = 0; n <= p; n++)
      for (int m = -n; m <= n; m++)
        for (int n2 = 0; n2 <= p; n2++)
          for (int m2 = -n2; m2 <= n2; m2++) {
            int qq = abs(m2 - m);
            mass[(size_t)idx(n, m) * NC + idx(n2, m2)] += f * cabs(phat(Pt, n, m)) * cabs(phat(Ps, n2, m2)) * cabs(J[qq]);
          }
  }
  for (int i = 0; i < NC * NC; i++) out[i] = 4.0 * PI / kt * mass[i];
  free(mass);
  free(Pt);
  free(Ps);
  free(J);
  free_rule(&qr);
}

void orc_reaction_T(int L, const double *d, const double *k, int l, int a, int lp, int b, double dx, double dy,
                    double zt, double zs, int p, double qb, double *out) {
  stack_t st;
  make_stack(&st, L, d, k);
  int NC = (p + 1) * (p + 1);
  cplx *T = (cplx *)malloc(sizeof(cplx) * NC * NC);
  reaction_T(&st, l, a, lp, b, dx, dy, zt, zs, p, qb, T);
  for (int i = 0; i < NC * NC; i++) {
    out[2 * i] = creal(T[i]);
    out[2 * i + 1] = cimag(T[i]);
  }
  free(T);
}

/* Reaction kernel of one component in the polarisation frame (see above) at a
 * single pair; and the same with a constant density sigma = 1 (sigma_one != 0)
 * for the Sommerfeld-identity check. */
void orc_reaction_kernel(int L, const double *d, const double *k, int l, int a, int lp, int b, double rho,
                         double ht, double hs, double qb, double *out) {
  stack_t st;
  make_stack(&st, L, d, k);
  qrule_t qr = make_rule(qb, stack_kmax(&st), ht + hs, rho, 0);
  cplx s = 0, J[2];
  for (int i = 0; i < qr.n; i++) {
    cplx kr = qr.kr[i], kzt = kz_of(k[l], kr), kzs = kz_of(k[lp], kr);
    cplx sig[2][2];
    orc_densities_c(&st, kr, l, lp, sig);
    orc_bessel_J(0, kr * rho, J);
    s += qr.w[i] * kr * J[0] * cexp(I * kzt * ht + I * kzs * hs) * sig[a][b] / kzt;
  }
  s /= k[l];
  out[0] = creal(s);
  out[1] = cimag(s);
  free_rule(&qr);
}

/* Multipole expansion basis of a reaction component in the polarisation frame
 * (eq. (mebasis), alpha-integrated per Section 3.5): for a target at (rho, phi)
 * laterally from the source centre and height ht, centre depth hc,
 *   F_nm = (1/k_t) (-i)^n i^m e^{i m phi} int k_rho J_m(k_rho rho)
 *          e^{i kz_t ht + i kz_s hc} sigma/kz_t Phat_n^m(kz_s/k_s) dk_rho,
 * so that G(r, r_s) = sum_nm M_nm F_nm with M_nm = 4 pi j_n(k_s r') conj(Y_n^m(r'^))
 * and r' = image - centre (frame coordinates).  out: 2*NC doubles. */
void orc_reaction_me_basis(int L, const double *d, const double *k, int l, int a, int lp, int b, double dx,
                           double dy, double ht, double hc, int p, double qb, double *out) {
  stack_t st;
  make_stack(&st, L, d, k);
  int NC = (p + 1) * (p + 1), NT = (p + 1) * (p + 2) / 2;
  double rho = sqrt(dx * dx + dy * dy), phi = atan2(dy, dx);
  double kt = k[l], ks = k[lp];
  qrule_t qr = make_rule(qb, stack_kmax(&st), ht + hc, rho, p + 1);
  cplx *F = (cplx *)calloc(NC, sizeof(cplx));
  cplx *Ps = (cplx *)malloc(sizeof(cplx) * NT), *J = (cplx *)malloc(sizeof(cplx) * (p + 1));
  for (int i = 0; i < qr.n; i++) {
    cplx kr = qr.kr[i], kzt = kz_of(kt, kr), kzs = kz_of(ks, kr);
    cplx sig[2][2];
    orc_densities_c(&st, kr, l, lp, sig);
    cplx f = qr.w[i] * kr * cexp(I * kzt * ht + I * kzs * hc) * sig[a][b] / kzt;
    orc_bessel_J(p, kr * rho, J);
    orc_legendre(p, kzs / ks, orc_branch_sqrt(kzs / ks), Ps);
    for (int n = 0; n <= p; n++)
      for (int m = -n; m <= n; m++) {
        cplx Jm = m >= 0 ? J[m] : msign(m) * J[-m];
        F[idx(n, m)] += f * Jm * phat(Ps, n, m);
      }
  }
  for (int n = 0; n <= p; n++)
    for (int m = -n; m <= n; m++) {
      cplx v = F[idx(n, m)] / kt * ipow(-n) * ipow(m) * cexp(I * (double)m * phi);
      out[2 * idx(n, m)] = creal(v);
      out[2 * idx(n, m) + 1] = cimag(v);
    }
  free(F);
  free(Ps);
  free(J);
  free_rule(&qr);
}

/* ------------------------------------------------------------------------- */
/* Plain FMM (Section 3.4 Algorithm 1 for each reaction component; the classic */
/* FMM for each free-space component)                                         */
/* ------------------------------------------------------------------------- */
/* Tree rule (the paper builds its trees adaptively, by bisection; the library and
 * this oracle use uniform-depth octrees):
 *  - free tree of layer l: root = bounding cube of the layer's particles
 *    (centre = bounding-box midpoint, side S = largest extent, S = 1 if zero);
 *  - all reaction trees share one root: x,y as the bounding box of all particles,
 *    z in the polarisation frame [-S/2, S/2] split at the interface z = 0, with
 *    S = max(x extent, y extent, 2 * largest particle-to-interface distance);
 *  - cell of a coordinate v on an axis at depth D: floor(((v - lo)/S) * 2^D) clamped
 *    to [0, 2^D - 1]; in the reaction frame a target at height h > 0 gets
 *    z-cell 2^{D-1} + min(floor((h/S) 2^D), 2^{D-1}-1) and a polarisation source
 *    at depth h > 0 gets 2^{D-1} - 1 - min(floor((h/S) 2^D), 2^{D-1}-1);
 *  - depth: the smallest D (>= 0 for free trees, >= 1 for reaction sets) whose
 *    fullest cell holds <= leaf_max points, at most 8; all reaction trees use the
 *    largest depth over every target set (l,a) and polarisation-source set (lp,b);
 *  - lists: M2L from level 2 down between cells whose parents are adjacent and
 *    which are not adjacent themselves; direct interaction between adjacent leaves. */

typedef struct {
  int n;
  int *ix, *iy, *iz;      /* cells at depth DMAX */
  double *fx, *fy, *fz;   /* frame coordinates (reaction: +height / -depth) */
  cplx *q;                /* charges (sources) */
  int *id;                /* particle index */
} pset_t;

typedef struct {
  pset_t ps;
  int D, frame;
  double lo[3], S;
  int **cnt;              /* per level: points per cell */
  int *lstart, *lorder;   /* leaf level: start (nc+1) and point order */
} tree_t;

static size_t cell_lin(int ix, int iy, int iz, int l) {
  size_t s = (size_t)1 << l;
  return ((size_t)ix * s + (size_t)iy) * s + (size_t)iz;
}
static int axis_cell(double v, double lo, double S, int D) {
  double u = (v - lo) / S;
  double f = floor(u * (double)(1 << D));
  int m = (1 << D) - 1;
  if (f < 0.0) return 0;
  if (f > (double)m) return m;
  return (int)f;
}
static int half_cell(double h, double S, int D) {
  double u = h / S;
  double f = floor(u * (double)(1 << D));
  int m = (1 << (D - 1)) - 1;
  if (f < 0.0) return 0;
  if (f > (double)m) return m;
  return (int)f;
}

static void pset_alloc(pset_t *ps, int n) {
  ps->n = n;
  ps->ix = (int *)malloc(sizeof(int) * (n + 1));
  ps->iy = (int *)malloc(sizeof(int) * (n + 1));
  ps->iz = (int *)malloc(sizeof(int) * (n + 1));
  ps->fx = (double *)malloc(sizeof(double) * (n + 1));
  ps->fy = (double *)malloc(sizeof(double) * (n + 1));
  ps->fz = (double *)malloc(sizeof(double) * (n + 1));
  ps->q = (cplx *)malloc(sizeof(cplx) * (n + 1));
  ps->id = (int *)malloc(sizeof(int) * (n + 1));
}
static void pset_free(pset_t *ps) {
  free(ps->ix); free(ps->iy); free(ps->iz);
  free(ps->fx); free(ps->fy); free(ps->fz);
  free(ps->q); free(ps->id);
}

static int occupancy_depth(const pset_t *ps, int leaf_max, int Dmin, int Dlim) {
  for (int D = Dmin; D <= Dlim; D++) {
    size_t nc = (size_t)1 << (3 * D);
    int *cnt = (int *)calloc(nc, sizeof(int));
    int mx = 0, sh = DMAX - D;
    for (int i = 0; i < ps->n; i++) {
      size_t c = cell_lin(ps->ix[i] >> sh, ps->iy[i] >> sh, ps->iz[i] >> sh, D);
      if (++cnt[c] > mx) mx = cnt[c];
    }
    free(cnt);
    if (mx <= leaf_max) return D;
  }
  return Dlim;
}

static void tree_build(tree_t *t) {
  int D = t->D;
  t->cnt = (int **)malloc(sizeof(int *) * (D + 1));
  for (int l = 0; l <= D; l++) {
    size_t nc = (size_t)1 << (3 * l);
    t->cnt[l] = (int *)calloc(nc, sizeof(int));
    int sh = DMAX - l;
    for (int i = 0; i < t->ps.n; i++) t->cnt[l][cell_lin(t->ps.ix[i] >> sh, t->ps.iy[i] >> sh, t->ps.iz[i] >> sh, l)]++;
  }
  size_t nc = (size_t)1 << (3 * D);
  t->lstart = (int *)calloc(nc + 1, sizeof(int));
  for (size_t c = 0; c < nc; c++) t->lstart[c + 1] = t->lstart[c] + t->cnt[D][c];
  int *fill = (int *)calloc(nc, sizeof(int));
  t->lorder = (int *)malloc(sizeof(int) * (t->ps.n + 1));
  int sh = DMAX - D;
  for (int i = 0; i < t->ps.n; i++) {
    size_t c = cell_lin(t->ps.ix[i] >> sh, t->ps.iy[i] >> sh, t->ps.iz[i] >> sh, D);
    t->lorder[t->lstart[c] + fill[c]++] = i;
  }
  free(fill);
}
static void tree_free(tree_t *t) {
  for (int l = 0; l <= t->D; l++) free(t->cnt[l]);
  free(t->cnt);
  free(t->lstart);
  free(t->lorder);
}

static void cell_center(const tree_t *t, int l, int ix, int iy, int iz, double *c) {
  double h = t->S / (double)(1 << l);
  c[0] = t->lo[0] + (ix + 0.5) * h;
  c[1] = t->lo[1] + (iy + 0.5) * h;
  c[2] = t->frame ? (iz + 0.5) * h - 0.5 * t->S : t->lo[2] + (iz + 0.5) * h;
}

/* Gaunt table G(nu,mu; q, m-mu; n) for all (n,m), (nu,mu), q = 0..2p, built once per p. */
static double *gaunt_tab = NULL;
static int gaunt_p = -1;
static void gaunt_init(int p) {
  if (gaunt_p == p) return;
  free(gaunt_tab);
  int NC = (p + 1) * (p + 1), Q = 2 * p;
  gaunt_tab = (double *)calloc((size_t)NC * NC * (Q + 1), sizeof(double));
#pragma omp parallel for schedule(dynamic, 1)
  for (int a = 0; a < NC; a++) {
    int n = (int)floor(sqrt((double)a)), m = a - n * n - n;
    for (int nu = 0; nu <= p; nu++)
      for (int mu = -nu; mu <= nu; mu++)
        for (int qq = abs(n - nu); qq <= n + nu; qq++) {
          if (((n + nu + qq) & 1) || abs(m - mu) > qq) continue;
          gaunt_tab[((size_t)a * NC + idx(nu, mu)) * (Q + 1) + qq] = orc_gaunt(nu, mu, qq, m - mu, n);
        }
  }
  gaunt_p = p;
}

/* Same operator as orc_translation, using the cached Gaunt table. */
static void translation_op(int kind, double k, const double *bv, int p, cplx *Op) {
  int NC = (p + 1) * (p + 1), Q = 2 * p;
  double bb = sqrt(bv[0] * bv[0] + bv[1] * bv[1] + bv[2] * bv[2]);
  cplx zq[64];
  if (kind == 0) {
    double jj[64];
    orc_sph_j(Q, k * bb, jj);
    for (int qq = 0; qq <= Q; qq++) zq[qq] = jj[qq];
  } else {
    sph_h(Q, k * bb, zq);
  }
  cplx *Yq = (cplx *)malloc(sizeof(cplx) * (Q + 1) * (Q + 1));
  orc_sph_harm(Q, bv[0], bv[1], bv[2], Yq);
  for (int n = 0; n <= p; n++)
    for (int m = -n; m <= n; m++)
      for (int nu = 0; nu <= p; nu++)
        for (int mu = -nu; mu <= nu; mu++) {
          int s = m - mu;
          cplx acc = 0;
          const double *g = &gaunt_tab[((size_t)idx(n, m) * NC + idx(nu, mu)) * (Q + 1)];
          for (int qq = abs(n - nu); qq <= n + nu; qq++) {
            if (((n + nu + qq) & 1) || abs(s) > qq || g[qq] == 0.0) continue;
            acc += ipow(qq) * zq[qq] * conj(Yq[idx(qq, s)]) * g[qq];
          }
          Op[(size_t)idx(n, m) * NC + idx(nu, mu)] = 4.0 * PI * ipow(n - nu) * acc;
        }
  free(Yq);
}

static void matvec_acc(int NC, const cplx *A, const cplx *x, cplx *y) {
  for (int r = 0; r < NC; r++) {
    cplx s = 0;
    for (int c = 0; c < NC; c++) s += A[(size_t)r * NC + c] * x[c];
    y[r] += s;
  }
}

/* Upward pass: P2M at the leaves and M2M up to level 2, wavenumber k.
 * Returns M[l] (dense over cells) for l = 2..D, NULL for l < 2. */
static cplx **upward(const tree_t *t, double k, int p) {
  int D = t->D, NC = (p + 1) * (p + 1);
  cplx **M = (cplx **)calloc(D + 1, sizeof(cplx *));
  if (D < 2) return M;
  for (int l = 2; l <= D; l++) M[l] = (cplx *)calloc(((size_t)1 << (3 * l)) * NC, sizeof(cplx));
  size_t nc = (size_t)1 << (3 * D);
  int s = 1 << D;
#pragma omp parallel for schedule(dynamic, 16)
  for (size_t c = 0; c < nc; c++) {
    if (t->cnt[D][c] == 0) continue;
    int ix = (int)(c / ((size_t)s * s)), iy = (int)((c / s) % s), iz = (int)(c % s);
    double ctr[3];
    cell_center(t, D, ix, iy, iz, ctr);
    double *buf = (double *)malloc(sizeof(double) * 2 * NC);
    for (int ii = t->lstart[c]; ii < t->lstart[c + 1]; ii++) {
      int i = t->lorder[ii];
      double rv[3] = {t->ps.fx[i] - ctr[0], t->ps.fy[i] - ctr[1], t->ps.fz[i] - ctr[2]};
      orc_point_expansion(0, k, rv, p, buf);
      for (int a = 0; a < NC; a++) M[D][c * NC + a] += t->ps.q[i] * (buf[2 * a] + I * buf[2 * a + 1]);
    }
    free(buf);
  }
  for (int l = D; l >= 3; l--) {
    cplx *ops = (cplx *)malloc(sizeof(cplx) * 8 * NC * NC);
    for (int ch = 0; ch < 8; ch++) {
      /* child (parity ch) centre minus parent centre = (+-h/2 per axis), h = child size */
      double h = t->S / (double)(1 << l);
      double bv[3] = {-(((ch >> 2) & 1) - 0.5) * h, -(((ch >> 1) & 1) - 0.5) * h, -((ch & 1) - 0.5) * h};
      translation_op(0, k, bv, p, ops + (size_t)ch * NC * NC); /* b = P - c */
    }
    int sl = 1 << l;
    size_t ncl = (size_t)1 << (3 * l);
    cplx *Mp = M[l - 1];
#pragma omp parallel for schedule(dynamic, 16)
    for (size_t pc = 0; pc < ((size_t)1 << (3 * (l - 1))); pc++) {
      int sp = sl / 2;
      int px = (int)(pc / ((size_t)sp * sp)), py = (int)((pc / sp) % sp), pz = (int)(pc % sp);
      for (int ch = 0; ch < 8; ch++) {
        int cx = 2 * px + ((ch >> 2) & 1), cy = 2 * py + ((ch >> 1) & 1), cz = 2 * pz + (ch & 1);
        size_t c = cell_lin(cx, cy, cz, l);
        if (t->cnt[l][c] == 0) continue;
        matvec_acc(NC, ops + (size_t)ch * NC * NC, M[l] + c * NC, Mp + pc * NC);
      }
    }
    (void)ncl;
    free(ops);
  }
  return M;
}

/* Downward pass skeleton shared by free and reaction components.  m2l(ctx, l,
 * target cell, source cell, out Op) supplies the M2L operator. */
typedef void (*m2l_fn)(void *ctx, int l, const int *tc, const int *sc, cplx *Op);

static cplx **downward(const tree_t *tt, const tree_t *ts, cplx **M, double kt, int p, m2l_fn m2l, void *ctx) {
  int D = tt->D, NC = (p + 1) * (p + 1);
  cplx **Lc = (cplx **)calloc(D + 1, sizeof(cplx *));
  if (D < 2) return Lc;
  for (int l = 2; l <= D; l++) Lc[l] = (cplx *)calloc(((size_t)1 << (3 * l)) * NC, sizeof(cplx));
  for (int l = 2; l <= D; l++) {
    int sl = 1 << l;
    size_t ncl = (size_t)1 << (3 * l);
    cplx *l2l = NULL;
    if (l >= 3) {
      l2l = (cplx *)malloc(sizeof(cplx) * 8 * NC * NC);
      for (int ch = 0; ch < 8; ch++) {
        double h = tt->S / (double)(1 << l);
        double bv[3] = {(((ch >> 2) & 1) - 0.5) * h, (((ch >> 1) & 1) - 0.5) * h, ((ch & 1) - 0.5) * h};
        translation_op(0, kt, bv, p, l2l + (size_t)ch * NC * NC); /* b = c - P */
      }
    }
#pragma omp parallel for schedule(dynamic, 4)
    for (size_t c = 0; c < ncl; c++) {
      if (tt->cnt[l][c] == 0) continue;
      int tc[3] = {(int)(c / ((size_t)sl * sl)), (int)((c / sl) % sl), (int)(c % sl)};
      cplx *Lb = Lc[l] + c * NC;
      if (l >= 3) {
        int ch = ((tc[0] & 1) << 2) | ((tc[1] & 1) << 1) | (tc[2] & 1);
        size_t pc = cell_lin(tc[0] >> 1, tc[1] >> 1, tc[2] >> 1, l - 1);
        matvec_acc(NC, l2l + (size_t)ch * NC * NC, Lc[l - 1] + pc * NC, Lb);
      }
      cplx *Op = (cplx *)malloc(sizeof(cplx) * NC * NC);
      int px = tc[0] >> 1, py = tc[1] >> 1, pz = tc[2] >> 1, sp = sl / 2;
      for (int qx = px - 1; qx <= px + 1; qx++)
        for (int qy = py - 1; qy <= py + 1; qy++)
          for (int qz = pz - 1; qz <= pz + 1; qz++) {
            if (qx < 0 || qy < 0 || qz < 0 || qx >= sp || qy >= sp || qz >= sp) continue;
            for (int ch = 0; ch < 8; ch++) {
              int sc[3] = {2 * qx + ((ch >> 2) & 1), 2 * qy + ((ch >> 1) & 1), 2 * qz + (ch & 1)};
              if (abs(sc[0] - tc[0]) <= 1 && abs(sc[1] - tc[1]) <= 1 && abs(sc[2] - tc[2]) <= 1) continue;
              size_t s = cell_lin(sc[0], sc[1], sc[2], l);
              if (ts->cnt[l][s] == 0) continue;
              m2l(ctx, l, tc, sc, Op);
              matvec_acc(NC, Op, M[l] + s * NC, Lb);
            }
          }
      free(Op);
    }
    free(l2l);
  }
  return Lc;
}

/* L2P at every target: phi[id] += sum L_nm j_n(k r) Y_n^m. */
static void eval_local(const tree_t *tt, cplx **Lc, double kt, int p, cplx *phi) {
  int D = tt->D, NC = (p + 1) * (p + 1);
  if (D < 2) return;
  int sh = DMAX - D;
#pragma omp parallel for schedule(static)
  for (int i = 0; i < tt->ps.n; i++) {
    int ix = tt->ps.ix[i] >> sh, iy = tt->ps.iy[i] >> sh, iz = tt->ps.iz[i] >> sh;
    double ctr[3];
    cell_center(tt, D, ix, iy, iz, ctr);
    double rv[3] = {tt->ps.fx[i] - ctr[0], tt->ps.fy[i] - ctr[1], tt->ps.fz[i] - ctr[2]};
    double *co = (double *)malloc(sizeof(double) * 2 * NC);
    const cplx *L = Lc[D] + cell_lin(ix, iy, iz, D) * NC;
    for (int a = 0; a < NC; a++) {
      co[2 * a] = creal(L[a]);
      co[2 * a + 1] = cimag(L[a]);
    }
    double out[2];
    orc_eval_expansion(1, kt, co, rv, p, out);
    phi[tt->ps.id[i]] += out[0] + I * out[1];
    free(co);
  }
}

typedef struct {
  double k;
  int p;
  double S;
  cplx *cache;   /* 343 slots per level */
  char *have;
  int D;
} free_ctx_t;

static void free_m2l(void *vctx, int l, const int *tc, const int *sc, cplx *Op) {
  free_ctx_t *c = (free_ctx_t *)vctx;
  int NC = (c->p + 1) * (c->p + 1);
  int dx = tc[0] - sc[0], dy = tc[1] - sc[1], dz = tc[2] - sc[2];
  size_t slot = (size_t)(l * 343 + (dx + 3) * 49 + (dy + 3) * 7 + (dz + 3));
  memcpy(Op, c->cache + slot * NC * NC, sizeof(cplx) * NC * NC);
  (void)Op;
}

/* Free-space FMM of one layer (targets = sources = the layer's particles). */
static void fmm_free_layer(const stack_t *st, int l, int p, int leaf_max, int Dlim, int N, const double *x, const double *y,
                           const double *z, const int *lay, const double *q, cplx *phi, int *depth_out) {
  int n = 0;
  for (int i = 0; i < N; i++) n += (lay[i] == l);
  if (n == 0) {
    *depth_out = -1;
    return;
  }
  tree_t t;
  memset(&t, 0, sizeof(t));
  pset_alloc(&t.ps, n);
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  int c = 0;
  for (int i = 0; i < N; i++) {
    if (lay[i] != l) continue;
    t.ps.fx[c] = x[i];
    t.ps.fy[c] = y[i];
    t.ps.fz[c] = z[i];
    t.ps.q[c] = q[2 * i] + I * q[2 * i + 1];
    t.ps.id[c] = i;
    c++;
  }
  for (int i = 0; i < n; i++) {
    double v[3] = {t.ps.fx[i], t.ps.fy[i], t.ps.fz[i]};
    for (int a = 0; a < 3; a++) {
      if (v[a] < lo[a]) lo[a] = v[a];
      if (v[a] > hi[a]) hi[a] = v[a];
    }
  }
  double S = 0;
  for (int a = 0; a < 3; a++)
    if (hi[a] - lo[a] > S) S = hi[a] - lo[a];
  if (S == 0.0) S = 1.0;
  for (int a = 0; a < 3; a++) t.lo[a] = 0.5 * (lo[a] + hi[a]) - 0.5 * S;
  t.S = S;
  t.frame = 0;
  for (int i = 0; i < n; i++) {
    t.ps.ix[i] = axis_cell(t.ps.fx[i], t.lo[0], S, DMAX);
    t.ps.iy[i] = axis_cell(t.ps.fy[i], t.lo[1], S, DMAX);
    t.ps.iz[i] = axis_cell(t.ps.fz[i], t.lo[2], S, DMAX);
  }
  t.D = occupancy_depth(&t.ps, leaf_max, 0, Dlim);
  *depth_out = t.D;
  tree_build(&t);
  double k = st->k[l];
  int NC = (p + 1) * (p + 1), D = t.D;
  cplx **M = upward(&t, k, p);
  if (D >= 2) {
    free_ctx_t ctx;
    ctx.k = k;
    ctx.p = p;
    ctx.S = S;
    ctx.D = D;
    ctx.cache = (cplx *)malloc(sizeof(cplx) * (size_t)(D + 1) * 343 * NC * NC);
    for (int lv = 2; lv <= D; lv++) {
      double h = S / (double)(1 << lv);
#pragma omp parallel for schedule(dynamic, 1)
      for (int o = 0; o < 343; o++) {
        int dx = o / 49 - 3, dy = (o / 7) % 7 - 3, dz = o % 7 - 3;
        if (abs(dx) <= 1 && abs(dy) <= 1 && abs(dz) <= 1) continue;
        double bv[3] = {dx * h, dy * h, dz * h};
        translation_op(1, k, bv, p, ctx.cache + ((size_t)lv * 343 + o) * NC * NC);
      }
    }
    cplx **Lc = downward(&t, &t, M, k, p, free_m2l, &ctx);
    eval_local(&t, Lc, k, p, phi);
    for (int lv = 0; lv <= D; lv++) free(Lc[lv]);
    free(Lc);
    free(ctx.cache);
  }
  /* near field: adjacent leaves, j != i */
  int s = 1 << D, sh = DMAX - D;
#pragma omp parallel for schedule(dynamic, 32)
  for (int i = 0; i < n; i++) {
    int ix = t.ps.ix[i] >> sh, iy = t.ps.iy[i] >> sh, iz = t.ps.iz[i] >> sh;
    cplx acc = 0;
    for (int ax = ix - 1; ax <= ix + 1; ax++)
      for (int ay = iy - 1; ay <= iy + 1; ay++)
        for (int az = iz - 1; az <= iz + 1; az++) {
          if (ax < 0 || ay < 0 || az < 0 || ax >= s || ay >= s || az >= s) continue;
          size_t cc = cell_lin(ax, ay, az, D);
          for (int jj = t.lstart[cc]; jj < t.lstart[cc + 1]; jj++) {
            int j = t.lorder[jj];
            if (j == i) continue;
            double dx = t.ps.fx[i] - t.ps.fx[j], dy = t.ps.fy[i] - t.ps.fy[j], dz = t.ps.fz[i] - t.ps.fz[j];
            double r = sqrt(dx * dx + dy * dy + dz * dz);
            if (r > 0.0) acc += t.ps.q[j] * h0(k * r);
          }
        }
    phi[t.ps.id[i]] += acc;
  }
  for (int lv = 0; lv <= D; lv++) free(M[lv]);
  free(M);
  tree_free(&t);
  pset_free(&t.ps);
}

/* ---- reaction components ---- */
typedef struct {
  const stack_t *st;
  int l, a, lp, b, p;
  double S, qb;
  cplx **icache;   /* per level: [j][i][r2] integral matrices (NULL until computed) */
  int D;
} react_ctx_t;

/* T operator from the per-geometry integral, eq. (me2lesimplified) in the
 * polarisation frame; see reaction_T. */
static void react_m2l(void *vctx, int l, const int *tc, const int *sc, cplx *Op) {
  react_ctx_t *c = (react_ctx_t *)vctx;
  int p = c->p, NC = (p + 1) * (p + 1);
  int dx = tc[0] - sc[0], dy = tc[1] - sc[1];
  int j = tc[2] - (1 << (l - 1)), i = (1 << (l - 1)) - 1 - sc[2];
  int r2 = dx * dx + dy * dy;
  const cplx *Im = c->icache[l] + ((size_t)((j * 2 + i) * 19 + r2)) * NC * NC;
  double phi = atan2((double)dy, (double)dx);
  double kt = c->st->k[c->l];
  for (int n = 0; n <= p; n++)
    for (int m = -n; m <= n; m++)
      for (int n2 = 0; n2 <= p; n2++)
        for (int m2 = -n2; m2 <= n2; m2++) {
          int qq = m2 - m;
          cplx cf = (4.0 * PI / kt) * ipow(n) * ipow(-n2) * ipow(qq) * cexp(I * (double)qq * phi);
          Op[(size_t)idx(n, m) * NC + idx(n2, m2)] = cf * Im[(size_t)idx(n, m) * NC + idx(n2, m2)];
        }
}

/* The integral part of the reaction M2L operator (no prefactor):
 * I_{nm,n'm'} = int k_rho J_q(k_rho rho) e^{i kz_t zt + i kz_s zs} sigma/kz_t Phat_n^m Phat_{n'}^{m'} dk_rho */
static void reaction_I(const stack_t *st, int l, int a, int lp, int b, double rho, double zt, double zs, int p,
                       double qb, cplx *I_) {
  int NC = (p + 1) * (p + 1), NT = (p + 1) * (p + 2) / 2, Q = 2 * p;
  double kt = st->k[l], ks = st->k[lp];
  qrule_t qr = make_rule(qb, stack_kmax(st), zt + zs, rho, 2 * p + 1);
  memset(I_, 0, sizeof(cplx) * NC * NC);
  cplx *Pt = (cplx *)malloc(sizeof(cplx) * NT), *Ps = (cplx *)malloc(sizeof(cplx) * NT);
  cplx *J = (cplx *)malloc(sizeof(cplx) * (Q + 1));
  for (int i = 0; i < qr.n; i++) {
    cplx kr = qr.kr[i], kzt = kz_of(kt, kr), kzs = kz_of(ks, kr);
    cplx sig[2][2];
    orc_densities_c(st, kr, l, lp, sig);
    cplx f = qr.w[i] * kr * cexp(I * kzt * zt + I * kzs * zs) * sig[a][b] / kzt;
    orc_bessel_J(Q, kr * rho, J);
    orc_legendre(p, kzt / kt, orc_branch_sqrt(kzt / kt), Pt);
    orc_legendre(p, kzs / ks, orc_branch_sqrt(kzs / ks), Ps);
    for (int n = 0; n <= p; n++)
      for (int m = -n; m <= n; m++) {
        cplx pt = phat(Pt, n, m) * f;
        for (int n2 = 0; n2 <= p; n2++)
          for (int m2 = -n2; m2 <= n2; m2++) {
            int qq = m2 - m;
            cplx Jq = qq >= 0 ? J[qq] : msign(qq) * J[-qq];
            I_[(size_t)idx(n, m) * NC + idx(n2, m2)] += pt * phat(Ps, n2, m2) * Jq;
          }
      }
  }
  free(Pt);
  free(Ps);
  free(J);
  free_rule(&qr);
}

static void fill_react_cache(react_ctx_t *c, const tree_t *tt, const tree_t *ts) {
  int p = c->p, NC = (p + 1) * (p + 1), D = tt->D;
  c->icache = (cplx **)calloc(D + 1, sizeof(cplx *));
  for (int l = 2; l <= D; l++) {
    /* which (j, i, r2) classes are used at this level */
    char need[2][2][19];
    memset(need, 0, sizeof(need));
    int sl = 1 << l, hf = 1 << (l - 1);
    for (int tz = hf; tz <= hf + 1 && tz < sl; tz++)
      for (int tx = 0; tx < sl; tx++)
        for (int ty = 0; ty < sl; ty++) {
          if (tt->cnt[l][cell_lin(tx, ty, tz, l)] == 0) continue;
          for (int sz = hf - 2; sz <= hf - 1; sz++) {
            if (sz < 0) continue;
            if (((tz >> 1) - (sz >> 1)) > 1) continue;
            for (int sx = 0; sx < sl; sx++)
              for (int sy = 0; sy < sl; sy++) {
                if (abs((sx >> 1) - (tx >> 1)) > 1 || abs((sy >> 1) - (ty >> 1)) > 1) continue;
                if (abs(sx - tx) <= 1 && abs(sy - ty) <= 1 && abs(sz - tz) <= 1) continue;
                if (ts->cnt[l][cell_lin(sx, sy, sz, l)] == 0) continue;
                int dx = tx - sx, dy = ty - sy;
                need[tz - hf][hf - 1 - sz][dx * dx + dy * dy] = 1;
              }
          }
        }
    c->icache[l] = (cplx *)calloc((size_t)4 * 19 * NC * NC, sizeof(cplx));
    int list[76], nl = 0;
    for (int j = 0; j < 2; j++)
      for (int i = 0; i < 2; i++)
        for (int r2 = 0; r2 < 19; r2++)
          if (need[j][i][r2]) list[nl++] = (j * 2 + i) * 19 + r2;
    double h = c->S / (double)(1 << l);
#pragma omp parallel for schedule(dynamic, 1)
    for (int e = 0; e < nl; e++) {
      int key = list[e], r2 = key % 19, ji = key / 19, j = ji / 2, i = ji % 2;
      reaction_I(c->st, c->l, c->a, c->lp, c->b, h * sqrt((double)r2), (j + 0.5) * h, (i + 0.5) * h, p, c->qb,
                 c->icache[l] + (size_t)key * NC * NC);
    }
  }
}

/* Reaction FMM for all components; common root and depth for every reaction tree. */
static void fmm_reaction(const stack_t *st, int p, int leaf_max, int Dlim, double qb, int N, const double *x, const double *y,
                         const double *z, const int *lay, const double *q, cplx *phi, int *depth_out) {
  int L = st->L;
  if (L < 1) {
    *depth_out = -1;
    return;
  }
  double xlo = INFINITY, xhi = -INFINITY, ylo = INFINITY, yhi = -INFINITY, H = 0;
  for (int i = 0; i < N; i++) {
    if (x[i] < xlo) xlo = x[i];
    if (x[i] > xhi) xhi = x[i];
    if (y[i] < ylo) ylo = y[i];
    if (y[i] > yhi) yhi = y[i];
    for (int a = 0; a < 2; a++)
      if (has_dir(st, lay[i], a)) {
        double hh = hdist(st, lay[i], a, z[i]);
        if (hh > H) H = hh;
      }
  }
  double S = xhi - xlo;
  if (yhi - ylo > S) S = yhi - ylo;
  if (2.0 * H > S) S = 2.0 * H;
  double lox = 0.5 * (xlo + xhi) - 0.5 * S, loy = 0.5 * (ylo + yhi) - 0.5 * S;
  /* point sets per (layer, direction): targets (+h) and sources (-h) */
  pset_t tset[LMAXL + 1][2], sset[LMAXL + 1][2];
  int Dr = 1;
  for (int l = 0; l <= L; l++)
    for (int a = 0; a < 2; a++) {
      int n = 0;
      for (int i = 0; i < N; i++) n += (lay[i] == l);
      pset_alloc(&tset[l][a], has_dir(st, l, a) ? n : 0);
      pset_alloc(&sset[l][a], has_dir(st, l, a) ? n : 0);
      if (!has_dir(st, l, a)) continue;
      int c = 0;
      for (int i = 0; i < N; i++) {
        if (lay[i] != l) continue;
        double hh = hdist(st, l, a, z[i]);
        pset_t *T = &tset[l][a], *Sx = &sset[l][a];
        T->fx[c] = Sx->fx[c] = x[i];
        T->fy[c] = Sx->fy[c] = y[i];
        T->fz[c] = hh;
        Sx->fz[c] = -hh;
        T->q[c] = Sx->q[c] = q[2 * i] + I * q[2 * i + 1];
        T->id[c] = Sx->id[c] = i;
        T->ix[c] = Sx->ix[c] = axis_cell(x[i], lox, S, DMAX);
        T->iy[c] = Sx->iy[c] = axis_cell(y[i], loy, S, DMAX);
        T->iz[c] = (1 << (DMAX - 1)) + half_cell(hh, S, DMAX);
        Sx->iz[c] = (1 << (DMAX - 1)) - 1 - half_cell(hh, S, DMAX);
        c++;
      }
      int d1 = occupancy_depth(&tset[l][a], leaf_max, 1, Dlim), d2 = occupancy_depth(&sset[l][a], leaf_max, 1, Dlim);
      if (d1 > Dr) Dr = d1;
      if (d2 > Dr) Dr = d2;
    }
  /* and deep enough that the finest boxes are no thicker than the smallest
   * particle-to-interface distance: then no target and no polarisation image
   * share the two boxes next to the interface, and the near field of the
   * reaction components is empty (within the depth limit) */
  double gmin = INFINITY;
  for (int i = 0; i < N; i++)
    for (int a = 0; a < 2; a++)
      if (has_dir(st, lay[i], a)) {
        double hh = hdist(st, lay[i], a, z[i]);
        if (hh < gmin) gmin = hh;
      }
  int Dg = 1;
  while (Dg < Dlim && S / (double)(1 << Dg) > gmin) Dg++;
  if (Dg > Dr) Dr = Dg;
  *depth_out = Dr;
  for (int l = 0; l <= L; l++)
    for (int a = 0; a < 2; a++) {
      if (!has_dir(st, l, a) || tset[l][a].n == 0) continue;
      tree_t tt;
      memset(&tt, 0, sizeof(tt));
      tt.ps = tset[l][a];
      tt.D = Dr;
      tt.frame = 1;
      tt.lo[0] = lox;
      tt.lo[1] = loy;
      tt.lo[2] = -0.5 * S;
      tt.S = S;
      tree_build(&tt);
      for (int lp = 0; lp <= L; lp++)
        for (int b = 0; b < 2; b++) {
          if (!has_dir(st, lp, b) || sset[lp][b].n == 0) continue;
          tree_t ts;
          memset(&ts, 0, sizeof(ts));
          ts.ps = sset[lp][b];
          ts.D = Dr;
          ts.frame = 1;
          ts.lo[0] = lox;
          ts.lo[1] = loy;
          ts.lo[2] = -0.5 * S;
          ts.S = S;
          tree_build(&ts);
          double kt = st->k[l], ks = st->k[lp];
          cplx **M = upward(&ts, ks, p);
          react_ctx_t ctx;
          ctx.st = st;
          ctx.l = l;
          ctx.a = a;
          ctx.lp = lp;
          ctx.b = b;
          ctx.p = p;
          ctx.S = S;
          ctx.qb = qb;
          ctx.D = Dr;
          fill_react_cache(&ctx, &tt, &ts);
          cplx **Lc = downward(&tt, &ts, M, kt, p, react_m2l, &ctx);
          eval_local(&tt, Lc, kt, p, phi);
          /* near field between adjacent leaves across the interface */
          {
            int D = Dr, s = 1 << D, sh = DMAX - D;
            double hmin_t = INFINITY, hmin_s = INFINITY;
            for (int i = 0; i < tt.ps.n; i++)
              if (tt.ps.fz[i] < hmin_t) hmin_t = tt.ps.fz[i];
            for (int i = 0; i < ts.ps.n; i++)
              if (-ts.ps.fz[i] < hmin_s) hmin_s = -ts.ps.fz[i];
            double hD = S / (double)(1 << D);
            qrule_t qr = make_rule(qb, stack_kmax(st), hmin_t + hmin_s, 2.0 * sqrt(2.0) * hD, 0);
            cplx *fac = (cplx *)malloc(sizeof(cplx) * qr.n);
            cplx *kzt = (cplx *)malloc(sizeof(cplx) * qr.n), *kzs = (cplx *)malloc(sizeof(cplx) * qr.n);
            for (int nd = 0; nd < qr.n; nd++) {
              cplx sig[2][2];
              orc_densities_c(st, qr.kr[nd], l, lp, sig);
              kzt[nd] = kz_of(kt, qr.kr[nd]);
              kzs[nd] = kz_of(ks, qr.kr[nd]);
              fac[nd] = qr.w[nd] * qr.kr[nd] * sig[a][b] / kzt[nd] / kt;
            }
#pragma omp parallel for schedule(dynamic, 8)
            for (int i = 0; i < tt.ps.n; i++) {
              int ix = tt.ps.ix[i] >> sh, iy = tt.ps.iy[i] >> sh, iz = tt.ps.iz[i] >> sh;
              cplx acc = 0, J[2];
              for (int ax = ix - 1; ax <= ix + 1; ax++)
                for (int ay = iy - 1; ay <= iy + 1; ay++)
                  for (int az = iz - 1; az <= iz + 1; az++) {
                    if (ax < 0 || ay < 0 || az < 0 || ax >= s || ay >= s || az >= s) continue;
                    size_t cc = cell_lin(ax, ay, az, D);
                    for (int jj = ts.lstart[cc]; jj < ts.lstart[cc + 1]; jj++) {
                      int j = ts.lorder[jj];
                      double dx = tt.ps.fx[i] - ts.ps.fx[j], dy = tt.ps.fy[i] - ts.ps.fy[j];
                      double rho = sqrt(dx * dx + dy * dy), ht = tt.ps.fz[i], hs = -ts.ps.fz[j];
                      cplx g = 0;
                      for (int nd = 0; nd < qr.n; nd++) {
                        orc_bessel_J(0, qr.kr[nd] * rho, J);
                        g += fac[nd] * J[0] * cexp(I * kzt[nd] * ht + I * kzs[nd] * hs);
                      }
                      acc += ts.ps.q[j] * g;
                    }
                  }
              phi[tt.ps.id[i]] += acc;
            }
            free(fac);
            free(kzt);
            free(kzs);
            free_rule(&qr);
          }
          for (int lv = 0; lv <= Dr; lv++) {
            free(M[lv]);
            free(Lc[lv]);
            if (ctx.icache) free(ctx.icache[lv]);
          }
          free(M);
          free(Lc);
          free(ctx.icache);
          tree_free(&ts);
        }
      tree_free(&tt);
    }
  for (int l = 0; l <= L; l++)
    for (int a = 0; a < 2; a++) {
      pset_free(&tset[l][a]);
      pset_free(&sset[l][a]);
    }
}

/* Plain FMM potentials Phi_l(r_i) for every particle (targets = sources).
 * what: 1 free part, 2 reaction part, 3 both.  info_out[0..L] = free-tree depths
 * (-1 for an empty layer), info_out[L+1] = depth of the reaction trees.
 *
 * Tree rule (the paper leaves tree construction to its FMM package): every tree is
 * a uniform octree.  A layer's free-space tree has the bounding cube of the
 * layer's particles as root and the smallest depth at which no cell holds more
 * than leaf_max particles.  The reaction trees share one root of side
 * max(x extent, y extent, 2 H) (H the largest particle-to-interface distance),
 * split at the interface into the target half and the polarisation-image half;
 * they all get the largest depth (>= 1) that any of them needs by the occupancy
 * rule, and at least the smallest depth at which the finest boxes are no thicker
 * than the smallest particle-to-interface distance.  Depths are capped at
 * max_depth (1..8). */
void orc_fmm(int L, const double *d, const double *k, int p, int leaf_max, int max_depth, double qb, int N,
             const double *x, const double *y, const double *z, const int *lay, const double *q, int what,
             double *phi_out, int *info_out) {
  const int Dlim = (max_depth >= 1 && max_depth <= DMAX) ? max_depth : DMAX;
  stack_t st;
  make_stack(&st, L, d, k);
  gl_init();
  gaunt_init(p);
  cplx *phi = (cplx *)calloc(N, sizeof(cplx));
  for (int l = 0; l <= L; l++) {
    info_out[l] = -1;
    if (what & 1) fmm_free_layer(&st, l, p, leaf_max, Dlim, N, x, y, z, lay, q, phi, &info_out[l]);
  }
  info_out[L + 1] = -1;
  if (what & 2) fmm_reaction(&st, p, leaf_max, Dlim, qb, N, x, y, z, lay, q, phi, &info_out[L + 1]);
  for (int i = 0; i < N; i++) {
    phi_out[2 * i] = creal(phi[i]);
    phi_out[2 * i + 1] = cimag(phi[i]);
  }
  free(phi);
}

/* Translation operator through the cached Gaunt table (for tests of the cache). */
void orc_translation_cached(int kind, double k, const double *bv, int p, double *op_out) {
  gaunt_init(p);
  int NC = (p + 1) * (p + 1);
  cplx *Op = (cplx *)malloc(sizeof(cplx) * NC * NC);
  translation_op(kind, k, bv, p, Op);
  for (int i = 0; i < NC * NC; i++) {
    op_out[2 * i] = creal(Op[i]);
    op_out[2 * i + 1] = cimag(Op[i]);
  }
  free(Op);
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
