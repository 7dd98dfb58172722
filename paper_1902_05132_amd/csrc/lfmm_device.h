// Device-side mathematics of the layered-media Helmholtz FMM (gfx950, FP64).
//
// Conventions (paper Section 2.1): Y_n^m = Phat_n^m(cos t) e^{i m phi} with Phat
// free of the Condon-Shortley phase and Phat_n^{-m} = (-1)^m Phat_n^m; coefficient
// index idx(n,m) = n*n + n + m; triangular Legendre index tix(n,m) = n(n+1)/2 + m.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#define LFMM_PI 3.14159265358979323846
#define LFMM_DMAX 8
#define LFMM_PMAX 10  // largest expansion order a plan accepts
#define LFMM_MAXL 16

struct cd {
  double x, y;
};

__host__ __device__ __forceinline__ cd mk(double a, double b) { cd r; r.x = a; r.y = b; return r; }
__host__ __device__ __forceinline__ cd operator+(cd a, cd b) { return mk(a.x + b.x, a.y + b.y); }
__host__ __device__ __forceinline__ cd operator-(cd a, cd b) { return mk(a.x - b.x, a.y - b.y); }
__host__ __device__ __forceinline__ cd operator-(cd a) { return mk(-a.x, -a.y); }
__host__ __device__ __forceinline__ cd operator*(cd a, cd b) { return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__host__ __device__ __forceinline__ cd operator*(double s, cd a) { return mk(s * a.x, s * a.y); }
__host__ __device__ __forceinline__ cd operator*(cd a, double s) { return mk(s * a.x, s * a.y); }
__host__ __device__ __forceinline__ cd cconj(cd a) { return mk(a.x, -a.y); }
__host__ __device__ __forceinline__ double cabs2(cd a) { return a.x * a.x + a.y * a.y; }
__host__ __device__ __forceinline__ double cmod(cd a) { return hypot(a.x, a.y); }
__host__ __device__ __forceinline__ cd operator/(cd a, cd b) {
  // scaled division (Smith's method)
  if (fabs(b.x) >= fabs(b.y)) {
    double r = b.y / b.x, den = b.x + b.y * r;
    return mk((a.x + a.y * r) / den, (a.y - a.x * r) / den);
  } else {
    double r = b.x / b.y, den = b.x * r + b.y;
    return mk((a.x * r + a.y) / den, (a.y * r - a.x) / den);
  }
}
__host__ __device__ __forceinline__ cd operator/(cd a, double s) { return mk(a.x / s, a.y / s); }
__host__ __device__ __forceinline__ cd cmul_i(cd a) { return mk(-a.y, a.x); }  // i*a
__host__ __device__ __forceinline__ cd cexpd(cd a) {
  double e = exp(a.x), s, c;
  sincos(a.y, &s, &c);
  return mk(e * c, e * s);
}
// principal square root (branch cut on the negative real axis)
__host__ __device__ __forceinline__ cd csqrtd(cd z) {
  double r = hypot(z.x, z.y);
  if (r == 0.0) return mk(0.0, 0.0);
  if (z.x >= 0.0) {
    double t = sqrt(0.5 * (r + z.x));
    return mk(t, z.y / (2.0 * t));
  } else {
    double t = sqrt(0.5 * (r - z.x));
    return mk(fabs(z.y) / (2.0 * t), copysign(t, z.y));
  }
}
// i^n for integer n
__host__ __device__ __forceinline__ cd ipow(int n) {
  int r = n & 3;
  return r == 0 ? mk(1, 0) : r == 1 ? mk(0, 1) : r == 2 ? mk(-1, 0) : mk(0, -1);
}
__host__ __device__ __forceinline__ int cidx(int n, int m) { return n * n + n + m; }
__host__ __device__ __forceinline__ int tix(int n, int m) { return n * (n + 1) / 2 + m; }

// ---------------------------------------------------------------------------
// Spherical Bessel functions of real argument.
// j_n(x), n = 0..p: power series for x < 1, otherwise Miller's backward
// recurrence normalised to sin(x)/x or the closed form of j_1.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double sph_j_series(int n, double x) {
  // j_n(x) = x^n/(2n+1)!! sum_k (-x^2/2)^k / (k! (2n+3)(2n+5)...(2n+2k+1))
  double xn = 1.0, dfac = 1.0;
  for (int i = 1; i <= n; i++) {
    xn *= x;
    dfac *= (2.0 * i + 1.0);
  }
  double x2 = 0.5 * x * x, term = 1.0, s = 1.0;
  for (int k = 1; k < 30; k++) {
    term *= -x2 / (k * (2.0 * n + 2.0 * k + 1.0));
    s += term;
    if (fabs(term) < 1e-17 * fabs(s)) break;
  }
  return xn / dfac * s;
}
__device__ __forceinline__ void dev_sph_j(int p, double x, double* j) {
  if (x < 1e-3) {  // two terms of the series per order are exact to rounding
    double xn = 1.0, dfac = 1.0, x2 = 0.5 * x * x;
    for (int n = 0; n <= p; n++) {
      if (n > 0) {
        xn *= x;
        dfac *= (2.0 * n + 1.0);
      }
      j[n] = xn / dfac * (1.0 - x2 / (2.0 * n + 3.0) + x2 * x2 / (2.0 * (2.0 * n + 3.0) * (2.0 * n + 5.0)));
    }
    return;
  }
  if (x < 1.0) {  // series for the two highest orders, then the stable downward recurrence
    double jp = sph_j_series(p + 1, x), jc = sph_j_series(p, x);
    j[p] = jc;
    for (int n = p; n >= 1; n--) {
      double jm = (2.0 * n + 1.0) / x * jc - jp;
      jp = jc;
      jc = jm;
      j[n - 1] = jc;
    }
    return;
  }
  int N = p + 24 + (int)x;
  double fp1 = 0.0, f = 1e-200;
  for (int n = N; n >= 1; n--) {
    double fm = (2.0 * n + 1.0) / x * f - fp1;
    fp1 = f;
    f = fm;  // f_{n-1}
    if (n - 1 <= p) j[n - 1] = f;
    if (fabs(f) > 1e200) {
      f *= 1e-200;
      fp1 *= 1e-200;
      for (int m = n - 1; m <= p; m++) j[m] *= 1e-200;
    }
  }
  // f = f_0, fp1 = f_1 (consistently scaled with j[])
  double s, c;
  sincos(x, &s, &c);
  double j0 = s / x, j1 = s / (x * x) - c / x;
  double sc = (fabs(j0) >= fabs(j1)) ? j0 / f : j1 / fp1;
  for (int n = 0; n <= p; n++) j[n] *= sc;
}

// Same as dev_sph_j with a compile-time order so that j[] stays in registers.
template <int P>
__device__ __forceinline__ void dev_sph_j_t(double x, double (&j)[P + 1]) {
  if (x < 1e-3) {
    double xn = 1.0, dfac = 1.0, x2 = 0.5 * x * x;
#pragma unroll
    for (int n = 0; n <= P; n++) {
      if (n > 0) {
        xn *= x;
        dfac *= (2.0 * n + 1.0);
      }
      j[n] = xn / dfac * (1.0 - x2 / (2.0 * n + 3.0) + x2 * x2 / (2.0 * (2.0 * n + 3.0) * (2.0 * n + 5.0)));
    }
    return;
  }
  double fp1, f;
  if (x < 1.0) {
    fp1 = sph_j_series(P + 1, x);
    f = sph_j_series(P, x);
    j[P] = f;
#pragma unroll
    for (int n = P; n >= 1; n--) {
      double fm = (2.0 * n + 1.0) / x * f - fp1;
      fp1 = f;
      f = fm;
      j[n - 1] = f;
    }
    return;
  }
  // one reciprocal for the whole recurrence: the backward recurrence is stable, so the
  // extra rounding of (2n+1) * (1/x) against (2n+1) / x stays at the last digit
  const double ix = 1.0 / x;
  int N = P + 24 + (int)x;
  fp1 = 0.0;
  f = 1e-200;
  for (int n = N; n >= P + 2; n--) {  // f_{n-1} from f_n, f_{n+1}; nothing stored yet
    double fm = (2.0 * n + 1.0) * ix * f - fp1;
    fp1 = f;
    f = fm;
    if (fabs(f) > 1e200) {
      f *= 1e-200;
      fp1 *= 1e-200;
    }
  }
  // f = f_{P+1}, fp1 = f_{P+2}
#pragma unroll
  for (int n = P + 1; n >= 1; n--) {
    double fm = (2.0 * n + 1.0) * ix * f - fp1;
    fp1 = f;
    f = fm;
    j[n - 1] = f;
  }
  double s, c;
  sincos(x, &s, &c);
  double j0 = s * ix, j1 = (s * ix - c) * ix;
  double sc = (fabs(j0) >= fabs(j1)) ? j0 / j[0] : j1 / j[1];
#pragma unroll
  for (int n = 0; n <= P; n++) j[n] *= sc;
}

// h_n^{(1)}(x) = j_n + i y_n, n = 0..p, x > 0 (y_n by upward recurrence)
__device__ __forceinline__ void dev_sph_h(int p, double x, cd* h) {
  double jj[48];
  dev_sph_j(p, x, jj);
  double s, c;
  sincos(x, &s, &c);
  double y0 = -c / x, y1 = -c / (x * x) - s / x;
  h[0] = mk(jj[0], y0);
  if (p >= 1) h[1] = mk(jj[1], y1);
  for (int n = 1; n < p; n++) {
    double y2 = (2.0 * n + 1.0) / x * y1 - y0;
    y0 = y1;
    y1 = y2;
    h[n + 1] = mk(jj[n + 1], y1);
  }
}

// Hankel's asymptotic expansions of J_0 and J_1 (|z| >= 25, |arg z| < pi/2):
// J_nu ~ sqrt(2/(pi z)) (P cos w - Q sin w), w = z - nu pi/2 - pi/4.
__device__ __forceinline__ void dev_hankel_J01(cd z, cd* J0, cd* J1) {
  cd iz = mk(1, 0) / z;
  cd P0 = mk(1, 0), Q0 = mk(0, 0), P1 = mk(1, 0), Q1 = mk(0, 0), t0 = mk(1, 0), t1 = mk(1, 0);
  for (int k = 1; k < 40; k++) {
    double o = (2.0 * k - 1.0) * (2.0 * k - 1.0);
    t0 = t0 * ((0.0 - o) / (8.0 * k)) * iz;
    t1 = t1 * ((4.0 - o) / (8.0 * k)) * iz;
    double sg = (k & 1) ? ((((k - 1) >> 1) & 1) ? -1.0 : 1.0) : (((k >> 1) & 1) ? -1.0 : 1.0);
    if (k & 1) {
      Q0 = Q0 + sg * t0;
      Q1 = Q1 + sg * t1;
    } else {
      P0 = P0 + sg * t0;
      P1 = P1 + sg * t1;
    }
    if (cabs2(t0) < 1e-36 && cabs2(t1) < 1e-36) break;
  }
  cd pre = csqrtd(mk(2.0 / LFMM_PI, 0) / z);
  for (int nu = 0; nu < 2; nu++) {
    cd w = mk(z.x - (0.25 + 0.5 * nu) * LFMM_PI, z.y);
    double sx, cx;
    sincos(w.x, &sx, &cx);
    double ch = cosh(w.y), sh = sinh(w.y);
    cd cw = mk(cx * ch, -sx * sh), sw = mk(sx * ch, cx * sh);
    if (nu == 0) *J0 = pre * (P0 * cw - Q0 * sw);
    else *J1 = pre * (P1 * cw - Q1 * sw);
  }
}

// ---------------------------------------------------------------------------
// Cylindrical Bessel J_q(z), q = 0..qmax, complex z.
// |z| < 2: power series; otherwise Miller's backward recurrence started well
// above max(qmax, |z|) and normalised with the generating-function identity
// e^{+-iz} = J_0 + 2 sum_{n>=1} (+-i)^n J_n (the sign giving the larger modulus).
// Writes to out[q * stride].
// ---------------------------------------------------------------------------
__device__ __forceinline__ void dev_besselJ(int qmax, cd z, cd* out, int stride) {
  double az = cmod(z);
  if (az == 0.0) {
    out[0] = mk(1, 0);
    for (int q = 1; q <= qmax; q++) out[q * stride] = mk(0, 0);
    return;
  }
  if (az < 2.0) {
    cd h = 0.5 * z, h2 = h * h, hq = mk(1, 0);
    double fq = 1.0;
    for (int q = 0; q <= qmax; q++) {
      if (q > 0) { hq = hq * h; fq *= q; }
      cd term = hq / fq, s = term;
      for (int k = 1; k < 30; k++) {
        term = term * (-1.0 / (k * (double)(q + k))) * h2;
        s = s + term;
        if (cabs2(term) < 1e-36 * cabs2(s)) break;
      }
      out[q * stride] = s;
    }
    return;
  }
  if (az > 25.0 && az > 2.0 * qmax) {
    // Hankel's expansion for J_0, J_1 then forward recurrence (stable for q < |z|)
    cd J0, J1;
    dev_hankel_J01(z, &J0, &J1);
    out[0] = J0;
    if (qmax >= 1) out[stride] = J1;
    cd inv2 = mk(2.0, 0) / z, jm = J0, jc = J1;
    for (int q = 1; q < qmax; q++) {
      cd jn = (double)q * (inv2 * jc) - jm;
      jm = jc;
      jc = jn;
      out[(q + 1) * stride] = jc;
    }
    return;
  }
  int N = qmax + (int)az + 30 + (int)(6.0 * cbrt(az));
  bool lower = (z.y <= 0.0);
  // w = +i (lower half plane) or -i; track w^n
  cd inv = mk(1, 0) / z;
  cd fp1 = mk(0, 0), f = mk(1e-250, 0);
  cd S = mk(0, 0);
  int r = N & 3;
  // w^N
  cd wn = lower ? ipow(r) : ipow(-r);
  S = 2.0 * (wn * f);
  if (N <= qmax) out[N * stride] = f;
  cd winv = lower ? mk(0, -1) : mk(0, 1);  // 1/w
  for (int n = N; n >= 1; n--) {
    cd fm = (2.0 * n) * (inv * f) - fp1;
    fp1 = f;
    f = fm;
    wn = wn * winv;
    if (n - 1 <= qmax) out[(n - 1) * stride] = f;
    S = S + ((n == 1) ? 1.0 : 2.0) * (wn * f);
    double mag = fabs(f.x) + fabs(f.y);
    if (mag > 1e250) {
      f = 1e-250 * f;
      fp1 = 1e-250 * fp1;
      S = 1e-250 * S;
      for (int m = n - 1; m <= qmax; m++) out[m * stride] = 1e-250 * out[m * stride];
    }
  }
  cd e = lower ? cexpd(mk(-z.y, z.x)) : cexpd(mk(z.y, -z.x));  // e^{iz} or e^{-iz}
  cd sc = e / S;
  for (int q = 0; q <= qmax; q++) out[q * stride] = out[q * stride] * sc;
}

// J_0(z) alone: series (|z| <= 8), Miller (8 < |z| <= 24), Hankel expansion beyond.
__device__ __forceinline__ cd dev_besselJ0(cd z) {
  double az = cmod(z);
  if (az <= 8.0) {
    cd h2 = 0.25 * (z * z), term = mk(1, 0), s = mk(1, 0);
    for (int k = 1; k < 60; k++) {
      term = term * (-1.0 / ((double)k * k)) * h2;
      s = s + term;
      if (cabs2(term) < 1e-36 * cabs2(s) && k > 2) break;
    }
    return s;
  }
  if (az <= 24.0) {
    cd J0;
    dev_besselJ(0, z, &J0, 1);
    return J0;
  }
  // Hankel's expansion: J_0 ~ sqrt(2/(pi z)) (P cos w - Q sin w), w = z - pi/4
  cd iz = mk(1, 0) / z, P = mk(1, 0), Q = mk(0, 0), term = mk(1, 0);
  for (int k = 1; k < 60; k++) {
    double c = -((2.0 * k - 1.0) * (2.0 * k - 1.0)) / (8.0 * k);
    term = term * c * iz;
    if (k & 1) Q = Q + ((((k - 1) >> 1) & 1) ? -1.0 : 1.0) * term;
    else P = P + (((k >> 1) & 1) ? -1.0 : 1.0) * term;
    if (cabs2(term) < 1e-36) break;
  }
  cd w = mk(z.x - 0.25 * LFMM_PI, z.y);
  // cos w, sin w for complex w
  double sx, cx;
  sincos(w.x, &sx, &cx);
  double ch = cosh(w.y), sh = sinh(w.y);
  cd cw = mk(cx * ch, -sx * sh), sw = mk(sx * ch, cx * sh);
  cd pre = csqrtd(mk(2.0 / LFMM_PI, 0) / z);
  return pre * (P * cw - Q * sw);
}

// ---------------------------------------------------------------------------
// Normalised associated Legendre Phat_n^m at complex x with s = sqrt(1-x^2)
// given (on the contour s = k_rho/k, which is the branch of the paper's
// eq. (branch)); out[tix(n,m) * stride], 0 <= m <= n <= p.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void dev_legendre_c(int p, cd x, cd s, cd* out, int stride) {
  cd pmm = mk(0.28209479177387814347, 0);  // 1/sqrt(4 pi)
  for (int m = 0; m <= p; m++) {
    if (m > 0) pmm = sqrt((2.0 * m + 1.0) / (2.0 * m)) * (s * pmm);
    out[tix(m, m) * stride] = pmm;
    if (m + 1 <= p) {
      cd p1 = sqrt(2.0 * m + 3.0) * (x * pmm), p0 = pmm;
      out[tix(m + 1, m) * stride] = p1;
      for (int n = m + 2; n <= p; n++) {
        double a = sqrt((2.0 * n - 1.0) * (2.0 * n + 1.0) / ((double)(n - m) * (n + m)));
        double b = sqrt((2.0 * n + 1.0) * (n - m - 1.0) * (n + m - 1.0) / ((2.0 * n - 3.0) * (n + m) * (double)(n - m)));
        cd p2 = a * (x * p1) - b * p0;
        out[tix(n, m) * stride] = p2;
        p0 = p1;
        p1 = p2;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Layered medium.  Densities by generalised reflection / transmission
// coefficients (the 2x2 reduction the paper mentions at the end of Section 3.1):
// with a_m = k_m kz_m, r = (a_m - a_{m+1})/(a_m + a_{m+1}) and E_m the phase over
// layer m, the down-looking coefficient obeys R_m = (r + R_{m+1}E_{m+1}^2)/(1 + r R_{m+1}E_{m+1}^2),
// the up-looking one the mirror recursion; in the source layer the two
// reflections close the 2x2 system U = R_b(X_b + E D), D = R_t(X_t + E U);
// other layers follow by generalised transmission.  sig[a][b] (a, b: 0 up, 1 down).
// ---------------------------------------------------------------------------
struct Stack {
  int L;
  double d[LFMM_MAXL];
  double k[LFMM_MAXL + 1];
};

// LL > 0: the stack has exactly LL interfaces (arrays stay in registers);
// LL = 0: any L <= LFMM_MAXL.
// With one != nullptr, *one also receives sig[asel][bsel], chosen among register
// values (a caller that indexes sig with runtime values would keep the array in
// memory, which the compiler places in LDS).
template <int LL>
__device__ __forceinline__ void dev_densities_t(const Stack& st, cd kr, int l, int lp, cd sig[2][2], int asel = 0,
                                                int bsel = 0, cd* one = nullptr) {
  constexpr int NL = (LL > 0) ? LL : LFMM_MAXL;
  const int L = (LL > 0) ? LL : st.L;
  cd kz[NL + 1], a[NL + 1], E[NL + 1], Rd[NL + 1], Ru[NL + 1];
  cd kr2 = kr * kr;
#pragma unroll
  for (int m = 0; m <= NL; m++) {
    kz[m] = mk(1, 0);
    a[m] = mk(1, 0);
    E[m] = mk(0, 0);
    if (m > L) continue;
    kz[m] = csqrtd(mk(st.k[m] * st.k[m], 0) - kr2);
    a[m] = st.k[m] * kz[m];
    if (m >= 1 && m <= L - 1) E[m] = cexpd(cmul_i(kz[m] * (st.d[m - 1] - st.d[m])));
  }
  // Rd[m]: reflection looking down from layer m at d_m; Ru[m]: looking up from layer m at d_{m-1}
#pragma unroll
  for (int m = NL; m >= 0; m--) {
    Rd[m] = mk(0, 0);
    if (m >= L) continue;
    cd r = (a[m] - a[m + 1]) / (a[m] + a[m + 1]);
    cd rho = (m + 1 <= L - 1) ? Rd[(m + 1 <= NL) ? m + 1 : NL] * E[(m + 1 <= NL) ? m + 1 : NL] * E[(m + 1 <= NL) ? m + 1 : NL] : mk(0, 0);
    Rd[m] = (r + rho) / (mk(1, 0) + r * rho);
  }
#pragma unroll
  for (int m = 0; m <= NL; m++) {
    Ru[m] = mk(0, 0);
    if (m < 1 || m > L) continue;
    cd r = (a[m] - a[m - 1]) / (a[m] + a[m - 1]);
    cd rho = (m - 1 >= 1) ? Ru[m - 1] * E[m - 1] * E[m - 1] : mk(0, 0);
    Ru[m] = (r + rho) / (mk(1, 0) + r * rho);
  }
  cd Rb = mk(0, 0), Rt = mk(0, 0), Ep = mk(0, 0);
#pragma unroll
  for (int m = 0; m <= NL; m++)
    if (m == lp) {
      if (lp <= L - 1) Rb = Rd[m];
      if (lp >= 1) Rt = Ru[m];
      if (lp >= 1 && lp <= L - 1) Ep = E[m];
    }
  cd Delta = mk(1, 0) - Rb * Rt * Ep * Ep;
#pragma unroll
  for (int b = 0; b < 2; b++) {
    bool exists = (b == 0) ? (lp <= L - 1) : (lp >= 1);
    sig[0][b] = mk(0, 0);
    sig[1][b] = mk(0, 0);
    if (!exists) continue;
    cd Xb = (b == 0) ? mk(1, 0) : mk(0, 0), Xt = (b == 1) ? mk(1, 0) : mk(0, 0);
    cd U = Rb * (Xb + Ep * Rt * Xt) / Delta;  // up-going in the source layer (ref. d_lp)
    cd D = Rt * (Xt + Ep * Rb * Xb) / Delta;  // down-going (ref. d_{lp-1})
    cd Ul = U, Dl = D;
    if (l < lp) {
      // total up-going wave at the top of the source layer, transmitted upward layer by layer
      cd Um = Xt + ((lp <= L - 1) ? Ep * U : mk(0, 0));
#pragma unroll
      for (int m = NL; m >= 1; m--) {
        if (m > lp || m <= l) continue;
        cd r = (a[m] - a[m - 1]) / (a[m] + a[m - 1]);
        cd rho = (m - 1 >= 1) ? Ru[m - 1] * E[m - 1] * E[m - 1] : mk(0, 0);
        cd T = (kz[m - 1] / kz[m]) * (mk(1, 0) + r) / (mk(1, 0) + r * rho);
        Um = T * Um;                        // U_{m-1}, referenced at d_{m-1}
        if (m - 1 > l) Um = E[m - 1] * Um;  // carried to the top of layer m-1
      }
      Ul = Um;
      Dl = mk(0, 0);
#pragma unroll
      for (int m = 0; m <= NL; m++)
        if (m == l && l >= 1) Dl = Ru[m] * E[m] * Ul;
    } else if (l > lp) {
      cd Dm = Xb + ((lp >= 1) ? Ep * D : mk(0, 0));
#pragma unroll
      for (int m = 0; m < NL; m++) {
        if (m < lp || m >= l) continue;
        cd r = (a[m] - a[m + 1]) / (a[m] + a[m + 1]);
        cd rho = (m + 1 <= L - 1) ? Rd[m + 1] * E[m + 1] * E[m + 1] : mk(0, 0);
        cd T = (kz[m + 1] / kz[m]) * (mk(1, 0) + r) / (mk(1, 0) + r * rho);
        Dm = T * Dm;                        // D_{m+1}, referenced at d_m
        if (m + 1 < l) Dm = E[m + 1] * Dm;
      }
      Dl = Dm;
      Ul = mk(0, 0);
#pragma unroll
      for (int m = 0; m <= NL; m++)
        if (m == l && l <= L - 1) Ul = Rd[m] * E[m] * Dl;
    }
    sig[0][b] = (l <= L - 1) ? Ul : mk(0, 0);
    sig[1][b] = (l >= 1) ? Dl : mk(0, 0);
    if (one && b == bsel) *one = asel == 0 ? ((l <= L - 1) ? Ul : mk(0, 0)) : ((l >= 1) ? Dl : mk(0, 0));
  }
}

__device__ __forceinline__ void dev_densities(const Stack& st, cd kr, int l, int lp, cd sig[2][2]) {
  dev_densities_t<0>(st, kr, l, lp, sig);
}

// ---------------------------------------------------------------------------
// Contour quadrature rule.  Gamma1: k_rho = -i s, s in [0, b] (NP1 panels);
// Gamma2: k_rho = t - i b with a near part [0, T0] in panels of length HN and a
// far part [T0, T0 + nfar * hf] in panels of length hf.  Gauss-Legendre with
// NGL points per panel (nodes/weights in the rule's constant table).
// ---------------------------------------------------------------------------
#define LFMM_NGL 16
#define LFMM_NP1 2
// Far panels: the first kg grow geometrically from width hf by the factor g (panel
// k is hf g^k wide), the rest are wmax wide; kg = 0 gives equal panels of width hf.
struct Rule {
  double b, T0, hn, hf, g, wmax;
  int nnear, nfar, kg, pad;
};
__host__ __device__ __forceinline__ int rule_nodes(const Rule& r) { return (LFMM_NP1 + r.nnear + r.nfar) * LFMM_NGL; }

__device__ __forceinline__ void rule_node(const Rule& r, int i, const double* glx, const double* glw, cd* kr, cd* w) {
  int pnl = i / LFMM_NGL, g = i % LFMM_NGL;
  double x = glx[g], ww = glw[g];
  if (pnl < LFMM_NP1) {
    double hw = 0.5 * r.b / LFMM_NP1, mid = (pnl + 0.5) * 2.0 * hw;
    *kr = mk(0.0, -(mid + hw * x));
    *w = mk(0.0, -hw * ww);
    return;
  }
  pnl -= LFMM_NP1;
  double t0, h;
  if (pnl < r.nnear) {
    h = r.hn;
    t0 = pnl * h;
  } else if (r.kg == 0) {
    h = r.hf;
    t0 = r.T0 + (pnl - r.nnear) * h;
  } else {
    const int k = pnl - r.nnear, kk = k < r.kg ? k : r.kg;
    double gk = 1.0, sum = 0.0;  // g^kk and 1 + g + ... + g^(kk-1)
    for (int j = 0; j < kk; j++) {
      sum += gk;
      gk *= r.g;
    }
    t0 = r.T0 + r.hf * sum + (k - kk) * r.wmax;
    h = k < r.kg ? r.hf * gk : r.wmax;
  }
  *kr = mk(t0 + 0.5 * h * (1.0 + x), -r.b);
  *w = mk(0.5 * h * ww, 0.0);
}
