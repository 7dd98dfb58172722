// The surrogate network of the reaction M2L integrals: a multilayer perceptron
// (hidden layers with the SiLU activation, linear output), BF16 weights and
// activations on the matrix cores with FP32 accumulation, FP32 master weights,
// trained on the mean squared error with Adam.
//
// All products of a training step are one kernel, k_mlp_gemm: C = A B with BF16
// operands of arbitrary strides (the forward product X W^T, the input gradient
// dZ W and the weight gradient dZ^T X differ only in which operand dimension is
// contiguous).  A 256-thread workgroup computes a 64 x 64 tile of C: the operand
// tiles (64 x 32) are staged in LDS with k contiguous, and each wave runs 2 x 2
// v_mfma_f32_16x16x16_bf16 blocks (A lane l: row l%16, k 4(l/16)..+3; B lane l:
// column l%16, the same k; D element r of lane l: row 4(l/16)+r, column l%16).
// The epilogue adds the bias and applies SiLU (forward) or multiplies by SiLU'
// of the saved pre-activation (backward).
#include <hip/hip_runtime.h>

#include "lfmm_internal.h"

typedef float v4f __attribute__((ext_vector_type(4)));
typedef short v4s __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short f2bf(float f) {  // round to nearest, ties to even
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float((unsigned)h << 16); }
__device__ __forceinline__ float silu_f(float z) { return z / (1.0f + expf(-z)); }
__device__ __forceinline__ float dsilu_f(float z) {
  float s = 1.0f / (1.0f + expf(-z));
  return s * (1.0f + z * (1.0f - s));
}

#define MG_T 64
#define MG_K 32
#define MG_LDK (MG_K + 8)

__global__ __launch_bounds__(256) void k_mlp_gemm(MlpGemm g) {
  __shared__ unsigned short As[MG_T * MG_LDK], Bs[MG_T * MG_LDK];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int m0 = blockIdx.y * MG_T, n0 = blockIdx.x * MG_T;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  v4f acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; i++)
#pragma unroll
    for (int j = 0; j < 2; j++) acc[i][j] = (v4f){0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < g.K; k0 += MG_K) {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < MG_T * MG_K / 256; i++) {
      const int e = tid + 256 * i;
      int r, k;
      if (g.ak == 1) {
        r = e / MG_K;
        k = e % MG_K;
      } else {
        r = e % MG_T;
        k = e / MG_T;
      }
      const int gr = m0 + r, gk = k0 + k;
      As[r * MG_LDK + k] = (gr < g.M && gk < g.K) ? g.A[(long)gr * g.am + (long)gk * g.ak] : (unsigned short)0;
      if (g.bk == 1) {
        r = e / MG_K;
        k = e % MG_K;
      } else {
        r = e % MG_T;
        k = e / MG_T;
      }
      const int gn = n0 + r, gk2 = k0 + k;
      Bs[r * MG_LDK + k] = (gn < g.N && gk2 < g.K) ? g.B[(long)gk2 * g.bk + (long)gn * g.bn] : (unsigned short)0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < MG_K; kk += 16) {
      v4s a[2], b[2];
#pragma unroll
      for (int t = 0; t < 2; t++) {
        a[t] = *(const v4s*)&As[(wm + 16 * t + (lane & 15)) * MG_LDK + kk + 4 * (lane >> 4)];
        b[t] = *(const v4s*)&Bs[(wn + 16 * t + (lane & 15)) * MG_LDK + kk + 4 * (lane >> 4)];
      }
#pragma unroll
      for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  }
#pragma unroll
  for (int i = 0; i < 2; i++)
#pragma unroll
    for (int j = 0; j < 2; j++)
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const int m = m0 + wm + 16 * i + 4 * (lane >> 4) + r, n = n0 + wn + 16 * j + (lane & 15);
        if (m >= g.M || n >= g.N) continue;
        float v = acc[i][j][r];
        if (g.bias) v += g.bias[n];
        if (g.mode == MLP_EPI_STORE) {
          g.C[(long)m * g.ldc + n] = v;
        } else if (g.mode == MLP_EPI_SILU) {
          g.C[(long)m * g.ldc + n] = v;
          g.Cb[(long)m * g.ldcb + n] = f2bf(silu_f(v));
        } else {  // MLP_EPI_DSILU
          g.Cb[(long)m * g.ldcb + n] = f2bf(v * dsilu_f(g.Zs[(long)m * g.ldz + n]));
        }
      }
}
extern "C" void lk_mlp_gemm(const MlpGemm& g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0) return;
  dim3 grid((g.N + MG_T - 1) / MG_T, (g.M + MG_T - 1) / MG_T);
  k_mlp_gemm<<<grid, 256, 0, s>>>(g);
}

// Output-layer gradient of the mean squared error, d = 2 (y - t) / (B nout) in
// BF16, and per-workgroup FP64 partial sums of (y - t)^2.
__global__ __launch_bounds__(256) void k_mlp_mse(int B, int nout, const float* y, const float* t, long ldt,
                                                 unsigned short* d, double* partial) {
  __shared__ double red[256];
  const long n = (long)B * nout;
  const float sc = 2.0f / (float)n;
  double acc = 0.0;
  for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < n; e += (long)gridDim.x * 256) {
    const long b = e / nout, o = e % nout;
    const float r = y[e] - t[b * ldt + o];
    acc += (double)r * (double)r;
    if (d) d[e] = f2bf(sc * r);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}
__global__ __launch_bounds__(256) void k_sum_partials(int n, const double* partial, double scale, double* out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) acc += partial[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0] * scale;
}
extern "C" void lk_mlp_mse(int B, int nout, const float* y, const float* t, long ldt, unsigned short* d,
                           double* partial, double* loss, hipStream_t s) {
  const int nb = MLP_MSE_BLOCKS;
  k_mlp_mse<<<nb, 256, 0, s>>>(B, nout, y, t, ldt, d, partial);
  k_sum_partials<<<1, 256, 0, s>>>(nb, partial, 1.0 / ((double)B * nout), loss);
}

// Bias gradient: column sums of the BF16 gradient, rows in order.
__global__ __launch_bounds__(256) void k_mlp_colsum(int M, int N, const unsigned short* d, float* gb) {
  const int n = blockIdx.x * 256 + threadIdx.x;
  if (n >= N) return;
  float acc = 0.f;
  for (int m = 0; m < M; m++) acc += bf2f(d[(long)m * N + n]);
  gb[n] = acc;
}
extern "C" void lk_mlp_colsum(int M, int N, const unsigned short* d, float* gb, hipStream_t s) {
  if (N > 0) k_mlp_colsum<<<(N + 255) / 256, 256, 0, s>>>(M, N, d, gb);
}

// Adam on the FP32 master parameters (c1, c2: the bias corrections 1 - beta^t),
// refreshing the BF16 copy.
__global__ __launch_bounds__(256) void k_mlp_adam(long n, float* w, float* m, float* v, const float* g, float lr,
                                                  float b1, float b2, float eps, float c1, float c2,
                                                  unsigned short* wb) {
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    wb[i] = f2bf(wi);
  }
}
extern "C" void lk_mlp_adam(long n, float* w, float* m, float* v, const float* g, float lr, float b1, float b2,
                            float eps, float c1, float c2, unsigned short* wb, hipStream_t s) {
  if (n > 0) k_mlp_adam<<<(unsigned)std::min<long>((n + 255) / 256, 2048), 256, 0, s>>>(n, w, m, v, g, lr, b1, b2, eps, c1, c2, wb);
}

__global__ __launch_bounds__(256) void k_f2bf(long n, const float* x, unsigned short* y) {
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) y[i] = f2bf(x[i]);
}
extern "C" void lk_f2bf(long n, const float* x, unsigned short* y, hipStream_t s) {
  if (n > 0) k_f2bf<<<(unsigned)std::min<long>((n + 255) / 256, 2048), 256, 0, s>>>(n, x, y);
}

// ---------------------------------------------------------------------------
// Surrogate of the reaction M2L integrals.  A class's matrix
// I[(n,m),(n',m')] (m >= 0; the rows with -m follow by symmetry, as in the
// quadrature) is predicted entry by entry in a normalised form:
//   I = env (mu + sd y),   env = [(n+n')! / ((k_t R)^n (k_s R)^{n'}) + 1] / R,
// with R = sqrt(rho^2 + (zt + zs + D)^2).  The first term is the size of the
// entry in the low-frequency limit (k_z -> i k_rho, Phat_n^m ~ (k_rho/k)^n, so
// the integral behaves like the (n+n')-th derivative of 1/R), the second its
// size once k R exceeds the order (an oscillating 1/R); D is the component's
// extra decay length, the rate at which its density sigma(k_rho) falls off at
// large k_rho (the thickness of the layers a transmitted wave crosses; 0 for a
// reflection).  mu and sd are per-output statistics over the training classes,
// sd divided by the entry's weight in the gate's error norm for boxes about
// 1.5 h apart, (n+n')! / ((2n+1)!! (2n'+1)!! 1.5^{n+n'}) (at least 1e-3), so
// that the mean squared error of the network weighs the entries as the gate does.  Output o = 2 (r NC + c) (+1 for the
// imaginary part), r = tix(n, m) the row, c = idx(n', m') the column.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void sur_row_nm(int r, int* n, int* m) {
  int a = 0;
  while ((a + 1) * (a + 2) / 2 <= r) a++;
  *n = a;
  *m = r - a * (a + 1) / 2;
}
__device__ __forceinline__ void sur_col_nm(int c, int* n, int* m) {
  int a = (int)sqrt((double)c);
  while (a * a > c) a--;
  while ((a + 1) * (a + 1) <= c) a++;
  *n = a;
  *m = c - a * a - a;
}
__device__ double sur_env(const ClassDesc& C, double D, double kt, double ks, int n, int n2) {
  const double Z = C.zt + C.zs + D, R = sqrt(C.rho * C.rho + Z * Z);
  double f = 1.0;
  for (int i = 2; i <= n + n2; i++) f *= (double)i;
  return (f / (pow(kt * R, (double)n) * pow(ks * R, (double)n2)) + 1.0) / R;
}
__device__ double sur_weight(int n, int n2) {
  double f = 1.0;
  for (int i = 1; i <= n + n2; i++) f *= (double)i / 1.5;
  for (int i = 3; i <= 2 * n + 1; i += 2) f /= (double)i;
  for (int i = 3; i <= 2 * n2 + 1; i += 2) f /= (double)i;
  return f > 1e-3 ? f : 1e-3;
}
// Quadrature matrices -> normalised targets T [ncls x nout] (mu == nullptr: I / env only).
__global__ __launch_bounds__(256) void k_sur_targets(const ClassDesc* cls, const double* dadd, Stack st,
                                                     const double* Iall, int p, int NC, const float* mu,
                                                     const float* sd, float* T) {
  const ClassDesc C = cls[blockIdx.y];
  const int NT = (p + 1) * (p + 2) / 2, nh = NT * NC;
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= nh) return;
  const int r = e / NC, c = e % NC;
  int n, m, n2, m2;
  sur_row_nm(r, &n, &m);
  sur_col_nm(c, &n2, &m2);
  const double env = sur_env(C, dadd[blockIdx.y], st.k[C.lt], st.k[C.ls], n, n2);
  const double* I = Iall + (size_t)C.out * NC * NC * 2 + 2 * ((size_t)cidx(n, m) * NC + c);
  double vr = I[0] / env, vi = I[1] / env;
  float* o = T + (size_t)blockIdx.y * 2 * nh + 2 * e;
  if (mu) {
    vr = (vr - mu[2 * e]) / sd[2 * e];
    vi = (vi - mu[2 * e + 1]) / sd[2 * e + 1];
  }
  o[0] = (float)vr;
  o[1] = (float)vi;
}
extern "C" void lk_sur_targets(int ncls, const ClassDesc* cls, const double* dadd, Stack st, const double* Iall,
                               int p, int NC, const float* mu, const float* sd, float* T, hipStream_t s) {
  const int nh = (p + 1) * (p + 2) / 2 * NC;
  if (ncls > 0) k_sur_targets<<<dim3((nh + 255) / 256, ncls), 256, 0, s>>>(cls, dadd, st, Iall, p, NC, mu, sd, T);
}
// Per-output mean and standard deviation of the first n rows of T (FP64 sums, rows
// in order), the deviation divided by the output's weight.
__global__ __launch_bounds__(256) void k_sur_colstats(int n, int nout, int NC, const float* T, float* mu, float* sd) {
  const int o = blockIdx.x * 256 + threadIdx.x;
  if (o >= nout) return;
  double s = 0.0;
  for (int i = 0; i < n; i++) s += T[(size_t)i * nout + o];
  const double mean = n > 0 ? s / n : 0.0;
  double v = 0.0;
  for (int i = 0; i < n; i++) {
    const double d = T[(size_t)i * nout + o] - mean;
    v += d * d;
  }
  const double sdev = n > 1 ? sqrt(v / n) : 0.0;
  int rn, rm, cn, cm;
  sur_row_nm((o / 2) / NC, &rn, &rm);
  sur_col_nm((o / 2) % NC, &cn, &cm);
  mu[o] = (float)mean;
  sd[o] = sdev > 1e-30 ? (float)(sdev / sur_weight(rn, cn)) : 1.0f;
}
extern "C" void lk_sur_colstats(int n, int nout, int NC, const float* T, float* mu, float* sd, hipStream_t s) {
  if (nout > 0) k_sur_colstats<<<(nout + 255) / 256, 256, 0, s>>>(n, nout, NC, T, mu, sd);
}
// Network outputs -> integral matrices of the classes (both the m and the -m rows).
__global__ __launch_bounds__(256) void k_sur_write(const ClassDesc* cls, const double* dadd, Stack st, const float* Y,
                                                   int p, int NC, const float* mu, const float* sd, double* Iall) {
  const ClassDesc C = cls[blockIdx.y];
  const int NT = (p + 1) * (p + 2) / 2, nh = NT * NC;
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= nh) return;
  const int r = e / NC, c = e % NC;
  int n, m, n2, m2;
  sur_row_nm(r, &n, &m);
  sur_col_nm(c, &n2, &m2);
  const double env = sur_env(C, dadd[blockIdx.y], st.k[C.lt], st.k[C.ls], n, n2);
  const float* y = Y + (size_t)blockIdx.y * 2 * nh + 2 * e;
  const double vr = env * ((double)mu[2 * e] + (double)sd[2 * e] * (double)y[0]);
  const double vi = env * ((double)mu[2 * e + 1] + (double)sd[2 * e + 1] * (double)y[1]);
  double* out = Iall + (size_t)C.out * NC * NC * 2;
  const size_t o1 = (size_t)cidx(n, m) * NC + c;
  out[2 * o1] = vr;
  out[2 * o1 + 1] = vi;
  if (m > 0) {
    const size_t o2 = (size_t)cidx(n, -m) * NC + cidx(n2, -m2);
    out[2 * o2] = vr;
    out[2 * o2 + 1] = vi;
  }
}
extern "C" void lk_sur_write(int ncls, const ClassDesc* cls, const double* dadd, Stack st, const float* Y, int p,
                             int NC, const float* mu, const float* sd, double* Iall, hipStream_t s) {
  const int nh = (p + 1) * (p + 2) / 2 * NC;
  if (ncls > 0) k_sur_write<<<dim3((nh + 255) / 256, ncls), 256, 0, s>>>(cls, dadd, st, Y, p, NC, mu, sd, Iall);
}
// Error of predicted against reference matrices of each class, in the norm that
// weighs entry (n, n') by its effect on expansions of boxes of size h:
//   w = (k_t h)^n (k_s h)^{n'} / ((2n+1)!! (2n'+1)!!)   (|j_n(k r)| <= (k r)^n / (2n+1)!!),
// err = |w (I_pred - I_ref)|_F / |w I_ref|_F over the m >= 0 rows.  One workgroup per class.
__global__ __launch_bounds__(256) void k_sur_err(const ClassDesc* cls, Stack st, const double* hcls, const double* Ipred,
                                                 const double* Iref, int p, int NC, double* err) {
  __shared__ double r1[256], r2[256];
  const ClassDesc C = cls[blockIdx.x];
  const int NT = (p + 1) * (p + 2) / 2, nh = NT * NC;
  const double h = hcls[blockIdx.x], kt = st.k[C.lt], ks = st.k[C.ls];
  double a1 = 0.0, a2 = 0.0;
  for (int e = threadIdx.x; e < nh; e += 256) {
    const int r = e / NC, c = e % NC;
    int n, m, n2, m2;
    sur_row_nm(r, &n, &m);
    sur_col_nm(c, &n2, &m2);
    double w = pow(kt * h, (double)n) * pow(ks * h, (double)n2);
    for (int i = 3; i <= 2 * n + 1; i += 2) w /= (double)i;
    for (int i = 3; i <= 2 * n2 + 1; i += 2) w /= (double)i;
    const size_t o = 2 * ((size_t)C.out * NC * NC + (size_t)cidx(n, m) * NC + c);
    const double dr = Ipred[o] - Iref[o], di = Ipred[o + 1] - Iref[o + 1];
    a1 += w * w * (dr * dr + di * di);
    a2 += w * w * (Iref[o] * Iref[o] + Iref[o + 1] * Iref[o + 1]);
  }
  r1[threadIdx.x] = a1;
  r2[threadIdx.x] = a2;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      r1[threadIdx.x] += r1[threadIdx.x + s];
      r2[threadIdx.x] += r2[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) err[blockIdx.x] = r2[0] > 0 ? sqrt(r1[0] / r2[0]) : (r1[0] > 0 ? 1e300 : 0.0);
}
extern "C" void lk_sur_err(int ncls, const ClassDesc* cls, Stack st, const double* hcls, const double* Ipred,
                           const double* Iref, int p, int NC, double* err, hipStream_t s) {
  if (ncls > 0) k_sur_err<<<ncls, 256, 0, s>>>(cls, st, hcls, Ipred, Iref, p, NC, err);
}
// Row gather for mini-batches: dst[i] = src[idx[i]] (rows of ncol elements of esz bytes, esz 2 or 4).
__global__ __launch_bounds__(256) void k_gather_rows2(int nrows, const int* idx, int ncol, const unsigned short* src,
                                                      unsigned short* dst) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= (long)nrows * ncol) return;
  const int i = (int)(e / ncol), c = (int)(e % ncol);
  dst[e] = src[(size_t)idx[i] * ncol + c];
}
__global__ __launch_bounds__(256) void k_gather_rows4(int nrows, const int* idx, int ncol, const float* src, float* dst) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= (long)nrows * ncol) return;
  const int i = (int)(e / ncol), c = (int)(e % ncol);
  dst[e] = src[(size_t)idx[i] * ncol + c];
}
extern "C" void lk_gather_rows(int nrows, const int* idx, int ncol, int esz, const void* src, void* dst,
                               hipStream_t s) {
  const long n = (long)nrows * ncol;
  if (n <= 0) return;
  const unsigned nb = (unsigned)((n + 255) / 256);
  if (esz == 2) k_gather_rows2<<<nb, 256, 0, s>>>(nrows, idx, ncol, (const unsigned short*)src, (unsigned short*)dst);
  else k_gather_rows4<<<nb, 256, 0, s>>>(nrows, idx, ncol, (const float*)src, (float*)dst);
}
// T = (T - mu) / sd per output, first n rows.
__global__ __launch_bounds__(256) void k_sur_norm(long n, int nout, float* T, const float* mu, const float* sd) {
  for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < n * nout; e += (long)gridDim.x * 256) {
    const int o = (int)(e % nout);
    T[e] = (T[e] - mu[o]) / sd[o];
  }
}
extern "C" void lk_sur_norm(long n, int nout, float* T, const float* mu, const float* sd, hipStream_t s) {
  if (n > 0) k_sur_norm<<<2048, 256, 0, s>>>(n, nout, T, mu, sd);
}
// Network inputs of n classes: one-hot geometry combination, then t (the box size
// on a log scale mapped to [-1, 1]), 256 times its BF16 rounding residual, T_2(t)
// and T_3(t); BF16 [n][nin].
__global__ __launch_bounds__(256) void k_sur_features(int n, const int* combo, const double* h, int nin, int c0,
                                                      double lh0, double lh1, unsigned short* X) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= (long)n * nin) return;
  const int c = (int)(e / nin), k = (int)(e % nin);
  unsigned short v = 0;
  if (k == combo[c]) {
    v = f2bf(1.0f);
  } else if (k >= c0 && k < c0 + 4) {
    const double t = 2.0 * (log(h[c]) - lh0) / (lh1 - lh0) - 1.0;
    double f = t;
    if (k == c0 + 1) f = 256.0 * (t - (double)bf2f(f2bf((float)t)));
    if (k == c0 + 2) f = 2.0 * t * t - 1.0;
    if (k == c0 + 3) f = 4.0 * t * t * t - 3.0 * t;
    v = f2bf((float)f);
  }
  X[e] = v;
}
extern "C" void lk_sur_features(int n, const int* combo, const double* h, int nin, int c0, double lh0, double lh1,
                                unsigned short* X, hipStream_t s) {
  const long tot = (long)n * nin;
  if (tot > 0) k_sur_features<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(n, combo, h, nin, c0, lh0, lh1, X);
}

// ---------------------------------------------------------------------------
// Pre-computed tables of the reaction M2L integrals (the paper's tabulation of
// Section 3.5, in the form a uniform tree needs): for every geometry combination
// the normalised matrix I / env (as above) as a function of t = log h, on panels
// in t with Chebyshev points of the second kind; an evaluation interpolates it
// (barycentric formula, weights from the host) and multiplies env back.
// Table layout: [slot][entry] complex FP64, slot = (combo * npanel + panel) *
// nnode + node, entry = tix(n, m) NC + idx(n', m').
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_tab_store(const ClassDesc* cls, const double* dadd, const int* slot, Stack st,
                                                   const double* Iall, int p, int NC, double* tab) {
  const ClassDesc C = cls[blockIdx.y];
  const int NT = (p + 1) * (p + 2) / 2, nh = NT * NC;
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= nh) return;
  const int r = e / NC, c = e % NC;
  int n, m, n2, m2;
  sur_row_nm(r, &n, &m);
  sur_col_nm(c, &n2, &m2);
  const double env = sur_env(C, dadd[blockIdx.y], st.k[C.lt], st.k[C.ls], n, n2);
  const double* I = Iall + (size_t)C.out * NC * NC * 2 + 2 * ((size_t)cidx(n, m) * NC + c);
  double* o = tab + ((size_t)slot[blockIdx.y] * nh + e) * 2;
  o[0] = I[0] / env;
  o[1] = I[1] / env;
}
extern "C" void lk_tab_store(int ncls, const ClassDesc* cls, const double* dadd, const int* slot, Stack st,
                             const double* Iall, int p, int NC, double* tab, hipStream_t s) {
  const int nh = (p + 1) * (p + 2) / 2 * NC;
  if (ncls > 0) k_tab_store<<<dim3((nh + 255) / 256, ncls), 256, 0, s>>>(cls, dadd, slot, st, Iall, p, NC, tab);
}
// Interpolated matrices of the classes into Iall (both the m and the -m rows):
// class c uses the nnode table slots from slot0[c] on with weights w[c][j] (they sum to 1).
__global__ __launch_bounds__(256) void k_tab_interp(const ClassDesc* cls, const double* dadd, const int* slot0,
                                                    const double* w, int nnode, Stack st, const double* tab, int p,
                                                    int NC, double* Iall) {
  const ClassDesc C = cls[blockIdx.y];
  const int NT = (p + 1) * (p + 2) / 2, nh = NT * NC;
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= nh) return;
  const int r = e / NC, c = e % NC;
  int n, m, n2, m2;
  sur_row_nm(r, &n, &m);
  sur_col_nm(c, &n2, &m2);
  const double* wc = w + (size_t)blockIdx.y * nnode;
  const double* t = tab + ((size_t)slot0[blockIdx.y] * nh + e) * 2;
  double vr = 0.0, vi = 0.0;
  for (int j = 0; j < nnode; j++) {
    const double wj = wc[j];
    vr += wj * t[(size_t)j * nh * 2];
    vi += wj * t[(size_t)j * nh * 2 + 1];
  }
  const double env = sur_env(C, dadd[blockIdx.y], st.k[C.lt], st.k[C.ls], n, n2);
  vr *= env;
  vi *= env;
  double* out = Iall + (size_t)C.out * NC * NC * 2;
  const size_t o1 = (size_t)cidx(n, m) * NC + c;
  out[2 * o1] = vr;
  out[2 * o1 + 1] = vi;
  if (m > 0) {
    const size_t o2 = (size_t)cidx(n, -m) * NC + cidx(n2, -m2);
    out[2 * o2] = vr;
    out[2 * o2 + 1] = vi;
  }
}
extern "C" void lk_tab_interp(int ncls, const ClassDesc* cls, const double* dadd, const int* slot0, const double* w,
                              int nnode, Stack st, const double* tab, int p, int NC, double* Iall, hipStream_t s) {
  const int nh = (p + 1) * (p + 2) / 2 * NC;
  if (ncls > 0)
    k_tab_interp<<<dim3((nh + 255) / 256, ncls), 256, 0, s>>>(cls, dadd, slot0, w, nnode, st, tab, p, NC, Iall);
}
