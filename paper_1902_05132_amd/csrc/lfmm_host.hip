// Host orchestration and C ABI of the layered-media Helmholtz FMM library.
//
// One lfmm_eval_device call runs every stage of the method on the GPU:
// layer classification, octrees (free-space tree per layer; target and
// polarisation-source trees per reaction direction sharing one root split at
// the interface), operator generation, the upward pass (P2M, M2M), M2L (free and
// the four reaction types), the downward pass (L2L, L2P), near-field sums and
// the component sum.  The host only does bookkeeping on counts read back at a
// few synchronisation points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <atomic>
#include <map>
#include <mutex>
#include <random>
#include <chrono>
#include <set>
#include <thread>
#include <string>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "../../include/lfmm.h"
#include "lfmm_internal.h"

namespace {

struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
};

// Workspace of an allocation-free evaluation: consecutive 256-byte aligned pieces
// of a region the caller did not have to allocate (the library's static device
// scratch).  take() throws LFMM_ENOMEM when the region is exhausted.
struct Arena {
  char* base = nullptr;
  size_t cap = 0, used = 0;
  void* take(size_t bytes);
};

// The library's last failed HIP call, from any thread (for lfmm_last_hip_error).
static std::mutex g_hip_err_mu;
static char g_hip_err[2][160] = {"", ""};
static int g_hip_err_cur = 0;
static void note_hip_error(hipError_t e, int line) {
  std::lock_guard<std::mutex> g(g_hip_err_mu);
  const int nx = g_hip_err_cur ^ 1;
  snprintf(g_hip_err[nx], sizeof(g_hip_err[nx]), "%s (%d) at lfmm_host.hip:%d", hipGetErrorName(e), (int)e, line);
  g_hip_err_cur = nx;
}
#define HIPCHK(x)                       \
  do {                                  \
    hipError_t _e = (x);                \
    if (_e != hipSuccess) {             \
      note_hip_error(_e, __LINE__);     \
      throw Fail{LFMM_EHIP};            \
    }                                   \
  } while (0)

struct Fail {
  int code;
};

void* Arena::take(size_t bytes) {
  const size_t off = (used + 255) & ~(size_t)255;
  if (off > cap || bytes > cap - off) throw Fail{LFMM_ENOMEM};
  used = off + bytes;
  return base + off;
}

enum {
  ST_CLASSIFY, ST_TREE, ST_OPS_FREE, ST_REACT_TABLES, ST_REACT_MFMA, ST_REACT_EXPAND, ST_JOBS, ST_P2M, ST_M2M,
  ST_M2L, ST_L2L, ST_L2P, ST_P2P, ST_NEAR_REACT, ST_SUM, ST_REACT_SUR, ST_REACT_TAB, ST_COUNT
};
const char* kStageNames[ST_COUNT] = {"classify", "tree",  "ops_free", "react_tables",  "react_mfma", "react_expand",
                                     "jobs",     "p2m",   "m2m",      "m2l",           "l2l",        "l2p",
                                     "p2p_free", "near_reaction", "sum", "react_surrogate", "react_table"};

// ---------------------------------------------------------------------------
// Host-side constants owned by the library (independent of any checker):
// Gauss-Legendre rules by Newton iteration on P_n and Gaunt coefficients by
// exact Gauss-Legendre quadrature of triple products of normalised Legendre
// functions, G(nu,mu; q,s; n) = 2 pi int_{-1}^{1} Phat_nu^mu Phat_q^s Phat_n^{mu+s} dx.
// ---------------------------------------------------------------------------
void gauss_rule(int n, std::vector<double>& x, std::vector<double>& w) {
  x.resize(n);
  w.resize(n);
  for (int i = 0; i < n; i++) {
    double t = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; it++) {
      double p0 = 1.0, p1 = t;
      for (int kk = 2; kk <= n; kk++) {
        double p2 = ((2.0 * kk - 1.0) * t * p1 - (kk - 1.0) * p0) / kk;
        p0 = p1;
        p1 = p2;
      }
      double dp = n * (t * p1 - p0) / (t * t - 1.0);
      double dt = p1 / dp;
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    double p0 = 1.0, p1 = t;
    for (int kk = 2; kk <= n; kk++) {
      double p2 = ((2.0 * kk - 1.0) * t * p1 - (kk - 1.0) * p0) / kk;
      p0 = p1;
      p1 = p2;
    }
    double dp = n * (t * p1 - p0) / (t * t - 1.0);
    x[i] = t;
    w[i] = 2.0 / ((1.0 - t * t) * dp * dp);
  }
}

// Phat_n^m(x) for 0 <= m <= n <= P at real x, table [n][m]
void host_phat(int P, double x, std::vector<double>& T) {
  T.assign((P + 1) * (P + 1), 0.0);
  double s = std::sqrt(std::max(0.0, 1.0 - x * x));
  double pmm = 1.0 / std::sqrt(4.0 * M_PI);
  for (int m = 0; m <= P; m++) {
    if (m > 0) pmm *= std::sqrt((2.0 * m + 1.0) / (2.0 * m)) * s;
    T[m * (P + 1) + m] = pmm;
    if (m + 1 <= P) {
      double p0 = pmm, p1 = std::sqrt(2.0 * m + 3.0) * x * pmm;
      T[(m + 1) * (P + 1) + m] = p1;
      for (int n = m + 2; n <= P; n++) {
        double a = std::sqrt((2.0 * n - 1.0) * (2.0 * n + 1.0) / ((double)(n - m) * (n + m)));
        double b = std::sqrt((2.0 * n + 1.0) * (n - m - 1.0) * (n + m - 1.0) / ((2.0 * n - 3.0) * (n + m) * (double)(n - m)));
        double p2 = a * x * p1 - b * p0;
        T[n * (P + 1) + m] = p2;
        p0 = p1;
        p1 = p2;
      }
    }
  }
}

std::vector<double> gaunt_table(int p) {
  int NC = (p + 1) * (p + 1), P2 = 2 * p, NQ = 3 * p + 4;
  std::vector<double> gx, gw;
  gauss_rule(NQ, gx, gw);
  std::vector<std::vector<double>> tabs(NQ);
  for (int g = 0; g < NQ; g++) host_phat(P2, gx[g], tabs[g]);
  auto ph = [&](int g, int n, int m) {
    double v = tabs[g][n * (P2 + 1) + std::abs(m)];
    return (m < 0 && (std::abs(m) & 1)) ? -v : v;
  };
  std::vector<double> G((size_t)NC * NC * (p + 1), 0.0);
  for (int n = 0; n <= p; n++)
    for (int m = -n; m <= n; m++)
      for (int nu = 0; nu <= p; nu++)
        for (int mu = -nu; mu <= nu; mu++) {
          int s = m - mu, q0 = std::abs(n - nu);
          int jmax = std::min(n, nu);
          for (int j = 0; j <= jmax; j++) {
            int q = q0 + 2 * j;
            if (std::abs(s) > q) continue;
            double acc = 0.0;
            for (int g = 0; g < NQ; g++) acc += gw[g] * ph(g, nu, mu) * ph(g, q, s) * ph(g, n, m);
            G[((size_t)cidx(n, m) * NC + cidx(nu, mu)) * (p + 1) + j] = 2.0 * M_PI * acc;
          }
        }
  return G;
}

// x such that the decay x^N e^{-x} has fallen by e^{-c} from its peak at x = N
double decay_length(int N, double c) {
  if (N <= 0) return c;
  double lo = N, hi = N + c + 10.0 * N + 10.0;
  for (int it = 0; it < 200; it++) {
    double mid = 0.5 * (lo + hi);
    double v = mid - N * std::log(mid / N) - N;
    if (v >= c) hi = mid;
    else lo = mid;
  }
  return hi;
}

}  // namespace

// ---------------------------------------------------------------------------
// Surrogate network runtime (kernels in lfmm_mlp.hip): parameters packed per
// layer as the weight matrix [out][in] row-major, then the bias [out]; FP32
// master copy, BF16 copy for the matrix cores, Adam moments, gradient.
// ---------------------------------------------------------------------------
struct MlpNet {
  int nin = 0, width = 0, nh = 0, nout = 0;
  long np = 0;
  std::vector<int> lo, li;
  std::vector<long> woff, boff;
  std::map<std::string, DevBuf> bufs;
  // during an allocation-free evaluation: pieces of the arena for buffers that
  // would otherwise have to grow (forward-pass activations of more rows)
  Arena* arena = nullptr;
  std::map<std::string, DevBuf> abufs;
  void setup(int nin_, int width_, int nh_, int nout_) {
    nin = nin_;
    width = width_;
    nh = nh_;
    nout = nout_;
    lo.clear();
    li.clear();
    woff.clear();
    boff.clear();
    np = 0;
    for (int l = 0; l <= nh; l++) {
      int i = l == 0 ? nin : width, o = l == nh ? nout : width;
      li.push_back(i);
      lo.push_back(o);
      woff.push_back(np);
      np += (long)o * i;
      boff.push_back(np);
      np += o;
    }
  }
  template <typename T>
  T* dev(const std::string& name, size_t count) {
    size_t bytes = std::max<size_t>(count * sizeof(T), 256);
    DevBuf& B = bufs[name];
    if (B.cap < bytes && arena) {
      DevBuf& A = abufs[name];
      if (A.cap < bytes) {
        A.p = arena->take(bytes);
        A.cap = bytes;
      }
      return (T*)A.p;
    }
    if (B.cap < bytes) {
      if (B.p) HIPCHK(hipFree(B.p));
      B.p = nullptr;
      B.cap = 0;
      if (hipMalloc(&B.p, bytes) != hipSuccess) {
        B.p = nullptr;
        throw Fail{LFMM_ENOMEM};
      }
      B.cap = bytes;
    }
    return (T*)B.p;
  }
  void release() {
    for (auto& kv : bufs)
      if (kv.second.p) (void)hipFree(kv.second.p);
    bufs.clear();
  }
  float* w() { return dev<float>("w", np); }
  unsigned short* wb() { return dev<unsigned short>("wb", np); }
  float* z(int l, int B) { return dev<float>("z" + std::to_string(l), (size_t)B * width); }
  unsigned short* a(int l, int B) { return dev<unsigned short>("a" + std::to_string(l), (size_t)B * width); }
  float* y(int B) { return dev<float>("y", (size_t)B * nout); }
  // forward pass of B rows of x (BF16, [B][nin]) -> y [B][nout] (FP32)
  void forward(int B, const unsigned short* x, hipStream_t s) {
    const unsigned short* in = x;
    for (int l = 0; l <= nh; l++) {
      MlpGemm g;
      memset(&g, 0, sizeof(g));
      g.M = B;
      g.N = lo[l];
      g.K = li[l];
      g.A = in;
      g.am = li[l];
      g.ak = 1;
      g.B = wb() + woff[l];
      g.bk = 1;
      g.bn = li[l];
      g.bias = w() + boff[l];
      if (l < nh) {
        g.mode = MLP_EPI_SILU;
        g.C = z(l, B);
        g.ldc = width;
        g.Cb = a(l, B);
        g.ldcb = width;
        in = g.Cb;
      } else {
        g.mode = MLP_EPI_STORE;
        g.C = y(B);
        g.ldc = nout;
      }
      lk_mlp_gemm(g, s);
    }
  }
  // gradient of the mean squared error against t ([B][ldt] FP32) after forward();
  // the loss goes to loss_out (device, one double)
  void backward(int B, const unsigned short* x, const float* t, long ldt, double* loss_out, hipStream_t s) {
    const int dmax = std::max(nout, std::max(width, nin));
    unsigned short* d = dev<unsigned short>("d0", (size_t)B * dmax);
    unsigned short* dn = dev<unsigned short>("d1", (size_t)B * dmax);
    float* grad = dev<float>("g", np);
    lk_mlp_mse(B, nout, y(B), t, ldt, d, dev<double>("partial", MLP_MSE_BLOCKS), loss_out, s);
    for (int l = nh; l >= 0; l--) {
      const unsigned short* ain = l == 0 ? x : a(l - 1, B);
      MlpGemm g;
      memset(&g, 0, sizeof(g));
      g.M = lo[l];  // weight gradient: gW[o][i] = sum_b d[b][o] ain[b][i]
      g.N = li[l];
      g.K = B;
      g.A = d;
      g.am = 1;
      g.ak = lo[l];
      g.B = ain;
      g.bk = li[l];
      g.bn = 1;
      g.mode = MLP_EPI_STORE;
      g.C = grad + woff[l];
      g.ldc = li[l];
      lk_mlp_gemm(g, s);
      lk_mlp_colsum(B, lo[l], d, grad + boff[l], s);
      if (l == 0) break;
      memset(&g, 0, sizeof(g));
      g.M = B;  // dn[b][i] = (sum_o d[b][o] W[o][i]) silu'(z_{l-1}[b][i])
      g.N = li[l];
      g.K = lo[l];
      g.A = d;
      g.am = lo[l];
      g.ak = 1;
      g.B = wb() + woff[l];
      g.bk = li[l];
      g.bn = 1;
      g.mode = MLP_EPI_DSILU;
      g.Cb = dn;
      g.ldcb = li[l];
      g.Zs = z(l - 1, B);
      g.ldz = width;
      lk_mlp_gemm(g, s);
      std::swap(d, dn);
    }
  }
  void adam(int step, float lr, hipStream_t s) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.f - std::pow(b1, (float)step), c2 = 1.f - std::pow(b2, (float)step);
    lk_mlp_adam(np, w(), dev<float>("m", np), dev<float>("v", np), dev<float>("g", np), lr, b1, b2, eps, c1, c2,
                wb(), s);
  }
  // FP32 parameters from the host; BF16 copy and zero Adam moments
  void load_params(const float* host, hipStream_t s) {
    HIPCHK(hipMemcpyAsync(w(), host, np * sizeof(float), hipMemcpyHostToDevice, s));
    lk_f2bf(np, w(), wb(), s);
    HIPCHK(hipMemsetAsync(dev<float>("m", np), 0, np * sizeof(float), s));
    HIPCHK(hipMemsetAsync(dev<float>("v", np), 0, np * sizeof(float), s));
  }
};

// The trained surrogate of the reaction M2L integrals of one plan, and its gate.
struct Surrogate {
  bool ready = false;
  double tol = 0.0;  // gate: classes whose held-out error bound is <= tol use the network
  double h_lo = 0.0, h_hi = 0.0;
  int ncomp = 0;
  std::vector<int> comp_of;  // [(l * 2 + a) * 2 * NL... ] component id of (l, a, lp, b) or -1
  std::vector<double> bound; // [comp][j][i][ri] held-out error bound (inf: none)
  std::vector<float> mu, sd; // per-output statistics (host copies)
  std::vector<double> Dc;    // per component: extra decay length of its density at large k_rho
  MlpNet net;
  lfmm_train_report trep;
  int version = 0;  // changes whenever the network does
};

// Pre-computed tables of the reaction M2L integrals of one plan, and their gate.
// For every geometry combination the normalised integral matrix is tabulated as a
// function of u = ln h + alpha h (alpha = 4 max_l k_l: logarithmic in h where the
// matrices vary as powers of h, linear where they oscillate with h) on npanel equal
// panels of Chebyshev points of the second kind (nnode per panel).
struct OpTables {
  bool ready = false;
  double tol = 0.0;  // gate: classes whose validated bound is <= tol use the tables
  double h_lo = 0.0, h_hi = 0.0, alpha = 0.0, u0 = 0.0, du = 0.0;
  int npanel = 0, nnode = 0, ndense = 0, version = 0;
  std::vector<int> dense;     // [comp][j][i][ri] -> dense combination index, -1 where none
  std::vector<double> bound;  // [comp][j][i][ri] validated error bound (inf: none)
  DevBuf tab;                 // [dense][panel][node] normalised matrices (NT x NC complex FP64)
  lfmm_table_report rep;
  void release() {
    if (tab.p) (void)hipFree(tab.p);
    tab.p = nullptr;
    tab.cap = 0;
    ready = false;
  }
};

// widest far panel of the Sommerfeld contour rule (tuning override LFMM_FAR_CAP)
static const double P_FAR_CAP_DEFAULT = 16.0;

struct lfmm_plan_s {
  Stack st;
  int p, leaf_max, NC, NCK, NRT, NKS, NT, opsz;
  double b, min_gap;
  int max_depth, profile;
  int prec;      // 0: FP64; 1: mixed (FP32 near field and FP32-MFMA M2L)
  int physical = 0;  // 1: return physical potentials instead of the paper's normalisation
  int reuse_ops = 0;  // 1: keep the operators of the last evaluation when its trees are the same
  std::string last_opsig;  // what those operators were generated from
  int prec_parts;  // which stages the mixed path runs in FP32: 1 near field, 2 M2L (both by default)
  int gemm_ks;   // M2L GEMM: waves sharing a 16-target tile, 1, 2, 4 or 8 (0: 4)
  int p2p_ta;    // near field: targets per wave step (64 / p2p_ta sources)
  int p2p_ch;    // near field: sources per LDS tile
  double kmax;
  double far_cap = P_FAR_CAP_DEFAULT;
  double quad_c = 40.0;  // the contour ends where the integrands' envelope has fallen by e^{-quad_c}
  double far_grow = 1.5;  // growth of the far panels beyond the cap (1: none; tuning override LFMM_FAR_GROW)
  int64_t quad_max_nodes = (int64_t)1 << 20;  // contour nodes one class may take (more: LFMM_ENOCONV)
  double* d_gaunt = nullptr;
  std::map<std::string, DevBuf> bufs;
  std::vector<char> hbuf;
  lfmm_report rep;
  hipEvent_t evb[ST_COUNT], eve[ST_COUNT];  // begin / end of each stage (profiling)
  bool ev_ok = false;
  // second stream for the operator generation (free-space operators, then the
  // reaction chain), which depends only on the trees and runs beside the job
  // tables, P2M and near field of the main stream
  hipStream_t s2 = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr, ops_ev = nullptr;
  // third stream for the GEMM job tables, beside the main stream's P2M and near field
  hipStream_t s3 = nullptr;
  hipEvent_t jobs_ev = nullptr;
  Surrogate sur;
  OpTables tab;
  std::vector<int> rop_idx;       // reaction operator of each (trees, level, heights, offset) key
  std::vector<size_t> rop_dirty;  // keys the last evaluation set
  // The charge-dependent launches of the last evaluation, in the order they were
  // queued on its main stream (zeroing, P2M, near field, M2M, M2L, L2L, L2P,
  // reaction near field, component sum).  Everything they read besides the charges
  // stays in the plan's workspace, so replaying them after gathering new charges into
  // tree order evaluates the same positions again (lfmm_apply).
  std::vector<std::function<void(hipStream_t, const double*, double*)>> apply_list;
  bool apply_ready = false;  // the list and its workspace are valid (set by lfmm_prepare / lfmm_eval_device)
  bool prep_only = false;    // the evaluation records the list without running it (lfmm_prepare)
  int64_t apply_n = 0;       // particles of the prepared evaluation
  int apply_ntp = 0;         // tree points (particles plus polarisation images)
  const int* apply_orig = nullptr;  // particle index of each tree point in tree order
  double* apply_pq = nullptr;       // tree-order charges

  // device workspace in use: the plan's own, or one lent by a batch worker
  std::map<std::string, DevBuf>* bufp = &bufs;
  // allocation-free evaluation: every workspace buffer is a piece of this arena
  // (bufp then points at a map of such pieces, which nobody frees)
  Arena* arena = nullptr;
  int device = 0;  // the device the plan's streams belong to
  template <typename T>
  T* dev(const char* name, size_t count) {
    size_t bytes = std::max<size_t>(count * sizeof(T), 256);
    DevBuf& B = (*bufp)[name];
    if (arena) {
      if (B.cap < bytes) {
        B.p = arena->take(bytes);
        B.cap = bytes;
      }
      return (T*)B.p;
    }
    if (B.cap < bytes) {
      if (B.p) HIPCHK(hipFree(B.p));
      B.p = nullptr;
      B.cap = 0;
      size_t nb = bytes + bytes / 8;
      if (hipMalloc(&B.p, nb) != hipSuccess) {
        B.p = nullptr;
        throw Fail{LFMM_ENOMEM};
      }
      B.cap = nb;
    }
    return (T*)B.p;
  }
  // Host-to-device uploads go through a pinned staging arena so that they are
  // truly asynchronous (a copy from pageable memory can hold the host until the
  // stream drains).  The arena is reset at the start of every evaluation, after
  // the last copy out of it has completed; it grows to the size the previous
  // evaluation needed (uploads that do not fit fall back to pageable copies).
  char* pin = nullptr;
  size_t pin_cap = 0, pin_used = 0, pin_need = 0;
  hipEvent_t pin_ev = nullptr;
  bool pin_pending = false;
  void pin_reset() {
    if (pin_pending) {
      HIPCHK(hipEventSynchronize(pin_ev));
      pin_pending = false;
    }
    if (pin_need > pin_cap && !arena) {
      if (pin) (void)hipHostFree(pin);
      pin = nullptr;
      pin_cap = 0;
      size_t nb = pin_need + pin_need / 4;
      if (hipHostMalloc((void**)&pin, nb, hipHostMallocDefault) == hipSuccess) pin_cap = nb;
      else pin = nullptr;
    }
    pin_used = 0;
    pin_need = 0;
  }
  template <typename T>
  T* upload(const char* name, const std::vector<T>& v, hipStream_t s) {
    T* d = dev<T>(name, std::max<size_t>(v.size(), 1));
    size_t bytes = v.size() * sizeof(T);
    if (!bytes) return d;
    size_t off = (pin_used + 255) & ~(size_t)255;
    pin_used = off + bytes;
    pin_need = std::max(pin_need, pin_used);
    if (pin && off + bytes <= pin_cap) {
      memcpy(pin + off, v.data(), bytes);
      HIPCHK(hipMemcpyAsync(d, pin + off, bytes, hipMemcpyHostToDevice, s));
      HIPCHK(hipEventRecord(pin_ev, s));
      pin_pending = true;
    } else {
      HIPCHK(hipMemcpyAsync(d, v.data(), bytes, hipMemcpyHostToDevice, s));
    }
    return d;
  }
  // Device-to-host readbacks of small tables: queued into a pinned buffer, then
  // waited for by polling an event (a blocking sync on a pageable copy has shown
  // millisecond-scale wake-up delays, during which the device idles).
  char* rb = nullptr;
  size_t rb_cap = 0, rb_used = 0;
  hipEvent_t rb_ev = nullptr;
  std::vector<std::pair<void*, std::pair<size_t, size_t>>> rb_list;  // (host dst, (offset, bytes))
  std::vector<std::pair<void*, std::pair<const void*, size_t>>> rb_direct;  // (host dst, (device src, bytes))
  void rb_add(void* dst, const void* src, size_t bytes, hipStream_t s) {
    size_t off = (rb_used + 255) & ~(size_t)255;
    if (arena && off + bytes > rb_cap) {
      // no pinned buffer may be allocated now: copy this one at the flush
      rb_direct.push_back({dst, {src, bytes}});
      return;
    }
    if (off + bytes > rb_cap) {
      rb_flush(s);  // empties the buffer (and waits for what it holds)
      off = 0;
      if (bytes > rb_cap) {
        if (rb) (void)hipHostFree(rb);
        rb = nullptr;
        rb_cap = 0;
        size_t nb = std::max<size_t>(bytes, 1 << 20);
        if (hipHostMalloc((void**)&rb, nb, hipHostMallocDefault) != hipSuccess) throw Fail{LFMM_ENOMEM};
        rb_cap = nb;
      }
    }
    HIPCHK(hipMemcpyAsync(rb + off, src, bytes, hipMemcpyDeviceToHost, s));
    rb_list.push_back({dst, {off, bytes}});
    rb_used = off + bytes;
  }
  void rb_flush(hipStream_t s) {
    rb_mark(s);
    rb_wait();
  }
  // rb_flush in two halves, so that work queued on the stream between them runs while
  // the host waits for the copies
  void rb_mark(hipStream_t s) { HIPCHK(hipEventRecord(rb_ev, s)); }
  void rb_wait() {
    hipError_t e;
    while ((e = hipEventQuery(rb_ev)) == hipErrorNotReady) {
    }
    if (e != hipSuccess) throw Fail{LFMM_EHIP};
    for (auto& d : rb_list) memcpy(d.first, rb + d.second.first, d.second.second);
    rb_list.clear();
    rb_used = 0;
    for (auto& d : rb_direct) HIPCHK(hipMemcpy(d.first, d.second.first, d.second.second, hipMemcpyDeviceToHost));
    rb_direct.clear();
  }
  mutable std::map<int, double> decay_memo;
  double decay_cached(int npow) const {
    auto it = decay_memo.find(npow);
    if (it != decay_memo.end()) return it->second;
    double U = decay_length(npow, quad_c);
    decay_memo[npow] = U;
    return U;
  }
  Rule make_rule(double dz, double rho, int npow) const {
    Rule r;
    memset(&r, 0, sizeof(r));
    r.b = b;
    r.T0 = 0.5 * std::ceil(2.0 * (kmax + 2.0));
    r.hn = 0.5;
    r.nnear = (int)std::lround(r.T0 / r.hn);
    double U = decay_cached(npow);
    double tfar = U / dz;
    // far panels: a few decay lengths of e^{-t dz} wide, at most a fraction of the
    // oscillation period 2 pi / rho of J_q(t rho)
    double wlim = 8.0 / dz;
    if (rho > 0.0) wlim = std::min(wlim, 7.0 / rho);
    double hf = std::min(wlim, far_cap);
    r.g = 1.0;
    if (far_grow > 1.0 && wlim > hf * (1.0 + 1e-12)) {
      // the cap holds near T0, where the densities' faster-decaying terms (multiple
      // reflections, e^{-2 t d}) still matter; beyond, only the polynomial and the
      // exponential remain, and the panels widen geometrically up to wlim
      r.hf = hf;
      r.g = far_grow;
      r.wmax = wlim;
      double w = hf;
      while (w < wlim && r.kg < 64) {
        r.kg++;
        w *= far_grow;
      }
      // panels the budget leaves for the far part (LFMM_NP1 + nnear are taken)
      const int64_t kbud = quad_max_nodes / LFMM_NGL - LFMM_NP1 - r.nnear;
      double t = r.T0, wk = hf;
      int64_t k = 0;
      while (t < tfar && k < r.kg) {  // the growing panels
        t += wk;
        wk *= far_grow;
        k++;
      }
      if (t < tfar) {  // then panels of width wlim up to tfar
        const double more = std::ceil((tfar - t) / wlim);
        if (!(more <= (double)kbud)) throw Fail{LFMM_ENOCONV};
        k += (int64_t)more;
      }
      if (k > kbud) throw Fail{LFMM_ENOCONV};
      r.nfar = std::max<int>(1, (int)k);
      return r;
    }
    const double nf = std::ceil(tfar / hf);
    if (!(nf <= (double)(quad_max_nodes / LFMM_NGL - LFMM_NP1 - r.nnear))) throw Fail{LFMM_ENOCONV};
    r.nfar = std::max(1, (int)nf);
    r.hf = tfar / r.nfar;
    r.wmax = r.hf;
    return r;
  }
};

namespace {

// The plan's parameters from the arguments of lfmm_plan, on the host only.
int plan_params(int L, const double* d, const double* k, int p, int leaf_max, const lfmm_options* opt,
                lfmm_plan_s* P) {
  if (L < 0 || L > LFMM_MAXL || p < 1 || p > LFMM_PMAX || leaf_max < 1) return LFMM_EINVAL;
  if (L > 0 && !d) return LFMM_EINVAL;
  if (!k) return LFMM_EINVAL;
  for (int i = 0; i <= L; i++)
    if (!(k[i] > 0.0) || !std::isfinite(k[i])) return LFMM_EINVAL;
  for (int i = 0; i < L; i++) {
    if (!std::isfinite(d[i])) return LFMM_EINVAL;
    if (i > 0 && !(d[i] < d[i - 1])) return LFMM_EINVAL;
  }
  P->st.L = L;
  for (int i = 0; i < LFMM_MAXL; i++) P->st.d[i] = (i < L) ? d[i] : 0.0;
  P->kmax = 0;
  for (int i = 0; i <= LFMM_MAXL; i++) {
    P->st.k[i] = (i <= L) ? k[i] : 1.0;
    if (i <= L) P->kmax = std::max(P->kmax, k[i]);
  }
  P->p = p;
  P->leaf_max = leaf_max;
  P->NC = (p + 1) * (p + 1);
  P->NCK = (P->NC + 3) / 4 * 4;
  P->NRT = (P->NC + 15) / 16;
  P->NKS = P->NCK / 4;
  P->NT = (p + 1) * (p + 2) / 2;
  P->opsz = P->NRT * P->NKS * 128;
  P->gemm_ks = 0;
  P->p2p_ta = 8;
  P->p2p_ch = 256;
  if (const char* e = getenv("LFMM_P2P_TA")) P->p2p_ta = atoi(e);  // tile-shape overrides for tuning runs
  if (const char* e = getenv("LFMM_P2P_CH")) P->p2p_ch = atoi(e);
  if (const char* e = getenv("LFMM_GEMM_KS")) {  // tile-shape override for tuning runs
    int v = atoi(e);
    if (v == 1 || v == 2 || v == 4 || v == 8) P->gemm_ks = v;
  }
  if (const char* e = getenv("LFMM_FAR_CAP")) P->far_cap = atof(e);
  if (const char* e = getenv("LFMM_FAR_GROW")) P->far_grow = atof(e);
  P->b = 0.5;
  P->min_gap = 1e-9;
  P->max_depth = 8;
  P->profile = 0;
  P->prec = 0;
  P->prec_parts = 3;
  if (const char* e = getenv("LFMM_PREC_PARTS")) P->prec_parts = atoi(e) & 3;  // accuracy studies
  if (opt) {
    if (opt->contour_b > 0) P->b = opt->contour_b;
    if (opt->max_depth > 0) P->max_depth = std::min(8, opt->max_depth);
    if (opt->min_gap > 0) P->min_gap = opt->min_gap;
    P->profile = opt->profile;
    if (opt->precision < 0 || opt->precision > 1) {
      return LFMM_EINVAL;
    }
    P->prec = opt->precision;
    if (opt->physical < 0 || opt->physical > 1) {
      return LFMM_EINVAL;
    }
    P->physical = opt->physical;
    if (opt->reuse_operators < 0 || opt->reuse_operators > 1) {
      return LFMM_EINVAL;
    }
    P->reuse_ops = opt->reuse_operators;
    if (opt->quad_tol < 0 || opt->quad_tol >= 1 || std::isnan(opt->quad_tol)) {
      return LFMM_EINVAL;
    }
    if (opt->quad_tol > 0) P->quad_c = -std::log(opt->quad_tol);
    if (opt->quad_max_nodes < 0) return LFMM_EINVAL;
    if (opt->quad_max_nodes > 0) P->quad_max_nodes = opt->quad_max_nodes;
  }
  return LFMM_OK;
}

int plan_impl(int L, const double* d, const double* k, int p, int leaf_max, const lfmm_options* opt,
              lfmm_plan_t** out) {
  if (!out) return LFMM_EINVAL;
  *out = nullptr;
  lfmm_plan_s* P = new lfmm_plan_s();
  if (int rc = plan_params(L, d, k, p, leaf_max, opt, P)) {
    delete P;
    return rc;
  }
  memset(&P->rep, 0, sizeof(P->rep));
  try {
    std::vector<double> gx, gw;
    gauss_rule(LFMM_NGL, gx, gw);
    lk_set_gl(gx.data(), gw.data());
    lk_m2l_gemm_init();
    std::vector<double> G = gaunt_table(p);
    HIPCHK(hipMalloc(&P->d_gaunt, G.size() * sizeof(double)));
    HIPCHK(hipMemcpy(P->d_gaunt, G.data(), G.size() * sizeof(double), hipMemcpyHostToDevice));
    P->ev_ok = true;
    for (int i = 0; i < ST_COUNT; i++)
      if (hipEventCreate(&P->evb[i]) != hipSuccess || hipEventCreate(&P->eve[i]) != hipSuccess) P->ev_ok = false;
    HIPCHK(hipStreamCreateWithFlags(&P->s2, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&P->fork_ev, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&P->join_ev, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&P->ops_ev, hipEventDisableTiming));
    HIPCHK(hipStreamCreateWithFlags(&P->s3, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&P->jobs_ev, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&P->pin_ev, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&P->rb_ev, hipEventDisableTiming));
    // the readback buffer exists before the first evaluation, so that an
    // allocation-free evaluation finds one
    if (hipHostMalloc((void**)&P->rb, (size_t)1 << 20, hipHostMallocDefault) != hipSuccess) throw Fail{LFMM_ENOMEM};
    P->rb_cap = (size_t)1 << 20;
    HIPCHK(hipGetDevice(&P->device));
  } catch (Fail& f) {
    lfmm_destroy(P);
    return f.code;
  }
  *out = P;
  return LFMM_OK;
}

// Reaction integral matrices of the given classes into Iall (class c at c.out):
// node tables per rule group (classes with the same quadrature rule and rho),
// F per class, then the MFMA node sum.  reaction_prep does the host bookkeeping
// and the uploads (on stream up), reaction_launch the kernels (on stream s), so
// that an evaluation can upload everything on its main stream before it forks
// the kernels onto the second one (copies of both streams share one DMA queue:
// an upload queued on the second stream behind its kernels would hold up every
// later upload of the main stream).
struct RIPrep {
  ClassDesc* cls = nullptr;
  RGDesc* rgs = nullptr;
  SCDesc* scs = nullptr;
  int* mem = nullptr;
  double *J = nullptr, *Pt = nullptr, *F = nullptr, *Lt = nullptr;
  int nrg = 0, ncls = 0, nsc = 0, nwg = 0, Ntot = 0, Ftot = 0;
};
static RIPrep reaction_prep(lfmm_plan_s* P, const char* tag, std::vector<ClassDesc>& classes, hipStream_t up) {
  RIPrep R;
  if (classes.empty()) return R;
  const int p = P->p, Q = 2 * p, NT = P->NT, NL = P->st.L + 1;
  // rule groups in order of first appearance (a hash map: this bookkeeping runs while
  // the GPU waits for the operator stream's first kernels)
  typedef std::tuple<double, double, double, double, int, int, double, double, int> RGKey;
  struct RGKeyHash {
    size_t operator()(const RGKey& k) const {
      size_t h = 1469598103934665603ull;
      auto mix = [&h](size_t v) { h = (h ^ v) * 1099511628211ull; };
      const std::hash<double> hd;
      mix(hd(std::get<0>(k)));
      mix(hd(std::get<1>(k)));
      mix(hd(std::get<2>(k)));
      mix(hd(std::get<3>(k)));
      mix((size_t)std::get<4>(k));
      mix((size_t)std::get<5>(k));
      mix(hd(std::get<6>(k)));
      mix(hd(std::get<7>(k)));
      mix((size_t)std::get<8>(k));
      return h;
    }
  };
  std::unordered_map<RGKey, int, RGKeyHash> key_rg;
  key_rg.reserve(classes.size());
  std::vector<RGDesc> rgs;
  int Ntot = 0, Ftot = 0;
  for (auto& C : classes) {
    const RGKey key(C.rule.b, C.rule.T0, C.rule.hn, C.rule.hf, C.rule.nnear, C.rule.nfar, C.rho, C.rule.wmax,
                    C.rule.kg);
    auto it = key_rg.find(key);
    int nn = rule_nodes(C.rule);
    if (it == key_rg.end()) {
      RGDesc R;
      memset(&R, 0, sizeof(R));
      R.rule = C.rule;
      R.rho = C.rho;
      R.off = Ntot;
      R.nn = nn;
      Ntot += nn;
      it = key_rg.emplace(key, (int)rgs.size()).first;
      rgs.push_back(R);
    }
    C.rg_off = rgs[it->second].off;
    C.f_off = Ftot;
    Ftot += nn;
  }
  // stacks: classes with the same rule group and source layer, at most SC_GMAX
  // of them and three target layers each
  // (rule group, source layer) in ascending order, each with its classes by target
  // layer and then by index: one sort of (rg_off, ls, lt, class) entries
  const int NTILE = (P->NC + 15) / 16;
  std::vector<std::array<int, 4>> ord(classes.size());
  for (int c = 0; c < (int)classes.size(); c++) ord[c] = {classes[c].rg_off, classes[c].ls, classes[c].lt, c};
  std::sort(ord.begin(), ord.end());
  std::vector<SCDesc> scs;
  std::vector<int> members;
  int nwg = 0;
  std::vector<int> mem;
  for (size_t o0 = 0; o0 < ord.size();) {
    size_t o1 = o0;
    mem.clear();
    while (o1 < ord.size() && ord[o1][0] == ord[o0][0] && ord[o1][1] == ord[o0][1]) mem.push_back(ord[o1++][3]);
    size_t i = 0;
    while (i < mem.size()) {
      SCDesc S;
      memset(&S, 0, sizeof(S));
      S.rg_off = ord[o0][0];
      S.ls = ord[o0][1];
      S.nn = rule_nodes(classes[mem[i]].rule);
      S.mem0 = (int)members.size();
      while (i < mem.size() && S.G < SC_GMAX) {
        int lt = classes[mem[i]].lt, slot = -1;
        for (int k = 0; k < S.nlt; k++)
          if (S.lt[k] == lt) slot = k;
        if (slot < 0) {
          if (S.nlt == 3) break;
          S.lt[S.nlt++] = lt;
        }
        members.push_back(mem[i]);
        S.G++;
        i++;
      }
      for (int m = 0; m <= p; m++) S.NU += ((S.G * (p + 1 - m) + 15) / 16) * NTILE;
      S.wg0 = nwg;
      nwg += (S.NU + 8 * SC_UPW - 1) / (8 * SC_UPW);
      scs.push_back(S);
    }
    o0 = o1;
  }
  std::string t(tag);
  R.cls = P->upload((t + "_cls").c_str(), classes, up);
  R.rgs = P->upload((t + "_rgs").c_str(), rgs, up);
  R.scs = P->upload((t + "_scs").c_str(), scs, up);
  R.mem = P->upload((t + "_mem").c_str(), members, up);
  R.J = P->dev<double>((t + "_J").c_str(), (size_t)Ntot * (Q + 1) * 2);
  R.Pt = P->dev<double>((t + "_P").c_str(), (size_t)NL * Ntot * NT * 2);
  R.F = P->dev<double>((t + "_F").c_str(), (size_t)Ftot * 2);
  // stacks deeper than the specialised density kernels: the layer recursions once
  // per node (6 quantities per layer), shared by every class on that node
  if (P->st.L > 4) R.Lt = P->dev<double>((t + "_Lt").c_str(), (size_t)6 * NL * Ntot * 2);
  R.nrg = (int)rgs.size();
  R.ncls = (int)classes.size();
  R.nsc = (int)scs.size();
  R.nwg = nwg;
  R.Ntot = Ntot;
  R.Ftot = Ftot;
  return R;
}
static void reaction_launch(lfmm_plan_s* P, const RIPrep& R, double* Iall, hipStream_t s,
                            const std::function<void()>& after_tables = nullptr) {
  if (!R.ncls) return;
  lk_react_tables(R.nrg, R.rgs, R.Ntot, P->st, P->p, R.J, R.Pt, R.Lt, s);
  lk_react_F(R.ncls, R.cls, R.Ftot, P->st, R.Ntot, R.Lt, R.F, s);
  if (after_tables) after_tables();
  lk_react_mfma(R.nwg, R.nsc, R.scs, R.mem, R.cls, P->p, R.Ntot, R.J, R.Pt, R.F, Iall, P->NC, s);
}
static void reaction_integrals(lfmm_plan_s* P, const char* tag, std::vector<ClassDesc>& classes, double* Iall,
                               hipStream_t s) {
  RIPrep R = reaction_prep(P, tag, classes, s);
  reaction_launch(P, R, Iall, s);
}

inline int has_dir(const Stack& st, int l, int a) { return a == 0 ? (l <= st.L - 1) : (l >= 1); }

// ---------------------------------------------------------------------------
// Surrogate training.  Geometry combinations of a component: heights j, i of the
// target and source boxes (in boxes above / below the interface) and the lateral
// offset class r2 = (dx^2 + dy^2) / h^2; (j, i) = (0, 0) has no r2 <= 2 (adjacent
// boxes are near field).  Input features (built on the GPU, k_sur_features): one-hot
// geometry combination (component, j, i, r2 class), and t = the box size on a log
// scale mapped to [-1, 1] (with its rounding residual, scaled by 256, so that BF16
// inputs still resolve h) plus T_2(t), T_3(t).
// ---------------------------------------------------------------------------
const int kR2[10] = {0, 1, 2, 4, 5, 8, 9, 10, 13, 18};
inline int sur_nin(int ncomp) { return (ncomp * 40 + 4 + 31) / 32 * 32; }
inline int sur_combo(int comp, int j, int i, int ri) { return ((comp * 2 + j) * 2 + i) * 10 + ri; }
void sur_components(lfmm_plan_s* P) {
  Surrogate& S = P->sur;
  const Stack& st = P->st;
  const int NL = st.L + 1;
  S.comp_of.assign((size_t)NL * 2 * NL * 2, -1);
  S.ncomp = 0;
  for (int l = 0; l < NL; l++)
    for (int a = 0; a < 2; a++)
      for (int lp = 0; lp < NL; lp++)
        for (int b = 0; b < 2; b++)
          if (has_dir(st, l, a) && has_dir(st, lp, b)) S.comp_of[((l * 2 + a) * NL + lp) * 2 + b] = S.ncomp++;
}
inline int sur_comp(const lfmm_plan_s* P, int l, int a, int lp, int b) {
  const int NL = P->st.L + 1;
  return P->sur.comp_of[((l * 2 + a) * NL + lp) * 2 + b];
}
// Extra decay length of each component's density: -d ln|sigma| / d k_rho between
// k_rho = 30 and 60 (beyond every wavenumber the plan accepts as typical), i.e.
// the thickness of the layers between the two interfaces the component couples.
void sur_decay(lfmm_plan_s* P) {
  Surrogate& S = P->sur;
  const int NL = P->st.L + 1;
  S.Dc.assign(S.ncomp, 0.0);
  const double kr[4] = {30.0, 0.0, 60.0, 0.0};
  double* dk = P->dev<double>("sur_dk", 4);
  double* ds = P->dev<double>("sur_ds", 16);
  HIPCHK(hipMemcpy(dk, kr, sizeof(kr), hipMemcpyHostToDevice));
  for (int l = 0; l < NL; l++)
    for (int lp = 0; lp < NL; lp++) {
      double out[16];
      lk_dbg_dens(2, dk, P->st, l, lp, ds, nullptr);
      HIPCHK(hipMemcpy(out, ds, sizeof(out), hipMemcpyDeviceToHost));
      for (int a = 0; a < 2; a++)
        for (int b = 0; b < 2; b++) {
          const int c = sur_comp(P, l, a, lp, b);
          if (c < 0) continue;
          const int e = 2 * (2 * a + b);
          const double s1 = std::hypot(out[e], out[e + 1]), s2 = std::hypot(out[8 + e], out[8 + e + 1]);
          S.Dc[c] = (s1 > 0 && s2 > 0) ? std::max(0.0, -std::log(s2 / s1) / 30.0) : 0.0;
        }
    }
}

void sur_train_impl(lfmm_plan_s* P, int64_t n_samples, uint64_t seed, const lfmm_train_opts& o,
                    lfmm_train_report& R) {
  Surrogate& S = P->sur;
  const Stack& st = P->st;
  const int NL = st.L + 1, p = P->p, NC = P->NC, NT = P->NT;
  hipStream_t s = P->s2;
  auto wall = []() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
  };
  S.ready = false;
  S.h_lo = o.h_min;
  S.h_hi = o.h_max;
  sur_components(P);
  sur_decay(P);
  const int nout = 2 * NT * NC, nin = sur_nin(S.ncomp);
  S.net.setup(nin, o.width, o.nhidden, nout);
  S.bound.assign((size_t)S.ncomp * 40, INFINITY);
  memset(&R, 0, sizeof(R));
  R.n_combos = S.ncomp * 37;
  R.nin = nin;
  R.nout = nout;
  // ---- sampling: stratified log-uniform box sizes per combination, evenly spaced strata held out
  struct Smp {
    int comp, j, i, ri;
    double h;
  };
  std::vector<Smp> tr, ho;
  const int nper = n_samples > 0 ? std::max<int>(4, (int)((n_samples + R.n_combos - 1) / R.n_combos)) : 48;
  const int nhold = std::max(1, (int)std::lround(o.holdout * nper));
  const int stride = std::max(1, nper / nhold);
  std::mt19937_64 rng(seed);
  std::uniform_real_distribution<double> U(0.0, 1.0);
  const double lh0 = std::log(S.h_lo), lh1 = std::log(S.h_hi);
  for (int l = 0; l < NL; l++)
    for (int a = 0; a < 2; a++)
      for (int lp = 0; lp < NL; lp++)
        for (int b = 0; b < 2; b++) {
          const int comp = sur_comp(P, l, a, lp, b);
          if (comp < 0) continue;
          for (int j = 0; j < 2; j++)
            for (int i = 0; i < 2; i++)
              for (int ri = 0; ri < 10; ri++) {
                if (i == 0 && j == 0 && kR2[ri] <= 2) continue;
                int held = 0;
                for (int k = 0; k < nper; k++) {
                  Smp m{comp, j, i, ri, std::exp(lh0 + (k + U(rng)) / nper * (lh1 - lh0))};
                  if (k % stride == stride / 2 && held < nhold) {
                    ho.push_back(m);
                    held++;
                  } else {
                    tr.push_back(m);
                  }
                }
              }
        }
  std::vector<int4> comp_lab(S.ncomp);
  for (int l = 0; l < NL; l++)
    for (int a = 0; a < 2; a++)
      for (int lp = 0; lp < NL; lp++)
        for (int b = 0; b < 2; b++) {
          int c = sur_comp(P, l, a, lp, b);
          if (c >= 0) comp_lab[c] = make_int4(l, a, lp, b);
        }
  auto make_class = [&](const Smp& m, int out) {
    ClassDesc C;
    memset(&C, 0, sizeof(C));
    C.zt = (m.j + 0.5) * m.h;
    C.zs = (m.i + 0.5) * m.h;
    C.rho = m.h * std::sqrt((double)kR2[m.ri]);
    C.rule = P->make_rule(C.zt + C.zs, C.rho, 2 * p + 1);
    C.lt = comp_lab[m.comp].x;
    C.a = comp_lab[m.comp].y;
    C.ls = comp_lab[m.comp].z;
    C.b = comp_lab[m.comp].w;
    C.out = out;
    return C;
  };
  const int64_t ntr = (int64_t)tr.size(), nho = (int64_t)ho.size(), ntot = ntr + nho;
  R.n_train = ntr;
  R.n_holdout = nho;
  R.n_values = ntr * NT * NC;
  const size_t mat = (size_t)NC * NC * 2;
  // ---- labels by quadrature, in chunks
  double t0 = wall();
  MlpNet& N = S.net;
  float* T = N.dev<float>("T", (size_t)ntr * nout);
  double* Iref = N.dev<double>("Iref", (size_t)nho * mat);
  const int CHK = 1024;
  double* Ich = N.dev<double>("Ich", (size_t)CHK * mat);
  for (int64_t c0 = 0; c0 < ntot; c0 += CHK) {
    const int nc = (int)std::min<int64_t>(CHK, ntot - c0);
    HIPCHK(hipStreamSynchronize(s));
    P->pin_reset();
    std::vector<ClassDesc> cls(nc);
    for (int c = 0; c < nc; c++) {
      const int64_t g = c0 + c;
      cls[c] = make_class(g < ntr ? tr[g] : ho[g - ntr], c);
    }
    std::vector<double> dadd(nc);
    for (int c = 0; c < nc; c++) {
      const int64_t g = c0 + c;
      dadd[c] = S.Dc[(g < ntr ? tr[g] : ho[g - ntr]).comp];
    }
    reaction_integrals(P, "sur", cls, Ich, s);
    ClassDesc* dcls = P->upload("sur_lab_cls", cls, s);
    double* ddadd = P->upload("sur_lab_dadd", dadd, s);
    const int ntrain_here = (int)std::max<int64_t>(0, std::min<int64_t>(ntr - c0, nc));
    if (ntrain_here > 0)
      lk_sur_targets(ntrain_here, dcls, ddadd, st, Ich, p, NC, nullptr, nullptr, T + (size_t)c0 * nout, s);
    if (ntrain_here < nc) {
      const int64_t h0 = c0 + ntrain_here - ntr;
      HIPCHK(hipMemcpyAsync(Iref + (size_t)h0 * mat, Ich + (size_t)ntrain_here * mat,
                            (size_t)(nc - ntrain_here) * mat * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
  }
  float* mu = N.dev<float>("mu", nout);
  float* sd = N.dev<float>("sd", nout);
  lk_sur_colstats((int)ntr, nout, NC, T, mu, sd, s);
  lk_sur_norm(ntr, nout, T, mu, sd, s);
  HIPCHK(hipStreamSynchronize(s));
  R.ms_labels = wall() - t0;
  // ---- inputs
  std::vector<int> xc(ntot);
  std::vector<double> xh(ntot);
  for (int64_t g = 0; g < ntot; g++) {
    const Smp& m = g < ntr ? tr[g] : ho[g - ntr];
    xc[g] = sur_combo(m.comp, m.j, m.i, m.ri);
    xh[g] = m.h;
  }
  int* dxc = N.dev<int>("xc", ntot);
  double* dxh = N.dev<double>("xh", ntot);
  HIPCHK(hipMemcpy(dxc, xc.data(), ntot * sizeof(int), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(dxh, xh.data(), ntot * sizeof(double), hipMemcpyHostToDevice));
  unsigned short* dX = N.dev<unsigned short>("X", (size_t)ntot * nin);
  lk_sur_features((int)ntot, dxc, dxh, nin, S.ncomp * 40, std::log(S.h_lo), std::log(S.h_hi), dX, s);
  // ---- initialisation: uniform +-sqrt(6 / fan_in) weights, zero biases
  t0 = wall();
  std::vector<float> w0(N.np, 0.0f);
  for (int l = 0; l <= N.nh; l++) {
    const double lim = std::sqrt(6.0 / N.li[l]);
    for (long e = 0; e < (long)N.lo[l] * N.li[l]; e++) w0[N.woff[l] + e] = (float)(lim * (2.0 * U(rng) - 1.0));
  }
  N.load_params(w0.data(), s);
  // ---- Adam on shuffled mini-batches, cosine-decayed step size
  const int B = o.batch, spe = (int)((ntr + B - 1) / B), total = o.epochs * spe;
  int* didx = N.dev<int>("idx", ntr);
  unsigned short* xb = N.dev<unsigned short>("xb", (size_t)B * nin);
  float* tb = N.dev<float>("tb", (size_t)B * nout);
  double* losses = N.dev<double>("losses", o.epochs + 1);
  double* lossb = N.dev<double>("lossb", 1);
  std::vector<int> perm(ntr);
  for (int64_t i = 0; i < ntr; i++) perm[i] = (int)i;
  int step = 0;
  for (int e = 0; e < o.epochs; e++) {
    std::shuffle(perm.begin(), perm.end(), rng);
    HIPCHK(hipStreamSynchronize(s));
    HIPCHK(hipMemcpy(didx, perm.data(), perm.size() * sizeof(int), hipMemcpyHostToDevice));
    for (int sb = 0; sb < spe; sb++) {
      const int b0 = sb * B, nb = (int)std::min<int64_t>(B, ntr - b0);
      lk_gather_rows(nb, didx + b0, nin, 2, dX, xb, s);
      lk_gather_rows(nb, didx + b0, nout, 4, T, tb, s);
      N.forward(nb, xb, s);
      double* lo = (step == 0) ? losses : (sb == spe - 1 ? losses + e + 1 : lossb);
      N.backward(nb, xb, tb, nout, lo, s);
      const double lr = o.lr * (0.01 + 0.99 * 0.5 * (1.0 + std::cos(LFMM_PI * step / std::max(1, total))));
      N.adam(++step, (float)lr, s);
    }
  }
  std::vector<double> hl(o.epochs + 1);
  HIPCHK(hipStreamSynchronize(s));
  HIPCHK(hipMemcpy(hl.data(), losses, hl.size() * sizeof(double), hipMemcpyDeviceToHost));
  R.ms_train = wall() - t0;
  R.epochs = o.epochs;
  R.steps = step;
  R.loss_first = hl[0];
  R.loss_last = hl[o.epochs];
  // ---- held-out errors -> gate bounds
  S.mu.resize(nout);
  S.sd.resize(nout);
  HIPCHK(hipMemcpy(S.mu.data(), mu, nout * sizeof(float), hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(S.sd.data(), sd, nout * sizeof(float), hipMemcpyDeviceToHost));
  if (nho > 0) {
    double* Ipred = N.dev<double>("Ipred", (size_t)nho * mat);
    std::vector<ClassDesc> hc(nho);
    std::vector<double> hh(nho), hd(nho);
    for (int64_t g = 0; g < nho; g++) {
      hc[g] = make_class(ho[g], (int)g);
      hh[g] = ho[g].h;
      hd[g] = S.Dc[ho[g].comp];
    }
    ClassDesc* dhc = N.dev<ClassDesc>("hold_cls", nho);
    double* dhh = N.dev<double>("hold_h", nho);
    double* dhd = N.dev<double>("hold_d", nho);
    double* derr = N.dev<double>("hold_err", nho);
    HIPCHK(hipMemcpy(dhc, hc.data(), nho * sizeof(ClassDesc), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(dhh, hh.data(), nho * sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(dhd, hd.data(), nho * sizeof(double), hipMemcpyHostToDevice));
    const int FB = 2048;
    for (int64_t c0 = 0; c0 < nho; c0 += FB) {
      const int nc = (int)std::min<int64_t>(FB, nho - c0);
      N.forward(nc, dX + (size_t)(ntr + c0) * nin, s);
      lk_sur_write(nc, dhc + c0, dhd + c0, st, N.y(nc), p, NC, mu, sd, Ipred, s);
    }
    lk_sur_err((int)nho, dhc, st, dhh, Ipred, Iref, p, NC, derr, s);
    std::vector<double> err(nho);
    HIPCHK(hipStreamSynchronize(s));
    HIPCHK(hipMemcpy(err.data(), derr, nho * sizeof(double), hipMemcpyDeviceToHost));
    std::vector<double> worst(S.bound.size(), -1.0);
    for (int64_t g = 0; g < nho; g++) {
      const int cb = sur_combo(ho[g].comp, ho[g].j, ho[g].i, ho[g].ri);
      worst[cb] = std::max(worst[cb], err[g]);
    }
    for (size_t cb = 0; cb < worst.size(); cb++)
      if (worst[cb] >= 0.0) S.bound[cb] = 2.0 * worst[cb];
    std::vector<double> se = err;
    std::sort(se.begin(), se.end());
    R.err_median = se[se.size() / 2];
    R.err_max = se.back();
  }
  for (const char* nm : {"T", "Iref", "Ich", "Ipred", "X", "xc", "xh", "idx", "xb", "tb", "hold_cls", "hold_h",
                         "hold_d", "hold_err"}) {
    auto it = N.bufs.find(nm);
    if (it != N.bufs.end()) {
      if (it->second.p) (void)hipFree(it->second.p);
      N.bufs.erase(it);
    }
  }
  S.trep = R;
  S.version++;
  S.ready = true;
}

// ---------------------------------------------------------------------------
// Pre-computed tables of the reaction M2L integrals (the tabulation of Section
// 3.5 and the table form of Algorithm 1, restricted to what a uniform tree asks
// for).  Every reaction class of an evaluation is a geometry combination (component,
// j, i, lateral class) at a box size h, its centres at heights (j + 1/2) h and
// (i + 1/2) h and lateral distance sqrt(r2) h: the paper's tables over (rho, z, z')
// are, along that curve, one table in h per combination.  Entries are normalised as
// the surrogate's targets (I / env) and interpolated in u = ln h + alpha h by the
// barycentric formula on Chebyshev points of the second kind.  Bounds: the largest
// weighted relative error (the surrogate's norm) over validation classes halfway
// (in angle) between nodes, against the quadrature, times two.
// ---------------------------------------------------------------------------
static std::vector<int4> component_labels(lfmm_plan_s* P) {
  const int NL = P->st.L + 1;
  std::vector<int4> lab(P->sur.ncomp);
  for (int l = 0; l < NL; l++)
    for (int a = 0; a < 2; a++)
      for (int lp = 0; lp < NL; lp++)
        for (int b = 0; b < 2; b++) {
          const int c = sur_comp(P, l, a, lp, b);
          if (c >= 0) lab[c] = make_int4(l, a, lp, b);
        }
  return lab;
}
static ClassDesc combo_class(lfmm_plan_s* P, const int4& lab, int j, int i, int ri, double h, int out) {
  ClassDesc C;
  memset(&C, 0, sizeof(C));
  C.zt = (j + 0.5) * h;
  C.zs = (i + 0.5) * h;
  C.rho = h * std::sqrt((double)kR2[ri]);
  C.rule = P->make_rule(C.zt + C.zs, C.rho, 2 * P->p + 1);
  C.lt = lab.x;
  C.a = lab.y;
  C.ls = lab.z;
  C.b = lab.w;
  C.out = out;
  return C;
}
inline double tab_u(const OpTables& T, double h) { return std::log(h) + T.alpha * h; }
// h of u: Newton on f(t) = t + alpha e^t - u (increasing, convex) from t = u, where
// f >= 0, so the iterates decrease monotonically to the root
static double tab_h(const OpTables& T, double u) {
  double t = u;
  for (int it = 0; it < 400; it++) {
    const double e = T.alpha * std::exp(t), f = t + e - u, dt = f / (1.0 + e);
    t -= dt;
    if (std::fabs(dt) <= 1e-15 * std::max(1.0, std::fabs(t))) break;
  }
  return std::exp(t);
}
inline double tab_node_x(int n, int j) { return std::cos(LFMM_PI * j / (n - 1)); }
// panel of h and the barycentric weights of its nodes (w[0..n-1], summing to 1);
// Chebyshev points of the second kind have the weights (-1)^j, halved at both ends
static int tab_weights(const OpTables& T, double h, double* w) {
  const int n = T.nnode;
  const double u = tab_u(T, h);
  int k = (int)std::floor((u - T.u0) / T.du);
  k = std::min(std::max(k, 0), T.npanel - 1);
  const double x = std::min(1.0, std::max(-1.0, 2.0 * (u - (T.u0 + k * T.du)) / T.du - 1.0));
  double sum = 0.0;
  for (int j = 0; j < n; j++) {
    const double xj = tab_node_x(n, j);
    if (x == xj) {
      for (int i = 0; i < n; i++) w[i] = i == j ? 1.0 : 0.0;
      return k;
    }
    w[j] = ((j & 1) ? -1.0 : 1.0) * ((j == 0 || j == n - 1) ? 0.5 : 1.0) / (x - xj);
    sum += w[j];
  }
  for (int j = 0; j < n; j++) w[j] /= sum;
  return k;
}
// node j of panel k -> x = cos(pi j / (n - 1)) -> u = u_k + (x + 1) du / 2
static double tab_node_h(const OpTables& T, int k, double x) {
  return tab_h(T, T.u0 + k * T.du + 0.5 * (x + 1.0) * T.du);
}

void tab_build_impl(lfmm_plan_s* P, const lfmm_table_opts& o, lfmm_table_report& R) {
  OpTables& T = P->tab;
  const Stack& st = P->st;
  const int p = P->p, NC = P->NC, NT = P->NT;
  hipStream_t s = P->s2;
  auto wall = []() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
  };
  T.release();
  sur_components(P);
  sur_decay(P);
  const int ncomp = P->sur.ncomp;
  const std::vector<int4> lab = component_labels(P);
  T.h_lo = o.h_min;
  T.h_hi = o.h_max;
  T.alpha = 4.0 * P->kmax;
  T.nnode = o.nnode;
  T.u0 = tab_u(T, T.h_lo);
  const double u1 = tab_u(T, T.h_hi);
  T.npanel = std::max(1, (int)std::ceil((u1 - T.u0) / o.du - 1e-9));
  T.du = (u1 - T.u0) / T.npanel;
  T.dense.assign((size_t)ncomp * 40, -1);
  T.bound.assign((size_t)ncomp * 40, INFINITY);
  struct Cmb {
    int comp, j, i, ri;
  };
  std::vector<Cmb> cmbs;
  for (int c = 0; c < ncomp; c++)
    for (int j = 0; j < 2; j++)
      for (int i = 0; i < 2; i++)
        for (int ri = 0; ri < 10; ri++) {
          if (i == 0 && j == 0 && kR2[ri] <= 2) continue;
          T.dense[sur_combo(c, j, i, ri)] = (int)cmbs.size();
          cmbs.push_back(Cmb{c, j, i, ri});
        }
  T.ndense = (int)cmbs.size();
  const size_t nh = (size_t)NT * NC, mat = (size_t)NC * NC * 2;
  const int64_t nslot = (int64_t)T.ndense * T.npanel * T.nnode;
  memset(&R, 0, sizeof(R));
  R.n_combos = T.ndense;
  R.npanel = T.npanel;
  R.nnode = T.nnode;
  R.n_slots = nslot;
  R.bytes = nslot * (int64_t)nh * 16;
  if (hipMalloc(&T.tab.p, (size_t)R.bytes) != hipSuccess) {
    T.tab.p = nullptr;
    throw Fail{LFMM_ENOMEM};
  }
  T.tab.cap = (size_t)R.bytes;
  double* tab = (double*)T.tab.p;
  const int CHK = 1024;
  double* Ich = P->dev<double>("tab_Ich", (size_t)CHK * mat);
  // ---- nodes: quadrature, normalised into their slots
  double t0 = wall();
  for (int64_t g0 = 0; g0 < nslot; g0 += CHK) {
    const int nc = (int)std::min<int64_t>(CHK, nslot - g0);
    HIPCHK(hipStreamSynchronize(s));
    P->pin_reset();
    std::vector<ClassDesc> cls(nc);
    std::vector<double> dadd(nc);
    std::vector<int> slot(nc);
    for (int c = 0; c < nc; c++) {
      const int64_t g = g0 + c;
      const int jn = (int)(g % T.nnode), k = (int)((g / T.nnode) % T.npanel), d = (int)(g / ((int64_t)T.nnode * T.npanel));
      const Cmb& m = cmbs[d];
      cls[c] = combo_class(P, lab[m.comp], m.j, m.i, m.ri, tab_node_h(T, k, tab_node_x(T.nnode, jn)), c);
      dadd[c] = P->sur.Dc[m.comp];
      slot[c] = (int)g;
    }
    reaction_integrals(P, "tab", cls, Ich, s);
    ClassDesc* dcls = P->upload("tab_cls", cls, s);
    double* dd = P->upload("tab_dadd", dadd, s);
    int* ds = P->upload("tab_slot", slot, s);
    lk_tab_store(nc, dcls, dd, ds, st, Ich, p, NC, tab, s);
  }
  HIPCHK(hipStreamSynchronize(s));
  R.ms_build = wall() - t0;
  // ---- validation halfway (in angle) between nodes, spread over each panel
  t0 = wall();
  const int nval = std::min(o.nval, T.nnode - 1);
  const int64_t nv = (int64_t)T.ndense * T.npanel * nval;
  R.n_validation = nv;
  std::vector<double> worst(T.bound.size(), -1.0), all;
  double* Ipred = P->dev<double>("tab_Ipred", (size_t)CHK * mat);
  double* derr = P->dev<double>("tab_err", CHK);
  for (int64_t g0 = 0; g0 < nv; g0 += CHK) {
    const int nc = (int)std::min<int64_t>(CHK, nv - g0);
    HIPCHK(hipStreamSynchronize(s));
    P->pin_reset();
    std::vector<ClassDesc> cls(nc);
    std::vector<double> dadd(nc), hv(nc), w((size_t)nc * T.nnode);
    std::vector<int> slot0(nc), cb(nc);
    for (int c = 0; c < nc; c++) {
      const int64_t g = g0 + c;
      const int v = (int)(g % nval), k = (int)((g / nval) % T.npanel), d = (int)(g / ((int64_t)nval * T.npanel));
      const int jv = nval > 1 ? (int)std::lround((double)v * (T.nnode - 2) / (nval - 1)) : (T.nnode - 2) / 2;
      const double x = std::cos(LFMM_PI * (jv + 0.5) / (T.nnode - 1));
      const Cmb& m = cmbs[d];
      hv[c] = tab_node_h(T, k, x);
      cls[c] = combo_class(P, lab[m.comp], m.j, m.i, m.ri, hv[c], c);
      dadd[c] = P->sur.Dc[m.comp];
      const int kk = tab_weights(T, hv[c], &w[(size_t)c * T.nnode]);
      slot0[c] = (d * T.npanel + kk) * T.nnode;
      cb[c] = sur_combo(m.comp, m.j, m.i, m.ri);
    }
    reaction_integrals(P, "tab", cls, Ich, s);
    ClassDesc* dcls = P->upload("tab_cls", cls, s);
    double* dd = P->upload("tab_dadd", dadd, s);
    int* ds = P->upload("tab_slot", slot0, s);
    double* dw = P->upload("tab_w", w, s);
    double* dh = P->upload("tab_h", hv, s);
    lk_tab_interp(nc, dcls, dd, ds, dw, T.nnode, st, tab, p, NC, Ipred, s);
    lk_sur_err(nc, dcls, st, dh, Ipred, Ich, p, NC, derr, s);
    std::vector<double> err(nc);
    HIPCHK(hipStreamSynchronize(s));
    HIPCHK(hipMemcpy(err.data(), derr, nc * sizeof(double), hipMemcpyDeviceToHost));
    for (int c = 0; c < nc; c++) {
      worst[cb[c]] = std::max(worst[cb[c]], err[c]);
      all.push_back(err[c]);
    }
  }
  for (size_t c = 0; c < worst.size(); c++)
    if (worst[c] >= 0.0) T.bound[c] = 2.0 * worst[c];
  if (!all.empty()) {
    std::sort(all.begin(), all.end());
    R.err_median = all[all.size() / 2];
    R.err_max = all.back();
  }
  R.ms_validate = wall() - t0;
  for (const char* nm : {"tab_Ich", "tab_Ipred", "tab_err"}) {
    auto it = P->bufs.find(nm);
    if (it != P->bufs.end()) {
      if (it->second.p) (void)hipFree(it->second.p);
      P->bufs.erase(it);
    }
  }
  T.rep = R;
  T.version++;
  T.ready = true;
}

struct Group {
  int seq0, K;
};

// Build the GEMM block table of one job from its sorted group ids and counts.
void build_blocks(const std::vector<int>& counts, const std::vector<Group>& groups, std::vector<GBlock>& blocks,
                  std::vector<int>& gstart, std::vector<int>& blk_first, std::vector<int>& blk_count,
                  const std::vector<int>& group_level, int nlev, int bsize) {
  int ng = (int)groups.size();
  gstart.assign(ng + 1, 0);
  for (int g = 0; g < ng; g++) gstart[g + 1] = gstart[g] + counts[g];
  blocks.clear();
  blk_first.assign(nlev, -1);
  blk_count.assign(nlev, 0);
  for (int g = 0; g < ng; g++) {
    int lv = group_level.empty() ? 0 : group_level[g];
    for (int e = gstart[g]; e < gstart[g + 1]; e += bsize) {
      GBlock b;
      b.e0 = e;
      b.nt = std::min(bsize, gstart[g + 1] - e);
      b.seq0 = groups[g].seq0;
      b.K = groups[g].K;
      if (blk_first[lv] < 0) blk_first[lv] = (int)blocks.size();
      blk_count[lv]++;
      blocks.push_back(b);
    }
  }
}

int eval_impl(lfmm_plan_t* P, int64_t n64, const double* xyz, const int32_t* layer_in, const double* q,
              double* phi, hipStream_t s) {
  if (!P || n64 < 0 || n64 >= (int64_t)1 << 31) return LFMM_EINVAL;
  if (n64 > 0 && (!xyz || (!P->prep_only && (!q || !phi)))) return LFMM_EINVAL;
  int n = (int)n64;
  lfmm_report& rep = P->rep;
  memset(&rep, 0, sizeof(rep));
  rep.precision = P->prec;
  (void)hipGetLastError();  // the launch check below is for this evaluation's own launches
  P->apply_list.clear();
  P->apply_ready = false;
  P->apply_n = n;
  P->apply_ntp = 0;
  if (n == 0) return LFMM_OK;
  // a charge-dependent launch: queued now (unless only preparing) and recorded
  const bool run_q = !P->prep_only;
  auto qrun = [&](std::function<void(hipStream_t, const double*, double*)> f) {
    if (run_q) f(s, q, phi);
    P->apply_list.push_back(std::move(f));
  };
  P->pin_reset();
  std::string prev_opsig;  // signature of the operators in the buffer (cleared until this evaluation succeeds)
  prev_opsig.swap(P->last_opsig);
  const Stack& st = P->st;
  const int L = st.L, NL = L + 1, p = P->p, NC = P->NC, NCK = P->NCK, NKS = P->NKS, opsz = P->opsz;
  const double* x = xyz;
  const double* y = xyz + n;
  const double* z = xyz + 2 * (size_t)n;
  bool prof = P->profile && P->ev_ok;
  // profile 2: only the stages of the kernels whose rates a benchmark reports (each
  // recorded event is a marker in its stream; on the main stream they cost about 0.1 ms
  // per evaluation at the bench workload)
  auto staged = [&](int i) {
    return prof && (P->profile != 2 || i == ST_M2L || i == ST_P2P || i == ST_REACT_MFMA || i == ST_P2M ||
                    i == ST_L2P);
  };
  auto sbeg = [&](int i, hipStream_t st_) {
    if (staged(i)) HIPCHK(hipEventRecord(P->evb[i], st_));
  };
  auto send = [&](int i, hipStream_t st_) {
    if (staged(i)) HIPCHK(hipEventRecord(P->eve[i], st_));
  };
  auto mark = [&](int i) {  // boundary between stages i-1 and i on the main stream
    if (i > 0) send(i - 1, s);
    if (i < ST_COUNT) sbeg(i, s);
  };
  hipStream_t s2 = P->s2;
  mark(0);
  // ---------------- classification and statistics
  int nbk = std::min(1024, (n + 255) / 256);
  double* partial = P->dev<double>("partial", (size_t)nbk * NL * LFMM_NSTAT);
  double* stats = P->dev<double>("stats", (size_t)NL * LFMM_NSTAT);
  int* layer = P->dev<int>("layer", n);
  lk_classify(n, x, y, z, layer_in, layer, st, partial, nbk, s);
  lk_reduce_stats(nbk, NL, partial, stats, s);
  std::vector<double> hs((size_t)NL * LFMM_NSTAT);
  P->rb_add(hs.data(), stats, hs.size() * sizeof(double), s);
  P->rb_flush(s);
  double bad = 0;
  for (int l = 0; l < NL; l++) bad += hs[l * LFMM_NSTAT + 11];
  if (bad > 0) return LFMM_EINVAL;
  std::vector<int> cnt(NL), layer_start(NL + 1, 0);
  for (int l = 0; l < NL; l++) {
    const double* S = &hs[l * LFMM_NSTAT];
    cnt[l] = (int)std::llround(S[0]);
    layer_start[l + 1] = layer_start[l] + cnt[l];
    if (cnt[l] > 0) {
      if (l <= L - 1 && S[7] < P->min_gap) return LFMM_EINVAL;
      if (l >= 1 && S[9] < P->min_gap) return LFMM_EINVAL;
    }
  }
  mark(1);
  // ---------------- trees
  std::vector<TreeInfo> trees;
  std::vector<int> free_tree(NL, -1);
  double xlo = INFINITY, xhi = -INFINITY, ylo = INFINITY, yhi = -INFINITY, H = 0;
  for (int l = 0; l < NL; l++) {
    if (cnt[l] == 0) continue;
    const double* S = &hs[l * LFMM_NSTAT];
    xlo = std::min(xlo, S[1]);
    xhi = std::max(xhi, S[2]);
    ylo = std::min(ylo, S[3]);
    yhi = std::max(yhi, S[4]);
    if (l <= L - 1) H = std::max(H, S[8]);
    if (l >= 1) H = std::max(H, S[10]);
    TreeInfo T;
    memset(&T, 0, sizeof(T));
    double ext[3] = {S[2] - S[1], S[4] - S[3], S[6] - S[5]};
    double Sd = std::max(ext[0], std::max(ext[1], ext[2]));
    if (Sd == 0.0) Sd = 1.0;
    T.lo[0] = 0.5 * (S[1] + S[2]) - 0.5 * Sd;
    T.lo[1] = 0.5 * (S[3] + S[4]) - 0.5 * Sd;
    T.lo[2] = 0.5 * (S[5] + S[6]) - 0.5 * Sd;
    T.S = Sd;
    T.k = st.k[l];
    T.kind = 0;
    T.layer = l;
    T.dir = 0;
    T.npts = cnt[l];
    free_tree[l] = (int)trees.size();
    trees.push_back(T);
  }
  double Sr = std::max(xhi - xlo, std::max(yhi - ylo, 2.0 * H));
  double rlox = 0.5 * (xlo + xhi) - 0.5 * Sr, rloy = 0.5 * (ylo + yhi) - 0.5 * Sr;
  std::vector<int> tgt_tree(2 * NL, -1), src_tree(2 * NL, -1);
  for (int kind = 1; kind <= 2 && L >= 1; kind++)
    for (int l = 0; l < NL; l++)
      for (int a = 0; a < 2; a++) {
        if (!has_dir(st, l, a) || cnt[l] == 0) continue;
        TreeInfo T;
        memset(&T, 0, sizeof(T));
        T.lo[0] = rlox;
        T.lo[1] = rloy;
        T.lo[2] = -0.5 * Sr;
        T.S = Sr;
        T.k = st.k[l];
        T.kind = kind;
        T.layer = l;
        T.dir = a;
        T.npts = cnt[l];
        (kind == 1 ? tgt_tree : src_tree)[2 * l + a] = (int)trees.size();
        trees.push_back(T);
      }
  int ntrees = (int)trees.size();
  int ntp = 0;
  for (auto& T : trees) {
    T.pt_off = ntp;
    T.depth = 8;
    ntp += T.npts;
  }
  rep.n_trees = ntrees;
  // ---------------- stable partition of the particles by layer
  int* perm = P->dev<int>("perm", n);
  int* inv_perm = P->dev<int>("inv_perm", n);
  const int nbl = (n + 255) / 256;
  int* lcnt = P->dev<int>("layer_cnt", (size_t)NL * nbl + 1);
  int* loff = P->dev<int>("layer_off", (size_t)NL * nbl + 1);
  if (n) {
    lk_layer_count(n, NL, layer, lcnt, s);
    int* ts1 = P->dev<int>("scan_ts1", lk_scan_tsum_size((long long)NL * nbl));
    lk_scan_excl(lcnt, (long long)NL * nbl, loff, ts1, s);
    lk_layer_scatter(n, NL, layer, loff, perm, inv_perm, s);
  }
  int* d_lstart = P->upload("layer_start", layer_start, s);
  TreeInfo* d_trees = P->upload("trees", trees, s);
  // ---------------- keys and sort
  unsigned* keys = P->dev<unsigned>("keys", ntp);
  unsigned* skeys = P->dev<unsigned>("skeys", ntp);
  int* vals = P->dev<int>("vals", ntp);
  int* sg = P->dev<int>("sg", ntp);
  double* rec = P->dev<double>("tp_rec", 5 * (size_t)ntp);
  lk_tree_points(ntp, ntrees, d_trees, perm, d_lstart, x, y, z, q, st, keys, vals, rec, s);
  if (ntrees > 96) throw Fail{LFMM_ENOTSUP};  // at most 5 L + 1 trees: never for L <= 16
  {
    // the points come grouped by tree (the key's top bits), so each tree's run is
    // sorted on its own on the 24 Morton bits
    std::vector<int> seg(ntrees + 1);
    for (int t = 0; t < ntrees; t++) seg[t] = trees[t].pt_off;
    seg[ntrees] = ntp;
    unsigned* ktmp = P->dev<unsigned>("keys_tmp", ntp);
    int* vtmp = P->dev<int>("vals_tmp", ntp);
    int* rsw = P->dev<int>("rs_scratch", (size_t)lk_radix_sort_scratch(ntp, ntrees));
    if (lk_radix_sort_segs(keys, vals, skeys, sg, ktmp, vtmp, ntp, ntrees, seg.data(), 24, 0xffffffffu, rsw, s))
      throw Fail{LFMM_ENOTSUP};  // more trees than segments (excluded above)
  }
  // fullest cell per (tree, level), then the slab flags: one fill, one readback
  int* occ = P->dev<int>("occ", ntrees * 27);
  int* slab = occ + ntrees * 9;
  lk_fill_int(occ, (size_t)ntrees * 27, 0, s);
  lk_occupancy(ntp, ntrees, skeys, d_trees, P->leaf_max, occ, slab, s);
  std::vector<int> hos(ntrees * 27);
  P->rb_add(hos.data(), occ, sizeof(int) * ntrees * 27, s);
  P->rb_mark(s);
  // particle data in sorted order (frame coordinates) and each tree point's particle:
  // they need only the sort, and run while the host reads the occupancy back
  double* px = P->dev<double>("px", ntp);
  double* py = P->dev<double>("py", ntp);
  double* pz = P->dev<double>("pz", ntp);
  double* pq = P->dev<double>("pq", 2 * (size_t)ntp);
  lk_gather(ntp, sg, rec, px, py, pz, pq, s);
  int* tp_orig = P->dev<int>("tp_orig", ntp);
  lk_point_origin(ntp, ntrees, d_trees, perm, d_lstart, sg, tp_orig, s);
  P->rb_wait();
  const std::vector<int> hocc(hos.begin(), hos.begin() + ntrees * 9), hslab(hos.begin() + ntrees * 9, hos.end());
  // depth rule: smallest depth whose fullest cell holds <= leaf_max points
  int Dr = -1;
  for (int t = 0; t < ntrees; t++) {
    int dmin = trees[t].kind == 0 ? 0 : 1;
    int D = P->max_depth;
    for (int l = dmin; l <= P->max_depth; l++)
      if (hocc[t * 9 + l] <= P->leaf_max) {
        D = l;
        break;
      }
    trees[t].depth = D;
    if (trees[t].kind != 0) Dr = std::max(Dr, D);
  }
  if (Dr >= 0) {
    // and deep enough that the finest boxes are no thicker than the smallest
    // particle-to-interface distance, so that (within the depth limit) no target
    // and no polarisation image share the two boxes next to the interface and the
    // reaction near field is empty
    double gmin = INFINITY;
    for (int l = 0; l < NL; l++) {
      const double* S = &hs[(size_t)l * LFMM_NSTAT];
      if (S[0] <= 0) continue;
      if (l <= L - 1) gmin = std::min(gmin, S[7]);
      if (l >= 1) gmin = std::min(gmin, S[9]);
    }
    int Dg = 1;
    while (Dg < P->max_depth && Sr / (double)(1 << Dg) > gmin) Dg++;
    Dr = std::max(Dr, Dg);
  }
  for (int t = 0; t < ntrees; t++)
    if (trees[t].kind != 0) trees[t].depth = Dr;
  int Dmax = 0;
  for (auto& T : trees) Dmax = std::max(Dmax, T.depth);
  for (int l = 0; l < 17; l++) rep.free_depth[l] = -1;
  for (int l = 0; l < NL && l < 17; l++)
    if (free_tree[l] >= 0) rep.free_depth[l] = trees[free_tree[l]].depth;
  rep.reaction_depth = Dr;
  d_trees = P->upload("trees", trees, s);
  // ---------------- boxes
  int nlev = Dmax + 1;
  const int nbt = lk_box_tiles(ntp);
  int* box_tcnt = P->dev<int>("box_tcnt", (size_t)nlev * nbt + 1);
  int* box_toff = P->dev<int>("box_toff", (size_t)nlev * nbt + 1);
  int* tb = P->dev<int>("tb", ntrees * 18);  // every entry written by lk_tree_box_range_all
  // boxes opened per tile and level, one scan over all levels (global box rows), box ranges
  if ((size_t)nlev * ntp >= ((size_t)1 << 31)) throw Fail{LFMM_ENOTSUP};
  int* ts3 = P->dev<int>("scan_ts3", lk_scan_tsum_size((long long)nlev * nbt + 1));
  if (ntp) {
    lk_box_count(ntp, nlev, skeys, d_trees, box_tcnt, s);
    lk_scan_excl(box_tcnt, (long long)nlev * nbt + 1, box_toff, ts3, s);
  }
  lk_tree_box_range_all(ntrees, nlev, ntp, skeys, d_trees, box_toff, tb, s);
  std::vector<int> htb(ntrees * 18);
  P->rb_add(htb.data(), tb, sizeof(int) * ntrees * 18, s);
  P->rb_flush(s);
  std::vector<int> lvl_count(9, 0), lvl_off(10, 0);
  for (int l = 0; l < nlev; l++)
    for (int t = 0; t < ntrees; t++) lvl_count[l] += htb[(t * 9 + l) * 2 + 1];
  for (int l = 0; l < 9; l++) lvl_off[l + 1] = lvl_off[l] + lvl_count[l];
  int NR = lvl_off[nlev];
  rep.n_boxes = NR;
  auto first_row = [&](int t, int l) { return lvl_off[l] + htb[(t * 9 + l) * 2]; };
  auto nbox = [&](int t, int l) { return htb[(t * 9 + l) * 2 + 1]; };
  int* box_start = P->dev<int>("box_start", NR + 1);
  int* box_code = P->dev<int>("box_code", NR + 1);
  int* box_tree = P->dev<int>("box_tree", NR + 1);
  int* box_level = P->dev<int>("box_level", NR + 1);
  int* box_cnt = P->dev<int>("box_cnt", NR + 1);
  int* leafrow = P->dev<int>("leafrow", ntp);
  lk_box_fill_all(ntp, nlev, skeys, box_toff, d_trees, box_start, box_code, box_tree, box_level, leafrow, s);
  // dense cell -> row grids
  std::vector<long long> grid_off(ntrees * 9, -1);
  long long gtot = 0;
  for (int t = 0; t < ntrees; t++)
    for (int l = 0; l <= trees[t].depth; l++) {
      grid_off[t * 9 + l] = gtot;
      gtot += 1LL << (3 * l);
    }
  int* grid = P->dev<int>("grid", (size_t)gtot);
  lk_fill_int(grid, (size_t)gtot, -1, s);
  long long* d_grid_off = P->upload("grid_off", grid_off, s);
  lk_grid_fill_all(NR, box_start, box_code, box_tree, box_level, d_trees, d_grid_off, grid, box_cnt, s);
  P->apply_ntp = ntp;
  P->apply_orig = tp_orig;
  P->apply_pq = pq;
  send(ST_TREE, s);
  // the operator stream (and the job stream) may start from here: everything the
  // operator stream reads is uploaded on it ahead of its kernels (copies of all
  // streams share one DMA queue, so an upload queued behind its kernels would hold
  // up the other streams' later ones)
  unsigned long long* d_cnt = P->dev<unsigned long long>("pair_counts", 4);
  HIPCHK(hipMemsetAsync(d_cnt, 0, sizeof(unsigned long long) * 4, s));
  HIPCHK(hipEventRecord(P->fork_ev, s));
  HIPCHK(hipStreamWaitEvent(s2, P->fork_ev, 0));
  const bool m2l32 = P->prec && (P->prec_parts & 2), p2p32 = P->prec && (P->prec_parts & 1);
  // ---------------- P2M needs the trees only: it goes first and keeps the GPU busy
  // while the host builds the operator tables
  double* M = P->dev<double>("M", (size_t)NR * NCK * 2);
  double* Lx = P->dev<double>("L", (size_t)NR * NCK * 2);
  qrun([=](hipStream_t ss, const double*, double*) {
    lk_zero(M, (size_t)NR * NCK * 2, ss);
    lk_zero(Lx, (size_t)NR * NCK * 2, ss);
  });
  // leaf segments of trees with a far field
  std::vector<int> seg_row0, seg_prefix;
  int ptot = 0;
  for (int t = 0; t < ntrees; t++) {
    const TreeInfo& T = trees[t];
    if ((T.kind == 0 || T.kind == 2) && T.depth >= 2) {
      seg_row0.push_back(first_row(t, T.depth));
      seg_prefix.push_back(ptot);
      ptot += nbox(t, T.depth);
      rep.p2m_points += T.npts;
    }
  }
  rep.p2m_leaves = ptot;
  sbeg(ST_P2M, s);
  if (ptot) {
    int* d_r0 = P->upload("p2m_r0", seg_row0, s);
    int* d_pf = P->upload("p2m_pf", seg_prefix, s);
    const int nseg = (int)seg_row0.size();
    qrun([=](hipStream_t ss, const double*, double*) {
      lk_p2m(nseg, d_r0, d_pf, ptot, box_start, box_cnt, box_code, box_tree, box_level, d_trees, px, py, pz, pq, p,
             NCK, M, ss);
    });
  }
  send(ST_P2M, s);
  // the free-space near field, right after the P2M: the main stream is then busy while
  // the host builds the operator tables
  double* phi_tp = P->dev<double>("phi_tp", 2 * (size_t)ntp);
  qrun([=](hipStream_t ss, const double*, double*) { lk_zero(phi_tp, 2 * (size_t)ntp, ss); });
  // ---------------- free-space near field (its stage brackets the kernel alone)
  {
    std::vector<int> r0, pf;
    int tot = 0;
    double krmax = 0.0;  // bound on k r over adjacent leaves: the diagonal of two boxes side by side
    for (int t = 0; t < ntrees; t++) {
      const TreeInfo& T = trees[t];
      if (T.kind != 0) continue;
      r0.push_back(first_row(t, T.depth));
      pf.push_back(tot);
      tot += nbox(t, T.depth);
      double h = T.S / (double)(1 << T.depth);
      krmax = std::max(krmax, T.k * 2.0 * h * std::sqrt(3.0));
    }
    if (tot) {
      int* d_r0 = P->upload("p2p_r0", r0, s);
      int* d_pf = P->upload("p2p_pf", pf, s);
      // the series form where k r <= 1 on every pair, shorter series where k r <= 1/2
      rep.p2p_series = krmax <= 0.5 ? 2 : (krmax <= 1.0 ? 1 : 0);
      const int series = rep.p2p_series;
      sbeg(ST_P2P, s);
      const int nr0 = (int)r0.size(), ta = P->p2p_ta, ch = P->p2p_ch, f32 = p2p32 ? 1 : 0;
      unsigned long long* cnt3 = d_cnt + 3;
      qrun([=](hipStream_t ss, const double*, double*) {
        lk_p2p_free(nr0, d_r0, d_pf, tot, box_start, box_cnt, box_code, box_tree, box_level, d_trees, d_grid_off, grid,
                    px, py, pz, pq, sg, phi_tp, series, ta, ch, f32, cnt3, ss);
      });
    } else {
      sbeg(ST_P2P, s);
    }
    send(ST_P2P, s);
  }
  // ---------------- operators
  // expansion scale exponents of the mixed-precision M2L: c = 2^e, e = round(log2(1/(k h))) per (tree, level)
  std::vector<int> hse((size_t)ntrees * 9, 0);
  for (int t = 0; t < ntrees; t++)
    for (int l = 0; l <= trees[t].depth && l < 9; l++) {
      double h = trees[t].S / (double)(1 << l);
      hse[(size_t)t * 9 + l] = (int)std::lround(std::log2(1.0 / (trees[t].k * h)));
    }
  auto scl = [&](int t, int l) { return hse[(size_t)t * 9 + l]; };
  std::vector<int> opse;  // (e_target, e_source) per operator (M2L operators only)
  auto set_opsc = [&](int op, int et, int es) {
    if ((size_t)(2 * op + 2) > opse.size()) opse.resize(2 * (size_t)op + 2, 0);
    opse[2 * (size_t)op] = et;
    opse[2 * (size_t)op + 1] = es;
  };
  // M2L operators (free and reaction) and shift operators (M2M, L2L) are numbered
  // separately, each array with the zero operator at index 0
  int nops = 1, nsh = 1;
  std::vector<OpDesc> fops;
  std::vector<int> m2l_op((size_t)ntrees * 9 * 343, 0), m2m_op((size_t)ntrees * 9 * 8, 0),
      l2l_op((size_t)ntrees * 9 * 8, 0);
  for (int t = 0; t < ntrees; t++) {
    const TreeInfo& T = trees[t];
    int D = T.depth;
    for (int l = 2; l <= D; l++) {
      double h = T.S / (double)(1 << l);
      if (T.kind == 0)
        for (int o = 0; o < 343; o++) {
          int dx = o / 49 - 3, dy = (o / 7) % 7 - 3, dz = o % 7 - 3;
          if (std::abs(dx) <= 1 && std::abs(dy) <= 1 && std::abs(dz) <= 1) continue;
          OpDesc od{dx * h, dy * h, dz * h, T.k, 1, nops};
          set_opsc(nops, scl(t, l), scl(t, l));
          m2l_op[((size_t)t * 9 + l) * 343 + o] = nops++;
          fops.push_back(od);
        }
      if (l >= 3)
        for (int ch = 0; ch < 8; ch++) {
          double cx = (((ch >> 2) & 1) - 0.5) * h, cy = (((ch >> 1) & 1) - 0.5) * h, cz = ((ch & 1) - 0.5) * h;
          if (T.kind == 0 || T.kind == 2) {  // M2M: b = parent - child
            OpDesc od{-cx, -cy, -cz, T.k, 0, nsh};
            m2m_op[((size_t)t * 9 + l) * 8 + ch] = nsh++;
            fops.push_back(od);
          }
          if (T.kind == 0 || T.kind == 1) {  // L2L: b = child - parent
            OpDesc od{cx, cy, cz, T.k, 0, nsh};
            l2l_op[((size_t)t * 9 + l) * 8 + ch] = nsh++;
            fops.push_back(od);
          }
        }
    }
  }
  rep.n_ops_free = (int64_t)fops.size();
  // reaction M2L classes and operators
  std::vector<ClassDesc> classes;
  std::vector<int4> cls_meta;  // (j, i, r2 class) of each class
  std::vector<double> cls_h;   // its box size
  std::vector<ROpDesc> rops;
  // rop index: [tt][ts][l][j][i][dx+3][dy+3] (0 = the zero operator); kept by the
  // plan, and only the entries the previous evaluation wrote are cleared
  const size_t nrop_keys = (size_t)ntrees * ntrees * 9 * 2 * 2 * 49;
  if (P->rop_idx.size() < nrop_keys) {
    P->rop_idx.assign(nrop_keys, 0);
    P->rop_dirty.clear();
  }
  for (size_t k : P->rop_dirty) P->rop_idx[k] = 0;
  P->rop_dirty.clear();
  std::vector<int>& rop_id = P->rop_idx;
  auto rkey = [&](int tt, int ts, int l, int j, int i, int dx, int dy) {
    return (((((size_t)tt * ntrees + ts) * 9 + l) * 2 + j) * 2 + i) * 49 + (size_t)(dx + 3) * 7 + (dy + 3);
  };
  const int r2vals[10] = {0, 1, 2, 4, 5, 8, 9, 10, 13, 18};
  int64_t nodes_total = 0;
  if (L >= 1)
    for (int l = 0; l < NL; l++)
      for (int a = 0; a < 2; a++) {
        int tt = tgt_tree[2 * l + a];
        if (tt < 0) continue;
        for (int lp = 0; lp < NL; lp++)
          for (int b = 0; b < 2; b++) {
            int ts = src_tree[2 * lp + b];
            if (ts < 0) continue;
            for (int lv = 2; lv <= Dr; lv++) {
              double h = Sr / (double)(1 << lv);
              for (int j = 0; j < 2; j++) {
                if (!hslab[(tt * 9 + lv) * 2 + j]) continue;
                for (int i = 0; i < 2; i++) {
                  if (!hslab[(ts * 9 + lv) * 2 + i]) continue;
                  int cls_of_r2[19];
                  for (int r = 0; r < 19; r++) cls_of_r2[r] = -1;
                  for (int ri = 0; ri < 10; ri++) {
                    int r2 = r2vals[ri];
                    if (i == 0 && j == 0 && r2 <= 2) continue;
                    ClassDesc C;
                    memset(&C, 0, sizeof(C));
                    C.zt = (j + 0.5) * h;
                    C.zs = (i + 0.5) * h;
                    C.rho = h * std::sqrt((double)r2);
                    C.rule = P->make_rule(C.zt + C.zs, C.rho, 2 * p + 1);
                    C.lt = l;
                    C.ls = lp;
                    C.a = a;
                    C.b = b;
                    C.out = (int)classes.size();
                    nodes_total += rule_nodes(C.rule);
                    cls_of_r2[r2] = C.out;
                    classes.push_back(C);
                    cls_meta.push_back(make_int4(j, i, ri, 0));
                    cls_h.push_back(h);
                  }
                  for (int dx = -3; dx <= 3; dx++)
                    for (int dy = -3; dy <= 3; dy++) {
                      if (i == 0 && j == 0 && std::abs(dx) <= 1 && std::abs(dy) <= 1) continue;
                      ROpDesc R;
                      R.dx = dx * h;
                      R.dy = dy * h;
                      R.kt = st.k[l];
                      R.cls = cls_of_r2[dx * dx + dy * dy];
                      set_opsc(nops, scl(tt, lv), scl(ts, lv));
                      R.op = nops++;
                      rop_id[rkey(tt, ts, lv, j, i, dx, dy)] = R.op;
                      P->rop_dirty.push_back(rkey(tt, ts, lv, j, i, dx, dy));
                      rops.push_back(R);
                    }
                }
              }
            }
          }
      }
  rep.n_react_classes = (int64_t)classes.size();
  rep.n_react_nodes = nodes_total;
  rep.n_ops_react = (int64_t)rops.size();
  // every operator in the GEMMs' k-step-major layout: shift operators in FP64, M2L
  // operators in FP32 on the mixed path and FP64 otherwise
  const int opsz_m = 2 * NKS * (m2l_nrt(NC) * 64 + 4 * m2l_xr(NC));
  double* sops = P->dev<double>("sops", (size_t)nsh * opsz_m);
  double* ops = m2l32 ? nullptr : P->dev<double>("ops", (size_t)nops * opsz_m);
  float* ops32 = nullptr;
  int* d_opsc = nullptr;
  int* d_sc = P->upload("exp_scale", hse, s);
  if (m2l32) {
    ops32 = P->dev<float>("ops32", (size_t)nops * opsz_m);
    opse.resize(2 * (size_t)nops, 0);
    d_opsc = P->upload("op_scale", opse, s2);
  }
  // gates: classes whose combination the pre-computed tables, else the surrogate,
  // give within its tolerance take those integrals, the others the quadrature's
  std::vector<ClassDesc> qcls, scls, tcls;
  std::vector<int> sC, tSlot;
  std::vector<double> sH, sD, tW, tD;
  const bool use_sur = P->sur.ready && P->sur.tol > 0.0 && !classes.empty();
  const bool use_tab = P->tab.ready && P->tab.tol > 0.0 && !classes.empty();
  if (use_sur || use_tab) {
    const Surrogate& S = P->sur;
    const OpTables& T = P->tab;
    for (size_t c = 0; c < classes.size(); c++) {
      const ClassDesc& C = classes[c];
      const int comp = sur_comp(P, C.lt, C.a, C.ls, C.b);
      const int j = cls_meta[c].x, i = cls_meta[c].y, ri = cls_meta[c].z;
      const double h = cls_h[c];
      const int cb = comp >= 0 ? sur_combo(comp, j, i, ri) : -1;
      if (use_tab && cb >= 0 && h >= T.h_lo && h <= T.h_hi && T.dense[cb] >= 0 && T.bound[cb] <= T.tol) {
        tcls.push_back(C);
        const size_t w0 = tW.size();
        tW.resize(w0 + T.nnode);
        const int k = tab_weights(T, h, &tW[w0]);
        tSlot.push_back((T.dense[cb] * T.npanel + k) * T.nnode);
        tD.push_back(S.Dc[comp]);
      } else if (use_sur && cb >= 0 && h >= S.h_lo && h <= S.h_hi && S.bound[cb] <= S.tol) {
        scls.push_back(C);
        sC.push_back(cb);
        sH.push_back(h);
        sD.push_back(S.Dc[comp]);
      } else {
        qcls.push_back(C);
      }
    }
  }
  std::vector<ClassDesc>& qref = (use_sur || use_tab) ? qcls : classes;
  rep.n_react_surrogate = (int64_t)scls.size();
  rep.n_react_table = (int64_t)tcls.size();
  // operators of the previous evaluation are kept when the plan asks for it and
  // everything they are generated from is the same (trees, classes, precision,
  // surrogate gate, buffers); a failed evaluation leaves no signature behind
  std::string opsig;
  if (P->reuse_ops) {
    auto app = [&](const void* q, size_t nb) { opsig.append((const char*)q, nb); };
    app(fops.data(), fops.size() * sizeof(OpDesc));
    app(classes.data(), classes.size() * sizeof(ClassDesc));
    app(rops.data(), rops.size() * sizeof(ROpDesc));
    app(opse.data(), opse.size() * sizeof(int));
    const int fl[7] = {P->prec, P->prec_parts, (int)scls.size(), P->physical, (int)tcls.size(), P->sur.version,
                       P->tab.version};
    app(fl, sizeof(fl));
    app(&P->sur.tol, sizeof(double));
    app(&P->tab.tol, sizeof(double));
    app(&ops, sizeof(ops));
    app(&ops32, sizeof(ops32));
    app(&sops, sizeof(sops));
  }
  const bool reuse = P->reuse_ops && P->bufp == &P->bufs && !prev_opsig.empty() && opsig == prev_opsig;
  rep.ops_reused = reuse ? 1 : 0;
  if (reuse) {
    for (int st_i : {ST_OPS_FREE, ST_REACT_TABLES, ST_REACT_MFMA, ST_REACT_SUR, ST_REACT_TAB, ST_REACT_EXPAND}) {
      sbeg(st_i, s2);
      send(st_i, s2);
    }
    HIPCHK(hipEventRecord(P->ops_ev, s2));
  } else {
    // the operator stream: its uploads, then free-space operators (the main stream
    // waits for them before the M2M), then the reaction chain (joined before the M2L)
    OpDesc* d_fops = P->upload("fops", fops, s2);
    RIPrep rip = reaction_prep(P, "ri", qref, s2);
    // reaction operators grouped by class (counting sort, stable): one expansion
    // workgroup per class
    std::vector<ROpDesc> rops_c(rops.size());
    std::vector<int> rgrp;
    if (!classes.empty()) {
      std::vector<int> ccnt(classes.size() + 1, 0);
      for (const ROpDesc& R : rops) ccnt[R.cls + 1]++;
      for (size_t c = 0; c < classes.size(); c++) {
        if (ccnt[c + 1] > 8) throw Fail{LFMM_ENOTSUP};  // (a class has at most 8 lateral offsets)
        if (ccnt[c + 1] > 0) {
          rgrp.push_back(ccnt[c]);
          rgrp.push_back(ccnt[c + 1]);
        }
        ccnt[c + 1] += ccnt[c];
      }
      std::vector<int> pos(ccnt.begin(), ccnt.end() - 1);
      for (const ROpDesc& R : rops) rops_c[pos[R.cls]++] = R;
    }
    ROpDesc* d_rops = classes.empty() ? nullptr : P->upload("rops", rops_c, s2);
    int* d_rgrp = rgrp.empty() ? nullptr : P->upload("rop_groups", rgrp, s2);
    ClassDesc* d_gcls = nullptr;
    int* d_gcombo = nullptr;
    double *d_gh = nullptr, *d_gd = nullptr;
    if (!scls.empty()) {
      d_gcls = P->upload("gate_cls", scls, s2);
      d_gcombo = P->upload("gate_combo", sC, s2);
      d_gh = P->upload("gate_h", sH, s2);
      d_gd = P->upload("gate_d", sD, s2);
    }
    ClassDesc* d_tcls = nullptr;
    int* d_tslot = nullptr;
    double *d_tw = nullptr, *d_td = nullptr;
    if (!tcls.empty()) {
      d_tcls = P->upload("tab_gcls", tcls, s2);
      d_tslot = P->upload("tab_gslot", tSlot, s2);
      d_tw = P->upload("tab_gw", tW, s2);
      d_td = P->upload("tab_gd", tD, s2);
    }
    double* Iall = classes.empty() ? nullptr : P->dev<double>("Iall", classes.size() * (size_t)NC * NC * 2);
    lk_zero(sops, opsz_m, s2);  // operator 0 of both arrays: the zero operator
    if (m2l32) lk_zero((double*)ops32, opsz_m / 2, s2);
    else lk_zero(ops, opsz_m, s2);
    sbeg(ST_OPS_FREE, s2);
    lk_transop((int)fops.size(), d_fops, sops, opsz_m, ops, opsz_m, p, NC, NKS, P->d_gaunt, ops32, d_opsc, s2);
    send(ST_OPS_FREE, s2);
    HIPCHK(hipEventRecord(P->ops_ev, s2));
    sbeg(ST_REACT_TABLES, s2);
    if (!classes.empty()) {
      if (!qref.empty()) {
        reaction_launch(P, rip, Iall, s2, [&]() {
          send(ST_REACT_TABLES, s2);
          sbeg(ST_REACT_MFMA, s2);
        });
      } else {
        send(ST_REACT_TABLES, s2);
        sbeg(ST_REACT_MFMA, s2);
      }
      send(ST_REACT_MFMA, s2);
      sbeg(ST_REACT_SUR, s2);
      if (!scls.empty()) {
        MlpNet& Nn = P->sur.net;
        const int ns = (int)scls.size();
        unsigned short* d_sx = P->dev<unsigned short>("gate_x", (size_t)ns * Nn.nin);
        const Surrogate& S = P->sur;
        lk_sur_features(ns, d_gcombo, d_gh, Nn.nin, S.ncomp * 40, std::log(S.h_lo), std::log(S.h_hi), d_sx, s2);
        Nn.forward(ns, d_sx, s2);
        lk_sur_write(ns, d_gcls, d_gd, st, Nn.y(ns), p, NC, Nn.dev<float>("mu", Nn.nout), Nn.dev<float>("sd", Nn.nout),
                     Iall, s2);
      }
      send(ST_REACT_SUR, s2);
      sbeg(ST_REACT_TAB, s2);
      if (!tcls.empty())
        lk_tab_interp((int)tcls.size(), d_tcls, d_td, d_tslot, d_tw, P->tab.nnode, st, (const double*)P->tab.tab.p, p,
                      NC, Iall, s2);
      send(ST_REACT_TAB, s2);
      sbeg(ST_REACT_EXPAND, s2);
      lk_react_expand((int)rgrp.size() / 2, d_rgrp, d_rops, Iall, ops, opsz_m, p, NC, NKS, ops32, d_opsc, s2);
    } else {
      send(ST_REACT_TABLES, s2);
      sbeg(ST_REACT_MFMA, s2);
      send(ST_REACT_MFMA, s2);
      sbeg(ST_REACT_SUR, s2);
      send(ST_REACT_SUR, s2);
      sbeg(ST_REACT_TAB, s2);
      send(ST_REACT_TAB, s2);
      sbeg(ST_REACT_EXPAND, s2);
    }
  }
  send(ST_REACT_EXPAND, s2);
  HIPCHK(hipEventRecord(P->join_ev, s2));
  // ---------------- GEMM jobs, on a third stream (they need the trees only, and
  // their count readbacks then wait for the job kernels alone, not for the near field)
  hipStream_t sj = P->s3;
  HIPCHK(hipStreamWaitEvent(sj, P->fork_ev, 0));
  sbeg(ST_JOBS, sj);
  // group tables (host): M2M groups per (tree, parent level), level-major descending;
  // L2L groups per (tree, level, class) level-major ascending; M2L groups per (tree, level, class)
  std::vector<int> gb_m2m(ntrees * 9, -1), gb_l2l(ntrees * 9, -1), gb_m2l(ntrees * 9, -1);
  std::vector<Group> g_m2m, g_l2l, g_m2l;
  std::vector<int> lv_m2m, lv_l2l;
  std::vector<int> seq_m2m, seq_l2l, seq_m2l;
  std::vector<Tmpl> tmpl_m2l;
  for (int lp = Dmax - 1; lp >= 2; lp--)
    for (int t = 0; t < ntrees; t++) {
      const TreeInfo& T = trees[t];
      if (!(T.kind == 0 || T.kind == 2) || lp + 1 > T.depth) continue;
      gb_m2m[t * 9 + lp] = (int)g_m2m.size();
      Group G{(int)seq_m2m.size(), 8};
      for (int ch = 0; ch < 8; ch++) seq_m2m.push_back(m2m_op[((size_t)t * 9 + lp + 1) * 8 + ch]);
      g_m2m.push_back(G);
      lv_m2m.push_back(lp);
    }
  for (int l = 3; l <= Dmax; l++)
    for (int t = 0; t < ntrees; t++) {
      const TreeInfo& T = trees[t];
      if (!(T.kind == 0 || T.kind == 1) || l > T.depth) continue;
      gb_l2l[t * 9 + l] = (int)g_l2l.size();
      for (int c = 0; c < 8; c++) {
        Group G{(int)seq_l2l.size(), 1};
        seq_l2l.push_back(l2l_op[((size_t)t * 9 + l) * 8 + c]);
        g_l2l.push_back(G);
        lv_l2l.push_back(l);
      }
    }
  int kmax_m2l = 1;
  for (int t = 0; t < ntrees; t++) {
    const TreeInfo& T = trees[t];
    if (T.kind == 2) continue;
    for (int l = 2; l <= T.depth; l++) {
      gb_m2l[t * 9 + l] = (int)g_m2l.size();
      for (int c = 0; c < 8; c++) {
        Group G{(int)seq_m2l.size(), 0};
        if (T.kind == 0) {
          int cx = (c >> 2) & 1, cy = (c >> 1) & 1, cz = c & 1;
          for (int dx = -3 + cx; dx <= 2 + cx; dx++)
            for (int dy = -3 + cy; dy <= 2 + cy; dy++)
              for (int dz = -3 + cz; dz <= 2 + cz; dz++) {
                if (std::abs(dx) <= 1 && std::abs(dy) <= 1 && std::abs(dz) <= 1) continue;
                int o = (dx + 3) * 49 + (dy + 3) * 7 + (dz + 3);
                Tmpl tm;
                tm.op = m2l_op[((size_t)t * 9 + l) * 343 + o];
                tm.stree = t;
                tm.dx = (short)dx;
                tm.dy = (short)dy;
                tm.dz = (short)dz;
                tm.zabs = 0;
                tmpl_m2l.push_back(tm);
                seq_m2l.push_back(tm.op);
                G.K++;
              }
        } else {
          int j = c >> 2, cx = (c >> 1) & 1, cy = c & 1;
          if (hslab[(t * 9 + l) * 2 + j])
            for (int lp = 0; lp < NL; lp++)
              for (int b = 0; b < 2; b++) {
                int ts = src_tree[2 * lp + b];
                if (ts < 0) continue;
                for (int i = 0; i < 2; i++) {
                  if (!hslab[(ts * 9 + l) * 2 + i]) continue;
                  for (int dx = -3 + cx; dx <= 2 + cx; dx++)
                    for (int dy = -3 + cy; dy <= 2 + cy; dy++) {
                      if (i == 0 && j == 0 && std::abs(dx) <= 1 && std::abs(dy) <= 1) continue;
                      Tmpl tm;
                      tm.op = rop_id[rkey(t, ts, l, j, i, dx, dy)];
                      tm.stree = ts;
                      tm.dx = (short)dx;
                      tm.dy = (short)dy;
                      tm.dz = (short)((1 << (l - 1)) - 1 - i);
                      tm.zabs = 1;
                      tmpl_m2l.push_back(tm);
                      seq_m2l.push_back(tm.op);
                      G.K++;
                    }
                }
              }
        }
        kmax_m2l = std::max(kmax_m2l, G.K);
        g_m2l.push_back(G);
      }
    }
  }
  // device: group ids for every box row, sort, count
  struct JobDev {
    int* gid;
    int* rowid;
    int* sgid;
    int* srowid;
    int* cnt;
  };
  auto job_prep = [&](const char* tag, int mode, const std::vector<int>& gbase, int ngroups, JobDev& J) {
    std::string t(tag);
    J.gid = P->dev<int>((t + "_gid").c_str(), NR + 1);
    J.rowid = P->dev<int>((t + "_row").c_str(), NR + 1);
    J.sgid = P->dev<int>((t + "_sgid").c_str(), NR + 1);
    J.srowid = P->dev<int>((t + "_srow").c_str(), NR + 1);
    J.cnt = P->dev<int>((t + "_cnt").c_str(), ngroups + 1);
    int* d_gb = P->upload((t + "_gb").c_str(), gbase, sj);
    lk_group_ids(NR, 0, mode, box_code, box_tree, box_level, d_trees, d_gb, 9, J.gid, J.rowid, sj);
    // sort keys: group ids (M2L: group * M2L_BCLS + boundary class); rows in no group
    // carry 0x7fffffff and sort as the largest key
    const long long kend = mode == 2 ? (long long)ngroups * M2L_BCLS : (long long)ngroups;
    int nbits = 1;
    while ((1LL << nbits) <= kend) nbits++;
    unsigned* kt = P->dev<unsigned>((t + "_ktmp").c_str(), NR + 1);
    int* vt = P->dev<int>((t + "_vtmp").c_str(), NR + 1);
    int* rsw = P->dev<int>((t + "_rs").c_str(), (size_t)lk_radix_sort_scratch(NR, 1));
    lk_radix_sort_pairs((const unsigned*)J.gid, J.rowid, (unsigned*)J.sgid, J.srowid, kt, vt, NR, nbits,
                        (unsigned)((1LL << nbits) - 1), rsw, sj);
    if (mode == 2) lk_m2l_key_to_group(NR, J.sgid, sj);
    // sizes of the groups
    lk_fill_int(J.cnt, ngroups + 1, 0, sj);
    lk_hist_ids(J.sgid, NR, ngroups, J.cnt, sj);
  };
  JobDev J_m2m{}, J_l2l{}, J_m2l{};
  int ng_m2m = (int)g_m2m.size(), ng_l2l = (int)g_l2l.size(), ng_m2l = (int)g_m2l.size();
  if (ng_m2m) job_prep("m2m", 0, gb_m2m, ng_m2m, J_m2m);
  if (ng_l2l) job_prep("l2l", 1, gb_l2l, ng_l2l, J_l2l);
  if ((int64_t)ng_m2l * M2L_BCLS >= 0x7fffffff) throw Fail{LFMM_ENOTSUP};
  if (ng_m2l) job_prep("m2l", 2, gb_m2l, ng_m2l, J_m2l);
  std::vector<int> c_m2m(ng_m2m + 1), c_l2l(ng_l2l + 1), c_m2l(ng_m2l + 1);
  if (ng_m2m) P->rb_add(c_m2m.data(), J_m2m.cnt, sizeof(int) * ng_m2m, sj);
  if (ng_l2l) P->rb_add(c_l2l.data(), J_l2l.cnt, sizeof(int) * ng_l2l, sj);
  if (ng_m2l) P->rb_add(c_m2l.data(), J_m2l.cnt, sizeof(int) * ng_m2l, sj);
  P->rb_flush(sj);
  c_m2m.resize(ng_m2m);
  c_l2l.resize(ng_l2l);
  c_m2l.resize(ng_m2l);
  std::vector<GBlock> b_m2m, b_l2l, b_m2l;
  std::vector<int> gs_m2m, gs_l2l, gs_m2l, bf_m2m, bc_m2m, bf_l2l, bc_l2l, bf_m2l, bc_m2l;
  // M2L: four waves share each 16-target tile and split its operator sequence
  // (fastest on both shallow and deep trees); eight, in workgroups of 512 threads,
  // where the 16-target tiles are too few to fill the GPU twice over, so that the
  // longest lists (reaction tiles of several hundred operators) end sooner
  // (a larger split where one wave's operator list would not fit the CU's LDS)
  int ks_m2l = P->gemm_ks;
  if (ks_m2l <= 0) {
    int64_t tiles = 0;
    for (int g = 0; g < ng_m2l; g++) tiles += (c_m2l[g] + 15) / 16;
    ks_m2l = tiles <= 2 * 256 ? 8 : 4;
  }
  while (ks_m2l < 4 && lk_m2l_lds_bytes(kmax_m2l, ks_m2l) > lk_m2l_lds_max()) ks_m2l *= 2;
  if (lk_m2l_lds_bytes(kmax_m2l, ks_m2l) > lk_m2l_lds_max()) throw Fail{LFMM_ENOTSUP};
  rep.m2l_ks = ks_m2l;
  // M2M: the waves of a 16-target tile split each parent's eight child operators
  // (a level's parents alone give too few 64-target blocks to fill the GPU)
  static const int ks_m2m = [] {  // tuning override: 1, 2 or 4
    const int v = getenv("LFMM_M2M_KS") ? atoi(getenv("LFMM_M2M_KS")) : 4;
    return (v == 1 || v == 2) ? v : 4;
  }();
  build_blocks(c_m2m, g_m2m, b_m2m, gs_m2m, bf_m2m, bc_m2m, lv_m2m, 9, 64 / ks_m2m);
  build_blocks(c_l2l, g_l2l, b_l2l, gs_l2l, bf_l2l, bc_l2l, lv_l2l, 9, 64);
  // (a 16-target tile per workgroup of four waves at K-split 4, of eight at 8)
  build_blocks(c_m2l, g_m2l, b_m2l, gs_m2l, bf_m2l, bc_m2l, {}, 1, ks_m2l == 8 ? 16 : 64 / ks_m2l);
  int ne_m2m = ng_m2m ? gs_m2m[ng_m2m] : 0, ne_l2l = ng_l2l ? gs_l2l[ng_l2l] : 0,
      ne_m2l = ng_m2l ? gs_m2l[ng_m2l] : 0;
  int64_t m2l_slots = 0;
  for (int g = 0; g < ng_m2l; g++) m2l_slots += (int64_t)c_m2l[g] * g_m2l[g].K;
  rep.m2l_slots = m2l_slots;
  // source rows
  int* sr_m2m = P->dev<int>("sr_m2m", (size_t)ne_m2m * 8 + 1);
  int* sr_l2l = P->dev<int>("sr_l2l", (size_t)ne_l2l + 1);
  int* sr_m2l = P->dev<int>("sr_m2l", (size_t)ne_m2l * kmax_m2l + 1);
  if (ne_m2m) lk_src_m2m(ne_m2m, J_m2m.srowid, box_code, box_tree, box_level, d_grid_off, grid, sr_m2m, d_cnt + 1, sj);
  if (ne_l2l) lk_src_l2l(ne_l2l, J_l2l.srowid, box_code, box_tree, box_level, d_grid_off, grid, sr_l2l, d_cnt + 2, sj);
  std::vector<int> gseq0(ng_m2l), gK(ng_m2l);
  for (int g = 0; g < ng_m2l; g++) {
    gseq0[g] = g_m2l[g].seq0;
    gK[g] = g_m2l[g].K;
  }
  int* d_gseq0 = P->upload("m2l_gseq0", gseq0, sj);
  int* d_gK = P->upload("m2l_gK", gK, sj);
  Tmpl* d_tmpl = P->upload("m2l_tmpl", tmpl_m2l, sj);
  if (ne_m2l)
    lk_src_m2l(ne_m2l, J_m2l.srowid, J_m2l.sgid, d_gseq0, d_gK, d_tmpl, kmax_m2l, box_code, box_level, d_grid_off,
               grid, sr_m2l, d_cnt + 0, sj);
  GBlock* d_bm2m = P->upload("b_m2m", b_m2m, sj);
  GBlock* d_bm2l = P->upload("b_m2l", b_m2l, sj);
  GBlock* d_bl2l = P->upload("b_l2l", b_l2l, sj);
  int* d_sq_m2m = P->upload("sq_m2m", seq_m2m, sj);
  int* d_sq_l2l = P->upload("sq_l2l", seq_l2l, sj);
  int* d_sq_m2l = P->upload("sq_m2l", seq_m2l, sj);
  send(ST_JOBS, sj);
  HIPCHK(hipEventRecord(P->jobs_ev, sj));
  HIPCHK(hipStreamWaitEvent(s, P->jobs_ev, 0));
  // the free-space operators are needed from here on
  HIPCHK(hipStreamWaitEvent(s, P->ops_ev, 0));
  sbeg(ST_M2M, s);
  {
    const int ksm = ks_m2m;
    const int* srow = J_m2m.srowid;
    qrun([=](hipStream_t ss, const double*, double*) {
      for (int lp = Dmax - 1; lp >= 2; lp--)
        if (bc_m2m[lp] > 0)
          lk_shift_gemm64(NC, ksm, bc_m2m[lp], d_bm2m + bf_m2m[lp], d_sq_m2m, srow, sr_m2m, 8, sops, opsz_m, NKS, M, M,
                        NCK, ss);
    });
  }
  // mixed precision: rescaled FP32 copy of the multipole expansions (it needs only the
  // upward pass, so it runs before the wait for the reaction operators; its time is
  // counted with the upward pass, so that the m2l stage brackets the GEMM alone)
  float* M32 = nullptr;
  if (!b_m2l.empty() && m2l32) {
    M32 = P->dev<float>("M32", (size_t)NR * NCK * 2);
    qrun([=](hipStream_t ss, const double*, double*) { lk_m_to_f32(NR, NCK, NC, box_tree, box_level, d_sc, M, M32, ss); });
  }
  send(ST_M2M, s);
  // and the reaction operators from here on
  HIPCHK(hipStreamWaitEvent(s, P->join_ev, 0));
  sbeg(ST_M2L, s);
  // ---------------- M2L (every level, free and reaction)
  if (!b_m2l.empty() && m2l32) {
    const int nb = (int)b_m2l.size();
    const int* srow = J_m2l.srowid;
    qrun([=](hipStream_t ss, const double*, double*) {
      lk_gemm32(NC, ks_m2l, nb, d_bm2l, d_sq_m2l, srow, sr_m2l, kmax_m2l, ops32, opsz_m, NKS, M32, Lx, NCK, box_tree,
                box_level, d_sc, ss);
    });
  } else if (!b_m2l.empty()) {
    const int nb = (int)b_m2l.size();
    const int* srow = J_m2l.srowid;
    qrun([=](hipStream_t ss, const double*, double*) {
      lk_m2l_gemm64(NC, ks_m2l, nb, d_bm2l, d_sq_m2l, srow, sr_m2l, kmax_m2l, ops, opsz_m, NKS, M, Lx, NCK, ss);
    });
  }
  mark(10);
  // ---------------- downward pass
  {
    const int* srow = J_l2l.srowid;
    qrun([=](hipStream_t ss, const double*, double*) {
      for (int l = 3; l <= Dmax; l++)
        if (bc_l2l[l] > 0)
          lk_shift_gemm64(NC, 1, bc_l2l[l], d_bl2l + bf_l2l[l], d_sq_l2l, srow, sr_l2l, 1, sops, opsz_m, NKS, Lx, Lx,
                        NCK, ss);
    });
  }
  mark(11);
  {
    std::vector<int> s0, pf;
    int tot = 0;
    for (int t = 0; t < ntrees; t++) {
      const TreeInfo& T = trees[t];
      if ((T.kind == 0 || T.kind == 1) && T.depth >= 2) {
        s0.push_back(T.pt_off);
        pf.push_back(tot);
        tot += T.npts;
        rep.l2p_leaves += nbox(t, T.depth);
      }
    }
    rep.l2p_points = tot;
    if (tot) {
      int* d_s0 = P->upload("l2p_s0", s0, s);
      int* d_pf = P->upload("l2p_pf", pf, s);
      const int ns0 = (int)s0.size();
      qrun([=](hipStream_t ss, const double*, double*) {
        lk_l2p(ns0, d_s0, d_pf, tot, leafrow, box_code, box_tree, box_level, d_trees, px, py, pz, sg, p, NCK, Lx,
               phi_tp, ss);
      });
    }
  }
  send(ST_L2P, s);
  sbeg(ST_NEAR_REACT, s);
  // ---------------- reaction near field (adjacent leaves across the interface)
  if (L >= 1 && Dr >= 1) {
    for (int l = 0; l < NL; l++)
      for (int a = 0; a < 2; a++) {
        int tt = tgt_tree[2 * l + a];
        if (tt < 0 || !hslab[(tt * 9 + Dr) * 2 + 0]) continue;
        std::vector<NFComp> comps;
        std::vector<Rule> rules;
        std::vector<int> lts, lss, as, bs;
        int node_tot = 0;
        double ht_min = hs[l * LFMM_NSTAT + (a == 0 ? 7 : 9)];
        for (int lp = 0; lp < NL; lp++)
          for (int b = 0; b < 2; b++) {
            int ts = src_tree[2 * lp + b];
            if (ts < 0 || !hslab[(ts * 9 + Dr) * 2 + 0]) continue;
            double hs_min = hs[lp * LFMM_NSTAT + (b == 0 ? 7 : 9)];
            double hD = Sr / (double)(1 << Dr);
            Rule r = P->make_rule(ht_min + hs_min, 2.0 * std::sqrt(2.0) * hD, 0);
            NFComp C;
            C.node0 = node_tot;
            C.nnodes = rule_nodes(r);
            C.stree = ts;
            C.pad = 0;
            node_tot += C.nnodes;
            comps.push_back(C);
            rules.push_back(r);
            lts.push_back(l);
            lss.push_back(lp);
            as.push_back(a);
            bs.push_back(b);
          }
        if (comps.empty()) continue;
        std::string tag = "nf" + std::to_string(tt);
        double* nkr = P->dev<double>((tag + "kr").c_str(), 2 * (size_t)node_tot);
        double* nfac = P->dev<double>((tag + "fac").c_str(), 2 * (size_t)node_tot);
        double* nkzt = P->dev<double>((tag + "kzt").c_str(), 2 * (size_t)node_tot);
        double* nkzs = P->dev<double>((tag + "kzs").c_str(), 2 * (size_t)node_tot);
        for (size_t c = 0; c < comps.size(); c++)
          lk_nf_nodes(comps[c].nnodes, rules[c], st, lts[c], lss[c], as[c], bs[c], nkr + 2 * comps[c].node0,
                      nfac + 2 * comps[c].node0, nkzt + 2 * comps[c].node0, nkzs + 2 * comps[c].node0, s);
        NFComp* d_comps = P->upload((tag + "comps").c_str(), comps, s);
        const int nbt = nbox(tt, Dr), fr = first_row(tt, Dr), nco = (int)comps.size();
        qrun([=](hipStream_t ss, const double*, double*) {
          lk_nf_react(nbt, fr, tt, nco, d_comps, box_start, box_cnt, box_code, d_trees, d_grid_off, grid, px, py, pz, pq,
                      sg, nkr, nfac, nkzt, nkzs, phi_tp, ss);
        });
        rep.nf_react_pairs += 1;
      }
  }
  mark(14);
  // ---------------- component sum
  int max_tt = 3;
  std::vector<int> tgt_list(NL * max_tt, -1);
  for (int l = 0; l < NL; l++) {
    tgt_list[l * max_tt + 0] = free_tree[l];
    tgt_list[l * max_tt + 1] = tgt_tree[2 * l + 0];
    tgt_list[l * max_tt + 2] = tgt_tree[2 * l + 1];
  }
  int* d_tl = P->upload("tgt_list", tgt_list, s);
  {
    const Stack stk = st;
    const int phys = P->physical;
    qrun([=](hipStream_t ss, const double*, double* ph) {
      lk_final_sum(n, layer, inv_perm, d_lstart, d_tl, max_tt, d_trees, phi_tp, ph, stk, phys, ss);
    });
  }
  send(ST_SUM, s);
  // every stream has joined the main one by now: the staging arena's last use is
  // complete once the main stream gets here
  if (P->pin_pending) HIPCHK(hipEventRecord(P->pin_ev, s));
  HIPCHK(hipGetLastError());
  unsigned long long hcnt[4] = {0, 0, 0, 0};
  P->rb_add(hcnt, d_cnt, sizeof(hcnt), s);
  P->rb_flush(s);
  // the readback waited for the main stream, which every other stream had joined:
  // the staging arena is free again, and no later call waits on an event recorded on
  // the caller's stream (which may be gone by then, as a batch worker's is)
  P->pin_pending = false;
  rep.m2l_pairs = (int64_t)hcnt[0];
  rep.m2m_pairs = (int64_t)hcnt[1];
  rep.l2l_pairs = (int64_t)hcnt[2];
  rep.p2p_pairs = (int64_t)hcnt[3];
  if (prof) {
    for (int i = 0; i < ST_COUNT; i++) {
      float ms = 0;
      if (staged(i) && hipEventElapsedTime(&ms, P->evb[i], P->eve[i]) == hipSuccess) rep.stage_ms[i] = ms;
    }
  }
  // operators generated into a lent workspace (a batch worker's) are gone once the
  // worker frees it, and a later allocation may reuse its addresses: keep no
  // signature then, so that the next evaluation on the plan's own workspace
  // generates its operators again
  if (P->bufp == &P->bufs) P->last_opsig.swap(opsig);
  else P->last_opsig.clear();
  if (P->arena) {
    rep.workspace_bytes = (int64_t)P->arena->used;
  } else {
    for (auto& kv : *P->bufp) rep.workspace_bytes += (int64_t)kv.second.cap;
  }
  return LFMM_OK;
}

}  // namespace

extern "C" {

int lfmm_plan(int L, const double* d, const double* k, int p, int leaf_max, const lfmm_options* opt,
              lfmm_plan_t** out) {
  return plan_impl(L, d, k, p, leaf_max, opt, out);
}

int lfmm_quad_nodes(int L, const double* d, const double* k, int p, const lfmm_options* opt, double dz,
                    double rho, int64_t* nodes) {
  if (!nodes) return LFMM_EINVAL;
  *nodes = 0;
  if (!(dz > 0) || !std::isfinite(dz) || !(rho >= 0) || !std::isfinite(rho)) return LFMM_EINVAL;
  lfmm_plan_s P;
  if (int rc = plan_params(L, d, k, p, 1, opt, &P)) return rc;
  // the count the rule would reach with an unlimited budget, reported beside LFMM_ENOCONV
  const int64_t budget = P.quad_max_nodes;
  P.quad_max_nodes = (int64_t)1 << 30;
  try {
    Rule r = P.make_rule(dz, rho, 2 * p + 1);
    *nodes = ((int64_t)LFMM_NP1 + r.nnear + r.nfar) * LFMM_NGL;
  } catch (Fail& f) {
    return f.code;
  }
  return *nodes > budget ? LFMM_ENOCONV : LFMM_OK;
}

int lfmm_eval_device(lfmm_plan_t* plan, int64_t n, const double* xyz, const int32_t* layer, const double* q,
                     double* phi, void* stream) {
  try {
    int rc = eval_impl(plan, n, xyz, layer, q, phi, (hipStream_t)stream);
    // the recorded launches stay valid while the workspace is the plan's own
    if (rc == LFMM_OK && plan->bufp == &plan->bufs && !plan->arena) plan->apply_ready = true;
    return rc;
  } catch (Fail& f) {
    // drain what this call queued before its staging buffers are reused
    (void)hipStreamSynchronize((hipStream_t)stream);
    (void)hipStreamSynchronize(plan->s2);
    if (plan->s3) (void)hipStreamSynchronize(plan->s3);
    plan->rb_list.clear();
    plan->rb_direct.clear();
    plan->rb_used = 0;
    plan->pin_pending = false;  // the streams are drained
    return f.code;
  }
}

int lfmm_prepare(lfmm_plan_t* plan, int64_t n, const double* xyz, const int32_t* layer, void* stream) {
  if (!plan) return LFMM_EINVAL;
  if (plan->bufp != &plan->bufs || plan->arena) return LFMM_EINVAL;  // only on the plan's own workspace
  hipStream_t s = (hipStream_t)stream;
  int rc;
  plan->prep_only = true;
  try {
    rc = eval_impl(plan, n, xyz, layer, nullptr, nullptr, s);
    if (rc == LFMM_OK && hipStreamSynchronize(s) != hipSuccess) rc = LFMM_EHIP;
  } catch (Fail& f) {
    (void)hipStreamSynchronize(s);
    (void)hipStreamSynchronize(plan->s2);
    if (plan->s3) (void)hipStreamSynchronize(plan->s3);
    plan->rb_list.clear();
    plan->rb_direct.clear();
    plan->rb_used = 0;
    plan->pin_pending = false;  // the streams are drained
    rc = f.code;
  }
  plan->prep_only = false;
  plan->apply_ready = rc == LFMM_OK;
  if (rc != LFMM_OK) plan->apply_list.clear();
  return rc;
}

int lfmm_apply(lfmm_plan_t* plan, const double* q, double* phi, void* stream) {
  if (!plan || !plan->apply_ready) return LFMM_EINVAL;
  if (plan->apply_n == 0) return LFMM_OK;
  if (!q || !phi) return LFMM_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  (void)hipGetLastError();  // the check below is for these launches
  lk_gather_q(plan->apply_ntp, plan->apply_orig, q, plan->apply_pq, s);
  for (auto& f : plan->apply_list) f(s, q, phi);
  return hipPeekAtLastError() == hipSuccess ? LFMM_OK : LFMM_EHIP;
}

int lfmm_eval(lfmm_plan_t* plan, int64_t n, const double* xyz, const int32_t* layer, const double* q, double* phi) {
  if (!plan || n < 0) return LFMM_EINVAL;
  if (n == 0) return LFMM_OK;
  if (!xyz || !q || !phi) return LFMM_EINVAL;
  try {
    double* dx = plan->dev<double>("h_xyz", 3 * (size_t)n);
    double* dq = plan->dev<double>("h_q", 2 * (size_t)n);
    double* dp = plan->dev<double>("h_phi", 2 * (size_t)n);
    int* dl = nullptr;
    HIPCHK(hipMemcpy(dx, xyz, sizeof(double) * 3 * n, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(dq, q, sizeof(double) * 2 * n, hipMemcpyHostToDevice));
    if (layer) {
      dl = plan->dev<int>("h_layer", n);
      HIPCHK(hipMemcpy(dl, layer, sizeof(int) * n, hipMemcpyHostToDevice));
    }
    int rc = eval_impl(plan, n, dx, dl, dq, dp, nullptr);
    if (rc != LFMM_OK) return rc;
    HIPCHK(hipMemcpy(phi, dp, sizeof(double) * 2 * n, hipMemcpyDeviceToHost));
    return LFMM_OK;
  } catch (Fail& f) {
    (void)hipStreamSynchronize(nullptr);
    (void)hipStreamSynchronize(plan->s2);
    if (plan->s3) (void)hipStreamSynchronize(plan->s3);
    plan->rb_list.clear();
    plan->rb_direct.clear();
    plan->rb_used = 0;
    plan->pin_pending = false;  // the streams are drained
    return f.code;
  }
}

// Targets apart from the sources: the union (sources, then targets with zero
// charge) goes through the ordinary evaluation; zero charges add nothing and the
// free part skips coincident points, so the union's potentials at the target
// entries are the requested ones.
static int eval_targets_impl(lfmm_plan_t* P, int64_t ns, const double* sxyz, const int32_t* slay, const double* q,
                             int64_t nt, const double* txyz, const int32_t* tlay, double* phi, hipStream_t s) {
  if (!P || ns < 0 || nt < 0 || ns + nt >= ((int64_t)1 << 31)) return LFMM_EINVAL;
  if (nt == 0) return LFMM_OK;
  if ((ns > 0 && (!sxyz || !q)) || !txyz || !phi) return LFMM_EINVAL;
  if ((slay == nullptr) != (tlay == nullptr) && ns > 0) return LFMM_EINVAL;  // both or neither
  const size_t nu = (size_t)(ns + nt);
  double* ux = P->dev<double>("u_xyz", 3 * nu);
  double* uq = P->dev<double>("u_q", 2 * nu);
  double* up = P->dev<double>("u_phi", 2 * nu);
  int* ul = nullptr;
  for (int c = 0; c < 3; c++) {
    if (ns) HIPCHK(hipMemcpyAsync(ux + c * nu, sxyz + c * (size_t)ns, sizeof(double) * ns, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(ux + c * nu + ns, txyz + c * (size_t)nt, sizeof(double) * nt, hipMemcpyDeviceToDevice, s));
  }
  if (ns) HIPCHK(hipMemcpyAsync(uq, q, sizeof(double) * 2 * ns, hipMemcpyDeviceToDevice, s));
  lk_zero(uq + 2 * ns, 2 * (size_t)nt, s);
  if (tlay) {
    ul = P->dev<int>("u_layer", nu);
    if (ns) HIPCHK(hipMemcpyAsync(ul, slay, sizeof(int) * ns, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(ul + ns, tlay, sizeof(int) * nt, hipMemcpyDeviceToDevice, s));
  }
  int rc = eval_impl(P, (int64_t)nu, ux, ul, uq, up, s);
  if (rc != LFMM_OK) return rc;
  HIPCHK(hipMemcpyAsync(phi, up + 2 * ns, sizeof(double) * 2 * nt, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  return LFMM_OK;
}

int lfmm_eval_targets_device(lfmm_plan_t* plan, int64_t n_src, const double* src_xyz, const int32_t* src_layer,
                             const double* q, int64_t n_tgt, const double* tgt_xyz, const int32_t* tgt_layer,
                             double* phi, void* stream) {
  try {
    return eval_targets_impl(plan, n_src, src_xyz, src_layer, q, n_tgt, tgt_xyz, tgt_layer, phi, (hipStream_t)stream);
  } catch (Fail& f) {
    (void)hipStreamSynchronize((hipStream_t)stream);
    if (plan) {
      (void)hipStreamSynchronize(plan->s2);
      if (plan->s3) (void)hipStreamSynchronize(plan->s3);
      plan->rb_list.clear();
      plan->rb_direct.clear();
      plan->rb_used = 0;
      plan->pin_pending = false;  // the streams are drained
    }
    return f.code;
  }
}

int lfmm_eval_targets(lfmm_plan_t* plan, int64_t n_src, const double* src_xyz, const int32_t* src_layer,
                      const double* q, int64_t n_tgt, const double* tgt_xyz, const int32_t* tgt_layer, double* phi) {
  if (!plan || n_src < 0 || n_tgt < 0) return LFMM_EINVAL;
  if (n_tgt == 0) return LFMM_OK;
  if ((n_src > 0 && (!src_xyz || !q)) || !tgt_xyz || !phi) return LFMM_EINVAL;
  try {
    double* ds = plan->dev<double>("hs_xyz", 3 * (size_t)std::max<int64_t>(n_src, 1));
    double* dq = plan->dev<double>("hs_q", 2 * (size_t)std::max<int64_t>(n_src, 1));
    double* dt = plan->dev<double>("ht_xyz", 3 * (size_t)n_tgt);
    double* dp = plan->dev<double>("ht_phi", 2 * (size_t)n_tgt);
    int *dsl = nullptr, *dtl = nullptr;
    if (n_src) {
      HIPCHK(hipMemcpy(ds, src_xyz, sizeof(double) * 3 * n_src, hipMemcpyHostToDevice));
      HIPCHK(hipMemcpy(dq, q, sizeof(double) * 2 * n_src, hipMemcpyHostToDevice));
    }
    HIPCHK(hipMemcpy(dt, tgt_xyz, sizeof(double) * 3 * n_tgt, hipMemcpyHostToDevice));
    if (src_layer && n_src) {
      dsl = plan->dev<int>("hs_layer", n_src);
      HIPCHK(hipMemcpy(dsl, src_layer, sizeof(int) * n_src, hipMemcpyHostToDevice));
    }
    if (tgt_layer) {
      dtl = plan->dev<int>("ht_layer", n_tgt);
      HIPCHK(hipMemcpy(dtl, tgt_layer, sizeof(int) * n_tgt, hipMemcpyHostToDevice));
    }
    int rc = eval_targets_impl(plan, n_src, ds, dsl, dq, n_tgt, dt, dtl, dp, nullptr);
    if (rc != LFMM_OK) return rc;
    HIPCHK(hipMemcpy(phi, dp, sizeof(double) * 2 * n_tgt, hipMemcpyDeviceToHost));
    return LFMM_OK;
  } catch (Fail& f) {
    (void)hipStreamSynchronize(nullptr);
    (void)hipStreamSynchronize(plan->s2);
    if (plan->s3) (void)hipStreamSynchronize(plan->s3);
    plan->rb_list.clear();
    plan->rb_direct.clear();
    plan->rb_used = 0;
    plan->pin_pending = false;  // the streams are drained
    return f.code;
  }
}

int lfmm_eval_batch(int nprob, lfmm_plan_t* const* plans, const int64_t* n, const double* const* xyz,
                    const int32_t* const* layer, const double* const* q, double* const* phi, int nworkers,
                    int* status) {
  if (nprob < 0 || (nprob > 0 && (!plans || !n || !xyz || !q || !phi))) return LFMM_EINVAL;
  if (nprob == 0) return LFMM_OK;
  {
    std::set<const lfmm_plan_t*> seen;
    for (int i = 0; i < nprob; i++)
      if (!plans[i] || !seen.insert(plans[i]).second) return LFMM_EINVAL;
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return LFMM_EHIP;
  const int nw = std::max(1, std::min(nworkers > 0 ? nworkers : 8, nprob));
  std::vector<int> st(nprob, LFMM_OK);
  std::atomic<int> next(0);
  // each worker owns one device workspace and lends it to the plans it runs, so
  // the batch needs nworkers workspaces rather than one per problem
  auto worker = [&]() {
    hipStream_t ws = nullptr;
    if (hipSetDevice(dev) != hipSuccess || hipStreamCreateWithFlags(&ws, hipStreamNonBlocking) != hipSuccess) {
      for (int i; (i = next.fetch_add(1)) < nprob;) st[i] = LFMM_EHIP;
      return;
    }
    std::map<std::string, DevBuf> wbufs;
    for (int i; (i = next.fetch_add(1)) < nprob;) {
      plans[i]->bufp = &wbufs;
      st[i] = lfmm_eval_device(plans[i], n[i], xyz[i], layer ? layer[i] : nullptr, q[i], phi[i], ws);
      plans[i]->bufp = &plans[i]->bufs;
    }
    (void)hipStreamSynchronize(ws);
    (void)hipStreamDestroy(ws);
    for (auto& kv : wbufs)
      if (kv.second.p) (void)hipFree(kv.second.p);
  };
  std::vector<std::thread> th;
  for (int w = 0; w < nw; w++) th.emplace_back(worker);
  for (auto& t : th) t.join();
  int rc = LFMM_OK;
  for (int i = 0; i < nprob; i++) {
    if (status) status[i] = st[i];
    if (rc == LFMM_OK && st[i] != LFMM_OK) rc = st[i];
  }
  return rc;
}

struct lfmm_batch_s {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

int lfmm_batch_prepare(int nprob, lfmm_plan_t* const* plans, const int64_t* n, const double* const* xyz,
                       const int32_t* const* layer, int nworkers, int* status) {
  if (nprob <= 0 || !plans || !n || !xyz) return LFMM_EINVAL;
  {
    std::set<const lfmm_plan_t*> seen;
    for (int i = 0; i < nprob; i++) {
      if (!plans[i] || !seen.insert(plans[i]).second || n[i] < 0) return LFMM_EINVAL;
      if (n[i] > 0 && !xyz[i]) return LFMM_EINVAL;
    }
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return LFMM_EHIP;
  const int nw = std::max(1, std::min(nworkers > 0 ? nworkers : 8, nprob));
  std::vector<int> st(nprob, LFMM_OK);
  std::atomic<int> next(0);
  auto worker = [&]() {
    hipStream_t ws = nullptr;
    if (hipSetDevice(dev) != hipSuccess || hipStreamCreateWithFlags(&ws, hipStreamNonBlocking) != hipSuccess) {
      for (int i; (i = next.fetch_add(1)) < nprob;) st[i] = LFMM_EHIP;
      return;
    }
    for (int i; (i = next.fetch_add(1)) < nprob;)
      st[i] = lfmm_prepare(plans[i], n[i], xyz[i], layer ? layer[i] : nullptr, ws);
    (void)hipStreamDestroy(ws);
  };
  std::vector<std::thread> th;
  for (int w = 0; w < nw; w++) th.emplace_back(worker);
  for (auto& t : th) t.join();
  int rc = LFMM_OK;
  for (int i = 0; i < nprob; i++) {
    if (status) status[i] = st[i];
    if (rc == LFMM_OK && st[i] != LFMM_OK) rc = st[i];
  }
  return rc;
}

int lfmm_batch_capture(int nprob, lfmm_plan_t* const* plans, const double* const* q, double* const* phi,
                       int nbranch, lfmm_batch_t** out, lfmm_batch_report* rep) {
  if (!out) return LFMM_EINVAL;
  *out = nullptr;
  if (nprob <= 0 || !plans || !q || !phi) return LFMM_EINVAL;
  {
    std::set<const lfmm_plan_t*> seen;
    for (int i = 0; i < nprob; i++) {
      if (!plans[i] || !seen.insert(plans[i]).second || !plans[i]->apply_ready) return LFMM_EINVAL;
      if (plans[i]->apply_n > 0 && (!q[i] || !phi[i])) return LFMM_EINVAL;
    }
  }
  const auto t1 = std::chrono::steady_clock::now();
  int rc = LFMM_OK;
  // the problems over the branches, largest first, each to the least loaded branch
  const int nb = std::max(1, std::min(nbranch > 0 ? nbranch : 4, std::min(nprob, 16)));
  std::vector<int> order(nprob);
  for (int i = 0; i < nprob; i++) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return plans[a]->apply_n > plans[b]->apply_n; });
  std::vector<int64_t> load(nb, 0);
  std::vector<std::vector<int>> members(nb);
  for (int i : order) {
    const int b = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    members[b].push_back(i);
    load[b] += plans[i]->apply_n;
  }
  hipStream_t cs = nullptr;
  std::vector<hipStream_t> br(nb, nullptr);
  std::vector<hipEvent_t> ev(nb + 1, nullptr);
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool capturing = false;
  auto cleanup = [&]() {
    if (capturing) {
      hipGraph_t g = nullptr;
      (void)hipStreamEndCapture(cs, &g);
      if (g) (void)hipGraphDestroy(g);
    }
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
    for (auto& b : br)
      if (b) (void)hipStreamDestroy(b);
    if (cs) (void)hipStreamDestroy(cs);
  };
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) rc = LFMM_EHIP;
  for (int b = 0; b < nb && rc == LFMM_OK; b++)
    if (hipStreamCreateWithFlags(&br[b], hipStreamNonBlocking) != hipSuccess) rc = LFMM_EHIP;
  for (int b = 0; b <= nb && rc == LFMM_OK; b++)
    if (hipEventCreateWithFlags(&ev[b], hipEventDisableTiming) != hipSuccess) rc = LFMM_EHIP;
  if (rc == LFMM_OK && hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) rc = LFMM_EHIP;
  capturing = rc == LFMM_OK;
  if (rc == LFMM_OK && hipEventRecord(ev[nb], cs) != hipSuccess) rc = LFMM_EHIP;
  for (int b = 0; b < nb && rc == LFMM_OK; b++) {
    if (hipStreamWaitEvent(br[b], ev[nb], 0) != hipSuccess) {
      rc = LFMM_EHIP;
      break;
    }
    for (int i : members[b])
      if ((rc = lfmm_apply(plans[i], q[i], phi[i], br[b])) != LFMM_OK) break;
    if (rc == LFMM_OK && (hipEventRecord(ev[b], br[b]) != hipSuccess || hipStreamWaitEvent(cs, ev[b], 0) != hipSuccess))
      rc = LFMM_EHIP;
  }
  if (capturing) {
    capturing = false;
    if (hipStreamEndCapture(cs, &graph) != hipSuccess && rc == LFMM_OK) rc = LFMM_EHIP;
  }
  if (rc == LFMM_OK && hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) rc = LFMM_EHIP;
  cleanup();
  if (rc != LFMM_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  lfmm_batch_s* B = new lfmm_batch_s();
  B->graph = graph;
  B->exec = exec;
  if (rep) {
    memset(rep, 0, sizeof(*rep));
    for (int i = 0; i < nprob; i++) rep->n_total += plans[i]->apply_n;
    size_t nn = 0;
    if (hipGraphGetNodes(graph, nullptr, &nn) == hipSuccess) rep->graph_nodes = (int64_t)nn;
    rep->branches = nb;
    rep->capture_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t1).count();
  }
  *out = B;
  return LFMM_OK;
}

int lfmm_batch_launch(lfmm_batch_t* batch, void* stream) {
  if (!batch || !batch->exec) return LFMM_EINVAL;
  return hipGraphLaunch(batch->exec, (hipStream_t)stream) == hipSuccess ? LFMM_OK : LFMM_EHIP;
}

void lfmm_batch_destroy(lfmm_batch_t* batch) {
  if (!batch) return;
  if (batch->exec) (void)hipGraphExecDestroy(batch->exec);
  if (batch->graph) (void)hipGraphDestroy(batch->graph);
  delete batch;
}

// ---- allocation-free evaluation ----
// The library's static device scratch: every device that loads the library holds
// one copy of it until the process ends.  In host code the array's name is only a
// stand-in; its device address on each device comes from hipGetSymbolAddress,
// called once per device with that device current, and only that address is used.
static __device__ __align__(256) char scratch[LFMM_NOALLOC_BYTES];
#define LFMM_NOALLOC_MAXDEV 64
static std::mutex g_scratch_mu;
static char* g_scratch_ptr[LFMM_NOALLOC_MAXDEV] = {};

static int scratch_of_device(int dev, char** out) {
  if (dev < 0 || dev >= LFMM_NOALLOC_MAXDEV) return LFMM_ENOTSUP;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return LFMM_EHIP;
    g_scratch_ptr[dev] = (char*)ptr;
  }
  *out = g_scratch_ptr[dev];
  return LFMM_OK;
}

int lfmm_eval_device_noalloc(lfmm_plan_t* plan, int64_t n, const double* xyz, const int32_t* layer, const double* q,
                             double* phi, void* stream) {
  if (!plan) return LFMM_EINVAL;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return LFMM_EHIP;
  if (dev != plan->device) return LFMM_EINVAL;  // the plan's streams live on another device
  char* base = nullptr;
  int rc = scratch_of_device(dev, &base);
  if (rc != LFMM_OK) return rc;
  Arena A;
  A.base = base;
  A.cap = (size_t)LFMM_NOALLOC_BYTES;
  std::map<std::string, DevBuf> pieces;  // names -> pieces of the scratch; never freed
  plan->arena = &A;
  plan->bufp = &pieces;
  plan->sur.net.arena = &A;
  rc = lfmm_eval_device(plan, n, xyz, layer, q, phi, stream);
  // the next call on this device reuses the scratch: nothing of this one may still run
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess && rc == LFMM_OK) rc = LFMM_EHIP;
  if (hipStreamSynchronize(plan->s2) != hipSuccess && rc == LFMM_OK) rc = LFMM_EHIP;
  if (plan->s3 && hipStreamSynchronize(plan->s3) != hipSuccess && rc == LFMM_OK) rc = LFMM_EHIP;
  plan->arena = nullptr;
  plan->bufp = &plan->bufs;
  plan->sur.net.arena = nullptr;
  plan->sur.net.abufs.clear();
  return rc;
}

int lfmm_last_report(const lfmm_plan_t* plan, lfmm_report* rep) {
  if (!plan || !rep) return LFMM_EINVAL;
  *rep = plan->rep;
  return LFMM_OK;
}

const char* lfmm_stage_name(int i) { return (i >= 0 && i < ST_COUNT) ? kStageNames[i] : nullptr; }

void lfmm_destroy(lfmm_plan_t* plan) {
  if (!plan) return;
  for (auto& kv : plan->bufs)
    if (kv.second.p) (void)hipFree(kv.second.p);
  if (plan->d_gaunt) (void)hipFree(plan->d_gaunt);
  if (plan->pin_pending) (void)hipEventSynchronize(plan->pin_ev);
  if (plan->pin) (void)hipHostFree(plan->pin);
  if (plan->pin_ev) (void)hipEventDestroy(plan->pin_ev);
  if (plan->rb) (void)hipHostFree(plan->rb);
  if (plan->rb_ev) (void)hipEventDestroy(plan->rb_ev);
  for (int i = 0; i < ST_COUNT; i++) {
    if (plan->evb[i]) (void)hipEventDestroy(plan->evb[i]);
    if (plan->eve[i]) (void)hipEventDestroy(plan->eve[i]);
  }
  if (plan->s2) {
    (void)hipStreamSynchronize(plan->s2);
    (void)hipStreamDestroy(plan->s2);
  }
  if (plan->fork_ev) (void)hipEventDestroy(plan->fork_ev);
  if (plan->join_ev) (void)hipEventDestroy(plan->join_ev);
  if (plan->ops_ev) (void)hipEventDestroy(plan->ops_ev);
  if (plan->s3) {
    (void)hipStreamSynchronize(plan->s3);
    (void)hipStreamDestroy(plan->s3);
  }
  if (plan->jobs_ev) (void)hipEventDestroy(plan->jobs_ev);
  plan->sur.net.release();
  plan->tab.release();
  delete plan;
}

const char* lfmm_last_hip_error(void) {
  std::lock_guard<std::mutex> g(g_hip_err_mu);
  return g_hip_err[g_hip_err_cur];
}

const char* lfmm_status_string(int status) {
  switch (status) {
    case LFMM_OK: return "ok";
    case LFMM_EINVAL: return "invalid argument";
    case LFMM_ENOMEM: return "out of memory";
    case LFMM_EHIP: return "HIP runtime error";
    case LFMM_ENOTSUP: return "not supported";
    case LFMM_EIO: return "surrogate file unreadable, unwritable or not for this plan";
    case LFMM_ENOCONV: return "Sommerfeld quadrature needs more contour nodes than the plan allows";
    default: return "unknown status";
  }
}

// Operator from its packed form: the GEMMs' k-step-major layout with its last-row entries.
static void unpack_op(const std::vector<double>& pk, int NC, int NKS, double* out) {
  const int NRT = m2l_nrt(NC), XR = m2l_xr(NC), SZ = NRT * 64 + 4 * XR;
  for (int r = 0; r < NC; r++)
    for (int c = 0; c < NC; c++) {
      size_t pp;
      if (r < NRT * 16) pp = 2 * ((size_t)(c >> 2) * SZ + (r >> 4) * 64 + (r & 15) + 16 * (c & 3));
      else pp = 2 * ((size_t)(c >> 2) * SZ + NRT * 64 + (c & 3));
      out[2 * ((size_t)r * NC + c)] = pk[pp];
      out[2 * ((size_t)r * NC + c) + 1] = pk[pp + 1];
    }
}

int lfmm_translation(lfmm_plan_t* plan, int kind, double kw, const double* b, double* out) {
  if (!plan || !b || !out || (kind != 0 && kind != 1) || !(kw > 0)) return LFMM_EINVAL;
  if (kind == 1 && b[0] == 0 && b[1] == 0 && b[2] == 0) return LFMM_EINVAL;
  try {
    std::vector<OpDesc> d(1);
    d[0] = OpDesc{b[0], b[1], b[2], kw, kind, 0};
    OpDesc* dd = plan->upload("dbg_op", d, nullptr);
    double* ops = plan->dev<double>("dbg_ops", plan->opsz);
    lk_transop(1, dd, ops, plan->opsz, ops, plan->opsz, plan->p, plan->NC, plan->NKS, plan->d_gaunt, nullptr, nullptr,
               nullptr);
    std::vector<double> pk(plan->opsz);
    HIPCHK(hipMemcpy(pk.data(), ops, sizeof(double) * plan->opsz, hipMemcpyDeviceToHost));
    unpack_op(pk, plan->NC, plan->NKS, out);
  } catch (Fail& f) {
    return f.code;
  }
  return LFMM_OK;
}

int lfmm_reaction_operator(lfmm_plan_t* plan, int l, int a, int lp, int b, double dx, double dy, double zt, double zs,
                           double* out) {
  if (!plan || !out) return LFMM_EINVAL;
  const Stack& st = plan->st;
  if (st.L < 1 || l < 0 || l > st.L || lp < 0 || lp > st.L || (a != 0 && a != 1) || (b != 0 && b != 1))
    return LFMM_EINVAL;
  if (!has_dir(st, l, a) || !has_dir(st, lp, b) || !(zt > 0) || !(zs > 0)) return LFMM_EINVAL;
  try {
    int NC = plan->NC;
    std::vector<ClassDesc> c(1);
    memset(&c[0], 0, sizeof(ClassDesc));
    c[0].zt = zt;
    c[0].zs = zs;
    c[0].rho = std::sqrt(dx * dx + dy * dy);
    c[0].rule = plan->make_rule(zt + zs, c[0].rho, 2 * plan->p + 1);
    c[0].lt = l;
    c[0].ls = lp;
    c[0].a = a;
    c[0].b = b;
    c[0].out = 0;
    double* I = plan->dev<double>("dbg_I", (size_t)NC * NC * 2);
    reaction_integrals(plan, "dbg", c, I, nullptr);
    std::vector<ROpDesc> r(1);
    r[0] = ROpDesc{dx, dy, st.k[l], 0, 0};
    ROpDesc* dr = plan->upload("dbg_rop", r, nullptr);
    double* ops = plan->dev<double>("dbg_ops", plan->opsz);
    std::vector<int> g1 = {0, 1};
    int* dg = plan->upload("dbg_rgrp", g1, nullptr);
    lk_react_expand(1, dg, dr, I, ops, plan->opsz, plan->p, NC, plan->NKS, nullptr, nullptr, nullptr);
    std::vector<double> pk(plan->opsz);
    HIPCHK(hipMemcpy(pk.data(), ops, sizeof(double) * plan->opsz, hipMemcpyDeviceToHost));
    unpack_op(pk, NC, plan->NKS, out);
  } catch (Fail& f) {
    return f.code;
  }
  return LFMM_OK;
}

int lfmm_densities(lfmm_plan_t* plan, int n, const double* krho, int l, int lp, double* out) {
  if (!plan || n < 0 || (n > 0 && (!krho || !out))) return LFMM_EINVAL;
  if (l < 0 || l > plan->st.L || lp < 0 || lp > plan->st.L) return LFMM_EINVAL;
  if (n == 0) return LFMM_OK;
  try {
    double* dk = plan->dev<double>("dbg_kr", 2 * (size_t)n);
    double* dout = plan->dev<double>("dbg_sig", 8 * (size_t)n);
    HIPCHK(hipMemcpy(dk, krho, sizeof(double) * 2 * n, hipMemcpyHostToDevice));
    lk_dbg_dens(n, dk, plan->st, l, lp, dout, nullptr);
    HIPCHK(hipMemcpy(out, dout, sizeof(double) * 8 * n, hipMemcpyDeviceToHost));
  } catch (Fail& f) {
    return f.code;
  }
  return LFMM_OK;
}

int lfmm_surrogate_train(lfmm_plan_t* plan, int64_t n_samples, uint64_t seed, const lfmm_train_opts* opts,
                         lfmm_train_report* rep) {
  if (!plan || n_samples < 0) return LFMM_EINVAL;
  if (plan->st.L < 1) return LFMM_EINVAL;
  lfmm_train_opts o;
  memset(&o, 0, sizeof(o));
  if (opts) o = *opts;
  if (o.h_min <= 0) o.h_min = 0.02;
  if (o.h_max <= 0) o.h_max = 2.0;
  if (o.epochs <= 0) o.epochs = 150;
  if (o.batch <= 0) o.batch = 256;
  if (o.lr <= 0) o.lr = 2e-3;
  if (o.holdout <= 0) o.holdout = 0.1;
  if (o.width <= 0) o.width = 128;
  if (o.nhidden <= 0) o.nhidden = 4;
  if (!(o.h_max > o.h_min) || !std::isfinite(o.h_max) || o.holdout >= 1.0 || o.width > 1024 || o.nhidden > 16 ||
      o.batch > 65536 || n_samples > ((int64_t)1 << 26))
    return LFMM_EINVAL;
  lfmm_train_report R;
  try {
    sur_train_impl(plan, n_samples, seed, o, R);
  } catch (Fail& f) {
    (void)hipStreamSynchronize(plan->s2);
    if (plan->s3) (void)hipStreamSynchronize(plan->s3);
    plan->sur.ready = false;
    return f.code;
  }
  if (rep) *rep = R;
  return LFMM_OK;
}

// File: "LFMMSUR1", then int32 {version 1, p, L, ncomp, nin, width, nhidden, nout},
// double k[L+1], d[L], h_lo, h_hi, bound[ncomp*40], float mu[nout], sd[nout], w[np].
int lfmm_surrogate_save(const lfmm_plan_t* plan, const char* path) {
  if (!plan || !path || !plan->sur.ready) return LFMM_EINVAL;
  const Surrogate& S = plan->sur;
  MlpNet& N = const_cast<MlpNet&>(S.net);
  std::vector<float> w(N.np);
  if (hipMemcpy(w.data(), N.w(), N.np * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess) return LFMM_EHIP;
  FILE* f = fopen(path, "wb");
  if (!f) return LFMM_EIO;
  const int L = plan->st.L;
  int32_t hd[8] = {1, plan->p, L, S.ncomp, N.nin, N.width, N.nh, N.nout};
  bool ok = fwrite("LFMMSUR1", 1, 8, f) == 8 && fwrite(hd, sizeof(hd), 1, f) == 1 &&
            fwrite(plan->st.k, sizeof(double), L + 1, f) == (size_t)(L + 1) &&
            (L == 0 || fwrite(plan->st.d, sizeof(double), L, f) == (size_t)L) &&
            fwrite(&S.h_lo, sizeof(double), 1, f) == 1 && fwrite(&S.h_hi, sizeof(double), 1, f) == 1 &&
            fwrite(S.bound.data(), sizeof(double), S.bound.size(), f) == S.bound.size() &&
            fwrite(S.mu.data(), sizeof(float), S.mu.size(), f) == S.mu.size() &&
            fwrite(S.sd.data(), sizeof(float), S.sd.size(), f) == S.sd.size() &&
            fwrite(w.data(), sizeof(float), w.size(), f) == w.size();
  if (fclose(f) != 0) ok = false;
  return ok ? LFMM_OK : LFMM_EIO;
}

int lfmm_surrogate_load(lfmm_plan_t* plan, const char* path) {
  if (!plan || !path) return LFMM_EINVAL;
  FILE* f = fopen(path, "rb");
  if (!f) return LFMM_EIO;
  const int L = plan->st.L, NL = L + 1;
  char magic[8];
  int32_t hd[8];
  std::vector<double> kk(NL), dd(L);
  bool ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, "LFMMSUR1", 8) == 0 && fread(hd, sizeof(hd), 1, f) == 1 &&
            hd[0] == 1 && hd[1] == plan->p && hd[2] == L;
  ok = ok && fread(kk.data(), sizeof(double), NL, f) == (size_t)NL && (L == 0 || fread(dd.data(), sizeof(double), L, f) == (size_t)L);
  for (int i = 0; ok && i < NL; i++) ok = kk[i] == plan->st.k[i];
  for (int i = 0; ok && i < L; i++) ok = dd[i] == plan->st.d[i];
  Surrogate T;
  if (ok) {
    int ncomp = 0;  // the component numbering depends on L only
    for (int l = 0; l < NL; l++)
      for (int a = 0; a < 2; a++)
        for (int lp = 0; lp < NL; lp++)
          for (int b = 0; b < 2; b++) ncomp += has_dir(plan->st, l, a) && has_dir(plan->st, lp, b);
    ok = hd[3] == ncomp && hd[4] == sur_nin(hd[3]) && hd[5] > 0 && hd[5] <= 1024 && hd[6] > 0 && hd[6] <= 16 &&
         hd[7] == 2 * plan->NT * plan->NC;
  }
  std::vector<float> w;
  if (ok) {
    T.net.setup(hd[4], hd[5], hd[6], hd[7]);
    T.bound.resize((size_t)hd[3] * 40);
    T.mu.resize(hd[7]);
    T.sd.resize(hd[7]);
    w.resize(T.net.np);
    ok = fread(&T.h_lo, sizeof(double), 1, f) == 1 && fread(&T.h_hi, sizeof(double), 1, f) == 1 &&
         fread(T.bound.data(), sizeof(double), T.bound.size(), f) == T.bound.size() &&
         fread(T.mu.data(), sizeof(float), T.mu.size(), f) == T.mu.size() &&
         fread(T.sd.data(), sizeof(float), T.sd.size(), f) == T.sd.size() &&
         fread(w.data(), sizeof(float), w.size(), f) == w.size() && T.h_hi > T.h_lo && T.h_lo > 0;
    char extra;
    ok = ok && fread(&extra, 1, 1, f) == 0;
  }
  fclose(f);
  if (!ok) return LFMM_EIO;
  Surrogate& S = plan->sur;
  try {
    S.ready = false;
    S.net.release();
    S.net.setup(T.net.nin, T.net.width, T.net.nh, T.net.nout);
    S.net.load_params(w.data(), nullptr);
    HIPCHK(hipMemcpy(S.net.dev<float>("mu", S.net.nout), T.mu.data(), T.mu.size() * sizeof(float),
                     hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(S.net.dev<float>("sd", S.net.nout), T.sd.data(), T.sd.size() * sizeof(float),
                     hipMemcpyHostToDevice));
    HIPCHK(hipDeviceSynchronize());
  } catch (Fail& fl) {
    return fl.code;
  }
  sur_components(plan);
  try {
    sur_decay(plan);
  } catch (Fail& fl) {
    return fl.code;
  }
  S.h_lo = T.h_lo;
  S.h_hi = T.h_hi;
  S.bound = T.bound;
  S.mu = T.mu;
  S.sd = T.sd;
  memset(&S.trep, 0, sizeof(S.trep));
  S.version++;
  S.ready = true;
  return LFMM_OK;
}

int lfmm_surrogate_gate(lfmm_plan_t* plan, double tol) {
  if (!plan || !(tol >= 0.0)) return LFMM_EINVAL;
  plan->sur.tol = tol;
  return LFMM_OK;
}

int lfmm_surrogate_bounds(const lfmm_plan_t* plan, int n, double* bounds, int* count) {
  if (!plan || !count || n < 0 || (n > 0 && !bounds)) return LFMM_EINVAL;
  const Surrogate& S = plan->sur;
  if (!S.ready) {
    *count = 0;
    return LFMM_EINVAL;
  }
  int w = 0;
  for (int c = 0; c < S.ncomp; c++)
    for (int j = 0; j < 2; j++)
      for (int i = 0; i < 2; i++)
        for (int ri = 0; ri < 10; ri++) {
          if (i == 0 && j == 0 && kR2[ri] <= 2) continue;
          if (w < n) bounds[w] = S.bound[sur_combo(c, j, i, ri)];
          w++;
        }
  *count = w;
  return LFMM_OK;
}

int lfmm_tables_build(lfmm_plan_t* plan, const lfmm_table_opts* opts, lfmm_table_report* rep) {
  if (!plan) return LFMM_EINVAL;
  if (plan->st.L < 1) return LFMM_EINVAL;
  lfmm_table_opts o;
  memset(&o, 0, sizeof(o));
  if (opts) o = *opts;
  if (o.h_min <= 0) o.h_min = 0.02;
  if (o.h_max <= 0) o.h_max = 2.0;
  if (o.nnode <= 0) o.nnode = 16;
  if (o.du <= 0) o.du = 1.5;
  if (o.nval <= 0) o.nval = 4;
  if (!(o.h_max > o.h_min) || !std::isfinite(o.h_max) || o.nnode < 2 || o.nnode > 32 || o.nval > 32 ||
      !std::isfinite(o.du))
    return LFMM_EINVAL;
  OpTables& T = plan->tab;
  T.alpha = 4.0 * plan->kmax;
  const double span = (std::log(o.h_max) + T.alpha * o.h_max) - (std::log(o.h_min) + T.alpha * o.h_min);
  if (span / o.du > 4096) return LFMM_EINVAL;
  lfmm_table_report R;
  try {
    tab_build_impl(plan, o, R);
  } catch (Fail& f) {
    (void)hipStreamSynchronize(plan->s2);
    T.release();
    return f.code;
  }
  if (rep) *rep = R;
  return LFMM_OK;
}

int lfmm_tables_gate(lfmm_plan_t* plan, double tol) {
  if (!plan || !(tol >= 0.0)) return LFMM_EINVAL;
  plan->tab.tol = tol;
  return LFMM_OK;
}

int lfmm_tables_bounds(const lfmm_plan_t* plan, int n, double* bounds, int* count) {
  if (!plan || !count || n < 0 || (n > 0 && !bounds)) return LFMM_EINVAL;
  const OpTables& T = plan->tab;
  if (!T.ready) {
    *count = 0;
    return LFMM_EINVAL;
  }
  int w = 0;
  for (size_t c = 0; c < T.bound.size(); c++)
    if (T.dense[c] >= 0) {
      if (w < n) bounds[w] = T.bound[c];
      w++;
    }
  *count = w;
  return LFMM_OK;
}

int lfmm_tables_release(lfmm_plan_t* plan) {
  if (!plan) return LFMM_EINVAL;
  (void)hipStreamSynchronize(plan->s2);
  (void)hipDeviceSynchronize();
  plan->tab.release();
  plan->tab.version++;
  return LFMM_OK;
}

// File: "LFMMTAB1", then int32 {version 1, p, L, ncomp, npanel, nnode, NT * NC, ndense},
// double k[L+1], d[L], h_lo, h_hi, alpha, u0, du, bound[ncomp*40], then the table
// (ndense * npanel * nnode matrices of NT * NC complex FP64).
static const size_t TAB_IO_CHUNK = (size_t)64 << 20;
int lfmm_tables_save(const lfmm_plan_t* plan, const char* path) {
  if (!plan || !path || !plan->tab.ready) return LFMM_EINVAL;
  const OpTables& T = plan->tab;
  FILE* f = fopen(path, "wb");
  if (!f) return LFMM_EIO;
  const int L = plan->st.L;
  const int32_t hd[8] = {1, plan->p, L, plan->sur.ncomp, T.npanel, T.nnode, plan->NT * plan->NC, T.ndense};
  const double geo[5] = {T.h_lo, T.h_hi, T.alpha, T.u0, T.du};
  bool ok = fwrite("LFMMTAB1", 1, 8, f) == 8 && fwrite(hd, sizeof(hd), 1, f) == 1 &&
            fwrite(plan->st.k, sizeof(double), L + 1, f) == (size_t)(L + 1) &&
            (L == 0 || fwrite(plan->st.d, sizeof(double), L, f) == (size_t)L) && fwrite(geo, sizeof(geo), 1, f) == 1 &&
            fwrite(T.bound.data(), sizeof(double), T.bound.size(), f) == T.bound.size();
  std::vector<char> buf;
  for (size_t off = 0; ok && off < T.tab.cap; off += TAB_IO_CHUNK) {
    const size_t nb = std::min(TAB_IO_CHUNK, T.tab.cap - off);
    buf.resize(nb);
    ok = hipMemcpy(buf.data(), (const char*)T.tab.p + off, nb, hipMemcpyDeviceToHost) == hipSuccess &&
         fwrite(buf.data(), 1, nb, f) == nb;
  }
  if (fclose(f) != 0) ok = false;
  return ok ? LFMM_OK : LFMM_EIO;
}

int lfmm_tables_load(lfmm_plan_t* plan, const char* path) {
  if (!plan || !path) return LFMM_EINVAL;
  if (plan->st.L < 1) return LFMM_EINVAL;
  FILE* f = fopen(path, "rb");
  if (!f) return LFMM_EIO;
  const int L = plan->st.L, NL = L + 1;
  char magic[8];
  int32_t hd[8];
  double geo[5];
  std::vector<double> kk(NL), dd(L);
  sur_components(plan);
  const int ncomp = plan->sur.ncomp;
  int ndense = 0;
  for (int c = 0; c < ncomp; c++)
    for (int j = 0; j < 2; j++)
      for (int i = 0; i < 2; i++)
        for (int ri = 0; ri < 10; ri++) ndense += !(i == 0 && j == 0 && kR2[ri] <= 2);
  bool ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, "LFMMTAB1", 8) == 0 && fread(hd, sizeof(hd), 1, f) == 1 &&
            hd[0] == 1 && hd[1] == plan->p && hd[2] == L && hd[3] == ncomp && hd[4] >= 1 && hd[4] <= 4096 &&
            hd[5] >= 2 && hd[5] <= 32 && hd[6] == plan->NT * plan->NC && hd[7] == ndense;
  ok = ok && fread(kk.data(), sizeof(double), NL, f) == (size_t)NL && fread(dd.data(), sizeof(double), L, f) == (size_t)L &&
       fread(geo, sizeof(geo), 1, f) == 1;
  for (int i = 0; ok && i < NL; i++) ok = kk[i] == plan->st.k[i];
  for (int i = 0; ok && i < L; i++) ok = dd[i] == plan->st.d[i];
  ok = ok && geo[1] > geo[0] && geo[0] > 0 && geo[4] > 0 && geo[2] == 4.0 * plan->kmax;
  std::vector<double> bound((size_t)ncomp * 40);
  ok = ok && fread(bound.data(), sizeof(double), bound.size(), f) == bound.size();
  if (!ok) {
    fclose(f);
    return LFMM_EIO;
  }
  OpTables& T = plan->tab;
  (void)hipStreamSynchronize(plan->s2);
  (void)hipDeviceSynchronize();
  T.release();
  const size_t bytes = (size_t)hd[7] * hd[4] * hd[5] * hd[6] * 16;
  if (hipMalloc(&T.tab.p, bytes) != hipSuccess) {
    T.tab.p = nullptr;
    fclose(f);
    return LFMM_ENOMEM;
  }
  T.tab.cap = bytes;
  std::vector<char> buf;
  for (size_t off = 0; ok && off < bytes; off += TAB_IO_CHUNK) {
    const size_t nb = std::min(TAB_IO_CHUNK, bytes - off);
    buf.resize(nb);
    ok = fread(buf.data(), 1, nb, f) == nb &&
         hipMemcpy((char*)T.tab.p + off, buf.data(), nb, hipMemcpyHostToDevice) == hipSuccess;
  }
  char extra;
  ok = ok && fread(&extra, 1, 1, f) == 0;
  fclose(f);
  if (ok) {
    try {
      sur_decay(plan);
    } catch (Fail& fl) {
      T.release();
      return fl.code;
    }
  }
  if (!ok) {
    T.release();
    return LFMM_EIO;
  }
  T.h_lo = geo[0];
  T.h_hi = geo[1];
  T.alpha = geo[2];
  T.u0 = geo[3];
  T.du = geo[4];
  T.npanel = hd[4];
  T.nnode = hd[5];
  T.ndense = hd[7];
  T.bound = bound;
  T.dense.assign((size_t)ncomp * 40, -1);
  int dn = 0;
  for (int c = 0; c < ncomp; c++)
    for (int j = 0; j < 2; j++)
      for (int i = 0; i < 2; i++)
        for (int ri = 0; ri < 10; ri++)
          if (!(i == 0 && j == 0 && kR2[ri] <= 2)) T.dense[sur_combo(c, j, i, ri)] = dn++;
  memset(&T.rep, 0, sizeof(T.rep));
  T.version++;
  T.ready = true;
  return LFMM_OK;
}

int lfmm_mlp_forward_backward(int B, int nin, int width, int nhidden, int nout, const float* x, const float* params,
                              const float* t, float* y, float* grad, double* loss) {
  if (B < 1 || nin < 1 || width < 1 || nhidden < 0 || nout < 1 || B > 65536 || nin > 4096 || width > 4096 ||
      nhidden > 16 || nout > 65536 || !x || !params || !t || !y || !grad || !loss)
    return LFMM_EINVAL;
  MlpNet N;
  int rc = LFMM_OK;
  try {
    N.setup(nin, width, nhidden, nout);
    N.load_params(params, nullptr);
    float* dxf = N.dev<float>("xf", (size_t)B * nin);
    unsigned short* dx = N.dev<unsigned short>("x", (size_t)B * nin);
    float* dt = N.dev<float>("t", (size_t)B * nout);
    double* dl = N.dev<double>("loss", 1);
    HIPCHK(hipMemcpy(dxf, x, sizeof(float) * B * nin, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(dt, t, sizeof(float) * B * nout, hipMemcpyHostToDevice));
    lk_f2bf((long)B * nin, dxf, dx, nullptr);
    N.forward(B, dx, nullptr);
    N.backward(B, dx, dt, nout, dl, nullptr);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpy(y, N.y(B), sizeof(float) * B * nout, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(grad, N.dev<float>("g", N.np), sizeof(float) * N.np, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(loss, dl, sizeof(double), hipMemcpyDeviceToHost));
  } catch (Fail& f) {
    rc = f.code;
  }
  N.release();
  return rc;
}

int lfmm_set_tiles(lfmm_plan_t* plan, int gemm_ks, int p2p_ta, int p2p_ch) {
  if (!plan) return LFMM_EINVAL;
  if (gemm_ks != 1 && gemm_ks != 2 && gemm_ks != 4 && gemm_ks != 8) return LFMM_EINVAL;
  if (p2p_ta != 4 && p2p_ta != 8 && p2p_ta != 16) return LFMM_EINVAL;
  if (p2p_ch != 128 && p2p_ch != 256 && p2p_ch != 512) return LFMM_EINVAL;
  plan->gemm_ks = gemm_ks;
  plan->p2p_ta = p2p_ta;
  plan->p2p_ch = p2p_ch;
  return LFMM_OK;
}

int lfmm_autotune(lfmm_plan_t* plan, int64_t n, const double* xyz, const int32_t* layer, const double* q, double* phi,
                  void* stream, lfmm_tune_report* rep) {
  if (!plan) return LFMM_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  lfmm_tune_report R;
  memset(&R, 0, sizeof(R));
  auto timed = [&](double* ms) -> int {
    int rc = eval_impl(plan, n, xyz, layer, q, phi, s);  // warm-up (sizes buffers)
    if (rc != LFMM_OK) return rc;
    double best = 1e300;
    for (int r = 0; r < 2; r++) {
      if (hipStreamSynchronize(s) != hipSuccess) return LFMM_EHIP;
      auto t0 = std::chrono::steady_clock::now();
      rc = eval_impl(plan, n, xyz, layer, q, phi, s);
      if (rc != LFMM_OK) return rc;
      if (hipStreamSynchronize(s) != hipSuccess) return LFMM_EHIP;
      best = std::min(best, std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count());
    }
    R.trials += 3;
    *ms = best;
    return LFMM_OK;
  };
  const int ks0 = plan->gemm_ks > 0 ? plan->gemm_ks : 4, ta0 = plan->p2p_ta, ch0 = plan->p2p_ch;
  plan->gemm_ks = ks0;
  double best;
  int rc = timed(&best);
  if (rc != LFMM_OK) return rc;
  R.ms_default = best;
  int bks = ks0, bta = ta0, bch = ch0;
  for (int ks : {1, 2, 4, 8}) {
    if (ks == ks0) continue;
    plan->gemm_ks = ks;
    double ms;
    if ((rc = timed(&ms)) != LFMM_OK) break;
    if (ms < best) {
      best = ms;
      bks = ks;
    }
  }
  plan->gemm_ks = bks;
  if (rc == LFMM_OK && plan->prec == 0) {
    const int shapes[][2] = {{4, 256}, {16, 256}, {8, 128}, {8, 512}, {4, 128}, {16, 512}};
    for (auto& sh : shapes) {
      if (sh[0] == ta0 && sh[1] == ch0) continue;
      plan->p2p_ta = sh[0];
      plan->p2p_ch = sh[1];
      double ms;
      if ((rc = timed(&ms)) != LFMM_OK) break;
      if (ms < best) {
        best = ms;
        bta = sh[0];
        bch = sh[1];
      }
    }
  }
  plan->p2p_ta = bta;
  plan->p2p_ch = bch;
  if (rc != LFMM_OK) {  // keep the defaults after a failure
    plan->gemm_ks = ks0;
    plan->p2p_ta = ta0;
    plan->p2p_ch = ch0;
    return rc;
  }
  if ((rc = eval_impl(plan, n, xyz, layer, q, phi, s)) != LFMM_OK) return rc;
  R.gemm_ks = plan->gemm_ks;
  R.p2p_ta = plan->p2p_ta;
  R.p2p_ch = plan->p2p_ch;
  R.ms_best = best;
  if (rep) *rep = R;
  return LFMM_OK;
}

}  // extern "C"
