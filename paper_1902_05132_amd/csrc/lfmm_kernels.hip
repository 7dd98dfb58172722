// HIP kernels of the layered-media Helmholtz FMM for gfx950 (MI355X).
//
// Stages (paper Section 3.4, Algorithm 1 per reaction component plus the classic
// FMM per free-space layer): layer classification, octree construction on
// Morton keys, operator generation (free-space translations from the addition
// theorems of Section 2.1; reaction M2L operators from the Sommerfeld-type
// integrals of Section 3.5 by contour quadrature), P2M, M2M / M2L / L2L as
// batched complex GEMMs on FP64 MFMA, L2P, near-field sums.
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <type_traits>

#include "lfmm_internal.h"

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

__constant__ double c_glx[LFMM_NGL];
__constant__ double c_glw[LFMM_NGL];
// three-term recurrence coefficients of Phat_n^m (Section 2.2): a_n^m, b_n^m, and the
// diagonal factors sqrt((2m+1)/(2m)); index n * 16 + m, n, m <= 15
__constant__ double c_la[256];
__constant__ double c_lb[256];
__constant__ double c_ld[16];

extern "C" void lk_set_gl(const double* x, const double* w) {
  (void)hipMemcpyToSymbol(HIP_SYMBOL(c_glx), x, sizeof(double) * LFMM_NGL);
  (void)hipMemcpyToSymbol(HIP_SYMBOL(c_glw), w, sizeof(double) * LFMM_NGL);
  double la[256], lb[256], ld[16];
  for (int n = 0; n < 16; n++) {
    ld[n] = n > 0 ? sqrt((2.0 * n + 1.0) / (2.0 * n)) : 1.0;
    for (int m = 0; m < 16; m++) {
      double a = 0.0, b = 0.0;
      if (n > m) a = sqrt((2.0 * n - 1.0) * (2.0 * n + 1.0) / ((double)(n - m) * (n + m)));
      if (n > m + 1) b = sqrt((2.0 * n + 1.0) * (n - m - 1.0) * (n + m - 1.0) / ((2.0 * n - 3.0) * (n + m) * (double)(n - m)));
      la[n * 16 + m] = a;
      lb[n * 16 + m] = b;
    }
  }
  (void)hipMemcpyToSymbol(HIP_SYMBOL(c_la), la, sizeof(la));
  (void)hipMemcpyToSymbol(HIP_SYMBOL(c_lb), lb, sizeof(lb));
  (void)hipMemcpyToSymbol(HIP_SYMBOL(c_ld), ld, sizeof(ld));
}

static inline int nblk(size_t n, int b) { return (int)((n + b - 1) / b); }

// ---------------------------------------------------------------------------
// Utilities
// ---------------------------------------------------------------------------
__global__ void k_zero(double* p, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0.0;
}
__global__ void k_fill_int(int* p, size_t n, int v) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}
extern "C" void lk_zero(double* p, size_t n, hipStream_t s) {
  if (n == 0) return;
  int g = (int)((n + 255) / 256);
  if (g > 65536) g = 65536;
  k_zero<<<g, 256, 0, s>>>(p, n);
}
extern "C" void lk_fill_int(int* p, size_t n, int v, hipStream_t s) {
  if (n == 0) return;
  int g = (int)((n + 255) / 256);
  if (g > 65536) g = 65536;
  k_fill_int<<<g, 256, 0, s>>>(p, n, v);
}

__device__ __forceinline__ unsigned morton3(unsigned ix, unsigned iy, unsigned iz) {
  unsigned c = 0;
  for (int b = 0; b < 8; b++) {
    c |= ((ix >> b) & 1u) << (3 * b + 2);
    c |= ((iy >> b) & 1u) << (3 * b + 1);
    c |= ((iz >> b) & 1u) << (3 * b);
  }
  return c;
}
__device__ __forceinline__ void demorton3(unsigned c, int l, int* ix, int* iy, int* iz) {
  unsigned x = 0, y = 0, z = 0;
  for (int b = 0; b < l; b++) {
    x |= ((c >> (3 * b + 2)) & 1u) << b;
    y |= ((c >> (3 * b + 1)) & 1u) << b;
    z |= ((c >> (3 * b)) & 1u) << b;
  }
  *ix = (int)x;
  *iy = (int)y;
  *iz = (int)z;
}
__device__ __forceinline__ int axis_cell(double v, double lo, double S) {
  double u = (v - lo) / S;
  double f = floor(u * 256.0);
  if (f < 0.0) return 0;
  if (f > 255.0) return 255;
  return (int)f;
}
__device__ __forceinline__ int half_cell(double h, double S) {
  double u = h / S;
  double f = floor(u * 256.0);
  if (f < 0.0) return 0;
  if (f > 127.0) return 127;
  return (int)f;
}
__device__ __forceinline__ double layer_h(const Stack& st, int l, int dir, double z) {
  return dir == 0 ? z - st.d[l] : st.d[l - 1] - z;
}
__device__ __forceinline__ int tree_of(const TreeInfo* trees, int ntrees, int g) {
  int t = 0;
  while (t + 1 < ntrees && g >= trees[t + 1].pt_off) t++;
  return t;
}
// frame coordinates of a tree point (free: physical; reaction target: +height; source: -depth)
__device__ __forceinline__ void frame_xyz(const TreeInfo& T, const Stack& st, double x, double y, double z,
                                          double* fx, double* fy, double* fz) {
  *fx = x;
  *fy = y;
  if (T.kind == 0) *fz = z;
  else if (T.kind == 1) *fz = layer_h(st, T.layer, T.dir, z);
  else *fz = -layer_h(st, T.layer, T.dir, z);
}
__device__ __forceinline__ void box_center(const TreeInfo& T, unsigned code, int l, double* c) {
  int ix, iy, iz;
  demorton3(code, l, &ix, &iy, &iz);
  double h = T.S / (double)(1 << l);
  c[0] = T.lo[0] + (ix + 0.5) * h;
  c[1] = T.lo[1] + (iy + 0.5) * h;
  c[2] = (T.kind == 0) ? T.lo[2] + (iz + 0.5) * h : (iz + 0.5) * h - 0.5 * T.S;
}

// ---------------------------------------------------------------------------
// Layer classification and per-layer statistics
// stats per layer: 0 count, 1/2 x min/max, 3/4 y, 5/6 z, 7/8 up-height min/max,
// 9/10 down-height min/max, 11 invalid count
// ---------------------------------------------------------------------------
#define NSTAT LFMM_NSTAT
__global__ __launch_bounds__(256) void k_classify(int n, const double* x, const double* y, const double* z,
                                                  const int* lin, int* lout, Stack st, double* partial) {
  __shared__ double red[256];
  int L = st.L;
  double v[NSTAT];
  for (int l = 0; l <= L; l++) {
    double cnt = 0, bad = 0;
    double xmn = INFINITY, xmx = -INFINITY, ymn = INFINITY, ymx = -INFINITY, zmn = INFINITY, zmx = -INFINITY;
    double umn = INFINITY, umx = -INFINITY, dmn = INFINITY, dmx = -INFINITY;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
      double zi = z[i];
      int lc = 0;
      for (int j = 0; j < L; j++) lc += (zi < st.d[j]) ? 1 : 0;
      bool ok = isfinite(x[i]) && isfinite(y[i]) && isfinite(zi);
      for (int j = 0; j < L; j++) ok = ok && (zi != st.d[j]);
      if (lin && lin[i] != lc) ok = false;
      if (l == 0) lout[i] = ok ? lc : -1;
      if (!ok) {
        if (l == 0) bad += 1;
        continue;
      }
      if (lc != l) continue;
      cnt += 1;
      xmn = fmin(xmn, x[i]); xmx = fmax(xmx, x[i]);
      ymn = fmin(ymn, y[i]); ymx = fmax(ymx, y[i]);
      zmn = fmin(zmn, zi); zmx = fmax(zmx, zi);
      if (l <= L - 1) { double h = zi - st.d[l]; umn = fmin(umn, h); umx = fmax(umx, h); }
      if (l >= 1) { double h = st.d[l - 1] - zi; dmn = fmin(dmn, h); dmx = fmax(dmx, h); }
    }
    v[0] = cnt; v[1] = xmn; v[2] = xmx; v[3] = ymn; v[4] = ymx; v[5] = zmn; v[6] = zmx;
    v[7] = umn; v[8] = umx; v[9] = dmn; v[10] = dmx; v[11] = bad;
    for (int s = 0; s < NSTAT; s++) {
      bool ismin = (s == 1 || s == 3 || s == 5 || s == 7 || s == 9);
      bool ismax = (s == 2 || s == 4 || s == 6 || s == 8 || s == 10);
      red[threadIdx.x] = v[s];
      __syncthreads();
      for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
          double a = red[threadIdx.x], b = red[threadIdx.x + w];
          red[threadIdx.x] = ismin ? fmin(a, b) : ismax ? fmax(a, b) : a + b;
        }
        __syncthreads();
      }
      if (threadIdx.x == 0) partial[((size_t)blockIdx.x * (L + 1) + l) * NSTAT + s] = red[0];
      __syncthreads();
    }
  }
}
// one wave per (layer, statistic): lanes stride over the per-block partials
__global__ __launch_bounds__(64) void k_reduce_stats(int nblocks, int nl, const double* partial, double* stats) {
  int idx = blockIdx.x, lane = threadIdx.x;
  int s = idx % NSTAT;
  bool ismin = (s == 1 || s == 3 || s == 5 || s == 7 || s == 9);
  bool ismax = (s == 2 || s == 4 || s == 6 || s == 8 || s == 10);
  double acc = ismin ? INFINITY : ismax ? -INFINITY : 0.0;
  for (int b = lane; b < nblocks; b += 64) {
    double v = partial[(size_t)b * nl * NSTAT + idx];
    acc = ismin ? fmin(acc, v) : ismax ? fmax(acc, v) : acc + v;
  }
  for (int off = 32; off > 0; off >>= 1) {
    double v = __shfl_xor(acc, off, 64);
    acc = ismin ? fmin(acc, v) : ismax ? fmax(acc, v) : acc + v;
  }
  if (lane == 0) stats[idx] = acc;
}
extern "C" void lk_classify(int n, const double* x, const double* y, const double* z, const int* lin, int* lout,
                            Stack st, double* partial, int nblocks, hipStream_t s) {
  k_classify<<<nblocks, 256, 0, s>>>(n, x, y, z, lin, lout, st, partial);
}
extern "C" void lk_reduce_stats(int nblocks, int nl, const double* partial, double* stats, hipStream_t s) {
  k_reduce_stats<<<nl * NSTAT, 64, 0, s>>>(nblocks, nl, partial, stats);
}

// ---------------------------------------------------------------------------
// Stable partition of the particles by layer (a counting sort: at most LFMM_MAXL + 1
// layers).  Block b holds particles [256 b, 256 b + 256).  k_layer_count writes each
// layer's count per block, cnt[l * nb + b]; an exclusive scan of that layer-major
// array gives every (layer, block) its first output slot; k_layer_scatter puts each
// particle at that slot plus its rank among the block's earlier particles of its
// layer (wave ballots, then the earlier waves' counts).  Layers are in [0, NL).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_layer_count(int n, int NL, const int* layer, int* cnt) {
  __shared__ int wc[4][LFMM_MAXL + 1];
  const int i = blockIdx.x * 256 + threadIdx.x, wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int my = i < n ? layer[i] : -1;
  for (int l = 0; l < NL; l++) {
    const unsigned long long m = __ballot(my == l);
    if (lane == 0) wc[wave][l] = __popcll(m);
  }
  __syncthreads();
  if (threadIdx.x < NL) {
    const int l = threadIdx.x;
    cnt[(size_t)l * gridDim.x + blockIdx.x] = wc[0][l] + wc[1][l] + wc[2][l] + wc[3][l];
  }
}
__global__ __launch_bounds__(256) void k_layer_scatter(int n, int NL, const int* layer, const int* off, int* perm,
                                                       int* inv) {
  __shared__ int wc[4][LFMM_MAXL + 1];
  const int i = blockIdx.x * 256 + threadIdx.x, wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int my = i < n ? layer[i] : -1;
  const unsigned long long below = lane ? (~0ull >> (64 - lane)) : 0ull;
  int rank = 0;
  for (int l = 0; l < NL; l++) {
    const unsigned long long m = __ballot(my == l);
    if (my == l) rank = __popcll(m & below);
    if (lane == 0) wc[wave][l] = __popcll(m);
  }
  __syncthreads();
  if (i < n) {
    int pos = off[(size_t)my * gridDim.x + blockIdx.x] + rank;
    for (int w = 0; w < wave; w++) pos += wc[w][my];
    perm[pos] = i;
    inv[i] = pos;
  }
}
extern "C" void lk_layer_count(int n, int NL, const int* layer, int* cnt, hipStream_t s) {
  if (n) k_layer_count<<<nblk(n, 256), 256, 0, s>>>(n, NL, layer, cnt);
}
extern "C" void lk_layer_scatter(int n, int NL, const int* layer, const int* off, int* perm, int* inv,
                                 hipStream_t s) {
  if (n) k_layer_scatter<<<nblk(n, 256), 256, 0, s>>>(n, NL, layer, off, perm, inv);
}

__global__ void k_dbg_dens(int n, const double* kr, Stack st, int l, int lp, double* out) {
  int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  cd sig[2][2];
  dev_densities(st, mk(kr[2 * i], kr[2 * i + 1]), l, lp, sig);
  for (int a = 0; a < 2; a++)
    for (int b = 0; b < 2; b++) {
      out[8 * i + 2 * (2 * a + b)] = sig[a][b].x;
      out[8 * i + 2 * (2 * a + b) + 1] = sig[a][b].y;
    }
}
extern "C" void lk_dbg_dens(int n, const double* kr, Stack st, int l, int lp, double* out, hipStream_t s) {
  if (n) k_dbg_dens<<<nblk(n, 256), 256, 0, s>>>(n, kr, st, l, lp, out);
}

// ---------------------------------------------------------------------------
// Tree points: keys = (tree << 24) | Morton code of the depth-8 cell
// ---------------------------------------------------------------------------
// Each tree point also gets its record (frame x, y, z, Re q, Im q) here, in tree
// point order: the gather into sorted order then reads one 40-byte record per
// point instead of following the layer permutation into five separate arrays.
__global__ void k_tree_points(int ntp, int ntrees, const TreeInfo* trees, const int* perm, const int* layer_start,
                              const double* x, const double* y, const double* z, const double* q, Stack st,
                              unsigned* keys, int* vals, double* rec) {
  int g = blockIdx.x * 256 + threadIdx.x;
  if (g >= ntp) return;
  int t = tree_of(trees, ntrees, g);
  TreeInfo T = trees[t];
  int i = perm[layer_start[T.layer] + (g - T.pt_off)];
  double fx, fy, fz;
  frame_xyz(T, st, x[i], y[i], z[i], &fx, &fy, &fz);
  int ix = axis_cell(fx, T.lo[0], T.S), iy = axis_cell(fy, T.lo[1], T.S), iz;
  if (T.kind == 0) iz = axis_cell(fz, T.lo[2], T.S);
  else if (T.kind == 1) iz = 128 + half_cell(fz, T.S);
  else iz = 127 - half_cell(-fz, T.S);
  keys[g] = ((unsigned)t << 24) | morton3(ix, iy, iz);
  vals[g] = g;
  double* r = rec + 5 * (size_t)g;
  r[0] = fx;
  r[1] = fy;
  r[2] = fz;
  r[3] = q ? q[2 * i] : 0.0;  // no charges yet when only the geometry is prepared
  r[4] = q ? q[2 * i + 1] : 0.0;
}
extern "C" void lk_tree_points(int ntp, int ntrees, const TreeInfo* trees, const int* perm, const int* layer_start,
                               const double* x, const double* y, const double* z, const double* q, Stack st,
                               unsigned* keys, int* vals, double* rec, hipStream_t s) {
  if (ntp)
    k_tree_points<<<nblk(ntp, 256), 256, 0, s>>>(ntp, ntrees, trees, perm, layer_start, x, y, z, q, st, keys, vals,
                                                 rec);
}

// occupancy[t*9 + l] = fullest cell of tree t at level l, capped at leaf_max + 1 (the
// depth rule asks only whether it exceeds leaf_max: one probe leaf_max points ahead
// of a cell's first point answers that); slab flags of reaction trees.
// A workgroup scans a contiguous segment of the sorted keys and keeps its maxima
// and flags in LDS (the keys are sorted by tree, so a segment touches few
// trees); one flush per workgroup then updates the global tables.  A point's two
// probes (its predecessor and the point leaf_max ahead) serve every level, and a
// wave whose points all lie in one tree updates each LDS entry once (by ballots).
#define OCC_SEG 2048
#define OCC_TMAX 96
__global__ __launch_bounds__(256) void k_occupancy(int ntp, int ntrees, const unsigned* skeys, const TreeInfo* trees,
                                                   int leaf_max, int* occ, int* slab) {
  __shared__ int s_occ[OCC_TMAX * 9], s_slab[OCC_TMAX * 18];
  for (int i = threadIdx.x; i < ntrees * 9; i += 256) s_occ[i] = 0;
  for (int i = threadIdx.x; i < ntrees * 18; i += 256) s_slab[i] = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int seg0 = blockIdx.x * OCC_SEG, seg1 = min(ntp, seg0 + OCC_SEG);
  for (int b0 = seg0; b0 < seg1; b0 += 256) {
    // every lane of a wave takes part in the ballots; points past the segment are idle
    const int s = b0 + threadIdx.x;
    const bool valid = s < seg1;
    const unsigned key = valid ? skeys[s] : 0u;
    const int t = (int)(key >> 24);
    const TreeInfo& T = trees[t];
    const int pt0 = T.pt_off, hi = T.pt_off + T.npts;
    const bool has_prev = valid && s > pt0;
    const unsigned prev = has_prev ? skeys[s - 1] : 0u;
    const bool has_far = valid && leaf_max < hi - s;
    const unsigned far = has_far ? skeys[s + leaf_max] : 0u;
    int ix, iy, iz;
    demorton3(key & 0xFFFFFFu, 8, &ix, &iy, &iz);
    const int kind = T.kind;
    const unsigned long long act = __ballot(valid);
    const int t0 = __shfl(t, act ? __ffsll((long long)act) - 1 : 0);
    const bool one_tree = __ballot(valid && t != t0) == 0ull;
    const bool leader = act && lane == __ffsll((long long)act) - 1;
    for (int l = 0; l <= 8; l++) {
      const int sh = 3 * (8 - l);
      const bool first = valid && (!has_prev || (prev >> sh) != (key >> sh));
      const bool full = has_far && (far >> sh) == (key >> sh);
      int hgt = -1;
      if (l >= 1 && kind != 0) {
        const int izl = iz >> (8 - l), half = 1 << (l - 1);
        hgt = (kind == 1) ? izl - half : half - 1 - izl;
      }
      if (one_tree) {
        const unsigned long long bf = __ballot(first), bfull = __ballot(first && full);
        const unsigned long long b0s = __ballot(first && hgt == 0), b1s = __ballot(first && hgt == 1);
        if (leader) {
          if (bf) atomicMax(&s_occ[t0 * 9 + l], bfull ? leaf_max + 1 : 1);
          if (b0s) s_slab[(t0 * 9 + l) * 2] = 1;
          if (b1s) s_slab[(t0 * 9 + l) * 2 + 1] = 1;
        }
      } else if (first) {
        atomicMax(&s_occ[t * 9 + l], full ? leaf_max + 1 : 1);
        if (hgt == 0 || hgt == 1) s_slab[(t * 9 + l) * 2 + hgt] = 1;
      }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < ntrees * 9; i += 256)
    if (s_occ[i] > 0) atomicMax(&occ[i], s_occ[i]);
  for (int i = threadIdx.x; i < ntrees * 18; i += 256)
    if (s_slab[i]) slab[i] = 1;
}
extern "C" void lk_occupancy(int ntp, int ntrees, const unsigned* skeys, const TreeInfo* trees, int leaf_max,
                             int* occ, int* slab, hipStream_t s) {
  if (ntp) k_occupancy<<<(ntp + OCC_SEG - 1) / OCC_SEG, 256, 0, s>>>(ntp, ntrees, skeys, trees, leaf_max, occ, slab);
}

// Box numbering.  Sorted point s opens a box of level l (of its tree, if the tree
// reaches level l) where its key differs from its predecessor's above bit 3 (8 - l);
// the boxes of all levels are numbered in level-major order (all level-0 boxes, then
// level 1, ...), each level in point order.  The flags are not stored: one pass
// counts them per tile of BOX_TILE points and level, one exclusive scan of those
// counts (level-major) gives each tile's first row per level, and the passes that
// need rows recount within the tile.
#define BOX_TILE 2048
__device__ __forceinline__ bool box_opens(const unsigned* skeys, const TreeInfo* trees, int s, int l) {
  const unsigned key = skeys[s];
  if (l > trees[key >> 24].depth) return false;
  const int sh = 3 * (8 - l);
  return s == 0 || (skeys[s - 1] >> sh) != (key >> sh);
}
// cnt[l * ntiles + tile] = boxes of level l opened in the tile; cnt[nlev * ntiles] = 0
__global__ __launch_bounds__(256) void k_box_count(int ntp, int nlev, int ntiles, const unsigned* skeys,
                                                   const TreeInfo* trees, int* cnt) {
  __shared__ int c[9];
  const int lane = threadIdx.x & 63, tile = blockIdx.x;
  if (threadIdx.x < 9) c[threadIdx.x] = 0;
  __syncthreads();
  for (int r = 0; r < BOX_TILE / 256; r++) {
    const int s = tile * BOX_TILE + r * 256 + threadIdx.x;
    const bool valid = s < ntp;
    const unsigned key = valid ? skeys[s] : 0u;
    const unsigned prev = valid && s > 0 ? skeys[s - 1] : 0u;
    const int D = valid ? trees[key >> 24].depth : -1;
    for (int l = 0; l < nlev; l++) {
      const int sh = 3 * (8 - l);
      const bool f = valid && l <= D && (s == 0 || (prev >> sh) != (key >> sh));
      const unsigned long long b = __ballot(f);
      if (lane == 0 && b) atomicAdd(&c[l], __popcll(b));
    }
  }
  __syncthreads();
  if (threadIdx.x < nlev) cnt[(size_t)threadIdx.x * ntiles + tile] = c[threadIdx.x];
  if (tile == 0 && threadIdx.x == 0) cnt[(size_t)nlev * ntiles] = 0;
}
extern "C" int lk_box_tiles(int ntp) { return (ntp + BOX_TILE - 1) / BOX_TILE; }
extern "C" void lk_box_count(int ntp, int nlev, const unsigned* skeys, const TreeInfo* trees, int* cnt,
                             hipStream_t s) {
  const int nt = lk_box_tiles(ntp);
  if (nt && nlev) k_box_count<<<nt, 256, 0, s>>>(ntp, nlev, nt, skeys, trees, cnt);
}
// global row of the first level-l box opened at or after point pos (pos <= ntp):
// the tile's first row plus the boxes opened in the tile before pos
__device__ int box_row_at(const unsigned* skeys, const TreeInfo* trees, const int* off, int ntiles, int l, int pos,
                          int* red) {
  const int tile = pos / BOX_TILE, t0 = tile * BOX_TILE;
  int n = 0;
  for (int s = t0 + (int)threadIdx.x; s < pos; s += 256) n += box_opens(skeys, trees, s, l) ? 1 : 0;
  red[threadIdx.x] = n;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const int r = off[(size_t)l * ntiles + tile] + red[0];
  __syncthreads();
  return r;
}
// per (tree, level < 9): first box (level-local) and number of boxes (zeros past the
// tree's depth or the last level); one workgroup each
__global__ __launch_bounds__(256) void k_tree_box_range_all(int ntrees, int nlev, int ntp, const unsigned* skeys,
                                                            const TreeInfo* trees, const int* off, int* tb) {
  __shared__ int red[256];
  const int t = blockIdx.x / 9, level = blockIdx.x % 9;
  const int ntiles = (ntp + BOX_TILE - 1) / BOX_TILE;
  const TreeInfo T = trees[t];
  int first = 0, cnt = 0;
  if (ntp > 0 && T.npts > 0 && level < nlev && level <= T.depth) {
    const int r0 = box_row_at(skeys, trees, off, ntiles, level, T.pt_off, red);
    const int r1 = box_row_at(skeys, trees, off, ntiles, level, T.pt_off + T.npts, red);
    first = r0 - off[(size_t)level * ntiles];
    cnt = r1 - r0;
  }
  if (threadIdx.x == 0) {
    tb[(t * 9 + level) * 2] = first;
    tb[(t * 9 + level) * 2 + 1] = cnt;
  }
}
extern "C" void lk_tree_box_range_all(int ntrees, int nlev, int ntp, const unsigned* skeys, const TreeInfo* trees,
                                      const int* off, int* tb, hipStream_t s) {
  if (ntrees) k_tree_box_range_all<<<ntrees * 9, 256, 0, s>>>(ntrees, nlev, ntp, skeys, trees, off, tb);
}
// Box records (first point, Morton code at its level, tree, level) of every box, and
// each point's leaf row (its box at its tree's depth); one workgroup per (tile,
// level).  The point counts follow from the next box's first point (k_grid_fill_all).
__global__ __launch_bounds__(256) void k_box_fill_all(int ntp, int nlev, const unsigned* skeys, const int* off,
                                                      const TreeInfo* trees, int* box_start, int* box_code,
                                                      int* box_tree, int* box_level, int* leafrow) {
  __shared__ int wc[4];
  const int tile = blockIdx.x, level = blockIdx.y, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ntiles = gridDim.x, sh = 3 * (8 - level);
  const unsigned long long below = lane ? (~0ull >> (64 - lane)) : 0ull;
  int run = off[(size_t)level * ntiles + tile];
  for (int r = 0; r < BOX_TILE / 256; r++) {
    const int s = tile * BOX_TILE + r * 256 + threadIdx.x;
    const bool valid = s < ntp;
    const unsigned key = valid ? skeys[s] : 0u;
    const int t = key >> 24;
    const int D = valid ? trees[t].depth : -1;
    const bool f = valid && level <= D && (s == 0 || (skeys[s - 1] >> sh) != (key >> sh));
    const unsigned long long b = __ballot(f);
    if (lane == 0) wc[wave] = __popcll(b);
    __syncthreads();
    int R = run + __popcll(b & below);
    for (int w = 0; w < wave; w++) R += wc[w];
    if (f) {
      box_start[R] = s;
      box_code[R] = (int)((key & 0xFFFFFFu) >> sh);
      box_tree[R] = t;
      box_level[R] = level;
    }
    if (valid && D == level) leafrow[s] = R + (f ? 1 : 0) - 1;
    run += wc[0] + wc[1] + wc[2] + wc[3];
    __syncthreads();
  }
}
extern "C" void lk_box_fill_all(int ntp, int nlev, const unsigned* skeys, const int* off, const TreeInfo* trees,
                                int* box_start, int* box_code, int* box_tree, int* box_level, int* leafrow,
                                hipStream_t s) {
  const int nt = lk_box_tiles(ntp);
  if (nt && nlev)
    k_box_fill_all<<<dim3(nt, nlev), 256, 0, s>>>(ntp, nlev, skeys, off, trees, box_start, box_code, box_tree,
                                                   box_level, leafrow);
}
// Each box's point count (a box ends where the next box of its tree and level starts,
// or at the tree's last point) and its row in the dense cell -> row grid.
__global__ void k_grid_fill_all(int nrows, const int* box_start, const int* box_code, const int* box_tree,
                                const int* box_level, const TreeInfo* trees, const long long* grid_off, int* grid,
                                int* box_cnt) {
  const int R = blockIdx.x * 256 + threadIdx.x;
  if (R >= nrows) return;
  const int t = box_tree[R], l = box_level[R];
  const bool next = R + 1 < nrows && box_tree[R + 1] == t && box_level[R + 1] == l;
  box_cnt[R] = (next ? box_start[R + 1] : trees[t].pt_off + trees[t].npts) - box_start[R];
  const long long go = grid_off[t * 9 + l];
  if (go < 0) return;
  grid[go + box_code[R]] = R;
}
extern "C" void lk_grid_fill_all(int nrows, const int* box_start, const int* box_code, const int* box_tree,
                                 const int* box_level, const TreeInfo* trees, const long long* grid_off, int* grid,
                                 int* box_cnt, hipStream_t s) {
  if (nrows)
    k_grid_fill_all<<<nblk(nrows, 256), 256, 0, s>>>(nrows, box_start, box_code, box_tree, box_level, trees,
                                                      grid_off, grid, box_cnt);
}

// tree point records into Morton-sorted order, split into coordinate and charge arrays
__global__ void k_gather(int ntp, const int* sg, const double* rec, double* px, double* py, double* pz, double* pq) {
  int s = blockIdx.x * 256 + threadIdx.x;
  if (s >= ntp) return;
  const double* r = rec + 5 * (size_t)sg[s];
  double fx = r[0], fy = r[1], fz = r[2], qr = r[3], qi = r[4];
  px[s] = fx;
  py[s] = fy;
  pz[s] = fz;
  pq[2 * s] = qr;
  pq[2 * s + 1] = qi;
}
extern "C" void lk_gather(int ntp, const int* sg, const double* rec, double* px, double* py, double* pz, double* pq,
                          hipStream_t s) {
  if (ntp) k_gather<<<nblk(ntp, 256), 256, 0, s>>>(ntp, sg, rec, px, py, pz, pq);
}

// particle index of every tree point in tree order (the particle whose charge it carries)
__global__ void k_point_origin(int ntp, int ntrees, const TreeInfo* trees, const int* perm, const int* layer_start,
                               const int* sg, int* orig) {
  int s = blockIdx.x * 256 + threadIdx.x;
  if (s >= ntp) return;
  const int g = sg[s];
  const TreeInfo& T = trees[tree_of(trees, ntrees, g)];
  orig[s] = perm[layer_start[T.layer] + (g - T.pt_off)];
}
extern "C" void lk_point_origin(int ntp, int ntrees, const TreeInfo* trees, const int* perm, const int* layer_start,
                                const int* sg, int* orig, hipStream_t s) {
  if (ntp) k_point_origin<<<nblk(ntp, 256), 256, 0, s>>>(ntp, ntrees, trees, perm, layer_start, sg, orig);
}

// tree-order charges from the particles' charges
__global__ void k_gather_q(int ntp, const int* orig, const double* q, double* pq) {
  int s = blockIdx.x * 256 + threadIdx.x;
  if (s >= ntp) return;
  const int i = orig[s];
  pq[2 * s] = q[2 * i];
  pq[2 * s + 1] = q[2 * i + 1];
}
extern "C" void lk_gather_q(int ntp, const int* orig, const double* q, double* pq, hipStream_t s) {
  if (ntp) k_gather_q<<<nblk(ntp, 256), 256, 0, s>>>(ntp, orig, q, pq);
}

// ---------------------------------------------------------------------------
// Operator layout for the MFMA GEMM: an (NRT*16) x (NKS*4) complex matrix is
// stored as tiles of 16 rows x 4 columns; tile (rt, ks) holds 64 (re, im) pairs
// in MFMA A-operand lane order (lane = row%16 + 16*(col%4)), so each lane loads
// its operand with one 128-bit load.  Padding rows/columns are zero.
// ---------------------------------------------------------------------------
__device__ __forceinline__ size_t packed_pos(int row, int col, int NKS) {
  return ((size_t)((row >> 4) * NKS + (col >> 2)) << 7) + 2 * (size_t)((row & 15) | ((col & 3) << 4));
}
__device__ __forceinline__ void decode_nm(int r, int* n, int* m) {
  int nn = (int)floor(sqrt((double)r) + 1e-9);
  while (nn * nn > r) nn--;
  while ((nn + 1) * (nn + 1) <= r) nn++;
  *n = nn;
  *m = r - nn * nn - nn;
}
// (n, m) of every index idx(n, m) < NC, in LDS (one entry per thread, then a barrier)
#define NM_TAB 128
__device__ __forceinline__ void fill_nm(int NC, int2* tab) {
  for (int r = threadIdx.x; r < NC; r += blockDim.x) {
    int n, m;
    decode_nm(r, &n, &m);
    tab[r] = make_int2(n, m);
  }
}
// Entry e of an operator in the FP32 M2L layout (k-step major; see m2l32_nrt):
// k-step e / SZ, then within it the NRT tiles in lane order and the last row.
__device__ __forceinline__ void m2l_packed_rc(int e, int NRT, int XR, int* row, int* col) {
  const int SZ = NRT * 64 + 4 * XR, ks = e / SZ, r = e - ks * SZ;
  if (r < NRT * 64) {
    *row = (r >> 6) * 16 + (r & 15);
    *col = ks * 4 + ((r & 63) >> 4);
  } else {
    *row = NRT * 16;
    *col = ks * 4 + (r - NRT * 64);
  }
}

// Free-space translation operators (Section 2.1 addition theorems):
//   Op[(n,m),(nu,mu)] = 4 pi i^{n-nu} sum_q i^q z_q(k|b|) conj(Y_q^{m-mu}(b^)) G(nu,mu; q,m-mu; n)
// G tabulated per (row, col, j), q = |n - nu| + 2 j.  One workgroup per operator.
// With ops32 given, singular (M2L) operators are written in FP32 to ops32 instead,
// scaled as Op[(n,m),(nu,mu)] 2^{-(e_t n + e_s nu)} with (e_t, e_s) = opse[op] (the
// per-level expansion scale exponents of the FP32 path).
__global__ __launch_bounds__(256) void k_transop(const OpDesc* descs, double* sops, int opsz, double* ops, int opsz_m,
                                                 int p, int NC, int NKS, const double* gaunt, float* ops32,
                                                 const int2* opse) {
  __shared__ cd zq[64];
  __shared__ cd Yq[(2 * LFMM_PMAX + 1) * (2 * LFMM_PMAX + 1)];  // idx(q, s), q <= 2p
  __shared__ int2 nmt[NM_TAB];
  OpDesc D = descs[blockIdx.x];
  fill_nm(NC, nmt);
  int Q = 2 * p;
  double bb = sqrt(D.bx * D.bx + D.by * D.by + D.bz * D.bz);
  __shared__ double jj[64];
  if (threadIdx.x == 0) {
    double x = D.k * bb;
    dev_sph_j(Q, x, jj);
    if (D.kind == 0) {
      for (int q = 0; q <= Q; q++) zq[q] = mk(jj[q], 0);
    } else {
      double sn, cs;
      sincos(x, &sn, &cs);
      double y0 = -cs / x, y1 = -cs / (x * x) - sn / x;
      zq[0] = mk(jj[0], y0);
      if (Q >= 1) zq[1] = mk(jj[1], y1);
      for (int n = 1; n < Q; n++) {
        double y2 = (2.0 * n + 1.0) / x * y1 - y0;
        y0 = y1;
        y1 = y2;
        zq[n + 1] = mk(jj[n + 1], y1);
      }
    }
  }
  int m = threadIdx.x;
  if (m <= Q) {
    double ct = D.bz / bb, st = sqrt(D.bx * D.bx + D.by * D.by) / bb;
    double ph = atan2(D.by, D.bx);
    double pmm = 0.28209479177387814347;
    for (int mm = 1; mm <= m; mm++) pmm *= sqrt((2.0 * mm + 1.0) / (2.0 * mm)) * st;
    double sn, cs;
    sincos(m * ph, &sn, &cs);
    double sgn = (m & 1) ? -1.0 : 1.0;
    double p0 = pmm, p1 = 0.0;
    for (int q = m; q <= Q; q++) {
      double val;
      if (q == m) val = pmm;
      else if (q == m + 1) { p1 = sqrt(2.0 * m + 3.0) * ct * pmm; val = p1; }
      else {
        double a = sqrt((2.0 * q - 1.0) * (2.0 * q + 1.0) / ((double)(q - m) * (q + m)));
        double b = sqrt((2.0 * q + 1.0) * (q - m - 1.0) * (q + m - 1.0) / ((2.0 * q - 3.0) * (q + m) * (double)(q - m)));
        double p2 = a * ct * p1 - b * p0;
        p0 = p1;
        p1 = p2;
        val = p2;
      }
      Yq[cidx(q, m)] = mk(val * cs, val * sn);
      if (m > 0) Yq[cidx(q, -m)] = mk(sgn * val * cs, -sgn * val * sn);
    }
  }
  __syncthreads();
  // shift operators (regular) in their own array; M2L operators (singular) in the
  // M2L array, FP32 when one is given; both in the GEMMs' k-step-major layout
  const bool f32 = ops32 != nullptr && D.kind == 1;
  double* out = D.kind == 0 ? sops + (size_t)D.op * opsz : (f32 ? nullptr : ops + (size_t)D.op * opsz_m);
  float* out32 = f32 ? ops32 + (size_t)D.op * opsz_m : nullptr;
  const int2 se = f32 ? opse[D.op] : make_int2(0, 0);
  int P1 = p + 1;
  const int nrtl = m2l_nrt(NC), xrl = m2l_xr(NC);
  const int ntot = NKS * (nrtl * 64 + 4 * xrl);
  for (int e = threadIdx.x; e < ntot; e += 256) {
    int row, col;
    m2l_packed_rc(e, nrtl, xrl, &row, &col);
    cd val = mk(0, 0);
    if (row < NC && col < NC) {
      const int n = nmt[row].x, mm = nmt[row].y, nu = nmt[col].x, mu = nmt[col].y;
      int s = mm - mu;
      const double* g = gaunt + ((size_t)row * NC + col) * P1;
      int q0 = abs(n - nu);
      cd acc = mk(0, 0);
      int jmax = (n < nu) ? n : nu;
      for (int j = 0; j <= jmax; j++) {
        int q = q0 + 2 * j;
        if (abs(s) > q) continue;
        double gv = g[j];
        if (gv == 0.0) continue;
        acc = acc + gv * (ipow(q) * zq[q] * cconj(Yq[cidx(q, s)]));
      }
      val = (4.0 * LFMM_PI) * (ipow(n - nu) * acc);
      if (f32) {
        int sh = -(se.x * n + se.y * nu);
        val = mk(ldexp(val.x, sh), ldexp(val.y, sh));
      }
    }
    if (f32) {
      ((float2*)out32)[e] = make_float2((float)val.x, (float)val.y);
    } else {
      ((double2*)out)[e] = make_double2(val.x, val.y);
    }
  }
}
extern "C" void lk_transop(int nops, const OpDesc* descs, double* sops, int opsz, double* ops, int opsz_m, int p,
                           int NC, int NKS, const double* gaunt, float* ops32, const int* opse, hipStream_t s) {
  if (nops)
    k_transop<<<nops, 256, 0, s>>>(descs, sops, opsz, ops, opsz_m, p, NC, NKS, gaunt, ops32, (const int2*)opse);
}

// ---------------------------------------------------------------------------
// Reaction M2L integrals (Section 3.5 eq. (me2lesimplified) in the polarisation
// frame of Section 3.3): for a class (target/source layer and direction, target
// height zt, source depth zs, lateral distance rho)
//   I[(n,m),(n',m')] = int_Gamma k_rho J_q(k_rho rho) e^{i kz_t zt + i kz_s zs}
//                      sigma_ab(k_rho) / kz_t  Phat_n^m(kz_t/k_t) Phat_{n'}^{m'}(kz_s/k_s) dk_rho,
// q = m' - m, by Gauss-Legendre panels on the contour.  Only m >= 0 is
// integrated: Phat_n^{-m} = (-1)^m Phat_n^m and J_{-q} = (-1)^q J_q give the rest.  Classes with the same
// (zt + zs, rho) share the quadrature nodes and J_q, and Phat depends only on
// the layer and the node, so the node tables are built once per rule group:
//   k_react_tables: J_q(k rho) (q = 0..2p) and Phat(kz_l/k_l) for every layer l;
//   k_react_F:      F = w k_rho e^{...} sigma_ab / kz_t per class and node;
//   k_react_mfma:   the node sum as FP64 MFMA products (below).
// ---------------------------------------------------------------------------
// Per-node layer quantities of the density recursion (stacks with more than four
// interfaces, whose densities k_react_F then assembles from them): for every layer
// m, kz_m, the phase E_m over the layer, the generalised reflections Rd_m (looking
// down at d_m) and Ru_m (looking up at d_{m-1}), and the generalised transmissions
// Tu_m (from layer m up into m-1) and Td_m (from m down into m+1), the same
// expressions as dev_densities_t.  Layout: Ltab[(field * (L + 1) + m) * Ntot + node],
// fields LT_KZ, LT_E, LT_RD, LT_RU, LT_TU, LT_TD (zero where a quantity does not exist).
enum { LT_KZ, LT_E, LT_RD, LT_RU, LT_TU, LT_TD, LT_NF };
__device__ void layer_tables_node(const Stack& st, cd kr, int Ntot, int g, cd* Lt) {
  const int L = st.L, NLm = L + 1;
  auto at = [&](int f, int m) -> cd& { return Lt[((size_t)f * NLm + m) * Ntot + g]; };
  const cd kr2 = kr * kr, zero = mk(0, 0), one = mk(1, 0);
  auto kzf = [&](int m) { return csqrtd(mk(st.k[m] * st.k[m], 0) - kr2); };
  auto Ef = [&](int m, cd kz) {
    return (m >= 1 && m <= L - 1) ? cexpd(cmul_i(kz * (st.d[m - 1] - st.d[m]))) : zero;
  };
  for (int m = 0; m <= L; m++) {
    const cd kz = kzf(m);
    at(LT_KZ, m) = kz;
    at(LT_E, m) = Ef(m, kz);
  }
  // looking down: m = L-1 .. 0 from the layer below
  at(LT_RD, L) = zero;
  at(LT_TD, L) = zero;
  {
    cd kzn = kzf(L), an = st.k[L] * kzn, Rdn = zero, En = zero;
    for (int m = L - 1; m >= 0; m--) {
      const cd kz = kzf(m), a = st.k[m] * kz;
      const cd r = (a - an) / (a + an);
      const cd rho = (m + 1 <= L - 1) ? Rdn * En * En : zero;
      const cd Rd = (r + rho) / (one + r * rho);
      at(LT_RD, m) = Rd;
      at(LT_TD, m) = (kzn / kz) * (one + r) / (one + r * rho);
      kzn = kz;
      an = a;
      Rdn = Rd;
      En = Ef(m, kz);
    }
  }
  // looking up: m = 1 .. L from the layer above
  at(LT_RU, 0) = zero;
  at(LT_TU, 0) = zero;
  {
    cd kzp = kzf(0), ap = st.k[0] * kzp, Rup = zero, Ep = zero;
    for (int m = 1; m <= L; m++) {
      const cd kz = kzf(m), a = st.k[m] * kz;
      const cd r = (a - ap) / (a + ap);
      const cd rho = (m - 1 >= 1) ? Rup * Ep * Ep : zero;
      const cd Ru = (r + rho) / (one + r * rho);
      at(LT_RU, m) = Ru;
      at(LT_TU, m) = (kzp / kz) * (one + r) / (one + r * rho);
      kzp = kz;
      ap = a;
      Rup = Ru;
      Ep = Ef(m, kz);
    }
  }
}
__global__ __launch_bounds__(256) void k_react_tables(const RGDesc* rgs, int nrg, int Ntot, Stack st, int p,
                                                      cd* Jtab, cd* Ptab, cd* Ltab) {
  const int NL = st.L + 1, Q = 2 * p, NT = (p + 1) * (p + 2) / 2;
  long long t = (long long)blockIdx.x * 256 + threadIdx.x;
  if (t >= (long long)(NL + (Ltab ? 2 : 1)) * Ntot) return;
  int kind = (int)(t / Ntot), g = (int)(t % Ntot);
  int lo = 0, hi = nrg - 1;  // rule group holding global node g
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (rgs[mid].off <= g) lo = mid;
    else hi = mid - 1;
  }
  const RGDesc R = rgs[lo];
  cd kr, w;
  rule_node(R.rule, g - R.off, c_glx, c_glw, &kr, &w);
  if (kind == 0) {
    dev_besselJ(Q, kr * R.rho, Jtab + (size_t)g * (Q + 1), 1);
  } else if (kind == NL + 1) {
    layer_tables_node(st, kr, Ntot, g, Ltab);
  } else {
    int l = kind - 1;
    double kl = st.k[l];
    cd kz = csqrtd(mk(kl * kl, 0) - kr * kr);
    dev_legendre_c(p, kz / kl, kr / kl, Ptab + ((size_t)l * Ntot + g) * NT, 1);
  }
}
// The F values of all classes are one array (class c's nodes from cls[c].f_off on,
// in class order): one thread per entry, its class by bisection on f_off.
__device__ __forceinline__ int class_of_entry(const ClassDesc* cls, int ncls, int f) {
  int lo = 0, hi = ncls - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (cls[mid].f_off <= f) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}
template <int LL>
__global__ __launch_bounds__(256) void k_react_F(const ClassDesc* cls, int ncls, int Ftot, Stack st, cd* Ftab) {
  const int f = blockIdx.x * 256 + threadIdx.x;
  if (f >= Ftot) return;
  const ClassDesc C = cls[class_of_entry(cls, ncls, f)];
  const int node = f - C.f_off;
  cd kr, w;
  rule_node(C.rule, node, c_glx, c_glw, &kr, &w);
  double kt = st.k[C.lt], ks = st.k[C.ls];
  cd kr2 = kr * kr;
  cd kzt = csqrtd(mk(kt * kt, 0) - kr2), kzs = csqrtd(mk(ks * ks, 0) - kr2);
  // the one density this class needs, as a register value: reading sig with the
  // class's runtime (a, b) would keep the array in memory, which the compiler
  // places in LDS (16 KB per workgroup), so that the kernel could not share CUs
  // with the near field
  cd sig[2][2], sab = mk(0, 0);
  dev_densities_t<LL>(st, kr, C.lt, C.ls, sig, C.a, C.b, &sab);
  cd ex = cexpd(cmul_i(kzt * C.zt + kzs * C.zs));
  Ftab[C.f_off + node] = w * kr * ex * sab / kzt;
}
// k_react_F for stacks with more than four interfaces: the density of the class's
// component from the per-node layer tables (closure in the source layer, then the
// generalised transmissions to the target layer), the same steps as
// dev_densities_t without repeating the recursions for every class of a node.
__global__ __launch_bounds__(256) void k_react_F_lt(const ClassDesc* cls, int ncls, int Ftot, Stack st, int Ntot,
                                                    const cd* Lt, cd* Ftab) {
  const int f = blockIdx.x * 256 + threadIdx.x;
  if (f >= Ftot) return;
  const ClassDesc C = cls[class_of_entry(cls, ncls, f)];
  const int node = f - C.f_off;
  cd kr, w;
  rule_node(C.rule, node, c_glx, c_glw, &kr, &w);
  const int L = st.L, NLm = L + 1, g = C.rg_off + node, l = C.lt, lp = C.ls;
  auto at = [&](int f, int m) { return Lt[((size_t)f * NLm + m) * Ntot + g]; };
  const cd zero = mk(0, 0), one = mk(1, 0);
  const cd kzt = at(LT_KZ, l), kzs = at(LT_KZ, lp);
  const cd Rb = (lp <= L - 1) ? at(LT_RD, lp) : zero, Rt = (lp >= 1) ? at(LT_RU, lp) : zero;
  const cd Ep = (lp >= 1 && lp <= L - 1) ? at(LT_E, lp) : zero;
  const cd Delta = one - Rb * Rt * Ep * Ep;
  const cd Xb = (C.b == 0) ? one : zero, Xt = (C.b == 1) ? one : zero;
  const cd U = Rb * (Xb + Ep * Rt * Xt) / Delta, D = Rt * (Xt + Ep * Rb * Xb) / Delta;
  cd Ul = U, Dl = D;
  if (l < lp) {
    cd Um = Xt + ((lp <= L - 1) ? Ep * U : zero);
    for (int m = lp; m > l; m--) {
      Um = at(LT_TU, m) * Um;
      if (m - 1 > l) Um = at(LT_E, m - 1) * Um;
    }
    Ul = Um;
    Dl = (l >= 1) ? at(LT_RU, l) * at(LT_E, l) * Ul : zero;
  } else if (l > lp) {
    cd Dm = Xb + ((lp >= 1) ? Ep * D : zero);
    for (int m = lp; m < l; m++) {
      Dm = at(LT_TD, m) * Dm;
      if (m + 1 < l) Dm = at(LT_E, m + 1) * Dm;
    }
    Dl = Dm;
    Ul = (l <= L - 1) ? at(LT_RD, l) * at(LT_E, l) * Dl : zero;
  }
  const cd sab = (C.a == 0) ? ((l <= L - 1) ? Ul : zero) : ((l >= 1) ? Dl : zero);
  cd ex = cexpd(cmul_i(kzt * C.zt + kzs * C.zs));
  Ftab[C.f_off + node] = w * kr * ex * sab / kzt;
}
// The node sum on the FP64 matrix cores.  For a fixed order m the block
//   I_g[(n, m), (n', m')] = sum_c (F_{g,c} Phat_n^m(t_c)) (s J_{|q|}(k_c rho) Phat_{n'}^{|m'|}(s_c))
// of class g (s = the sign from the negative orders m' < 0 and q < 0) is a
// product of a (p+1-m) x nodes matrix and a nodes x NC matrix.  The right-hand
// factor depends only on the quadrature rule group and the source layer, so the
// classes sharing both (a stack of G <= 16 classes, with at most three target
// layers) are contracted together: for each m the left-hand rows (g, n) of all
// G classes are packed into 16-row tiles, and the products run as 16x16x4
// complex MFMA steps (three real MFMAs each in Gauss's form, four otherwise)
// against column tiles (n', m') in NC order.  The (m, row tile, column tile) units of a stack are spread over the
// eight waves of one or more workgroups (UPW units per wave); the node tables of
// a chunk of CH nodes are staged in LDS.  Entries with -m, -m' equal those with
// m, m' and are written too.
template <int UPW, int CH, bool G3>
__global__ __launch_bounds__(512) void k_react_mfma(const SCDesc* scs, int nsc, const int* members,
                                                    const ClassDesc* cls, int p, int Ntot, const cd* Jtab,
                                                    const cd* Ptab, const cd* Ftab, double* Iout, int NC) {
  extern __shared__ cd sh[];
  const int Q = 2 * p, NT = (p + 1) * (p + 2) / 2, NTILE = (NC + 15) / 16;
  __shared__ int s_slot[SC_GMAX], s_out[SC_GMAX], s_foff[SC_GMAX];
  int lo = 0, hi = nsc - 1;  // stack of this workgroup
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (scs[mid].wg0 <= (int)blockIdx.x) lo = mid;
    else hi = mid - 1;
  }
  const SCDesc S = scs[lo];
  const int ug = blockIdx.x - S.wg0, G = S.G, nlt = S.nlt;
  cd* FJ = sh;                  // [CH][Q+1]
  cd* PS = FJ + CH * (Q + 1);   // [CH][NT]
  cd* PT = PS + CH * NT;        // [nlt][CH][NT]
  cd* F = PT + 3 * CH * NT;     // [G][CH]
  if (threadIdx.x < G) {
    const ClassDesc C = cls[members[S.mem0 + threadIdx.x]];
    int slot = 0;
    for (int i = 0; i < nlt; i++)
      if (S.lt[i] == C.lt) slot = i;
    s_slot[threadIdx.x] = slot;
    s_out[threadIdx.x] = C.out;
    s_foff[threadIdx.x] = C.f_off;
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int col = lane & 15, kq = lane >> 4;
  int um[UPW], urt[UPW], uct[UPW], apt[UPW], ag[UPW], psi[UPW], jq[UPW];
  double sgn[UPW];
  bool uv[UPW];
  const int u0 = (ug * 8 + wave) * UPW;
#pragma unroll
  for (int i = 0; i < UPW; i++) {
    int u = u0 + i;
    uv[i] = u < S.NU;
    int m = 0, rem = uv[i] ? u : 0;
    while (m <= p) {
      int nu_m = ((G * (p + 1 - m) + 15) / 16) * NTILE;
      if (rem < nu_m) break;
      rem -= nu_m;
      m++;
    }
    if (m > p) {  // not reached for u < NU
      uv[i] = false;
      m = 0;
      rem = 0;
    }
    const int Rm = p + 1 - m, rt = rem / NTILE, ct = rem % NTILE;
    um[i] = m;
    urt[i] = rt;
    uct[i] = ct;
    // left-hand row of this lane
    int r = rt * 16 + col;
    ag[i] = -1;
    apt[i] = 0;
    if (uv[i] && r < G * Rm) {
      int g = r / Rm, n = m + r % Rm;
      ag[i] = g;
      apt[i] = s_slot[g] * CH * NT + tix(n, m);
    }
    // right-hand column of this lane
    int j = 16 * ct + col;
    psi[i] = 0;
    jq[i] = 0;
    sgn[i] = 0.0;
    if (uv[i] && j < NC) {
      int n2 = (int)sqrt((double)j);
      while (n2 * n2 > j) n2--;
      while ((n2 + 1) * (n2 + 1) <= j) n2++;
      int m2 = j - n2 * n2 - n2, am = m2 < 0 ? -m2 : m2, q = m2 - m;
      int sg = 1;
      if (m2 < 0 && (am & 1)) sg = -sg;
      if (q < 0 && ((-q) & 1)) sg = -sg;
      psi[i] = tix(n2, am);
      jq[i] = q < 0 ? -q : q;
      sgn[i] = (double)sg;
    }
  }
  // Gauss's form (G3): P1 = Ar Br, P2 = Ai Bi, P3 = (Ar + Ai)(Br + Bi) in accr, accg,
  // acci; re = P1 - P2, im = P3 - P1 - P2.  Otherwise four real products.
  v4d accr[UPW], acci[UPW], accg[G3 ? UPW : 1];
#pragma unroll
  for (int i = 0; i < UPW; i++) {
    accr[i] = (v4d){0, 0, 0, 0};
    acci[i] = (v4d){0, 0, 0, 0};
    if constexpr (G3) accg[i] = (v4d){0, 0, 0, 0};
  }
  const int nn = S.nn;
  const cd* Jg = Jtab + (size_t)S.rg_off * (Q + 1);
  const cd* PSg = Ptab + ((size_t)S.ls * Ntot + S.rg_off) * NT;
  for (int c0 = 0; c0 < nn; c0 += CH) {
    const int nc = nn - c0 < CH ? nn - c0 : CH;
    __syncthreads();
    for (int e = threadIdx.x; e < CH * (Q + 1); e += 512)
      FJ[e] = e < nc * (Q + 1) ? Jg[(size_t)c0 * (Q + 1) + e] : mk(0, 0);
    for (int e = threadIdx.x; e < CH * NT; e += 512) PS[e] = e < nc * NT ? PSg[(size_t)c0 * NT + e] : mk(0, 0);
    for (int sl = 0; sl < nlt; sl++) {
      const cd* PTg = Ptab + ((size_t)S.lt[sl] * Ntot + S.rg_off + c0) * NT;
      for (int e = threadIdx.x; e < CH * NT; e += 512) PT[sl * CH * NT + e] = e < nc * NT ? PTg[e] : mk(0, 0);
    }
    for (int e = threadIdx.x; e < G * CH; e += 512) {
      int g = e / CH, c = e % CH;
      F[e] = c < nc ? Ftab[s_foff[g] + c0 + c] : mk(0, 0);
    }
    __syncthreads();
    for (int kst = 0; kst < (nc + 3) / 4; kst++) {
      const int c = kst * 4 + kq;
      int cm = -1, crt = -1;
      double ar = 0.0, ai = 0.0;
#pragma unroll
      for (int i = 0; i < UPW; i++) {
        if (!uv[i]) continue;
        if (um[i] != cm || urt[i] != crt) {
          cm = um[i];
          crt = urt[i];
          cd x = ag[i] >= 0 ? F[ag[i] * CH + c] * PT[apt[i] + c * NT] : mk(0, 0);
          ar = x.x;
          ai = x.y;
        }
        cd y = sgn[i] * (FJ[c * (Q + 1) + jq[i]] * PS[c * NT + psi[i]]);
        if constexpr (G3) {
          accr[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, y.x, accr[i], 0, 0, 0);
          accg[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, y.y, accg[i], 0, 0, 0);
          acci[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar + ai, y.x + y.y, acci[i], 0, 0, 0);
        } else {
          accr[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, y.x, accr[i], 0, 0, 0);
          acci[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, y.y, acci[i], 0, 0, 0);
          accr[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai, y.y, accr[i], 0, 0, 0);
          acci[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, y.x, acci[i], 0, 0, 0);
        }
      }
    }
  }
#pragma unroll
  for (int i = 0; i < UPW; i++) {
    if (!uv[i]) continue;
    const int m = um[i], Rm = p + 1 - m, j = 16 * uct[i] + col;
    if (j >= NC) continue;
    int n2 = (int)sqrt((double)j);
    while (n2 * n2 > j) n2--;
    while ((n2 + 1) * (n2 + 1) <= j) n2++;
    const int m2 = j - n2 * n2 - n2;
#pragma unroll
    for (int r = 0; r < 4; r++) {
      int row = urt[i] * 16 + kq + 4 * r;
      if (row >= G * Rm) continue;
      int g = row / Rm, n = m + row % Rm;
      double* out = Iout + (size_t)s_out[g] * NC * NC * 2;
      double vr = accr[i][r], vi = acci[i][r];
      if constexpr (G3) {
        vi = vi - vr - accg[i][r];
        vr = vr - accg[i][r];
      }
      size_t o1 = (size_t)cidx(n, m) * NC + j;
      out[2 * o1] = vr;
      out[2 * o1 + 1] = vi;
      if (m > 0) {
        size_t o2 = (size_t)cidx(n, -m) * NC + cidx(n2, -m2);
        out[2 * o2] = vr;
        out[2 * o2 + 1] = vi;
      }
    }
  }
}
extern "C" void lk_react_tables(int nrg, const RGDesc* rgs, int Ntot, Stack st, int p, double* Jtab, double* Ptab,
                                double* Ltab, hipStream_t s) {
  long long nt = (long long)(st.L + (Ltab ? 3 : 2)) * Ntot;
  if (nrg && nt)
    k_react_tables<<<(unsigned)((nt + 255) / 256), 256, 0, s>>>(rgs, nrg, Ntot, st, p, (cd*)Jtab, (cd*)Ptab,
                                                                (cd*)Ltab);
}
extern "C" void lk_react_F(int ncls, const ClassDesc* cls, int Ftot, Stack st, int Ntot, const double* Ltab,
                           double* Ftab, hipStream_t s) {
  if (!ncls || !Ftot) return;
  const unsigned g = (unsigned)((Ftot + 255) / 256);
  if (Ltab) {
    k_react_F_lt<<<g, 256, 0, s>>>(cls, ncls, Ftot, st, Ntot, (const cd*)Ltab, (cd*)Ftab);
    return;
  }
  switch (st.L) {
    case 1: k_react_F<1><<<g, 256, 0, s>>>(cls, ncls, Ftot, st, (cd*)Ftab); break;
    case 2: k_react_F<2><<<g, 256, 0, s>>>(cls, ncls, Ftot, st, (cd*)Ftab); break;
    case 3: k_react_F<3><<<g, 256, 0, s>>>(cls, ncls, Ftot, st, (cd*)Ftab); break;
    case 4: k_react_F<4><<<g, 256, 0, s>>>(cls, ncls, Ftot, st, (cd*)Ftab); break;
    default: k_react_F<0><<<g, 256, 0, s>>>(cls, ncls, Ftot, st, (cd*)Ftab); break;
  }
}
template <int UPW, int CH>
static void launch_react_mfma(int nwg, int nsc, const SCDesc* scs, const int* members, const ClassDesc* cls, int p,
                              int Ntot, const cd* J, const cd* P, const cd* F, double* Iout, int NC, size_t lds,
                              hipStream_t s) {
  k_react_mfma<UPW, CH, SC_G3><<<nwg, 512, lds, s>>>(scs, nsc, members, cls, p, Ntot, J, P, F, Iout, NC);
}
extern "C" void lk_react_mfma(int nwg, int nsc, const SCDesc* scs, const int* members, const ClassDesc* cls, int p,
                              int Ntot, const double* Jtab, const double* Ptab, const double* Ftab, double* Iout,
                              int NC, hipStream_t s) {
  if (!nwg) return;
  const int Q = 2 * p, NT = (p + 1) * (p + 2) / 2;
  const cd *J = (const cd*)Jtab, *P = (const cd*)Ptab, *F = (const cd*)Ftab;
  static const int ch_env = getenv("LFMM_REACT_CH") ? atoi(getenv("LFMM_REACT_CH")) : 0;  // tuning override
  if (p <= 8 && ch_env != 16) {
    const size_t lds = sizeof(cd) * (32 * (Q + 1 + 4 * NT) + SC_GMAX * 32);
    launch_react_mfma<SC_UPW, 32>(nwg, nsc, scs, members, cls, p, Ntot, J, P, F, Iout, NC, lds, s);
  } else {
    const size_t lds = sizeof(cd) * (16 * (Q + 1 + 4 * NT) + SC_GMAX * 16);
    launch_react_mfma<SC_UPW, 16>(nwg, nsc, scs, members, cls, p, Ntot, J, P, F, Iout, NC, lds, s);
  }
}

// T[(n,m),(n',m')] = (4 pi/k_t) i^n (-i)^{n'} i^q e^{i q phi} I[(n,m),(n',m')], q = m' - m,
// phi = arg of the lateral offset target - source.  One workgroup per operator.
// One workgroup per class: the class's integral matrix is read once and written out as
// each of its operators (at most eight lateral offsets share a class), which differ
// only in the phases e^{i q phi}; operators of one class share k_t and the FP32 scale
// exponents.  grp[g] = (first operator in rops, count).
#define RX_MAXOPS 8
__global__ __launch_bounds__(256) void k_react_expand(const int2* grp, const ROpDesc* rops, const double* Iall,
                                                      double* ops, int opsz, int p, int NC, int NKS, float* ops32,
                                                      const int2* opse) {
  __shared__ cd ph[RX_MAXOPS][64];  // i^q e^{i q phi} of each operator, q = -2p..2p
  __shared__ int s_op[RX_MAXOPS];
  __shared__ int2 nmt[NM_TAB];
  const int2 G = grp[blockIdx.x];
  const int nop = G.y;
  fill_nm(NC, nmt);
  const int Q = 2 * p;
  for (int t = threadIdx.x; t < nop * (2 * Q + 1); t += 256) {
    const int o = t / (2 * Q + 1), q = t % (2 * Q + 1) - Q;
    const ROpDesc R = rops[G.x + o];
    double sn, cs;
    sincos(q * atan2(R.dy, R.dx), &sn, &cs);
    ph[o][q + Q] = ipow(q) * mk(cs, sn);
    if (q == -Q) s_op[o] = R.op;
  }
  __syncthreads();
  const ROpDesc R0 = rops[G.x];
  const double* I = Iall + (size_t)R0.cls * NC * NC * 2;
  const int2 se = ops32 ? opse[R0.op] : make_int2(0, 0);
  const double pre = 4.0 * LFMM_PI / R0.kt;
  const int nrtl = m2l_nrt(NC), xrl = m2l_xr(NC);
  const int ntot = NKS * (nrtl * 64 + 4 * xrl);
  for (int e = threadIdx.x; e < ntot; e += 256) {
    int row, col;
    m2l_packed_rc(e, nrtl, xrl, &row, &col);
    const bool in = row < NC && col < NC;
    cd base = mk(0, 0);
    int q = 0;
    if (in) {
      const int n = nmt[row].x, m = nmt[row].y, n2 = nmt[col].x, m2 = nmt[col].y;
      base = pre * (ipow(n - n2) * mk(I[2 * ((size_t)row * NC + col)], I[2 * ((size_t)row * NC + col) + 1]));
      if (ops32) {
        const int sh = -(se.x * n + se.y * n2);
        base = mk(ldexp(base.x, sh), ldexp(base.y, sh));
      }
      q = m2 - m + Q;
    }
    for (int o = 0; o < nop; o++) {
      const cd val = in ? ph[o][q] * base : mk(0, 0);
      if (ops32) ((float2*)(ops32 + (size_t)s_op[o] * opsz))[e] = make_float2((float)val.x, (float)val.y);
      else ((double2*)(ops + (size_t)s_op[o] * opsz))[e] = make_double2(val.x, val.y);
    }
  }
}
extern "C" void lk_react_expand(int ngrp, const int* grp, const ROpDesc* rops, const double* Iall, double* ops,
                                int opsz, int p, int NC, int NKS, float* ops32, const int* opse, hipStream_t s) {
  if (ngrp)
    k_react_expand<<<ngrp, 256, 0, s>>>((const int2*)grp, rops, Iall, ops, opsz, p, NC, NKS, ops32,
                                        (const int2*)opse);
}

// ---------------------------------------------------------------------------
// P2M: M_nm = sum_j Q_j 4 pi j_n(k r_j) conj(Y_n^m(r_j^)) about the leaf centre
// (eq. (melecoeffree); at polarisation sources for reaction trees, eq.
// (melayerupgoingimage)).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int seg_find(const int* prefix, int nseg, int x) {
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= x) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// One workgroup of 128 threads per leaf, the particles taken in chunks of 64.  Per
// chunk the first wave computes 4 pi j_n(k r), cos(theta) and the charge of each
// particle, the second wave Phat_m^m(theta) e^{i m phi} for every order m (the
// diagonal start of the Legendre recurrence and the azimuthal factor), all into LDS.
// Then thread (m, stripe) runs the recurrence in n for order m, normalised to start at
// 1, over its stripe of the chunk and accumulates both M_{n,m} and M_{n,-m}, which share
// every recurrence value; the stripes are summed through LDS in a fixed order, one sign
// at a time.  The two signs' accumulators need three waves per SIMD's registers.
template <int P>
__global__ __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(3))) void k_p2m(int nseg, const int* seg_row0, const int* seg_prefix,
                                             const int* box_start, const int* box_cnt, const int* box_code,
                                             const int* box_tree, const int* box_level, const TreeInfo* trees,
                                             const double* px, const double* py, const double* pz, const double* pq,
                                             int NCK, double* M) {
  constexpr int P1 = P + 1, NSTR = 128 / P1, CH = 64, ES = CH + 1;
  constexpr int NTRI = P1 * (P1 + 1) / 2;  // (m, n >= m) pairs of one sign
  // staging: cos(theta), charge, j_n rows, then the Phat_m^m e^{i m phi} rows (padded by
  // one entry so that the orders of one particle fall in different banks)
  constexpr int NSTAGE = 3 * CH + P1 * CH + 2 * P1 * ES, NRED = NSTR * NTRI * 2;
  __shared__ __align__(16) double smem[NSTAGE > NRED ? NSTAGE : NRED];
  // recurrence coefficients (a_n^m, b_n^m) at n P1 + m.  On and below the diagonal they
  // are set to (0, -1): started from p_{-2} = p_{-1} = 1 the steps n <= m then give 1,
  // the normalised start of order m, with no branch (the values below the diagonal are
  // accumulated but never stored); b vanishes one above the diagonal
  __shared__ double2 s_ab[P1 * P1];
  double* s_ct = smem;
  double2* s_q = reinterpret_cast<double2*>(smem + CH);
  double(*s_j)[CH] = reinterpret_cast<double(*)[CH]>(smem + 3 * CH);
  double2(*s_e)[ES] = reinterpret_cast<double2(*)[ES]>(smem + 3 * CH + P1 * CH);
  double* red = smem;  // [stripe][(m, n >= m)] (re, im), one sign at a time
  const int tid = threadIdx.x;
  const int li = blockIdx.x;
  const int sgm = seg_find(seg_prefix, nseg, li);
  const int R = seg_row0[sgm] + (li - seg_prefix[sgm]);
  const TreeInfo T = trees[box_tree[R]];
  double c[3];
  box_center(T, (unsigned)box_code[R], box_level[R], c);
  const int s0 = box_start[R], nt = box_cnt[R];
  for (int o = tid; o < P1 * P1; o += 128) {
    const int n = o / P1, mm = o % P1;
    s_ab[o] = n <= mm ? make_double2(0.0, -1.0) : make_double2(c_la[n * 16 + mm], c_lb[n * 16 + mm]);
  }
  const int m = tid % P1, str = tid / P1;
  const bool active = str < NSTR;
  const double cm = (m & 1) ? -1.0 : 1.0;
  cd accp[P1], accn[P1];
#pragma unroll
  for (int n = 0; n <= P; n++) {
    accp[n] = mk(0, 0);
    accn[n] = mk(0, 0);
  }
  for (int c0 = 0; c0 < nt; c0 += CH) {
    const int nc = nt - c0 < CH ? nt - c0 : CH;
    const int pl = tid & (CH - 1);
    __syncthreads();
    if (pl < nc) {
      const int i = s0 + c0 + pl;
      const double dx = px[i] - c[0], dy = py[i] - c[1], dz = pz[i] - c[2];
      const double rho = sqrt(dx * dx + dy * dy), r = sqrt(rho * rho + dz * dz);
      if (tid < CH) {
        double jn[P1];
        dev_sph_j_t<P>(T.k * r, jn);
#pragma unroll
        for (int n = 0; n <= P; n++) s_j[n][pl] = 4.0 * LFMM_PI * jn[n];
        s_ct[pl] = r > 0 ? dz / r : 1.0;
        s_q[pl] = make_double2(pq[2 * i], pq[2 * i + 1]);
      } else {
        const double st = r > 0 ? rho / r : 0.0;
        // e^{i m phi} by repeated multiplication with e^{i phi} = (dx + i dy) / rho
        const double cp = rho > 0 ? dx / rho : 1.0, sp = rho > 0 ? dy / rho : 0.0;
        double pmm = 0.28209479177387814347, cs = 1.0, sn = 0.0;
        s_e[0][pl] = make_double2(pmm, 0.0);
#pragma unroll
        for (int mm = 1; mm <= P; mm++) {
          pmm *= c_ld[mm] * st;
          const double t = cs * cp - sn * sp;
          sn = sn * cp + cs * sp;
          cs = t;
          s_e[mm][pl] = make_double2(pmm * cs, pmm * sn);
        }
      }
    }
    __syncthreads();
    if (active) {
      // the second particle of an iteration past the end of the chunk is a zero-weight
      // copy of the first
#pragma unroll 1
      for (int i = str; i < nc; i += NSTR) {
        const double ct = s_ct[i];
        const double2 e = s_e[m][i], q = s_q[i];
        const cd qp = mk(q.x, q.y) * mk(e.x, -e.y), qn = cm * (mk(q.x, q.y) * mk(e.x, e.y));
        double p0 = 1.0, p1 = 1.0;
#pragma unroll
        for (int n = 0; n <= P; n++) {
          const double2 ab = s_ab[n * P1 + m];
          const double val = ab.x * ct * p1 - ab.y * p0;
          p0 = p1;
          p1 = val;
          const double u = s_j[n][i] * val;
          accp[n] = accp[n] + u * qp;
          accn[n] = accn[n] + u * qn;
        }
      }
    }
  }
  // (m, n) at m P1 - m (m - 1) / 2 + (n - m) within one stripe's block
  const int tri = m * P1 - m * (m - 1) / 2 - m;
  double* Mr = M + (size_t)R * NCK * 2;
#pragma unroll
  for (int h = 0; h < 2; h++) {
    __syncthreads();
    if (active) {
#pragma unroll
      for (int n = 0; n <= P; n++) {
        if (n < m) continue;
        const cd a = h ? accn[n] : accp[n];
        const size_t o = ((size_t)str * NTRI + tri + n) * 2;
        red[o] = a.x;
        red[o + 1] = a.y;
      }
    }
    __syncthreads();
    // one thread per output (m, n >= m; no sign 1 for m = 0): the stripes are summed in
    // a fixed order
    for (int o = tid; o < NTRI; o += 128) {
      int mm = 0, r = o;
      while (r >= P1 - mm) {
        r -= P1 - mm;
        mm++;
      }
      const int n = mm + r;
      if (h == 0 || mm > 0) {
        double sx = 0.0, sy = 0.0;
        for (int k = 0; k < NSTR; k++) {
          sx += red[((size_t)k * NTRI + o) * 2];
          sy += red[((size_t)k * NTRI + o) * 2 + 1];
        }
        const int oc = cidx(n, h ? -mm : mm);
        Mr[2 * oc] = sx;
        Mr[2 * oc + 1] = sy;
      }
    }
  }
}
extern "C" void lk_p2m(int nseg, const int* seg_row0, const int* seg_prefix, int total, const int* box_start,
                       const int* box_cnt, const int* box_code, const int* box_tree, const int* box_level,
                       const TreeInfo* trees, const double* px, const double* py, const double* pz, const double* pq,
                       int p, int NCK, double* M, hipStream_t s) {
  if (!total) return;
#define P2M_CASE(PP)                                                                                          \
  case PP:                                                                                                    \
    k_p2m<PP><<<total, 128, 0, s>>>(nseg, seg_row0, seg_prefix, box_start, box_cnt, box_code, box_tree,       \
                                    box_level, trees, px, py, pz, pq, NCK, M);                                \
    break;
  switch (p) { P2M_CASE(1) P2M_CASE(2) P2M_CASE(3) P2M_CASE(4) P2M_CASE(5) P2M_CASE(6) P2M_CASE(7) P2M_CASE(8)
               P2M_CASE(9) P2M_CASE(10) default: break; }
#undef P2M_CASE
}

// ---------------------------------------------------------------------------
// L2P: phi += sum_nm L_nm j_n(k r) Y_n^m(r^) (eq. (freespace3dlocexp) / (lelayerimage)),
// one thread per target point of the listed trees (sorted-position segments).
// ---------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(256) void k_l2p(int nseg, const int* seg_s0, const int* seg_prefix, int total,
                                             const int* leafrow, const int* box_code, const int* box_tree,
                                             const int* box_level, const TreeInfo* trees, const double* px,
                                             const double* py, const double* pz, const int* sg, int NCK,
                                             const double* Lc, double* phi_tp) {
  int gid = blockIdx.x * 256 + threadIdx.x;
  if (gid >= total) return;
  int sgm = seg_find(seg_prefix, nseg, gid);
  int s = seg_s0[sgm] + (gid - seg_prefix[sgm]);
  int R = leafrow[s];
  TreeInfo T = trees[box_tree[R]];
  double c[3];
  box_center(T, (unsigned)box_code[R], box_level[R], c);
  double dx = px[s] - c[0], dy = py[s] - c[1], dz = pz[s] - c[2];
  double r = sqrt(dx * dx + dy * dy + dz * dz);
  double jn[P + 1];
  dev_sph_j_t<P>(T.k * r, jn);
  const double rho = sqrt(dx * dx + dy * dy);
  double ct = r > 0 ? dz / r : 1.0, st = r > 0 ? rho / r : 0.0;
  // e^{i m phi} by repeated multiplication with e^{i phi} = (dx + i dy) / rho
  const double cp = rho > 0 ? dx / rho : 1.0, sp = rho > 0 ? dy / rho : 0.0;
  double cs = 1.0, sn = 0.0;
  const double* L = Lc + (size_t)R * NCK * 2;
  cd acc = mk(0, 0);
  double pmm = 0.28209479177387814347;
#pragma unroll 1
  for (int m = 0; m <= P; m++) {
    if (m > 0) {
      pmm *= c_ld[m] * st;
      const double t = cs * cp - sn * sp;
      sn = sn * cp + cs * sp;
      cs = t;
    }
    double cm = (m & 1) ? -1.0 : 1.0;
    double p0 = 0.0, p1 = pmm;
#pragma unroll
    for (int n = 0; n <= P; n++) {
      if (n < m) continue;
      double val;
      if (n == m) val = pmm;
      else {
        val = c_la[n * 16 + m] * ct * p1 - c_lb[n * 16 + m] * p0;
        p0 = p1;
        p1 = val;
      }
      double base = jn[n] * val;
      cd Lp = mk(L[2 * cidx(n, m)], L[2 * cidx(n, m) + 1]);
      acc = acc + Lp * mk(base * cs, base * sn);
      if (m > 0) {
        cd Ln = mk(L[2 * cidx(n, -m)], L[2 * cidx(n, -m) + 1]);
        acc = acc + Ln * mk(cm * base * cs, -cm * base * sn);
      }
    }
  }
  int g = sg[s];
  phi_tp[2 * g] += acc.x;
  phi_tp[2 * g + 1] += acc.y;
}
extern "C" void lk_l2p(int nseg, const int* seg_s0, const int* seg_prefix, int total, const int* leafrow,
                       const int* box_code, const int* box_tree, const int* box_level, const TreeInfo* trees,
                       const double* px, const double* py, const double* pz, const int* sg, int p, int NCK,
                       const double* Lc, double* phi_tp, hipStream_t s) {
  if (!total) return;
  int g = nblk(total, 256);
#define L2P_CASE(PP)                                                                                          \
  case PP:                                                                                                    \
    k_l2p<PP><<<g, 256, 0, s>>>(nseg, seg_s0, seg_prefix, total, leafrow, box_code, box_tree, box_level,      \
                                trees, px, py, pz, sg, NCK, Lc, phi_tp);                                      \
    break;
  switch (p) { L2P_CASE(1) L2P_CASE(2) L2P_CASE(3) L2P_CASE(4) L2P_CASE(5) L2P_CASE(6) L2P_CASE(7) L2P_CASE(8)
               L2P_CASE(9) L2P_CASE(10) default: break; }
#undef L2P_CASE
}

// ---------------------------------------------------------------------------
// Workgroups are dispatched round-robin over the 8 XCDs (each with its own L2):
// map the dispatch index so that consecutive logical blocks -- which share their
// group's operator sequence -- run on the same XCD and reuse its L2.
__device__ __forceinline__ int xcd_block(int b, int nb) {
  const int q = nb >> 3, r = nb & 7, x = b & 7;
  return x * q + (x < r ? x : r) + (b >> 3);
}
// ---------------------------------------------------------------------------
// FP32 path of the M2L (mixed precision).  Expansions of a box at level l of a
// tree with wavenumber k are rescaled by powers c^n of c = 2^e, e = round(log2(1/(k h_l)))
// (h_l the box size), which brings M_n ~ (k h)^n and L_n ~ (k h)^{-n} to O(1) and
// keeps FP32 away from overflow (h_{2p}(k r) reaches 1e44 at p = 10 on fine
// levels); the operators are stored pre-scaled, T[(n,m),(nu,mu)] c_t^{-n} c_s^{-nu}
// (powers of two: the scalings are exact).
// The GEMM runs on v_mfma_f32_16x16x4f32 (D element r of lane l = (row
// 4 (l/16) + r, col l%16)); each operator's FP32 partial sum is moved into FP64
// accumulators when the operator is done, and the result is added, unscaled, to
// the FP64 local expansions.
// ---------------------------------------------------------------------------
__global__ void k_m_to_f32(int nrows, int NCK, int NC, const int* box_tree, const int* box_level, const int* se,
                           const double2* M, float2* M32) {
  long long e = (long long)blockIdx.x * 256 + threadIdx.x;
  if (e >= (long long)nrows * NCK) return;
  int row = (int)(e / NCK), col = (int)(e % NCK);
  float2 v = make_float2(0.f, 0.f);
  if (col < NC) {
    int n = (int)sqrt((double)col);
    while (n * n > col) n--;
    int sh = se[box_tree[row] * 9 + box_level[row]] * n;
    double2 m = M[e];
    v = make_float2((float)ldexp(m.x, sh), (float)ldexp(m.y, sh));
  }
  M32[e] = v;
}
extern "C" void lk_m_to_f32(int nrows, int NCK, int NC, const int* box_tree, const int* box_level, const int* se,
                            const double* M, float* M32, hipStream_t s) {
  long long n = (long long)nrows * NCK;
  if (n) k_m_to_f32<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(nrows, NCK, NC, box_tree, box_level, se,
                                                                (const double2*)M, (float2*)M32);
}
// M2L on the matrix cores (FP32 in the mixed path, FP64 otherwise).  A wave owns
// 16 targets of one group (the B columns: source expansions gathered by row) and
// every row of the output; the KS waves of a workgroup take every KS-th operator of
// the group's sequence and add their partial sums through LDS at the end, in a
// fixed order.  Before the loop each wave lists the operators for which at least
// one of its targets has a source (the others would only multiply zeros), with the
// source rows, in LDS; the loop then runs over the (operator, k-step) steps of that
// list with the operands of the next PF steps in flight in registers.  Operators
// are stored k-step major (see m2l_nrt), so one step's operand is NRT contiguous
// 512-byte (FP32) or 1 KB (FP64) tiles.  The complex product takes three real
// MFMAs (Gauss's method: P1 = Ar Br, P2 = Ai Bi, P3 = (Ar + Ai)(Br + Bi),
// re = P1 - P2, im = P3 - P1 - P2) where the registers allow, four otherwise; a
// last row that would be alone in its sixteen-row tile (XR) is summed on the
// vector ALU.  The FP32 kernel moves each operator's sums into FP64 accumulators
// when the operator is done.
template <typename R>
struct M2LT {
  typedef typename std::conditional<sizeof(R) == 4, float2, double2>::type C2;
  typedef typename std::conditional<sizeof(R) == 4, v4f, v4d>::type V4;
};
__device__ __forceinline__ v4f mfma16(float a, float b, v4f c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
__device__ __forceinline__ v4d mfma16(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
// lst: this wave's lists in LDS: lmax operator ids, then lmax x 16 source rows (one
// per target column).  Every load of the main loop is unconditional (addresses
// clamped, absent sources zeroed by a flag where the value is used), so that the
// compiler can keep PF steps of loads in flight instead of waiting for all of them.
template <typename R, int NRT, int XR, int KS, int PF, bool G3>
__device__ __forceinline__ void m2l_body(const GBlock& bd, const int* seq, const int* srow, int srow_stride,
                                         const typename M2LT<R>::C2* __restrict__ ops, size_t opstride, int NKS,
                                         const typename M2LT<R>::C2* __restrict__ S, int NCK, v4d (&dre)[NRT],
                                         v4d (&dim)[NRT], double& dxre, double& dxim, int* lst, int lmax) {
  typedef typename M2LT<R>::C2 C2;
  typedef typename M2LT<R>::V4 V4;
  constexpr bool F32 = sizeof(R) == 4;
  constexpr int SZ = NRT * 64 + 4 * XR;
  constexpr int NA = NRT + XR;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, col = lane & 15, kr = lane >> 4;
  const int cg = wave / KS, kw = wave % KS;
  const int tt = cg * 16 + col;
  const bool tv = tt < bd.nt;
  const int* my_srow = srow + (size_t)(bd.e0 + (tv ? tt : 0)) * srow_stride;
  int* lop = lst;
  int* lsr = lst + lmax;
  // this wave's operators with a source for at least one of its targets, with the
  // source row of each target column
  int nv = 0;
  for (int k = kw; k < bd.K; k += KS) {
    const int sr = tv ? my_srow[k] : -1;
    if (__ballot(sr >= 0)) {
      if (lane == 0) lop[nv] = seq[bd.seq0 + k];
      if (kr == 0) lsr[nv * 16 + col] = sr;
      nv++;
    }
  }
  if (nv == 0) return;
  __builtin_amdgcn_wave_barrier();
  const int T = nv * NKS;
  int ak = 0, aks = 0, ls = 0;  // next step to load: operator ak of the list, k-step aks; its index ls
  auto load = [&](C2 (&a)[NA], C2& b, bool& bv) {
    const int akc = ak < nv ? ak : nv - 1;  // past the end: a valid address, the value unused
    const C2* A = ops + (size_t)lop[akc] * opstride + (size_t)aks * SZ;
#pragma unroll
    for (int rt = 0; rt < NRT; rt++) a[rt] = A[rt * 64 + lane];
    if constexpr (XR) a[NRT] = A[NRT * 64 + kr];
    const int sr = lsr[akc * 16 + col];
    bv = sr >= 0 && ls < T;
    b = S[(size_t)(sr >= 0 ? sr : 0) * NCK + 4 * aks + kr];
    ls++;
    aks++;
    ak += aks == NKS;
    aks = aks == NKS ? 0 : aks;
  };
  V4 p1[NRT], p2[NRT], p3[NRT];
#pragma unroll
  for (int rt = 0; rt < NRT; rt++) {
    p1[rt] = V4{0, 0, 0, 0};
    p2[rt] = V4{0, 0, 0, 0};
    p3[rt] = V4{0, 0, 0, 0};
  }
  R xre = 0, xim = 0;
  C2 af[PF][NA], bf[PF];
  bool bv[PF];
#pragma unroll
  for (int u = 0; u < PF; u++) load(af[u], bf[u], bv[u]);
  int cks = 0;
  auto flush = [&]() {
#pragma unroll
    for (int rt = 0; rt < NRT; rt++) {
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const double q1 = (double)p1[rt][r], q3 = (double)p3[rt][r];
        if constexpr (G3) {
          const double q2 = (double)p2[rt][r];
          dre[rt][r] += q1 - q2;
          dim[rt][r] += q3 - q1 - q2;
        } else {
          dre[rt][r] += q1;
          dim[rt][r] += q3;
        }
      }
      p1[rt] = V4{0, 0, 0, 0};
      p2[rt] = V4{0, 0, 0, 0};
      p3[rt] = V4{0, 0, 0, 0};
    }
    if constexpr (XR) {
      dxre += (double)xre;
      dxim += (double)xim;
      xre = 0;
      xim = 0;
    }
  };
  auto step = [&](C2 (&a)[NA], C2& b_, bool& bv_) {
    const C2 b = bv_ ? b_ : C2{0, 0};
    if constexpr (G3) {
      const R bs = b.x + b.y;
#pragma unroll
      for (int rt = 0; rt < NRT; rt++) {
        p1[rt] = mfma16(a[rt].x, b.x, p1[rt]);
        p2[rt] = mfma16(a[rt].y, b.y, p2[rt]);
        p3[rt] = mfma16(a[rt].x + a[rt].y, bs, p3[rt]);
      }
    } else {
#pragma unroll
      for (int rt = 0; rt < NRT; rt++) {
        p1[rt] = mfma16(a[rt].x, b.x, p1[rt]);
        p3[rt] = mfma16(a[rt].x, b.y, p3[rt]);
        p1[rt] = mfma16(-a[rt].y, b.y, p1[rt]);
        p3[rt] = mfma16(a[rt].y, b.x, p3[rt]);
      }
    }
    if constexpr (XR) {
      xre += a[NRT].x * b.x - a[NRT].y * b.y;
      xim += a[NRT].x * b.y + a[NRT].y * b.x;
    }
    load(a, b_, bv_);  // the step PF ahead into the registers just used
    // FP32: one operator done -> its sums into FP64 (FP64 keeps accumulating)
    if (++cks == NKS) {
      cks = 0;
      if constexpr (F32) flush();
    }
    // keep the scheduler from moving the loads of this step down to their uses
    __builtin_amdgcn_sched_barrier(0);
  };
  // steps past T (up to the next multiple of UN) multiply zeros; the loop body runs
  // UN = 4 PF steps, since the compiler's wait at the top of the loop drains every
  // load in flight: once per 4 PF steps instead of once per PF
  constexpr int UN = 4 * PF;
  for (int i = 0; i < T; i += UN) {
#pragma unroll
    for (int u = 0; u < UN; u++) step(af[u % PF], bf[u % PF], bv[u % PF]);
  }
  flush();
  if constexpr (XR) {
    // the four k-lanes of a target hold partial sums of the last row
    dxre += __shfl_xor(dxre, 16);
    dxim += __shfl_xor(dxim, 16);
    dxre += __shfl_xor(dxre, 32);
    dxim += __shfl_xor(dxim, 32);
  }
}
// Partial sums of the KS waves of a 16-target tile through LDS (fixed order), then
// the rows of wave kw = 0 added to the local expansions (rows of FP32 results
// unscaled by the level's power of two first).
template <int NRT, int XR, int KS>
__device__ __forceinline__ void m2l_store(const GBlock& bd, const int* trow, double2* D, int NCK, int NC, bool f32row,
                                          int e_t_or_0, const int* box_tree, const int* box_level, const int* se,
                                          v4d (&dre)[NRT], v4d (&dim)[NRT], double& dxre, double& dxim) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, col = lane & 15, kr = lane >> 4;
  const int cg = wave / KS, kw = wave % KS;
  if constexpr (KS > 1) {
    __shared__ double red[KS > 4 ? KS : 4][8][64];
#pragma unroll
    for (int rt = 0; rt < NRT + XR; rt++) {
      if (kw > 0) {
        if (rt < NRT) {
#pragma unroll
          for (int r = 0; r < 4; r++) {
            red[wave][r][lane] = dre[rt < NRT ? rt : 0][r];
            red[wave][4 + r][lane] = dim[rt < NRT ? rt : 0][r];
          }
        } else {
          red[wave][0][lane] = dxre;
          red[wave][4][lane] = dxim;
        }
      }
      __syncthreads();
      if (kw == 0) {
        for (int w = 1; w < KS; w++) {
          if (rt < NRT) {
#pragma unroll
            for (int r = 0; r < 4; r++) {
              dre[rt < NRT ? rt : 0][r] += red[wave + w][r][lane];
              dim[rt < NRT ? rt : 0][r] += red[wave + w][4 + r][lane];
            }
          } else {
            dxre += red[wave + w][0][lane];
            dxim += red[wave + w][4][lane];
          }
        }
      }
      __syncthreads();
    }
  }
  const int tt = cg * 16 + col;
  if (kw != 0 || tt >= bd.nt) return;
  const int tr = trow[bd.e0 + tt];
  const int e_t = f32row ? se[box_tree[tr] * 9 + box_level[tr]] : 0;
  double2* Dr = D + (size_t)tr * NCK;
  auto put = [&](int row, double vr, double vi) {
    if (f32row) {
      int n = (int)sqrt((double)row);
      while (n * n > row) n--;
      vr = ldexp(vr, e_t * n);
      vi = ldexp(vi, e_t * n);
    }
    double2 v = Dr[row];
    v.x += vr;
    v.y += vi;
    Dr[row] = v;
  };
#pragma unroll
  for (int rt = 0; rt < NRT; rt++)
#pragma unroll
    for (int r = 0; r < 4; r++) {
      // D layouts: FP32 element r of lane l = row 4 (l/16) + r; FP64: row l/16 + 4 r
      const int row = rt * 16 + (f32row ? 4 * kr + r : kr + 4 * r);
      if (row < NC) put(row, dre[rt][r], dim[rt][r]);
    }
  if constexpr (XR) {
    if (kr == 0) put(NRT * 16, dxre, dxim);
  }
}
template <int NRT, int XR, int KS>
__global__ __launch_bounds__(KS == 8 ? 512 : 256, KS == 8 ? 1 : 2) __attribute__((amdgpu_waves_per_eu(1, 2))) void k_m2l_gemm32(const GBlock* blocks, const int* seq, const int* trow,
                                                       const int* srow, int srow_stride,
                                                       const float2* __restrict__ ops, int opstride2, int NKS,
                                                       const float2* __restrict__ S, double2* D, int NCK, int NC,
                                                       const int* box_tree, const int* box_level, const int* se,
                                                       int lmax) {
  extern __shared__ int m2l_lists[];  // per wave: lmax operator ids, then lmax x 16 source rows
  const GBlock bd = blocks[xcd_block(blockIdx.x, gridDim.x)];
  v4d dre[NRT], dim[NRT];
#pragma unroll
  for (int rt = 0; rt < NRT; rt++) {
    dre[rt] = (v4d){0, 0, 0, 0};
    dim[rt] = (v4d){0, 0, 0, 0};
  }
  double dxre = 0.0, dxim = 0.0;
  const int wave = threadIdx.x >> 6;
  m2l_body<float, NRT, XR, KS, (NRT <= 6 ? 3 : 2), (NRT <= 6)>(bd, seq, srow, srow_stride, ops, (size_t)opstride2, NKS, S, NCK, dre,
                                               dim, dxre, dxim, m2l_lists + 17 * lmax * wave, lmax);
  m2l_store<NRT, XR, KS>(bd, trow, D, NCK, NC, true, 0, box_tree, box_level, se, dre, dim, dxre, dxim);
}
// (two waves per SIMD is the target: at a higher one the scheduler would sink the
// prefetch loads to their uses to free registers)
template <int NRT, int XR, int KS>
__global__ __launch_bounds__(KS == 8 ? 512 : 256, KS == 8 ? 1 : 2) __attribute__((amdgpu_waves_per_eu(1, 2))) void k_m2l_gemm64(const GBlock* blocks, const int* seq, const int* trow,
                                                       const int* srow, int srow_stride,
                                                       const double2* __restrict__ ops, int opstride2, int NKS,
                                                       const double2* __restrict__ S, double2* D, int NCK, int NC,
                                                       int lmax) {
  extern __shared__ int m2l_lists[];  // per wave: lmax operator ids, then lmax x 16 source rows
  const GBlock bd = blocks[xcd_block(blockIdx.x, gridDim.x)];
  v4d dre[NRT], dim[NRT];
#pragma unroll
  for (int rt = 0; rt < NRT; rt++) {
    dre[rt] = (v4d){0, 0, 0, 0};
    dim[rt] = (v4d){0, 0, 0, 0};
  }
  double dxre = 0.0, dxim = 0.0;
  const int wave = threadIdx.x >> 6;
  m2l_body<double, NRT, XR, KS, 2, (NRT <= 5)>(bd, seq, srow, srow_stride, ops, (size_t)opstride2, NKS, S, NCK, dre,
                                                dim, dxre, dxim, m2l_lists + 17 * lmax * wave, lmax);
  m2l_store<NRT, XR, KS>(bd, trow, D, NCK, NC, false, 0, nullptr, nullptr, nullptr, dre, dim, dxre, dxim);
}
// M2M and L2L: the same GEMM over the 8 (M2M) or 1 (L2L) shift operators of a
// target's level; a kernel of its own so that profiles tell it from the M2L.
template <int NRT, int XR, int KS>
__global__ __launch_bounds__(256, 2) __attribute__((amdgpu_waves_per_eu(1, 2))) void k_shift_gemm64(
    const GBlock* blocks, const int* seq, const int* trow, const int* srow, int srow_stride,
    const double2* __restrict__ ops, int opstride2, int NKS, const double2* __restrict__ S, double2* D, int NCK,
    int NC, int lmax) {
  extern __shared__ int m2l_lists[];
  const GBlock bd = blocks[xcd_block(blockIdx.x, gridDim.x)];
  v4d dre[NRT], dim[NRT];
#pragma unroll
  for (int rt = 0; rt < NRT; rt++) {
    dre[rt] = (v4d){0, 0, 0, 0};
    dim[rt] = (v4d){0, 0, 0, 0};
  }
  double dxre = 0.0, dxim = 0.0;
  const int wave = threadIdx.x >> 6;
  m2l_body<double, NRT, XR, KS, 2, (NRT <= 5)>(bd, seq, srow, srow_stride, ops, (size_t)opstride2, NKS, S, NCK, dre,
                                                dim, dxre, dxim, m2l_lists + 17 * lmax * wave, lmax);
  m2l_store<NRT, XR, KS>(bd, trow, D, NCK, NC, false, 0, nullptr, nullptr, nullptr, dre, dim, dxre, dxim);
}
extern "C" void lk_shift_gemm64(int NC, int ks, int nblocks, const GBlock* blocks, const int* seq, const int* trow,
                                const int* srow, int srow_stride, const double* ops, int opsz, int NKS,
                                const double* S, double* D, int NCK, hipStream_t s) {
  if (!nblocks) return;
  const int lmax = (srow_stride + ks - 1) / ks;
  const size_t lds = sizeof(int) * 17 * (size_t)lmax * 4;
  const int nrt = m2l_nrt(NC), xr = m2l_xr(NC);
  const double2* o2 = (const double2*)ops;
  const int os2 = opsz / 2;
#define SHIFT_CASE(N, X, K)                                                                                     \
  if (nrt == N && xr == X && ks == K) {                                                                         \
    k_shift_gemm64<N, X, K><<<nblocks, 256, lds, s>>>(blocks, seq, trow, srow, srow_stride, o2, os2, NKS,       \
                                                      (const double2*)S, (double2*)D, NCK, NC, lmax);           \
    return;                                                                                                     \
  }
#define SHIFT_KS(N, X) SHIFT_CASE(N, X, 1) SHIFT_CASE(N, X, 2) SHIFT_CASE(N, X, 4)
  SHIFT_KS(1, 0) SHIFT_KS(2, 0) SHIFT_KS(3, 1) SHIFT_KS(3, 0) SHIFT_KS(4, 0) SHIFT_KS(5, 1) SHIFT_KS(7, 0)
  SHIFT_KS(8, 0)
#undef SHIFT_KS
#undef SHIFT_CASE
}
// Every M2L GEMM instance may use the CU's 160 KB of LDS, less its static LDS, for its
// operator lists (17 ints per listed operator and wave), and the reaction node sums
// for their tables; set once per plan, outside any capture and any evaluation (so no
// attribute call races another thread's launches).  The smallest allowance over the
// M2L instances bounds an M2L launch.
static size_t g_m2l_lds_max = 64 * 1024 - 16 * 1024;
template <typename K>
static size_t m2l_allow_lds(K* kern) {
  hipFuncAttributes fa;
  if (hipFuncGetAttributes(&fa, (const void*)kern) != hipSuccess) return 64 * 1024 - 16 * 1024;
  const size_t lim = 160 * 1024 - fa.sharedSizeBytes;
  if (hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lim) != hipSuccess)
    return 64 * 1024 - fa.sharedSizeBytes;
  return lim;
}
extern "C" void lk_m2l_gemm_init() {
  size_t lim = 160 * 1024;
#define M2L_ATTR(N, X, K)                                          \
  lim = std::min(lim, m2l_allow_lds(k_m2l_gemm32<N, X, K>));     \
  lim = std::min(lim, m2l_allow_lds(k_m2l_gemm64<N, X, K>));
#define M2L_ATTR_KS(N, X) M2L_ATTR(N, X, 1) M2L_ATTR(N, X, 2) M2L_ATTR(N, X, 4) M2L_ATTR(N, X, 8)
  M2L_ATTR_KS(1, 0) M2L_ATTR_KS(2, 0) M2L_ATTR_KS(3, 1) M2L_ATTR_KS(3, 0) M2L_ATTR_KS(4, 0) M2L_ATTR_KS(5, 1)
  M2L_ATTR_KS(7, 0) M2L_ATTR_KS(8, 0)
#undef M2L_ATTR_KS
#undef M2L_ATTR
  g_m2l_lds_max = lim;
  // the reaction node sums' LDS (32 or 16 classes' tables per workgroup)
  (void)m2l_allow_lds(k_react_mfma<SC_UPW, 32, SC_G3>);
  (void)m2l_allow_lds(k_react_mfma<SC_UPW, 16, SC_G3>);
  (void)hipGetLastError();  // a refused attribute leaves no error behind: its smaller limit is kept
}
extern "C" size_t lk_m2l_lds_max() { return g_m2l_lds_max; }
extern "C" size_t lk_m2l_lds_bytes(int srow_stride, int ks) {
  return sizeof(int) * 17 * (size_t)((srow_stride + ks - 1) / ks) * (ks == 8 ? 8 : 4);  // every wave's lists
}

extern "C" void lk_gemm32(int NC, int ks, int nblocks, const GBlock* blocks, const int* seq, const int* trow,
                          const int* srow, int srow_stride, const float* ops, int opsz, int NKS, const float* S,
                          double* D, int NCK, const int* box_tree, const int* box_level, const int* se,
                          hipStream_t s) {
  if (!nblocks) return;
  const int lmax = (srow_stride + ks - 1) / ks;  // a wave lists at most ceil(K / ks) operators
  const size_t lds = sizeof(int) * 17 * (size_t)lmax * (ks == 8 ? 8 : 4);  // every wave's lists
  const int nrt = m2l_nrt(NC), xr = m2l_xr(NC);
  const float2* o2 = (const float2*)ops;
  const int os2 = opsz / 2;  // operator stride in float2 (opsz floats per operator)
#define GEMM32_CASE(N, X, K)                                                                                        \
  if (nrt == N && xr == X && ks == K) {                                                                             \
    k_m2l_gemm32<N, X, K><<<nblocks, K == 8 ? 512 : 256, lds, s>>>(blocks, seq, trow, srow, srow_stride, o2, os2, NKS,             \
                                                    (const float2*)S, (double2*)D, NCK, NC, box_tree, box_level, se, \
                                                    lmax);                                                          \
    return;                                                                                                         \
  }
#define GEMM32_KS(N, X) GEMM32_CASE(N, X, 1) GEMM32_CASE(N, X, 2) GEMM32_CASE(N, X, 4) GEMM32_CASE(N, X, 8)
  GEMM32_KS(1, 0) GEMM32_KS(2, 0) GEMM32_KS(3, 1) GEMM32_KS(3, 0) GEMM32_KS(4, 0) GEMM32_KS(5, 1) GEMM32_KS(7, 0)
  GEMM32_KS(8, 0)
#undef GEMM32_KS
#undef GEMM32_CASE
}
extern "C" void lk_m2l_gemm64(int NC, int ks, int nblocks, const GBlock* blocks, const int* seq, const int* trow,
                              const int* srow, int srow_stride, const double* ops, int opsz, int NKS,
                              const double* S, double* D, int NCK, hipStream_t s) {
  if (!nblocks) return;
  const int lmax = (srow_stride + ks - 1) / ks;  // a wave lists at most ceil(K / ks) operators
  const size_t lds = sizeof(int) * 17 * (size_t)lmax * (ks == 8 ? 8 : 4);  // every wave's lists
  const int nrt = m2l_nrt(NC), xr = m2l_xr(NC);
  const double2* o2 = (const double2*)ops;
  const int os2 = opsz / 2;  // operator stride in double2 (opsz doubles per operator)
#define GEMM64_CASE(N, X, K)                                                                                  \
  if (nrt == N && xr == X && ks == K) {                                                                       \
    k_m2l_gemm64<N, X, K><<<nblocks, K == 8 ? 512 : 256, lds, s>>>(blocks, seq, trow, srow, srow_stride, o2, os2, NKS,       \
                                                    (const double2*)S, (double2*)D, NCK, NC, lmax);           \
    return;                                                                                                   \
  }
#define GEMM64_KS(N, X) GEMM64_CASE(N, X, 1) GEMM64_CASE(N, X, 2) GEMM64_CASE(N, X, 4) GEMM64_CASE(N, X, 8)
  GEMM64_KS(1, 0) GEMM64_KS(2, 0) GEMM64_KS(3, 1) GEMM64_KS(3, 0) GEMM64_KS(4, 0) GEMM64_KS(5, 1) GEMM64_KS(7, 0)
  GEMM64_KS(8, 0)
#undef GEMM64_KS
#undef GEMM64_CASE
}

// ---------------------------------------------------------------------------
// Device-wide exclusive prefix sum of int32 values in three passes over tiles of
// SCAN_TILE: the sum of every tile, an exclusive scan of the tile sums in one
// workgroup, then every tile scanned again from its offset.  out may equal in.
// ---------------------------------------------------------------------------
#define SCAN_TILE 4096
__device__ __forceinline__ int block_excl_scan256(int v, int* sh, int* total) {
  // Hillis-Steele scan of one value per thread of a 256-thread block
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const int a = t >= off ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += a;
    __syncthreads();
  }
  const int incl = sh[t];
  *total = sh[255];
  __syncthreads();
  return incl - v;
}
__global__ __launch_bounds__(256) void k_scan_tiles(const int* in, long long n, int* tsum) {
  __shared__ int sh[256];
  const long long base = (long long)blockIdx.x * SCAN_TILE + threadIdx.x;
  int s = 0;
#pragma unroll
  for (int k = 0; k < 16; k++)
    if (base + 256 * k < n) s += in[base + 256 * k];
  int tot;
  block_excl_scan256(s, sh, &tot);
  if (threadIdx.x == 0) tsum[blockIdx.x] = tot;
}
__global__ __launch_bounds__(256) void k_scan_sums(int* tsum, int nt) {
  __shared__ int sh[256];
  int carry = 0;
  for (int c = 0; c < nt; c += 256) {
    const int i = c + threadIdx.x;
    const int v = i < nt ? tsum[i] : 0;
    int tot;
    const int ex = block_excl_scan256(v, sh, &tot);
    if (i < nt) tsum[i] = carry + ex;
    carry += tot;
  }
}
__global__ __launch_bounds__(256) void k_scan_apply(const int* in, long long n, const int* toff, int* out) {
  // the tile in 16 rounds of 256 consecutive values: a shuffle scan in each wave,
  // the waves' totals in wave order, the rounds in order
  __shared__ int wt[4];
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  int carry = toff[blockIdx.x];
  for (int r = 0; r < 16; r++) {
    const long long g = (long long)blockIdx.x * SCAN_TILE + r * 256 + t;
    const int v = g < n ? in[g] : 0;
    int x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int y = __shfl_up(x, d);
      if (lane >= d) x += y;
    }
    if (lane == 63) wt[wave] = x;
    __syncthreads();
    int wpre = 0;
    for (int w = 0; w < wave; w++) wpre += wt[w];
    const int rtot = wt[0] + wt[1] + wt[2] + wt[3];
    if (g < n) out[g] = carry + wpre + x - v;
    carry += rtot;
    __syncthreads();
  }
}
extern "C" void lk_scan_excl(const int* in, long long n, int* out, int* tsum, hipStream_t s) {
  if (n <= 0) return;
  const int nt = (int)((n + SCAN_TILE - 1) / SCAN_TILE);
  k_scan_tiles<<<nt, 256, 0, s>>>(in, n, tsum);
  k_scan_sums<<<1, 256, 0, s>>>(tsum, nt);
  k_scan_apply<<<nt, 256, 0, s>>>(in, n, tsum, out);
}
extern "C" int lk_scan_tsum_size(long long n) { return (int)((n + SCAN_TILE - 1) / SCAN_TILE) + 1; }

// ---------------------------------------------------------------------------
// Stable LSD radix sort of (u32 key, int32 value) pairs, 8 key bits per pass,
// within segments: the pairs come grouped in consecutive segments (the trees of
// the particle sort, whose keys differ above the sorted bits) and each segment is
// sorted on its own, so the bits that tell the segments apart need no pass.
// Per pass: digit counts of every tile of at most RS_TILE pairs of one segment
// (segment-major, then digit-major), one exclusive scan of the counts (each
// segment's digits in order, each digit's tiles in order), then a stable scatter.
// A tile is taken in rounds of 256 consecutive pairs; within a wave the pairs with
// the same digit are found by eight ballots and ranked by lane, and the waves'
// counts are added in wave order, the rounds in order.  The scatter first places
// the tile's pairs in LDS in digit order, then writes each digit's run to its
// consecutive global positions.  Keys above kcap sort as kcap (a sentinel of the
// caller) but keep their value.
// ---------------------------------------------------------------------------
#define RS_TILE 4096
#define RS_ROUNDS (RS_TILE / 256)
#define RS_MAXSEG 96
struct RsSegs {
  int nseg;
  int tile0[RS_MAXSEG + 1];  // first tile of each segment; tile0[nseg] = all tiles
  int off[RS_MAXSEG + 1];    // first pair of each segment; off[nseg] = all pairs
};
// the workgroup's tile: first pair, end, and where its digit counts sit (digit d at
// cbase + d * cstride)
struct RsTile {
  long long base, end;
  size_t cbase, cstride;
};
__device__ __forceinline__ RsTile rs_tile(const RsSegs& S, int b) {
  int lo = 0, hi = S.nseg - 1;  // last segment whose first tile is <= b
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (S.tile0[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  const int j = b - S.tile0[lo], ntl = S.tile0[lo + 1] - S.tile0[lo];
  RsTile T;
  T.base = S.off[lo] + (long long)j * RS_TILE;
  T.end = T.base + RS_TILE < S.off[lo + 1] ? T.base + RS_TILE : S.off[lo + 1];
  T.cbase = (size_t)256 * S.tile0[lo] + j;
  T.cstride = (size_t)ntl;
  return T;
}
__device__ __forceinline__ unsigned rs_digit(unsigned key, unsigned kcap, int shift) {
  return ((key < kcap ? key : kcap) >> shift) & 255u;
}
// lanes of the wave whose valid pair has digit d (d < 256)
__device__ __forceinline__ unsigned long long rs_same(unsigned d, bool valid) {
  unsigned long long same = __ballot(valid);
#pragma unroll
  for (int b = 0; b < 8; b++) {
    const unsigned long long m = __ballot((d >> b) & 1u);
    same &= ((d >> b) & 1u) ? m : ~m;
  }
  return same;
}
__global__ __launch_bounds__(256) void k_rs_count(const unsigned* keys, unsigned kcap, int shift, int* cnt,
                                                  const RsSegs S) {
  __shared__ int h[256];
  const int tid = threadIdx.x, lane = tid & 63;
  const unsigned long long below = lane ? (~0ull >> (64 - lane)) : 0ull;
  const RsTile T = rs_tile(S, blockIdx.x);
  h[tid] = 0;
  __syncthreads();
  for (int r = 0; r < RS_ROUNDS; r++) {
    const long long g = T.base + r * 256 + tid;
    const bool valid = g < T.end;
    const unsigned d = rs_digit(valid ? keys[g] : 0u, kcap, shift);
    const unsigned long long same = rs_same(d, valid);
    if (valid && (same & below) == 0) atomicAdd(&h[d], __popcll(same));
  }
  __syncthreads();
  cnt[T.cbase + tid * T.cstride] = h[tid];
}
__global__ __launch_bounds__(256) void k_rs_scatter(const unsigned* kin, const int* vin, unsigned kcap, int shift,
                                                    const int* cnt, const int* off, unsigned* kout, int* vout,
                                                    const RsSegs S) {
  __shared__ unsigned sk[RS_TILE];
  __shared__ int sv[RS_TILE];
  __shared__ int lstart[256], run[256], goff[256], sh[256];
  __shared__ int wcnt[4][256];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const unsigned long long below = lane ? (~0ull >> (64 - lane)) : 0ull;
  const RsTile T = rs_tile(S, blockIdx.x);
  // where each digit's pairs start in the tile's digit order, and globally
  int tot;
  const int mine = cnt[T.cbase + tid * T.cstride];
  const int ls = block_excl_scan256(mine, sh, &tot);
  lstart[tid] = ls;
  run[tid] = ls;
  goff[tid] = off[T.cbase + tid * T.cstride];
  for (int r = 0; r < RS_ROUNDS; r++) {
    for (int w = 0; w < 4; w++) wcnt[w][tid] = 0;
    __syncthreads();
    const long long g = T.base + r * 256 + tid;
    const bool valid = g < T.end;
    const unsigned key = valid ? kin[g] : 0u;
    const int val = valid ? vin[g] : 0;
    const unsigned d = rs_digit(key, kcap, shift);
    const unsigned long long same = rs_same(d, valid);
    const int rank = __popcll(same & below);
    if (valid && rank == 0) wcnt[wave][d] = __popcll(same);
    __syncthreads();
    if (valid) {
      int pos = run[d] + rank;
      for (int w = 0; w < wave; w++) pos += wcnt[w][d];
      sk[pos] = key;
      sv[pos] = val;
    }
    __syncthreads();
    run[tid] += wcnt[0][tid] + wcnt[1][tid] + wcnt[2][tid] + wcnt[3][tid];
  }
  __syncthreads();
  const int nt = (int)(T.end - T.base);
  for (int i = tid; i < nt; i += 256) {
    const unsigned key = sk[i];
    const unsigned d = rs_digit(key, kcap, shift);
    const int gp = goff[d] + (i - lstart[d]);
    kout[gp] = key;
    vout[gp] = sv[i];
  }
}
// Scratch (ints) the sort needs for n pairs in nseg segments: the counts, their
// offsets and the scan's tile sums.
extern "C" long long lk_radix_sort_scratch(int n, int nseg) {
  const long long nt = (n + RS_TILE - 1) / RS_TILE + (nseg > 1 ? nseg : 1);
  return 2LL * 256 * nt + lk_scan_tsum_size(256LL * nt);
}
// Sorts kin/vin (left unchanged) into kout/vout, with ktmp/vtmp (all n long) between
// passes; each of the nseg segments [seg_off[i], seg_off[i+1]) (host array;
// seg_off[0] = 0, seg_off[nseg] = n, nondecreasing) is sorted on its own.
extern "C" int lk_radix_sort_segs(const unsigned* kin, const int* vin, unsigned* kout, int* vout, unsigned* ktmp,
                                  int* vtmp, int n, int nseg, const int* seg_off, int nbits, unsigned kcap,
                                  int* scratch, hipStream_t s) {
  if (n <= 0) return 0;
  if (nseg < 1 || nseg > RS_MAXSEG || seg_off[0] != 0 || seg_off[nseg] != n) return -1;
  RsSegs S;
  S.nseg = nseg;
  S.tile0[0] = 0;
  for (int i = 0; i < nseg; i++) {
    const int len = seg_off[i + 1] - seg_off[i];
    if (len < 0) return -1;
    S.off[i] = seg_off[i];
    S.tile0[i + 1] = S.tile0[i] + (len + RS_TILE - 1) / RS_TILE;
  }
  S.off[nseg] = n;
  const int nb = S.tile0[nseg];
  const int passes = nbits <= 0 ? 1 : (nbits + 7) / 8;
  int* cnt = scratch;
  int* off = scratch + 256LL * nb;
  int* tsum = off + 256LL * nb;
  const unsigned* ks = kin;
  const int* vs = vin;
  for (int pss = 0; pss < passes; pss++) {
    const bool to_out = ((passes - 1 - pss) & 1) == 0;
    unsigned* kd = to_out ? kout : ktmp;
    int* vd = to_out ? vout : vtmp;
    k_rs_count<<<nb, 256, 0, s>>>(ks, kcap, 8 * pss, cnt, S);
    lk_scan_excl(cnt, 256LL * nb, off, tsum, s);
    k_rs_scatter<<<nb, 256, 0, s>>>(ks, vs, kcap, 8 * pss, cnt, off, kd, vd, S);
    ks = kd;
    vs = vd;
  }
  return 0;
}
// The whole array as one segment.
extern "C" void lk_radix_sort_pairs(const unsigned* kin, const int* vin, unsigned* kout, int* vout, unsigned* ktmp,
                                    int* vtmp, int n, int nbits, unsigned kcap, int* scratch, hipStream_t s) {
  const int so[2] = {0, n};
  lk_radix_sort_segs(kin, vin, kout, vout, ktmp, vtmp, n, 1, so, nbits, kcap, scratch, s);
}
// Sizes of groups of sorted ids in [0, ng) (ids outside are skipped): one LDS
// histogram per workgroup, added to cnt (zeroed by the caller).
__global__ __launch_bounds__(256) void k_hist_ids(const int* ids, int n, int ng, int* cnt) {
  extern __shared__ int hh[];
  for (int g = threadIdx.x; g < ng; g += 256) hh[g] = 0;
  __syncthreads();
  // lanes with equal ids (runs, as the ids are sorted) are counted together: one
  // atomic per distinct id in a wave
  const int lane = threadIdx.x & 63;
  for (int i0 = blockIdx.x * 4096; i0 < n && i0 < (blockIdx.x + 1) * 4096; i0 += 256) {
    const int i = i0 + threadIdx.x;
    const int g = i < n ? ids[i] : -1;
    bool todo = g >= 0 && g < ng;
    while (__ballot(todo)) {
      const int lead = __ffsll((long long)__ballot(todo)) - 1;
      const int gl = __shfl(g, lead);
      const unsigned long long same = __ballot(todo && g == gl);
      if (lane == lead) atomicAdd(&hh[gl], __popcll(same));
      if (g == gl) todo = false;
    }
  }
  __syncthreads();
  for (int g = threadIdx.x; g < ng; g += 256)
    if (hh[g]) atomicAdd(&cnt[g], hh[g]);
}
__global__ __launch_bounds__(256) void k_hist_ids_global(const int* ids, int n, int ng, int* cnt) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n && ids[i] >= 0 && ids[i] < ng) atomicAdd(&cnt[ids[i]], 1);
}
extern "C" void lk_hist_ids(const int* ids, int n, int ng, int* cnt, hipStream_t s) {
  if (n <= 0 || ng <= 0) return;
  if (ng <= 16384) k_hist_ids<<<(n + 4095) / 4096, 256, sizeof(int) * (size_t)ng, s>>>(ids, n, ng, cnt);
  else k_hist_ids_global<<<(n + 255) / 256, 256, 0, s>>>(ids, n, ng, cnt);
}

// ---------------------------------------------------------------------------
// GEMM job construction: group ids per target box, then source rows.
// mode 0: M2M targets (parents), mode 1: L2L targets, mode 2: M2L targets.
// gbase[t*9 + l] = first group id of (tree, level) or -1.
// ---------------------------------------------------------------------------
__global__ void k_group_ids(int nrows, int row0, int mode, const int* box_code, const int* box_tree,
                            const int* box_level, const TreeInfo* trees, const int* gbase, int* gid, int* rowid) {
  int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= nrows) return;
  int R = row0 + r;
  int t = box_tree[R], l = box_level[R];
  unsigned code = (unsigned)box_code[R];
  int gb = gbase[t * 9 + l];
  int g = 0x7fffffff;
  if (gb >= 0) {
    if (mode == 0) g = gb;
    else if (mode == 1) g = gb + (int)(code & 7u);
    else {
      // M2L: the group, then (sort key only) the box's boundary class, so that
      // targets with the same missing interaction offsets share GEMM tiles and a
      // tile skips every operator none of its targets has
      TreeInfo T = trees[t];
      int ix, iy, iz;
      demorton3(code, l, &ix, &iy, &iz);
      const int n = 1 << l;
      auto axis = [n](int x) { return min(x, 3) * 4 + min(n - 1 - x, 3); };
      if (T.kind == 0) {
        g = (gb + (int)(code & 7u)) * M2L_BCLS + (axis(ix) * 16 + axis(iy)) * 16 + axis(iz);
      } else {
        int j = iz - (1 << (l - 1));
        if (j == 0 || j == 1) g = (gb + j * 4 + (((ix & 1) << 1) | (iy & 1))) * M2L_BCLS + (axis(ix) * 16 + axis(iy)) * 16;
      }
    }
  }
  gid[r] = g;
  rowid[r] = R;
}
// sorted M2L sort keys back to group ids
__global__ void k_m2l_key_to_group(int n, int* key) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n && key[i] != 0x7fffffff) key[i] /= M2L_BCLS;
}
extern "C" void lk_m2l_key_to_group(int n, int* key, hipStream_t s) {
  if (n) k_m2l_key_to_group<<<nblk(n, 256), 256, 0, s>>>(n, key);
}
extern "C" void lk_group_ids(int nrows, int row0, int mode, const int* box_code, const int* box_tree,
                             const int* box_level, const TreeInfo* trees, const int* gbase, int nlev1, int* gid,
                             int* rowid, hipStream_t s) {
  (void)nlev1;
  if (nrows) k_group_ids<<<nblk(nrows, 256), 256, 0, s>>>(nrows, row0, mode, box_code, box_tree, box_level, trees, gbase, gid, rowid);
}

__device__ __forceinline__ int grid_get(const long long* grid_off, const int* grid, int t, int l, int ix, int iy,
                                        int iz) {
  int n = 1 << l;
  if (ix < 0 || iy < 0 || iz < 0 || ix >= n || iy >= n || iz >= n) return -1;
  long long go = grid_off[t * 9 + l];
  if (go < 0) return -1;
  return grid[go + morton3(ix, iy, iz)];
}

// adds the wave's per-lane counts to *npairs (a wave sum, one atomic per wave); every
// lane of the wave calls it
__device__ __forceinline__ void count_wave(int cnt, unsigned long long* npairs) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) cnt += __shfl_xor(cnt, m, 64);
  if ((threadIdx.x & 63) == 0 && cnt) atomicAdd(npairs, (unsigned long long)cnt);
}
// M2L sources from interaction templates (free: offsets within the same tree;
// reaction: absolute source depth in a polarisation-source tree)
// Also counts the products with a source present (a wave sum, one atomic per wave).
// (restrict: the table written never aliases the lookups, so the loads of several
// template entries can be in flight at once)
__global__ void k_src_m2l(int nent, const int* __restrict__ trow, const int* __restrict__ egrp,
                          const int* __restrict__ grp_seq0, const int* __restrict__ grp_K,
                          const Tmpl* __restrict__ tmpl, int stride, const int* __restrict__ box_code,
                          const int* __restrict__ box_level, const long long* __restrict__ grid_off,
                          const int* __restrict__ grid, int* __restrict__ srow, unsigned long long* npairs) {
  int e = blockIdx.x * 256 + threadIdx.x;
  int cnt = 0;
  if (e < nent) {
    int g = egrp[e];
    int R = trow[e];
    int l = box_level[R];
    int ix, iy, iz;
    demorton3((unsigned)box_code[R], l, &ix, &iy, &iz);
    int s0 = grp_seq0[g], K = grp_K[g];
    const unsigned n = 1u << l;
#pragma unroll 4
    for (int kk = 0; kk < K; kk++) {
      const Tmpl T = tmpl[s0 + kk];
      const int x = ix - T.dx, y = iy - T.dy, z = T.zabs ? T.dz : iz - T.dz;
      // the lookup of grid_get without branches (an empty cell or a cell outside the
      // grid reads entry 0, which always exists, and is then discarded)
      const long long go = grid_off[T.stree * 9 + l];
      const bool ok = (unsigned)x < n && (unsigned)y < n && (unsigned)z < n && go >= 0;
      const int v = grid[ok ? go + morton3(x, y, z) : 0];
      const int sr = ok ? v : -1;
      srow[(size_t)e * stride + kk] = sr;
      cnt += sr >= 0;
    }
  }
  count_wave(cnt, npairs);
}
extern "C" void lk_src_m2l(int nent, const int* trow, const int* egrp, const int* grp_seq0, const int* grp_K,
                           const Tmpl* tmpl, int stride, const int* box_code, const int* box_level,
                           const long long* grid_off, const int* grid, int* srow, unsigned long long* npairs,
                           hipStream_t s) {
  if (nent) k_src_m2l<<<nblk(nent, 256), 256, 0, s>>>(nent, trow, egrp, grp_seq0, grp_K, tmpl, stride, box_code,
                                                      box_level, grid_off, grid, srow, npairs);
}

// number of (target, source) products with a source present
// M2M and L2L sources of each target row; each kernel also counts the products with
// a source present
__global__ void k_src_m2m(int nent, const int* trow, const int* box_code, const int* box_tree, const int* box_level,
                          const long long* grid_off, const int* grid, int* srow, unsigned long long* npairs) {
  int e = blockIdx.x * 256 + threadIdx.x;
  int cnt = 0;
  if (e < nent) {
    int R = trow[e];
    int t = box_tree[R], l = box_level[R] + 1;
    unsigned code = (unsigned)box_code[R];
    long long go = grid_off[t * 9 + l];
    for (int ch = 0; ch < 8; ch++) {
      const int sr = (go < 0) ? -1 : grid[go + code * 8 + ch];
      srow[(size_t)e * 8 + ch] = sr;
      cnt += sr >= 0;
    }
  }
  count_wave(cnt, npairs);
}
extern "C" void lk_src_m2m(int nent, const int* trow, const int* box_code, const int* box_tree, const int* box_level,
                           const long long* grid_off, const int* grid, int* srow, unsigned long long* npairs,
                           hipStream_t s) {
  if (nent)
    k_src_m2m<<<nblk(nent, 256), 256, 0, s>>>(nent, trow, box_code, box_tree, box_level, grid_off, grid, srow, npairs);
}

__global__ void k_src_l2l(int nent, const int* trow, const int* box_code, const int* box_tree, const int* box_level,
                          const long long* grid_off, const int* grid, int* srow, unsigned long long* npairs) {
  int e = blockIdx.x * 256 + threadIdx.x;
  int cnt = 0;
  if (e < nent) {
    int R = trow[e];
    int t = box_tree[R], l = box_level[R];
    unsigned code = (unsigned)box_code[R];
    long long go = grid_off[t * 9 + (l - 1)];
    const int sr = (go < 0) ? -1 : grid[go + (code >> 3)];
    srow[e] = sr;
    cnt = sr >= 0;
  }
  count_wave(cnt, npairs);
}
extern "C" void lk_src_l2l(int nent, const int* trow, const int* box_code, const int* box_tree, const int* box_level,
                           const long long* grid_off, const int* grid, int* srow, unsigned long long* npairs,
                           hipStream_t s) {
  if (nent)
    k_src_l2l<<<nblk(nent, 256), 256, 0, s>>>(nent, trow, box_code, box_tree, box_level, grid_off, grid, srow, npairs);
}

// ---------------------------------------------------------------------------
// Free-space near field: phi_i += sum_{j in adjacent leaves, j != i} Q_j h0(k r_ij),
// h0(x) = e^{ix}/(ix) = sin(x)/x - i cos(x)/x (eq. (totalinteraction)).
// One workgroup per target leaf.  The targets of the leaf and tiles of the
// sources of its 27 neighbour leaves are staged in LDS (SoA).  A wave works on
// TA targets x (64/TA) sources per step (lane = target row a, source column b),
// so a leaf of any size keeps nearly every lane busy; the partial sums of the
// 64/TA source columns are combined by a butterfly over lanes, and each wave owns
// whole target blocks, so the sums are formed in a fixed order.
// When k r <= 1 holds for every pair the kernel can meet (host-checked bound),
// sin(x)/x and cos(x) are evaluated as polynomials in u = x^2 fitted on the range
// of u (errors below FP64 rounding), and 1/r comes from the hardware reciprocal
// square root refined by two Newton steps, so a pair costs no division, no square
// root and no argument reduction.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double rsqrt_nr(double r2) {
  double y = __builtin_amdgcn_rsq(r2);
  double hh = 0.5 * r2;
  y = y * fma(-hh, y * y, 1.5);
  y = y * fma(-hh, y * y, 1.5);
  return y;
}
// h0(x) = sin(x)/x - i cos(x)/x for x = k r, from u = x^2 > 0 and y = 1/x (hr + i hi).
// FORM 1: fitted polynomials of degree 7 in u for x <= 1; FORM 2: of degree 5 for
// x <= 1/2; FORM 0: sincos.
template <int FORM>
__device__ __forceinline__ void h0_pair(double u, double y, double& hr, double& hi) {
  if constexpr (FORM > 0) {
    static_assert(FORM == 1 || FORM == 2, "series forms 1 and 2");
    double ps, pc;
    if constexpr (FORM == 1) {
      // where x <= 1: polynomials of degree 7 in u fitted on [0, 1] (least squares on
      // Chebyshev nodes; largest error 1.1e-18 for sin(x)/x, 1.6e-17 for cos x)
      ps = fma(-7.5354880644876129003e-13, u, 1.6057233337039861802e-10);
      ps = fma(ps, u, -2.5052093083699723249e-8);
      ps = fma(ps, u, 2.7557319152309194144e-6);
      ps = fma(ps, u, -1.9841269841087476663e-4);
      ps = fma(ps, u, 8.3333333333331054536e-3);
      ps = fma(ps, u, -1.6666666666666665582e-1);
      ps = fma(ps, u, 9.9999999999999999992e-1);
      pc = fma(-1.1281052794952459614e-11, u, 2.0873682510844004151e-9);
      pc = fma(pc, u, -2.7557293243107711753e-7);
      pc = fma(pc, u, 2.480158717989726233e-5);
      pc = fma(pc, u, -1.3888888888579294079e-3);
      pc = fma(pc, u, 4.1666666666662798174e-2);
      pc = fma(pc, u, -4.9999999999999981584e-1);
      pc = fma(pc, u, 9.9999999999999999856e-1);
    } else {
      // where x <= 1/2: polynomials of degree 5 in u fitted on [0, 1/4] (least squares
      // on Chebyshev nodes; largest error 1.9e-17 for sin(x)/x, 2.5e-16 for cos x)
      ps = fma(-2.493193700544346251e-8, u, 2.7556981496282984831e-6);
      ps = fma(ps, u, -1.9841269403639427146e-4);
      ps = fma(ps, u, 8.3333333330769671683e-3);
      ps = fma(ps, u, -1.6666666666666117393e-1);
      ps = fma(ps, u, 9.9999999999999998093e-1);
      pc = fma(-2.740115064302131569e-7, u, 2.4801148458800499824e-5);
      pc = fma(pc, u, -1.3888888320265660306e-3);
      pc = fma(pc, u, 4.1666666663335758195e-2);
      pc = fma(pc, u, -4.9999999999992863579e-1);
      pc = fma(pc, u, 9.9999999999999975224e-1);
    }
    hr = ps;       // sin(x)/x
    hi = -pc * y;  // -cos(x)/x
  } else {
    double sn, cs;
    sincos(u * y, &sn, &cs);
    hr = sn * y;
    hi = -cs * y;
  }
}
#define P2P_TMAX 256
template <int FORM, int TA, int CH>
__global__ __launch_bounds__(256, 5) void k_p2p_free(int nseg, const int* seg_row0, const int* seg_prefix,
                                                  const int* box_start, const int* box_cnt, const int* box_code,
                                                  const int* box_tree, const int* box_level, const TreeInfo* trees,
                                                  const long long* grid_off, const int* grid, const double* px,
                                                  const double* py, const double* pz, const double* pq, const int* sg,
                                                  double* phi_tp, unsigned long long* npairs) {
  constexpr int TB = 64 / TA;
  // one record per source (k x, k y, k z, Re q, Im q): the five reads of a pair share
  // one address register, their offsets folded into the instructions
  __shared__ double s_src[5 * CH];
  __shared__ double t_x[P2P_TMAX], t_y[P2P_TMAX], t_z[P2P_TMAX], acc_r[P2P_TMAX], acc_i[P2P_TMAX];
  __shared__ int nb_start[27], nb_pre[28];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int a = lane / TB, b = lane % TB;
  int li = blockIdx.x;
  int sgm = seg_find(seg_prefix, nseg, li);
  int R = seg_row0[sgm] + (li - seg_prefix[sgm]);
  int t = box_tree[R], l = box_level[R];
  const double k = trees[t].k;
  int ix, iy, iz;
  demorton3((unsigned)box_code[R], l, &ix, &iy, &iz);
  const int s0 = box_start[R], nt = box_cnt[R];
  if (tid < 27) {
    // the own leaf (offset 0, 0, 0) first: only its sources can coincide with a target
    // (coincident points share a leaf), so only they need the select that drops them
    const int o = tid == 0 ? 13 : (tid <= 13 ? tid - 1 : tid);
    int dx = o / 9 - 1, dy = (o / 3) % 3 - 1, dz = o % 3 - 1;
    int Rn = grid_get(grid_off, grid, t, l, ix + dx, iy + dy, iz + dz);
    nb_start[tid] = Rn >= 0 ? box_start[Rn] : 0;
    nb_pre[tid + 1] = Rn >= 0 ? box_cnt[Rn] : 0;
  }
  __syncthreads();
  if (tid == 0) {
    nb_pre[0] = 0;
    for (int i = 1; i <= 27; i++) nb_pre[i] += nb_pre[i - 1];
    if (nt) atomicAdd(npairs, (unsigned long long)nt * (unsigned long long)(nb_pre[27] - 1));
  }
  __syncthreads();
  const int total = nb_pre[27];
  for (int c0 = 0; c0 < nt; c0 += P2P_TMAX) {
    const int ntp = nt - c0 < P2P_TMAX ? nt - c0 : P2P_TMAX;
    const int ntb = (ntp + TA - 1) / TA;
    if (tid < ntp) {  // coordinates in units of 1/k: r^2 is then (k r)^2
      t_x[tid] = k * px[s0 + c0 + tid];
      t_y[tid] = k * py[s0 + c0 + tid];
      t_z[tid] = k * pz[s0 + c0 + tid];
      acc_r[tid] = 0.0;
      acc_i[tid] = 0.0;
    }
    for (int base = 0; base < total; base += CH) {
      const int nch = total - base < CH ? total - base : CH;
      __syncthreads();
      for (int f = tid; f < nch; f += 256) {
        int g = base + f;
        int lo = 0, hi = 26;  // last neighbour whose prefix is <= g
        while (lo < hi) {
          int mid = (lo + hi + 1) >> 1;
          if (nb_pre[mid] <= g) lo = mid;
          else hi = mid - 1;
        }
        int ss = nb_start[lo] + (g - nb_pre[lo]);
        double* rec = s_src + 5 * f;
        rec[0] = k * px[ss];
        rec[1] = k * py[ss];
        rec[2] = k * pz[ss];
        rec[3] = pq[2 * ss];
        rec[4] = pq[2 * ss + 1];
      }
      __syncthreads();
      for (int tb = wave; tb < ntb; tb += 4) {
        const int ti = tb * TA + a;
        const bool tv = ti < ntp;
        const int tr = tv ? ti : 0;
        const double x0 = t_x[tr], y0 = t_y[tr], z0 = t_z[tr];
        double ax = 0.0, ay = 0.0;
        // one pair: SELF where the source may be the target itself (its own leaf)
        auto pair = [&](int j, auto self_tag) {
          constexpr bool SELF = decltype(self_tag)::value;
          const double* rec = s_src + 5 * j;
          double dx = x0 - rec[0], dy = y0 - rec[1], dz = z0 - rec[2];
          double u = fma(dx, dx, fma(dy, dy, dz * dz));  // (k r)^2
          const bool ok = !SELF || u > 0.0;  // the target itself (and coincident points) contribute nothing
          const double us = ok ? u : 1.0;    // (a select of the input keeps the loop free of branches)
          double hr, hi;
          h0_pair<FORM>(us, rsqrt_nr(us), hr, hi);  // 1 / (k r) from the refined rsq
          hr = ok ? hr : 0.0;
          hi = ok ? hi : 0.0;
          double qr = rec[3], qi = rec[4];
          ax = fma(qr, hr, fma(-qi, hi, ax));
          ay = fma(qr, hi, fma(qi, hr, ay));
        };
        // the chunk's sources of the own leaf (the first nt of the concatenation), then the rest
        const int nown = nt - base < nch ? (nt - base > 0 ? nt - base : 0) : nch;
        int j = b;
#pragma unroll 2
        for (; j < nown; j += TB) pair(j, std::true_type{});
#pragma unroll 2
        for (; j < nch; j += TB) pair(j, std::false_type{});
#pragma unroll
        for (int m = TB / 2; m >= 1; m >>= 1) {
          ax += __shfl_xor(ax, m, 64);
          ay += __shfl_xor(ay, m, 64);
        }
        if (b == 0 && tv) {
          acc_r[ti] += ax;
          acc_i[ti] += ay;
        }
      }
    }
    __syncthreads();
    if (tid < ntp) {
      int g = sg[s0 + c0 + tid];
      phi_tp[2 * g] += acc_r[tid];
      phi_tp[2 * g + 1] += acc_i[tid];
    }
    __syncthreads();
  }
}
// FP32 variant of the near field (mixed precision).  Coordinates relative to the
// target leaf's first particle, scaled by k, are formed in FP64 and kept as FP32 hi + lo
// pairs, so a pair difference (hi - hi) + (lo - lo) is accurate to FP32 rounding of the
// difference itself, also for the closest pairs; pairs are evaluated and partially
// summed in FP32, and each target's sum is accumulated in FP64.  With coordinates in
// units of 1/k, r2 is (k r)^2 and the reciprocal square root gives 1/(k r) directly.
// A source is one 32-byte LDS record (x, y, z, xl | yl, zl, Re q, Im q): two 16-byte
// reads at offsets the compiler folds into the instruction.  NS selects how sin(x)/x and
// cos(x), x = k r, are evaluated (v_rsq_f32 for 1/x): 7, where x <= 1 on every pair,
// polynomials of degree 4 in u = x^2 fitted on [0, 1]; 5, where x <= 1/2, polynomials
// of degree 3 fitted on [0, 1/4] (least squares on Chebyshev nodes; with the
// coefficients rounded to FP32 the largest errors are 7.1e-9 and 4.7e-9 on [0, 1],
// 8.4e-11 and 7.5e-10 on [0, 1/4], against 6e-8 for one FP32 rounding); 0 takes
// sincosf.  The neighbour leaves are taken with the target's
// own leaf first: only its sources can coincide with a target (coincident points
// share a leaf), so only they go through the select that drops coincident pairs.
template <int NS, int TA, int CH>
__global__ __launch_bounds__(256) void k_p2p_free32(int nseg, const int* seg_row0, const int* seg_prefix,
                                                    const int* box_start, const int* box_cnt, const int* box_code,
                                                    const int* box_tree, const int* box_level, const TreeInfo* trees,
                                                    const long long* grid_off, const int* grid, const double* px,
                                                    const double* py, const double* pz, const double* pq,
                                                    const int* sg, double* phi_tp, unsigned long long* npairs) {
  constexpr int TB = 64 / TA;
  __shared__ float4 s_src[2 * CH];  // per source: (x, y, z, xl), (yl, zl, qr, qi)
  __shared__ float t_x[P2P_TMAX], t_y[P2P_TMAX], t_z[P2P_TMAX], t_xl[P2P_TMAX], t_yl[P2P_TMAX], t_zl[P2P_TMAX];
  __shared__ double acc_r[P2P_TMAX], acc_i[P2P_TMAX];
  __shared__ int nb_start[27], nb_pre[28];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int a = lane / TB, b = lane % TB;
  int li = blockIdx.x;
  int sgm = seg_find(seg_prefix, nseg, li);
  int R = seg_row0[sgm] + (li - seg_prefix[sgm]);
  int t = box_tree[R], l = box_level[R];
  const double k = trees[t].k;
  int ix, iy, iz;
  demorton3((unsigned)box_code[R], l, &ix, &iy, &iz);
  const int s0 = box_start[R], nt = box_cnt[R];
  if (tid < 27) {
    const int o = tid == 0 ? 13 : (tid <= 13 ? tid - 1 : tid);  // the own leaf (offset 0, 0, 0) first
    int dx = o / 9 - 1, dy = (o / 3) % 3 - 1, dz = o % 3 - 1;
    int Rn = grid_get(grid_off, grid, t, l, ix + dx, iy + dy, iz + dz);
    nb_start[tid] = Rn >= 0 ? box_start[Rn] : 0;
    nb_pre[tid + 1] = Rn >= 0 ? box_cnt[Rn] : 0;
  }
  __syncthreads();
  if (tid == 0) {
    nb_pre[0] = 0;
    for (int i = 1; i <= 27; i++) nb_pre[i] += nb_pre[i - 1];
    if (nt) atomicAdd(npairs, (unsigned long long)nt * (unsigned long long)(nb_pre[27] - 1));
  }
  __syncthreads();
  if (nt == 0) return;
  const int total = nb_pre[27];
  const double xr = px[s0], yr = py[s0], zr = pz[s0];
  for (int c0 = 0; c0 < nt; c0 += P2P_TMAX) {
    const int ntp = nt - c0 < P2P_TMAX ? nt - c0 : P2P_TMAX;
    const int ntb = (ntp + TA - 1) / TA;
    if (tid < ntp) {
      double ux = k * (px[s0 + c0 + tid] - xr), uy = k * (py[s0 + c0 + tid] - yr), uz = k * (pz[s0 + c0 + tid] - zr);
      t_x[tid] = (float)ux;
      t_y[tid] = (float)uy;
      t_z[tid] = (float)uz;
      t_xl[tid] = (float)(ux - (double)t_x[tid]);
      t_yl[tid] = (float)(uy - (double)t_y[tid]);
      t_zl[tid] = (float)(uz - (double)t_z[tid]);
      acc_r[tid] = 0.0;
      acc_i[tid] = 0.0;
    }
    for (int base = 0; base < total; base += CH) {
      const int nch = total - base < CH ? total - base : CH;
      __syncthreads();
      for (int f = tid; f < nch; f += 256) {
        int g = base + f;
        int lo = 0, hi = 26;
        while (lo < hi) {
          int mid = (lo + hi + 1) >> 1;
          if (nb_pre[mid] <= g) lo = mid;
          else hi = mid - 1;
        }
        int ss = nb_start[lo] + (g - nb_pre[lo]);
        double ux = k * (px[ss] - xr), uy = k * (py[ss] - yr), uz = k * (pz[ss] - zr);
        float hx = (float)ux, hy = (float)uy, hz = (float)uz;
        s_src[2 * f] = make_float4(hx, hy, hz, (float)(ux - (double)hx));
        s_src[2 * f + 1] = make_float4((float)(uy - (double)hy), (float)(uz - (double)hz), (float)pq[2 * ss],
                                       (float)pq[2 * ss + 1]);
      }
      __syncthreads();
      for (int tb = wave; tb < ntb; tb += 4) {
        const int ti = tb * TA + a;
        const bool tv = ti < ntp;
        const int tr = tv ? ti : 0;
        const float x0 = t_x[tr], y0 = t_y[tr], z0 = t_z[tr], x0l = t_xl[tr], y0l = t_yl[tr], z0l = t_zl[tr];
        float ax = 0.f, ay = 0.f;
        // one pair: SELF where the source may be the target itself (its own leaf)
        auto pair = [&](int j, auto self_tag) {
          constexpr bool SELF = decltype(self_tag)::value;
          const float4 A = s_src[2 * j], B = s_src[2 * j + 1];
          float dx = (x0 - A.x) + (x0l - A.w), dy = (y0 - A.y) + (y0l - B.x), dz = (z0 - A.z) + (z0l - B.y);
          float u = fmaf(dx, dx, fmaf(dy, dy, dz * dz));  // (k r)^2
          const bool ok = !SELF || u > 0.f;               // coincident points contribute nothing
          const float y = ok ? __builtin_amdgcn_rsqf(u) : 0.f;  // 1 / (k r)
          float hr, hi;
          if constexpr (NS > 0) {
            static_assert(NS == 5 || NS == 7, "series of 5 or 7 terms");
            float ps, pc;
            if constexpr (NS == 7) {
              // the fitted quartics in u on [0, 1]
              ps = fmaf(2.6937597576e-06f, u, -1.9835866409e-04f);
              ps = fmaf(ps, u, 8.3333140695e-03f);
              ps = fmaf(ps, u, -1.6666666426e-01f);
              ps = fmaf(ps, u, 9.9999999995e-01f);
              pc = fmaf(2.4121201082e-05f, u, -1.3882960343e-03f);
              pc = fmaf(pc, u, 4.1666455375e-02f);
              pc = fmaf(pc, u, -4.9999997362e-01f);
              pc = fmaf(pc, u, 9.9999999947e-01f);
            } else {
              // the fitted cubics in u on [0, 1/4]
              ps = fmaf(-1.9703922747e-04f, u, 8.3331189572e-03f);
              ps = fmaf(ps, u, -1.6666665595e-01f);
              ps = fmaf(ps, u, 9.9999999992e-01f);
              pc = fmaf(-1.3765364239e-03f, u, 4.1664739108e-02f);
              pc = fmaf(pc, u, -4.9999990368e-01f);
              pc = fmaf(pc, u, 9.9999999925e-01f);
            }
            hr = ok ? ps : 0.f;
            hi = -pc * y;
          } else {
            const float kr = u * y;
            float sn, cs;
            sincosf(kr, &sn, &cs);
            hr = sn * y;
            hi = -cs * y;
          }
          const float qr = B.z, qi = B.w;
          ax = fmaf(qr, hr, fmaf(-qi, hi, ax));
          ay = fmaf(qr, hi, fmaf(qi, hr, ay));
        };
        // the chunk's sources of the own leaf (the first nt of the concatenation), then the rest
        const int nown = nt - base < nch ? (nt - base > 0 ? nt - base : 0) : nch;
        int j = b;
#pragma unroll 4
        for (; j < nown; j += TB) pair(j, std::true_type{});
#pragma unroll 4
        for (; j < nch; j += TB) pair(j, std::false_type{});
#pragma unroll
        for (int m = TB / 2; m >= 1; m >>= 1) {
          ax += __shfl_xor(ax, m, 64);
          ay += __shfl_xor(ay, m, 64);
        }
        if (b == 0 && tv) {
          acc_r[ti] += (double)ax;
          acc_i[ti] += (double)ay;
        }
      }
    }
    __syncthreads();
    if (tid < ntp) {
      int g = sg[s0 + c0 + tid];
      phi_tp[2 * g] += acc_r[tid];
      phi_tp[2 * g + 1] += acc_i[tid];
    }
    __syncthreads();
  }
}
extern "C" void lk_p2p_free(int nseg, const int* seg_row0, const int* seg_prefix, int total, const int* box_start,
                            const int* box_cnt, const int* box_code, const int* box_tree, const int* box_level,
                            const TreeInfo* trees, const long long* grid_off, const int* grid, const double* px,
                            const double* py, const double* pz, const double* pq, const int* sg, double* phi_tp,
                            int poly, int ta, int ch, int f32, unsigned long long* npairs, hipStream_t s) {
  if (!total) return;
  if (f32) {
#define P2P32(NS)                                                                                               \
  k_p2p_free32<NS, 8, 256><<<total, 256, 0, s>>>(nseg, seg_row0, seg_prefix, box_start, box_cnt, box_code,      \
                                                 box_tree, box_level, trees, grid_off, grid, px, py, pz, pq, sg, \
                                                 phi_tp, npairs)
    if (poly == 2) P2P32(5);
    else if (poly) P2P32(7);
    else P2P32(0);
#undef P2P32
    return;
  }
#define P2P_CASE(FO, T, C)                                                                                      \
  if (poly == FO && ta == T && ch == C) {                                                                       \
    k_p2p_free<FO, T, C><<<total, 256, 0, s>>>(nseg, seg_row0, seg_prefix, box_start, box_cnt, box_code,        \
                                              box_tree, box_level, trees, grid_off, grid, px, py, pz, pq, sg,   \
                                              phi_tp, npairs);                                                  \
    return;                                                                                                     \
  }
  P2P_CASE(1, 4, 128) P2P_CASE(1, 8, 128) P2P_CASE(1, 16, 128)
  P2P_CASE(1, 4, 256) P2P_CASE(1, 8, 256) P2P_CASE(1, 16, 256)
  P2P_CASE(1, 4, 512) P2P_CASE(1, 8, 512) P2P_CASE(1, 16, 512)
  P2P_CASE(2, 4, 128) P2P_CASE(2, 8, 128) P2P_CASE(2, 16, 128)
  P2P_CASE(2, 4, 256) P2P_CASE(2, 8, 256) P2P_CASE(2, 16, 256)
  P2P_CASE(2, 4, 512) P2P_CASE(2, 8, 512) P2P_CASE(2, 16, 512)
  P2P_CASE(0, 4, 256) P2P_CASE(0, 8, 256) P2P_CASE(0, 16, 256)
#undef P2P_CASE
  // any other request falls back to the general-purpose shape
  if (poly == 2)
    k_p2p_free<2, 8, 256><<<total, 256, 0, s>>>(nseg, seg_row0, seg_prefix, box_start, box_cnt, box_code, box_tree,
                                                box_level, trees, grid_off, grid, px, py, pz, pq, sg, phi_tp,
                                                npairs);
  else if (poly)
    k_p2p_free<1, 8, 256><<<total, 256, 0, s>>>(nseg, seg_row0, seg_prefix, box_start, box_cnt, box_code, box_tree,
                                                box_level, trees, grid_off, grid, px, py, pz, pq, sg, phi_tp,
                                                npairs);
  else
    k_p2p_free<0, 8, 256><<<total, 256, 0, s>>>(nseg, seg_row0, seg_prefix, box_start, box_cnt, box_code, box_tree,
                                                box_level, trees, grid_off, grid, px, py, pz, pq, sg, phi_tp,
                                                npairs);
}

// ---------------------------------------------------------------------------
// Reaction near field (Algorithm 1, local direct interactions): for adjacent
// leaves across the interface, the kernel
//   G = (1/k_t) int k_rho J0(k_rho rho) e^{i kz_t h + i kz_s h'} sigma/kz_t dk_rho
// by contour quadrature.  Node tables per component: kr, fac = w kr sigma/(kz_t k_t), kz_t, kz_s.
// ---------------------------------------------------------------------------
__global__ void k_nf_nodes(int nnodes, Rule rule, Stack st, int lt, int ls, int a, int b, double* nkr, double* nfac,
                           double* nkzt, double* nkzs) {
  int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= nnodes) return;
  cd kr, w;
  rule_node(rule, i, c_glx, c_glw, &kr, &w);
  double kt = st.k[lt], ks = st.k[ls];
  cd kr2 = kr * kr;
  cd kzt = csqrtd(mk(kt * kt, 0) - kr2), kzs = csqrtd(mk(ks * ks, 0) - kr2);
  cd sig[2][2];
  dev_densities(st, kr, lt, ls, sig);
  cd fac = w * kr * sig[a][b] / kzt / kt;
  nkr[2 * i] = kr.x; nkr[2 * i + 1] = kr.y;
  nfac[2 * i] = fac.x; nfac[2 * i + 1] = fac.y;
  nkzt[2 * i] = kzt.x; nkzt[2 * i + 1] = kzt.y;
  nkzs[2 * i] = kzs.x; nkzs[2 * i + 1] = kzs.y;
}
extern "C" void lk_nf_nodes(int nnodes, Rule rule, Stack st, int lt, int ls, int a, int b, double* nkr, double* nfac,
                             double* nkzt, double* nkzs, hipStream_t s) {
  if (nnodes) k_nf_nodes<<<nblk(nnodes, 256), 256, 0, s>>>(nnodes, rule, st, lt, ls, a, b, nkr, nfac, nkzt, nkzs);
}

__global__ __launch_bounds__(256) void k_nf_react(int nleaf, int row0, int ttree, int ncomp, const NFComp* comps,
                                                  const int* box_start, const int* box_cnt, const int* box_code,
                                                  const TreeInfo* trees, const long long* grid_off, const int* grid,
                                                  const double* px, const double* py, const double* pz,
                                                  const double* pq, const int* sg, const double* nkr,
                                                  const double* nfac, const double* nkzt, const double* nkzs,
                                                  double* phi_tp) {
  int R = row0 + blockIdx.x;
  TreeInfo T = trees[ttree];
  int l = T.depth;
  int ix, iy, iz;
  demorton3((unsigned)box_code[R], l, &ix, &iy, &iz);
  if (iz != (1 << (l - 1))) return;  // only leaves touching the interface
  int s0 = box_start[R], nt = box_cnt[R];
  for (int tt = threadIdx.x; tt < nt; tt += 256) {
    int st = s0 + tt;
    double x0 = px[st], y0 = py[st], h0 = pz[st];
    cd acc = mk(0, 0);
    for (int c = 0; c < ncomp; c++) {
      NFComp C = comps[c];
      for (int dx = -1; dx <= 1; dx++)
        for (int dy = -1; dy <= 1; dy++) {
          int Rs = grid_get(grid_off, grid, C.stree, l, ix + dx, iy + dy, (1 << (l - 1)) - 1);
          if (Rs < 0) continue;
          int a0 = box_start[Rs], cn = box_cnt[Rs];
          for (int j = 0; j < cn; j++) {
            int ss = a0 + j;
            double ddx = x0 - px[ss], ddy = y0 - py[ss];
            double rho = sqrt(ddx * ddx + ddy * ddy), hs = -pz[ss];
            cd g = mk(0, 0);
            for (int nd = C.node0; nd < C.node0 + C.nnodes; nd++) {
              cd kr = mk(nkr[2 * nd], nkr[2 * nd + 1]);
              cd kzt = mk(nkzt[2 * nd], nkzt[2 * nd + 1]), kzs = mk(nkzs[2 * nd], nkzs[2 * nd + 1]);
              cd fac = mk(nfac[2 * nd], nfac[2 * nd + 1]);
              cd e = cexpd(cmul_i(kzt * h0 + kzs * hs));
              g = g + fac * dev_besselJ0(kr * rho) * e;
            }
            acc = acc + mk(pq[2 * ss], pq[2 * ss + 1]) * g;
          }
        }
    }
    int gg = sg[st];
    phi_tp[2 * gg] += acc.x;
    phi_tp[2 * gg + 1] += acc.y;
  }
}
extern "C" void lk_nf_react(int nleaf, int row0, int ttree, int ncomp, const NFComp* comps, const int* box_start,
                             const int* box_cnt, const int* box_code, const TreeInfo* trees, const long long* grid_off,
                             const int* grid, const double* px, const double* py, const double* pz, const double* pq,
                             const int* sg, const double* nkr, const double* nfac, const double* nkzt,
                             const double* nkzs, double* phi_tp, hipStream_t s) {
  if (nleaf && ncomp)
    k_nf_react<<<nleaf, 256, 0, s>>>(nleaf, row0, ttree, ncomp, comps, box_start, box_cnt, box_code, trees, grid_off,
                                     grid, px, py, pz, pq, sg, nkr, nfac, nkzt, nkzs, phi_tp);
}

// ---------------------------------------------------------------------------
// Final sum over the trees in which particle i is a target (eq. (totalinteraction))
// ---------------------------------------------------------------------------
// phys: return the physical potential, the sum times i k_l / (4 pi) (the paper's
// Phi normalisation divides the physical potential by it)
__global__ void k_final_sum(int n, const int* layer, const int* inv_perm, const int* layer_start, const int* tgt_trees,
                            int max_tt, const TreeInfo* trees, const double* phi_tp, double* phi, Stack st,
                            int phys) {
  int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  int l = layer[i];
  double sx = 0, sy = 0;
  if (l >= 0) {
    int j = inv_perm[i] - layer_start[l];
    for (int c = 0; c < max_tt; c++) {
      int t = tgt_trees[l * max_tt + c];
      if (t < 0) continue;
      int g = trees[t].pt_off + j;
      sx += phi_tp[2 * g];
      sy += phi_tp[2 * g + 1];
    }
  }
  if (phys && l >= 0) {
    const double c = st.k[l] / (4.0 * LFMM_PI);
    const double rx = -sy * c, ry = sx * c;
    sx = rx;
    sy = ry;
  }
  phi[2 * i] = sx;
  phi[2 * i + 1] = sy;
}
extern "C" void lk_final_sum(int n, const int* layer, const int* inv_perm, const int* layer_start, const int* tgt_trees,
                             int max_tt, const TreeInfo* trees, const double* phi_tp, double* phi, Stack st, int phys,
                             hipStream_t s) {
  if (n)
    k_final_sum<<<nblk(n, 256), 256, 0, s>>>(n, layer, inv_perm, layer_start, tgt_trees, max_tt, trees, phi_tp, phi,
                                             st, phys);
}
