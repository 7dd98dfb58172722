// Shared declarations between the host orchestration and the kernels.
#pragma once
#include "lfmm_device.h"

#define LFMM_NSTAT 12  // per-layer statistics gathered by the classification kernel
#define M2L_BCLS 4096  // boundary classes of M2L targets (16 per axis) in the job sort key

// One octree of the evaluation: a free-space tree of one layer, a reaction
// target tree (layer l, direction a) or a reaction polarisation-source tree
// (layer lp, direction b).  kind: 0 free, 1 reaction target, 2 reaction source.
struct TreeInfo {
  double lo[3];
  double S;
  double k;
  int kind;
  int layer;
  int dir;     // 0 up, 1 down (reaction trees)
  int depth;
  int npts;
  int pt_off;  // first tree-point index
  int pad0, pad1;
};

// One product of the surrogate network, C = A B with BF16 operands
// (A(m, k) = A[m am + k ak], B(k, n) = B[k bk + n bn]) and an epilogue:
//   MLP_EPI_STORE  C = A B (+ bias[n]) in FP32
//   MLP_EPI_SILU   C = A B + bias[n] in FP32 and Cb = bf16(silu(C))
//   MLP_EPI_DSILU  Cb = bf16((A B) silu'(Zs))
enum { MLP_EPI_STORE = 0, MLP_EPI_SILU = 1, MLP_EPI_DSILU = 2 };
#define MLP_MSE_BLOCKS 256
struct MlpGemm {
  int M, N, K, mode;
  const unsigned short* A;
  long am, ak;
  const unsigned short* B;
  long bk, bn;
  const float* bias;
  float* C;
  long ldc;
  unsigned short* Cb;
  long ldcb;
  const float* Zs;
  long ldz;
};

// Free-space translation operator request.
struct OpDesc {
  double bx, by, bz, k;
  int kind;  // 0: regular (j_q), 1: singular (h_q)
  int op;    // destination index: in the shift array (kind 0) or the M2L array (kind 1)
};

// One geometry class of the reaction M2L integrals.
struct ClassDesc {
  Rule rule;
  double zt, zs, rho;
  int lt, ls, a, b;  // target layer, source layer, directions
  int out;           // index of the integral matrix
  int rg_off;        // first node of its rule group in the node tables
  int f_off;         // first entry of its F values
  int pad;
};

// A stack of reaction classes contracted together: same quadrature rule group
// and source layer, at most SC_GMAX classes and three target layers.
#define SC_GMAX 16
#define SC_UPW 5     // MFMA units per wave
#define SC_G3 true  // complex products in Gauss's three-product form
struct SCDesc {
  int rg_off, nn, ls, G;
  int mem0;   // first member in the member list
  int nlt;    // distinct target layers
  int lt[3];
  int wg0;    // first workgroup
  int NU;     // (m, row tile, column tile) units
  int pad;
};

// Quadrature rule group: classes with the same (zt + zs, rho) share these nodes.
struct RGDesc {
  Rule rule;
  double rho;
  int off;  // first node in the node tables
  int nn;
};

// One reaction M2L operator: phase/prefactor applied to a class integral.
struct ROpDesc {
  double dx, dy;  // lateral offset target - source (in box units times h)
  double kt;
  int cls;        // integral matrix index
  int op;         // destination operator index
};

// Interaction template entry of a GEMM group.
struct Tmpl {
  int op;
  int stree;
  short dx, dy, dz, zabs;
};

// GEMM block: up to 64 * NCT targets of one group (NCT column tiles per wave).
struct GBlock {
  int e0;     // first entry
  int nt;     // targets in the block
  int seq0;   // first template / op entry of the group
  int K;      // number of operators in the group
};

// M2L operators (FP64, and FP32 in the mixed path) are stored k-step by k-step (4
// source coefficients each): the NRT full tiles of 16 rows in MFMA A-operand lane
// order (lane = row % 16 + 16 (col % 4)), then, when (p+1)^2 = 16 NRT + 1, the 4
// values of the last row, which the GEMM accumulates on the vector ALU instead of
// in a sixteen-row tile that would hold one useful row.  (M2M and L2L operators keep
// the row-tile-major layout of the shift GEMM.)
__host__ __device__ inline int m2l_nrt(int NC) { return (NC % 16 == 1) ? NC / 16 : (NC + 15) / 16; }
__host__ __device__ inline int m2l_xr(int NC) { return (NC % 16 == 1) ? 1 : 0; }
// Near-field reaction pair table for one (target tree, source tree) component.
struct NFComp {
  int node0, nnodes;  // node range in the node tables
  int stree;
  int pad;
};

extern "C" {
// kernel launch wrappers (lfmm_kernels.hip)
void lk_set_gl(const double* x, const double* w);
void lk_zero(double* p, size_t n, hipStream_t s);
void lk_fill_int(int* p, size_t n, int v, hipStream_t s);
// stable partition by layer: per-block counts cnt[l * nb + b] (nb = ceil(n / 256)),
// then, with off = their exclusive scan, perm[slot] = particle and inv[particle] = slot
void lk_layer_count(int n, int NL, const int* layer, int* cnt, hipStream_t s);
void lk_layer_scatter(int n, int NL, const int* layer, const int* off, int* perm, int* inv, hipStream_t s);
void lk_dbg_dens(int n, const double* kr, Stack st, int l, int lp, double* out, hipStream_t s);
void lk_classify(int n, const double* x, const double* y, const double* z, const int* lin, int* lout, Stack st,
                 double* partial, int nblocks, hipStream_t s);
void lk_reduce_stats(int nblocks, int nl, const double* partial, double* stats, hipStream_t s);
void lk_tree_points(int ntp, int ntrees, const TreeInfo* trees, const int* perm, const int* layer_start,
                    const double* x, const double* y, const double* z, const double* q, Stack st, unsigned* keys,
                    int* vals, double* rec, hipStream_t s);
void lk_occupancy(int ntp, int ntrees, const unsigned* skeys, const TreeInfo* trees, int leaf_max, int* occ,
                  int* slab, hipStream_t s);
void lk_gather(int ntp, const int* sg, const double* rec, double* px, double* py, double* pz, double* pq,
               hipStream_t s);
void lk_point_origin(int ntp, int ntrees, const TreeInfo* trees, const int* perm, const int* layer_start,
                     const int* sg, int* orig, hipStream_t s);
void lk_gather_q(int ntp, const int* orig, const double* q, double* pq, hipStream_t s);
void lk_transop(int nops, const OpDesc* descs, double* sops, int opsz, double* ops, int opsz_m, int p, int NC,
                int NKS, const double* gaunt, float* ops32, const int* opse, hipStream_t s);
// Ltab != nullptr (stacks with more than four interfaces): per-node layer tables,
// 6 (L + 1) Ntot complex, from which k_react_F assembles the densities.
void lk_react_tables(int nrg, const RGDesc* rgs, int Ntot, Stack st, int p, double* Jtab, double* Ptab,
                     double* Ltab, hipStream_t s);
void lk_react_F(int ncls, const ClassDesc* cls, int Ftot, Stack st, int Ntot, const double* Ltab, double* Ftab,
                hipStream_t s);
void lk_react_mfma(int nwg, int nsc, const SCDesc* scs, const int* members, const ClassDesc* cls, int p, int Ntot,
                   const double* Jtab, const double* Ptab, const double* Ftab, double* Iout, int NC, hipStream_t s);
// grp: (first, count) per class over rops sorted by class, at most 8 operators a class
void lk_react_expand(int ngrp, const int* grp, const ROpDesc* rops, const double* Iall, double* ops, int opsz, int p,
                     int NC, int NKS, float* ops32, const int* opse, hipStream_t s);
void lk_p2m(int nseg, const int* seg_row0, const int* seg_prefix, int total, const int* box_start,
            const int* box_cnt, const int* box_code, const int* box_tree, const int* box_level,
            const TreeInfo* trees, const double* px, const double* py, const double* pz, const double* pq, int p,
            int NCK, double* M, hipStream_t s);
void lk_l2p(int nseg, const int* seg_s0, const int* seg_prefix, int total, const int* leafrow, const int* box_code,
            const int* box_tree, const int* box_level, const TreeInfo* trees, const double* px, const double* py,
            const double* pz, const int* sg, int p, int NCK, const double* Lc, double* phi_tp, hipStream_t s);
void lk_group_ids(int nrows, int row0, int mode, const int* box_code, const int* box_tree, const int* box_level,
                  const TreeInfo* trees, const int* gbase, int nlev1, int* gid, int* rowid, hipStream_t s);
// also adds the number of slots with a source present to *npairs
void lk_src_m2l(int nent, const int* trow, const int* egrp, const int* grp_seq0, const int* grp_K,
                const Tmpl* tmpl, int stride, const int* box_code, const int* box_level, const long long* grid_off,
                const int* grid, int* srow, unsigned long long* npairs, hipStream_t s);
void lk_src_m2m(int nent, const int* trow, const int* box_code, const int* box_tree, const int* box_level,
                const long long* grid_off, const int* grid, int* srow, unsigned long long* npairs, hipStream_t s);
void lk_src_l2l(int nent, const int* trow, const int* box_code, const int* box_tree, const int* box_level,
                const long long* grid_off, const int* grid, int* srow, unsigned long long* npairs, hipStream_t s);
void lk_p2p_free(int nseg, const int* seg_row0, const int* seg_prefix, int total, const int* box_start,
                 const int* box_cnt, const int* box_code, const int* box_tree, const int* box_level,
                 const TreeInfo* trees, const long long* grid_off, const int* grid, const double* px,
                 const double* py, const double* pz, const double* pq, const int* sg, double* phi_tp, int poly,
                 int ta, int ch, int f32, unsigned long long* npairs, hipStream_t s);
void lk_m_to_f32(int nrows, int NCK, int NC, const int* box_tree, const int* box_level, const int* se,
                 const double* M, float* M32, hipStream_t s);
// M2L GEMMs: blocks of 16 x (4 / ks) targets, ks waves splitting each tile's operator
// sequence; srow_stride is the longest sequence
// M2L GEMMs: allow every instance the CU's LDS (less its static LDS); the dynamic LDS
// any instance may take; the LDS one launch needs for its operator lists
// M2M and L2L on the same GEMM design (shift operators in the M2L layout, FP64)
void lk_shift_gemm64(int NC, int ks, int nblocks, const GBlock* blocks, const int* seq, const int* trow,
                     const int* srow, int srow_stride, const double* ops, int opsz, int NKS, const double* S,
                     double* D, int NCK, hipStream_t s);
void lk_m2l_gemm_init();
size_t lk_m2l_lds_max();
size_t lk_m2l_lds_bytes(int srow_stride, int ks);
void lk_gemm32(int NC, int ks, int nblocks, const GBlock* blocks, const int* seq, const int* trow, const int* srow,
               int srow_stride, const float* ops, int opsz, int NKS, const float* S, double* D, int NCK,
               const int* box_tree, const int* box_level, const int* se, hipStream_t s);
void lk_m2l_gemm64(int NC, int ks, int nblocks, const GBlock* blocks, const int* seq, const int* trow, const int* srow,
                   int srow_stride, const double* ops, int opsz, int NKS, const double* S, double* D, int NCK,
                   hipStream_t s);
void lk_nf_nodes(int nnodes, Rule rule, Stack st, int lt, int ls, int a, int b, double* nkr, double* nfac,
                 double* nkzt, double* nkzs, hipStream_t s);
void lk_nf_react(int nleaf, int row0, int ttree, int ncomp, const NFComp* comps, const int* box_start,
                 const int* box_cnt, const int* box_code, const TreeInfo* trees, const long long* grid_off,
                 const int* grid, const double* px, const double* py, const double* pz, const double* pq,
                 const int* sg, const double* nkr, const double* nfac, const double* nkzt, const double* nkzs,
                 double* phi_tp, hipStream_t s);
void lk_final_sum(int n, const int* layer, const int* inv_perm, const int* layer_start, const int* tgt_trees,
                  int max_tt, const TreeInfo* trees, const double* phi_tp, double* phi, Stack st, int phys,
                  hipStream_t s);
void lk_mlp_gemm(const MlpGemm& g, hipStream_t s);
void lk_mlp_mse(int B, int nout, const float* y, const float* t, long ldt, unsigned short* d, double* partial,
                double* loss, hipStream_t s);
void lk_mlp_colsum(int M, int N, const unsigned short* d, float* gb, hipStream_t s);
void lk_mlp_adam(long n, float* w, float* m, float* v, const float* g, float lr, float b1, float b2, float eps,
                 float c1, float c2, unsigned short* wb, hipStream_t s);
void lk_f2bf(long n, const float* x, unsigned short* y, hipStream_t s);
void lk_sur_targets(int ncls, const ClassDesc* cls, const double* dadd, Stack st, const double* Iall, int p, int NC,
                    const float* mu, const float* sd, float* T, hipStream_t s);
void lk_sur_colstats(int n, int nout, int NC, const float* T, float* mu, float* sd, hipStream_t s);
void lk_sur_write(int ncls, const ClassDesc* cls, const double* dadd, Stack st, const float* Y, int p, int NC,
                  const float* mu, const float* sd, double* Iall, hipStream_t s);
void lk_sur_err(int ncls, const ClassDesc* cls, Stack st, const double* hcls, const double* Ipred, const double* Iref,
                int p, int NC, double* err, hipStream_t s);
void lk_gather_rows(int nrows, const int* idx, int ncol, int esz, const void* src, void* dst, hipStream_t s);
void lk_sur_norm(long n, int nout, float* T, const float* mu, const float* sd, hipStream_t s);
void lk_sur_features(int n, const int* combo, const double* h, int nin, int c0, double lh0, double lh1,
                     unsigned short* X, hipStream_t s);
// box numbering: per tile of points and level the boxes opened there (lk_box_tiles(ntp)
// tiles; cnt holds nlev * tiles + 1 ints), the exclusive scan of those counts gives
// the tiles' first rows (off), from which the ranges and the box records follow
int lk_box_tiles(int ntp);
void lk_box_count(int ntp, int nlev, const unsigned* skeys, const TreeInfo* trees, int* cnt, hipStream_t s);
void lk_tree_box_range_all(int ntrees, int nlev, int ntp, const unsigned* skeys, const TreeInfo* trees,
                           const int* off, int* tb, hipStream_t s);
void lk_box_fill_all(int ntp, int nlev, const unsigned* skeys, const int* off, const TreeInfo* trees, int* box_start,
                     int* box_code, int* box_tree, int* box_level, int* leafrow, hipStream_t s);
void lk_grid_fill_all(int nrows, const int* box_start, const int* box_code, const int* box_tree,
                      const int* box_level, const TreeInfo* trees, const long long* grid_off, int* grid,
                      int* box_cnt, hipStream_t s);
void lk_m2l_key_to_group(int n, int* key, hipStream_t s);
// exclusive prefix sum of n ints (out may equal in); tsum: lk_scan_tsum_size(n) ints
void lk_scan_excl(const int* in, long long n, int* out, int* tsum, hipStream_t s);
int lk_scan_tsum_size(long long n);
// stable radix sort of (key, value) pairs on the low nbits bits of min(key, kcap);
// scratch: lk_radix_sort_scratch(n, 1) ints
long long lk_radix_sort_scratch(int n, int nseg);
void lk_radix_sort_pairs(const unsigned* kin, const int* vin, unsigned* kout, int* vout, unsigned* ktmp, int* vtmp,
                         int n, int nbits, unsigned kcap, int* scratch, hipStream_t s);
// the same within each of nseg <= 96 consecutive segments (host offsets, nseg + 1 of
// them); scratch: lk_radix_sort_scratch(n, nseg) ints; -1 on a bad segment list
int lk_radix_sort_segs(const unsigned* kin, const int* vin, unsigned* kout, int* vout, unsigned* ktmp, int* vtmp,
                       int n, int nseg, const int* seg_off, int nbits, unsigned kcap, int* scratch, hipStream_t s);
// group sizes of ids in [0, ng), added to cnt
void lk_hist_ids(const int* ids, int n, int ng, int* cnt, hipStream_t s);
void lk_tab_store(int ncls, const ClassDesc* cls, const double* dadd, const int* slot, Stack st, const double* Iall,
                  int p, int NC, double* tab, hipStream_t s);
void lk_tab_interp(int ncls, const ClassDesc* cls, const double* dadd, const int* slot0, const double* w, int nnode,
                   Stack st, const double* tab, int p, int NC, double* Iall, hipStream_t s);
}
