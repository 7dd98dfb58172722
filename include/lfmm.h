/*
 * lfmm -- fast multipole method for the 3-D Helmholtz equation in layered media
 * on AMD MI355X (gfx950).  C ABI of the HIP library liblfmm.so.
 *
 * Method: Wang, Zhang & Cai, "Fast multipole method for 3-D Helmholtz equation
 * in layered media", SIAM J. Sci. Comput. (2019).  The library evaluates, for N
 * particles with complex charges Q_j in a medium of L+1 layers,
 *
 *   Phi_l(r_i) = sum_{j in layer l, j != i} Q_j h0(k_l |r_i - r_j|)
 *              + sum over the four reaction components (up/down target part x
 *                up/down source part) of sum_j Q_j u^{**}_{l l'}(r_i, r_j),
 *
 * the total interaction of Section 3.4 eq. (totalinteraction), with the reaction
 * components (Section 3.1 eqs. (greenfuncomponent), (totaldensity)) scaled by
 * 4 pi / (i k_l) so that the free part is h0(x) = e^{ix}/(ix).  The reaction
 * components are evaluated by FMMs on equivalent polarisation sources
 * (Section 3.3 eq. (eqpolarizedsource), Algorithm 1), the free part by the classic
 * FMM, truncated at order p.
 *
 * Geometry: L interfaces z = d[0] > d[1] > ... > d[L-1]; layer 0 is z > d[0],
 * layer l (0 < l < L) is d[l] < z < d[l-1], layer L is z < d[L-1]; k[0..L] are
 * the real wavenumbers, layer 0 first.  Particles must not lie on an interface.
 *
 * Error behaviour: every call returns an lfmm_status code; nothing is printed
 * and no call aborts the process.
 */
#ifndef LFMM_H
#define LFMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LFMM_OK = 0,
  LFMM_EINVAL = 1,  /* invalid argument: plan parameters, particle data (non-finite coordinate,
                       layer id inconsistent with z, particle closer than min_gap to an interface) */
  LFMM_ENOMEM = 2,  /* device or host allocation failed */
  LFMM_EHIP = 3,    /* a HIP runtime call failed */
  LFMM_ENOTSUP = 4, /* the configuration is outside what the library supports */
  LFMM_EIO = 5,     /* a surrogate or table file could not be read or written, or does not match the plan */
  LFMM_ENOCONV = 6  /* the Sommerfeld quadrature of a reaction class (Section 3.5) would need more contour
                       nodes than the plan's budget (quad_max_nodes) to reach its truncation tolerance */
} lfmm_status;

/* Plan options; pass NULL for the defaults shown. */
typedef struct {
  double contour_b; /* depth of the deformed Sommerfeld contour (Section 3.5, b): 0.5 */
  int max_depth;    /* largest octree depth, <= 8: 8 */
  double min_gap;   /* smallest allowed particle-to-interface distance: 1e-9 */
  int profile;      /* 1: record per-stage times (adds stream events); 2: only the M2L, near field,
                       node sums, P2M and L2P stages: 0 */
  int precision;    /* 0: FP64 throughout.  1: mixed precision -- near field in FP32 and the M2L
                       on FP32 matrix cores (operators and multipole expansions rescaled per
                       level), with the Bessel/Legendre recurrences, the Sommerfeld quadrature,
                       the local-expansion accumulation and the final sums in FP64: 0 */
  int physical;     /* 0: potentials in the paper's normalisation Phi (eq. (totalinteraction): the
                       free part is sum Q_j h0(k_l r), h0(x) = e^{ix}/(ix)); 1: physical potentials,
                       Phi times i k_l / (4 pi) (free part sum Q_j e^{i k_l r} / (4 pi r)): 0 */
  int reuse_operators; /* 1: an evaluation whose trees, classes, precision and surrogate gate are the
                          same as the previous successful one's keeps that evaluation's free-space and
                          reaction operators instead of generating them again ("warm"); not in
                          lfmm_eval_batch, whose workers lend their workspaces: 0 */
  double quad_tol;     /* truncation of the Sommerfeld contour (Section 3.5): the far panels end where
                          the envelope t^N e^{-t dz} of a class's integrands has fallen to quad_tol
                          times its largest value (N = 2p + 1); in (0, 1), or 0 for e^{-40} (4e-18) */
  int64_t quad_max_nodes; /* the most contour nodes one reaction class (or one near-field reaction
                          component) may take.  The far panels' count grows as 1/dz when the target and
                          source boxes' images approach each other (dz = z_t + z_s -> 0); a class that
                          needs more fails the evaluation with LFMM_ENOCONV: 0 for 2^20 */
} lfmm_options;

typedef struct lfmm_plan_s lfmm_plan_t;

/* Per-evaluation report of the last lfmm_eval / lfmm_eval_device call. */
typedef struct {
  int n_trees;
  int free_depth[17];      /* octree depth of each layer's free-space tree (-1: empty layer) */
  int reaction_depth;      /* common depth of every reaction tree (-1: none) */
  int64_t n_boxes;         /* boxes over all trees and levels */
  int64_t n_ops_free;      /* free-space translation operators generated */
  int64_t n_react_classes; /* reaction M2L integral classes (each an (p+1)^2 x (p+1)^2 matrix) */
  int64_t n_react_nodes;   /* contour nodes summed over the classes */
  int64_t n_ops_react;     /* reaction M2L operators */
  int64_t m2l_pairs;       /* (target box, source box) M2L products, free + reaction */
  int64_t m2l_slots;       /* M2L products issued to the GEMM (including absent sources) */
  int64_t m2m_pairs;       /* (parent, child) M2M products */
  int64_t l2l_pairs;       /* (child, parent) L2L products */
  int64_t p2p_pairs;       /* free-space near-field (target, source) pairs evaluated */
  int64_t nf_react_pairs;  /* near-field reaction pairs */
  int p2p_series;          /* near field's form of h0: 1 the series (k r <= 1 on every pair), 2 the shorter
                              series (k r <= 1/2), 0 the library sin and cos */
  int precision;           /* the plan's precision option */
  double stage_ms[24];     /* per-stage device time when profiling is on (see lfmm_stage_name) */
  int64_t n_react_surrogate; /* reaction classes whose integrals came from the surrogate (gate hits);
                                the other n_react_classes - n_react_surrogate used the quadrature */
  int ops_reused;            /* 1: the operators of the previous evaluation were kept (reuse_operators) */
  int64_t n_react_table;     /* reaction classes whose integrals came from the pre-computed tables */
  int64_t workspace_bytes;   /* device workspace the evaluation used (its buffers' capacities; for
                                lfmm_eval_device_noalloc, the part of the static scratch it took) */
  int64_t p2m_points, p2m_leaves; /* points (particles and polarisation images) and leaves of the P2M */
  int64_t l2p_points, l2p_leaves; /* targets and leaves of the L2P */
  int m2l_ks;                     /* M2L K-split the evaluation used (waves sharing a 16-target tile) */
} lfmm_report;

/*
 * lfmm_plan -- fix the layered medium and the FMM parameters: the stack of Section 3.1
 * (interfaces z = d_l, layer l between d_l and d_{l-1}, wavenumber k_l in layer l), the
 * truncation order p of the expansions of Sections 2 and 3.3 and the leaf bound of the
 * trees of Section 3.4.
 *   L        number of interfaces (0 <= L <= 16; L = 0 is free space)
 *   d        host array of L interface heights, strictly decreasing (copied)
 *   k        host array of L+1 wavenumbers, each > 0 (copied)
 *   p        truncation order of the expansions, 1 <= p <= 10 ((p+1)^2 coefficients)
 *   leaf_max largest number of particles allowed in a leaf before refinement (>= 1)
 *   opt      NULL or options
 *   out      receives the plan (owned by the library; release with lfmm_destroy)
 * Returns LFMM_EINVAL for invalid parameters, LFMM_EHIP/LFMM_ENOMEM on device errors.
 */
int lfmm_plan(int L, const double* d, const double* k, int p, int leaf_max, const lfmm_options* opt,
              lfmm_plan_t** out);

/*
 * lfmm_eval_device -- Phi at every particle (targets = sources), device memory: the total
 * interaction of Section 3.4 eq. (totalinteraction) -- the free-space sum within each
 * layer plus the four reaction components of every layer pair (Section 3.1 eq.
 * (greenfuncomponent)) -- by Algorithm 1 (Section 3.4) on the polarisation sources of
 * Section 3.3 eq. (eqpolarizedsource).
 *   n        number of particles (0 <= n < 2^31)
 *   xyz      device, 3*n doubles, structure of arrays: x[0..n), y[0..n), z[0..n)
 *   layer    device, n int32 layer ids or NULL (then derived from z); when given,
 *            each id must equal the layer containing z, else LFMM_EINVAL
 *   q        device, 2*n doubles, charges interleaved (re, im)
 *   phi      device, 2*n doubles, output interleaved (re, im); written entirely
 *   stream   hipStream_t to run on (NULL: the default stream); the call returns
 *            after the result is complete on that stream
 * Buffers are owned by the caller and must not overlap phi.  The plan keeps a
 * device workspace between calls; calls on one plan must not overlap.
 */
int lfmm_eval_device(lfmm_plan_t* plan, int64_t n, const double* xyz, const int32_t* layer, const double* q,
                     double* phi, void* stream);

/*
 * lfmm_eval_device_noalloc -- lfmm_eval_device without any allocation: for callers
 * that cannot allocate (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  The evaluation's whole device workspace is
 * taken from a static device array of LFMM_NOALLOC_BYTES that the library holds
 * on every device it runs on until the process ends; no device or pinned host
 * memory is allocated (host bookkeeping uses ordinary heap memory).  Arguments,
 * layout and results are those of lfmm_eval_device, and the potentials are
 * bit-identical to its own.  The call is synchronous: it returns after every
 * stream it used has finished.
 *   - must be called with the plan's device current (else LFMM_EINVAL);
 *   - LFMM_ENOMEM if the evaluation needs more workspace than LFMM_NOALLOC_BYTES
 *     (lfmm_report.workspace_bytes of an ordinary evaluation of the same problem
 *     tells how much it needs); nothing is allocated instead, and phi is then
 *     undefined;
 *   - the operators of an earlier evaluation are never kept (reuse_operators does
 *     not apply);
 *   - every call on one device shares that device's scratch: calls that overlap in
 *     time on one device (from several threads or plans) race and must not be made.
 */
#define LFMM_NOALLOC_BYTES ((size_t)512 << 20)
int lfmm_eval_device_noalloc(lfmm_plan_t* plan, int64_t n, const double* xyz, const int32_t* layer, const double* q,
                             double* phi, void* stream);

/* lfmm_eval -- the same with host buffers (copied to and from the device). */
int lfmm_eval(lfmm_plan_t* plan, int64_t n, const double* xyz, const int32_t* layer, const double* q, double* phi);

/*
 * lfmm_eval_targets_device -- Phi at a separate set of target points (the total
 * interaction of Section 3.4 eq. (totalinteraction) evaluated at r = target):
 *   Phi_l(t) = sum_{sources j in layer l, |t - r_j| > 0} Q_j h0(k_l |t - r_j|)
 *            + sum over all sources of the reaction components,
 * l being the target's layer.  A source at exactly the target's position is left
 * out of the free part (the kernel is singular there), as for targets = sources.
 *   n_src, src_xyz, src_layer, q   sources as in lfmm_eval_device
 *   n_tgt, tgt_xyz, tgt_layer      targets (device, SoA 3*n_tgt doubles; layer ids or NULL --
 *                                  src_layer and tgt_layer are both given or both NULL)
 *   phi                            device, 2*n_tgt doubles, output interleaved (re, im)
 * The method runs on the union of sources and targets (targets with zero charge),
 * so the plan's trees cover both; n_src + n_tgt < 2^31.  Errors as lfmm_eval_device.
 */
int lfmm_eval_targets_device(lfmm_plan_t* plan, int64_t n_src, const double* src_xyz, const int32_t* src_layer,
                             const double* q, int64_t n_tgt, const double* tgt_xyz, const int32_t* tgt_layer,
                             double* phi, void* stream);

/* lfmm_eval_targets -- the same with host buffers. */
int lfmm_eval_targets(lfmm_plan_t* plan, int64_t n_src, const double* src_xyz, const int32_t* src_layer,
                      const double* q, int64_t n_tgt, const double* tgt_xyz, const int32_t* tgt_layer, double* phi);

/*
 * lfmm_eval_batch -- many independent problems at once (each its own medium and
 * particles, each with its own plan).  Problem i evaluates Phi at its n[i]
 * particles exactly as lfmm_eval_device(plans[i], n[i], xyz[i], layer ? layer[i]
 * : NULL, q[i], phi[i], ...) would.  nworkers host threads (<= 0: 8) take problems
 * in turn, each on a stream of its own, so the problems' kernels overlap on the
 * GPU.  All pointers in xyz/layer/q/phi are device pointers; layer may be NULL.
 * The plans must be distinct.  status (host, nprob ints, may be NULL) receives
 * each problem's code; the return value is LFMM_OK if every problem succeeded,
 * else the first failing code.  Returns after every problem is complete.
 */
int lfmm_eval_batch(int nprob, lfmm_plan_t* const* plans, const int64_t* n, const double* const* xyz,
                    const int32_t* const* layer, const double* const* q, double* const* phi, int nworkers,
                    int* status);

/*
 * Positions once, charges many times.
 *
 * lfmm_prepare -- the charge-independent part of lfmm_eval_device for these positions
 * (n, xyz, layer as there): classification, the trees of Section 3.4, interaction
 * lists, and the free-space and reaction translation operators (Section 2; Section 3.5,
 * eq. (me2lesimplified)).  No charges are read.  Returns once the work is complete.
 *
 * lfmm_apply -- Phi at the prepared positions for charges q (device, 2n doubles,
 * interleaved re/im as in lfmm_eval_device) into phi (device, 2n doubles): the
 * charge-dependent kernels of Algorithm 1 (Section 3.4) from the upward pass on -- P2M,
 * M2M, M2L, L2L, L2P, the near fields and the component sum -- queued on `stream` in one
 * stream order.  The call synchronises nothing, allocates nothing and clears memory with
 * kernels only, so it can be captured into a HIP graph.  The result equals
 * lfmm_eval_device's for the same positions and charges bit for bit.  Valid after
 * lfmm_prepare, or lfmm_eval_device on the plan's own workspace, until the plan's next
 * evaluation (LFMM_EINVAL otherwise); calls on one plan must not overlap.
 */
int lfmm_prepare(lfmm_plan_t* plan, int64_t n, const double* xyz, const int32_t* layer, void* stream);
int lfmm_apply(lfmm_plan_t* plan, const double* q, double* phi, void* stream);

/*
 * lfmm_batch -- many independent layered problems (each its own medium, particles and
 * plan) evaluated by one launch of one HIP graph.
 *
 * lfmm_batch_prepare runs lfmm_prepare for every problem on nworkers host threads
 * (<= 0: 8), each on a stream of its own; status (host, nprob ints, may be NULL)
 * receives each problem's code, the return value the first failing one.
 *
 * lfmm_batch_capture captures lfmm_apply of every prepared problem, with charges q[i]
 * and output phi[i] (device pointers), on nbranch (<= 0: 4, at most 16) independent
 * branches of one graph, the problems spread over the branches by size (largest first,
 * each to the least loaded branch), and instantiates it.  No problem is evaluated.
 *
 * lfmm_batch_launch launches that graph on `stream`: every problem's phi[i] then equals
 * lfmm_eval_device(plans[i], n[i], xyz[i], layer[i], q[i], ...) bit for bit, for
 * whatever q[i] holds when the graph runs.  The plans must be distinct, and must be
 * neither evaluated, prepared again nor destroyed while the batch is used; the q and
 * phi buffers must stay allocated.  rep (may be NULL) receives the batch's sizes.
 */
typedef struct lfmm_batch_s lfmm_batch_t;
typedef struct {
  int64_t n_total;     /* particles over all problems */
  int64_t graph_nodes; /* kernel and dependency nodes of the captured graph */
  int branches;        /* independent branches of the graph */
  double capture_ms;   /* host wall time of the capture and instantiation */
} lfmm_batch_report;
int lfmm_batch_prepare(int nprob, lfmm_plan_t* const* plans, const int64_t* n, const double* const* xyz,
                       const int32_t* const* layer, int nworkers, int* status);
int lfmm_batch_capture(int nprob, lfmm_plan_t* const* plans, const double* const* q, double* const* phi,
                       int nbranch, lfmm_batch_t** out, lfmm_batch_report* rep);
int lfmm_batch_launch(lfmm_batch_t* batch, void* stream);
void lfmm_batch_destroy(lfmm_batch_t* batch);

/* Report of the last evaluation on this plan. */
int lfmm_last_report(const lfmm_plan_t* plan, lfmm_report* rep);

/* Name of stage index i of lfmm_report.stage_ms (NULL past the last). */
const char* lfmm_stage_name(int i);

/* Release a plan and its device memory (NULL is ignored). */
void lfmm_destroy(lfmm_plan_t* plan);

/* Text of a status code. */
const char* lfmm_status_string(int status);

/* The HIP error behind the library's last LFMM_EHIP, from any thread (its name, code and
 * the library source line that saw it), or "" if there was none.  The string belongs to
 * the library and stays valid until the next failing HIP call after the next one. */
const char* lfmm_last_hip_error(void);

/* Contour nodes of the Sommerfeld quadrature (Section 3.5: the deformed contour, then panels of
 * the real axis truncated where the integrand envelope t^{2p+1} e^{-t dz} has decayed to quad_tol,
 * widened up to the J_q(t rho) oscillation limit) that a plan with these arguments uses for one
 * reaction class at vertical image distance dz = z_t + z_s > 0 and horizontal distance rho >= 0.
 * Arguments as lfmm_plan; no device is touched, so it serves for budgeting on any host.
 * *nodes receives the count; LFMM_ENOCONV when it exceeds opt->quad_max_nodes (*nodes then still
 * holds the count, or 0 beyond 2^30), LFMM_EINVAL for invalid arguments. */
int lfmm_quad_nodes(int L, const double* d, const double* k, int p, const lfmm_options* opt, double dz,
                    double rho, int64_t* nodes);

/* ---- tile-shape autotuning ---- */
typedef struct {
  int gemm_ks;          /* chosen M2L K-split (waves sharing a 16-target tile's operator sequence) */
  int p2p_ta, p2p_ch;   /* chosen near-field tile shape (FP64 series path: targets per wave step,
                           sources per LDS tile); the mixed path has one shape */
  int trials;           /* evaluations timed */
  double ms_default, ms_best; /* time per evaluation with the default and the chosen shapes */
} lfmm_tune_report;

/*
 * Time whole evaluations of the given particles (device buffers, as lfmm_eval_device,
 * on the given stream) over the tile shapes the library carries -- M2L K-split 1, 2, 4, 8;
 * for FP64 plans the near-field shapes (4, 8, 16 targets per wave step x 128, 256, 512
 * sources per tile) -- one coordinate at a time, and keep the fastest for later
 * evaluations of this plan.  phi receives the last evaluation's potentials.  The shapes
 * change only the summation order, so results agree to rounding.  rep is optional (host).
 * Errors: as lfmm_eval_device.
 */
int lfmm_autotune(lfmm_plan_t* plan, int64_t n, const double* xyz, const int32_t* layer, const double* q, double* phi,
                  void* stream, lfmm_tune_report* rep);

/* Set a plan's tile shapes to ones lfmm_autotune carries (for instance those it chose on
 * a representative problem): M2L K-split gemm_ks in {1, 2, 4, 8}; near-field p2p_ta in
 * {4, 8, 16} targets per wave step and p2p_ch in {128, 256, 512} sources per tile.
 * Later evaluations use them; LFMM_EINVAL for other values. */
int lfmm_set_tiles(lfmm_plan_t* plan, int gemm_ks, int p2p_ta, int p2p_ch);

/* ---- learned surrogate of the reaction M2L integrals ----
 *
 * The integral matrices I[(n,m),(n',m')] of the reaction M2L operators (Section 3.5,
 * eq. (me2lesimplified) with the integrals written out in Section 3.5) depend on a
 * class geometry: component (target layer and direction, source layer and direction),
 * box size h, the heights j, i in {0, 1} of the target and source boxes above and
 * below the interface and the lateral offset class rho^2/h^2 in {0,1,2,4,5,8,9,10,13,18}.
 * The surrogate is a multilayer perceptron (SiLU hidden layers, linear output) that
 * maps this geometry to the whole matrix (the m >= 0 rows), normalised by the
 * low-frequency size of each entry and per-output statistics.  It stands where the
 * paper uses pre-computed interpolation tables; the quadrature stays the fallback
 * and the reference for every value.  Its weights and activations are BF16 on the matrix
 * cores with FP32 accumulation; the FP32 master weights are trained on the GPU by
 * the library's own forward and backward kernels (mean squared error, Adam).
 *
 * Gate: training holds out a fraction of the sampled classes and records, for every
 * geometry combination (component, j, i, rho class), twice the largest held-out
 * error of the predicted matrices in the norm that weighs entry (n, n') by
 * (k_t h)^n (k_s h)^n' / ((2n+1)!! (2n'+1)!!) (the size of its effect on expansions of
 * boxes of size h).  An evaluation uses the network for a class only if its h lies in
 * the trained range and its combination's bound is <= the gate tolerance; every other
 * class is integrated by quadrature.  With the gate closed (tolerance 0, the default)
 * the evaluation is bit-identical to one without a surrogate.
 */
typedef struct {
  double h_min, h_max; /* box sizes covered: 0.02 .. 2.0 */
  int epochs;          /* passes over the training classes: 150 */
  int batch;           /* classes per Adam step: 256 */
  double lr;           /* initial Adam step size, cosine-decayed to 1/100 of it: 2e-3 */
  double holdout;      /* fraction of each combination's classes held out for the gate: 0.1 */
  int width, nhidden;  /* hidden-layer width and count: 128, 4 */
} lfmm_train_opts;

typedef struct {
  int64_t n_train, n_holdout; /* classes (one integral matrix each) */
  int64_t n_values;           /* complex integral values in the training set */
  int n_combos;               /* geometry combinations of the plan's medium */
  int nin, nout;              /* network input and output widths */
  int epochs, steps;
  double loss_first, loss_last; /* training loss (normalised mean squared error): first step, last epoch */
  double err_median, err_max;   /* held-out weighted relative errors of the integral matrices */
  double ms_labels, ms_train;   /* wall time of the quadrature labels and of the training */
} lfmm_train_report;

/*
 * Train the plan's surrogate: n_samples classes (0: 48 per geometry combination)
 * with log-uniform box sizes, labelled by the library's quadrature on the GPU;
 * seed fixes the sampling, initialisation and batch order.  opts and rep are
 * optional (host).  Replaces a previous surrogate; the gate keeps its tolerance.
 * Errors: LFMM_EINVAL (L = 0: no reaction field; bad options), LFMM_ENOMEM, LFMM_EHIP.
 */
int lfmm_surrogate_train(lfmm_plan_t* plan, int64_t n_samples, uint64_t seed, const lfmm_train_opts* opts,
                         lfmm_train_report* rep);

/* Write the surrogate (network, statistics, gate bounds, medium) to a file; LFMM_EINVAL if none, LFMM_EIO. */
int lfmm_surrogate_save(const lfmm_plan_t* plan, const char* path);

/* Read a surrogate written for the same medium and order p; LFMM_EIO if unreadable or mismatched. */
int lfmm_surrogate_load(lfmm_plan_t* plan, const char* path);

/* Gate tolerance (>= 0; 0 closes the gate) for later evaluations of this plan. */
int lfmm_surrogate_gate(lfmm_plan_t* plan, double tol);

/*
 * Held-out error bound of each geometry combination of the plan's surrogate
 * (host, capacity n; ordered by component, then j, i, rho class; +inf where a
 * combination had no held-out class), and the number written in *count.
 */
int lfmm_surrogate_bounds(const lfmm_plan_t* plan, int n, double* bounds, int* count);

/* ---- pre-computed tables of the reaction M2L integrals ----
 *
 * The paper's alternative to integrating every class at run time (Section 3.5:
 * tables of the integrals on a grid, polynomial interpolation in the FMM), in the
 * form a uniform tree needs: a class is a geometry combination (as for the
 * surrogate) at a box size h, so the paper's tables over (rho, z, z') reduce along
 * the tree's geometry to one table in h per combination.  Each holds the
 * normalised matrix (the m >= 0 rows) at Chebyshev points of the second kind on
 * equal panels of u = ln h + alpha h, alpha = 4 max_l k_l, built by the library's
 * quadrature on the GPU, and is interpolated by the barycentric formula (FP64,
 * in HBM).  Bound of a combination: twice the largest error, in the surrogate's
 * norm, at validation points halfway (in angle) between nodes against the
 * quadrature.  Gate: a class uses the tables if its h lies in the tabulated range
 * and its combination's bound is <= the gate tolerance; the tables take precedence
 * over the surrogate; a closed gate (0, the default) leaves evaluations
 * bit-identical to ones without tables.
 */
typedef struct {
  double h_min, h_max; /* box sizes covered: 0.02 .. 2.0 */
  int nnode;           /* Chebyshev points per panel: 16 (2 .. 32) */
  double du;           /* largest panel width in u: 1.5 */
  int nval;            /* validation points per panel: 4 (at most nnode - 1) */
} lfmm_table_opts;

typedef struct {
  int n_combos, npanel, nnode;
  int64_t n_slots;            /* tabulated matrices (combinations x panels x nodes) */
  int64_t n_validation;       /* validation classes */
  int64_t bytes;              /* device memory of the tables */
  double err_median, err_max; /* validation errors (weighted relative, as the bounds) */
  double ms_build, ms_validate;
} lfmm_table_report;

/*
 * Build the plan's tables (opts and rep optional, host).  Replaces previous tables;
 * the gate keeps its tolerance.  Errors: LFMM_EINVAL (L = 0; bad options, more than
 * 4096 panels), LFMM_ENOMEM, LFMM_EHIP.
 */
int lfmm_tables_build(lfmm_plan_t* plan, const lfmm_table_opts* opts, lfmm_table_report* rep);

/* Gate tolerance (>= 0; 0 closes the gate) for later evaluations of this plan. */
int lfmm_tables_gate(lfmm_plan_t* plan, double tol);

/* Validated bound of each geometry combination (ordered as lfmm_surrogate_bounds). */
int lfmm_tables_bounds(const lfmm_plan_t* plan, int n, double* bounds, int* count);

/* Free the tables' device memory (the gate then has nothing to select). */
int lfmm_tables_release(lfmm_plan_t* plan);

/* Write the tables (layout, bounds, medium, values) to a file; LFMM_EINVAL if none, LFMM_EIO. */
int lfmm_tables_save(const lfmm_plan_t* plan, const char* path);

/* Read tables written for the same medium and order p; LFMM_EIO if unreadable or mismatched. */
int lfmm_tables_load(lfmm_plan_t* plan, const char* path);

/*
 * One forward and backward pass of a network of the surrogate's form on the GPU
 * (component check of the kernels): B rows of x [B][nin], parameters packed per
 * layer as W [out][in] row-major then b [out] (FP32; weights and x are rounded to
 * BF16 as the network holds them), targets t [B][nout].  Out: y [B][nout], the
 * gradient of the mean squared error in the parameters' packing, and the loss.
 * All host arrays.  Errors: LFMM_EINVAL, LFMM_ENOMEM, LFMM_EHIP.
 */
int lfmm_mlp_forward_backward(int B, int nin, int width, int nhidden, int nout, const float* x, const float* params,
                              const float* t, float* y, float* grad, double* loss);

/* ---- component entry points (the same kernels the evaluation runs) ---- */

/*
 * Free-space translation operator of the addition theorems (Section 2.1):
 * new_{nm} = sum_{nu,mu} Op[(n,m)][(nu,mu)] old_{nu,mu}; kind 0 regular (M2M with
 * b = parent - child centre, L2L with b = child - parent centre), kind 1 singular
 * (M2L with b = target - source centre).  Computed on the GPU for wavenumber kw;
 * out: host, (p+1)^4 complex as re/im pairs, row-major over idx(n,m) = n*n+n+m.
 */
int lfmm_translation(lfmm_plan_t* plan, int kind, double kw, const double* b, double* out);

/*
 * Reaction M2L operator T (Section 3.3 eqs. (metoleimage1)-(metoleimage2), in the
 * Phi normalisation and the polarisation frame): target layer l with direction a
 * (0 up, 1 down), source layer lp with direction b, lateral offset (dx, dy) of the
 * target centre from the polarisation-source centre, target-centre height zt > 0
 * above the interface and source-centre depth zs > 0 below it.  Computed on the
 * GPU by contour quadrature; out as for lfmm_translation.
 */
int lfmm_reaction_operator(lfmm_plan_t* plan, int l, int a, int lp, int b, double dx, double dy, double zt, double zs,
                           double* out);

/*
 * Reaction densities sigma^{ab}_{l,lp}(k_rho) (Section 3.1) at n complex points
 * (host, re/im pairs) computed on the GPU; out: host, n x 4 complex
 * (up-up, up-down, down-up, down-down), zero where the component does not exist.
 */
int lfmm_densities(lfmm_plan_t* plan, int n, const double* krho, int l, int lp, double* out);

#ifdef __cplusplus
}
#endif
#endif /* LFMM_H */
