/*
 * pfmm.h -- C ABI of the MI355X space-time FMM for the heat equation.
 *
 * Operators (Watschinger, Merta, Of, Zapletal, "A parallel fast multipole
 * method for a space-time boundary element method for the heat equation"):
 *
 *   V_h  single-layer Galerkin matrix, piecewise constant in space and time
 *        (Section 2, matrix V_h; kernel eq. heat_kernel), applied by the
 *        space-time FMM of Section 3 (Algorithm 2).
 *   K_h  double-layer Galerkin matrix with the kernel alpha dG/dn_y
 *        (Section 2, operator K), here with the same piecewise-constant trial
 *        space as V_h, applied by the same FMM with the source expansion
 *        differentiated along the normal.
 *
 * Vectors are indexed by (k_t - 1) E_x + k_x (time-major, Section 2) with
 * 0-based steps and triangles: index = step * n_triangles + triangle.
 *
 * Every call returns a pfmm_status.  Nothing throws or aborts across the
 * ABI.  On a non-OK status pfmm_last_error() returns a thread-local message
 * describing the failure.
 *
 * Memory: mesh and time arrays are HOST pointers, copied during
 * pfmm_build_tree (the caller may free them afterwards).  Vectors passed to
 * the apply calls are DEVICE pointers on the tree's device.  The tree owns
 * every device buffer it allocates; applies allocate nothing.
 *
 * Streams: `stream` is a hipStream_t passed as void* (NULL = the default
 * stream).  Applies are stream-ordered and asynchronous.  A tree may be used
 * by one stream at a time; concurrent applies on one tree race.
 *
 * Buffer lengths cannot be checked: passing shorter buffers than documented
 * is undefined behaviour.
 */
#ifndef PFMM_H
#define PFMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PFMM_OK = 0,
    PFMM_EINVAL = -1,        /* invalid argument, parameter or mesh            */
    PFMM_ENOMEM = -2,        /* host or device allocation failed / over budget */
    PFMM_EDEVICE = -3,       /* HIP runtime error or no usable gfx950 device   */
    PFMM_ENOTCONV = -4,      /* iterative solver did not converge              */
    PFMM_ENONFINITE = -5,    /* non-finite input detected                      */
    PFMM_EUNSUPPORTED = -6   /* valid input outside what this build supports   */
} pfmm_status;

typedef enum {
    PFMM_FP64 = 0,           /* farfield and nearfield in FP64                 */
    PFMM_MIXED_FP32 = 1,     /* M2L (eq. m2l) with FP32 moments and operator
                                entries on FP32 matrix cores with FP32
                                accumulation, on every level with >= 32 time
                                intervals; nearfield, S2M, M2M, L2L, L2T, the
                                locals and the final sum stay FP64           */
    PFMM_MIXED_BF16 = 2      /* as PFMM_MIXED_FP32 with moments, table entries
                                and operator entries rounded to bfloat16 and
                                multiplied on the BF16 matrix cores with FP32
                                accumulation (levels with equal intervals;
                                levels with unequal ones multiply the same
                                bfloat16 values on the FP32 matrix cores)    */
} pfmm_precision;

/* how the nearfield blocks (Section 3.4, eq. eval_sl_nf_block) are applied */
typedef enum {
    PFMM_NF_STORED = 0,      /* causal blocks assembled once and streamed from
                                device memory at every apply                  */
    PFMM_NF_TOEPLITZ = 1     /* uniform steps make a block entry depend on the
                                triangles and the step difference only: keep
                                the distinct values per (leaf spatial box, d)
                                and read them at every apply (no block storage);
                                needs uniform steps                          */
} pfmm_nearfield_mode;

/* which operators pfmm_build_tree assembles (bit mask).  PFMM_OP_K1: the
   double layer with trial functions piecewise linear and continuous in space
   (nodal hat functions at the mesh vertices, Section 2), stored nearfield
   only */
enum { PFMM_OP_V = 1, PFMM_OP_K = 2, PFMM_OP_K1 = 4 };

typedef struct pfmm_tree pfmm_tree;   /* opaque */

typedef struct {
    double   alpha;          /* heat capacity constant alpha > 0 (Section 2).       default 1   */
    int32_t  m_t;            /* Lagrange degree in time, 0..16 (eq. kernel_approx). default 6   */
    int32_t  m_x;            /* Chebyshev total degree in space, 0..16.             default 6   */
    int32_t  n_max;          /* refine a box iff it holds >= n_max elements (Alg. 1) default 64 */
    double   c_st;           /* box-size coupling constant (eq. rel_h_t_h_x).      default 0.9 */
    int32_t  n_tr;           /* spatial cut, grid distance (eq. 03:Iarea); -1 none. default 5   */
    int32_t  q_reg;          /* Gauss points per direction, regular panel pairs.   default 4   */
    int32_t  q_sing;         /* Gauss points per direction, touching panel pairs.  default 5   */
    int32_t  precision;      /* pfmm_precision of the applies; a MIXED tree also
                                keeps the FP64 path (pfmm_set_precision).     default FP64 */
    int32_t  operators;      /* PFMM_OP_V | PFMM_OP_K | PFMM_OP_K1.          default V and K */
    int32_t  check_finite;   /* 1: reject non-finite mesh/time input.              default 1   */
    int32_t  nearfield_mode; /* pfmm_nearfield_mode.                               default STORED */
    int32_t  nearfield_gemm; /* Toeplitz mode: 1 runs the leaf boxes whose leaves are
                                time translates as GEMMs on the FP64 matrix cores
                                (another summation order), 0 keeps the stored
                                mode's order everywhere.                   default 1   */
    uint64_t device_mem_budget; /* bytes the tree may allocate; 0 = 90% of free memory */
} pfmm_params;

typedef struct {
    int32_t  depth;              /* largest level of the box cluster tree            */
    int32_t  n_levels_far;       /* levels >= 2 that carry expansions                */
    int64_t  boxes;              /* boxes of the tree (all levels)                   */
    int64_t  leaves;             /* leaf boxes                                       */
    int64_t  near_entries;       /* causal nearfield entries of one operator's blocks
                                    (the block layout is the same for V_h and K_h)  */
    int64_t  m2l_pairs;          /* (target, source) pairs of all interaction lists  */
    int64_t  near_row_groups;    /* (leaf, time step) row groups of the nearfield    */
    int64_t  distinct_integrals; /* entries of the distinct panel-integral table    */
    uint64_t device_bytes;       /* device memory owned by the tree                  */
    int32_t  m2l_matrix_cores;   /* 1: M2L on FP64 matrix cores, 0: vector units,
                                    -1: not decided (host-only planning)           */
    int32_t  near_gemm_groups;   /* Toeplitz nearfield: leaf spatial boxes whose
                                    products run as GEMMs on the FP64 matrix cores
                                    (0 in the stored mode, -1 host-only planning)  */
    int32_t  n_time_classes;     /* largest number of distinct (target interval,
                                    source interval) geometries of the M2L over the
                                    levels >= 2 (2 when every level has equal
                                    intervals: the offsets of 2 and 3 intervals)  */
    int64_t  near_entries_V;     /* entries stored for V_h: near_entries if V_h is
                                    built in the stored mode, else 0               */
    int64_t  near_entries_K;     /* entries stored for K_h, likewise (coplanar zeros
                                    included: K_h shares V_h's block layout)       */
    int64_t  near_nonzero_K;     /* causal nearfield entries of K_h between panels
                                    that are not coplanar (the others are exactly
                                    zero): the entries K_h's product must read      */
    int64_t  near_entries_K1;    /* entries stored for the p1 double layer: three
                                    per source triangle and target element (its
                                    local vertices), 0 if not built             */
} pfmm_stats;

/* Fill *out with the default parameters above.  Returns PFMM_EINVAL on NULL. */
pfmm_status pfmm_default_params(pfmm_params* out);

/*
 * Build the space-time box cluster tree (Algorithm 1), its nearfield and
 * interaction lists (eqs. 03:ILtemp, 03:Iarea, def_st_nearfield,
 * def_st_interaction_list), the expansion tables, and assemble the stored
 * nearfield blocks of the requested operators on the GPU (Section 3.4,
 * eq. eval_sl_nf_block).
 *
 *  vertices    host, n_vertices x 3 doubles, row-major
 *  triangles   host, n_triangles x 3 int32, 0-based vertex indices; the
 *              surface must be closed and consistently oriented (outward
 *              normals by the right-hand rule)
 *  time_nodes  host, n_steps + 1 strictly increasing doubles.  Any step
 *              count: Algorithm 1 halves a time interval at the node nearest
 *              its midpoint (the earlier of two equally near), so intervals
 *              of one level may differ in length and leaves may sit on
 *              several levels of one time range.  Steps may differ in length
 *              (graded or adaptive grids, Section 3.2): then every stored
 *              nearfield entry is integrated for its own step pair and the
 *              M2L operators for each pair of interval lengths and distance;
 *              PFMM_NF_TOEPLITZ then returns PFMM_EUNSUPPORTED, and so do
 *              the learned preconditioner's calls (its features assume one
 *              step length).  Steps equal to within 1e-12 relative count as
 *              uniform.
 *  p           parameters (NULL = defaults)
 *  device      HIP device ordinal
 *  stream      hipStream_t as void* used for the assembly
 *  out         receives the tree; *out is NULL on failure
 *
 * Errors: PFMM_EINVAL (bad arguments/mesh), PFMM_ENONFINITE, PFMM_ENOMEM
 * (over budget, checked before allocating), PFMM_EDEVICE, PFMM_EUNSUPPORTED.
 */
pfmm_status pfmm_build_tree(const double* vertices, int64_t n_vertices,
                            const int32_t* triangles, int64_t n_triangles,
                            const double* time_nodes, int64_t n_steps,
                            const pfmm_params* p, int32_t device, void* stream,
                            pfmm_tree** out);

/*
 * f = V_h w by the FMM (Algorithm 2).  w_dev and f_dev are device arrays of
 * n_steps * n_triangles doubles in the natural order; f is overwritten.
 * w_dev and f_dev must not alias.  Asynchronous on `stream`.
 * Errors: PFMM_EINVAL (NULL, or V not built), PFMM_EDEVICE (launch failure).
 */
pfmm_status pfmm_apply_V(pfmm_tree* t, const double* w_dev, double* f_dev, void* stream);

/* f = K_h u, same conventions as pfmm_apply_V (K must have been built). */
pfmm_status pfmm_apply_K(pfmm_tree* t, const double* u_dev, double* f_dev, void* stream);

/*
 * f = K_h u for the double layer with p1-continuous trial functions in space
 * (Section 2: the Dirichlet datum's discretisation, nodal hat functions phi_v
 * at the mesh vertices, p0 in time; tested with p0 x p0):
 *   f[kt E_x + kx] = sum_{jt, v} K_h[(kt, kx), (jt, v)] u[jt n_vertices + v].
 * u_dev: device, n_steps * n_vertices doubles (time-major, the vertex order
 * of pfmm_build_tree); f_dev: n_steps * n_triangles doubles (natural order),
 * overwritten.  The FMM is the double layer's with per-vertex S2M moments;
 * the nearfield blocks hold three columns per source triangle.  Needs
 * PFMM_OP_K1 at build.  Asynchronous on `stream`; u_dev, f_dev must not alias.
 * Errors: PFMM_EINVAL (NULL, K1 not built), PFMM_EDEVICE.
 */
pfmm_status pfmm_apply_K1(pfmm_tree* t, const double* u_dev, double* f_dev, void* stream);

/*
 * Select the farfield precision of the following applies of t (and of the
 * solves, which call the same apply).  PFMM_FP64 is always available;
 * PFMM_MIXED_FP32 and PFMM_MIXED_BF16 need a tree built with either of them
 * (which holds FP32 moments and FP32 / BF16 tables besides the FP64 data).
 * Not stream-ordered: call it between applies, not while one is being
 * enqueued.  Errors: PFMM_EINVAL (NULL tree, unknown precision, FP32 data
 * not built).
 */
pfmm_status pfmm_set_precision(pfmm_tree* t, int32_t precision);

/*
 * Autotuner of the M2L launch configuration (eq. m2l on the matrix cores;
 * the paper's kernels are CPU code, so these choices are this library's
 * own).  For every level >= 2 with equal intervals and each farfield
 * precision the tree holds (FP64; FP32, whose choice BF16 shares), it times
 * the candidate configurations on this device -- interval blocks per
 * workgroup (32, 64 or 128 intervals) and interaction-list shares (1, 2, 3,
 * 4, 6, 8; 1..4 for levels with fewer than 32 intervals) -- with one warm-up
 * and three launches between HIP events each, and keeps the fastest for the
 * tree's later applies.  The choices are cached in the text file cache_path
 * (one JSON object; NULL: no cache), keyed by the device's architecture and
 * compute-unit count and the level's shape (coefficients per box, intervals,
 * slots, slot pairs of the interaction lists, precision); a later call for
 * the same shapes applies the cached choices without timing.  Results of
 * later applies change only by the summation order of the shares (FP64:
 * ~1e-15 relative).  Levels with unequal intervals keep their class-aware
 * kernel.  Synchronous on `stream`; may reallocate the tree's partial-locals
 * buffer; not allowed while stage profiling is on.  n_tuned and n_cached
 * (may be NULL) receive the (level, precision) pairs timed and those taken
 * from the cache.
 * Errors: PFMM_EINVAL (NULL tree, profiling on, cache not writable),
 * PFMM_ENOMEM, PFMM_EDEVICE.
 */
pfmm_status pfmm_autotune(pfmm_tree* t, const char* cache_path, void* stream, int32_t* n_tuned, int32_t* n_cached);

/* Counts and sizes of a built tree. */
pfmm_status pfmm_tree_stats(const pfmm_tree* t, pfmm_stats* out);

/*
 * Host-only planning: build the tree and lists of Algorithm 1 / Section 3.3
 * on the CPU and report their counts, without touching any GPU.  Same
 * argument conventions as pfmm_build_tree; device_bytes reports the memory a
 * build would allocate.
 */
pfmm_status pfmm_plan_stats(const double* vertices, int64_t n_vertices,
                            const int32_t* triangles, int64_t n_triangles,
                            const double* time_nodes, int64_t n_steps,
                            const pfmm_params* p, pfmm_stats* out);

/*
 * Stage timing with HIP events recorded on the apply stream.  When enabled,
 * each apply records an event pair around every stage; pfmm_profile_read
 * synchronises those events and returns accumulated milliseconds and launch
 * counts per stage (indices: 0 permute, 1 S2M, 2 M2M, 3 M2L, 4 L2L, 5 L2T,
 * 6 nearfield, 7 unpermute), then resets them.  n_stages receives 8.
 */
pfmm_status pfmm_profile_enable(pfmm_tree* t, int32_t enable);
pfmm_status pfmm_profile_read(pfmm_tree* t, double* ms, int64_t* counts, int32_t* n_stages);

/*
 * Dirichlet solve (Section 2, system 02:linear:system; Section 5 solves it
 * with GMRES without preconditioner to a relative precision of 1e-8).
 */
typedef struct pfmm_precond pfmm_precond;   /* learned preconditioner, below */

typedef struct {
    double  rtol;            /* stop when the relative residual
                                ||b - V_h w_k||_2 / ||b||_2 <= rtol.              default 1e-8 */
    int32_t max_iter;        /* Krylov dimension; no restart, 1..100000.         default 200  */
    int32_t inner_precision; /* pfmm_precision of the inner applies of the
                                refinement solve (see pfmm_solve_V_precond); a
                                reduced one needs a tree built in a MIXED mode.
                                default PFMM_FP64 */
    const double* x0_dev;    /* initial iterate (device, natural order, may equal
                                w_dev: the solve then resumes in place), NULL =
                                zero.  An iterate already within rtol returns it
                                unchanged after 0 iterations.     default NULL */
    const pfmm_precond* precond; /* learned preconditioner (pfmm_precond_create /
                                _load / _train) for the refinement solve, NULL =
                                none.                                 default NULL */
    const char* precond_path;    /* weights file (pfmm_precond_save format) loaded
                                for the call when precond is NULL; NULL = none.
                                default NULL */
} pfmm_solve_opts;

typedef struct {
    int32_t iters;               /* GMRES iterations (V_h applies in the Arnoldi loop)         */
    int32_t converged;           /* 1 if the estimate reached rtol                             */
    double  rel_residual;        /* GMRES estimate at exit                                     */
    double  true_rel_residual;   /* ||b - V_h w||_2 / ||b||_2, recomputed with one more apply  */
    double  seconds;             /* wall time of the call                                      */
    double* history;             /* optional caller-owned HOST array receiving the estimate
                                    before iteration 1 (= 1) and after every iteration; NULL = none */
    int32_t history_cap;         /* entries available in history                              */
    int32_t history_len;         /* entries written                                            */
    int32_t outer;               /* pfmm_solve_V_precond: refinement steps (FP64 residuals)    */
    int32_t precond_fallback;    /* pfmm_solve_V_precond: 1 if it fell back to plain GMRES     */
} pfmm_solve_info;

/* Fill *out with the defaults above.  Returns PFMM_EINVAL on NULL. */
pfmm_status pfmm_default_solve_opts(pfmm_solve_opts* out);

/*
 * Solve V_h w = b.  With the default options (no preconditioner, FP64 inner
 * precision) this is GMRES as in Section 5: no restart, FP64 Arnoldi with
 * classical Gram-Schmidt applied twice, Givens rotations, from w_0 = x0_dev
 * (zero when NULL) on the residual b - V_h w_0, stopped when the estimate of
 * ||b - V_h w_k||_2 / ||b||_2 reaches rtol.  With o->precond, o->precond_path
 * or a reduced o->inner_precision it runs the FP64 iterative refinement of
 * pfmm_solve_V_precond instead (judged by the FP64 residual), from x0_dev.
 * b_dev and w_dev are device arrays of n_steps * n_triangles doubles in the
 * natural order and must not alias.  o = NULL takes the defaults; info may
 * be NULL.  Synchronous: returns after the solve has finished on `stream`.
 * Allocates (max_iter + 1) Krylov vectors (about twice that for the
 * refinement solve) for the duration of the call and frees them.
 * Errors: PFMM_EINVAL (NULL, bad options, V not built, unreadable weights
 * file), PFMM_ENOMEM (workspace larger than free device memory),
 * PFMM_ENONFINITE (b, x0 or an Arnoldi value not finite), PFMM_ENOTCONV
 * (max_iter reached; w_dev then holds the last iterate and info is filled),
 * PFMM_EDEVICE.
 */
pfmm_status pfmm_solve_V(pfmm_tree* t, const double* b_dev, double* w_dev, const pfmm_solve_opts* o,
                         pfmm_solve_info* info, void* stream);

/*
 * b = (1/2 M_h + K_h) g, the right-hand side of the Dirichlet system, for the
 * projected datum g (device, natural order; M_h is the diagonal p0 x p0 mass
 * matrix |gamma_k| h_t).  Needs K_h built; asynchronous on `stream` like an
 * apply; g_dev and b_dev must not alias.  With it a caller can form b on a
 * tree holding only K_h, release it, and solve on a tree holding only V_h
 * (for problems whose two nearfields do not fit the device together).
 * Errors: PFMM_EINVAL (NULL, K not built), PFMM_EDEVICE.
 */
pfmm_status pfmm_dirichlet_rhs(pfmm_tree* t, const double* g_dev, double* b_dev, void* stream);

/*
 * Solve the Dirichlet problem V_h w = (1/2 M_h + K_h) g for the projected
 * datum g (device, natural order, the p0 coefficients of the Dirichlet data;
 * M_h is the diagonal p0 x p0 mass matrix |gamma_k| h_t).  Needs both V_h and
 * K_h built.  Same options (initial iterate, preconditioner, inner
 * precision), conventions and errors as pfmm_solve_V; one more
 * right-hand-side vector is allocated for the call.
 */
pfmm_status pfmm_solve_dirichlet(pfmm_tree* t, const double* g_dev, double* w_dev, const pfmm_solve_opts* o,
                                 pfmm_solve_info* info, void* stream);

/*
 * The Dirichlet system with the datum in p1-continuous functions (Section 2,
 * system 02:linear:system as discretised there): g_dev holds the
 * coefficients per step and vertex of the projected datum (device,
 * n_steps * n_vertices, time-major), M_h is the mixed mass matrix
 *   M_h[(kt, kx), (jt, v)] = delta_{kt jt} (t_{kt+1} - t_kt) |gamma_kx| / 3
 * for the vertices v of triangle kx, and K_h the p1 double layer
 * (pfmm_apply_K1).  pfmm_dirichlet_rhs_p1 forms b = (1/2 M_h + K_h) g
 * (n_steps * n_triangles, natural order; needs PFMM_OP_K1);
 * pfmm_solve_dirichlet_p1 solves V_h w = b as pfmm_solve_V does (needs V_h
 * and PFMM_OP_K1; same options, conventions and errors; one more
 * right-hand-side vector is allocated for the call).
 */
pfmm_status pfmm_dirichlet_rhs_p1(pfmm_tree* t, const double* g_dev, double* b_dev, void* stream);
pfmm_status pfmm_solve_dirichlet_p1(pfmm_tree* t, const double* g_dev, double* w_dev, const pfmm_solve_opts* o,
                                    pfmm_solve_info* info, void* stream);

/*
 * Batches of independent problems (trees on one device, each holding V_h).
 * pfmm_apply_V_batch computes f_i = V_h^(i) w_i for every tree i of the
 * batch in one stream-ordered call: the applies are captured once into a HIP
 * graph whose branches run on up to 8 internal streams (tree i on branch
 * i mod 8, in batch order: put the largest problems first), and the graph is
 * replayed while the vector pointers and the trees' farfield precisions
 * (pfmm_set_precision) stay the same (a change re-captures).
 * w_dev[i], f_dev[i]: device arrays of tree i's size, natural order, not
 * aliasing.  The batch keeps pointers to the trees: destroy it before them.
 * Stage profiling must be off for the trees of a batch.
 * Errors: PFMM_EINVAL (NULL or empty, a tree without V_h, trees on different
 * devices or repeated, profiling on), PFMM_ENOMEM, PFMM_EDEVICE.
 */
typedef struct pfmm_batch pfmm_batch;
pfmm_status pfmm_batch_create(pfmm_tree* const* trees, int32_t n, pfmm_batch** out);
pfmm_status pfmm_apply_V_batch(pfmm_batch* b, const double* const* w_dev, double* const* f_dev, void* stream);
/*
 * Cross-problem M2L of a batch (default on): the M2L of the levels whose
 * intervals differ in length (class-aware kernel) runs for all trees of the
 * batch in one launch per (precision, time offset) -- a 1D grid over every
 * (tree, level) unit's workgroups -- between the trees' upward passes and
 * nearfields and their downward passes, each in the graph's branches.
 * Applies to batches whose trees share the degrees m_t, m_x; otherwise, and
 * with enable = 0, every tree's apply runs whole in its branch.  Results
 * are the same either way (bitwise).  Changing the setting re-captures on
 * the next apply.  Errors: PFMM_EINVAL (NULL).
 */
pfmm_status pfmm_batch_set_cross_m2l(pfmm_batch* b, int32_t enable);
void pfmm_batch_destroy(pfmm_batch* b);

/*
 * Learned temporal-block preconditioner (not part of the paper, whose GMRES
 * is unpreconditioned).  It maps the local space-time neighbourhood of a
 * residual r to the correction z(j, k) = s (c . x + N(x)): with u = r / (D s)
 * (D the diagonal of V_h, s the root mean square of r / D), for each lag
 * f < features the inputs x are u(step j - f, k), the mean of u(j - f, .)
 * over the 3 edge neighbours of triangle k and its mean over their own
 * neighbours other than k (input index 3 f + ring).  c is a linear stencil
 * fitted by least squares; N is a small FP32 perceptron (3 x features ->
 * hidden -> hidden -> 1, tanh, no biases) fitted to what c leaves; with
 * hidden = 0 there is no N.  The weights are independent of the mesh, so a
 * preconditioner trained on one tree can be applied on another.
 *
 * pfmm_precond_create: stencil zero, random (Glorot-uniform, seeded)
 *   perceptron weights on a device; features (time lags) 1..32, hidden
 *   0..256.
 * pfmm_precond_train: runs a plain FP64 GMRES solve of V_h x = b on tree t
 *   to 1e-10, takes x_k at n_snap iterations spread over the solve and
 *   n_snap of its Krylov basis vectors v_j, forms the pairs
 *   (r = V_h e, e) for e = x* - x_k and e = v_j, fits c by least squares on
 *   about 2^20 samples of the pairs normalised by their s (seeded sampling),
 *   then N to the remaining error (mean squared error, Adam with a cosine
 *   decay of the step size from lr, `steps` minibatches of `batch` samples;
 *   skipped when hidden = 0).  Synchronous; allocates its workspace for the
 *   call.  final_loss (may be NULL) gets the perceptron's last batch loss,
 *   or with hidden = 0 the mean squared residual of the stencil fit.
 * pfmm_precond_apply: z for one vector v on tree t (device, natural order,
 *   v and z distinct); synchronous on `stream`.
 * pfmm_precond_save / _load: a small binary file of the weights: four int32
 *   (0x4d4c5031, version 4, features, hidden), then c (3 features), W1
 *   (3 features x hidden, row-major), W2 (hidden x hidden, row-major, input
 *   first) and w3 (hidden), all FP32 little-endian.
 * Errors: PFMM_EINVAL, PFMM_ENOMEM, PFMM_EDEVICE, PFMM_ENOTCONV (training
 *   solve did not converge), PFMM_ENONFINITE (degenerate normal equations).
 */
pfmm_status pfmm_precond_create(int32_t device, int32_t features, int32_t hidden, uint64_t seed, pfmm_precond** out);
pfmm_status pfmm_precond_train(pfmm_precond* pc, pfmm_tree* t, const double* b_dev, int32_t n_snap, int32_t steps,
                               int32_t batch, float lr, uint64_t seed, float* final_loss, void* stream);
pfmm_status pfmm_precond_apply(const pfmm_precond* pc, pfmm_tree* t, const double* v_dev, double* z_dev,
                               void* stream);
pfmm_status pfmm_precond_save(const pfmm_precond* pc, const char* path);
pfmm_status pfmm_precond_load(const char* path, int32_t device, pfmm_precond** out);
void pfmm_precond_destroy(pfmm_precond* pc);

/*
 * pfmm_precond_apply for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments and result as pfmm_precond_apply, but it
 * calls no hipMalloc / hipFree and does not synchronise: the work is only
 * enqueued on `stream`.  Its scratch (the diagonal of V_h per triangle, the
 * reduction partials and the three FP32 feature fields) is a device array of
 * PFMM_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it runs on
 * until the process ends; a tree needs 8 (round_up(n_triangles, 32) + 1024 +
 * ceil(3 N / 2)) bytes of it (N = n_steps * n_triangles; about 8.4M DOFs fit),
 * larger trees get PFMM_EINVAL.  All calls on one GPU share that GPU's array:
 * calls that overlap on one device (different streams or threads) race; calls
 * ordered on one stream do not.
 * Errors: PFMM_EINVAL (NULL, aliasing, V not built, tree too large),
 * PFMM_EDEVICE.
 */
#define PFMM_NOALLOC_SCRATCH_BYTES (96u << 20)
pfmm_status pfmm_precond_apply_noalloc(const pfmm_precond* pc, pfmm_tree* t, const double* v_dev, double* z_dev,
                                       void* stream);

/*
 * Solve V_h w = b by iterative refinement in FP64 around flexible GMRES
 * (right preconditioning with pc, or none when pc is NULL), the inner
 * products applied in the farfield precision `inner_precision`
 * (pfmm_precision; the reduced ones need a mixed tree); the refinement
 * starts from o->x0_dev (zero when NULL; o->precond, o->precond_path and
 * o->inner_precision are ignored here: the arguments decide).  Every refinement
 * step computes the true residual b - V_h w with the FP64 apply; the solve
 * stops when its norm relative to ||b|| reaches o->rtol, and it is judged by
 * that FP64 residual only.  Each inner solve stops at a relative reduction
 * of 1e-4 (or max_iter inner iterations).  If a refinement step fails to
 * halve the FP64 residual, or the preconditioned inner solve produces a
 * non-finite value, the solve falls back to plain FP64 GMRES from the
 * current iterate (info->precond_fallback = 1).  info->iters counts all
 * inner iterations (V_h applies), info->outer the refinement steps.  The
 * tree's precision setting is restored on return.  Workspace: about
 * 2 (max_iter + 2) vectors for the call, 1.5 more with a preconditioner
 * (its three FP32 feature fields).  Errors as pfmm_solve_V.
 */
pfmm_status pfmm_solve_V_precond(pfmm_tree* t, const pfmm_precond* pc, int32_t inner_precision, const double* b_dev,
                                 double* w_dev, const pfmm_solve_opts* o, pfmm_solve_info* info, void* stream);

/*
 * Representation formula at interior points (Section 2): for zero initial
 * data, the solution inside the domain is u = V~ w - W u with the
 * single-layer potential V~ (kernel G) of the Neumann trace w = alpha du/dn
 * and the double-layer potential W (kernel alpha dG/dn_y) of the Dirichlet
 * trace u.  For p0 x p0 traces on the tree's mesh and time grid (w from a
 * Dirichlet solve, u the projected datum) this evaluates
 *     out_i = (V~ w)(x_i, t_i) - (W u)(x_i, t_i)
 * at n_points space-time points.  Time integrals are closed-form (first
 * antiderivatives of G and G / (2 s)); each triangle's space integral uses
 * the collapsed Gauss rule with q points per direction (1..16), accurate for
 * points well inside the domain and less so as a point approaches the
 * surface (points on the surface are not supported).  Direct summation:
 * O(n_points N q^2) work, no tree expansions.
 *  w_dev, u_dev  device, natural order, N = n_steps * n_triangles doubles;
 *                either may be NULL (that potential is left out)
 *  xt_dev        device, n_points x 4 doubles (x, y, z, t) row-major
 *  out_dev       device, n_points doubles (overwritten)
 * Asynchronous on `stream`; allocates nothing once the tree is built.
 * Errors: PFMM_EINVAL (NULL tree / points / output, q or n_points out of
 * range), PFMM_EDEVICE.
 */
pfmm_status pfmm_representation(pfmm_tree* t, const double* w_dev, const double* u_dev, const double* xt_dev,
                                int64_t n_points, int32_t q, double* out_dev, void* stream);

/* Release every host and device resource of the tree.  NULL is a no-op. */
void pfmm_destroy(pfmm_tree* t);

/* Thread-local message for the last non-OK status on this thread ("" if none). */
const char* pfmm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PFMM_H */
