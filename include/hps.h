/*
 * hps.h - C ABI of the MI355X (gfx950) hierarchical Poincare-Steklov (HPS)
 * fast direct solver: batched leaf solves, level-by-level DtN merges and the
 * downward solve of arXiv 2503.17535 (Sections 3.1-3.4, Appendices A and C).
 *
 * Problem (Section 1, eqs. elliptic_BVP / dirichlet_data):
 *     L u = f  in  Omega = [lo, hi]^d,   u = g  on the boundary,
 *     L u = sum_t c_t(x) d_t u   (second-order, variable coefficients).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Uniform tree of depth L: n_leaves = 2^(d L) leaves, numbered depth first
 *   (the 2^d children of a node are contiguous; child order a,b,c,d =
 *   SW,SE,NE,NW, and in 3D e..h directly above a..d).
 * - Leaf points: p^d Chebyshev-Lobatto points (ascending -cos(pi j/(p-1))),
 *   point index ix + p*iy (+ p^2*iz).  hps_leaf_points() returns them.
 * - Coefficient terms (t): 2D  c_xx, c_xy, c_yy, c_x, c_y, c_0      (6);
 *                          3D  c_xx, c_yy, c_zz, c_xy, c_xz, c_yz,
 *                              c_x, c_y, c_z, c_0                    (10).
 * - Boundary data g lives at the q = p-2 Gauss-Legendre points of every leaf
 *   face on the domain boundary, in the order hps_boundary_points() returns
 *   (faces x-,x+,y-,y+,z-,z+ / sides S,E,N,W; each face the concatenation of
 *   its sub-faces in quadrant order).
 * - Arrays are fp64, C order, as documented per argument.  "dev" arrays are
 *   device (HBM) pointers, "host" arrays host pointers.  All array arguments
 *   are owned by the caller and only borrowed for the call (for dev arrays:
 *   until the work queued on the given stream has completed).
 * - Streams are hipStream_t passed as void* (NULL = default stream).
 * - Every int-returning function returns HPS_OK or an error code and never
 *   throws; hps_last_error() describes the last failure of the calling thread.
 */
#ifndef HPS_H_
#define HPS_H_

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  HPS_OK = 0,
  HPS_EINVAL = 1,        /* bad argument (null pointer, p or depth out of range) */
  HPS_ENOMEM = 2,        /* device or host allocation failed                      */
  HPS_ESINGULAR = 3,     /* zero pivot in a leaf (L_ii) or merge (D) factorization */
  HPS_EDEVICE = 4,       /* HIP runtime error (message has the HIP error string)  */
  HPS_EUNSUPPORTED = 5   /* valid request outside what this build implements      */
};

/* build flags */
enum {
  HPS_FLAG_ROOT_T = 1,     /* also form the root DtN matrix (unused by Dirichlet solves) */
  HPS_FLAG_NO_CHECK = 2,   /* do not synchronize at the end of hps_build to check pivots */
  HPS_FLAG_TIMING = 4,     /* record per-stage HIP events (read with hps_stage_times)   */
  HPS_FLAG_FP32_COPY = 8,  /* keep fp32 copies of the solve operators (mixed precision) */
  HPS_FLAG_FULL_PIVOT = 16, /* invert every merge matrix D whole with partial pivoting
                               (no block elimination around D's zero blocks; m <= 16384) */
  HPS_FLAG_FP32_ONLY = 32, /* with HPS_FLAG_FP32_COPY (implied): free the fp64 solve operators
                              once their fp32 copies exist; the operator then serves only
                              HPS_FP32_REFINED solves, at about half the resident bytes */
  HPS_FLAG_TEST_NO_REFINE = 1 << 30 /* test hook: skip the Newton-Schulz steps, so that an
                                       inaccurate block inverse takes the fallback below */
};

/* solve precision */
enum { HPS_FP64 = 0, HPS_FP32_REFINED = 1 };

typedef struct {
  int dim;        /* 2 or 3 */
  int depth;      /* L >= 1 (2D: L <= 12, 3D: L <= 5) */
  double lo;      /* domain [lo, hi]^dim */
  double hi;
} hps_tree_t;

typedef struct {
  long long n_leaves;     /* 2^(dim*depth)                           */
  int pts_per_leaf;       /* p^dim                                   */
  int n_terms;            /* 6 (2D) or 10 (3D)                       */
  long long n_root_bdry;  /* Gauss points on the domain boundary     */
  int n_interior;         /* (p-2)^dim interior points per leaf      */
  int n_leaf_bdry;        /* 2*dim*(p-2)^(dim-1) Gauss points / leaf */
  int n_levels;           /* merge levels = depth                    */
  long long root_D;       /* size of the root merge's D              */
} hps_sizes_t;

typedef struct hps_op hps_op_t;   /* opaque; owned by the library until hps_free */

/* Sizes of the discretization (host only, no device work). */
int hps_sizes(const hps_tree_t* tree, int p, hps_sizes_t* out);

/* Leaf Chebyshev points, host array xyz[n_leaves][p^dim][dim] (caller-allocated).
 * Callers sample coefficients and sources at these points (Section 1: the
 * method evaluates L, f, g at points of its choosing). */
int hps_leaf_points(const hps_tree_t* tree, int p, double* xyz);

/* Root-boundary Gauss points, host array xyz[n_root_bdry][dim]; the order in
 * which hps_solve reads boundary data. */
int hps_boundary_points(const hps_tree_t* tree, int p, double* xyz);

/* Accuracy of the merge inverses of one tree level (Algorithm merge,
 * "Invert D").  Every inverse Z = D^{-1} is probed with a fixed vector x:
 *   residual = max over the level's nodes of |Z (D x) - x|_inf / |x|_inf.
 * Large merge matrices (m > 112 unless HPS_FLAG_FULL_PIVOT) are inverted by
 * block elimination around their zero interface blocks, pivoting inside the
 * blocks only; for indefinite operators (Helmholtz) those blocks can be ill
 * conditioned while D is not.  Nodes whose probe residual exceeds 1e-12 then
 * get up to two Newton-Schulz steps Z <- 2Z - (Z D) Z (each squares I - Z D).
 * If a node stays above 1e-10, or a pivot inside a block is zero, the build
 * is redone with HPS_FLAG_FULL_PIVOT (partial pivoting over all of D); where
 * that is unsupported (m > 16384) hps_build returns HPS_ESINGULAR naming the
 * level and node. */
typedef struct {
  int level;            /* tree level of the parents (0 = root)                     */
  int m;                /* size of D                                                */
  long long nodes;      /* merges on the level                                      */
  int block_inverse;    /* 1: block elimination + refinement; 0: whole-D pivoting   */
  int ns_steps;         /* Newton-Schulz steps run on the worst node (0..2)         */
  double residual0;     /* max probe residual right after the inversion            */
  double residual;      /* max probe residual of the stored inverse                */
  long long worst_node; /* node index (within the level) of `residual`              */
} hps_level_info_t;

/* Per-level merge-inverse accuracy of a built operator: fills out[0..L-1]
 * (index = tree level) up to cap entries and returns the number written, or
 * a negative error code.  Synchronizes the op's build stream the first time. */
int hps_level_info(hps_op_t* op, hps_level_info_t* out, int cap);

/* Device bytes an operator built with these arguments keeps resident
 * (excluding the transient build workspace), for admission control. */
size_t hps_op_footprint(const hps_tree_t* tree, int p, int flags);

/* Build stage (Algorithm local_solve, Algorithm merge; App. A.1-A.2, C.1-C.2):
 * per leaf LU of L(I_i,I_i), Y = -L_ii^{-1} L_ie P, T = Q Y; per merge
 * D^{-1}, S = -D^{-1} C and the parent T = A - B D^{-1} C, for all levels.
 *   coeffs  dev  [n_leaves][n_terms][p^dim] coefficient samples
 *   flags   HPS_FLAG_*
 *   stream  hipStream_t the build is queued on
 *   out     receives the operator handle (NULL on error)
 * Device memory for the operator is allocated by the library.  Unless
 * HPS_FLAG_NO_CHECK is set the call synchronizes the stream once at its end:
 * it returns HPS_ESINGULAR if a pivot of a leaf or of a whole-D inversion was
 * exactly zero or not finite, and checks the merge-inverse probes (see
 * hps_level_info), redoing the build with HPS_FLAG_FULL_PIVOT when a
 * block-eliminated inverse stayed inaccurate.  With HPS_FLAG_NO_CHECK neither
 * check runs (hps_level_info still reports the probes). */
int hps_build(const hps_tree_t* tree, int p, const double* coeffs, int flags,
              void* stream, hps_op_t** out);

/* Build with subtree recomputation (Section 4.1, Algorithm "Subtree
 * recomputation strategy"), for trees whose stored operators exceed the
 * device memory.  The tree is cut subtree_depth levels above the leaves:
 * only the merge operators of the top depth - subtree_depth levels stay
 * resident, together with a device copy of the coefficients and the storage
 * of ONE subtree (its leaf factors and merges), which is rebuilt from the
 * coefficients for each subtree in turn.  The build passes over the
 * subtrees once to obtain the T of every subtree root, then merges the top
 * levels.  Every hps_solve then rebuilds each subtree, twice when a source is
 * given (once for the source's outgoing flux at the subtree root, once for
 * the downward pass from the boundary data the top levels hand down), so a
 * solve costs about the build of the subtrees plus a solve.
 *   tree           2D, depth >= 2
 *   subtree_depth  1 <= subtree_depth < depth
 *   coeffs, flags, stream, out  as for hps_build; HPS_FLAG_FP32_COPY and
 *                  HPS_FLAG_ROOT_T are rejected (HPS_EUNSUPPORTED)
 * The operator serves hps_solve with precision HPS_FP64 (same arguments,
 * results within rounding of an hps_build operator's: the arithmetic is the
 * same, only the merge inverses' Newton-Schulz gate and batch-size dependent
 * kernel choices may differ), hps_solve_adjoint (adjoint checkpointing: the
 * transposed passes in reverse order, every subtree rebuilt twice, once for
 * the g of its root and once more before its root-to-leaves part),
 * hps_coeff_grad, hps_free, hps_op_bytes (top levels + one subtree + the
 * coefficient copy), hps_level_info (the top levels) and hps_stage_times;
 * hps_solve_noalloc and hps_solve_batch return HPS_EUNSUPPORTED for it.
 * Solves and adjoint solves of one such operator rebuild its one subtree
 * plan: calls on different streams must be serialized by the caller.  The
 * build checks (see hps_build) run on every subtree and on the top levels;
 * if any asks for whole-D pivoting the whole build is redone with
 * HPS_FLAG_FULL_PIVOT, which later solves then use. */
int hps_build_subtrees(const hps_tree_t* tree, int p, const double* coeffs, int flags,
                       int subtree_depth, void* stream, hps_op_t** out);

/* Build of the ItI (impedance-to-impedance) variant (Appendix B), 2D: the
 * Poincare-Steklov operators map incoming impedance data g = u_n + i eta u to
 * outgoing data h = u_n - i eta u (Section 2), which keeps the merges well
 * posed for Helmholtz problems at any wavenumber (Section 2, related work).
 * Leaf stage (Algorithm "2D ItI local solve"): B = [G; L(I_i, :)] with the
 * Robin rows G = N~ + i eta I at the 4p - 4 boundary Chebyshev points, B^{-1}
 * by batched Gauss-Jordan, Y = B^{-1}(:, I_e) P, T = Q H Y.  Merges
 * (Appendix B.2): D = I + [[0, D12], [D21, 0]] inverted through its Schur
 * complement W = I - D12 D21 (eq. ItI_D_inv), S = -D^{-1} C, T = A + B S.
 * Every corner carries the Robin condition of the side that starts at it on a
 * counterclockwise walk of the leaf boundary (SW: S, SE: E, NE: N, NW: W).
 *   tree    2D (depth limited by W of the root merge: 8 (p - 2) 2^(depth-1)
 *           reals <= 16384, i.e. depth <= 8 at p = 16)
 *   eta     impedance parameter, > 0
 *   coeffs  dev  [n_leaves][6][p^2] real coefficient samples (as hps_build)
 *   flags   HPS_FLAG_NO_CHECK, HPS_FLAG_TIMING (others: HPS_EUNSUPPORTED)
 * Complex data are interleaved (re, im) doubles, the layout of complex128:
 * hps_solve on the returned operator reads bdry as [nrhs][n_root_bdry]
 * complex incoming impedance data at the root Gauss points (2 n_root_bdry
 * doubles per rhs), src as [nrhs][n_leaves][p^2] complex and writes u in the
 * same complex layout; precision must be HPS_FP64.  Unless HPS_FLAG_NO_CHECK
 * is set the call synchronizes once and returns HPS_ESINGULAR on a zero or
 * non-finite Gauss-Jordan pivot.  The operator serves hps_solve, hps_free,
 * hps_op_bytes and hps_stage_times; the adjoint, coefficient-gradient,
 * allocation-free, batched and level-info calls return HPS_EUNSUPPORTED. */
int hps_build_iti(const hps_tree_t* tree, int p, double eta, const double* coeffs, int flags,
                  void* stream, hps_op_t** out);

/* ---- Adaptive 3D discretization (Section 4.2) ----
 * An adaptive octree over the cube [lo, hi]^3: its leaves as int[n_leaves][4]
 * = (level, ix, iy, iz), the leaf being the box of side (hi - lo) / 2^level
 * with lower corner lo + side * (ix, iy, iz), listed in depth-first order
 * (the eight children of a node in the merge's child order: (x, y, z) offsets
 * 000, 100, 110, 010, 001, 101, 111, 011).  Leaves must tile the cube, the
 * root must be split, and face neighbours may differ by at most one level
 * (the level restriction); levels up to 20.  Host memory. */
typedef struct {
  double lo, hi;
  long long n_leaves;
  const int* leaves;
} hps_atree_t;

/* Build over an adaptive octree: the leaf stage of each leaf size (as
 * hps_build in 3D), then the non-uniform merges.  Each interior interface of
 * a merge is discretized on the coarser of its two sides, Gauss panel by
 * panel; where the other side has the four panels of a quadrant split, its
 * Dirichlet data are the coarse panel's interpolant at its Gauss points and
 * its Neumann data enter the flux balance through the interpolants of its
 * four panels evaluated at the coarse Gauss points.  D is inverted by
 * Gauss-Jordan with partial pivoting over all of D (m <= 16384).
 *   coeffs  dev  [n_leaves][10][p^3]  coefficient samples in the leaves' order
 *   flags   HPS_FLAG_TIMING or 0 (others: HPS_EUNSUPPORTED)
 * The call synchronizes once; HPS_ESINGULAR on a zero or non-finite pivot.
 * hps_solve then reads bdry as [nrhs][n_root] at the root's Gauss points (in
 * the order hps_adaptive_points(which = 2) lists them), src / u as
 * [nrhs][n_leaves][p^3] in the leaves' order; precision HPS_FP64.  The
 * operator serves hps_solve, hps_free, hps_op_bytes and hps_stage_times; the
 * adjoint, gradient, allocation-free, batched, level-info and refined-precision
 * calls return HPS_EUNSUPPORTED. */
int hps_build_adaptive(const hps_atree_t* tree, int p, const double* coeffs, int flags, void* stream,
                       hps_op_t** out);

/* Root boundary points of an adaptive operator (return value) and the size of
 * its root merge matrix D (*d_size, if non-NULL); negative on error. */
long long hps_adaptive_root_size(const hps_op_t* op, long long* d_size);

/* Points of an adaptive tree (host, [..][3] doubles, x fastest):
 *   which 0: every leaf's p^3 Chebyshev points [n_leaves][p^3][3];
 *   which 1: the Chebyshev points of every leaf's eight children
 *            [n_leaves][8][p^3][3] (the points x_1 of eq. refinement_check);
 *   which 2: the root's Gauss boundary points [n_root][3] (tree restricted).
 * hps_adaptive_root_points returns n_root (negative on error). */
int hps_adaptive_points(const hps_atree_t* tree, int p, int which, double* out);
long long hps_adaptive_root_points(const hps_atree_t* tree, int p);

/* Refinement criterion, eq. (refinement_check): split[i] = 1 unless
 * max |f1 - L_8f1 f0| < eps max |f| on leaf i, where f0 [nl][p^3] (dev) are
 * samples at the leaves' Chebyshev points, f1 [nl][8][p^3] (dev) at their
 * children's (hps_adaptive_points 0 and 1), L_8f1 the tensor interpolation
 * from a leaf's points to its children's, and max |f| the largest |f0| over
 * all leaves given.  split: host [nl].  nl <= 65535.  Synchronizes. */
int hps_adaptive_check(int p, long long nl, const double* f0, const double* f1, double eps, int* split,
                       void* stream);

/* Tree edits (host).  Each writes the resulting leaves in depth-first order
 * to out (int[..][4]) when cap is large enough and returns their number
 * (larger than cap: nothing written, call again); negative on error.
 *   split:   every leaf i with split[i] != 0 replaced by its eight children;
 *   union:   the leaves of the union of two trees (a node is split when
 *            either tree splits it);
 *   balance: leaves split until face neighbours differ by at most one level. */
long long hps_adaptive_split(const int* leaves, long long n, const int* split, int* out, long long cap);
long long hps_adaptive_union(const int* a, long long na, const int* b, long long nb, int* out, long long cap);
long long hps_adaptive_balance(const int* leaves, long long n, int* out, long long cap);

/* Build and first solve in one call, for a source known at build time (the
 * paper's form of the algorithm computes the particular solution's fluxes
 * during the merge stage, Section 3): the same operator and bitwise the same
 * u as hps_build followed by hps_solve.  The sources' leaf solves and the
 * upward pass through the merge levels that are already built run on a
 * second stream (created and destroyed by the call, default priority) beside
 * the Gauss-Jordan chains of the top merge levels; the rest follows on
 * `stream`.  Arguments as hps_build and hps_solve (precision HPS_FP64; src
 * NULL: build, then solve).  Synchronizes once, as the checked build does. */
int hps_build_solve(const hps_tree_t* tree, int p, const double* coeffs, int flags, const double* bdry,
                    const double* src, double* u, int nrhs, void* stream, hps_op_t** out);

/* Solve stage (Algorithm down_pass, with the source entering through the
 * linear upward pass of the particular solution, Section 3):
 *   bdry  dev  [nrhs][n_root_bdry]        Dirichlet data g at the root Gauss points
 *   src   dev  [nrhs][n_leaves][p^dim]    f at the leaf points, or NULL for f = 0
 *   u     dev  [nrhs][n_leaves][p^dim]    output: solution at every leaf point
 *   nrhs  >= 1; precision HPS_FP64 (HPS_FP32_REFINED needs HPS_FLAG_FP32_COPY)
 * Asynchronous on `stream`; errors from earlier device work surface as
 * HPS_EDEVICE on a later call. */
int hps_solve(hps_op_t* op, const double* bdry, const double* src, double* u,
              int nrhs, int precision, void* stream);

/* Bytes of the static device workspace of hps_solve_noalloc (per GPU). */
#define HPS_STATIC_WS_BYTES (384ull << 20)

/* Allocation-free fp64 solve, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, results and 16-rhs chunking as hps_solve with
 * precision HPS_FP64, and bitwise the same output, but the solve's working
 * vectors (boundary data and fluxes of every tree level, leaf particular
 * solutions, merge interface data, split-K partial products) live in a
 * static device array of HPS_STATIC_WS_BYTES that the library holds on every
 * GPU it runs on until the process ends, not in the operator.  The call
 * allocates nothing (no hipMalloc/hipFree, no hipMemset: what must start at
 * zero is cleared by a kernel; no stage timing).  The caller passes inputs
 * and outputs as for hps_solve, on the device the operator was built on.
 * Returns HPS_EINVAL, with both sizes in the message, if the operator's solve
 * workspace does not fit the array (for example 2D p = 16 trees deeper than
 * 6 levels).  Every call on one GPU shares that GPU's array and leaves its
 * contents behind: calls that overlap on one GPU (different streams or
 * threads) race on it and must be serialized by the caller. */
int hps_solve_noalloc(hps_op_t* op, const double* bdry, const double* src, double* u,
                      int nrhs, void* stream);

/* Mixed-precision solve (precision HPS_FP32_REFINED; operator built with
 * HPS_FLAG_FP32_COPY, 2D).  The stored operators are copied to fp32 at build
 * time (leaf LU and Y, merge D^{-1}, S and B's nonzero blocks); the solution
 * is refined in fp64 on the composite collocation system that HPS eliminates
 * (collocation rows at interior leaf points, boundary bordering, flux balance
 * on shared panels; Section 3): each sweep computes the fp64 residual from
 * the coefficients and applies an fp32 HPS solve to it.  The factorizations
 * themselves are never redone in fp32.  Sets the number of correction sweeps
 * used by later refined solves of `op` (sweeps == 0 only queries; the
 * default is 3: each sweep contracts the error by 1e-5 .. 1e-3 depending on
 * the operator, and two sweeps leave up to 2e-8); returns the previous
 * value, or a negative error code. */
int hps_refine_sweeps(hps_op_t* op, int sweeps);

/* Adjoint (transposed) solve.  The solve is linear in its data,
 * u = G_f f + G_g g; this returns lam_src = G_f^T w and lam_bdry = G_g^T w by
 * running the stored leaf and merge operators of the build transposed, in
 * reverse order (the transposes of the downward pass and of the upward source
 * pass of Section 3; derivative rules for the solver are the future work of
 * Section 6).  No factorization is redone.
 *   w         dev [nrhs][n_leaves][p^dim]   weight, laid out like u
 *   lam_src   dev [nrhs][n_leaves][p^dim]   output; zero at leaf boundary points
 *                                           (the source is not read there)
 *   lam_bdry  dev [nrhs][n_root_bdry]       output, or NULL if not wanted
 * Asynchronous on `stream`, like hps_solve. */
int hps_solve_adjoint(hps_op_t* op, const double* w, double* lam_src,
                      double* lam_bdry, int nrhs, void* stream);

/* Gradient with respect to the coefficient fields.  Only the collocation rows
 * at interior leaf points contain the coefficients (boundary bordering
 * replaces the others, Section 2), so for a scalar J(u) with lam = adjoint of
 * grad_u J:
 *   grad[leaf][t][pt] = - sum_r lam[r][leaf][pt] * (d_t u_r)(pt)   at interior pts,
 *                       0                                           at boundary pts,
 * with d_t the leaf's spectral derivative of term t.
 *   u     dev [nrhs][n_leaves][p^dim]   the solution (from hps_solve)
 *   lam   dev [nrhs][n_leaves][p^dim]   lam_src of hps_solve_adjoint
 *   grad  dev [n_leaves][n_terms][p^dim] output (overwritten)
 * Asynchronous on `stream`. */
int hps_coeff_grad(hps_op_t* op, const double* u, const double* lam, int nrhs,
                   double* grad, void* stream);

/* Interpolation of a leaf-point field at scattered points (host only): the
 * solution on a leaf is its tensor Chebyshev interpolant (Section 2).  For
 * each point x[m] (host [m][dim]) returns the containing leaf leaf[m] (on a
 * shared edge or face, the lowest leaf index) and the barycentric weights
 * w[m][p^dim] with u(x[m]) = sum_k w[m][k] u[leaf[m]][k].  Points outside the
 * domain give HPS_EINVAL. */
int hps_interp_weights(const hps_tree_t* tree, int p, const double* x, long long m,
                       long long* leaf, double* w);

/* Batched solve over several resident operators (continuous-batching
 * serving).  The solves of all items run as one sequence of launches in
 * which every launch covers the same pass stage of every item (the source
 * up-pass of Section 3 aligned at the leaves, the downward pass aligned at
 * the root), so a batch costs a fixed number of launches (5 L_max + 4)
 * whatever the number of operators and right-hand sides.  Each item is one
 * operator with 1..16 right-hand sides given as separate device vectors:
 *   bdry[j]  dev [n_root_bdry]            Dirichlet data of rhs j
 *   src[j]   dev [n_leaves][p^2]           source of rhs j, or NULL for f = 0
 *   u[j]     dev [n_leaves][p^2]           output of rhs j
 * Results equal those of hps_solve on the same data (the arithmetic of every
 * output entry is the same).  2D operators only; an operator may appear at
 * most once per batch, and must not be used by another solve on another
 * stream until this batch has completed (the batch uses the operator's solve
 * workspace).  The batcher owns two pinned host / device descriptor blocks
 * and alternates them: the host packs batch n+1 while the device runs batch
 * n, and waits only when it comes back to a block still in use.  Asynchronous
 * on `stream`. */
typedef struct hps_batcher hps_batcher_t;

typedef struct {
  hps_op_t* op;
  int nrhs;
  const double* bdry[16];
  const double* src[16];
  double* u[16];
} hps_batch_item_t;

int hps_batcher_create(hps_batcher_t** out);
int hps_solve_batch(hps_batcher_t* batcher, const hps_batch_item_t* items, int nitems, void* stream);
void hps_batcher_free(hps_batcher_t* batcher);

/* Per-stage device times (ms) of the last build/solve queued with
 * HPS_FLAG_TIMING: names[i] (static strings) and ms[i], up to cap entries.
 * Synchronizes the op's stream.  Returns the number of entries, or < 0. */
int hps_stage_times(hps_op_t* op, const char** names, double* ms, int cap);

/* Resident device bytes of a built operator. */
size_t hps_op_bytes(const hps_op_t* op);

/* Allocator callback (optional).  When set, every device block of an
 * operator (its stored operators, build and solve workspaces) comes from
 * alloc(bytes, ctx) and goes back through free(ptr, bytes, ctx), so that a
 * framework's caching allocator (PyTorch's, for example) can supply the
 * library's memory and account for it.  alloc returns a device pointer
 * aligned to 256 bytes, or NULL, which the library reports as HPS_ENOMEM
 * (after freeing what the failed call had allocated).  Both NULL restores the
 * library's own pool; exactly one NULL is HPS_EINVAL.  The setting applies to
 * allocations made after the call; every block goes back through the
 * allocator that supplied it, which must stay valid until the operators built
 * with it are freed.  free is called only after the device has finished with
 * the block (hps_free synchronizes the device first).  The small per-(p, leaf
 * size) constant tables are always the library's own. */
typedef void* (*hps_alloc_fn)(size_t bytes, void* ctx);
typedef void (*hps_free_fn)(void* ptr, size_t bytes, void* ctx);
int hps_set_allocator(hps_alloc_fn alloc, hps_free_fn free, void* ctx);

/* Device memory of the library (all operators and their build workspaces,
 * the peak memory the paper reports for 3D trees, Section 4): bytes currently
 * handed out (in_use) and
 * their high-water mark since the last reset (peak); either may be NULL.
 * reset_peak != 0 sets the mark to the current use after reading it.  Freed
 * blocks the library keeps cached for later builds are not counted. */
void hps_mem_stats(size_t* in_use, size_t* peak, int reset_peak);

/* Release the operator and its device memory (after its queued work). */
void hps_free(hps_op_t* op);

/* Message for the last non-OK return on this thread ("" if none). */
const char* hps_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HPS_H_ */
