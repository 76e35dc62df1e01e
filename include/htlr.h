/*
 * htlr.h -- C ABI of the MI355X library for hierarchical Tucker low-rank
 * (HTLR) matrices (Li & Liu, "Hierarchical Tucker Low-Rank Matrices:
 * Construction and Matrix-Vector Multiplication", arXiv 2508.05958).
 *
 * The operator is the Nystrom discretisation of the integral equation
 * a(x) u(x) + int_[0,1]^d k(x,y) u(y) dy = f(x)   (Sec. 1, eq. 1.1), i.e.
 *
 *     f_i = a_i u_i + sum_j K_ij |Omega_j| u_j                 (eq. 1.3 and
 *     K_ij = k(x_i, x_j) (j != i),  K_ii |Omega_i| = int_Omega_i k(x_i,y) dy
 *                                                      (eq. 1.4, Sec. 3.3)
 *
 * on a tensor grid {x_i} in [0,1]^d, compressed into an HTLR matrix
 * (Def. 3.7): a 2^d cluster tree (Def. 2.1, 3.5), a block cluster tree under
 * strong or weak admissibility (Defs. 2.2-2.4, 3.6), Tucker low-rank blocks
 * from tensor Chebyshev interpolation on admissible leaves (eq. 3.4-3.6,
 * Alg. 4.1) and dense blocks on inadmissible leaves (eq. 4.1).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Vectors are in natural grid order: multi-index (i_1,...,i_d), 0-based,
 *   maps to i_1 + n*i_2 + n^2*i_3 (first index fastest, Sec. 2.1).
 * - Several right-hand sides form an N x nrhs column-major array (each
 *   right-hand side contiguous).
 * - Pointers documented as "device" must point to GPU memory of the device
 *   current at the call (for example torch.Tensor.data_ptr()).  Pointers
 *   documented as "host" are read before the call returns.
 * - A "stream" argument is a hipStream_t passed as void*; NULL is the null
 *   stream.  Work enqueued on a stream completes asynchronously; the caller
 *   keeps the device buffers alive until the stream has finished.
 * - Every call returns an htlr_status; nothing crosses the ABI as an
 *   exception.  On failure htlr_last_error() returns a message (thread
 *   local, valid until the next call on the same thread).  A kernel fault
 *   surfaces at the next synchronising call as HTLR_ERR_HIP.
 */
#ifndef HTLR_H
#define HTLR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct htlr_matrix_s* htlr_matrix; /* opaque; owns all its device memory */

typedef enum {
  HTLR_OK = 0,
  HTLR_ERR_INVALID = -1,       /* bad argument (null pointer, size, order of nodes, ...) */
  HTLR_ERR_UNSUPPORTED = -2,   /* valid request the GPU path does not implement */
  HTLR_ERR_OOM = -3,           /* a device or host allocation failed */
  HTLR_ERR_HIP = -4,           /* a HIP runtime call failed */
  HTLR_ERR_NOT_CONVERGED = -5, /* solver stopped at its iteration limit */
  HTLR_ERR_NUMERIC = -6        /* NaN/Inf in an input or a breakdown */
} htlr_status;

/* Kernel functions k(x, y), r = |x - y| (Euclidean).  The paper's Sec. 5 uses
 * the Gaussian and single-layer-potential kernels; the unnormalised forms
 * are used here.  HTLR_K_POLY_TEST is the polynomial
 *   prod_l (1 + A_l (x_l - y_l))^(p-1),   A = (0.50, 0.30, 0.20),
 * of degree p-1 in every coordinate, which Chebyshev interpolation with p
 * points reproduces exactly (Lemma 3.1); it exists for testing. */
typedef enum {
  HTLR_K_INV_R = 0,      /* 1 / r                                   */
  HTLR_K_NEG_LOG = 1,    /* -log r                                  */
  HTLR_K_EXP = 2,        /* exp(-r)                                 */
  HTLR_K_GAUSS = 3,      /* exp(-r^2 / (2 sigma^2)), sigma^2 = d     */
  HTLR_K_POLY_TEST = 100
} htlr_kernel;

/* Arithmetic of a product.  HTLR_FP64: every step in double.  HTLR_FP32:
 * far-field contractions and near field in float.  HTLR_BF16_CORE: as FP32,
 * but the core apply multiplies bfloat16 cores by bfloat16 source tensors on
 * the matrix cores with float accumulation. */
typedef enum { HTLR_FP64 = 0, HTLR_FP32 = 1, HTLR_BF16_CORE = 2 } htlr_precision;

/* Element type of the vectors passed to htlr_matvec. */
typedef enum { HTLR_VEC_F64 = 0, HTLR_VEC_F32 = 1 } htlr_vec_dtype;

typedef enum { HTLR_ADM_STRONG = 0, HTLR_ADM_WEAK = 1 } htlr_admissibility;

typedef struct {
  /* eta^2 of strong admissibility, max(diam) <= eta * dist (Def. 2.3),
   * tested as max(diam^2) <= eta2 * dist^2; equality is admissible.
   * <= 0 selects 1.0 ("dist >= box diameter"). */
  double eta2;
  int admissibility;     /* htlr_admissibility (Def. 2.3 or Def. 2.2)             */
  int gl_order;          /* Gauss-Legendre points per dimension for the diagonal
                            integrals of eq. 1.4; 0 selects 16 (d=2) or 8 (d=3)   */
  const double* a;       /* host, N samples a(x_i) in natural order; NULL: a = 0   */
  int precisions;        /* bit mask of (1 << htlr_precision) the matrix will be
                            applied in; selects which core copies are kept;
                            0 selects all three                                    */
  int orthonormalize;    /* Alg. 4.1's QR step (uniform grids; otherwise
                            HTLR_ERR_UNSUPPORTED):
                            0: interpolation form (Lagrange factors U, V and
                               cores G = k(xi_t, eta_s), eq. 3.4);
                            1: thin QR of the factors, U = W R, V = Q T, stored
                               as W, Q with G <- G x_1 R ... x_{d+1} T ...; the
                               same operator up to rounding;
                            2: QR with column pivoting truncated at rank_tol
                               (Sec. 2.1): each level keeps its own rank r_l,
                               the number of pivots kept for its factor, and
                               its cores shrink to r_l^d x r_l^d (levels whose
                               boxes are at least p points wide keep p unless
                               rank_tol is loose)                              */
  double rank_tol;       /* orthonormalize = 2: keep pivots with
                            |R_kk| > rank_tol |R_00|; <= 0 selects 1e-13       */
  const double* edges;   /* host, d*(n+1) cell edges per dimension, dimension-
                            major (edges[l*(n+1) + k] = e_{l;k}), or NULL.  The
                            cells Omega_i of eq. 1.3 are their products: the
                            quadrature weights |Omega_i|, the diagonal integrals
                            of eq. 1.4 and the boxes Omega_tau of the cluster
                            tree (Sec. 2.2, Def. 3.5) follow them.  Each
                            dimension's edges increase strictly within [0, 1]
                            and node k lies in [e_{l;k}, e_{l;k+1}], otherwise
                            HTLR_ERR_INVALID.  NULL: the 1D Voronoi cells
                            (midpoints between neighbouring nodes, 0 and 1 at
                            the ends).  The grid takes the uniform path only if
                            nodes and edges both equal the uniform ones.  Copied
                            at build; htlr_build_quasi applies them to the
                            quasi-uniform cells (S and T)                     */
} htlr_build_opts;

/* Builds the HTLR matrix of the Nystrom operator above (Alg. 4.1).
 *
 * points : host, d*n doubles, or NULL.  Node coordinates per dimension,
 *          dimension-major: points[l*n + k] = x_{l;k}, strictly increasing
 *          inside (0, 1).  The grid is their tensor product; cells Omega_i
 *          are the products of opts->edges or, by default, of the 1D Voronoi
 *          cells (midpoints between neighbouring nodes, 0 and 1 at the ends;
 *          Sec. 2.2).  NULL means
 *          the uniform cell-centred grid x_{l;k} = (k + 1/2)/n (Example 2.2).
 *          A grid whose nodes equal the uniform ones to 1e-14 is treated as
 *          uniform (translation-invariant cores, exact integer geometry).
 * kernel : htlr_kernel.
 * d      : 2 or 3.
 * n      : points per dimension (N = n^d).
 * p      : Chebyshev points per dimension (Tucker rank, Sec. 3.1), 1..12.
 * leaf   : leaf threshold N_0 = leaf^d; a cluster is a leaf when it has at
 *          most N_0 points (Sec. 2.2).  n must halve exactly down to the
 *          leaf level, otherwise HTLR_ERR_UNSUPPORTED.
 * opts   : host, may be NULL (all defaults).
 * out    : host; receives the handle.  The handle keeps copies of points and
 *          a; the caller may free them on return.
 *
 * Runs synchronously on the null stream of the current device. */
htlr_status htlr_build(const double* points, htlr_kernel kernel, int d, int n, int p,
                       int leaf, const htlr_build_opts* opts, htlr_matrix* out);

/* Builds the same operator on a quasi-uniform tensor grid by the transfer
 * scheme of Sec. 3.3 (eq. 3.9): A ~ diag(a) + T Ahat S.
 *
 * Ahat is the HTLR matrix of the same kernel on the uniform cell-centred grid
 * of m^d cells, with a = 0 (built as htlr_build(NULL, kernel, d, m, p, leaf);
 * its diagonal integrals are those of the uniform cells).  S (m^d x n^d) and
 * T (n^d x m^d) move a vector between the grids, reading it as piecewise
 * constant on its cells:
 *     S[t,i] = |Omega_t^uni cap Omega_i| / |Omega_t^uni|,
 *     T[i,t] = |Omega_i cap Omega_t^uni| / |Omega_i|.
 * On a tensor grid both are Kronecker products of 1D cell-overlap matrices;
 * their rows sum to 1 and both conserve sum_i |Omega_i| u_i.  The term
 * a_i u_i is applied on the quasi-uniform grid itself.
 *
 * points : host, d*n doubles as in htlr_build (cells are the 1D Voronoi
 *          cells); NULL means the uniform grid of n cells.
 * m      : uniform cells per dimension (m = rho n with oversampling rho);
 *          m must halve exactly down to Ahat's leaf level, otherwise
 *          HTLR_ERR_UNSUPPORTED.
 * opts   : as in htlr_build; opts->a holds a(x_i) at the n^d points.
 * out    : host; receives the handle.
 *
 * The handle is used like any other: htlr_matvec and htlr_solve (vectors of
 * n^d rows), htlr_workspace_bytes, htlr_autotune (tunes Ahat's products),
 * htlr_profile_* (adds the steps "quasi_s" and "quasi_t"), htlr_info
 * (structure of Ahat with d, n of the quasi-uniform grid and uniform_m = m)
 * and htlr_free.  Runs synchronously on the null stream of the current
 * device; failures leave *out NULL. */
htlr_status htlr_build_quasi(const double* points, htlr_kernel kernel, int d, int n, int m, int p,
                             int leaf, const htlr_build_opts* opts, htlr_matrix* out);

/* Device bytes htlr_build would hold for the same arguments (cores, factors,
 * geometry, near-field tables, block lists), without allocating; used for
 * admission by memory footprint.  Work buffers of products and solves are
 * reported by htlr_workspace_bytes. */
htlr_status htlr_footprint(const double* points, htlr_kernel kernel, int d, int n, int p,
                           int leaf, const htlr_build_opts* opts, size_t* bytes);

/* Device bytes of the work buffers a product with nrhs right-hand sides in
 * precision prec needs (allocated inside the handle on first use).  Not
 * included: on uniform 3D grids with 8^3-point leaves and radial kernels, a
 * product with nrhs >= 2 on a handle whose workspace is not reserved runs the
 * near field on the matrix-core core apply.  On first use it builds one
 * 512 x 512 block per near offset in FP64 and FP32 (3 MB per offset; 117
 * offsets at 16^3 leaves) and leaf-major copies of u and of the near
 * result (2 N nrhs values) plus their K-split partial sums, and keeps them
 * with the handle.  Reserved workspaces (the server) and
 * htlr_matvec_noalloc use the table kernel instead. */
htlr_status htlr_workspace_bytes(htlr_matrix A, int nrhs, htlr_precision prec, size_t* bytes);

/* f = A u (overwrites f) by the HTLR product (Alg. 4.2, eq. 4.3).
 *
 * u, f   : device, N x nrhs column-major, element type vec_dtype; must not
 *          overlap.  HTLR_FP64 needs HTLR_VEC_F64; HTLR_FP32 and
 *          HTLR_BF16_CORE need HTLR_VEC_F32.
 * nrhs   : 1..64.
 * stream : hipStream_t or NULL.
 *
 * Uses work buffers owned by the handle: products on one handle must be
 * issued on one stream at a time. */
htlr_status htlr_matvec(htlr_matrix A, const void* u, void* f, int nrhs, htlr_precision prec,
                        htlr_vec_dtype vec_dtype, void* stream);

/* For callers that cannot allocate device memory (code under hipGraph
 * capture, serving loops or harnesses that forbid hipMalloc): f = A u as
 * htlr_matvec computes it, with the product's work buffers in a fixed array
 * of the library's own device memory of HTLR_NOALLOC_SCRATCH_BYTES, which
 * each device the library runs on holds until the process ends.  Calls no
 * hipMalloc or hipFree and no allocating library routine.
 *
 * Arguments, layouts and errors as htlr_matvec.  The product takes the
 * kernels that need no lazily built work lists: the plain core apply on
 * VALU instead of the matrix-core kernels, near-field kernels without K-split
 * partial sums, every launch on the caller's stream, no tuner choices.  So
 * its result equals htlr_matvec's to rounding, not bit for bit, and it is
 * slower on large problems.
 * HTLR_ERR_INVALID when the work buffers of this (matrix, nrhs) exceed the
 * fixed size (the message states both sizes; htlr_matvec still serves
 * them), HTLR_ERR_UNSUPPORTED for htlr_build_quasi handles.
 * Every call on one device shares that device's array: calls that overlap
 * on one device (on different streams, or from several threads) race and
 * must be serialised by the caller. */
#define HTLR_NOALLOC_SCRATCH_BYTES (64u << 20)
htlr_status htlr_matvec_noalloc(htlr_matrix A, const void* u, void* f, int nrhs, htlr_precision prec,
                                htlr_vec_dtype vec_dtype, void* stream);

/* Rows of the uncompressed Nystrom product (eq. 1.3-1.4):
 *     out_i = (a_i + D_i) u_i + sum_{j != i} k(x_i, x_j) |Omega_j| u_j,
 * evaluated directly over all N source points in FP64, for measuring the
 * HTLR approximation error as Sec. 5 does (e_apply;rand, the relative
 * 2-norm error against the exact A u on randomly chosen rows).
 *
 * u      : device, N x nrhs column-major doubles.
 * rows   : device, nrows int64 row indices in natural order; an index
 *          outside [0, N) gives NaN in its output rows.
 * out    : device, nrows x nrhs column-major doubles (out[q + r*nrows] is
 *          row rows[q] of right-hand side r).
 * nrhs   : 1..8.
 * Cost O(nrows N); deterministic.  Transfer-form handles return
 * HTLR_ERR_UNSUPPORTED. */
htlr_status htlr_exact_rows(htlr_matrix A, const double* u, const int64_t* rows, int nrows, double* out, int nrhs,
                            void* stream);

/* Solver options (the paper has no solver: solving A u = f is the
 * "backward evaluation" of Sec. 1).  Restarted GMRES(restart) with x0 = 0 and
 * classical Gram-Schmidt with reorthogonalisation in double, wrapped in
 * iterative refinement: the residual r = f - A x is formed with the FP64
 * product, the correction solves A d = r with products in inner_prec. */
typedef struct {
  double tol;          /* stop when ||f - A x||_2 / ||f||_2 <= tol (FP64 residual); <=0: 1e-10 */
  int restart;         /* Krylov dimension per cycle; <=0: 30 */
  int max_outer;       /* refinement steps; <=0: 20 */
  int max_inner;       /* inner iterations per refinement step; <=0: 300 */
  int inner_prec;      /* htlr_precision of the inner products */
  double inner_tol;    /* relative residual target of an inner solve; <=0: 1e-6 (FP32), 1e-2 (BF16), tol (FP64) */
} htlr_solve_opts;

typedef struct {
  int outer_iters;      /* refinement steps taken */
  int inner_iters;      /* total inner GMRES iterations */
  int matvecs_fp64;     /* FP64 products used */
  int matvecs_inner;    /* inner-precision products used */
  double rel_residual;  /* final ||f - A x|| / ||f|| with the FP64 product */
} htlr_solve_info;

/* Solves A u = f.  f, u: device, N doubles (nrhs must be 1).  On
 * HTLR_ERR_NOT_CONVERGED, u holds the best iterate and info its residual.
 * f = 0 returns u = 0.  NaN/Inf in f returns HTLR_ERR_NUMERIC.  Allocates
 * its Krylov basis (restart+1 vectors of N doubles) per call; synchronises
 * the stream for the scalar Givens updates. */
htlr_status htlr_solve(htlr_matrix A, const double* f, double* u, int nrhs,
                       const htlr_solve_opts* opts, htlr_solve_info* info, void* stream);

/* Structure statistics of a built matrix. */
typedef struct {
  int d, n, p, leaf_side, levels;     /* levels = depth L of the cluster tree        */
  int uniform;                        /* 1: translation-invariant (uniform) grid       */
  int64_t adm_pairs[16];              /* admissible leaves per level 0..15              */
  int64_t unique_cores[16];           /* stored cores per level (uniform grids)         */
  int64_t near_pairs;                 /* inadmissible leaves                            */
  size_t device_bytes;                /* what htlr_footprint reports                    */
  double diag0;                       /* D_0 = K_00 |Omega_0| (uniform: every D_i)       */
  int uniform_m;                      /* htlr_build_quasi handles: m; otherwise 0        */
  int rank;                           /* largest level rank of the stored factors and
                                         cores (p unless the QR step truncated it)        */
  int level_rank[16];                 /* Tucker rank of each level 0..15 with admissible
                                         leaves (its cores are level_rank^d squared);
                                         0 for levels without admissible leaves          */
} htlr_info_t;

htlr_status htlr_info(htlr_matrix A, htlr_info_t* info);

/* Kernel timing of products, for measurement: while enabled, every launch of
 * htlr_matvec on this handle is bracketed by hipEvents recorded on the
 * launch stream.  htlr_profile_read synchronises those events and returns,
 * per step name ("near", "up_l4", "core_l4", "down_l4", ...), the number of
 * launches and their summed duration in milliseconds since the last reset.
 * While enabled, a product issues all its launches on the caller's stream
 * in order (the levels do not run concurrently), so that each duration is
 * that launch's alone; results are bitwise the same either way.
 * Enabling or disabling clears the record. */
typedef struct {
  char name[32];
  int launches;
  double total_ms;
} htlr_profile_entry;

htlr_status htlr_profile_enable(htlr_matrix A, int enable);
htlr_status htlr_profile_read(htlr_matrix A, htlr_profile_entry* out, int cap, int* count);

/* Autotuner: times variants of the product's kernels for products with
 * nrhs right-hand sides in precision prec on this matrix (the core apply's
 * matrix-core tile shape, its class-tile or offset-major mode and the split of
 * its reduction over workgroups; the near-field kernel, its K splits, tiles
 * per wave and waves per leaf; concurrent or serial level launches), and keeps
 * the fastest for later products of that shape.  The choices change the
 * order of summation, so results agree to rounding, not bit for bit; a given
 * choice is deterministic.  With the environment variable HTLR_TUNE_CACHE naming a file, results
 * are read from and appended to it, keyed by (d, n, p, leaf, kernel, grid,
 * nrhs, prec).  Allocates scratch vectors; synchronises the device. */
typedef struct {
  int ks_target;        /* workgroups the core apply aims for when splitting its reduction
                           (0: automatic, at least 2048 and 4 per unsplit work item) */
  int near_kind;        /* 0: VALU row kernel, 1: matrix-core kernel */
  int near_waves;       /* waves per leaf of the VALU row kernel */
  int candidates;       /* variants timed (0: taken from the cache) */
  double ms_default;    /* product time with the built-in choice */
  double ms_best;       /* product time with the chosen variant */
} htlr_tune_result;

htlr_status htlr_autotune(htlr_matrix A, int nrhs, htlr_precision prec, htlr_tune_result* out);

/* Releases the handle and all its device memory (synchronises the device). */
void htlr_free(htlr_matrix A);

const char* htlr_last_error(void);

/* Host-only planner, for inspection and tests; touches no GPU.
 * Counts the leaves of the block cluster tree (Def. 2.4) for the given grid
 * (points and cell edges as in htlr_build and htlr_build_opts.edges, each
 * may be NULL), per level. */
htlr_status htlr_plan_counts(const double* points, const double* edges, int d, int n, int leaf, double eta2,
                             int admissibility, int* levels, int64_t* adm_per_level /*[16]*/,
                             int64_t* near_pairs);

/* Host-only planner: the admissible (level >= 0) or inadmissible (level < 0)
 * leaves of the block cluster tree as pairs of box indices at that level
 * (box multi-index b, linear index b_1 + B b_2 + B^2 b_3, B boxes per
 * dimension).  Writes up to cap pairs into tau[] and sigma[] (host), sorted
 * by (tau, sigma), and the total into *count. */
htlr_status htlr_plan_pairs(const double* points, const double* edges, int d, int n, int leaf, double eta2,
                            int admissibility, int level, int32_t* tau, int32_t* sigma,
                            int64_t cap, int64_t* count);

/* ------------------------------------------------------------------------
 * Request server: continuous batching of solve requests on one GPU.
 * (Not in the paper; a serving layer over htlr_build / htlr_solve.)
 *
 * Requests (A u = f for possibly different grids, kernels and ranks) are
 * queued by htlr_server_submit and advanced by htlr_server_step, one
 * scheduling tick per call:
 *  - admission: queued requests enter, first come first served, while the
 *    device bytes of resident structures plus request state stay within
 *    memory_budget; idle structures are evicted least recently used first;
 *  - structures (the HTLR matrices) stay resident across requests, keyed by
 *    (points, kernel, d, n, p, leaf, eta2, admissibility, a);
 *  - work is scheduled per unit (a group of structures, below, or one
 *    structure), each idle or with one step in flight: a tick issues, for
 *    every idle unit, one step of GMRES with FP64 iterative refinement for
 *    each of its active requests (the method of htlr_solve, with the
 *    refinement residual taken after every GMRES cycle), then waits until at
 *    least one unit in flight has finished its step and advances that unit's
 *    requests; so small structures take many steps while a large one
 *    computes one product.  The products of all requests of a structure in
 *    one step are fused into a single multi-right-hand-side product,
 *    optionally replayed from a captured hipGraph;
 *  - structures that share their factors (the uniform grid of the same d,
 *    n, p, leaf, eta2 and admissibility; e.g. different kernels) form a
 *    group: their fused products of one tick run as one grouped product, in
 *    which the up contraction and the down expansion of each level are one
 *    launch over the columns of every member (Alg. 4.2's factor steps do not
 *    depend on the kernel), and the core applies and near fields run per
 *    structure;
 *  - structures (or groups) run on separate streams, so their work overlaps.
 * A request's answer does not depend on which other requests share its
 * ticks beyond rounding (each column of a fused product is computed by the
 * same arithmetic as alone).
 * A server is used from one host thread at a time.
 * ------------------------------------------------------------------------ */
typedef struct htlr_server_s* htlr_server;

typedef struct {
  size_t memory_budget; /* device bytes for structures + request state; 0: 90% of free memory */
  int max_active;       /* requests in flight; <= 0: 64 */
  int max_batch;        /* requests of one structure fused per product (1..64); <= 0: 16 */
  int restart;          /* GMRES cycle length; <= 0: 30 */
  int inner_prec;       /* htlr_precision of the inner products; with HTLR_BF16_CORE,
                           structures on given points (tensor grids, which have no
                           bfloat16 cores) take FP32 inner products */
  int use_graphs;       /* 1: replay fused products from captured hipGraphs */
  int autotune;         /* 1: time kernel variants per (structure, batch width, precision) */
  int no_group_fusion;  /* 1: never fuse the products of different structures */
  double inner_tol;     /* relative residual an inner GMRES cycle aims at; <= 0: 1e-6 (FP32),
                           1e-4 (BF16-core), 1e-12 (FP64).  A refinement step stops its
                           cycle there (or at the request's own tolerance, if looser), or
                           after restart iterations */
} htlr_server_opts;

typedef struct {
  const double* points; /* host, as in htlr_build (NULL: uniform grid) */
  int kernel, d, n, p, leaf;
  double eta2;          /* <= 0: 1 */
  int admissibility;
  const double* a;      /* host, N values, or NULL (a = 0); copied at submit */
  const double* f;      /* host, N values; copied at submit */
  double tol;           /* target ||f - A u|| / ||f|| (FP64 product); <= 0: 1e-8 */
  int max_outer;        /* refinement cycles; <= 0: 50 */
} htlr_request;

typedef struct {
  int state;            /* 0 queued, 1 active, 2 done, 3 failed */
  int status;           /* htlr_status of a finished request */
  int outer_iters, inner_iters;
  double rel_residual;
  double t_submit, t_admit, t_done; /* seconds on the server clock */
} htlr_request_info;

typedef struct {
  int64_t ticks, fused_products, graph_launches, structures_built, evictions;
  int resident_structures, active, queued;
  size_t resident_bytes;
  int64_t group_products;     /* fused products that spanned several structures */
  int64_t grouped_launches;   /* up / down launches shared by several structures */
} htlr_server_stats_t;

htlr_status htlr_server_create(const htlr_server_opts* opts, htlr_server* out);
/* Copies the request; *id identifies it in htlr_server_result. */
htlr_status htlr_server_submit(htlr_server S, const htlr_request* req, int64_t* id);
/* One scheduling tick: admission, one fused step issued for every idle unit,
 * a wait until at least one unit's step has finished, the host updates of
 * that unit's requests, retirement.  Returns the number of active and queued
 * requests after the tick. */
htlr_status htlr_server_step(htlr_server S, int* active, int* queued);
/* For a finished request: copies u (host, N doubles, may be NULL) and its
 * info, then forgets the request.  For an unfinished one: fills info only
 * and returns HTLR_ERR_INVALID with state 0 or 1. */
htlr_status htlr_server_result(htlr_server S, int64_t id, double* u, htlr_request_info* info);
htlr_status htlr_server_stats(htlr_server S, htlr_server_stats_t* out);
double htlr_server_clock(htlr_server S);
void htlr_server_destroy(htlr_server S);

#ifdef __cplusplus
}
#endif

#endif /* HTLR_H */
