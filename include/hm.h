/*
 * hm.h - C ABI of the gfx950 hierarchical-matrix library with accumulated
 * updates (Boerm, "Hierarchical matrix arithmetic with accumulated updates").
 *
 * Conventions
 *  - Every function returns an hm_status; nothing throws across the ABI.
 *    hm_last_error() returns a thread-local message for the last failure.
 *  - All arithmetic runs on the GPU in hand-written HIP kernels, stream-ordered
 *    on the context's stream.  Calls that return results to the host
 *    (hm_lu, hm_addmul, hm_plan_run, hm_to_dense, ...) synchronise the stream.
 *  - Matrices are column-major.  Row and column indices of an H-matrix are in
 *    cluster order: position p holds the original index perm[p] (hm_perm).
 *  - Handles are owned by the caller and released with the matching *_free /
 *    *_destroy function.  Input arrays are borrowed and copied.
 */
#ifndef HM_H
#define HM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HM_OK = 0,
  HM_ERR_ARG = 1,      /* invalid argument (sizes, NULL handles, mismatched structure) */
  HM_ERR_ALLOC = 2,    /* device or host allocation failed */
  HM_ERR_HIP = 3,      /* a HIP runtime call failed */
  HM_ERR_SINGULAR = 4, /* zero pivot in a leaf LU */
  HM_ERR_NUMERIC = 5,  /* NaN/Inf, rank capacity or workspace exceeded (see message) */
  HM_ERR_STATE = 6     /* unsupported structure (e.g. H-LU needs a binary cluster tree) */
} hm_status;

/* How products reach the matrix being updated:
 *   HM_STANDARD           every low-rank product is applied at once by
 *                         truncated additions to the leaves below its target
 *                         (Fig. rkupdate, Sect. 4);
 *   HM_ACCUMULATED        products are gathered in accumulators and pushed
 *                         down the block tree (Figs. addproduct, split, flush);
 *   HM_ACCUMULATED_FUSED  as HM_ACCUMULATED, but in a split the low-rank
 *                         products that reach one son accumulator are added in
 *                         groups of three, each group truncated together with
 *                         the accumulator in one truncated addition of the
 *                         stacked sum (not in the paper: the multi-term form of
 *                         Fig. rkadd that the H^2-style motivation of the
 *                         accumulators suggests; fewer, larger truncations). */
typedef enum { HM_STANDARD = 0, HM_ACCUMULATED = 1, HM_ACCUMULATED_FUSED = 2 } hm_update_mode;

/* Arithmetic of the contractions of stacked factors and of the H-matrix by
 * thin-dense products (storage is FP64 in every mode; the core SVD, rank rule,
 * leaf LU and triangular solves are always FP64):
 *   HM_FP64    everything in FP64;
 *   HM_FP32    operands rounded to FP32, FP32 products and sums;
 *   HM_BF16X3  operands rounded to FP32 and split into three BF16 pieces, six
 *              cross products on the matrix cores with FP32 accumulation. */
typedef enum { HM_FP64 = 0, HM_FP32 = 1, HM_BF16X3 = 2 } hm_precision;

/* Order of execution of a plan's work items (chosen when the plan is made):
 *   HM_SCHEDULE_WAVES     dependency waves: every launch of a wave waits for
 *                         all launches of the wave before (the earliest wave
 *                         of every item; the late placement of the items that
 *                         only write temporaries when those exceed the
 *                         temporary budget); plans can be replayed from a
 *                         captured hipGraph;
 *   HM_SCHEDULE_DATAFLOW  every item waits only for the items it conflicts
 *                         with: launches on four streams ordered by estimated
 *                         earliest start, with event dependencies; more
 *                         temporary memory, no graph replay.  A plan whose
 *                         temporaries would exceed the budget falls back to
 *                         waves. */
typedef enum { HM_SCHEDULE_WAVES = 0, HM_SCHEDULE_DATAFLOW = 1 } hm_schedule;

typedef struct hm_ctx hm_ctx;       /* stream, device status words */
typedef struct hm_matrix hm_matrix; /* device-resident H-matrix (structure on the host) */
typedef struct hm_plan hm_plan;     /* a recorded and scheduled multiplication or H-LU */
typedef struct hm_mlp hm_mlp;       /* rank-predictor network (see the end of this header) */

/* Per-run information. */
typedef struct {
  double plan_seconds;      /* host recording + scheduling + upload */
  double run_seconds;       /* device time of the run (HIP events around the launches) */
  int64_t truncations;      /* truncations executed on the device */
  int64_t planned_truncations; /* truncation work items recorded (upper bound) */
  int64_t items[5];         /* work items per kind: GEMM, TRUNC, LU, TRSM, COPY */
  int64_t waves;            /* dependency waves */
  int64_t launches;         /* kernel launches per run */
  int64_t temp_bytes;       /* device memory of temporaries */
  int64_t workspace_bytes;  /* truncation workspace pool */
  int64_t counts[9];        /* trunc_update, trunc_accum, trunc_merge, dense_updates,
                               addproduct, pending, products, leaf_lu, merges (planned) */
  int32_t status_bits;      /* device status word of the run */
  int32_t schedule;         /* hm_schedule the plan was made with */
  int64_t trunc_bytes;      /* algorithmic bytes of the executed truncations, 8 (m+n)(l+k) */
  double op_seconds[5];     /* device time per work-item kind (only with HM_PROFILE_OPS=1) */
  double plan_phase_seconds[3]; /* recording, scheduling, upload */
  int64_t small_trunc_bytes;    /* the part of trunc_bytes done by the small-block kernel (m, n <= 64) */
  double small_trunc_seconds;   /* device time of the small-block truncation launches (HM_PROFILE_OPS=1) */
  int64_t small_trunc_launches; /* truncation launches per run: small-block kernel */
  int64_t general_trunc_launches; /* truncation launches per run: register-resident + general kernels */
  int64_t predicted;            /* truncations done by the rank predictor's range finder */
  int64_t predicted_fallback;   /* predicted truncations that failed the check and ran the exact path */
  int32_t graph_replay;         /* 1 when the run was replayed from a hipGraph (hm_plan_use_graph) */
  int32_t pad;
} hm_run_info;

/* Library version string. */
const char* hm_version(void);

/* Thread-local message describing the last error. */
const char* hm_last_error(void);

/* Create a context on the given hipStream_t (NULL = default stream) of the
 * current device.  Device memory comes from hipMalloc / hipFree. */
hm_status hm_ctx_create(void* hip_stream, hm_ctx** out);
/* Device allocator of a context (not in the paper): alloc(bytes, user) returns
 * device memory of at least `bytes` bytes usable on the context's stream (NULL
 * when it cannot), free(ptr, user) releases it.  Every device allocation of
 * the library made for this context -- matrices, plans, workspaces, networks
 * -- goes through them; objects keep the allocator and free through it even
 * after the context is destroyed, so `user` must outlive them.  The library
 * frees only memory whose last use it has synchronised. */
typedef void* (*hm_alloc_fn)(size_t bytes, void* user);
typedef void (*hm_free_fn)(void* ptr, void* user);
/* hm_ctx_create with the caller's allocator (alloc and free both set, or both
 * NULL for hipMalloc / hipFree; HM_ERR_ARG otherwise). */
hm_status hm_ctx_create_with_allocator(void* hip_stream, hm_alloc_fn alloc, hm_free_fn free_fn, void* user,
                                       hm_ctx** out);
void hm_ctx_destroy(hm_ctx* ctx);
/* Schedule (hm_schedule) of the plans made on ctx from now on; the default is
 * HM_SCHEDULE_DATAFLOW.  The environment variable HM_SCHEDULE (waves, late or
 * dataflow), when set, takes precedence.  HM_ERR_ARG for another value. */
hm_status hm_set_schedule(hm_ctx* ctx, int32_t schedule);

/* Host-only check of a schedule (no device, nothing allocated on one): records
 * the H-LU (mode as for hm_lu) of an H-matrix on a side^dim grid of points
 * (leaf_size, eta, kmax as for hm_build_csr), schedules it with `schedule`
 * (the environment's HM_SCHEDULE takes precedence) and checks the result
 * against the run rules alone: stream order, event waits and epoch joins for
 * the dataflow schedule, wave order for waves.  out[8]: launches; pairs of
 * conflicting operations; of them not ordered; pairs of temporaries sharing
 * memory; of them not ordered; waits on a launch that records no event; items
 * placed in no launch or in two; 1 if the dataflow schedule was used.  A
 * correct schedule has out[2] = out[4] = out[5] = out[6] = 0.  At most 2^22
 * points. */
hm_status hm_schedule_check(int32_t dim, int32_t side, int32_t leaf_size, double eta, int32_t kmax, int32_t mode,
                            int32_t schedule, int64_t* out);

/*
 * Build an H-matrix for n points x (n x dim, row-major, dim 1..3) from a sparse
 * matrix in CSR form (rowptr[n+1], colind, vals; original index order).
 * Structure (Defs. cluster tree and block tree, Sect. 2): geometric bisection
 * with clusters of at most leaf_size points; a block (t, s) is admissible when
 * max(diam t, diam s) <= eta dist(t, s) with dist > 0 (tight bounding boxes).
 * Inadmissible leaves are dense; admissible leaves are low-rank with capacity
 * min(#t, #s, kmax) columns.  An admissible leaf that holds CSR entries is
 * stored exactly as A = its nonzero columns, B = unit vectors.
 */
hm_status hm_build_csr(hm_ctx* ctx, int32_t dim, int64_t n, const double* x, const int64_t* rowptr,
                       const int32_t* colind, const double* vals, int32_t leaf_size, double eta, int32_t kmax,
                       hm_matrix** out);

/*
 * Source of the entries of an H-matrix built by hm_build.
 *   HM_SRC_CSR             a sparse matrix in CSR form (rowptr[n+1] int64,
 *                          colind int32, vals; original index order), stored
 *                          as hm_build_csr stores it;
 *   HM_SRC_STENCIL_5PT /   the (2 dim + 1)-point finite-difference Laplacian
 *   HM_SRC_STENCIL_7PT     of the points, which must lie on an integer lattice:
 *                          2 dim on the diagonal, -1 between points at
 *                          distance 1 (points absent from the lattice are a
 *                          Dirichlet boundary, eliminated); 5PT needs dim 2,
 *                          7PT dim 3.  Admissible blocks of such matrices are
 *                          zero (local rank zero, Sect. 3);
 *   HM_SRC_KERNEL_INVDIST  the kernel 1/|x_i - x_j|, with `diag` on the
 *                          diagonal and with two distinct points at the same
 *                          place an error (HM_ERR_ARG).  Inadmissible leaves
 *                          hold the kernel itself; every admissible leaf holds
 *                          the best rank-k approximation of its dense block
 *                          (Eckart-Young, Sect. 3) with the smallest k whose
 *                          discarded tail satisfies
 *                          sum_{i>k} s_i^2 <= eps^2 sum_i s_i^2 (options->eps),
 *                          stored as A = U_k, B = V_k S_k.  The GPU compresses
 *                          each block by a tree of truncations (Fig. rkadd) of
 *                          its 64-column slices at a relative tolerance of
 *                          1e-12 before the final truncation at eps, so its
 *                          singular values are those of the dense block up to
 *                          about 1e-12 |block|_F: the rank is the exact rule's
 *                          wherever the rule's decision is not that close to a
 *                          tie.
 *   HM_SRC_BEM_SINGLE /    the boundary-element matrices of Sect. 7: Galerkin
 *   HM_SRC_BEM_DOUBLE      with piecewise constants on the flat triangles
 *                          `tri` (dim 3; coords are the points the clusters
 *                          are built from, normally the centroids):
 *                          single layer V_ij = int_Ti int_Tj 1/(4 pi |x-y|),
 *                          or half the mass matrix plus the double layer
 *                          K_ij = |T_i|/2 delta_ij + int_Ti int_Tj
 *                          <y - x, n_y>/(4 pi |x - y|^3) with n_y the normal
 *                          (v1 - v0) x (v2 - v0) normalised; the integrals by
 *                          the 7-point rule of degree 5 on both triangles, the
 *                          single layer's diagonal by that rule outside and
 *                          the closed-form integral of 1/|x - y| over the
 *                          triangle inside.  Admissible blocks as for
 *                          HM_SRC_KERNEL_INVDIST.  A triangle of zero area is
 *                          an error (HM_ERR_ARG).
 * Pointers are host arrays, borrowed and copied.
 */
typedef enum {
  HM_SRC_CSR = 0,
  HM_SRC_STENCIL_5PT = 1,
  HM_SRC_STENCIL_7PT = 2,
  HM_SRC_KERNEL_INVDIST = 3,
  HM_SRC_BEM_SINGLE = 4,
  HM_SRC_BEM_DOUBLE = 5
} hm_source_kind;
typedef struct {
  int32_t kind; /* hm_source_kind */
  int32_t pad;
  const int64_t* rowptr; /* HM_SRC_CSR */
  const int32_t* colind;
  const double* vals;
  double diag;        /* HM_SRC_KERNEL_INVDIST: value of the diagonal entries */
  const double* tri;  /* HM_SRC_BEM_*: n x 9, the three vertices of each flat triangle */
} hm_source;

/*
 * Options of hm_build, hm_lu_opt and hm_addmul_opt (hm_options_init sets the
 * defaults given here).
 *   eps          relative Frobenius tolerance of every truncated addition
 *                (Fig. rkadd, the rank rule of its "choose new rank" step);
 *                for hm_build, the compression tolerance of admissible
 *                kernel blocks (default 1e-6);
 *   eta          admissibility max(diam t, diam s) <= eta dist(t, s) (Sect. 2,
 *                default 2);
 *   leaf_size    largest leaf cluster (geometric bisection, default 64);
 *   kmax         rank capacity of admissible leaves (default 64);
 *   mode         HM_STANDARD or HM_ACCUMULATED (default HM_ACCUMULATED);
 *   precision    hm_precision of the products (default HM_FP64);
 *   schedule     hm_schedule of the plan, or -1 for the context's (default -1);
 *   use_graph    replay the plan from a hipGraph (wave plans only, default 0);
 *   rank_override  NULL, or rank_override_count ranks, one per truncation work
 *                item of the plan in recording order (the order of
 *                hm_plan_trunc_log): an entry >= 0 replaces the rank rule's
 *                choice of that item (clamped to the number of singular
 *                values the item has and to its capacity), -1 keeps the rule.
 *                A test hook: with the ranks of one run it makes another run
 *                (another precision, another schedule) take the same rank
 *                decisions, so that their floating-point results can be
 *                compared apart from them.
 */
typedef struct {
  double eps;
  double eta;
  int32_t leaf_size;
  int32_t kmax;
  int32_t mode;
  int32_t precision;
  int32_t schedule;
  int32_t use_graph;
  const int32_t* rank_override;
  int64_t rank_override_count;
} hm_options;
void hm_options_init(hm_options* opt);

/*
 * Build an H-matrix for n points (coords: host, n x dim row-major, dim 1..3)
 * with entries from `src`: cluster tree by geometric bisection with clusters
 * of at most opt->leaf_size points (split at the middle of the longest side
 * of the bounding box), block tree with opt->eta-admissibility (Defs. cluster
 * tree and block tree, Sect. 2); inadmissible leaves dense, admissible leaves
 * low-rank with capacity min(#t, #s, opt->kmax).  opt may be NULL (defaults).
 * Kernel matrices are assembled and compressed on the GPU.  HM_ERR_ARG for
 * invalid arguments, HM_ERR_NUMERIC when an admissible block needs a rank
 * above its capacity.
 */
hm_status hm_build(hm_ctx* ctx, int32_t dim, int64_t n, const double* coords, const hm_source* src,
                   const hm_options* opt, hm_matrix** out);

/* Deep copy (same structure, same values). */
hm_status hm_clone(hm_ctx* ctx, const hm_matrix* src, hm_matrix** out);
/* Checkpoint of an H-matrix: its cluster tree, block tree, rank capacity,
 * ranks and values (the whole factor storage) to a binary file, after the
 * context's stream has finished its work.  hm_load builds a new matrix with
 * exactly that structure and those values (host byte order; a file that is
 * short, from another format or inconsistent with its structure gives
 * HM_ERR_ARG, as does a path that cannot be opened). */
hm_status hm_save(hm_ctx* ctx, const hm_matrix* m, const char* path);
hm_status hm_load(hm_ctx* ctx, const char* path, hm_matrix** out);
/* Host-only check of a checkpoint file (no device is used): reads its
 * structure and accepts it only if it is one hm_save could have written --
 * perm a permutation of 0..n-1; the cluster tree rooted at cluster 0, every
 * son stored after its father with the sons' index ranges splitting the
 * father's; every non-leaf block (t, s) followed later by its sons
 * sons(t) x sons(s) in row-major order, and every block reached once from
 * the root; ranks within capacity; and exactly as many values as the
 * structure and kmax fix.  hm_load applies the same checks.  n, nclusters,
 * nblocks (each may be NULL) receive the sizes.  HM_ERR_ARG for a file that
 * cannot be opened or fails a check. */
hm_status hm_file_info(const char* path, int64_t* n, int32_t* nclusters, int32_t* nblocks);
/* Same structure, all leaves zero (dense zeros, rank 0). */
hm_status hm_zeros_like(hm_ctx* ctx, const hm_matrix* src, hm_matrix** out);
/* Copy the values of src into dst (identical structure required). */
hm_status hm_copy_values(hm_ctx* ctx, const hm_matrix* src, hm_matrix* dst);
void hm_matrix_free(hm_matrix* m);

/*
 * Z <- blocktrunc(Z + alpha X Y) (Sect. 4).  mode HM_STANDARD applies every
 * low-rank product immediately by rkupdate; HM_ACCUMULATED gathers them in
 * accumulators (Figs. addproduct, split, flush).  eps is the relative
 * Frobenius truncation tolerance of every truncated addition (Fig. rkadd).
 * X, Y, Z must share one cluster tree.  info may be NULL.
 */
hm_status hm_addmul(hm_ctx* ctx, double alpha, hm_matrix* X, hm_matrix* Y, hm_matrix* Z, double eps, int32_t mode,
                    hm_run_info* info);

/*
 * In-place H-LU factorisation G = L R (Sect. 6, block LR pattern): L unit lower
 * and R upper triangular, stored in G's structure, no pivoting.  mode as for
 * hm_addmul.  Returns HM_ERR_SINGULAR on a zero leaf pivot.
 */
hm_status hm_lu(hm_ctx* ctx, hm_matrix* G, double eps, int32_t mode, hm_run_info* info);

/* hm_lu and hm_addmul with options: opt->eps, mode, precision, schedule,
 * use_graph and rank_override apply (opt may be NULL for the defaults). */
hm_status hm_lu_opt(hm_ctx* ctx, hm_matrix* G, const hm_options* opt, hm_run_info* info);
hm_status hm_addmul_opt(hm_ctx* ctx, double alpha, hm_matrix* X, hm_matrix* Y, hm_matrix* Z, const hm_options* opt,
                        hm_run_info* info);

/* Totals of a context since its creation (not in the paper): plans made and
 * their host seconds, runs and their device seconds, truncations executed and
 * their algorithmic bytes 8 (m + n)(l + k), builds and their seconds, and the
 * device memory of the context's allocator: bytes in use now, the most in use
 * at once, and allocations made. */
typedef struct {
  int64_t plans;
  double plan_seconds;
  int64_t runs;
  double run_seconds;
  int64_t truncations;
  int64_t trunc_bytes;
  int64_t builds;
  double build_seconds;
  int64_t device_bytes_in_use;
  int64_t device_bytes_peak;
  int64_t device_allocations;
} hm_stats;
hm_status hm_get_stats(const hm_ctx* ctx, hm_stats* out);

/*
 * In-place H-matrix inversion G <- G^{-1} (Sect. 6: the block inversion of a
 * 2 x 2 block matrix in six steps, G11^{-1}, H12 = G11^{-1} G12 and
 * H21 = G21 G11^{-1}, the Schur complement S = G22 - H21 G12, S^{-1}, the
 * off-diagonal blocks -H12 S^{-1} and -S^{-1} H21, and
 * G11^{-1} - H12 (-S^{-1} H21); recursively on a binary cluster tree, dense
 * inverses of the leaves).  mode HM_STANDARD forms every product by the
 * standard multiplication; HM_ACCUMULATED follows Fig. invert: updates of a
 * block gathered in accumulators, the Schur complement added without a flush,
 * the last product flushed into G11, and a leaf flushed before its inverse is
 * formed.  The auxiliary H12 and H21 are temporaries of the plan.  eps as for
 * hm_lu; HM_ERR_SINGULAR when a leaf meets a zero pivot (no pivoting: G and
 * its principal submatrices must be invertible, as the paper assumes),
 * HM_ERR_STATE for a cluster tree that is not binary.
 */
hm_status hm_inv(hm_ctx* ctx, hm_matrix* G, double eps, int32_t mode, hm_run_info* info);
hm_status hm_plan_inv(hm_ctx* ctx, hm_matrix* G, int32_t mode, hm_plan** out);

/*
 * In-place H-Cholesky factorisation G = L L^T of a symmetric positive
 * definite H-matrix (Sect. 6: treated like the block inversion and H-LU; the
 * reading is the recursion chol(t) = chol(t0); G10 <- G10 L00^{-T};
 * G11 <- G11 - G10 G10^T on the lower blocks of G11; chol(t1), with dense
 * Cholesky factors of the leaves).  L is stored in the blocks on and below
 * the diagonal (zeros above the diagonal of the diagonal leaves); the blocks
 * above the diagonal are neither read nor written.  mode HM_STANDARD applies
 * every product at once; HM_ACCUMULATED gathers the Schur complements in
 * accumulators (the accumulator of a diagonal block split into its lower sons
 * only) and flushes a block before it is solved or factorised.  eps as for
 * hm_lu; HM_ERR_SINGULAR when a leaf pivot is not positive.
 */
hm_status hm_chol(hm_ctx* ctx, hm_matrix* G, double eps, int32_t mode, hm_run_info* info);
hm_status hm_plan_chol(hm_ctx* ctx, hm_matrix* G, int32_t mode, hm_plan** out);

/*
 * Record and schedule once, run many times.  A plan is bound to the matrices it
 * was made for; each run uses their current values.  hm_plan_run takes eps.
 */
hm_status hm_plan_lu(hm_ctx* ctx, hm_matrix* G, int32_t mode, hm_plan** out);
hm_status hm_plan_addmul(hm_ctx* ctx, double alpha, hm_matrix* X, hm_matrix* Y, hm_matrix* Z, int32_t mode,
                         hm_plan** out);
/* One plan for the H-LU of `count` independent matrices G[0..count) (host
 * array of distinct handles; each keeps its own cluster and block tree).  The
 * instances' work items share the waves of one schedule, so each batched
 * launch carries the independent truncations, products and leaf
 * factorisations of all instances; every instance's result is the one that
 * hm_plan_lu gives it alone (same items, same arithmetic).  Run with
 * hm_plan_run; the run info sums over the instances. */
hm_status hm_plan_lu_batch(hm_ctx* ctx, hm_matrix* const* G, int32_t count, int32_t mode, hm_plan** out);
/* Solution with the H-LU factors stored in G (after hm_lu or a run of an
 * H-LU plan): X <- (L R)^{-1} X, forward substitution with the unit lower
 * factor and backward substitution with the upper one, by blocks of the
 * H-matrix (leaf triangular solves and H-matrix times dense products on the
 * GPU; Sect. 6).  X: device, n x c column-major with leading dimension
 * ldx >= n, rows in cluster order (position p holds unknown perm[p]), solved
 * in place.  hm_plan_lu_solve records the solve once for repeated runs
 * (hm_plan_run; its eps is not used); the plan is bound to X.  The result is
 * undefined when G does not hold H-LU factors. */
hm_status hm_plan_lu_solve(hm_ctx* ctx, hm_matrix* G, double* X, int64_t ldx, int32_t c, hm_plan** out);
hm_status hm_lu_solve(hm_ctx* ctx, hm_matrix* G, double* X, int64_t ldx, int32_t c);
hm_status hm_plan_run(hm_ctx* ctx, hm_plan* plan, double eps, hm_run_info* info);
/* Run the plan as a hipGraph (enable != 0): its launches are captured on the
 * next hm_plan_run and replayed by later ones; a change of eps or of the
 * context captures again.  Only wave plans on two streams (HM_WAVE_LANES=2)
 * of at most 24,000 launches are captured; dataflow plans, wave plans on four
 * streams and larger plans, and plans recorded with HM_PROFILE_OPS=1 or
 * HM_DEBUG=1, keep running launch by launch (hm_run_info.graph_replay tells
 * which happened).  Returns HM_ERR_ARG for a NULL plan. */
hm_status hm_plan_use_graph(hm_plan* plan, int32_t enable);
/* Arithmetic of the plan's dense products (GEMM items) and of its small-block
 * truncations (33 <= max(m, n) <= 64: the stacked-factor products
 * K = sum A_p B_p^T and D = K^T U_k); larger truncations, and blocks of at
 * most 32 x 32 (one wavefront per item, see hm_trunc_batch), stay FP64.  A
 * mixed plan meets the eps bound up to the FP32 rounding of those products.
 * Default HM_FP64; returns HM_ERR_ARG for an unknown precision. */
hm_status hm_plan_set_precision(hm_plan* plan, int32_t precision);
/* Attach the rank predictor `mlp` (NULL detaches) to the plan's small-block
 * truncations (m, n <= 64).  omega: device array, 64 x 32 column-major FP64,
 * the Gaussian test matrix of the sketches (drawn by the caller).  mode 0: the
 * truncations stay exact and only compute their 8 features (level, log2 m,
 * log2 n, log2(1 + l), log10 of the 4 singular values of K omega(:, 0:4)
 * relative to |K|_F); mode 1: the network's estimate k^ sizes a range
 * finder of width w = k^ + oversample: the column-pivoted QR of the exact
 * path stops after w steps, the core SVD runs on those w columns, and the
 * result is kept when the exact residual |K - Q_w Q_w^T K|_F^2 (the remaining
 * column norms) meets the eps bound of the rank rule; otherwise the same QR
 * continues to the exact path.  Only truncations whose pivoted QR would run
 * more than w steps are affected.  A kept result meets the eps bound with a
 * rank that can exceed the exact one.  Only the first 4 columns of omega are
 * read.  mlp and omega must outlive the plan's runs. */
hm_status hm_plan_set_predictor(hm_plan* plan, const hm_mlp* mlp, const double* omega, int32_t oversample,
                                int32_t mode);
/* Rank override of the plan's truncation items (see hm_options): count
 * entries in recording order (host array, copied), or ranks NULL to remove it.
 * HM_ERR_ARG when count differs from the plan's number of truncation items. */
hm_status hm_plan_set_rank_override(hm_plan* plan, const int32_t* ranks, int64_t count);
/* Per truncation item (recording order), 10 floats: the 8 features, k^ (-1
 * when not predicted) and the outcome (0 exact, 1 range finder, 2 fell back);
 * -NaN for items that did not run the small-block kernel.  Recorded when the
 * plan was made with HM_FEATURE_LOG=1 and a predictor is attached.  Copies at
 * most cap items, returns the number of items (0 without a log, -1 on error). */
int64_t hm_plan_feature_log(const hm_plan* plan, float* out, int64_t cap);
/* Autotuner: runs the plan once per variant of the small-block truncation
 * kernel (4 or 8 threads per column of the core), timing every launch with
 * HIP events, and keeps for each small-block launch the faster variant.  The
 * matrix the plan writes is restored from a device snapshot before each trial
 * and at the end, so it is left as it was.  The variants agree to rounding
 * (their column sums combine 4 or 8 partial sums).  chosen[0] / chosen[1]:
 * launches that kept 4 / 8 threads per column.  A plan recorded with the
 * environment variable HM_SMALL_TPC=8 starts with the 8-thread variant.
 * Costs two runs of the plan and one copy of the written matrix in device
 * memory; returns HM_ERR_NUMERIC if a trial run reports a device error. */
hm_status hm_plan_autotune(hm_ctx* ctx, hm_plan* plan, double eps, int64_t* chosen);
void hm_plan_free(hm_plan* plan);
/* Per truncation work item of the last run, in the order of the recursion,
 * 9 ints: m, n, l, k, Jacobi sweeps, the cycles/16 spent in the QR, core and
 * rebuild phases (these 8 are -1 for skipped items), and the item's wave;
 * recorded when the plan was made with the environment variable
 * HM_TRUNC_LOG=1.  Copies at most cap items into out (may be NULL)
 * and returns the number of items (-1 on error). */
int64_t hm_plan_trunc_log(const hm_plan* plan, int32_t* out, int64_t cap);
/* Per launch of the plan, 5 doubles: wave, work-item kind (0 GEMM, 1 TRUNC,
 * 2 LU, 3 TRSM, 4 COPY), variant (truncations: 0 general kernels, 1 / 2
 * small-block kernel with 4 / 8 threads per column), items, and the device
 * milliseconds of the last run (0 unless the plan was recorded with
 * HM_PROFILE_OPS=1).  Copies at most cap launches into out (may be NULL) and
 * returns the number of launches (-1 on error). */
int64_t hm_plan_launch_log(const hm_plan* plan, double* out, int64_t cap);

/*
 * Batched truncated addition (Fig. rkadd) on raw device factors:
 *   (Cout, Dout) <- trunc_eps(C D^T + alpha A B^T)
 * A: m x k1 (lda), B: n x k1 (ldb), C: m x k2 (ldc), D: n x k2 (ldd), all
 * column-major device arrays; Cout (m x kcap, ld m) and Dout (n x kcap, ld n)
 * receive the new factors with rank *rank_out <= kcap (device int).  The
 * outputs may alias C and D when their leading dimensions are m and n.
 * k1 == 0 leaves the outputs untouched (adding zero is a no-op).
 * descs is a HOST array of count descriptors.  precision (hm_precision)
 * applies to the items with 33 <= max(m, n) <= 64; larger items, and items of
 * at most 32 x 32, are FP64.  Items of at most 32 x 32 run one per wavefront
 * (four per workgroup); the environment variable HM_TINY=0 sends them through
 * the block-wide small-block path instead (the same steps, equal ranks,
 * results equal to rounding).  Larger items whose stacked rank k1 + k2 is at
 * most 16 and whose larger side is at most 512, 256 or 128 rows (for k1 + k2
 * at most 4, 8 or 16) also run one per wavefront; HM_THIN=0 sends them
 * through the register-resident path (the same steps, equal ranks, results
 * equal to rounding).  Plans (hm_plan_*) run their truncations through the
 * other paths only.  Returns HM_ERR_NUMERIC when a rank exceeded kcap (the
 * rank is then clamped to kcap).
 */
typedef struct {
  int32_t m, n, k1, k2, kcap;
  int32_t lda, ldb, ldc, ldd;
  int32_t pad;
  double alpha;
  const double* A;
  const double* B;
  const double* C;
  const double* D;
  double* Cout;
  double* Dout;
  int32_t* rank_out;
} hm_trunc_desc;
hm_status hm_trunc_batch(hm_ctx* ctx, int32_t count, const hm_trunc_desc* descs, double eps, int32_t precision,
                         int64_t* executed);
/* hm_trunc_batch with the descriptor array in DEVICE memory (count entries,
 * as hm_trunc_desc; every pointer in them a device pointer), for callers whose
 * descriptors are made on the GPU.  The host cannot see the sizes, so the
 * caller bounds them: every item has m, n <= max_rows and k1 + k2 <= max_stack
 * (items beyond the bounds set HM_ERR_ARG in the status and are skipped).  The
 * descriptors are lowered and classified on the device; the workspace is sized
 * from the bounds.  executed (host, may be NULL) receives the executed
 * truncations; the call returns after the stream has finished. */
hm_status hm_trunc_batch_device(hm_ctx* ctx, int32_t count, const hm_trunc_desc* descs, int32_t max_rows,
                                int32_t max_stack, double eps, int32_t precision, int64_t* executed);
/* hm_trunc_batch_device for callers that cannot allocate device memory (code
 * under hipGraph capture, serving loops, harnesses that forbid hipMalloc): the
 * same operation and arguments, with every scratch buffer (lowered
 * descriptors, claim counter, per-item marks, truncation workspace) in one
 * 64 MiB array that each device holds for the life of the process; nothing is
 * allocated.  Limits: at most 4096 items, and count x the workspace that the
 * bounds imply for one item must fit the array (HM_ERR_ARG otherwise, checked
 * before anything is launched).  With executed NULL the call only enqueues its
 * kernels on the context's stream and returns (no error of the run is
 * reported); with executed set it waits for the stream and reports as
 * hm_trunc_batch_device.  Calls on one device share the array: calls that
 * overlap on one device race (serialise them on one stream). */
hm_status hm_trunc_batch_device_noalloc(hm_ctx* ctx, int32_t count, const hm_trunc_desc* descs, int32_t max_rows,
                                        int32_t max_stack, double eps, int32_t precision, int64_t* executed);
/* hm_trunc_batch with the rank predictor on its small items (m, n <= 64), as
 * for hm_plan_set_predictor in mode 1 (omega: device, 64 x 32 column-major
 * FP64; level: the level feature given to every item).  Each item either
 * keeps the range finder's result, which meets the eps bound of the rank rule
 * with a rank at least the exact one, or runs the exact path.  counts (host,
 * 3): executed truncations, accepted predictions, fallbacks to the exact path. */
hm_status hm_trunc_batch_predicted(hm_ctx* ctx, int32_t count, const hm_trunc_desc* descs, double eps,
                                   const hm_mlp* mlp, const double* omega, int32_t oversample, int32_t level,
                                   int64_t* counts);

/* Structure export (host arrays). */
int64_t hm_n(const hm_matrix* m);
hm_status hm_perm(const hm_matrix* m, int32_t* perm);
int32_t hm_num_clusters(const hm_matrix* m);
/* Clusters in pre-order: offset, size, level, first son, second son (-1). */
hm_status hm_clusters(const hm_matrix* m, int32_t* off, int32_t* size, int32_t* level, int32_t* son0,
                      int32_t* son1);
int32_t hm_num_blocks(const hm_matrix* m);
/* Blocks in depth-first pre-order: row cluster, column cluster, kind
 * (0 non-leaf, 1 admissible, 2 inadmissible), current rank (-1 if not
 * admissible), parent block (-1 for the root).  Reads ranks from the device. */
hm_status hm_blocks(hm_ctx* ctx, const hm_matrix* m, int32_t* t, int32_t* s, int32_t* kind, int32_t* rank,
                    int32_t* parent);
/* Dense n x n matrix in cluster order (host, column-major). */
hm_status hm_to_dense(hm_ctx* ctx, const hm_matrix* m, double* out);
/* Values of leaf block `block` (pre-order index of hm_blocks) as a dense
 * #t x #s host array with leading dimension ld >= #t (column-major; zero for
 * a non-leaf block).  Synchronises the stream. */
hm_status hm_block_to_dense(hm_ctx* ctx, const hm_matrix* m, int64_t block, double* out, int64_t ld);

/*
 * Rank predictor (a small network trained on logged truncations).
 * 8 features of a truncation -> predicted log2(1 + k):
 *   h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), y = w3 . h2 + b3
 * with W1: 64 x 8, W2: 64 x 64, w3: 64.  Parameters as one FP32 vector of
 * HM_MLP_NPARAM entries: W1 (row-major) | b1 | W2 (row-major) | b2 | w3 | b3.
 * The forward and backward passes use BF16 copies of W1, W2, w3 (rounded to
 * nearest even) and FP32 accumulation; Adam updates FP32 master weights.
 * Arrays X (B x 8, row-major FP32), t and y (B FP32) are device pointers.
 */
#define HM_MLP_NPARAM 4801
/* init: host FP32 master weights, or NULL for a He initialisation drawn from
 * seed (splitmix64 + Box-Muller, zero biases). */
hm_status hm_mlp_create(hm_ctx* ctx, const float* init, uint64_t seed, hm_mlp** out);
void hm_mlp_free(hm_mlp* mlp);
/* master: the FP32 master weights; working: the weights the kernels use (the
 * BF16 matrices as FP32, the FP32 biases).  Either may be NULL (host arrays). */
hm_status hm_mlp_get(hm_ctx* ctx, const hm_mlp* mlp, float* master, float* working);
/* y = network(X) for B samples. */
hm_status hm_mlp_predict(hm_ctx* ctx, const hm_mlp* mlp, const float* X, int64_t B, float* y);
/* Gradient of 0.5 mean (y - t)^2 over the B samples with respect to every
 * parameter (host grad, HM_MLP_NPARAM entries) and the loss (host, may be NULL). */
hm_status hm_mlp_gradient(hm_ctx* ctx, const hm_mlp* mlp, const float* X, const float* t, int64_t B, float* grad,
                          double* loss);
/* Adam (beta 0.9, 0.999) with learning rate lr over `epochs` passes of the B
 * samples in consecutive mini-batches of `batch` (the caller shuffles); the
 * mean loss of each epoch goes to epoch_loss (host, may be NULL). */
hm_status hm_mlp_train(hm_ctx* ctx, hm_mlp* mlp, const float* X, const float* t, int64_t B, int32_t epochs,
                       int32_t batch, float lr, float* epoch_loss);

#ifdef __cplusplus
}
#endif
#endif /* HM_H */
