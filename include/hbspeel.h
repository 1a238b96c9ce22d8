/*
 * hbspeel -- randomized compression of rank-structured matrices on MI355X.
 *
 * C ABI of the library (libhbspeel.so).  It implements, on one GPU, the
 * method of Martinsson, "Compressing rank-structured matrices via randomized
 * sampling" (arXiv 1503.07152):
 *
 *   hodlr_compress     Fig. 2  (HODLR, SVD variant of eq. SVDtogetV/SVDtogetB)
 *   hbs_compress       Fig. 4  (storage-efficient HBS) + Fig. 5 (HBS-ID)
 *   hss_apply(_adjoint) Fig. 7 with m = L, plus the diagonal blocks
 *
 * Conventions for every entry point
 *   - Matrices are column-major; "ld" is the leading dimension in elements.
 *   - Array arguments are DEVICE pointers unless stated "host".  The caller
 *     owns them; the library never keeps them past the call (except the
 *     operator's points / dense matrix, which must stay valid for the
 *     duration of a compress call).
 *   - `stream` is a hipStream_t (NULL = the null stream).  Work is enqueued
 *     on it; calls return when the work is enqueued unless stated otherwise.
 *     Compress calls synchronise the stream before returning (they report
 *     statistics and status).
 *   - Return value: HM_OK (0) on success, a negative HM_ERR_* code on error,
 *     a positive HM_WARN_* code for a successful call with a warning.  On
 *     error no handle is returned (out-pointer set to NULL), partial state is
 *     freed, and hm_last_error() gives a message (thread-local).
 *   - Handles (hm_hbs, hm_hodlr) are owned by the library and immutable
 *     after creation; apply may run concurrently on different streams.
 */
#ifndef HBSPEEL_H
#define HBSPEEL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define HM_OK 0
#define HM_WARN_RANK_SATURATED 1   /* a revealed eps-rank reached the cap r - p (Sec. 2.5:
                                      the sample may not have captured the block) */
#define HM_ERR_ARG (-1)            /* invalid argument (sizes, ld, options)     */
#define HM_ERR_ALLOC (-2)          /* device allocation failed                  */
#define HM_ERR_HIP (-3)            /* a HIP runtime call failed                 */
#define HM_ERR_CALLBACK (-4)       /* the user's matvec callback returned != 0  */
#define HM_ERR_NONFINITE (-5)      /* NaN/Inf in an operator sample             */
#define HM_ERR_UNSUPPORTED (-6)    /* size beyond a documented limit            */
#define HM_ERR_SINGULAR (-7)       /* hbs_factor: a block had a zero pivot      */

/* ---- element types ------------------------------------------------------ */
#define HM_F64 0
#define HM_F32 1
#define HM_BF16 2

/* ---- limits ---------------------------------------------------------------
 * Samples per level r = rank + oversample <= HM_MAX_SAMPLES.  The per-node
 * factorisations hold a (2r x 2r) triangle pair in LDS (160 KB per CU). */
#define HM_MAX_SAMPLES 48
/* Leaves hold at most HM_MAX_LEAF indices when the tree has more than one
 * level (the interpolative decomposition of a leaf runs in LDS). */
#define HM_MAX_LEAF 256

/* ---- operators (the black box of Sec. 1: x -> A x and x -> A^* x) -------- */
#define HM_OP_CALLBACK 0   /* user function                                    */
#define HM_OP_KERNEL 1     /* built-in kernel matrix on 2-D points, tiled MFMA */
#define HM_OP_DENSE 2      /* explicit N x N matrix                            */
#define HM_OP_HBS 3        /* a matrix held as an HBS handle, applied in O(N k) */
#define HM_OP_HBS_PRODUCT 4 /* the product hbs * hbs2 of two HBS handles, each
                               applied in O(N k) (Sec. 5.2, operator multiplication) */
#define HM_OP_FRONTAL 5    /* the frontal matrix of nested dissection held in an
                              hm_frontal handle (Sec. 5.4), symmetric */

#define HM_KERNEL_LOG 0    /* A(i,j) = log|x_i - x_j| (i != j), A(i,i) = 1       */
#define HM_KERNEL_NEAR 1   /* A(i,j) = 1 / (|x_i - x_j| + kparam) (all i, j)     */

typedef struct hm_hbs_s hm_hbs;
typedef struct hm_hodlr_s hm_hodlr;
typedef struct hm_hbs_factor_s hm_hbs_factor;
typedef struct hm_frontal_s hm_frontal;

/*
 * Black-box product (Sec. 1, "T_mult"; applied to N x ncols blocks as in
 * Sec. 5.3).  Must write Y = A X (adjoint = 0) or Y = A^* X (adjoint = 1) for
 * X, Y device arrays (n x ncols, column-major, leading dims ldx, ldy) owned by
 * the library for the duration of the call.  `dtype` is the operator's
 * sample_dtype and fixes the element types:
 *   HM_F64   X double, Y double
 *   HM_F32   X float,  Y float
 *   HM_BF16  X bfloat16 (uint16 bit patterns), Y float (FP32 accumulation)
 * The library rounds its FP64 test block to the sample type (round to nearest
 * even) and reads Y back into FP64 samples; node factorisations stay FP64.
 * The work must be enqueued on `stream` (a hipStream_t) or finished before
 * returning; the pointers must not be kept.  Return 0 on success; any other
 * value aborts the compression with HM_ERR_CALLBACK.
 */
typedef int (*hm_matvec_fn)(void* user, int adjoint, int64_t n, int64_t ncols,
                            const void* X, int64_t ldx, void* Y, int64_t ldy,
                            int32_t dtype, void* stream);

typedef struct hm_operator {
  int32_t kind;          /* HM_OP_*                                              */
  int32_t sample_dtype;  /* precision of the sampling product, HM_OP_KERNEL:
                            HM_F64 (FP64 MFMA), HM_F32 (FP32 MFMA),
                            HM_BF16 (BF16 MFMA, FP32 accumulation);
                            HM_OP_CALLBACK: the types the callback receives
                            (see hm_matvec_fn).  The samples are returned in
                            FP64 in every case.                                 */
  hm_matvec_fn fn;       /* HM_OP_CALLBACK                                       */
  void* user;            /* HM_OP_CALLBACK: passed back to fn                    */
  const double* points;  /* HM_OP_KERNEL: device, n points as (x0,y0,x1,y1,...)  */
  int32_t kernel_id;     /* HM_OP_KERNEL: HM_KERNEL_*                            */
  double kparam;         /* HM_OP_KERNEL: delta of HM_KERNEL_NEAR                */
  const double* dense;   /* HM_OP_DENSE: device, n x n column-major FP64         */
  int64_t ld;            /* HM_OP_DENSE: leading dimension                       */
  const hm_hbs* hbs;     /* HM_OP_HBS, HM_OP_HBS_PRODUCT: an FP64 handle (left factor) */
  const hm_hbs* hbs2;    /* HM_OP_HBS_PRODUCT: the right factor, an FP64 handle of
                            the same size: A x = hbs (hbs2 x), A^* x = hbs2^* (hbs^* x) */
  const hm_frontal* frontal; /* HM_OP_FRONTAL: a handle of height n               */
} hm_operator;

/* Flags */
#define HM_FLAG_ORTHONORMAL 1  /* hbs_compress: stop after Fig. 4 (orthonormal
                                  nested bases, r columns per node), no Fig. 5 */
#define HM_FLAG_PERSISTENT_ID 2 /* run the Fig. 5 sweep as one persistent launch
                                  over every level, side and instance (a device work
                                  queue; a parent is taken up once both children are
                                  done) instead of the default level by level (two
                                  launches per level and side, the two sides on two
                                  streams); same result */
#define HM_FLAG_LOW_MEMORY_PLAN 4 /* with the built-in kernel operator sampled in BF16:
                                  one operator call per product instead of first
                                  products riding in shared calls of up to 288
                                  columns, so that one window of sample columns is
                                  held instead of several (more calls, more time);
                                  the plan the compression falls back to by itself
                                  when the shared windows would exceed 4 GiB */

typedef struct hm_options {
  int64_t n;            /* matrix size N >= 1                                    */
  int64_t leaf_size;    /* m of Sec. 2.7: intervals of more than m indices are split
                           (uniform depth L = ceil(log2(N/m)), left half ceil(n/2)) */
  int32_t rank;         /* k >= 1: fixed rank (tol == 0) or rank cap (tol > 0)   */
  int32_t oversample;   /* p >= 0 (Sec. 2.5); r = rank + p samples per level     */
  double tol;           /* eps in [0,1): relative per block (s_j > eps s_1,
                           |R_jj| > eps |R_11|); 0 selects fixed rank k          */
  uint64_t seed;        /* key of the Philox4x32-10 Gaussian stream               */
  int32_t flags;        /* HM_FLAG_*                                             */
  int32_t store_dtype;  /* HBS handles: HM_F64 (default) or HM_F32 -- the node
                           factorisations run in FP64, the resulting generators
                           are stored (and applied) in this type.  HODLR: HM_F64 */
} hm_options;

typedef struct hm_info {
  int64_t n, leaf_size;
  int32_t levels;        /* L                                                      */
  int32_t rank_pad;      /* R: padded rank of the stored generators               */
  int32_t max_rank, min_rank;   /* over non-root nodes (HBS) or sibling blocks (HODLR) */
  int32_t is_id;         /* HBS-ID form (identity on skeleton rows)               */
  int32_t dtype;         /* storage type of the generators                        */
  int64_t storage_reals; /* reals needed at the revealed ranks (M of Sec. 5)      */
  int64_t sample_columns;/* columns sent to the operator (4 r L + n_max)          */
  int32_t operator_calls;/* operator invocations: 2 L + 1 (Omega_1, Omega_2 merged).
                            Fewer for the built-in kernel operator sampled in
                            BF16 (symmetric, so A and A* are one product), whose
                            calls take up to 288 columns: one call takes the
                            first products of G = min(L, floor(288 / 2r))
                            levels, each level's second call those of the next
                            levels that fit beside its 2r columns; when every
                            instance has L levels and 2r + n_max <= 288 the
                            block identity rides in second calls too (spare
                            columns of the narrow ones, else the last level's);
                            L + 1 calls when all first products fit so       */
  int32_t saturated;     /* nodes whose revealed rank reached r - p               */
  double t_compress_ms;  /* wall time of the compress call                        */
  double t_operator_ms;  /* time inside the operator (T_compress - T_net)         */
  int32_t jacobi_sweeps; /* most one-sided Jacobi sweeps any node SVD needed       */
  int32_t adapt_rounds;  /* hbs_compress_adaptive: compressions run (else 1)      */
  double err_estimate;   /* hbs_compress_adaptive: the final posterior estimate E
                            of Sec. 5 (else -1)                                   */
} hm_info;

/* ---- library ------------------------------------------------------------- */
/* Message of the last error on this thread ("" if none). */
const char* hm_last_error(void);
/* Build identification string (static storage). */
const char* hm_version(void);

/* Device memory (not part of the method; for callers that manage device
 * memory themselves, e.g. a framework's caching allocator).
 * hm_set_allocator installs alloc / free for every device allocation the
 * library makes from then on: handle generators and node tables, and per-call
 * scratch of compress, apply and backward.  alloc(ctx, bytes, stream) returns
 * device memory of at least `bytes` bytes, 256-byte aligned, usable by work
 * enqueued on `stream` (the stream passed to the entry point; NULL for calls
 * without one), or NULL on failure (the call then fails with HM_ERR_ALLOC).
 * free(ctx, ptr, stream) returns it with the stream it was allocated for,
 * after the library's last use of it has been enqueued on that stream, so a
 * stream-ordered allocator may reuse it at once.  Handle memory is returned
 * by hm_hbs_free / hm_hodlr_free: work on other streams that reads the
 * handle must be complete by then.  Every buffer goes back to the allocator
 * that made it, even after hm_set_allocator is called again.  alloc == NULL
 * (with free == NULL) restores the default: hipMalloc'd blocks that the
 * library keeps when they are released and hands out again to allocations of
 * the same rounded size for the same stream (stream order makes the reuse
 * safe), and hipMallocAsync / hipFreeAsync for scratch.  Exactly one of
 * alloc, free NULL: HM_ERR_ARG.  Not to be called while other threads are
 * inside the library. */
typedef void* (*hm_alloc_fn)(void* ctx, size_t bytes, void* stream);
typedef void (*hm_free_fn)(void* ctx, void* ptr, void* stream);
int hm_set_allocator(hm_alloc_fn alloc, hm_free_fn free, void* ctx);
/* Returns the device blocks the default allocator keeps for reuse to the
 * driver (hipFree, after waiting for the device).  Blocks in use stay. */
int hm_release_cached_memory(void);

/* ---- test matrices (Sec. 2.5; the randn of Fig. 2/4) ---------------------
 * Writes G(i, j) for rows i = row0 .. row0+nrows-1 and columns j = 0..ncols-1
 * of the counter-based Gaussian stream: Philox4x32-10 (Salmon et al., SC'11)
 * with counter (i, j>>1, level, phase) and key (seed mod 2^32, seed>>32), two
 * 53-bit uniforms u1 in (0,1], u2 in [0,1), Box-Muller (even j: cos branch,
 * odd j: sin branch).  out: device FP64 nrows x ncols, leading dim ld. */
int hm_gauss(uint64_t seed, int32_t level, int32_t phase, int64_t row0,
             int64_t nrows, int32_t ncols, double* out, int64_t ld, void* stream);

/* ---- operators ----------------------------------------------------------------
 * Y = A X (adjoint = 0) or A^* X through the operator `op` (any kind), exactly
 * as the compression samples it: X, Y device FP64 n x ncols column-major.  For
 * HM_OP_KERNEL the product runs in op->sample_dtype and is returned in FP64.
 * Enqueued on `stream`; returns without waiting for it. */
int hm_operator_apply(const hm_operator* op, int64_t n, int32_t adjoint, int64_t ncols,
                      const double* X, int64_t ldx, double* Y, int64_t ldy, void* stream);

/* ---- compression ------------------------------------------------------------
 * hodlr_compress: Fig. 2.  Per level: Y = A [Omega_2 | Omega_1] - A^(l) [...],
 * U = qr(Y block), Z = A^* [Psi_2 | Psi_1] - (A^(l))^* [...], [V, B, U^] =
 * svd(Z block, eps or k), U <- U U^; then D from a block-identity sample.
 * hbs_compress: Fig. 4 then (unless HM_FLAG_ORTHONORMAL) Fig. 5.
 * Returns HM_OK or HM_WARN_RANK_SATURATED with *out set; errors as above. */
int hodlr_compress(const hm_options* opts, const hm_operator* op, void* stream,
                   hm_hodlr** out);
int hbs_compress(const hm_options* opts, const hm_operator* op, void* stream,
                 hm_hbs** out);

/* Adaptive sampling (the paper fixes the samples per level in advance and
 * notes that adaptive rank determination could be built in, Sec. 4.3;
 * Remark 1.1 and Sec. 2.5 on the failure risk): tolerance mode (opts->tol >
 * 0) with opts->rank as the first rank cap k.  After each compression, if a
 * node's revealed rank reached the cap k (HM_WARN_RANK_SATURATED: the r = k +
 * p samples may not have captured its block) or the posterior estimate E of
 * Sec. 5 exceeds e_target, the cap doubles (to at most HM_MAX_SAMPLES - p) and
 * the compression runs again with the same seed (the Gaussian blocks are
 * defined by row, column and level, so the first columns of every level's
 * block stay the same).  E = max over 10 probe vectors w of |A w - A_H w| /
 * |A w|, the probes from phase 1 of the Gaussian stream keyed by opts->seed.
 * Returns HM_OK, or HM_WARN_RANK_SATURATED if the cap reached its limit with
 * a node still saturated or E > e_target.  hm_info: adapt_rounds,
 * err_estimate; sample_columns, operator_calls and the times add up all
 * rounds (the probes' 10 columns per round not included). */
int hbs_compress_adaptive(const hm_options* opts, const hm_operator* op, double e_target,
                          void* stream, hm_hbs** out);

/* Autotuner of the compression's schedule and tiles for one workload shape
 * (N, samples r, levels, largest leaf, sampler).  For the built-in kernel
 * operator sampled in BF16 it times hbs_compress under every combination of:
 *   gfirst  levels whose first products share one sampler call (1 .. 288 / 2r)
 *   ride    later first products a second-product call may carry (0 .. 2)
 *   ksplit  K-splits of the narrow sampler form (2, 3, 4)
 * (reps timed calls each after one warm-up call, the fastest counted), then
 * keeps the fastest for every later hbs_compress of that shape in this
 * process; other operators have one schedule.  The choices change only the
 * order of the FP32 sums of the BF16 products.  out (host): the choice
 * (0 / -1: the built-in default), candidates timed, and the default's and
 * the best's time in ms.  reps == 0 restores the built-in defaults for the
 * shape without timing anything.  Not to be called while other threads
 * compress. */
typedef struct hm_tune {
  int32_t gfirst, ride, ksplit, candidates;
  double t_default_ms, t_best_ms;
} hm_tune;
int hm_autotune(const hm_options* opts, const hm_operator* op, int32_t reps, void* stream,
                hm_tune* out);

/* Many independent HBS compressions (count instances of uneven N and rank),
 * level-synchronous: each level's sampling, peeling and node factorisations
 * of all instances run in the same batched launches.  Every operator must be
 * HM_OP_HBS, HM_OP_KERNEL or HM_OP_DENSE; all instances share flags and
 * store_dtype.  outs: host array of count handle pointers. */
int hbs_compress_batched(int32_t count, const hm_options* opts,
                         const hm_operator* ops, void* stream, hm_hbs** outs);

/* ---- apply (Fig. 7 with m = L, plus D) --------------------------------------
 * y = A_H x  /  y = A_H^* x for an n x nrhs block x.  x, y: device arrays of
 * the handle's dtype (HM_F64 or HM_F32), column-major, leading dims >= n.
 * x and y must not overlap. */
int hss_apply(const hm_hbs* h, int64_t nrhs, const void* x, int64_t ldx,
              void* y, int64_t ldy, void* stream);
int hss_apply_adjoint(const hm_hbs* h, int64_t nrhs, const void* x, int64_t ldx,
                      void* y, int64_t ldy, void* stream);

/* Backward of y = A_H x (not in the paper): given gy, writes gx = A_H^* gy and
 * the gradients of <gy, A_H x> with respect to the generators in the flat
 * layout of hm_hbs_from_generators (any of the generator outputs may be NULL
 * to skip it).  Every entry of each requested output is written (blocks that
 * no node owns, and D columns past a leaf's size, are set to zero), so the
 * outputs need no initialisation.  Same dtype rules as hss_apply. */
int hss_apply_backward(const hm_hbs* h, int64_t nrhs, const void* x, int64_t ldx,
                       const void* gy, int64_t ldgy, void* gx, int64_t ldgx,
                       void* gU, void* gV, void* gUt, void* gVt, void* gB,
                       void* gD, void* stream);

/* hss_apply for callers that cannot allocate device memory (code under
 * stream capture, serving loops, harnesses that forbid allocation): the same
 * y = A_H x with the same kernels and argument rules, but it allocates
 * nothing -- no hipMalloc / hipFree and no call of an hm_set_allocator
 * allocator.  The kernels' scratch (per-node expansions, 2 R c values each,
 * and row-chunk partials) lives in a fixed array of 32 MiB in the library's
 * device memory, one per GPU, held until the process ends; the columns of x
 * are processed in passes of as many as fit (at most 128).  A handle whose
 * single column needs more than 32 MiB of scratch is rejected with
 * HM_ERR_UNSUPPORTED.  Every call on a GPU uses that GPU's one array: calls
 * that overlap on one GPU (other streams, other threads) race and must be
 * serialised by the caller; calls on one stream are ordered. */
int hss_apply_noalloc(const hm_hbs* h, int64_t nrhs, const void* x, int64_t ldx,
                      void* y, int64_t ldy, void* stream);

/* Direct solver for an HBS matrix (the consumer of the compressed form the
 * paper names in Sec. 1; the algorithm is the one of Gillman, Young and
 * Martinsson for HBS matrices).  hbs_factor builds, from the leaves up, per
 * node Dh = (V^* D^-1 U)^-1, E = D^-1 U Dh, F^* = Dh V^* D^-1 and
 * G = D^-1 - D^-1 U Dh V^* D^-1, where a parent's D is [Dh_a B_ab; B_ba Dh_b]
 * and its U, V are its transfer matrices, and inverts the root's block: then
 * A^-1 = E (Dh + A~)^-1 F^* + G level by level.  Requirements: an FP64,
 * single-tree handle with at least one level, every non-root node of the same
 * incoming and outgoing rank k (fixed-rank compressions and handles from
 * generators), leaves of at most 128 rows.  Block inversions are Gauss-Jordan
 * with partial pivoting; a zero or non-finite pivot gives HM_ERR_SINGULAR.
 * Other handles give HM_ERR_ARG (dtype, forest, rank 0) or HM_ERR_UNSUPPORTED
 * (mixed ranks, larger leaves).  No pivoting happens across levels, so the
 * error grows with the conditioning of the D blocks and of V^* D^-1 U, not
 * only with cond(A).  The factor is independent of the handle (which may be
 * freed) and owned by the library (hm_hbs_factor_free; NULL is a no-op);
 * hbs_factor returns when it is complete.  Device memory: 8 (3 N k + N nmax
 * + nodes (k^2 + 8 k^2)) bytes, plus the same again as work during the call.
 * hbs_solve: x = A_H^-1 b for an n x nrhs FP64 block b (device, column-major,
 * leading dims >= n; HM_ERR_ARG otherwise); enqueued on `stream`, in chunks
 * of 128 columns; x and b must not overlap. */
int hbs_factor(const hm_hbs* h, void* stream, hm_hbs_factor** out);
int hbs_solve(const hm_hbs_factor* f, int64_t nrhs, const double* b, int64_t ldb, double* x,
              int64_t ldx, void* stream);
void hm_hbs_factor_free(hm_hbs_factor* f);

/* ---- frontal matrix of nested dissection (Sec. 5.4, Fig. 13) -----------------
 * The black box of that section: a conduction grid of `height` rows and
 * `width` (odd; 41 in the paper) columns of nodes, a bar between every two
 * neighbouring nodes, B the network's matrix (graph Laplacian: the sum of the
 * conductivities of a node's bars on the diagonal, minus the bar's
 * conductivity between neighbours), I3 the middle column (by row), I1 / I2
 * the columns left / right of it, and
 *   A = B33 - B31 B11^-1 B13 - B32 B22^-1 B23     (height x height, symmetric).
 * hm_frontal_create factors B11 and B22 on the device (block cyclic
 * reduction over grid rows, FP64) and returns when the factor is complete.
 * ch: device, height x (width - 1) C-ordered, ch[i (width-1) + j] joins nodes
 * (i, j) and (i, j+1); cv: device, (height - 1) x width C-ordered, cv[i width +
 * j] joins (i, j) and (i+1, j) (may be NULL when height == 1).  Both are read
 * during the call only.  Conductivities must be positive and finite; a
 * non-positive pivot gives HM_ERR_SINGULAR.  width > 65 gives
 * HM_ERR_UNSUPPORTED, other bad sizes HM_ERR_ARG.  With w = (width - 1) / 2
 * and wp = w rounded up to a multiple of 4, the handle holds about
 * 8 (6 wp^2 + 19 wp + 19) height bytes of device memory (2.3 GB per 100k rows
 * at width 41: the factor and the small operators of its first two levels)
 * and the call uses 32 w^2 height bytes more as work.
 * hm_frontal_apply: Y = A X for X, Y device, column-major, height x ncols,
 * leading dims >= height (HM_ERR_ARG otherwise); FP64; enqueued on `stream`,
 * in passes of at most 128 columns with a work block of about
 * 8 (2 wp + 5) height c bytes for c columns (wp: w rounded up to a multiple
 * of 4); X and Y must not overlap.  The handle is also an operator
 * (HM_OP_FRONTAL) for the compressions.  hm_frontal_free(NULL) is a no-op. */
int hm_frontal_create(int64_t height, int32_t width, const double* ch, const double* cv,
                      void* stream, hm_frontal** out);
int hm_frontal_apply(const hm_frontal* f, int64_t ncols, const double* X, int64_t ldx, double* Y,
                     int64_t ldy, void* stream);
void hm_frontal_free(hm_frontal* f);

/* HODLR apply: y = A_H x (adjoint = 0) or A_H^* x; FP64. */
int hodlr_apply(const hm_hodlr* h, int32_t adjoint, int64_t nrhs,
                const double* x, int64_t ldx, double* y, int64_t ldy, void* stream);

/* ---- handles ----------------------------------------------------------------
 * hm_hbs_from_generators: an HBS handle from generators of uniform rank
 * k <= HM_MAX_SAMPLES in the flat layout (all device, column-major blocks;
 * nn = 2^(L+1)):
 *   U, V   n x k          rows I_t of leaf t hold its basis
 *   Ut, Vt nn blocks of 2k x k (block t at offset t*2k*k); rows 0..k-1 couple
 *          to the left child 2t, rows k..2k-1 to 2t+1; used for 2 <= t < 2^L
 *   B      nn blocks of k x k; B[v] maps the outgoing expansion of v to the
 *          incoming expansion of its sibling: A(I_sib(v), I_v) = U_sib B[v] V_v^*
 *   D      n x nmax; rows I_t of leaf t hold D_t in columns 0..n_t-1
 * dtype HM_F64 or HM_F32 (the arrays' type).  The data is copied. */
int hm_hbs_from_generators(int64_t n, int64_t leaf_size, int32_t k, int32_t dtype,
                           const void* U, const void* V, const void* Ut,
                           const void* Vt, const void* B, const void* D,
                           void* stream, hm_hbs** out);
/* Copy of a handle with its generators converted to another storage dtype
 * (HM_F64 / HM_F32, rounded to nearest); structure, ranks and skeletons are
 * kept.  The copy is complete when the call returns. */
int hm_hbs_convert(const hm_hbs* h, int32_t dtype, void* stream, hm_hbs** out);
int hm_hbs_info(const hm_hbs* h, hm_info* host_out);
/* Device views of the generators of an HBS matrix (Sec. 2.9: leaf bases U_t,
 * V_t, the nested bases' transfer matrices, the sibling couplings B and the
 * diagonal blocks D_t; Fig. 4 / Fig. 5 produce them).  The pointers alias the
 * handle's own memory (no copy): valid until hm_hbs_free, read-only (handles
 * are immutable).  Layout (column-major, R = rank_pad, nodes = 2^(L+1) - 1,
 * node with heap number t = 1..nodes at block index t - 1):
 *   U, V    n x R, ld n; rows I_t of leaf t hold its basis
 *   Ut, Vt  2R x R per node (ld 2R); rows 0..R-1 couple to the left child,
 *           R..2R-1 to the right child; used for internal non-root nodes
 *   B       R x R per node (ld R): A(I_sib(t), I_t) = U_sib(t) B_t V_t^*
 *           (through the nested bases above the leaves)
 *   D       n x nmax, ld n; rows I_t of leaf t hold D_t in columns 0..n_t-1
 * Entries beyond a node's revealed rank are zero.  Single-tree handles only
 * (every handle returned by the entry points is one). */
typedef struct hm_views {
  int32_t dtype;     /* HM_F64 or HM_F32: element type of every array */
  int32_t rank_pad;  /* R */
  int32_t levels;    /* L */
  int32_t nmax;      /* columns of D (largest leaf) */
  int64_t n;         /* rows */
  int64_t nodes;     /* 2^(L+1) - 1 */
  const void* U;
  const void* V;
  const void* Ut;
  const void* Vt;
  const void* B;
  const void* D;
} hm_views;
int hm_hbs_generators(const hm_hbs* h, hm_views* host_out);
int hm_hodlr_info(const hm_hodlr* h, hm_info* host_out);
/* Generators in the flat layout above with k = info.rank_pad (zero-padded
 * beyond each node's rank), written to caller device buffers of the handle's
 * dtype (any may be NULL).  ranks_u / ranks_v: host int32[nn] (may be NULL).
 * skel_in / skel_out: host int32[nn * rank_pad] global skeleton rows of the
 * HBS-ID form, -1 padded (may be NULL; -1 everywhere if not is_id). */
int hm_hbs_export(const hm_hbs* h, void* U, void* V, void* Ut, void* Vt, void* B,
                  void* D, int32_t* ranks_u, int32_t* ranks_v, int32_t* skel_in,
                  int32_t* skel_out, void* stream);
/* HODLR generators: per level l = 1..L, U_l, V_l (n x rank_pad, rows I_t of
 * the level's nodes), diagonal B entries s_l (nn x rank_pad: B_{sib(v),v} =
 * diag(s[v])), D (n x nmax).  U, V: device arrays of L*n*rank_pad (level l at
 * offset (l-1)*n*rank_pad); s: device nn*rank_pad; ranks: host int32[nn]. */
int hm_hodlr_export(const hm_hodlr* h, double* U, double* V, double* s, double* D,
                    int32_t* ranks, void* stream);
void hm_hbs_free(hm_hbs* h);
void hm_hodlr_free(hm_hodlr* h);

#ifdef __cplusplus
}
#endif
#endif /* HBSPEEL_H */
