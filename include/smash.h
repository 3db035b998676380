/*
 * smash.h -- C ABI of libsmash: SMASH H^2 / HSS construction and product on
 * AMD Instinct MI355X (gfx950).
 *
 * Method: D. Cai, E. Chow, Y. Saad, Y. Xi, "SMASH: Structured Matrix
 * Approximation by Separation and Hierarchy" (arXiv 1705.05443).  Given a
 * kernel kappa and point sets X, Y, build an H^2 (strong admissibility) or
 * HSS (weak admissibility) approximation A-hat of A = [kappa(x, y)]
 * (Sec. 3, statement of the construction problem) and apply it to blocks
 * of vectors (Sec. 3.4).
 *
 * Conventions for every entry point:
 *  - Pointers named "device" must point to device memory of the current HIP
 *    device; "host" pointers to host memory.  Row-major layouts throughout.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Work is enqueued on it; inputs are borrowed and must stay valid until
 *    the stream has passed the call (as for hipMemcpyAsync).
 *  - Return value: SMASH_OK (0) or a negative error code.  No exception
 *    crosses the ABI; on failure output handles are left NULL and nothing
 *    leaks.  smash_last_error() gives a thread-local message.
 *  - A handle owns every device allocation it makes and is freed by
 *    smash_destroy.  Calls on different handles may run on different host
 *    threads; one handle serves one product call at a time.
 */
#ifndef SMASH_H
#define SMASH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ---- */
#define SMASH_OK 0
#define SMASH_E_INVALID_ARG -1 /* bad size, pointer, parameter or option    */
#define SMASH_E_UNSUPPORTED -2 /* e.g. the 1/(x-y) kernel with dim != 1     */
#define SMASH_E_OOM -3         /* device or host allocation failed          */
#define SMASH_E_DEVICE -4      /* a HIP runtime call failed                 */
#define SMASH_E_NUMERIC -5     /* non-finite input, or the RRQR swap cap hit */

/* ---- kernels (Sec. 2, eq. (2.1) and the radial kernels of the tests) ---- */
#define SMASH_KERNEL_INV_R 0  /* 1/|x-y|,   kappa(x,x) = diag_value          */
#define SMASH_KERNEL_LOG_R 1  /* log|x-y|,  kappa(x,x) = diag_value          */
#define SMASH_KERNEL_EXP_R 2  /* exp(-|x-y|), its own value 1 at x = y       */
#define SMASH_KERNEL_CAUCHY 3 /* 1/(x-y) on the real line (dim 1 only), eq. (2.1) */
/* Laplace double layer in Nystrom form (Sec. 6.4, eq. (6.9)), dim 2, X = Y:
 * kappa(x, y) = -((y - x) . m_y) / (2 pi |x - y|^2) with m_y the column
 * point's weighted normal (quadrature weight times speed times outer unit
 * normal), and kappa(x, x) = the row point's own diagonal value.  Needs
 * options.point_data.  Coupling blocks are stored (not evaluated). */
#define SMASH_KERNEL_DOUBLE_LAYER 4

/* ---- admissibility (Sec. 3.2) ---- */
#define SMASH_ADM_WEAK 0   /* HSS: binary tree, (i,j) admissible iff i != j  */
#define SMASH_ADM_STRONG 1 /* H^2: 2^d-tree, admissible iff well separated (Def. 2.1) */

/* ---- precisions ---- */
#define SMASH_F64 0
#define SMASH_F32 1
#define SMASH_BF16 2 /* apply only: BF16 matrices, FP32 vectors and accumulation */

/* ---- storage of the coupling blocks B_ij (Sec. 1.1: a block is fixed by
 *      its row and column skeleton indices, so it may be stored or
 *      re-evaluated) ---- */
#define SMASH_COUPLING_AUTO 0      /* stored when they take at most 3/4 of the free
                                      device memory at build time, else evaluated */
#define SMASH_COUPLING_STORED 1    /* evaluated once by the build and kept */
#define SMASH_COUPLING_EVALUATED 2 /* evaluated by every product, a bounded chunk
                                      of pairs at a time, right before its
                                      contraction; nothing O(sum k_i k_j) is kept */

typedef struct smash_handle_s *smash_handle;

/* Options.  Initialise with smash_default_options(); a NULL options pointer
 * means the defaults.
 *   tau          separation ratio of Def. 2.1; default 0.6 for dim 1, else 0.7
 *   eps_svd      HSS near-field SVD relative truncation (eq. (3.8)); < 0: = tol
 *   srrqr_f      Gu-Eisenstat bound f = s of Thm. 2.4; default 2
 *   diag_value   d_x of eq. (2.1) for singular kernels; default 0
 *   eval_prec    precision of the stored coupling / near-field blocks
 *   apply_prec   precision of the product: SMASH_F64 or SMASH_F32 (G copies,
 *                blocks and vectors of that type), or SMASH_BF16 (G copies and
 *                blocks stored in BF16 and multiplied on the BF16 matrix cores
 *                with FP32 accumulation; vectors FP32).  The construction
 *                itself (basis, near-field SVD, RRQR) is FP64 in every case.
 *   has_root_box root box [root_lo, root_lo + root_side]^dim instead of the
 *                bounding cube of X and Y (points outside: SMASH_E_INVALID_ARG)
 *   max_depth    > 0 caps the number of tree levels (root = level 1)
 *   batched      1: all nodes of a level in one launch per phase (default);
 *                0: one launch per node (the plain per-node form)
 *   timing       1: bracket every phase's launches with HIP events on the
 *                stream they run on; smash_info reports the summed times
 *   mv_split_nodes  launch shape of the product sweeps: a tree level with at
 *                most this many nodes runs each node on four wavefronts
 *                (long grids, few nodes), a larger one on one wavefront per
 *                node; default 1024, 0 never splits
 *   mv_xcd_run   launch shape of the coupling and near products: workgroups
 *                go to the 8 XCDs in runs of this many consecutive nodes
 *                (tree-order neighbours share an L2); default 16, in [1, 4096]
 *   graphs       1 (default): smash_matvec captures its launch sequence into a
 *                HIP graph on the second call with the same (X, ldx, nrhs, Y,
 *                ldy) and replays it from then on (the eight most recent
 *                argument sets are kept; not with timing); 0: always eager
 *   coupling_mode SMASH_COUPLING_* (default AUTO).  Both forms give the same
 *                product bit for bit (the same block values enter the same
 *                contraction); EVALUATED trades memory for product time
 *   coupling_chunk  block entries per chunk of the evaluated form (the
 *                workspace holds one chunk plus at most one node's blocks);
 *                0 (default): 256 MiB worth of the apply precision
 */
/* Device allocator hooks (smash_options.alloc, .free, .alloc_ctx): when both
 * are set, every device allocation of the handle -- its build temporaries,
 * its arrays and its product workspaces -- comes from
 * alloc(ctx, bytes, stream) and goes back through
 * free(ctx, ptr, bytes, stream), with the stream it was allocated for, once
 * no queued work uses it (temporaries at the end of the build, the rest in
 * smash_destroy).  For a caller whose own allocator (e.g. torch's caching
 * allocator) should hold one device-memory budget.  alloc returns device
 * memory aligned to at least 256 bytes, or NULL (the call then fails with
 * SMASH_E_OOM); the hooks are called on the calling host thread and must not
 * call back into the library; ctx must outlive the handle.  The temporary
 * copy buffer of smash_export uses the device allocator directly. */
typedef void *(*smash_alloc_fn)(void *ctx, size_t bytes, void *stream);
typedef void (*smash_free_fn)(void *ctx, void *ptr, size_t bytes, void *stream);

typedef struct smash_options {
  uint32_t struct_size; /* sizeof(smash_options) */
  double tau;
  double eps_svd;
  double srrqr_f;
  double diag_value;
  int32_t eval_prec;
  int32_t apply_prec;
  int32_t has_root_box;
  double root_lo[3];
  double root_side;
  int32_t max_depth;
  int32_t batched;
  int32_t timing;
  int32_t mv_split_nodes;
  int32_t graphs;
  int32_t mv_xcd_run;
  int32_t coupling_mode;
  int64_t coupling_chunk;
  smash_alloc_fn alloc; /* both NULL (default): the library's own pool */
  smash_free_fn free;
  void *alloc_ctx;
  /* SMASH_KERNEL_DOUBLE_LAYER: device, n x 3 FP64 row-major in the points'
   * order, per point (m_1, m_2, diagonal value); borrowed like the points.
   * NULL for every other kernel. */
  const double *point_data;
  /* far-field basis: SMASH_BASIS_CHEBYSHEV (default), the interpolation
   * basis (2.2) on interp_order Chebyshev points per axis; or
   * SMASH_BASIS_TAYLOR (dim 1 only, not the double-layer kernel), the
   * Taylor basis (2.4)-(2.5) with r = interp_order terms, scaled by the box's
   * center and half width (Def. 2.1). */
  int32_t basis;
} smash_options;

#define SMASH_BASIS_CHEBYSHEV 0
#define SMASH_BASIS_TAYLOR 1

int smash_default_options(smash_options *opt);

/* Construction (Sec. 3.1 partition, Sec. 3.3.1 HSS or Sec. 3.3.2 H^2
 * level-wise compression, eqs. (3.15), (3.19), (3.20) blocks), with Y = X.
 *   points        device, n x dim FP64
 *   kernel_id     SMASH_KERNEL_*
 *   leaf_size     nu_0: a box holding more than nu_0 points of X or Y is bisected
 *   interp_order  p: Chebyshev points per axis of the interpolation basis (2.2)
 *   admissibility SMASH_ADM_WEAK or SMASH_ADM_STRONG
 *   tol           relative rank tolerance of the strong RRQR (Thm. 2.4)
 *   out           receives the handle (NULL on failure)
 * Synchronises `stream` a few times (level sizes, list lengths); the handle
 * is ready when the call returns. */
int smash_build(const double *points, int64_t n, int32_t dim, int32_t kernel_id,
                int32_t leaf_size, int32_t interp_order, int32_t admissibility, double tol,
                const smash_options *opt, void *stream, smash_handle *out);

/* Same with distinct X (nx x dim) and Y (ny x dim), both device FP64. */
int smash_build_xy(const double *x, int64_t nx, const double *y, int64_t ny, int32_t dim,
                   int32_t kernel_id, int32_t leaf_size, int32_t interp_order,
                   int32_t admissibility, double tol, const smash_options *opt, void *stream,
                   smash_handle *out);

/* Product Y = A-hat X (Sec. 3.4) in the ORIGINAL point order.
 *   X  device, ny x nrhs, leading dimension ldx (>= nrhs)
 *   Y  device, nx x nrhs, leading dimension ldy (>= nrhs); fully overwritten
 *   dtype  type of X and Y: SMASH_F64 for an FP64-apply handle, SMASH_F32 for
 *          an FP32- or BF16-apply handle
 * Asynchronous on `stream`; workspaces are owned by the handle.  Products of
 * one handle are ordered by the library: one enqueued on another stream than
 * the handle's previous product waits (on the device) for that product. */
int smash_matvec(smash_handle h, const void *X, int64_t ldx, int32_t nrhs, int32_t dtype,
                 void *Y, int64_t ldy, void *stream);

/* Product with a Cauchy-like matrix (Sec. 6.3, eqs. (6.1)-(6.2)):
 * a_ij = kappa(x_i, y_j) sum_l w_il v_jl, i.e. A = sum_l diag(w_l) C diag(v_l)
 * with C = [kappa(x_i, y_j)] the handle's matrix (for SMASH_KERNEL_CAUCHY the
 * Cauchy matrix, which makes A the Cauchy-like matrix of (6.1)).  Computes
 * Y = sum_l w_l o (C-hat (v_l o X)) with C-hat the handle's approximation:
 * the HSS/H^2 generators of each term are the handle's with U, D and V scaled
 * by the generator columns, and their sum is the merged representation of
 * A-hat, applied here as one product with the p * nrhs columns v_l o X side
 * by side, followed by the weighted sum over l (in the order l = 0, 1, ...).
 *   X, Y, ldx, ldy, nrhs, dtype  as smash_matvec
 *   w  device FP64, nx x p, row-major (w[i * p + l]): the row generators
 *   v  device FP64, ny x p, row-major: the column generators
 *   p  generator columns, 1 <= p <= SMASH_CAUCHY_LIKE_MAX_P
 * Takes 8 (FP64 apply) or 4 bytes x p x nrhs x (nx + ny) of device memory for
 * the stacked vectors while it runs (through the handle's allocator hooks if
 * set), given back stream-ordered.  Asynchronous on `stream`, ordered with
 * the handle's other products as smash_matvec is.
 * Errors: as smash_matvec; SMASH_E_INVALID_ARG for a NULL w or v or p out of
 * range; SMASH_E_OOM when the stacked vectors cannot be allocated. */
#define SMASH_CAUCHY_LIKE_MAX_P 16
int smash_matvec_cauchy_like(smash_handle h, const void *X, int64_t ldx, int32_t nrhs,
                             int32_t dtype, const double *w, const double *v, int32_t p,
                             void *Y, int64_t ldy, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * product as smash_matvec, same arguments and results, but it allocates
 * nothing.  The product's slot-space vectors (q and z, the only device
 * memory it needs beyond the handle, X and Y) come from one library-owned
 * array of SMASH_NOALLOC_SCRATCH_BYTES per device, held by every device the
 * library runs on until the process ends; the right-hand sides are taken in
 * passes of 64, 48, 32 or 16 columns, the widest whose vectors fit.  Always
 * eager launches (no graph capture, no phase timers).
 * The array is shared by every such call on the device and keeps the last
 * call's contents: calls that overlap on one device (on different streams or
 * host threads, without ordering between them) race and give wrong results.
 * Unlike smash_matvec, no ordering with the handle's other products is
 * added (no event is recorded or waited for, so the call can be captured
 * into a caller's graph): order them on the caller's streams.
 * Errors: as smash_matvec; SMASH_E_INVALID_ARG, naming the sizes, when the
 * handle's vectors for 16 columns exceed the array (row slots + column slots
 * times 16 times 8 bytes for FP64 apply, 4 bytes otherwise);
 * SMASH_E_DEVICE when the array's device address cannot be obtained. */
#define SMASH_NOALLOC_SCRATCH_BYTES ((int64_t)64 << 20)
int smash_matvec_noalloc(smash_handle h, const void *X, int64_t ldx, int32_t nrhs,
                         int32_t dtype, void *Y, int64_t ldy, void *stream);

/* Products of several handles in one call (Sec. 3.4 for each): Ys[c] =
 * A-hat_c Xs[c] for c < count, enqueued on `stream` in order, each exactly as
 * smash_matvec would (a captured-graph replay once its argument set repeats).
 * For a serving loop that serves several resident matrices at once: one call
 * and one validation pass for all of them.
 *   hs, Xs, ldx, nrhs, Ys, ldy   host arrays of `count` entries with the
 *                meaning of smash_matvec's arguments; a handle may repeat
 *                (its products then run one after the other)
 *   dtype        for every entry
 * Every entry is validated before anything is enqueued: on an invalid one
 * nothing runs and the message names its index.  count == 0 does nothing.
 * Errors: SMASH_E_INVALID_ARG (count < 0, a NULL array, or an entry that
 * smash_matvec would reject), then as smash_matvec. */
int smash_matvec_batched(int32_t count, const smash_handle *hs, const void *const *Xs,
                         const int64_t *ldx, const int32_t *nrhs, void *const *Ys,
                         const int64_t *ldy, int32_t dtype, void *stream);

/* Launch shape of the products of an existing handle (the options
 * mv_split_nodes and mv_xcd_run), as an autotuner sets it between timed
 * products.  The numbers are unchanged up to the summation order of the
 * split sweeps.  Drops captured graphs (waits for their last launches).
 * Errors: SMASH_E_INVALID_ARG for a NULL handle or out-of-range values. */
int smash_set_product_shape(smash_handle h, int32_t mv_split_nodes, int32_t mv_xcd_run);

/* Sizes and statistics of a construction (host struct). */
typedef struct smash_info_t {
  int64_t nx, ny;
  int32_t dim, nlevels;
  int64_t nnodes, nleaves;
  int64_t n_admissible;   /* |L|   */
  int64_t n_inadmissible; /* |L^-| */
  int64_t sum_rank_row, sum_rank_col; /* sum over nodes of |i-hat| */
  int32_t max_rank_row, max_rank_col;
  int64_t coupling_entries; /* sum over L of k_i k_j     */
  int64_t near_entries;     /* sum over L^- of |i| |j|   */
  int64_t g_entries_row, g_entries_col; /* sum (|i-bar| - k) k */
  int64_t index_entries;    /* stored int32 index entries */
  int64_t device_bytes;     /* bytes held by the handle   */
  int64_t total_swaps;      /* Gu-Eisenstat swaps performed */
  int32_t apply_prec, eval_prec;
  int32_t symmetric_reuse;  /* column side taken from the row side */
  double build_ms;          /* wall time of the last build on its stream */
  /* with options.timing: device time (ms) and launch groups per phase,
   * summed over the build and every product so far (SMASH_PHASE_*) */
  double phase_ms[16];
  int64_t phase_calls[16];
  int64_t graph_captures, graph_replays; /* products captured / replayed as graphs */
  int32_t coupling_evaluated; /* 1: coupling blocks are evaluated inside each product */
  int32_t coupling_chunks;    /* chunks of pairs per product in that case */
  int64_t coupling_ws_entries; /* entries of the chunk workspace in that case
                                  (0 when the evaluation is fused into the
                                  contraction: FP64 and FP32 apply) */
  /* Storage comparison in the manner of Sec. 6.6 (Table 6.6), in bytes with
   * every value in FP64 and every index in int32:
   *   bytes_dense  the dense matrix, 8 nx ny;
   *   bytes_hss0   generators stored as dense matrices: U_i (and V_i when the
   *                column side is not the row side) as |i-bar| x k_i per
   *                node, every B_ij over L, every near block over L^-;
   *   bytes_smash  the storage of Sec. 2.3 (end): per node G_i and the index
   *                lists of its grid (sel), the pair lists, and the near
   *                blocks; a coupling block is fixed by its skeleton index
   *                sets, so no B_ij is stored. */
  int64_t bytes_dense, bytes_hss0, bytes_smash;
  /* Device bytes the construction held at its peak: the handle's arrays
   * plus every temporary of the build (chunks of the library's pool, or of
   * the allocator hooks).  A caller that admits constructions by memory
   * reserves this much while one runs, and device_bytes once it is done. */
  int64_t build_peak_bytes;
} smash_info_t;

#define SMASH_PHASE_TREE 0
#define SMASH_PHASE_PAIRS 1
#define SMASH_PHASE_NEAR_SVD 2
#define SMASH_PHASE_COMPR 3
#define SMASH_PHASE_SLOTS 4
#define SMASH_PHASE_BLOCKS 5
#define SMASH_PHASE_MV_GATHER 6
#define SMASH_PHASE_MV_UP 7
#define SMASH_PHASE_MV_COUPLING 8
#define SMASH_PHASE_MV_DOWN 9
#define SMASH_PHASE_MV_NEAR_OUT 10

int smash_info(smash_handle h, smash_info_t *info);

/* Copy parts of the construction to host memory for inspection.  With
 * host_buf == NULL, *count receives the number of elements and nothing is
 * copied; otherwise *count must hold the buffer capacity in elements.
 * Element type is int32 unless stated. */
#define SMASH_EX_PERM_X 1   /* nx: original index of each permuted X point */
#define SMASH_EX_PERM_Y 2
#define SMASH_EX_NODES 3    /* nnodes x 8: level, parent, first_child (-1), nchild, xb, xe, yb, ye */
#define SMASH_EX_BOXES 4    /* nnodes x 6 FP64: lo[3], hi[3] */
#define SMASH_EX_L 5        /* |L| x 2 (i, j) sorted */
#define SMASH_EX_LM 6       /* |L^-| x 2 sorted */
#define SMASH_EX_NEAR_PTR 7 /* HSS: nnodes+1 CSR pointer of N_i (eq. (A.1)) */
#define SMASH_EX_NEAR_IDX 8
#define SMASH_EX_RANKS 9    /* nnodes x 6: m_row, k_row, m_col, k_col, ks_row, ks_col */
#define SMASH_EX_ROW_SEL 10 /* per non-root node, m entries: skeleton positions asc, then the rest asc */
#define SMASH_EX_ROW_G 11   /* FP64, per non-root node (m-k) x k */
#define SMASH_EX_COL_SEL 12
#define SMASH_EX_COL_G 13
#define SMASH_EX_ROW_GRID 14 /* per non-root node, m permuted point ids */
#define SMASH_EX_COL_GRID 15
#define SMASH_EX_SIZES 16    /* nx, ny, nnodes, nlevels, |L|, |L^-|, dim, admissibility */
#define SMASH_EX_LEVELS 17   /* nlevels+1: first node of each level, then nnodes */
#define SMASH_EX_COUPLING 18 /* entries of all B_ij over L in pair order, each block  */
                             /* column-major (row index fastest), F64 or F32 per the */
                             /* apply precision; a BF16 handle: SMASH_E_UNSUPPORTED  */
#define SMASH_EX_NEAR 19     /* the same for the near blocks over L^-                */

/* Copy parts of the construction to host memory for inspection (parity
 * tests, debugging).
 *   what      SMASH_EX_*
 *   host_buf  host memory, or NULL to query the size
 *   count     with host_buf == NULL receives the number of ELEMENTS of the
 *             export (not bytes; the element type is given per SMASH_EX_*);
 *             otherwise holds the buffer capacity in elements on entry
 * Synchronises the device.  Errors: SMASH_E_INVALID_ARG (NULL handle or
 * count, unknown `what`, capacity too small), SMASH_E_UNSUPPORTED (an export
 * that the handle does not hold, e.g. SMASH_EX_COUPLING of a BF16 or
 * evaluated-coupling handle), SMASH_E_DEVICE. */
int smash_export(smash_handle h, int32_t what, void *host_buf, int64_t *count);

/* Admission model for a serving loop: an upper estimate of the device
 * bytes a handle built with these parameters holds (points, tree, lists,
 * G copies, coupling and near blocks, a 64-column product workspace), from
 * the point count alone.  The block counts assume every node carries the
 * full basis rank min(order^dim, leaf) and the interaction-list sizes of
 * uniform boxes (H^2: (2*3)^dim - 3^dim far pairs and 3^dim near pairs per
 * node for tau <= 0.7; HSS: one of each), so real footprints are lower
 * (2-5x on the workloads measured); a caller may scale it by the ratio it
 * observes.  Host-only arithmetic: no device is touched.
 *   apply_prec  SMASH_F64, SMASH_F32 or SMASH_BF16
 * Errors: SMASH_E_INVALID_ARG for out-of-range parameters or a NULL bytes. */
int smash_estimate_footprint(int64_t n, int32_t dim, int32_t kernel_id, int32_t leaf_size,
                             int32_t interp_order, int32_t admissibility, double tol,
                             int32_t apply_prec, int64_t *bytes);

/* The same for a coupling storage form (SMASH_COUPLING_*; AUTO is estimated
 * as STORED, the larger): with SMASH_COUPLING_EVALUATED the coupling blocks
 * are replaced by the product's chunk workspace (at most 256 MiB plus one
 * node's blocks).  For a serving loop that falls back to the evaluated form
 * when the stored one does not fit.
 * Errors: as smash_estimate_footprint, and SMASH_E_INVALID_ARG for an
 * unknown coupling_mode. */
int smash_estimate_footprint_mode(int64_t n, int32_t dim, int32_t kernel_id, int32_t leaf_size,
                                  int32_t interp_order, int32_t admissibility, double tol,
                                  int32_t apply_prec, int32_t coupling_mode, int64_t *bytes);

/* Returns the library's cached device memory to the device: the idle chunks
 * that constructions keep for the next one, and the free part of the
 * device's default memory pool (which the library keeps from shrinking
 * between constructions).  For a caller about to allocate through another
 * allocator, e.g. a serving loop that moves handles onto torch's caching
 * allocator after stand-alone constructions.  Handles keep their memory.
 *   device  the device to trim; < 0: the calling thread's current device
 * Synchronises that device.  Errors: SMASH_E_DEVICE. */
int smash_trim(int32_t device);

int smash_destroy(smash_handle h);

/* Thread-local description of the last failure on this thread. */
const char *smash_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SMASH_H */
