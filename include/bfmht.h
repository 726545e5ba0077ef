/*
 * bfmht.h -- C ABI of the MI355X (gfx950) butterfly manifold harmonic transform.
 *
 * The transform is the matrix form of the manifold harmonic transform,
 * f = Phi c with Phi[j, k] = phi_k(x_j) (Sec. 1, eq. MHT-sum), and its adjoint,
 * which maps point values back to coefficients; Phi is real, so the adjoint is
 * Phi^T (Sec. 1, the adjoint transform).  Phi is given as a row-wise butterfly
 * factor set built on the host (Sec. 2, Alg. "Butterfly factorization" and the
 * set it returns: a basis per frequency leaf, a transfer block per block pair at
 * levels 1..L, a column basis per space leaf).  The factors are computed in
 * FP64, on the host or with the batched device calls near the end of this
 * file; the apply calls upload and apply them.
 *
 * Conventions
 *  - Both trees are complete binary trees of depth L (or 4-ary, see arity
 *    below).  At level l (0..L) space node i sits at depth l and frequency node
 *    j at depth L-l; the block id is q = i * 2^(L-l) + j ("space-major").  The
 *    two inputs of block (l, i, j) are blocks (l-1, i>>1, 2j) and (l-1, i>>1, 2j+1).
 *  - Column bases are submatrices of Phi (column interpolative decompositions),
 *    so a block (l, i, j) computes y_lij = P_lij [y_{l-1,i>>1,2j}; y_{l-1,i>>1,2j+1}],
 *    level 0 computes y_0j = P_0j c[koff[j] : koff[j+1]], and the last stage
 *    writes f[perm_x[xoff[i] + t]] = (U_i y_Li)[t].
 *  - Dense right-hand-side blocks are row-major: row r, column (RHS) s at
 *    ptr[r * ld + s], ld >= nrhs.  Rows are points (f) or modes (c).  A block
 *    with no rows (n = 0 or m = 0) is never read or written: it may be NULL
 *    and its ld is not checked.
 *  - All device pointers are caller-owned (PyTorch allocates them).  The plan
 *    owns host metadata only and refers to device memory inside the buffer
 *    given to bfmht_plan_upload.
 *  - Every call that takes a stream is asynchronous on that stream (a
 *    hipStream_t passed as void*; NULL = the default stream) and never
 *    synchronises, except bfmht_plan_upload, which synchronises its stream
 *    once before freeing its host staging copy.
 *  - Errors: every call returns a status; bfmht_last_error() gives a message
 *    for the calling thread.  No exception crosses the ABI.  nrhs == 0 is a
 *    no-op that returns BFMHT_OK.
 */
#ifndef BFMHT_H
#define BFMHT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bfmht_plan bfmht_plan;

/* Arithmetic of the apply.  F64: factors, level vectors and I/O in double
 * (the plain baseline).  F32: factors and vectors in float, FP32 MFMA with
 * FP32 accumulation.  F64 and F32 applies with at most 4 right-hand sides use
 * vector FMAs instead of MFMA tiles (same jobs, same sums per output up to the
 * order of the reduction).  BF16X2 / BF16X3: factors stored in FP32 and split
 * into 2 / 3 bfloat16 terms as they are loaded (hi = bf16(x), lo = bf16(x - hi),
 * lo2 = bf16(x - hi - lo), round to nearest even; 4 bytes per entry streamed),
 * activations split the same way per tile, BF16 MFMA
 * products hi*hi + hi*lo + lo*hi (X2) or the six products whose term indices
 * sum to at most 2 (X3), FP32 accumulation, FP32 level vectors and I/O. */
typedef enum {
  BFMHT_F64 = 0,
  BFMHT_F32 = 1,
  BFMHT_BF16X2 = 2,
  BFMHT_BF16X3 = 3
} bfmht_precision;

typedef enum {
  BFMHT_OK = 0,
  BFMHT_EINVAL = 1,   /* bad argument: null pointer, size, ld, inconsistent factors */
  BFMHT_ESTATE = 2,   /* call out of order, e.g. apply before upload */
  BFMHT_ENOSPACE = 3, /* device buffer or workspace smaller than required */
  BFMHT_EHIP = 4      /* a HIP runtime call failed */
} bfmht_status;

/* Host FP64 factor set (Sec. 2, the factor set returned by the factorization).
 * Caller-owned; read only during bfmht_plan_create, which copies what it needs.
 *  n, m      number of points (rows of Phi) and modes (columns), m, n >= 0
 *  L         tree depth, arity^L <= 2^24
 *  arity     children per tree node: 2 (binary trees), 4 (a quadtree in space
 *            with a 4-ary frequency tree, Sec. 2's k-ary generalization, the
 *            trees of Sec. 5's analysis), or 0 for 2; below, 2^ reads arity^ and
 *            a block's inputs are the arity consecutive blocks
 *            (l-1, i / arity, arity j + t), t < arity
 *  perm_x    [n]      tree position -> original point index (a permutation)
 *  xoff      [2^L+1]  space-leaf offsets into tree positions, xoff[0] = 0, xoff[2^L] = n
 *  koff      [2^L+1]  frequency-leaf offsets into columns (eigenvalue order), koff[2^L] = m
 *  rank      [(L+1) * 2^L]  r_{l,q} at rank[l * 2^L + q]
 *  ident     [(L+1) * 2^L]  1 where P_{l,q} is the identity (then r_{l,q} equals its
 *                           input row count and nothing is stored)
 *  P, P_off  P_{l,q} is rank x r_in, row-major, at P + P_off[l * 2^L + q]
 *            (r_in = koff[j+1]-koff[j] at level 0, else the two input ranks summed);
 *            P_off is ignored for identity blocks
 *  P_len     number of doubles readable at P (bounds check of P_off)
 *  U, U_off  U_i is (xoff[i+1]-xoff[i]) x rank[L * 2^L + i], row-major, at U + U_off[i]
 *  U_len     number of doubles readable at U */
typedef struct {
  int64_t n, m;
  int32_t L;
  int32_t arity;
  const int32_t *perm_x;
  const int64_t *xoff;
  const int64_t *koff;
  const int32_t *rank;
  const uint8_t *ident;
  const double *P;
  const int64_t *P_off;
  int64_t P_len;
  const double *U;
  const int64_t *U_off;
  int64_t U_len;
} bfmht_factors_host;

/* Validate the factor set (the bases, transfer blocks and leaf bases that
 * Alg. "Butterfly factorization" of Sec. 2 returns) and build the device
 * layout for one precision.
 * On success *plan owns host metadata (stage tables, converted factors staged
 * for upload); on failure *plan is set to NULL.  max_nrhs >= 1 records the
 * largest nrhs the caller means to use; it sizes nothing (workspace is per
 * call), and applies with more columns are accepted. */
bfmht_status bfmht_plan_create(const bfmht_factors_host *factors, bfmht_precision prec,
                               int32_t max_nrhs, bfmht_plan **plan);

/* Plan flags of bfmht_plan_create_ex. */
#define BFMHT_PLAN_FULL_BLOCKS 1 /* store every ID block as the full P (no compact form, no merged leaf blocks) */
#define BFMHT_PLAN_LEAF_STAGE 2  /* keep the leaf bases as a stage of their own (no merged leaf blocks) */

/* bfmht_plan_create with flags (0 = the default of bfmht_plan_create).  By
 * default a transfer or level-0 block whose P has the column-ID structure
 * P = [I T] Pi^T (Sec. 2: the skeleton columns of an interpolative
 * decomposition, each exactly a unit vector) is applied in compact form in the
 * forward direction: only T is stored and the skeleton rows are added, which
 * saves the identity part's bytes and flops; results agree with the full form
 * up to rounding.  BFMHT_PLAN_FULL_BLOCKS keeps the full P.
 * By default the leaf bases are also merged into the last transfer level
 * (Sec. 2: f_i = U_i y_{L,i} with y_{L,i} = P_{L,i} x, so the two products are
 * one with the block U_i P_{L,i}, formed once in FP64 on the host here, by up
 * to 16 threads that the call starts and joins) when
 * L >= 1, the last level is not all identities, and the merged blocks hold at
 * most 1/32 more entries than U_i and the stored P_{L,i} together (the case
 * when the last level's ranks equal the leaf sizes).  A merged plan has one
 * stage fewer per direction; its results agree with the separate stages up to
 * rounding.  BFMHT_PLAN_LEAF_STAGE keeps the separate leaf stage.  EINVAL on
 * unknown flags; otherwise as bfmht_plan_create. */
bfmht_status bfmht_plan_create_ex(const bfmht_factors_host *factors, bfmht_precision prec, int32_t max_nrhs,
                                  int32_t flags, bfmht_plan **plan);

/* Factor entries one apply reads (storage and apply cost coincide: every
 * stored block is applied once per vector, Sec. 6.2): transpose = 0 for the
 * forward direction, 1 for the transposed direction.  Compact blocks count T
 * only, merged leaf blocks n_i K_i; -1 if plan is NULL. */
int64_t bfmht_plan_stored_entries(const bfmht_plan *plan, int32_t transpose);

/* Bytes of device memory the plan needs for its factors (the Sec. 2 factor
 * set in the plan's precision) and tables. */
int64_t bfmht_plan_device_bytes(const bfmht_plan *plan);

/* Bytes of workspace one apply or apply_transpose with this nrhs needs: two
 * ping-pong level buffers for the level vectors y_l of the Sec. 2 recursion
 * (each level's products of V*, the transfer blocks R*, then U), each large enough for the longest level vector and
 * for f's n rows (apply_transpose first gathers f into tree order there);
 * -1 on a bad argument. */
int64_t bfmht_workspace_bytes(const bfmht_plan *plan, int32_t nrhs);

/* The factor upload: copy the plan's factors (the Sec. 2 factor set) and tables into dev_buf (device memory, at least
 * bfmht_plan_device_bytes bytes, 256-byte aligned), on `stream`; synchronises
 * that stream, then frees the host staging copy.  The plan keeps dev_buf's
 * address; the caller keeps dev_buf alive until bfmht_plan_destroy.  A plan is
 * uploaded once; ESTATE on a second upload. */
bfmht_status bfmht_plan_upload(bfmht_plan *plan, void *dev_buf, int64_t dev_bytes, void *stream);

/* Synthesis f = Phi~ c (Sec. 1, eq. MHT-sum: point values from expansion
 * coefficients), applied as the factored product of Sec. 2: level-0 bases,
 * transfer levels 1..L, leaf bases.  c: device, m x nrhs (ld ldc); f: device, n x nrhs
 * (ld ldf), fully overwritten.  Element type double for F64, float otherwise.
 * ws: device workspace of at least bfmht_workspace_bytes(plan, nrhs) bytes,
 * 256-byte aligned.  c and f must not overlap ws or each other. */
bfmht_status bfmht_apply(const bfmht_plan *plan, const void *c, int64_t ldc, void *f, int64_t ldf,
                         int32_t nrhs, void *ws, int64_t ws_bytes, void *stream);

/* Analysis g = Phi~^T f (Sec. 1: the adjoint maps point values to
 * coefficients; Phi is real): the exact transpose of bfmht_apply's steps, in
 * reverse order.  f: device n x nrhs (ld ldf); g: device m x nrhs (ld ldg),
 * fully overwritten.  Same workspace rule as bfmht_apply. */
bfmht_status bfmht_apply_transpose(const bfmht_plan *plan, const void *f, int64_t ldf, void *g,
                                   int64_t ldg, int32_t nrhs, void *ws, int64_t ws_bytes,
                                   void *stream);

/* Scaled synthesis f = Phi~ diag(s) c (Sec. 7.2, Gaussian random fields: the
 * truncated Karhunen-Loeve expansion, eq. KL-expansion, y = Phi S^(1/2) z is this call with
 * s = S^(1/2) and c = z).  s: device, m elements, same element type as c.
 * Otherwise as bfmht_apply; diag(s) c is formed in the workspace, c is left
 * unchanged.  EINVAL if s is NULL (and m > 0). */
bfmht_status bfmht_apply_scaled(const bfmht_plan *plan, const void *s, const void *c, int64_t ldc, void *f,
                                int64_t ldf, int32_t nrhs, void *ws, int64_t ws_bytes, void *stream);

/* Scaled analysis g = diag(s) Phi~^T f.  With s the spectral density S on the
 * eigenvalues, bfmht_apply(bfmht_apply_transpose_scaled(f)) is the covariance
 * matrix-vector product Phi S Phi^T f of the truncated kernel expansion
 * (Sec. 7.2, eq. kernel-representation).  Otherwise as bfmht_apply_transpose.  EINVAL if s is NULL
 * (and m > 0). */
bfmht_status bfmht_apply_transpose_scaled(const bfmht_plan *plan, const void *s, const void *f, int64_t ldf,
                                          void *g, int64_t ldg, int32_t nrhs, void *ws, int64_t ws_bytes,
                                          void *stream);

/* Inverse transform by least squares (Sec. 7.1, eq. inverse-MHT): for every
 * column of f, `iters` steps of LSQR (Paige and Saunders' Golub-Kahan
 * bidiagonalization with plane rotations) on min ||Phi~ x - f||_2, each step
 * one bfmht_apply and one bfmht_apply_transpose plus vector kernels; the whole
 * solve is enqueued on `stream` with no host synchronization.
 * f: device n x nrhs (ld ldf), read only; x: device m x nrhs (ld ldx), the
 * iterate after `iters` steps (zero for iters = 0); rnorm: device nrhs
 * elements (or NULL), LSQR's estimate of ||Phi~ x - f||_2 per column after the
 * last step.  Element type as bfmht_apply.  ws: device workspace of at least
 * bfmht_lsqr_workspace_bytes(plan, nrhs) bytes, 256-byte aligned, not
 * overlapping f, x or rnorm.  EINVAL on bad arguments or iters < 0, ESTATE if
 * not uploaded, ENOSPACE if ws is too small.  A column whose residual or
 * projected residual vanishes keeps its iterate and its residual estimate
 * from then on (the estimate stays ||f|| when Phi~^T f = 0). */
bfmht_status bfmht_lsqr(const bfmht_plan *plan, const void *f, int64_t ldf, void *x, int64_t ldx, int32_t nrhs,
                        int32_t iters, void *rnorm, void *ws, int64_t ws_bytes, void *stream);
int64_t bfmht_lsqr_workspace_bytes(const bfmht_plan *plan, int32_t nrhs);

/* Number of stages of one apply (the levels of the Sec. 2 recursion): L + 2 (level 0, the L transfer levels, the
 * leaf stage), or L + 1 when the leaf bases are merged into the last transfer
 * level (see bfmht_plan_create_ex), numbered in forward order; -1 for NULL.  Leading levels whose
 * blocks are all identities are folded into the next stage by single applies
 * (their tile shapes then have no effect). */
int32_t bfmht_plan_num_stages(const bfmht_plan *plan);

/* Tile shape of one stage of the forward (transpose = 0) or transposed
 * (transpose != 0) apply: `rows` output rows (64 or 128) by `cols`
 * right-hand-side columns (16, 32 or 64, or 0 for the smallest of those that
 * covers nrhs) per workgroup.  Default 64 x 0.  Results do not depend on it;
 * it is the knob the autotuner sets.  EINVAL on a bad stage or shape. */
bfmht_status bfmht_plan_set_tile(bfmht_plan *plan, int32_t transpose, int32_t stage, int32_t rows, int32_t cols);
/* The shape set for that stage. */
bfmht_status bfmht_plan_get_tile(const bfmht_plan *plan, int32_t transpose, int32_t stage, int32_t *rows,
                                 int32_t *cols);

/* Workspace bytes of a bfmht_apply_batched call with these plans and RHS
 * counts (count >= 0 plans, all of one precision); -1 on a bad argument. */
int64_t bfmht_batched_workspace_bytes(const bfmht_plan *const *plans, int32_t count, const int32_t *nrhs);

/* Mode bits of bfmht_apply_batched. */
#define BFMHT_BATCH_TRANSPOSE 1           /* transposed applies (else forward) */
#define BFMHT_BATCH_PERSISTENT 2          /* every stage of every instance in one launch */
#define BFMHT_BATCH_WIDTH(w) ((w) << 8)   /* persistent tile width 16, 32 or 64 (0: 32) */

/* Many instances of uneven size (the many right-hand sides and many instances
 * of one call that the apply is used for in practice, e.g. several fields on
 * several meshes).  Instance i applies plans[i] (forward, or transposed with
 * BFMHT_BATCH_TRANSPOSE in mode) to in[i] (rows x nrhs[i], ld ldin[i]) and
 * overwrites out[i] (ld ldout[i]); instances with nrhs[i] == 0 are skipped.
 * All plans must be uploaded and share one precision.
 * Instances that share one plan (the same handle) are applied as one block of
 * columns: their inputs are packed side by side into the workspace and their
 * outputs copied back, so the plan's factors are streamed once for all of them
 * (results as from one apply per instance; a member with at most 4 columns
 * then runs on the MFMA kernel instead of the vector-FMA one).
 * Default: launch k runs the k-th stage of every unit (a shared-plan group or
 * a single instance) at once, one work item per output tile, so the number of
 * launches is the largest stage count in the batch, not the sum over instances
 * (one launch per stage position and kernel shape, each unit with its plan's
 * tile shapes; the per-stage segment tables travel as launch arguments);
 * asynchronous.
 * BFMHT_BATCH_PERSISTENT: one launch of resident workgroups runs every stage of
 * every instance (64-row tiles, BFMHT_BATCH_WIDTH columns, the MFMA kernel for
 * every RHS count); workgroups take work items in stage order from per-XCD
 * ticket queues and wait for the instance's previous stage to finish.  This
 * mode synchronises `stream` once at its end, to read the launch's error word,
 * and returns EHIP if a wait gave up (bounded, seconds).  This mode is
 * currently switched off and returns EINVAL (its GPU run did not finish in
 * time); the per-stage launches are the batched path.
 * ws: device workspace, 256-byte aligned, at least bfmht_batched_workspace_bytes;
 * it holds each unit's level buffers, the packed blocks of shared-plan units
 * (and the persistent launch's tables), so calls that overlap on one workspace
 * race.  No output may overlap an input, another output or ws.  EINVAL on
 * unknown mode bits. */
bfmht_status bfmht_apply_batched(const bfmht_plan *const *plans, int32_t count, const void *const *in,
                                 const int64_t *ldin, void *const *out, const int64_t *ldout, const int32_t *nrhs,
                                 int32_t mode, void *ws, int64_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): bfmht_apply with its
 * workspace taken from a fixed device array that the library holds, so the
 * call takes no workspace argument and allocates nothing.  Every GPU the
 * library runs on holds its own array of BFMHT_NOALLOC_WORKSPACE_BYTES from
 * the first use of the library's device code there until the process ends;
 * its device address is resolved once per device, on this call's first use
 * there (the stream's device; the current device for the NULL stream).
 * Otherwise as bfmht_apply: f = Phi~ c, asynchronous on `stream`, same
 * operands and errors.  ENOSPACE, with nothing launched, when
 * bfmht_workspace_bytes(plan, nrhs) exceeds the array.  All calls on one GPU
 * share its array (the last call's level vectors stay there; no part of it
 * needs clearing), so calls that overlap on one GPU (different streams, or
 * different host threads) race: serialise them. */
#define BFMHT_NOALLOC_WORKSPACE_BYTES (256ll << 20)
bfmht_status bfmht_apply_noalloc(const bfmht_plan *plan, const void *c, int64_t ldc, void *f, int64_t ldf,
                                 int32_t nrhs, void *stream);

/* ---- The factorization on the device (FP64) ----
 * Every block that the butterfly factorization compresses is a submatrix of
 * Phi: with column interpolative decompositions the previous level's column
 * basis restricted to a space node is Phi at the previous skeleton columns
 * (Sec. 2, Alg. "Butterfly factorization"; Sec. 4, the streaming variant that
 * only ever evaluates such blocks).  A level is then a batch of independent
 * tall blocks of uneven size; these calls form such a batch from tables and
 * compute the column ID of every block.  The caller orders the levels.
 *
 * Metadata arguments are HOST arrays, checked on the host and staged into the
 * device workspace ws (at least bfmht_factor_meta_bytes(count, col_off[count])
 * bytes, 256-byte aligned); each call synchronises `stream` once after staging
 * (so the host arrays may be freed on return) and leaves its kernels running
 * asynchronously.  Block b has rows[b] rows and K_b = col_off[b+1] - col_off[b]
 * columns (col_off[0] = 0, nondecreasing) and lives column-major (ld = rows[b])
 * at a + a_off[b], inside a_len doubles.  count == 0 is a no-op.  Blocks must
 * not overlap (not checked). */
int64_t bfmht_factor_meta_bytes(int32_t count, int64_t total_cols);

/* Form the blocks: entry (t, s) of block b is
 *   tab0[ta[g] * ld0 + row0[b] + t] * tab1[tb[g] * ld1 + row0[b] + t],  g = col_off[b] + s.
 * tab0 / tab1: device, w0 / w1 columns of ld0 / ld1 rows (points in tree
 * order).  For the Fourier matrix the two tables hold cos and sin of k x per
 * coordinate (Sec. 1, eq. 2D-DFT); for a dense Phi (Sec. 7's eigenvectors)
 * tab0 = Phi^T in tree order and tab1 one row of ones (tb = 0).
 * EINVAL if a block's rows leave [0, min(ld0, ld1)), a table column index is
 * out of range, or a block leaves a. */
bfmht_status bfmht_form_blocks(int32_t count, const int64_t *row0, const int64_t *rows, const int64_t *col_off,
                               const int32_t *ta, const int32_t *tb, const int64_t *a_off, const double *tab0,
                               int64_t ld0, int64_t w0, const double *tab1, int64_t ld1, int64_t w1, double *a,
                               int64_t a_len, void *ws, int64_t ws_bytes, void *stream);

/* Column IDs of the blocks (Sec. 2: the low-rank factorization of every block,
 * here A ~ A(:, J) P): column-pivoted Householder QR of each block in place (the
 * block is overwritten by R and the reflectors), pivoting on the largest
 * remaining column norm (first column on ties), stopped at the first pivot
 * whose norm is not above tol times the first pivot's.  A block with more than
 * twice as many rows as columns is first reduced to its K x K triangular factor
 * by an unpivoted blocked QR, and the pivoting runs on that triangle (the same
 * pivots and R up to rounding).  Outputs (device):
 * rank[b] = k, the number of columns kept (0 for an all-zero block);
 * piv[col_off[b] + s] = the block column (0 .. K_b-1) at pivot position s, for
 * all K_b positions; J = piv[0 .. k).  EINVAL on tol < 0 or a block wider than
 * local memory holds (about 5000 columns). */
bfmht_status bfmht_column_id(int32_t count, const int64_t *rows, const int64_t *col_off, const int64_t *a_off,
                             double *a, int64_t a_len, double tol, int32_t *rank, int32_t *piv, void *ws,
                             int64_t ws_bytes, void *stream);

/* The interpolation matrices after bfmht_column_id, on the same a and piv:
 * for every block with p_off[b] >= 0, P (rank[b] x K_b, row-major, at
 * p + p_off[b], inside p_len doubles) with P(:, piv[s]) = e_s for s < k and
 * P(:, piv[s]) = column s - k of R11^-1 R12 for s >= k (back substitution on
 * the triangular factor).  rank, p_off: host arrays (rank as bfmht_column_id
 * returned it); blocks with p_off[b] < 0 are skipped (the caller skips blocks
 * that keep every column, whose P is the identity). */
bfmht_status bfmht_id_coefficients(int32_t count, const int64_t *rows, const int64_t *col_off, const int64_t *a_off,
                                   const double *a, int64_t a_len, const int32_t *rank, const int32_t *piv,
                                   const int64_t *p_off, double *p, int64_t p_len, void *ws, int64_t ws_bytes,
                                   void *stream);

/* Free the plan's host memory.  Does not touch device memory.  NULL is a no-op. */
void bfmht_plan_destroy(bfmht_plan *plan);

/* Message describing the last failed call on this thread ("" if none). */
const char *bfmht_last_error(void);

/* Library version string. */
const char *bfmht_version(void);

#ifdef __cplusplus
}
#endif

#endif /* BFMHT_H */
