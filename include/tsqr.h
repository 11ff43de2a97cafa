/*
 * tsqr.h -- C ABI of the MI355X (gfx950) TSQR / CAQR library (libtsqr.so).
 *
 * Method: Demmel, Grigori, Hoemmen, Langou, "Communication-optimal parallel
 * and sequential QR and LU factorizations" (arXiv 0808.2664).
 *   - TSQR: QR of a tall-skinny m x n matrix (m >= n) as a reduction of
 *     stacked R factors over a tree (Sec. 2.1, Eqs. TSQR_binarytree_1..4);
 *     the Q factor is kept as the implicit "tree of Q factors" and never
 *     multiplied out (Sec. 2.1, remark after Eq. TSQR_binarytree_4).
 *   - CAQR: right-looking QR whose panel factorisation is TSQR, followed by
 *     the tree-structured trailing update (Sec. 3 and 3.1).
 *
 * Conventions shared by every entry point
 *   - Matrices are dense, ROW-MAJOR, with an explicit leading dimension
 *     counted in elements (ld >= number of columns).
 *   - Matrix pointers are DEVICE pointers (memory from hipMalloc or a torch
 *     CUDA/HIP tensor) unless the argument says "host".
 *   - `stream` is a hipStream_t passed as a plain pointer (NULL = the null
 *     stream).  Every call is stream-ordered and asynchronous: it enqueues
 *     work and returns; results are valid once the stream reaches that point.
 *   - dtype: TSQR_F32 or TSQR_F64.
 *   - Householder convention: reflectors H = I - tau v v^T with unit topmost
 *     entry (Sec. 5.2); beta = -sign(alpha)*||x|| with sign(0) = +1, tau = 0
 *     when the part below the diagonal is already zero.  diag(R) may
 *     therefore be negative; tsqr_sign_normalize gives diag(R) >= 0.
 *
 * Return codes (LAPACK "info" style)
 *    0                  success
 *   -i                  argument i (1-based) is invalid; nothing was enqueued
 *    TSQR_ERR_HIP       a HIP runtime call failed (tsqr_last_hip_error)
 *    TSQR_ERR_NOMEM     device workspace allocation failed
 *    TSQR_ERR_PLAN      handle / shape mismatch
 *    TSQR_ERR_UNSUPPORTED  n > 64 for TSQR, or an unsupported option
 *    TSQR_ERR_TIMEOUT   (tsqr_check_status only) a bounded wait inside a
 *                       factorisation gave up; its results are invalid
 *    TSQR_ERR_SCRATCH   (tsqr_factor_noalloc only) the problem needs more
 *                       scratch memory than the fixed buffer holds
 * NaN/Inf inputs are not detected; they propagate to the outputs.
 */
#ifndef TSQR_H
#define TSQR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TSQR_F32 0
#define TSQR_F64 1

#define TSQR_SUCCESS 0
#define TSQR_ERR_HIP 1
#define TSQR_ERR_NOMEM 2
#define TSQR_ERR_PLAN 3
#define TSQR_ERR_UNSUPPORTED 4
#define TSQR_ERR_TIMEOUT 5
#define TSQR_ERR_SCRATCH 6

#define TSQR_MAX_N 64

/* Opaque implicit Q (the tree of Q factors). */
typedef struct tsqr_qtree_s* tsqr_qtree;

/* Tree shape.  0 in any field = the library default.
 *   block_rows : rows per block of the chain kernels: 64 (the default and
 *                the only value accepted).  Each block's reflectors carry one
 *                n x n T.
 *   chains     : number of contiguous row ranges reduced independently with
 *                the flat tree of sequential TSQR (Sec. 2.1); their R
 *                factors are then reduced on the tree.  Default:
 *                min(number of blocks, 1024).  chains = number of blocks
 *                gives the plain parallel TSQR of Eqs. TSQR_binarytree_1..4.
 *   arity      : fan-in of the tree over the chain R factors (default 2).
 *   flags      : 0 or any of TSQR_FLAG_TREE_LEVELWISE, TSQR_FLAG_ONE_WAVE,
 *                TSQR_FLAG_SHARED_CUS.
 *                TSQR_FLAG_ONE_WAVE: every chain on the one-wave engine
 *                (chains and tree in one launch) also where the default is
 *                the two-wave chain engine (FP64, more than 32 columns:
 *                two waves split a chain's columns, then the tree in a
 *                second launch); both give the same bits.
 *                TSQR_FLAG_TREE_LEVELWISE: By default a binary tree
 *                whose chains all fit on the device at once is reduced
 *                panel by panel (a node starts on its first 16 columns as
 *                soon as its children have finished theirs); with this flag,
 *                or when the tree is not binary or the chains do not fit,
 *                each node starts when its children are complete.  Both give
 *                the same bits; only the schedule differs (Sec. 2.1: the
 *                tree shape and order are free).
 *                TSQR_FLAG_SHARED_CUS (caqr_factor only; ignored
 *                elsewhere): by default, on a whole MI355X (256 CUs), once
 *                the trailing columns are few (8192 with the FP64 update,
 *                12288 with FP32 products), caqr_factor runs its panel
 *                factorisations on one to four compute units of every XCD
 *                (two chain workgroups of the first panel per unit) and its
 *                trailing updates on the other units, through two CU-masked
 *                streams of its own that it keeps until the process ends;
 *                with this flag both always run on every unit.  Same bits
 *                either way.
 *   max_polls  : in the panel-by-panel tree a wave waits for its children's
 *                progress, polling at most this many times (default 2^22,
 *                far beyond any real wait).  A wave that gives up sets the
 *                library's status word, which tsqr_check_status reports as
 *                TSQR_ERR_TIMEOUT, and finishes with whatever rows are in
 *                memory, so that factorisation's results are invalid while
 *                every kernel still ends.  Small values exist for tests of
 *                that error path.
 * The library reads no environment variable: these fields are the only
 * tuning inputs. */
#define TSQR_FLAG_TREE_LEVELWISE 1
#define TSQR_FLAG_ONE_WAVE 2
#define TSQR_FLAG_SHARED_CUS 4
#define TSQR_FLAGS_ALL (TSQR_FLAG_TREE_LEVELWISE | TSQR_FLAG_ONE_WAVE | TSQR_FLAG_SHARED_CUS)
typedef struct tsqr_opts {
    int32_t block_rows;
    int32_t chains;
    int32_t arity;
    int32_t flags;
    int32_t max_polls;
} tsqr_opts;

/* TSQR factorisation A = QR (Sec. 2.1).
 *   dtype, m, n (m >= n >= 1, n <= 64), A (device, m x n, lda >= n).
 *   A is OVERWRITTEN with the reflectors of the tree's leaves (in place,
 *   like LAPACK xGEQRF); the implicit Q borrows A, so A must stay alive and
 *   unmodified until tsqr_qtree_destroy.
 *   R: device n x n (ldr >= n) receives R (upper triangle; zeros below), or
 *   NULL.  q_out: receives the implicit Q, or NULL: then only R and the leaf
 *   reflectors are produced (the block T factors, tau and the tree's
 *   reflectors are not formed) and the workspace is released at the end of
 *   the stream work.
 *   Argument indices for errors: 1 dtype, 2 m, 3 n, 4 A, 5 lda, 6 R, 7 ldr,
 *   8 opts, 9 q_out. */
int tsqr_factor(int dtype, int64_t m, int64_t n, void* A, int64_t lda, void* R, int64_t ldr,
                const tsqr_opts* opts, tsqr_qtree* q_out, void* stream);

/* R-only TSQR that allocates nothing, for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, harnesses
 * that forbid allocation).  Same arguments, kernels and results (bit for
 * bit) as tsqr_factor with q_out = NULL: A is overwritten with the leaf
 * reflectors, R (device n x n, ldr >= n, required) receives R with zeros
 * below the diagonal.  The factor's scratch memory (the chains' published R
 * factors and the tree's counters) is a fixed device array of
 * tsqr_factor_noalloc_scratch_bytes() bytes (40 MiB) that each device the
 * library runs on holds until the process ends; the call makes no device
 * allocation and no free.  Problems whose scratch exceeds it (more than 1024
 * chains of 64 columns in FP64 with the default tree; the default geometry
 * of every m fits) return TSQR_ERR_SCRATCH before any launch.  Every call on
 * a device shares that device's array: calls that overlap on one device (two
 * streams or two host threads) race and must be serialised by the caller.
 *   Argument indices for errors: 1 dtype, 2 m, 3 n, 4 A, 5 lda, 6 R, 7 ldr,
 *   8 opts. */
int tsqr_factor_noalloc(int dtype, int64_t m, int64_t n, void* A, int64_t lda, void* R, int64_t ldr,
                        const tsqr_opts* opts, void* stream);
/* Size in bytes of tsqr_factor_noalloc's fixed scratch array (per device). */
size_t tsqr_factor_noalloc_scratch_bytes(void);

/* Layout the apply kernels take for k columns of B on this implicit Q
 * (panel `panel` of a CAQR handle, whose trailing updates are Q^T products
 * of the panel's tree; panel = 0 for a TSQR handle).  Host only, no GPU work.
 * Returns 1 for the wide layout (n = 64 and enough workgroups: each wave
 * applies a block's reflectors to a 16-column tile of B over all 64 rows),
 * 0 for the narrow one (each wave owns 16 rows of a block), or -i for an
 * invalid argument i (1 q, 2 panel, 3 k < 1).  Lets tests check which
 * kernels a case exercises. */
int tsqr_apply_layout(tsqr_qtree q, int64_t panel, int64_t k);

/* Waits for the work enqueued on `stream` (hipStreamSynchronize), then reads
 * and clears the status word of the current device: TSQR_ERR_TIMEOUT if a
 * bounded wait of a factorisation on this device gave up since the last
 * call (see tsqr_opts.max_polls; the word is shared by every stream of the
 * device), 0 otherwise, TSQR_ERR_HIP if the synchronisation or the read
 * failed.  Factorisations do not synchronise by themselves, so a caller that
 * needs the guarantee calls this after them. */
int tsqr_check_status(void* stream);

/* TSQR of a batch of `batch` independent m x n matrices (m >= n >= 1,
 * n <= 64) stored one after another: member b is rows b*m .. b*m + m - 1 of
 * the (batch*m) x n row-major array A (a contiguous [batch][m][n] tensor
 * when lda = n).  Each member is reduced on its own tree (Sec. 2.1; the
 * batch is a forest): its rows are cut into the same number of chains, a
 * power of the arity (opts.chains = chains per member; 0 picks about one
 * chain per SIMD over the whole batch), and its R is the root of its tree.
 *   A is OVERWRITTEN with the leaf reflectors and borrowed by the implicit Q
 *   as for tsqr_factor.  R: device, member b's n x n factor at R + b*strideR
 *   (ldr >= n, strideR >= n*ldr when batch > 1), or NULL.  q_out: the
 *   batch's implicit Q, or NULL (R only).  tsqr_apply_qt, tsqr_apply_q and
 *   tsqr_form_q then act on the stacked (batch*m) x k array, every member
 *   with its own Q (form_q writes each member's thin Q in its rows).
 *   1 <= batch <= 65535.  TSQR_ERR_UNSUPPORTED if opts.chains is not a power
 *   of the arity or the members are too short for that many chains.
 *   Argument indices for errors: 1 dtype, 2 batch, 3 m, 4 n, 5 A, 6 lda,
 *   8 ldr, 9 strideR, 10 opts, 11 q_out. */
int tsqr_factor_batched(int dtype, int64_t batch, int64_t m, int64_t n, void* A, int64_t lda, void* R, int64_t ldr,
                        int64_t strideR, const tsqr_opts* opts, tsqr_qtree* q_out, void* stream);

/* Members of an implicit Q: 1 for tsqr_factor and caqr_factor, `batch` for
 * tsqr_factor_batched.  members: host int64.  Errors: 1 q, 2 members. */
int tsqr_qtree_members(tsqr_qtree q, int64_t* members);

/* Batched tsqr_sign_normalize: member b's R (at R + b*strideR) and the m
 * rows of Q starting at row b*m (Q: the stacked (batch*m) x n array, or
 * NULL) are scaled by D_b = sign(diag R_b), sign(0) = +1.
 * Errors: 1 dtype, 2 batch, 3 m, 4 n, 6 ldq, 7 R, 8 ldr, 9 strideR. */
int tsqr_sign_normalize_batched(int dtype, int64_t batch, int64_t m, int64_t n, void* Q, int64_t ldq, void* R,
                                int64_t ldr, int64_t strideR, void* stream);

/* B <- Q^T B for the full m x m orthogonal Q (Sec. 1: apply the stored tree
 * of Q factors; "about the same cost as the traditionally represented Q").
 * B: device m x k (ldb >= k), in place.  Rows 0..n-1 then hold the thin
 * Q^T B (to the signs of diag R); rows n..m-1 depend on the tree shape.
 * tsqr_apply_qt, tsqr_apply_q and tsqr_form_q only read the implicit Q (the
 * tree steps' counters are stream-ordered allocations of each call), so
 * calls on distinct B may run concurrently on different streams; the caller
 * orders tsqr_qtree_destroy after all of them.
 * Errors: 1 q, 2 k, 3 B, 4 ldb. */
int tsqr_apply_qt(tsqr_qtree q, int64_t k, void* B, int64_t ldb, void* stream);

/* Linear least squares: for each of the k columns b of B, the x minimising
 * ||A x - b||_2 (Sec. 1: the remark on least squares problems solved with the
 * QR factorisation).  TSQR of A, then B <- Q^T B through the tree of Q
 * factors, then back substitution R x = (Q^T b)(0:n); Q preserves norms, so
 * the residual norm of b is the 2-norm of rows n..m-1 of Q^T b.
 *   dtype, m, n, A, lda as for tsqr_factor (m >= n >= 1, n <= 64); A must
 *   have full column rank (a zero diagonal entry of R gives Inf/NaN in X; it
 *   is not detected).  A is OVERWRITTEN with the leaf reflectors.
 *   B: device m x k (ldb >= k), OVERWRITTEN: rows 0..n-1 hold X (n x k), rows
 *   n..m-1 the trailing rows of Q^T B (LAPACK xGELS layout).  k = 0: A is
 *   factored (R only) and nothing else is written.
 *   rnorm: device array of k residual norms (in dtype; sums of squares in
 *   FP64, added in a fixed order), or NULL.
 *   All temporaries (R, the implicit Q's workspace, partial sums) are
 *   stream-ordered allocations released at the end of the stream work.
 *   Argument indices for errors: 1 dtype, 2 m, 3 n, 4 A, 5 lda, 6 k, 7 B,
 *   8 ldb, 10 opts. */
int tsqr_lstsq(int dtype, int64_t m, int64_t n, void* A, int64_t lda, int64_t k, void* B, int64_t ldb,
               void* rnorm, const tsqr_opts* opts, void* stream);

/* CholeskyQR, the fast but conditionally stable algorithm the paper compares
 * TSQR with (Sec. 2.3 and its sequential cost table): R = the upper Cholesky
 * factor of A^T A (positive diagonal), Q = A R^{-1}.  passes = 2 gives
 * CholeskyQR2: the same steps on Q, and R = R2 R1.  Provided for comparison:
 * one pass loses orthogonality like cond(A)^2 u and breaks down (NaN in Q
 * and R, not detected) once A^T A is not numerically positive definite.
 *   dtype, m, n (m >= n >= 1, n <= 64); A: device m x n (lda >= n), read
 *   only; Q: device m x n (ldq >= n), may be A itself; R: device n x n
 *   (ldr >= n), zeros below the diagonal.  A stream-ordered workspace is
 *   released at the end of the stream work.
 *   Argument indices for errors: 1 dtype, 2 m, 3 n, 4 A, 5 lda, 6 Q, 7 ldq,
 *   8 R, 9 ldr, 10 passes. */
int tsqr_cholqr(int dtype, int64_t m, int64_t n, const void* A, int64_t lda, void* Q, int64_t ldq, void* R,
                int64_t ldr, int passes, void* stream);

/* Modified Gram-Schmidt, the other fast but unstable algorithm the paper
 * compares TSQR with (Sec. 2.3): for j = 0..n-1, r_jj = ||a_j||,
 * q_j = a_j / r_jj, then r_jc = q_j^T a_c and a_c -= r_jc q_j for every later
 * column c (right-looking).  Its loss of orthogonality grows in proportion
 * to cond(A).  Provided for comparison: TSQR is the stable path.
 *   dtype, m, n (m >= n >= 1, n <= 64), A (device, m x n, lda >= n, not
 *   modified unless Q is A); Q: device m x n (ldq >= n), may be A itself
 *   (ldq = lda); R: device n x n (ldr >= n), upper triangular with a
 *   positive diagonal, zeros below it.  n + 1 streaming passes over the rows,
 *   each inner product reduced in a fixed order (the result does not depend
 *   on scheduling).  A rank-deficient A (a zero r_jj) is not detected: Inf or
 *   NaN propagate.  Partial sums live in a stream-ordered allocation released
 *   at the end of the stream work.
 *   Argument indices for errors: 1 dtype, 2 m, 3 n, 4 A, 5 lda, 6 Q, 7 ldq,
 *   8 R, 9 ldr. */
int tsqr_mgs(int dtype, int64_t m, int64_t n, const void* A, int64_t lda, void* Q, int64_t ldq, void* R,
             int64_t ldr, void* stream);

/* B <- Q B (reverse order of tsqr_apply_qt).  Same arguments. */
int tsqr_apply_q(tsqr_qtree q, int64_t k, void* B, int64_t ldb, void* stream);

/* Thin Q = Q [I_n; 0] (m x n, device, ldq >= n) (Sec. 2.1: Q factors with
 * n columns).  Errors: 1 q, 2 Q, 3 ldq. */
int tsqr_form_q(tsqr_qtree q, void* Q, int64_t ldq, void* stream);

/* The explicit thin Q with diag(R) made non-negative (the QR factorisation
 * is unique up to the signs of R's rows and Q's columns, Sec. 2.1): Q <- Q D
 * and R <- D R with D = diag(d), d_j = -1 where R_jj < 0, else +1, for every
 * member of the implicit Q.  For TSQR (tsqr_factor, tsqr_factor_batched)
 * the explicit-Q pass starts each member's tree from D instead of I_n, so Q D
 * costs no pass of its own; the result is bit for bit that of tsqr_form_q
 * followed by tsqr_sign_normalize(_batched).  For CAQR it is those two calls.
 *   Q: device m x n (ldq >= n), written.  R: device, member b's n x n R at
 *   R + b*strideR (ldr >= n; strideR >= n*ldr when there are several
 *   members), read for D, then its rows scaled in stream order.
 *   Errors: 1 q, 2 Q, 3 ldq, 4 R, 5 ldr, 6 strideR. */
int tsqr_form_q_signed(tsqr_qtree q, void* Q, int64_t ldq, void* R, int64_t ldr, int64_t strideR, void* stream);

/* Release the implicit Q (device workspace freed stream-ordered on the
 * stream of its creation).  NULL is accepted. */
int tsqr_qtree_destroy(tsqr_qtree q);

/* Host query of a handle: info[0..9] = m, n, block_rows, chains, arity,
 * levels, blocks, dtype, kind (0 TSQR, 1 CAQR), panel (CAQR).  info: host
 * array of 10. */
int tsqr_qtree_info(tsqr_qtree q, int64_t* info);

/* Geometry the library would use for (m, n, opts), without any GPU work.
 * out (host, 7): block_rows, rows per chain, chains, arity, levels, blocks,
 * padded width.  Errors: 1 m, 2 n, 3 opts, 4 out. */
int tsqr_plan_geometry(int64_t m, int64_t n, const tsqr_opts* opts, int64_t* out);

/* CAQR (Sec. 3): right-looking QR of a general m x n matrix (m >= n) whose
 * panel factorisation is TSQR; after panel k the panel's implicit Q^T is
 * applied to the trailing columns, first block by block (the leaf level),
 * then on the tree's n-row slabs (Sec. 3.1).
 *   dtype: storage type of A; update_dtype: arithmetic of the trailing
 *   updates (TSQR_F32 with FP64 storage = the mixed-precision update: the
 *   two products of each block reflector run on FP32 MFMA with FP32
 *   accumulation and are subtracted in FP64; the panel reflectors, their T
 *   factors and the tree combines stay in the storage type).
 *   A: device m x n (lda >= n), overwritten: R in the upper triangle of the
 *   first n rows, the panels' reflectors below (the implicit Q borrows A).
 *   panel: panel width b, 1..64 (0 = 64).  opts: tree shape of each panel.
 *   q_out: receives the implicit Q (apply it with tsqr_apply_q/_qt, form it
 *   with tsqr_form_q), or NULL.
 *   Errors: 1 dtype, 2 m, 3 n, 4 A, 5 lda, 6 panel, 7 update_dtype, 8 opts. */
int caqr_factor(int dtype, int64_t m, int64_t n, void* A, int64_t lda, int64_t panel, int update_dtype,
                const tsqr_opts* opts, tsqr_qtree* q_out, void* stream);

/* Left-looking CAQR over column blocks (Sec. 3.2: left-looking QR with TSQR
 * panels has the same costs as the right-looking form).  The columns are cut
 * into blocks of block_cols; block k first receives the implicit Q^T of
 * every panel factored before it, oldest first (each panel's leaves, then
 * its tree), and the panels inside the block are then factored and applied
 * right-looking to the block's later columns.  Each column thus receives the
 * same panel transformations in the same order as in caqr_factor; the
 * results agree with caqr_factor's to rounding (the apply kernels chosen for
 * a launch depend on its column count).  block_cols = panel is plain
 * left-looking, block_cols >= n right-looking without look-ahead.  Panel
 * trees: chains of eight 64-row blocks unless opts sets `chains`, combined
 * node by node.  Every kernel runs on `stream`, one after the other.
 *   dtype, m, n, A, lda, panel, update_dtype, opts, q_out: as caqr_factor
 *   (same output layout and implicit Q).
 *   block_cols: multiple of the panel width (0 = the panel width).
 *   Errors: 1 dtype, 2 m, 3 n, 4 A, 5 lda, 6 panel, 7 block_cols,
 *   8 update_dtype, 9 opts. */
int caqr_factor_left(int dtype, int64_t m, int64_t n, void* A, int64_t lda, int64_t panel, int64_t block_cols,
                     int update_dtype, const tsqr_opts* opts, tsqr_qtree* q_out, void* stream);

/* D = sign(diag R) with sign(0) = +1; R <- D R and Q <- Q D, so diag(R) >= 0
 * (the QR factorisation is unique up to these signs, Sec. 2.1).
 * Q: device m x n (ldq >= n) or NULL; R: device n x n (ldr >= n). */
int tsqr_sign_normalize(int dtype, int64_t m, int64_t n, void* Q, int64_t ldq, void* R, int64_t ldr,
                        void* stream);

/* Adjoint of the thin QR with diag(R) > 0 (the sign-normalised factors of
 * tsqr_sign_normalize), for reverse-mode differentiation.  Not in the paper:
 * the published QR adjoint (Walter & Lehmann; Liao et al. "copyltu" form)
 *     M = R triu(dR)^T - dQ^T Q,  C = tril(M) + tril(M,-1)^T,
 *     dA = (dQ + Q C) R^{-T}.
 * The m-long contraction dQ^T Q is reduced over row chunks like the TSQR tree;
 * dA is one streaming pass over dQ and Q.  No reflectors are needed.
 *   batch >= 1 matrices, each m x n (n <= 64), matrix b at pointer + b*stride.
 *   Q, R: forward outputs (R upper, positive diagonal).  dQ, dR: upstream
 *   gradients, either may be NULL (= zero); only triu(dR) is used.
 *   dA: output m x n.  All device pointers, row-major.
 *   Errors: 1 dtype, 2 batch, 3 m, 4 n, 5 Q, 6 ldq, 8 R, 9 ldr, 12 lddq,
 *   15 lddr, 17 dA, 18 ldda. */
int tsqr_backward(int dtype, int64_t batch, int64_t m, int64_t n, const void* Q, int64_t ldq, int64_t strideQ,
                  const void* R, int64_t ldr, int64_t strideR, const void* dQ, int64_t lddq, int64_t stridedQ,
                  const void* dR, int64_t lddr, int64_t stridedR, void* dA, int64_t ldda, int64_t stridedA,
                  void* stream);

/* R out of a factored matrix: dst (n x n) <- upper triangle of src (n x n
 * view, leading dimension lds), zeros below the diagonal.  Used to read R
 * from the first n rows of a CAQR-factored A.  Errors: 1 dtype, 2 n, 3 src,
 * 4 lds, 5 dst, 6 ldd. */
int tsqr_copy_r(int dtype, int64_t n, const void* src, int64_t lds, void* dst, int64_t ldd, void* stream);

/* Profiling hook.  When start/stop are hipEvent_t handles (plain pointers),
 * every later call records them on its stream right before and right after
 * the chain (leaf) kernel of `phase`: 0 tsqr_factor, 1 tsqr_apply_qt,
 * 2 tsqr_apply_q, 3 tsqr_form_q.  NULL disables.  Process-wide; not thread
 * safe.  Errors: 1 phase. */
int tsqr_set_phase_events(int phase, void* start, void* stop);

/* Release the CU-masked streams caqr_factor keeps (see TSQR_FLAG_SHARED_CUS)
 * on every device where it made them, after waiting for their work; a later
 * caqr_factor makes them again.  For callers that want no library-held
 * stream left at process exit (the Python binding calls it from an exit
 * handler), and for callers that go on to other GPU work after their CAQR
 * calls: while the masked streams exist, work on the process's other streams
 * was measured to run slower (a TSQR step 2.08 against 1.79 ms).  Not to be
 * called while a caqr_factor is running.  Errors:
 * TSQR_ERR_HIP. */
int tsqr_release_streams(void);

/* Workspaces (the implicit Q's, and the short-lived ones of the apply, least
 * squares, CholeskyQR, MGS and adjoint calls) come from a stream-ordered
 * memory pool of the library on each device, which keeps up to 2 GiB of freed
 * memory cached across synchronisations so that repeated calls do not map
 * their workspaces again.  This returns every pool's cached memory to the
 * device (hipMemPoolTrimTo); memory still in use is unaffected.  No HIP call
 * is made when no pool exists.  Errors: TSQR_ERR_HIP. */
int tsqr_release_workspace_pools(void);

/* Last HIP error code seen by this thread (0 if none) and a message. */
int tsqr_last_hip_error(void);
const char* tsqr_status_string(int status);

/* ---------------------------------------------------------------- batched
 * Many independent TSQR factorisations (Sec. 2.1 for each matrix) of uneven
 * shapes in one graph launch: the chains of all matrices form one work queue
 * (longest first) served by persistent one-wave workers, and each matrix's
 * tree nodes are performed by the worker that completes a node's last child.
 * The tree shape of each matrix (chains, arity) is a per-matrix option; the
 * Python autotuner chooses them per (dtype, column class, row range). */
typedef struct tsqr_batch_s* tsqr_batch;

/* Plan `count` factorisations.  m, n: HOST arrays of count entries with
 *   m[i] >= n[i] >= 1 and n[i] <= 64.  opts: NULL (defaults for every
 *   matrix) or a HOST array of count tsqr_opts (same meaning as for
 *   tsqr_factor, 0 = default).  Allocates the device workspace of every tree
 *   (owned by the plan, hipMalloc; the call synchronises the device) and a
 *   stream used for graph capture.  Errors: -2 count < 1, -3/-4 null or bad
 *   m/n entries (TSQR_ERR_UNSUPPORTED for n > 64), TSQR_ERR_NOMEM,
 *   TSQR_ERR_HIP. */
int tsqr_batch_plan_create(int dtype, int32_t count, const int64_t* m, const int64_t* n, const tsqr_opts* opts,
                           tsqr_batch* plan_out);

/* Factor every matrix of the plan on `stream`.
 *   A, lda, R, ldr: DEVICE arrays of count entries.  A[i] is matrix i
 *   (row-major, lda[i] >= n[i]), overwritten with its leaf reflectors; R[i]
 *   receives its n x n R (row-major, ldr[i] >= n[i], zeros below the
 *   diagonal) and may be NULL.  The four arrays are read by the device when
 *   the work runs, so their contents may change between calls.
 *   The first call captures a hipGraph (fill kernels that clear the work
 *   queue and the node counters, then one persistent kernel per column
 *   class 1..16, 17..32, 33..64) and launches it on `stream`; later calls
 *   with the same four array addresses only launch the graph again, other
 *   addresses capture a new one.  Calls on one plan must not overlap in time
 *   (they share the plan's workspace and counters). */
int tsqr_batch_factor(tsqr_batch plan, void* const* A, const int64_t* lda, void* const* R, const int64_t* ldr,
                      void* stream);

/* out[0] count, out[1] total chains, out[2] column classes launched,
 * out[3] workspace bytes, out[4] 1 if a graph is captured, out[5] persistent
 * workers launched over all classes.  out: host array of 6. */
int tsqr_batch_plan_info(tsqr_batch plan, int64_t* out);

/* Release the plan (synchronises the device first).  NULL is accepted. */
int tsqr_batch_plan_destroy(tsqr_batch plan);

#ifdef __cplusplus
}
#endif

#endif /* TSQR_H */
