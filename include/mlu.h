/*
 * mlu -- blocked LU factorization with partial pivoting on AMD Instinct MI355X
 * (gfx950): the loop-based algorithm variants of Catalan, Herrero,
 * Quintana-Orti, Rodriguez-Sanchez and van de Geijn, "A Case for Malleable
 * Thread-Level Linear Algebra Libraries: The LU Factorization with Partial
 * Pivoting" (arXiv 1611.06365).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  * Matrices are FP64 and ROW-MAJOR: element (i, j) of an m x n matrix X with
 *    leading dimension ldx >= max(1, n) is X[i*ldx + j].  (A C-contiguous
 *    torch tensor of shape (m, n) is such a matrix with ldx = n.)
 *  * Every pointer whose name starts with d_ / d is DEVICE memory owned by the
 *    caller; h_ pointers are host memory read during the call only.  The
 *    library never allocates or frees device memory in these calls.
 *  * `stream` is a hipStream_t (NULL = the default stream).  All device work is
 *    enqueued on it asynchronously; nothing synchronizes, except the two entry
 *    points whose loop is decided on the host (mlu_dgetrf_et waits for each
 *    panel's realized width, mlu_dsgesv_gmres_ir for each refinement and each
 *    chunk of GMRES steps), as documented there.  Results (including *d_info) are valid once
 *    the stream's work has completed.  The look-ahead
 *    variant additionally uses one library-owned stream per device (default
 *    priority), forked from and joined back into `stream` with events, so a
 *    caller's stream capture records the whole call.
 *  * Return value (synchronous, host-side argument check, LAPACK convention):
 *      0       the work was enqueued;
 *      -i      argument i (1-based, `stream` is argument 1) is invalid and
 *              nothing was enqueued;
 *      MLU_ERR_HIP  a HIP runtime call failed while enqueuing.
 *  * Calls that share a workspace must not overlap in time.
 */
#ifndef MLU_H
#define MLU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MLU_ERR_HIP (-1000)
#define MLU_ERR_NOINIT (-1001)  /* mlu_init has not run on the current device */

/* Device-side status written to *d_info (besides 0 and j > 0, see mlu_dgetrf). */
#define MLU_INFO_SYNC_TIMEOUT (-999)  /* a cross-workgroup wait exceeded its bound */
#define MLU_INFO_BAD_PIVOT (-998)     /* an interchange index was out of range    */

/* Algorithmic variants (Fig. "LU", Fig. "LU_la_blk", Section 4.2 of the paper). */
enum mlu_variant {
  MLU_RL = 0, /* blocked right-looking: RL1 panel, RL2 trsm, RL3 gemm                 */
  MLU_LL = 1, /* blocked left-looking: LL1 trsm, LL2 gemm, LL3 panel (lazy swaps)     */
  MLU_LA = 2, /* right-looking with look-ahead: T_PF (PF1-PF3) || T_RU (RU1-RU2), the  */
              /* panel's workgroups joining RU2 once PF3 is done (worker sharing,     */
              /* Section 4.1)                                                         */
  /* 3 is the batched kernel in mlu_select's answers, not a variant here */
  MLU_LA_NOWS = 4 /* MLU_LA without worker sharing: T_PF idles after PF3 (the      */
                  /* comparison of Section 5.2); same arithmetic, bitwise results */
};

/*
 * Precision of the products in the outer trailing updates (RL3, PF2, RU2, LL2)
 * of the mixed-precision factorization.  The matrix stays FP64 in memory: the
 * operands of each update are rounded to the lower precision (FP32, or BF16
 * through FP32 with round to nearest even), the product is accumulated in FP32
 * on the matrix cores, and it is subtracted from the FP64 trailing matrix.  The
 * panel factorization and its inner updates, the triangular solves and the
 * interchanges stay FP64.
 */
enum mlu_precision {
  MLU_PREC_FP64 = 0,
  MLU_PREC_FP32 = 1,
  MLU_PREC_BF16 = 2  /* BF16 operands, FP32 accumulation */
};

/* Largest order of a matrix in the batched factorization. */
#define MLU_BATCH_MAX_N 512

/* Largest inner block size b_i of the panel factorization (Section 4.2 uses
 * b_i = 16 and 32).  The diagonal-block kernel holds 16 columns in registers;
 * a 32-column block is eliminated by it in two passes. */
#define MLU_MAX_NB_INNER 32

/* Library version, e.g. 200 for 0.2.0. */
int mlu_version(void);

/*
 * Prepare the library on the current device: the look-ahead variant's
 * library-owned stream and events, created once per device.  Called by the
 * workspace queries; a caller that captures a look-ahead call into a graph
 * calls it (or a workspace query) on that device before the capture, since
 * the creation is not a stream operation.  Returns 0 or MLU_ERR_HIP.
 */
int mlu_init(void);

/*
 * Workspace (device bytes) that mlu_dgetrf needs.  Depends on nothing but the
 * library build; arguments are accepted for forward compatibility.  Also runs
 * mlu_init on the current device (its failure is not reported here: without a
 * device the size is still returned).
 * Returns 0, or -i for an invalid argument; *bytes receives the size.
 */
int mlu_dgetrf_workspace(int m, int n, int variant, int nb, int nb_inner, size_t *bytes);

/*
 * LU factorization with partial pivoting, P A = L U (Section 3, opening;
 * algorithms of Fig. "LU", Fig. "LU_la_blk" and Section 4.2).
 *
 * Precondition:  dA holds A_hat, m x n (any m, n >= 0).
 * Postcondition: dA holds {L\U}: the strictly lower part of the first min(m,n)
 *   columns is L (unit diagonal not stored), the upper part of the first
 *   min(m,n) rows is U; d_ipiv[c] (c < min(m,n)) is the 1-based row interchanged
 *   with row c+1 at step c (sequential interchanges, LAPACK getrf convention:
 *   P applies them in order).  Pivot choice: the largest |value| in the current
 *   column from the diagonal down; the first such row on ties.
 *   *d_info = 0, or j > 0 if U(j,j) (1-based) is exactly zero (first such j);
 *   the factorization is still completed, the division by that pivot skipped.
 *
 *  stream      hipStream_t.
 *  m, n        matrix size.
 *  dA, lda     device matrix, row-major, lda >= max(1, n); m <= 33280
 *              (512 + 32 * 1024 rows: the tallest panel the register-resident
 *              kernel holds).
 *  d_ipiv      device int32[min(m, n)].
 *  d_info      device int32[1].
 *  variant     MLU_RL, MLU_LL, MLU_LA or MLU_LA_NOWS.
 *  nb          outer block size b (>= 1); nb = 1 gives each variant's
 *              unblocked form, nb >= min(m,n) a single panel.
 *  nb_inner    block size b_i of the panel factorization, 0..32 (0 = min(nb,
 *              16)): the panel [A11; A21] is factored by the blocked `inner`
 *              algorithm with b_i, each b_i-column block by LU_unb in the
 *              register-resident diagonal-block kernel (16 columns per pass;
 *              a block of 17..32 columns takes two passes with a rank-16
 *              update between them, the same elimination); b_i >= b means
 *              LU_unb on the whole panel.
 *  inner       algorithm of the panel factorization (Section 4.2, "outer /
 *              inner LU"): MLU_RL (right-looking: after each b_i block its
 *              interchanges, the solve of its rows and the update of the
 *              panel's columns to its right) or MLU_LL (left-looking: each
 *              b_i block first receives the panel's earlier interchanges, then
 *              the solve and update with the panel's columns to its left, then
 *              its own factorization, whose interchanges go to the columns to
 *              its left only).  Both give the same factors up to rounding.
 *  h_schedule  optional host array of n_schedule block sizes (each >= 1) used
 *              for the first outer iterations instead of nb (the paper's
 *              "Determine block size b"; the last block is trimmed to what is
 *              left of min(m, n)); NULL = constant nb.
 *  n_schedule  length of h_schedule (ignored when it is NULL).
 *  iters_limit -1 = run to completion; s >= 0 = stop after s outer loop bodies
 *              (RL, LL: s panels done; LA: the initial panel and s bodies, so
 *              panel s is factored and its interchanges are pending outside
 *              it).  Used to check the loop invariant.
 *  d_work      device workspace of work_bytes >= mlu_dgetrf_workspace().
 */
int mlu_dgetrf(void *stream, int m, int n, double *dA, int lda, int32_t *d_ipiv, int32_t *d_info,
               int variant, int nb, int nb_inner, int inner, const int32_t *h_schedule, int n_schedule,
               int iters_limit, void *d_work, size_t work_bytes);

/*
 * mlu_dgetrf for callers that cannot allocate: code under stream capture,
 * serving loops and harnesses that forbid device allocation.  Same arguments
 * and results as mlu_dgetrf without the workspace (arguments 1..14 numbered
 * as there): the factorization's scratch (the panel kernel's exchange slots,
 * the tile queues, about 60 KB) lives in a fixed-size device array of the
 * library, one per device, held until the process ends; no call allocates or
 * frees device memory.  Its size does not depend on m or n, so the only size
 * limit is mlu_dgetrf's (m <= 33280, argument 2).  mlu_init (or a workspace
 * query) must have run on the current device first: it resolves the array's
 * device address and creates the library stream; otherwise the call returns
 * MLU_ERR_NOINIT and enqueues nothing.  Every call on a device shares that
 * device's array (cleared by a kernel at the start of each call): calls that
 * overlap in time on one device race, whatever their streams.
 */
int mlu_dgetrf_noalloc(void *stream, int m, int n, double *dA, int lda, int32_t *d_ipiv, int32_t *d_info,
                       int variant, int nb, int nb_inner, int inner, const int32_t *h_schedule, int n_schedule,
                       int iters_limit);

/*
 * LU with partial pivoting by the look-ahead variant with early termination of
 * the panel factorization (Section 4.2, "Early termination"; Fig.
 * "LU_LA_ET").  Each look-ahead panel PF3 is factored by the blocked
 * left-looking algorithm in nb_inner-wide blocks, which touches nothing to the
 * right of the current block; when the trailing update RU2 of the same outer
 * iteration completes, it raises a device flag, the panel stops at the end of
 * its current block, and the next outer iteration proceeds with the columns
 * factored so far as its block (the block size adapts).  Result: as
 * mlu_dgetrf (same factors, pivots, info), computed with the realized panel
 * widths as the schedule.
 *  m, n, dA, lda, d_ipiv, d_info, nb, nb_inner: as mlu_dgetrf (nb = the
 *              planned width of each panel).
 *  force       0 = the flag is raised by RU2 (the method); 1 = every
 *              look-ahead panel stops after its first block; 2 = no panel
 *              stops (plain look-ahead with a left-looking PF3).
 *  min_width   a look-ahead panel stops only once it has at least this many
 *              columns (0 = after any block, the method's rule; ignored with
 *              force = 1).
 *  h_widths    optional host int32[max_widths]: the realized panel widths, in
 *              order (they sum to min(m, n)); *n_widths = their number (also
 *              when it exceeds max_widths, of which only the first are stored).
 *  d_work      mlu_dgetrf_workspace() bytes.
 * The host waits on the device once per outer iteration (for the width the
 * panel reached), so the call returns when the last panel has been factored
 * and the final updates are enqueued.  FP64 only.
 * Returns 0, -i for an invalid argument i, or MLU_ERR_HIP.
 */
int mlu_dgetrf_et(void *stream, int m, int n, double *dA, int lda, int32_t *d_ipiv, int32_t *d_info, int nb,
                  int nb_inner, int force, int min_width, int32_t *h_widths, int max_widths, int *n_widths,
                  void *d_work, size_t work_bytes);

/*
 * Mixed-precision LU with partial pivoting: mlu_dgetrf with the outer trailing
 * updates' products in `precision` (MLU_PREC_FP32, MLU_PREC_BF16, or
 * MLU_PREC_FP64 for exactly mlu_dgetrf).  The factors are those of a matrix
 * within about u_low * ||A|| of A (u_low = 2^-24 for FP32, 2^-8 for BF16)
 * rather than u_64 * ||A||: meant
 * as the factorization inside iterative refinement (mlu_dsgesv_ir), the
 * precision ladder the paper's loop-based variants admit unchanged (Fig.
 * "LU", Fig. "LU_la_blk": only the update kernel differs).  Arguments as
 * mlu_dgetrf, with `precision` inserted as argument 12 (later arguments are
 * numbered one higher in the -i return codes).
 */
int mlu_dsgetrf(void *stream, int m, int n, double *dA, int lda, int32_t *d_ipiv, int32_t *d_info, int variant,
                int nb, int nb_inner, int inner, int precision, const int32_t *h_schedule, int n_schedule,
                int iters_limit, void *d_work, size_t work_bytes);

/*
 * Solve A X = B by mixed-precision LU and FP64 iterative refinement (the
 * precision ladder over the paper's variants; Section 3 for the
 * factorization):
 *   LU := A factored by mlu_dsgetrf(precision, variant, nb, nb_inner, MLU_RL);
 *   X  := U^-1 L^-1 P B;
 *   repeat: R := B - A X in FP64;
 *           berr := max_j ||R_j||_inf / (||A||_inf ||X_j||_inf + ||B_j||_inf);
 *           stop if berr <= tol (or after max_iter corrections, or once
 *             berr is not finite or above twice the smallest berr so far:
 *             the corrections diverge);
 *           X := X + U^-1 L^-1 P R.
 *  dA (n x n, lda), dB (n x nrhs, ldb): read only.  dX (n x nrhs, ldx): the
 *  solution.  d_ipiv (int32[n]) and d_info as mlu_dgetrf, for the factors.
 *  *d_iters = number of corrections applied when berr <= tol was reached (0 if
 *  the first solve met it), or -1 if it was not reached (max_iter corrections,
 *  or divergence); *d_berr = berr of the X returned.  Everything is enqueued;
 *  the stop test is a device flag that the rest of the enqueued loop reads.
 *  d_work: mlu_dsgesv_ir_workspace(n, nrhs) bytes (it holds the n x n factors).
 *  Returns 0, -i for an invalid argument i, or MLU_ERR_HIP.
 */
int mlu_dsgesv_ir_workspace(int n, int nrhs, size_t *bytes);
int mlu_dsgesv_ir(void *stream, int n, int nrhs, const double *dA, int lda, const double *dB, int ldb, double *dX,
                  int ldx, int precision, double tol, int max_iter, int variant, int nb, int nb_inner,
                  int32_t *d_ipiv, int32_t *d_info, int32_t *d_iters, double *d_berr, void *d_work,
                  size_t work_bytes);

/*
 * Solve A x = b (one right-hand side) by mixed-precision LU and FP64
 * refinement whose corrections may come from GMRES (GMRES-IR: Carson and
 * Higham, SIAM J. Sci. Comput. 2017 and 2018), for kappa(A) * u_low >~ 1,
 * where the plain corrections of mlu_dsgesv_ir stop converging.  M = P^T L U is
 * the factorization of mlu_dsgetrf(precision, variant, nb, nb_inner, MLU_RL) (Section 3),
 * applied in FP64 as the preconditioner.
 *   x := M^-1 b;
 *   repeat: r := b - A x in FP64;
 *           berr := ||r||_inf / (||A||_inf ||x||_inf + ||b||_inf);
 *           stop if berr <= tol (or after max_outer corrections);
 *           solver MLU_IR_LU:    d := M^-1 r (stopping as not converged
 *             once berr is not finite or above twice the smallest so far);
 *           solver MLU_IR_GMRES: d := GMRES on M^-1 A d = M^-1 r from d = 0,
 *             Arnoldi with classical Gram-Schmidt applied twice, Givens
 *             rotations; it stops when its residual estimate falls to
 *             gmres_tol * ||M^-1 r||_2, at max_krylov steps, or at a breakdown;
 *           solver MLU_IR_AUTO:  MLU_IR_LU while each correction at least
 *             halves berr, MLU_IR_GMRES from the first one that does not;
 *           x := x + d;
 *           stopping as not converged once berr is not finite or two GMRES
 *           corrections in a row have each failed to halve it.
 *  dA (n x n, lda), db (n): read only.  dx (n): the solution.  d_ipiv and
 *  d_info as mlu_dgetrf, for the factors.  On return (the call waits for the
 *  stream once per outer and per GMRES step, so it is not capturable):
 *  *h_outer = corrections applied when berr <= tol was reached (0 if the first
 *  solve met it), or -1 if it stopped without reaching it;
 *  *h_inner = GMRES steps over all corrections; *h_berr = berr of the x
 *  returned.  1 <= max_krylov <= MLU_GMRES_MAX_KRYLOV; n <= 33280 (as
 *  mlu_dgetrf).
 *  d_work: mlu_dsgesv_gmres_ir_workspace(n, max_krylov) bytes (the n x n
 *  factors and the Krylov basis).  Returns 0, -i for an invalid argument i,
 *  or MLU_ERR_HIP.
 */
enum mlu_ir_solver { MLU_IR_LU = 0, MLU_IR_GMRES = 1, MLU_IR_AUTO = 2 };
#define MLU_GMRES_MAX_KRYLOV 512
int mlu_dsgesv_gmres_ir_workspace(int n, int max_krylov, size_t *bytes);
int mlu_dsgesv_gmres_ir(void *stream, int n, const double *dA, int lda, const double *db, double *dx,
                        int precision, int solver, double tol, int max_outer, int max_krylov, double gmres_tol,
                        int variant, int nb, int nb_inner, int32_t *d_ipiv, int32_t *d_info, int32_t *h_outer,
                        int32_t *h_inner, double *h_berr, void *d_work, size_t work_bytes);

/*
 * Batched LU with partial pivoting of `batch` independent square matrices of
 * different orders, in one persistent launch (Section 3 applied to each
 * operand: blocked right-looking with an unblocked panel, Fig. "LU").
 *  d_n      device int32[batch]: order of matrix i, 0 <= n_i <= max_n.
 *  d_A      device array of batch device pointers: matrix i, row-major,
 *           leading dimension d_lda[i] >= max(1, n_i); factored in place into
 *           {L\U} as mlu_dgetrf.
 *  d_ipiv   device array of batch device pointers: int32[n_i] interchanges of
 *           matrix i (1-based, sequential, as mlu_dgetrf).
 *  d_info   device int32[batch]: 0, j > 0 for the first exactly zero pivot
 *           (factorization completed), or -1 if n_i or d_lda[i] is invalid
 *           (the matrix is left untouched).
 *  max_n    an upper bound on every n_i (<= MLU_BATCH_MAX_N).
 *  nb       panel width: 16 or 32 (a tuning choice, results differ only in
 *           rounding), 0 for the default (16).
 *  d_work   mlu_getrf_batched_workspace(batch) bytes.
 * Matrices are processed largest first (a device counting sort), one per
 * workgroup at a time from atomic queues, in three size classes (orders above
 * 256, above 128, the rest: workgroups of 512, 256 and 128 threads, one
 * persistent launch per class that max_n can reach).  The call enqueues
 * kernels only (no memset): it can be captured in a stream graph.
 * Returns 0, -i for an invalid argument i, or MLU_ERR_HIP.
 */
int mlu_getrf_batched_workspace(int batch, size_t *bytes);
int mlu_dgetrf_batched(void *stream, int batch, const int32_t *d_n, double *const *d_A, const int32_t *d_lda,
                       int32_t *const *d_ipiv, int32_t *d_info, int max_n, int nb, void *d_work,
                       size_t work_bytes);
/* The same in FP32 (float matrices). */
int mlu_sgetrf_batched(void *stream, int batch, const int32_t *d_n, float *const *d_A, const int32_t *d_lda,
                       int32_t *const *d_ipiv, int32_t *d_info, int max_n, int nb, void *d_work,
                       size_t work_bytes);

/*
 * The learned selector (the block-size study of Section 5.1 as a model):
 * given the order n, the number of matrices and the product precision,
 * choose the variant and block size.  Host function, no device work.
 *  model       host float array written by the selector's pack(): a header
 *              [2, 9, hidden, 3, n_cand, n_lo, n_hi, batch_hi, margin, sd,
 *              ll_max_panels, batch_max_n], n_cand (variant id, b) candidate
 *              pairs (variant id 0..2 = MLU_RL/LL/LA with outer block size b
 *              for mlu_dgetrf / mlu_dsgetrf, 3 = MLU_SELECT_BATCHED with panel
 *              width b for mlu_?getrf_batched), then three dense layers
 *              (row-major W, then b) of a 9 -> hidden -> hidden -> 1
 *              perceptron with ReLU predicting the scaled log time per flop
 *              of one configuration from its features (log2 n, its square,
 *              log2 batch, the FP32 flag, the variant one-hot, log2 b).
 *  model_len   its length in floats.
 *  n           matrix order (>= 1); batch: number of matrices (>= 1);
 *              precision MLU_PREC_FP64 or _FP32.
 *  variant, nb receive the choice: the candidate with the smallest
 *              prediction (the first on ties) among the batched ones when
 *              batch > 1 and n <= batch_max_n, else among the single-matrix
 *              ones (the left-looking variant only up to ll_max_panels
 *              panels).
 *  fallback    receives 1 when the exhaustive autotuner should decide instead
 *              (n outside [n_lo, n_hi] or batch above batch_hi, or the
 *              runner-up predicted within `margin` of the choice), else 0.
 * Returns 0 or -i for an invalid argument i (a malformed model is argument 1
 * or 2).
 */
#define MLU_SELECT_BATCHED 3
int mlu_select(const float *model, int model_len, int n, int batch, int precision, int *variant, int *nb,
               int *fallback);

/*
 * Triangular solve with several right-hand sides, left side, no transpose:
 * B := T^{-1} B (RL2 / PF1 / RU1 / LL1 use uplo 'L', diag 'U' on trilu(A11),
 * Fig. "LU").
 *  uplo   'L' lower or 'U' upper triangle of T is read (the other is ignored).
 *  diag   'U' unit diagonal (not read) or 'N' stored diagonal.
 *  m      order of T; nrhs columns of B.  dT (ldt >= max(1,m)), dB (ldb >= max(1,nrhs)).
 * A zero on a non-unit diagonal gives inf/nan, as in BLAS trsm.
 */
int mlu_dtrsm(void *stream, char uplo, char diag, int m, int nrhs, const double *dT, int ldt, double *dB,
              int ldb);

/*
 * Solve A X = B with the factorization from mlu_dgetrf (square n x n):
 * B := U^{-1} L^{-1} P B.  dLU/lda and d_ipiv as returned by mlu_dgetrf; dB is
 * n x nrhs (ldb >= max(1, nrhs)), overwritten by X.
 */
int mlu_dgetrs(void *stream, int n, int nrhs, const double *dLU, int lda, const int32_t *d_ipiv, double *dB,
               int ldb);

/*
 * Trailing update C := C - A B (RL3 / PF2 / RU2 / LL2; Fig. "LU", Fig.
 * "LU_la_blk", Section 4.2) on FP64 matrix cores.  A is m x k, B k x n, C m x n.
 */
int mlu_dgemm_update(void *stream, int m, int n, int k, const double *dA, int lda, const double *dB, int ldb,
                     double *dC, int ldc);

/*
 * Apply the sequential interchanges d_ipiv[k1 .. k2) (0-based positions,
 * 1-based row values v with k+1 <= v <= m for position k) to columns
 * [0, ncols) of the m-row matrix dA (the "row permutations" between the panel
 * factorization and the update, Section 3.1).  A value out of that range is
 * skipped and *d_info (if not NULL) is set to MLU_INFO_BAD_PIVOT.
 */
int mlu_dlaswp(void *stream, int m, int ncols, double *dA, int lda, int k1, int k2, const int32_t *d_ipiv,
               int32_t *d_info);

/*
 * Unblocked factorization of one m x bw block (bw <= m; 1 <= bw <= 16 at any
 * m <= 33280, 17 <= bw <= 32 for m <= 8192, else -3 or -2): the
 * diagonal-block kernel (LU_unb of Fig. "LU", left) alone, holding the block
 * in registers (two rows per thread for up to 16 columns, one row per thread
 * for up to 32).  Interchanges are applied inside the block only; d_ipiv[c]
 * (c < bw) receives the 1-based row.  *d_info as in mlu_dgetrf.  Needs the
 * mlu_dgetrf workspace.
 */
int mlu_dgetf2_block(void *stream, int m, int bw, double *dA, int lda, int32_t *d_ipiv, int32_t *d_info,
                     void *d_work, size_t work_bytes);

/*
 * Measurement hook: event timing of the outer trailing-update GEMM launches
 * (RL3, PF2, RU2 -- the kernel that carries nearly all of the flops).
 * mlu_trace_begin(capacity) makes every following such launch, on any stream,
 * record a pair of HIP events around itself (at most `capacity` launches; the
 * library creates the events once).  In the look-ahead variant, the helper
 * workgroups that join RU2's tile queue from the panel's stream (Section 4.1,
 * worker sharing) record a pair too: when they start before RU2's own launch
 * ends, RU2 counts until the later of the two ends (its last tile may be a
 * helper's).  mlu_trace_end waits for the recorded events and returns the
 * number of launches timed, their summed duration in ms, and their
 * algorithmic flops (2 m n k per launch) and bytes (8 (2 m n + m k + k n) per
 * launch); it stops the recording.  Process-wide state: not for use while
 * another thread factors.
 */
int mlu_trace_begin(int capacity);
int mlu_trace_end(int *launches, double *total_ms, double *flops, double *bytes);

#ifdef __cplusplus
}
#endif

#endif /* MLU_H */
