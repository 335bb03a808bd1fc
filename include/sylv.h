/*
 * sylv.h - C ABI of the MI355X factorized Krylov solver for the Sylvester equation
 *
 *      A X + X B = C1 C2^T                                     (problem statement, eq. (1.1))
 *
 * with sparse A (n x n), B (m x m) and a low-rank right-hand side C1 (n x s), C2 (m x s).
 * The solution is returned in factored form X = V Xc W^T (Corollary 3.3): V (n x r_v) and
 * W (m x r_w) have orthonormal columns spanning block Krylov spaces of A and B^T, Xc is a small
 * r_v x r_w core.
 *
 * Conventions for every call below
 *   - Sizes are int64_t. Dense arrays are row-major with an explicit leading dimension
 *     (elements between consecutive rows).
 *   - Array pointers are DEVICE pointers (memory of the GPU the context was created on),
 *     allocated and owned by the caller, unless the parameter is marked "host".
 *   - The library allocates no device memory: every device buffer it needs lives in the
 *     workspace the caller passes to sylv_create (size from sylv_workspace_bytes). The library
 *     allocates only the host-side context and small host arrays for histories.
 *   - All device work is issued on the stream given to sylv_create (a hipStream_t passed as
 *     void*; NULL is the default stream). Calls that return a status wait for their work.
 *   - Return codes: 0 success, > 0 a solver outcome with a valid iterate, < 0 an error that
 *     leaves the context unchanged. sylv_status_string() names each code.
 *   - A context is not thread-safe; use one context per stream.
 */
#ifndef SYLV_H
#define SYLV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  SYLV_OK = 0,              /* converged: ||R_{k+1}|| <= tol * ||R_0|| (Alg. 4.1/4.2)       */
  SYLV_NOT_CONVERGED = 1,   /* max_iter reached; the last iterate is kept                   */
  SYLV_BREAKDOWN = 2,       /* a denominator of the recurrences vanished (or <P,Q> <= 0 in
                               CG); the last completed iterate is kept                       */
  SYLV_ERR_INVALID = -1,    /* bad argument (sizes, NULL pointers, malformed CSR)           */
  SYLV_ERR_HIP = -2,        /* a HIP runtime call failed                                     */
  SYLV_ERR_WORKSPACE = -3,  /* workspace missing, misaligned or smaller than required        */
  SYLV_ERR_RHS_RANK = -4,   /* C1 or C2 is not of full column rank (its QR fails)           */
  SYLV_ERR_STATE = -5       /* call out of order (e.g. factors requested before a solve)     */
};

/* Methods: factorized CG (Algorithm 4.1) and BiCGSTAB (Algorithm 4.2), and the further Krylov
 * methods the factorization carries over to (Section 4's remark, Section 6): conjugate residual
 * (CR, symmetric A and B, block Lanczos bases), conjugate gradient squared (CGS) and
 * generalized product-type BiCG (GPBiCG), both with two operator applications per iteration
 * on block Arnoldi bases. */
enum {
  SYLV_METHOD_CG = 0,
  SYLV_METHOD_BICGSTAB = 1,
  SYLV_METHOD_CR = 2,
  SYLV_METHOD_CGS = 3,
  SYLV_METHOD_GPBICG = 4
};

/* Precision. SYLV_FP64: everything in FP64. SYLV_MIXED_FP32: the bases V, W (and the compact
 * panels the sparse products read) are stored in FP32, halving the dominant memory traffic of
 * the block Arnoldi/Lanczos steps; products are accumulated in FP64 and the H, G blocks, the
 * cores, the scalars and the residual evaluation stay FP64. The recurrence then reaches a
 * true-residual floor of roughly the FP32 unit roundoff times the conditioning of the operator;
 * the outer refinement options (refine_max and the other refine_* fields of sylv_options)
 * recover full accuracy. SYLV_MIXED_BF16SPLIT: FP64 bases and recurrence, with the Gram
 * contractions of the true-residual evaluation in split BF16 on the BF16 matrix cores (the same
 * as SYLV_FP64 with gram_precision 1, or gram_precision 2 when that is asked for; see
 * gram_precision below). */
enum { SYLV_FP64 = 0, SYLV_MIXED_FP32 = 1, SYLV_MIXED_BF16SPLIT = 2 };

/* Compressed sparse row matrix: rows x rows, int32 row_ptr (rows + 1 entries, row_ptr[0] = 0)
 * and col_idx (nnz entries, sorted and unique within each row, 0 <= col < rows), float64
 * values (nnz); rows < 2^31 and nnz < 2^31. Device pointers, borrowed until sylv_destroy. */
typedef struct {
  int64_t rows;
  int64_t nnz;
  const int32_t *row_ptr;
  const int32_t *col_idx;
  const double *values;
} sylv_csr;

/* One problem A X + X B = C1 C2^T (eq. (1.1)).
 * lyapunov != 0 selects the Lyapunov equation A X + X A^T = C1 C1^T (Section 4.3): B and C2
 * are ignored, n must equal m, and the solution is X = V Xc V^T.
 * C1 is n x s with leading dimension ldc1 >= s; C2 is m x s with ldc2 >= s. Both are read
 * during sylv_create only. 1 <= s <= 8 and s <= min(n, m). */
typedef struct {
  int64_t n, m, s;
  sylv_csr A;
  sylv_csr B;
  int lyapunov;
  const double *C1;
  int64_t ldc1;
  const double *C2;
  int64_t ldc2;
} sylv_problem;

/* Options. method and max_iter size the workspace (the basis grows by s columns per CG
 * iteration and by 2s per BiCGSTAB iteration). check_every: the host waits for the device's
 * convergence flag every this many iterations (iterations enqueued after convergence do no
 * work); <= 0 selects the default, 16. closure_tol: a new basis block whose norm after orthogonalization is at most
 * closure_tol times ||M V_j||_F is replaced by a zero block (Krylov space exhausted); <= 0
 * selects the default of the precision (1e-12 for FP64, 1e-6 for FP32 bases).
 * precision: SYLV_FP64, SYLV_MIXED_FP32 (storage of the bases) or SYLV_MIXED_BF16SPLIT, see
 * above.
 * Outer refinement (0 < refine_max <= 4; used with SYLV_MIXED_FP32): after the solve, the
 * residual R = C1 C2^T - A X - X B of the iterate is sketched, Y = R Omega with a Gaussian
 * m x refine_rank matrix, compressed to the rank-k right-hand side P (R^T P)^T with P an
 * orthonormal basis of Y, and a correction equation with that right-hand side is solved (with
 * at most refine_max_iter iterations); this repeats until the FP64 true residual of the summed
 * iterate meets the tolerance or refine_max corrections ran. refine_inner_tol > tol lets the
 * first solve stop earlier.
 * streams: 1 runs the whole solve on the stream given at create; 2 runs the block Krylov steps
 * (Arnoldi / Lanczos, which do not depend on the iterates) on a second, library-owned stream
 * one iteration ahead of the core recurrences, synchronized with HIP events; 0 chooses 2 when
 * the bases have at least 16384 rows in total and 1 otherwise. Results are identical either
 * way.
 * reorth (BiCGSTAB's block Arnoldi, classical Gram-Schmidt applied twice): 1 orthogonalizes each
 * new block twice in its own step (three passes over the basis per step); 2 takes the second
 * pass of each block one step later, together with the first pass of the next block (two passes
 * per step; FP64 bases and s <= 4 only); 0 chooses 2 where it is available. The bases agree to
 * rounding.
 * gram_precision (Gram products of the true-residual evaluation, sylv_residual_norm): 0 forms
 * every Gram block in FP64 on FP64 matrix cores; 1 forms the blocks that involve the basis
 * defects (A V - V H, B^T W - W G, the right-hand side's QR defects and the C2 columns stacked
 * with them) in split BF16 on the BF16 matrix cores (each value split into two BF16 parts, three
 * partial products, FP32 partial sums over at most 4096 rows, summed in FP64; about 1e-5
 * relative error per Gram entry) and the basis Grams V^T V, W^T W in FP64: the defect terms are
 * at rounding level, so their contribution to the residual norm stays accurate to far better
 * than 1e-5 of the norm; 2 forms every block in split BF16 (the norm then carries a relative
 * error of order 1e-5).
 * verify: 1 evaluates the true residual after a solve
 * that stopped on the recursive test and, when it exceeds tol, solves again with the recursive
 * target lowered (at most twice); the result then reports rel_res_true, and the status is
 * SYLV_OK only when the true residual meets tol (SYLV_NOT_CONVERGED otherwise). 0 returns on the
 * recursive test alone (the algorithms' stopping rule). sylv_default_options() fills sensible
 * values (streams 0, reorth 0, gram_precision 0, verify 1). */
typedef struct {
  int method;
  int max_iter;
  int check_every;
  int record_history;
  double closure_tol;
  int precision;
  int refine_max;
  int refine_max_iter;
  int refine_rank;
  double refine_inner_tol;
  int streams;
  int reorth;
  int gram_precision;
  int verify;
} sylv_options;

/* Outcome of one solve. rank_v / rank_w: number of columns of the returned V and W;
 * rel_res_recursive: ||R_k|| / ||R_0|| from the recurrence (the algorithm's stopping test).
 * With outer refinement: iters sums the iterations of all solves, outer_steps counts the
 * correction solves, the factors are those of the summed iterate and rel_res_true is its FP64
 * true relative residual (status SYLV_OK when it meets tol). With verify, rel_res_true is the
 * true relative residual of a converged solve. Otherwise rel_res_true < 0. */
typedef struct {
  int status;
  int iters;
  int64_t rank_v;
  int64_t rank_w;
  double rel_res_recursive;
  double seconds;
  int outer_steps;
  double rel_res_true;
} sylv_result;

void sylv_default_options(sylv_options *opt);

/* Bytes of device workspace sylv_create needs for this problem and these options. Returns 0
 * if the problem or options are invalid. */
size_t sylv_workspace_bytes(const sylv_problem *prob, const sylv_options *opt);

/* Validates the problem, forms B^T in CSR on the device (unless Lyapunov), and computes the
 * QR factorizations C1 = V_1 R_L, C2 = W_1 R_R (Alg. 4.1 step 1, Alg. 4.2 step 2).
 * workspace: device buffer of ws_bytes >= sylv_workspace_bytes(), 256-byte aligned, owned by
 * the caller and used exclusively by this context until sylv_destroy.
 * Errors: SYLV_ERR_INVALID, SYLV_ERR_WORKSPACE, SYLV_ERR_RHS_RANK, SYLV_ERR_HIP. */
int sylv_create(void **ctx, const sylv_problem *prob, const sylv_options *opt,
                void *workspace, size_t ws_bytes, void *stream);

/* Factorized CG, Algorithm 4.1 (A and B symmetric positive definite), zero initial guess,
 * stopping test ||R_{k+1}|| <= tol ||R_0||. max_iter <= the value the workspace was sized
 * for. On return the iterate X_{k+1} = V_{k+1} Xc W_{k+1}^T is available through
 * sylv_get_factors. Returns the status also stored in res (res may be NULL). */
int sylv_factored_cg(void *ctx, double tol, int max_iter, sylv_result *res);

/* Factorized BiCGSTAB, Algorithm 4.2 with R~0 = R0; on return X_{k+1} = V_{2k+2} Xc
 * W_{2k+2}^T. Same conventions as sylv_factored_cg. */
int sylv_factored_bicgstab(void *ctx, double tol, int max_iter, sylv_result *res);

/* Factorized conjugate residual (A and B symmetric; F need not be definite): the matrix-
 * oriented CR recurrence (S = F(R), alpha = <R, S> / <Q, Q> with Q = F(P) kept by recurrence,
 * beta = <R', S'> / <R, S>) with every iterate in the factored form of Corollary 3.3, sums on
 * the cores (eq. (3.9)), inner products of cores (eq. (3.10)) and S by eq. (3.11). One block
 * Lanczos step per side per iteration; X_{k+1} = V_{k+1} Xc W_{k+1}^T. Conventions and
 * statuses as sylv_factored_cg; the context must have been created with method
 * SYLV_METHOD_CR (it sizes one more basis block). SYLV_BREAKDOWN when <Q, Q> or <R, S> vanishes. */
int sylv_factored_cr(void *ctx, double tol, int max_iter, sylv_result *res);

/* Factorized conjugate gradient squared: V = F(P), alpha = rho / <R~0, V>, Q = U - alpha V,
 * X += alpha (U + Q), R -= alpha F(U + Q), beta = rho' / rho, U = R + beta Q,
 * P = U + beta (Q + beta P), with R~0 = R0, the cores as above and two block Arnoldi steps per
 * side per iteration; X_{k+1} = V_{2k+2} Xc W_{2k+2}^T. Context created with SYLV_METHOD_CGS. */
int sylv_factored_cgs(void *ctx, double tol, int max_iter, sylv_result *res);

/* Factorized GPBiCG: the residual r_{k+1} = t_k - eta_k y_k - zeta_k F(t_k) with zeta_k, eta_k
 * minimizing its norm over the pair (eta_0 = 0), the iterate updated through u_k, z_k, and
 * two block Arnoldi steps per side per iteration; X_{k+1} = V_{2k+2} Xc W_{2k+2}^T. The history's
 * omega entries hold zeta_k. Context created with SYLV_METHOD_GPBICG. */
int sylv_factored_gpbicg(void *ctx, double tol, int max_iter, sylv_result *res);

/* True residual of the current iterate in FP64: abs_res = ||A X + X B - C1 C2^T||_F and
 * rel_res = abs_res / ||C1 C2^T||_F (host pointers). Evaluated from the factors without
 * forming X, as traces of small Gram products of the tall factors (inner product of
 * Section 2 / eq. (3.10), operator eq. (3.11) plus the basis defect A V - V H). */
int sylv_residual_norm(void *ctx, double *abs_res, double *rel_res);

/* Copies the factors of the current iterate: V (n x rank_v, ldv), Xc (rank_v x rank_w, ldx),
 * W (m x rank_w, ldw), device pointers. Any of V, Xc, W may be NULL to skip it; rank_v and
 * rank_w (host) receive the ranks, so a first call with all arrays NULL queries the sizes.
 * For a Lyapunov problem W is V. SYLV_ERR_STATE before a solve. */
int sylv_get_factors(void *ctx, double *V, int64_t ldv, double *Xc, int64_t ldx,
                     double *W, int64_t ldw, int64_t *rank_v, int64_t *rank_w);

/* Low-rank compression of the current iterate (the step after the solve, Corollary 3.3's form):
 * with V and W of orthonormal columns the singular values of X = V Xc W^T are those of the
 * core, so a truncated SVD Xc ~= U_k diag(sigma) Y_k^T gives X ~= (V U_k) diag(sigma) (W Y_k)^T.
 * sylv_compress finds the smallest rank k (at most max_rank when max_rank >= 0) with
 * ||Xc - U_k diag(sigma) Y_k^T||_F <= rel_tol ||Xc||_F, evaluating that error directly; *rank
 * and *rel_err (host, may be NULL) receive k and the achieved relative error. The SVD is formed
 * in FP64 on the GPU from a randomized range of at most 256 columns (Gaussian test matrix, one
 * power step) and one-sided Jacobi rotations on the projected core. Returns 0, or
 * SYLV_NOT_CONVERGED when max_rank or the 256-column range cannot meet rel_tol (the best
 * rank-k factors are kept). SYLV_ERR_STATE before a solve or after a refined solve;
 * SYLV_ERR_INVALID with FP32 bases.
 * sylv_get_compressed copies Z1 = V U_k (n x k, ldz1), sigma (k, descending) and Z2 = W Y_k
 * (m x k, ldz2) into device buffers (any may be NULL; *rank receives k). A later solve discards
 * the compression (SYLV_ERR_STATE until sylv_compress runs again). */
int sylv_compress(void *ctx, double rel_tol, int64_t max_rank, int64_t *rank, double *rel_err);
int sylv_get_compressed(void *ctx, double *Z1, int64_t ldz1, double *sigma, double *Z2,
                        int64_t ldz2, int64_t *rank);

/* Per-iteration history of the last solve, host arrays of capacity cap (any may be NULL):
 * relres[k] = ||R_{k+1}|| / ||R_0||, alpha[k], beta[k], omega[k] (omega only for BiCGSTAB;
 * beta[k] is undefined for the final iteration). *count receives the number of iterations. */
int sylv_get_history(void *ctx, double *relres, double *alpha, double *beta, double *omega,
                     int cap, int *count);

void sylv_destroy(void *ctx);

const char *sylv_status_string(int status);

/* Text of the last HIP runtime error the library saw in this thread (empty if none); useful
 * after a SYLV_ERR_HIP return. The string stays valid until the next library call. */
const char *sylv_last_error(void);

/* ---- batches of independent problems (one GPU) ----
 * Many problems of uneven sizes solved together (not in the paper: the paper solves one
 * problem of eq. (1.1) at a time). Each instance gets its own context, carved from one
 * caller-owned workspace; instance i uses opts[i].method and opts[i].max_iter. Forms:
 *   SYLV_BATCH_STREAMS  instances spread over nstreams HIP streams (longest-first by estimated
 *                       cost), one host thread per stream solving its instances one after
 *                       another; results are bit-identical to solving each instance alone.
 *   SYLV_BATCH_GROUPED  instances with the same method (CG or BiCGSTAB), block size, form
 *                       (Sylvester or Lyapunov), max_iter and closure_tol, FP64 and without
 *                       refinement, form a group: the group's iterations advance in lock-step
 *                       on one stream, every phase one kernel launch over the group's instance
 *                       table; an instance that stopped (its device stop flag) drops out of the
 *                       launches; the host polls one word per group (instances still running)
 *                       every 16 iterations. Converged instances are verified on the true
 *                       residual as single solves are. Results equal single solves up to
 *                       rounding (other workgroup splits of the reductions). Instances that
 *                       cannot join a group run as in SYLV_BATCH_STREAMS on nstreams streams.
 *   SYLV_BATCH_GRAPH    SYLV_BATCH_GROUPED, with each 16-iteration segment of a group captured
 *                       once as a HIP graph (the first solve that reaches it) and replayed by
 *                       later solves with the same max_iter.
 * sylv_batch_workspace_bytes: the instances' workspaces plus the group tables (0 if any
 *   instance is invalid); the same size serves every form.
 * sylv_batch_create_ex: errors as sylv_create (the first failing instance's code),
 *   SYLV_ERR_INVALID for an unknown form. sylv_batch_create = the SYLV_BATCH_STREAMS form.
 * sylv_batch_solve: res[count] (host); returns the first error (< 0) or the largest status.
 * sylv_batch_context: context of instance i (for sylv_get_factors, sylv_residual_norm, ...);
 *   owned by the batch.
 * sylv_batch_groups: number of groups (0 in the streams form). */
#define SYLV_BATCH_STREAMS 0
#define SYLV_BATCH_GROUPED 1
#define SYLV_BATCH_GRAPH 2
size_t sylv_batch_workspace_bytes(int count, const sylv_problem *probs, const sylv_options *opts);
int sylv_batch_create(void **batch, int count, const sylv_problem *probs,
                      const sylv_options *opts, void *workspace, size_t ws_bytes, int nstreams);
int sylv_batch_create_ex(void **batch, int count, const sylv_problem *probs,
                         const sylv_options *opts, void *workspace, size_t ws_bytes, int nstreams,
                         int form);
int sylv_batch_solve(void *batch, double tol, sylv_result *res);
void *sylv_batch_context(void *batch, int i);
int sylv_batch_groups(void *batch);
void sylv_batch_destroy(void *batch);

/* ---- measurement hooks ---- */

/* Time per kernel family, summed over the iterations the solves actually ran. */
typedef struct {
  int family;        /* index; sylv_kernel_family_name() names it                        */
  int64_t launches;  /* timed launches                                                   */
  double ms;         /* summed launch durations (HIP events on the context's stream)     */
  double bytes;      /* summed algorithmic bytes (the data the method must move)         */
  double flops;      /* summed algorithmic floating-point operations                     */
} sylv_kernel_stat;

/* on != 0: later solves record HIP events around every launch of the timed kernel families
 * (this serializes nothing but adds event overhead; use it for measurement runs) and the
 * statistics restart from zero; on == 0 stops recording. */
int sylv_set_profiling(void *ctx, int on);

/* Copies up to cap family records into out (host); *count receives the number of families.
 * SYLV_ERR_STATE if profiling is off. */
int sylv_get_kernel_stats(void *ctx, sylv_kernel_stat *out, int cap, int *count);

const char *sylv_kernel_family_name(int family);

/* ---- building blocks, exposed for testing and reuse (same stream/ownership rules) ---- */

/* Y = A X for CSR A (rows x rows) and a row-major panel X (rows x s, leading dimension ldx),
 * Y rows x s with leading dimension ldy; 1 <= s <= 8. The CSR SpMM of the block Lanczos /
 * Arnoldi step (eq. (3.8)). Unlike the other calls, sylv_spmm and sylv_sell_spmm only enqueue
 * their kernel on `stream` and return without waiting, so that products issued back to back
 * run back to back; 0 means the launch was accepted, and the caller orders later work on the
 * same stream or synchronizes before reading Y on the host. */
int sylv_spmm(const sylv_csr *A, int64_t s, const double *X, int64_t ldx, double *Y,
              int64_t ldy, void *stream);

/* Sliced-ELLPACK copy of a CSR matrix, the layout the solver's SpMM streams (slices of 64 rows,
 * each stored column-major with the slice's maximum row length; short rows padded with zero
 * values). sylv_sell_bytes: device bytes of the copy (0 for an invalid matrix).
 * sylv_sell_build: builds it into the caller's buffer; SYLV_ERR_WORKSPACE when the padding
 * exceeds the reserved 25% (matrices with very uneven rows stay in CSR).
 * sylv_sell_spmm: Y = A X as sylv_spmm, reading the copy built from the same A. */
size_t sylv_sell_bytes(const sylv_csr *A);
int sylv_sell_build(const sylv_csr *A, void *sell, size_t bytes, void *stream);
int sylv_sell_spmm(const sylv_csr *A, const void *sell, int64_t s, const double *X, int64_t ldx,
                   double *Y, int64_t ldy, void *stream);

/* Transpose of a square CSR matrix (rows x rows, nnz entries) into caller buffers:
 * out_row_ptr (rows + 1), out_col_idx (nnz), out_values (nnz). The result is canonical
 * (sorted column indices), so it is bit-identical to any other exact transpose. scratch:
 * device buffer of at least sylv_csr_transpose_scratch_bytes(rows) bytes (0 for rows < 0 or
 * rows >= 2^31). */
size_t sylv_csr_transpose_scratch_bytes(int64_t rows);
int sylv_csr_transpose(const sylv_csr *A, int32_t *out_row_ptr, int32_t *out_col_idx,
                       double *out_values, void *scratch, void *stream);

/* CSR transpose for callers that cannot allocate device memory: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc. Same result as sylv_csr_transpose
 * (canonical, bit-identical), but its scratch (2 (rows + 2) ints of column counts and scatter
 * cursors) lives in a static device array of the library, one per GPU, held until the process
 * ends: at most SYLV_NOALLOC_TRANSPOSE_MAX_ROWS rows (16 MiB of scratch); larger matrices return
 * SYLV_ERR_WORKSPACE (sylv_last_error names the limit). The call allocates nothing and only
 * enqueues kernels on `stream` (no memset or memcpy, no synchronization, so it may be captured
 * into a HIP graph); the caller orders later work on the same stream or synchronizes before
 * reading the outputs on the host. Every call on one GPU shares that GPU's scratch array: calls
 * that overlap on one GPU (on different streams, or from different threads) race and must be
 * serialized by the caller. out_row_ptr (rows + 1), out_col_idx (nnz), out_values (nnz) are
 * caller-owned device buffers. */
#define SYLV_NOALLOC_TRANSPOSE_MAX_ROWS ((int64_t)1 << 21)
int sylv_csr_transpose_noalloc(const sylv_csr *A, int32_t *out_row_ptr, int32_t *out_col_idx,
                               double *out_values, void *stream);

/* C (M x N, ldc) = alpha * op(A) op(B) + beta * C in FP64 on FP64 MFMA, with element strides:
 * A(i,k) = A[i*a_rs + k*a_cs], B(k,j) = B[k*b_rs + j*b_cs] (a transpose is a swap of the two
 * strides). The dense contraction behind the Gram products of the residual evaluation and the
 * core operator eq. (3.11). beta == 0 ignores C's old contents. M, N, K < 2^31. */
int sylv_dgemm(int64_t M, int64_t N, int64_t K, double alpha, const double *A, int64_t a_rs,
               int64_t a_cs, const double *B, int64_t b_rs, int64_t b_cs, double beta, double *C,
               int64_t ldc, void *stream);

/* C (M x N, ldc) = A^T B, or C += A^T B with accumulate != 0, for row-major operands A (K x M,
 * lda) and B (K x N, ldb) read down their K rows: the tall-skinny Gram products of the stacked
 * factors that the true-residual evaluation forms (inner products of Section 2 between tall
 * factors, eq. (3.10)), on FP64 matrix cores. K >= 1; lda and ldb are multiples of 8 with
 * lda >= M and ldb >= N rounded up to a multiple of 64 (the columns up to there are read; their
 * values only reach entries of C that are not written). symmetric != 0 (M == N, B == A): only
 * the tiles on and below the diagonal are computed and the upper triangle of C is then copied
 * from the lower one. work: device scratch of work_bytes bytes (8-byte aligned; NULL allowed)
 * for partial tiles; with sylv_gram_work_bytes(M, N, K) bytes every product runs in its
 * fastest form (large Grams on 128 x 128 tiles, split over K where the output has few tiles),
 * with less some run with fewer workgroups. Waits for the product. */
size_t sylv_gram_work_bytes(int64_t M, int64_t N, int64_t K);
int sylv_gram(int64_t M, int64_t N, int64_t K, const double *A, int64_t lda, const double *B,
              int64_t ldb, int symmetric, int accumulate, double *C, int64_t ldc, void *work,
              size_t work_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* SYLV_H */
