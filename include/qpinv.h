/* qpinv -- Moore--Penrose pseudoinverse of dense quaternion matrices by hyperpower-family iterations
 * on AMD Instinct MI355X (gfx950).  C ABI of libqpinv.so.
 *
 * Methods (Karmakar, Bhadala & Behera, "A Family of Iterative Methods for Computing Generalized
 * Inverses of Quaternion Matrices and its Applications", Section 3):
 *   Newton--Schulz (order 2), the hyperpower iteration of order p (definition of the quaternion
 *   hyperpower iterative method), QSAI (Algorithm 2, order 10), QHPI19 (Algorithm 3, order 19) and
 *   QRAPID (Algorithm 1, step parameter N).  Every iteration is a chain of quaternion matrix
 *   products X_{j+1} = X_j p(R_j), R_j = I - A X_j, started from X_0 = alpha A^H (Theorem 1).
 *
 * Conventions
 *   - A quaternion matrix A = A_s + A_x i + A_y j + A_z k (Section 2) is described by qpinv_qmat:
 *     four real planes in ONE device allocation, plane p (p = 0..3 for s, x, y, z) starting at
 *     data + p * plane_stride elements, each plane row-major with row stride `ld` elements.
 *     Requirements: rows >= 0, cols >= 0, ld >= cols, plane_stride >= rows * ld.  The whole
 *     rows x ld extent of every plane must be readable: kernels may load a row up to ld (16-byte
 *     loads from a clamped chunk) and discard the elements beyond cols, whatever they hold.
 *   - All matrix pointers are DEVICE pointers owned by the caller; the library never frees or
 *     retains them beyond the call.  The library owns its workspace (grown on demand, freed by
 *     qpinv_finalize).
 *   - `hip_stream` is a hipStream_t (NULL = the default stream).  Calls enqueue their kernels on
 *     that stream; calls that return host scalars (solve, residuals, features) synchronise it.
 *   - Every function returns a status code (QPINV_OK = 0 or a negative error) and never throws or
 *     aborts across the ABI.  The message of the last error on the calling thread is available
 *     from qpinv_last_error().
 *   - Overlapping calls on one context from several host threads are not supported.
 */
#ifndef QPINV_H
#define QPINV_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------------------------- status codes */
#define QPINV_OK 0
#define QPINV_EINVAL (-1)        /* bad argument: shape, order, pointer, dtype, option */
#define QPINV_ENONFINITE (-2)    /* A (or a given X_0) holds NaN or Inf */
#define QPINV_EDIVERGED (-3)     /* the iteration diverged (alpha outside (0, 2/sigma_1^2), Theorem 1) */
#define QPINV_ENOTCONVERGED (-4) /* max_iter reached; X holds the last iterate (not fatal) */
#define QPINV_EHIP (-5)          /* HIP runtime error (no device, launch failure, ...) */
#define QPINV_ENOMEM (-6)        /* workspace allocation failed */
#define QPINV_ETIMEOUT (-7)      /* a persistent kernel hit its bounded wait and exited early */

/* ---------------------------------------------------------------------------------- types */
typedef enum { QPINV_F64 = 0, QPINV_F32 = 1 } qpinv_dtype; /* storage type of a qpinv_qmat */

typedef struct {
  void* data;           /* device pointer to element (0,0) of plane s */
  int64_t rows, cols;   /* matrix shape */
  int64_t ld;           /* row stride of each plane, in elements */
  int64_t plane_stride; /* distance between planes, in elements */
  int32_t dtype;        /* qpinv_dtype */
} qpinv_qmat;

typedef enum {
  QPINV_NS = 0,     /* Newton--Schulz X(2I - AX); order must be 2 (or 0 = default) */
  QPINV_HPI = 1,    /* hyperpower X sum_{k<p} R^k in Horner form; order = p >= 2 */
  QPINV_QSAI = 2,   /* Algorithm 2; order must be 10 (or 0) */
  QPINV_QHPI19 = 3, /* Algorithm 3; order must be 19 (or 0) */
  QPINV_QRAPID = 4  /* Algorithm 1; order = step parameter N >= 0 (-1 = default 5) */
} qpinv_method;

typedef enum {
  QPINV_ALPHA_POWER = 0,   /* alpha = mu / sigma1_est^2, sigma1_est^2 from power iteration on A^H A
                              (option power_steps, default 8); mu = alpha_or_mu if > 0 else 1 */
  QPINV_ALPHA_FROB = 1,    /* alpha = 1 / ||A||_F^2 (Section 4 experimental setup) */
  QPINV_ALPHA_GIVEN = 2,   /* alpha = alpha_or_mu (e.g. 1/sigma_max(A^C)^2 of Algorithms 1-3) */
  QPINV_ALPHA_LEARNED = 3, /* mu predicted by the scaling network (qpinv_mlp_*), clamped to
                              [sigma1_est^2 / min(||A||_F^2, ||A||_1 ||A||_inf), 1.9] (the lower end is
                              certified, the upper is not: sigma1_est^2 <= sigma_1^2); the solve restarts
                              with mu = 1 (POWER) when it diverges or reaches max_iter, and, for stop
                              rules other than E1_REL (whose test certifies the result), when mu > 1
                              and the first residual's 2-norm estimate (3 power steps) exceeds
                              1 + 1e-3; POWER when no network is loaded */
  QPINV_X0_GIVEN = 4       /* X holds X_0 on entry (warm start / resume) */
} qpinv_scaling;

typedef enum {
  QPINV_STOP_DX_ABS = 0, /* ||X_{j+1} - X_j||_F < tol  (stopping test of Algorithms 1-3) */
  QPINV_STOP_DX_REL = 1, /* ||X_{j+1} - X_j||_F <= tol ||X_{j+1}||_F */
  QPINV_STOP_E1_REL = 2, /* ||A X_{j+1} A - A||_F <= tol ||A||_F (two extra products per iteration) */
  QPINV_STOP_GUARDED = 3 /* relative change <= tol, or the first rise of the relative change after it
                            dropped below half its running maximum; then the better (smaller
                            ||XAX - X||_F / ||X||_F) of the two iterates around the minimum.  That
                            Penrose residual is formed from the residuals the iteration already
                            computed (in the solve's precision) when the minimum is the last update,
                            otherwise from scratch in FP64. */
} qpinv_stop;

typedef enum {
  QPINV_PREC_F64 = 0,          /* every product in FP64 (MFMA f64) */
  QPINV_PREC_F32 = 1,          /* every product in FP32 (MFMA f32, FP32 accumulate) */
  QPINV_PREC_F32_F64FINISH = 2,/* FP32 until its stop rule fires or the relative change d satisfies
                                  d <= 0.5 and d^p <= 1e-6 (the FP32 floor; p = convergence order),
                                  then FP64 iterations (option finish_method, default Newton--Schulz)
                                  until d <= tol, or d <= 0.5 and d^q <= tol (q >= 3, the finish method's
                                  order), or d rises, or option f64_finish_iters (default 2) FP64 updates */
  QPINV_PREC_MIXED = 3         /* BF16 operands (FP32 accumulate) first; leave BF16 when ||R||_2
                                  (power estimate, option mixed_rnorm_steps) or ||R||_2^p drops below
                                  option mixed_switch (1e-2), or ||R||_2 < 0.9 fails to halve in one
                                  update, or stops falling, or after max_bf16_iters (8) updates; then
                                  as F32_F64FINISH, with every product of FP32 storage (the FP32 phase,
                                  the finish's corrections) as GEMM_BF16X3 (option mixed_split = 1, the
                                  default; 0, and always in qpinv_solve_noalloc: native FP32 products) */
} qpinv_precision;

typedef enum { QPINV_GEMM_F64 = 0, QPINV_GEMM_F32 = 1, QPINV_GEMM_BF16 = 2, QPINV_GEMM_BF16X3 = 3 } qpinv_gemm_prec;

typedef enum { QPINV_SIDE_AUTO = 0, QPINV_SIDE_LEFT = 1, QPINV_SIDE_RIGHT = 2 } qpinv_side;

typedef enum {
  QPINV_REASON_TOL = 0, QPINV_REASON_RISE = 1, QPINV_REASON_MAX_ITER = 2, QPINV_REASON_DIVERGED = 3
} qpinv_reason;

typedef struct {
  int32_t iters;          /* updates performed, including the one that triggered the stop */
  int32_t iters_bf16, iters_f32, iters_f64; /* per-precision split of iters */
  int32_t returned;       /* index j of the returned iterate X_j */
  int32_t stop_reason;    /* qpinv_reason */
  int32_t side;           /* residual side used: 1 left (I_n - XA), 2 right (I_m - AX) */
  int32_t alpha_clamped;  /* learned mu was clamped into the admissible interval */
  int32_t fallback_used;  /* the classical alpha replaced a failed first choice */
  int32_t reserved;
  double alpha_used;      /* alpha of X_0 = alpha A^H (0 for X0_GIVEN) */
  double mu_used;         /* alpha * sigma1_est^2 */
  double sigma1_sq_est;   /* power-iteration estimate (0 if not computed) */
  double final_dx_rel;    /* ||X_j - X_{j-1}||_F / ||X_j||_F of the last update */
  double e1_rel;          /* ||AXA - A||_F / ||A||_F when the stop rule computed it, else -1 */
  double seconds;         /* host wall time of the call */
  double gemm_flops;      /* algorithmic flops of the quaternion products (32 M N K each) */
} qpinv_info;

typedef struct qpinv_ctx qpinv_ctx;

/* ---------------------------------------------------------------------------------- lifecycle */

/* Create a context on HIP device `device`.  `config` is NULL or "key=value;key=value" with the
 * keys of qpinv_set_option.  Errors: EINVAL (bad key/value), EHIP (no such device). */
int qpinv_init(qpinv_ctx** ctx, int device, const char* config);

/* Set a numeric option: side (qpinv_side), power_steps (>= 1), power_seed, autotune (0/1),
 * f64_finish_iters (1..4), finish_method (method of the FP64 finish updates: QPINV_NS (default),
 * QPINV_QSAI, QPINV_QHPI19, or -1 for the solve's own method), f64_refined (0/1, default 1: FP64
 * finish updates of NS, HPI, QSAI and QHPI19 form the residual R and the sum X + (T - I) X in FP64
 * and the polynomial T - I of R and its product with X in FP32, so the correction carries FP32
 * rounding relative to |(T - I) X| -- for the default Newton-Schulz finish T - I = R, and the second
 * update's correction is already at the FP64 level; 0: every finish product in FP64), mixed_switch (||R||_2
 * threshold, default 1e-2), mixed_rnorm_steps,
 * max_bf16_iters, mixed_split (0/1, default 1: the MIXED ladder's FP32-storage products as GEMM_BF16X3),
 * gemm_timing (0/1), gemm_cfg_f64 / gemm_cfg_f32 / gemm_cfg_bf16 / gemm_cfg_bf16x3 (tile configuration
 * index used for every product of that precision, -1 = tuned or heuristic choice), batched_cfg
 * (configuration of qpinv_solve_batched, -1 = tuned or default), batched_dynamic (phase-synchronous
 * batched form: 1 (default) workgroups claim work items from a counter, 0 workgroup g takes items
 * g, g + G, ...; the results are the same), small_path (0/1, default 1: single FP64 or FP32 solves of
 * NS, QSAI, QHPI19 or QRAPID(N <= 8) with at most 128 rows and columns run as one persistent launch),
 * small_gram (0/1, default 1: in such an FP64 solve the workgroups idle during the set-up form A^H A, or
 * A A^H on the right side, and the first update's side product alpha times it becomes an element-wise
 * step, one product phase fewer; the sums round differently from the product X_0 A), fault_small_giveup
 * (0/1, a test hook: the one-launch solve's grid-barrier give-up flag is raised before its launch, so every
 * workgroup leaves at its first barrier and the call returns QPINV_ETIMEOUT without waiting; the next
 * solve clears the flag), verbose (0/1), penrose_finish (projection of the returned
 * iterate in FP64, Section 2's Penrose conditions: 0 (default) none; 1 X <- X A X (condition (b)) after the
 * last update; 2 X <- (X A)^H X (A X)^H, which A^dagger leaves unchanged by conditions (b)-(d) and whose
 * rows lie in range(A^H) and columns in range(A), the invariants of every exact iterate (Proposition 3.1):
 * it removes the rounding that lower precisions leave outside them -- on a numerically rank-deficient A
 * that is what limits an FP32 solve, since the update multiplies it by its order in the near-null
 * directions.  It amplifies, to first order, what error the range directions still carry, so it is placed
 * before the last FP64 update: the FP64 finish then runs max(2, f64_finish_iters) updates (no early stop)
 * with the projection before the last; an F64 solve is projected after its last update and takes one
 * more FP64 Newton-Schulz update; F32 solves refuse it (EINVAL).  2 FP64 products for 1, 4 products and
 * 2 adjoints for 2).
 * Errors: EINVAL for an unknown key or out-of-range value. */
int qpinv_set_option(qpinv_ctx* ctx, const char* key, double value);

/* Free the workspace and the context.  NULL is accepted. */
int qpinv_finalize(qpinv_ctx* ctx);

/* Human-readable name of a status code (static storage). */
const char* qpinv_strerror(int status);

/* Message of the last failing call on this host thread (static per-thread storage). */
const char* qpinv_last_error(void);

/* ---------------------------------------------------------------------------------- the solve */

/* X ~= A^dagger for A (rows m, cols n) by `method` (Section 3; Algorithms 1-3).
 *   order        see qpinv_method.
 *   scaling      how X_0 = alpha A^H is chosen (Theorem 1; scaling step of Algorithms 1-3).
 *   alpha_or_mu  alpha for ALPHA_GIVEN, mu multiplier for ALPHA_POWER (<= 0 means 1).
 *   tol, max_iter, stop   stop rule (stopping test of Algorithms 1-3 and variants).
 *   precision    arithmetic of the products (qpinv_precision).  A may be F32 or F64 storage; the
 *                library converts into its workspace when the precision needs the other type.
 *   X            output, shape n x m, F32 or F64; for QPINV_X0_GIVEN it also holds X_0 on entry.
 *   info         may be NULL.
 * Return: OK; ENOTCONVERGED (X = last iterate); EDIVERGED (X = last finite iterate);
 *         ENONFINITE (A has NaN/Inf, X untouched); EINVAL; EHIP; ENOMEM. */
int qpinv_solve(qpinv_ctx* ctx, int method, int order, const qpinv_qmat* A, int scaling, double alpha_or_mu,
                double tol, int max_iter, int stop, int precision, qpinv_qmat* X, qpinv_info* info,
                void* hip_stream);

/* Bytes of the device array that qpinv_solve_noalloc carves its workspace from (one copy per GPU). */
#define QPINV_NOALLOC_SCRATCH_BYTES 67108864

/* qpinv_solve for callers that cannot allocate device memory during a call (serving loops with a fixed
 * memory budget, harnesses that forbid hipMalloc inside a call): the same arguments, the same iterates and
 * results as qpinv_solve with the same tiles, but every workspace buffer is carved from a static device
 * array of QPINV_NOALLOC_SCRATCH_BYTES (64 MiB) that each GPU holds from its first context until the
 * process ends.  The call makes no hipMalloc / hipFree / hipHostMalloc and no allocating library call;
 * qpinv_init has already allocated the context's scalar buffers and looked up the array's address on its
 * device.  Within the call: no tile autotuning (tiles tuned earlier on the context, else the defaults), no
 * per-product timing events (option gemm_timing is ignored), and a BF16 stage buffer that is never grown.
 * Limit: a shape whose workspace bound exceeds the array is rejected with EINVAL before anything is
 * launched (square FP64 solves up to 280 x 280, FP32 up to 371 x 371, FP32 with the FP64 finish or the
 * precision ladder up to 216 x 216; tall or wide shapes go further on the long side).  Sharing: every call on one GPU uses that
 * GPU's array, which keeps the last call's contents (each buffer is written before it is read within a
 * call): calls that overlap on one GPU -- two streams, threads or contexts -- race and must be serialised
 * by the caller.  Return codes as qpinv_solve. */
int qpinv_solve_noalloc(qpinv_ctx* ctx, int method, int order, const qpinv_qmat* A, int scaling,
                        double alpha_or_mu, double tol, int max_iter, int stop, int precision, qpinv_qmat* X,
                        qpinv_info* info, void* hip_stream);

/* Many independent solves in ONE persistent kernel launch (replayed from a captured hipGraph when the
 * batch signature repeats): power-iteration or given alpha, X_0 = alpha A^H, the product chain and the
 * stop rule per matrix, on the residual side of the smaller dimension.  Two kernel forms, chosen by the
 * autotuner (option autotune = 1) or option batched_cfg:
 *   queue:              each workgroup takes matrices from a device queue (largest work first) and
 *                       runs a whole solve on its own (no waits between workgroups);
 *   phase-synchronous:  all matrices advance one product at a time; every product's output tiles over
 *                       all active matrices are spread over all workgroups, which meet at a bounded
 *                       grid barrier (batch <= 2048; an expired wait returns ETIMEOUT).
 *   method       NS, QSAI or QHPI19 (order as for qpinv_solve).
 *   batch        number of matrices; A and X are HOST arrays of `batch` descriptors of DEVICE data.
 *   A[b]         m_b x n_b, FP32, 1 <= m_b, n_b <= 512;  X[b]: n_b x m_b, FP32 (output).
 *   scaling      ALPHA_POWER (option power_steps / power_seed) or ALPHA_GIVEN with alpha[b] > 0.
 *   stop         DX_ABS, DX_REL or GUARDED with tol; max_iter bounds every solve.
 *   infos        host array of `batch` (may be NULL); infos[b].reserved holds that solve's status.
 * The tile configuration is timed on the batch when option autotune = 1 (once per batch signature).
 * Return: OK; ENOTCONVERGED / EDIVERGED / ENONFINITE if any solve ended that way (see infos);
 *         EINVAL; EHIP; ENOMEM; ETIMEOUT.  The call waits for the batch to finish. */
int qpinv_solve_batched(qpinv_ctx* ctx, int method, int order, int batch, const qpinv_qmat* A, qpinv_qmat* X,
                        int scaling, const double* alpha, double tol, int max_iter, int stop, qpinv_info* infos,
                        void* hip_stream);

/* One iteration X_out = X_{j+1} from X_in = X_j (Algorithms 1-3, one pass of the loop body) in the
 * given product precision (qpinv_gemm_prec) on the given side (LEFT/RIGHT; AUTO picks the smaller).
 * A, X_in, X_out share one storage dtype (F64 for GEMM_F64, F32 otherwise).  `dx` (host, may be
 * NULL) receives {||X_out - X_in||_F^2, ||X_out||_F^2}.  Errors: EINVAL, EHIP, ENOMEM. */
int qpinv_step(qpinv_ctx* ctx, int method, int order, int side, int gemm_prec, const qpinv_qmat* A,
               const qpinv_qmat* X_in, qpinv_qmat* X_out, double dx[2], void* hip_stream);

/* Penrose residuals (Section 4, error metrics) computed in FP64 on the GPU:
 *   E_abs = {||AXA - A||_F, ||XAX - X||_F, ||(AX)^H - AX||_F, ||(XA)^H - XA||_F},
 *   E_rel = E_abs / {||A||_F, ||X||_F, ||AX||_F, ||XA||_F}  (host arrays of 4).
 * Errors: EINVAL, EHIP, ENOMEM. */
int qpinv_residuals(qpinv_ctx* ctx, const qpinv_qmat* A, const qpinv_qmat* X, double E_abs[4], double E_rel[4],
                    void* hip_stream);

/* ---------------------------------------------------------------------------------- building blocks */

/* Quaternion product (Section 2, Hamilton product): C = alpha A B + beta C + gamma I, with
 * A (M x K), B (K x N), C (M x N) of one storage dtype (F64 for GEMM_F64, F32 otherwise) and I the
 * quaternion identity (ones on the diagonal of the real plane).  C must not alias A or B.
 * GEMM_BF16 rounds the FP32 operands to BF16 (nearest even) and accumulates in FP32.  Its large
 * products (1024 or more 64 x 64 output tiles, or the "_staged" configurations) first copy the
 * operands into a BF16 stage buffer that the context owns: 2 * 4 * (Mp + Np) * Kp bytes, Mp and Np
 * the row counts of A and of B^T rounded up to 128, Kp = K rounded up to 32 (a product whose copy of one
 * operand would reach 2^31 bytes takes the direct form instead, with no copies).  The buffer grows on
 * demand (the stream is synchronised first) and is freed by qpinv_finalize; products on one context
 * share it, so they must not run concurrently on different streams.
 * GEMM_BF16X3 (FP32 storage) splits every FP32 operand element x into hi = bf16(x) and lo = bf16(x - hi)
 * (|x - hi - lo| <= 2^-16 |x|) and sums the three BF16 products hi.hi + hi.lo + lo.hi in one FP32-accumulated
 * product over 3 Kp, from split copies in the same stage buffer (three times the bytes above): every term of
 * the Hamilton product carries an error of at most about 3 2^-16 |a| |b| besides the FP32 accumulation, in
 * 0.39 of an FP32 product's time at 4096^3.  Products whose split copies would reach 2^31 bytes are refused
 * (EINVAL); the solver then keeps native FP32 products.
 * Errors: EINVAL, EHIP, ENOMEM (stage buffer). */
int qpinv_qgemm(qpinv_ctx* ctx, int gemm_prec, const qpinv_qmat* A, const qpinv_qmat* B, qpinv_qmat* C,
                double alpha, double beta, double gamma, void* hip_stream);

/* Initial iterate X = alpha A^H (Theorem 1): X (n x m) from A (m x n); dtypes may differ.
 * Errors: EINVAL, EHIP. */
int qpinv_x0(qpinv_ctx* ctx, const qpinv_qmat* A, double alpha, qpinv_qmat* X, void* hip_stream);

/* Submatrix B = A(rows, cols) (Section 5.1: the CUR factors C = A(:, J) and R = A(I, :)).  rows and
 * cols are DEVICE arrays of nrows / ncols 0-based indices, or NULL to take every row / column in order
 * (then nrows / ncols must equal A's).  B is nrows x ncols with A's dtype, written for all four planes.
 * An index outside A gives NaN in the corresponding row / column of B (the kernel never reads outside
 * A).  Errors: EINVAL (shapes, dtypes, counts). */
int qpinv_submatrix(qpinv_ctx* ctx, const qpinv_qmat* A, const int* rows, int nrows, const int* cols, int ncols,
                    qpinv_qmat* B, void* hip_stream);

/* Global quaternion Krylov solve of A X = B (Section 3.5 and Section 4, Example 4: Gl-QFOM and
 * Gl-QGMRES, optionally with a left preconditioner M such as a QSAI iterate: M A X = M B).
 *   method      QPINV_KRYLOV_FOM or QPINV_KRYLOV_GMRES; the basis is orthonormal in
 *               <X, Y> = Re tr(X^H Y) and never restarted (max_iter + 1 basis matrices of device memory).
 *   A, M        n x n (M may be NULL); B and X n x m; all FP64.  X holds X_0 on entry and the solution on
 *               return, and must be contiguous (ld = cols, plane_stride = rows * cols).
 *   tol         stop when RR = ||B - A X_j||_F / ||B - A X_0||_F <= tol (Example 4's test).  The method
 *               tracks the iterated system's ||M (B - A X_j)||_F / ||M (B - A X_0)||_F (M = I when NULL;
 *               GMRES: the rotated right-hand side, FOM: that norm over the last rotation's cosine);
 *               with M, RR itself is evaluated at every step once the tracked value is <= tol.
 *   iters, rr   steps taken and the tracked relative residual at the last step; true_rr = RR of the
 *               returned X; history[j] = tracked value after step j (host, history_cap entries; may be
 *               NULL with history_cap 0).  Any of iters, rr, true_rr may be NULL.
 * The call synchronises the stream (one host transfer of the new Hessenberg column per step).
 * Returns QPINV_OK, QPINV_ENOTCONVERGED (max_iter steps without reaching tol; X is still the step's
 * solution), EINVAL, ENOMEM, EHIP. */
#define QPINV_KRYLOV_FOM 0
#define QPINV_KRYLOV_GMRES 1
int qpinv_gl_krylov(qpinv_ctx* ctx, int method, const qpinv_qmat* A, const qpinv_qmat* B, const qpinv_qmat* M,
                    qpinv_qmat* X, double tol, int max_iter, int* iters, double* rr, double* true_rr, double* history,
                    int history_cap, void* hip_stream);

/* Masked merge of the impute-reconstruct loop (Section 5.1): Y = Omega (.) M + (1 - Omega) (.) X for all
 * four planes, Omega given as a DEVICE byte array (rows x cols, row stride mask_ld; nonzero = observed).
 * M, X and Y share one shape and dtype; Y may be M or X itself.  Errors: EINVAL. */
int qpinv_masked_merge(qpinv_ctx* ctx, const qpinv_qmat* M, const unsigned char* mask, int64_t mask_ld,
                       const qpinv_qmat* X, qpinv_qmat* Y, void* hip_stream);

/* Scaling features of A (used by ALPHA_POWER / ALPHA_LEARNED) into host out[7]:
 *   {sigma1_est^2 (power_steps steps on A^H A from the SplitMix64 start vector, seed power_seed),
 *    ||A||_F, ||A||_1, ||A||_inf, rows, cols, the estimate of the step before the last}.
 * `power_steps` <= 0 uses the context option.  Errors: EINVAL, ENONFINITE, EHIP. */
int qpinv_features(qpinv_ctx* ctx, const qpinv_qmat* A, int power_steps, double out[7], void* hip_stream);

/* ---------------------------------------------------------------------------------- learned scaling
 * A small network predicts mu = alpha * sigma1_est^2 for X_0 = alpha A^H from seven raw features per
 * matrix, given as rows of 7 doubles (sigma1_est^2, previous estimate, ||A||_F, ||A||_1, ||A||_inf,
 * rows, cols) -- the order qpinv_features reports them in, with the previous estimate moved second.
 * ALPHA_LEARNED solves use it once a network is loaded (trained or set); the predicted mu is clamped
 * into [sigma1_est^2 / min(||A||_F^2, ||A||_1 ||A||_inf), 1.9] (only the lower end is certified inside
 * Theorem 1's interval), and the classical alpha = 1/sigma1_est^2 replaces it when the iteration diverges
 * or reaches max_iter, or (stop rules other than E1_REL) when ||I - X_0 A||_2 is estimated above 1.
 * All arrays below are DEVICE arrays unless marked host. */

/* (Re)initialise the network weights (Xavier-uniform, SplitMix64 stream `seed`) and the optimiser. */
int qpinv_mlp_init(qpinv_ctx* ctx, uint64_t seed);

/* Standardisation of the network inputs from `count` raw feature rows.  Errors: EINVAL, EHIP. */
int qpinv_mlp_fit_normalization(qpinv_ctx* ctx, const double* raw, int count, void* hip_stream);

/* One Adam step (lr) on the minibatch rows idx[0..batch) (idx may be NULL: rows 0..batch) of raw
 * features and targets y = log(mu); batch <= 1024.  *loss (host) receives the minibatch mean squared
 * error before the step.  Errors: EINVAL, EHIP. */
int qpinv_mlp_train_step(qpinv_ctx* ctx, const double* raw, const double* target, const int* idx, int batch,
                         double lr, double* loss, void* hip_stream);

/* Gradient of the minibatch loss with respect to the parameters (FP32, qpinv_mlp_num_params entries)
 * into grad, without changing the weights; *loss as above.  Errors: EINVAL, EHIP. */
int qpinv_mlp_gradient(qpinv_ctx* ctx, const double* raw, const double* target, int batch, float* grad, double* loss,
                       void* hip_stream);

/* mu = exp(network output) for `count` raw rows into mu.  Errors: EINVAL, EHIP. */
int qpinv_mlp_predict(qpinv_ctx* ctx, const double* raw, int count, double* mu, void* hip_stream);

/* Number of parameters, and get/set of the parameters followed by the standardisation (mean[10],
 * std[10]) as host floats (n = qpinv_mlp_num_params() + 20).  get returns the required n. */
int qpinv_mlp_num_params(void);
int qpinv_mlp_get_params(qpinv_ctx* ctx, float* host, int n);
int qpinv_mlp_set_params(qpinv_ctx* ctx, const float* host, int n);

/* Training labels from spectra (Theorem 1's proof: X_0 = alpha A^H keeps every iterate V diag U^H, so
 * each singular value s_i follows rho <- g(rho) from rho = 1 - alpha s_i^2, with g the method's residual
 * map from its convergence theorem).  For matrix b with singular values spectra[offsets[b] ..
 * offsets[b+1]) the iteration count J(alpha) to ||AXA - A||_F / ||A||_F <= tol is evaluated on `ngrid`
 * points mu geometric in [mu_lo, mu_hi] (alpha = mu / s_max^2); the label is the point nearest
 * mu_target of the longest run of grid points attaining the minimum, reported relative to s1sq_est[b]
 * as mu_out[b] = alpha* s1sq_est[b]; j_best[b] is that minimum and j_classical[b] the count of
 * alpha = 1/s1sq_est[b] (max_iter + 1 when not reached; max_iter <= 64).  Errors: EINVAL, EHIP. */
int qpinv_spectral_labels(qpinv_ctx* ctx, int method, int order, const double* spectra, const int* offsets, int count,
                          const double* s1sq_est, double tol, int max_iter, int ngrid, double mu_lo, double mu_hi,
                          double mu_target, double* mu_out, int* j_best, int* j_classical, void* hip_stream);

/* Time every tile configuration of the product for shape (M, N, K) in `gemm_prec` and remember the
 * fastest for later solves on this context.  best_ms (host, may be NULL) receives its time.
 * Returns the chosen configuration id (>= 0) or an error. */
int qpinv_autotune(qpinv_ctx* ctx, int gemm_prec, int64_t M, int64_t N, int64_t K, double* best_ms,
                   void* hip_stream);

/* Persisted tile choices, so that a later process skips the autotuner's timing runs.  qpinv_tune_save
 * writes every configuration this context has tuned (products per precision and shape, batched solves per
 * batch signature) to the text file `path` (host string; replaced if it exists), by configuration name and
 * with a device token (architecture name and compute-unit count); returns the number of entries written or
 * EINVAL (no path, file not writable).  qpinv_tune_load merges such a file into this context's tuned
 * choices (an entry for the same shape or signature replaces the context's) and returns the number of
 * entries applied: 0 for a file written on another device; entries naming a configuration this library
 * does not have are skipped.  EINVAL for no path, an unreadable file or a malformed one (then nothing is
 * applied).  Neither call uses the GPU beyond reading the device's properties. */
int qpinv_tune_save(qpinv_ctx* ctx, const char* path);
int qpinv_tune_load(qpinv_ctx* ctx, const char* path);

/* Number of tile configurations for a product precision, and the name of one (static storage). */
int qpinv_num_tile_configs(int gemm_prec);
const char* qpinv_tile_config_name(int gemm_prec, int cfg);

/* Configurations of qpinv_solve_batched (option batched_cfg): count and static name ("" if out of
 * range).  Names starting with "batched_sync" are phase-synchronous, the others queue kernels. */
int qpinv_num_batched_configs(void);
const char* qpinv_batched_config_name(int cfg);

/* Same as qpinv_qgemm with an explicit tile configuration (for measurement). */
int qpinv_qgemm_cfg(qpinv_ctx* ctx, int gemm_prec, int cfg, const qpinv_qmat* A, const qpinv_qmat* B,
                    qpinv_qmat* C, double alpha, double beta, double gamma, void* hip_stream);

/* Product launch statistics.  With option gemm_timing = 1 every quaternion product this context
 * launches is bracketed by HIP events on its stream.  For each kernel used since the previous call
 * (product precision x tile configuration) one row of 5 doubles is written to `out` (host):
 * {gemm_prec, tile configuration, launches, algorithmic flops (32 M N K each), summed event ms}.
 * At most max_rows rows; returns the number of rows (>= 0) or an error (EINVAL, EHIP).  The call
 * waits for the recorded events and resets the counters. */
int qpinv_gemm_stats(qpinv_ctx* ctx, double* out, int max_rows);

/* Stop-rule controller replay (host only, no GPU use): feed per-update scalars
 * d_abs[j] = ||X_{j+1}-X_j||_F, x_norm[j] = ||X_{j+1}||_F, e1_rel[j] (may be NULL unless
 * stop = E1_REL) for j < count into the controller of `stop` with `tol`; writes the decision per
 * update into decision[j] (0 continue, 1 stop by tol, 2 stop by rise, 3 diverged, 4 new minimum
 * recorded) and returns the number of updates consumed before stopping (count if none). */
int qpinv_controller_replay(int stop, double tol, int count, const double* d_abs, const double* x_norm,
                            const double* e1_rel, int* decision);

#ifdef __cplusplus
}
#endif

#endif /* QPINV_H */
