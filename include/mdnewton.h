/*
 * mdnewton -- one Newton step on truncated power series for a polynomial
 * system in multiple-double arithmetic (double double, quad double, octo
 * double), on an AMD Instinct MI355X (gfx950).
 *
 * The method is that of Verschelde, "GPU Accelerated Newton for Taylor Series
 * Solutions of Polynomial Homotopies in Multiple Double Precision"
 * (arXiv:2301.12659): evaluate and differentiate every monomial at the series
 * x(t) by convolutions (Section 5.1), assemble the series Jacobian
 * A(t) = A_0 + A_1 t + ... and the residual b(t) = -p(x(t)), and solve the lower
 * triangular block Toeplitz system of Section 2 with a Householder QR of A_0
 * (Sections 1.1 and 5.3) and staged back substitutions with right-hand side
 * updates (Sections 4 and 5.4).
 *
 * System.  p_i(x) = c_{i,0}(t) + sum_{m in P_i} c_m x^{a_m}, i = 0..n-1, with a
 * constant series c_{i,0}(t) per polynomial, a scalar multiple-double
 * coefficient c_m per monomial and exponent vectors a_m >= 0.  Series are
 * truncated at degree d: D = d + 1 coefficients (the paper's "order D").
 *
 * Numbers.  A multiple double with L limbs (L = 2, 4 or 8; 1: a double) is an unevaluated
 * sum of L doubles (Section 1.2).  Every numeric array is stored limb-major
 * ("structure of arrays", Sections 1.2 and 6): limb l of element q of an array
 * of N elements is at ptr[l * N + q].  Element orders:
 *   series vectors  x, b, c_{i,0}, dx : [L][n][D]      (variable i, coefficient k)
 *   Jacobian series A                 : [L][n][n][D]   (row i, column j, coefficient k:
 *                                                      coefficient of t^k in dp_i/dx_j)
 *   dense matrices (A_0, QR)          : [L][n][n]      row-major
 *   monomial coefficients cff         : [L][m]
 *
 * Pointers.  Numeric pointers are DEVICE pointers; index arrays passed to
 * md_plan_create are HOST pointers, validated and copied to the device.  The
 * caller owns every numeric buffer and the workspace; the plan owns only its
 * device copies of the index tables.  Calls are asynchronous on the given
 * stream.
 *
 * Errors.  Functions return MD_OK or a negative code for errors the host can
 * detect (bad sizes, indices out of range, workspace too small, HIP failures);
 * md_last_error() then describes it.  Conditions found on the device (a
 * singular A_0, a non-finite result) are written to *dev_status (a device
 * int32) and can be read after the stream is synchronized.  No exception or
 * abort crosses this interface.
 */
#ifndef MDNEWTON_H
#define MDNEWTON_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MD_OK 0
#define MD_EINVAL (-1)     /* invalid argument */
#define MD_ESINGULAR (-2)  /* A_0 is singular: a Householder column or R_ii is zero */
#define MD_ENONFINITE (-3) /* a NaN or infinity appeared in the result */
#define MD_EHIP (-4)       /* a HIP runtime call failed */
#define MD_ENOSPACE (-5)   /* workspace too small */

/* Precision = number of limbs L.  MD_D is plain double arithmetic (the
 * paper's "D" in its comparisons across precisions, Section 7): every entry
 * point but the batches and complex data accepts it. */
#define MD_D 1
#define MD_DD 2
#define MD_QD 4
#define MD_OD 8

/* Largest supported number of series coefficients D = d + 1, dimension n and
 * exponent.  (The paper's experiments use order 64; Table 1 goes to 127.) */
#define MD_MAX_COEFFS 128
#define MD_MAX_DIM 1024
#define MD_MAX_EXPONENT 8

typedef struct md_plan md_plan;

/* Build a plan for a system of n polynomials in n variables with m monomials,
 * truncated at degree d (D = d + 1 <= MD_MAX_COEFFS), in precision prec
 * (MD_D, MD_DD, MD_QD or MD_OD).  Index tables (host pointers, CSR):
 *   poly_ptr[n+1] : monomials of polynomial i are poly_ptr[i] .. poly_ptr[i+1]-1
 *   mon_ptr[m+1]  : support entries of monomial j are mon_ptr[j] .. mon_ptr[j+1]-1
 *   var[nnz]      : variable of each entry, strictly increasing within a monomial
 *   exp[nnz]      : exponent of each entry, 1 <= exp <= MD_MAX_EXPONENT
 * Monomials with an empty support are allowed (constants).  The plan copies
 * the tables to the device.  Returns MD_EINVAL on any inconsistency. */
int md_plan_create(int prec, int n, int d, int m, const int32_t *poly_ptr, const int32_t *mon_ptr,
                   const int32_t *var, const int32_t *exp, md_plan **out);
int md_plan_destroy(md_plan *plan);

/* Workspace bytes needed by md_eval_diff and md_newton_step for this plan. */
int md_workspace_size(const md_plan *plan, size_t *bytes);

/* Evaluation and differentiation at a series (Sections 5.1 and 6):
 *   b(t) = -p(x(t)) mod t^D              -> b   [L][n][D]
 *   A(t) = dp/dx (x(t)) mod t^D           -> A   [L][n][n][D]
 * from cff [L][m], cst (the constant series c_{i,0}) [L][n][D] and x [L][n][D].
 * Each monomial is evaluated and differentiated by the reverse mode of
 * Section 5.1 (forward, backward and cross products, 3k-5 convolutions for k
 * variables with exponent one); exponents above one use a common factor. */
int md_eval_diff(const md_plan *plan, const double *cff, const double *cst, const double *x, double *b,
                 double *A, void *ws, size_t ws_bytes, hipStream_t stream);

/* Householder QR of an n x n multiple-double matrix (Sections 1.1 and 5.3),
 * in place: on return a0 [L][n][n] (row-major) holds R on and above the
 * diagonal and the Householder vectors below it (unit leading entry
 * implicit), tau [L][n] the reflector factors: A_0 = Q R with
 * Q = H_0 H_1 ... H_{n-1}, H_c = I - tau_c v_c v_c^T, v_c = e_c + (entries below).
 * A zero column sets *dev_status = MD_ESINGULAR.  The factorization runs on
 * several workgroups that hand the reflectors over through the workspace
 * (md_qr_workspace_size bytes: flags, a reflector board and the slots of the
 * reflector scalars); a hand-over
 * time-out sets MD_EHIP. */
int md_qr_workspace_size(int prec, int n, size_t *bytes);
int md_qr(int prec, int n, double *a0, double *tau, void *ws, size_t ws_bytes, hipStream_t stream,
          int32_t *dev_status);

/* md_qr for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * factorization, kernels and results as md_qr, with no workspace argument and
 * no allocation.  Its scratch (the flags, the reflector board and the slots of
 * the reflector scalars) is a static
 * device array of MD_QR_NOALLOC_MAX_BYTES bytes; each GPU the library runs on
 * holds its own copy until the process ends.  The call is refused with
 * MD_ENOSPACE when md_qr_workspace_size(prec, n) exceeds that size (octo
 * doubles up to n = 256, quad doubles up to n = 363, double doubles up to
 * n = 514).  Every call on a GPU uses that GPU's one array, which keeps the
 * last call's contents (a kernel clears the flags and empties the scalar
 * slots at every call):
 * calls that overlap in time on one GPU (several streams or host threads)
 * race and give wrong results; order them on one stream or serialize them.
 * Arguments, status and errors as md_qr. */
#define MD_QR_NOALLOC_MAX_BYTES (4u * 1024u * 1024u + 64u * 1024u)
int md_qr_noalloc(int prec, int n, double *a0, double *tau, hipStream_t stream, int32_t *dev_status);

/* Solve the lower triangular block Toeplitz system of Section 2,
 *   A_0 dx_k = b_k - sum_{j=1..k} A_j dx_{k-j},  k = 0..d,
 * given the QR factors of A_0 from md_qr (qr [L][n][n], tau [L][n]) and the
 * Jacobian series A [L][n][n][D] (coefficient 0 is not read).  rhs_dx [L][n][D]
 * holds b on entry and dx on return.  Q^T and the inverse of R are applied to
 * every stage (Q^H b and back substitution kernels, Section 5.3; the stage
 * updates of Section 5.4).  *dev_status gets MD_ESINGULAR for a zero R_ii. */
int md_solve_workspace_size(int prec, int n, int d, size_t *bytes);
int md_series_solve(int prec, int n, int d, const double *qr, const double *tau, const double *A,
                    double *rhs_dx, void *ws, size_t ws_bytes, hipStream_t stream, int32_t *dev_status);

/* One Newton step (Section 2): b = -p(x), A = p'(x), dx from the block
 * Toeplitz system, x := x + dx in place (x [L][n][D]).  On the device:
 * *dev_status = MD_OK, MD_ESINGULAR or MD_ENONFINITE; dev_norms [2][D]:
 * dev_norms[k] = max_i |b_{i,k}| and dev_norms[D + k] = max_i |dx_{i,k}|
 * (leading limbs), the quantities the paper's Newton loop monitors. */
int md_newton_step(const md_plan *plan, const double *cff, const double *cst, double *x, int32_t *dev_status,
                   double *dev_norms, void *ws, size_t ws_bytes, hipStream_t stream);

/* count plain Newton steps, x := x + dx each time, with results identical bit
 * for bit to count calls of md_newton_step.  The QR of A_0 is on the critical
 * path of a single step; here it is taken off: A_0 of the next step depends
 * only on coefficient 0 of the next iterate, x_0 + dx_0, and dx_0 = M b_0
 * (the first stage of the staged solve, Section 2) is formed as soon as the
 * current step has its factorization and its b.  The pre-pass, QR and
 * back substitution of step s+1 then run on the plan's second stream beside
 * the staged solve of step s and the evaluation of step s+1 (the QR is
 * still computed for every step; Section 5.3 computes it once per path).
 * This applies to plans whose staged solve runs in one persistent launch
 * (double or quad double, n <= 64) with supports of at most 8 variables;
 * other plans take count ordinary steps.  The factorization of step s+1
 * waits on the device for the launch that forms its x_0 on the caller's
 * stream, and the caller's stream for M of each step (counters in the
 * workspace, reset at the start of the call; the waits are bounded and
 * report MD_EHIP), so two calls on one workspace must not overlap.  dev_status: MD_OK, or the failure of any of the steps (the
 * steps overlap, so the status is not reset between them); dev_norms: those
 * of the last step.  Workspace as md_newton_step;
 * the last step leaves its factorization where md_newton_step does, for
 * md_newton_step_window with keep_factorization.  MD_EINVAL for count < 0. */
int md_newton_steps(const md_plan *plan, int count, const double *cff, const double *cst, double *x,
                    int32_t *dev_status, double *dev_norms, void *ws, size_t ws_bytes, hipStream_t stream);

/* One Newton step in mixed precision.  The introduction (Section 1) recalls
 * that the early coefficients must be computed more accurately than the late
 * ones, and Section 1.2 places multiple doubles in the trend of mixed
 * precision.  Here the residual b = -p(x) (monomial values, forward products
 * only), the update x := x + dx and the norms are computed at the plan's
 * precision L, while the Jacobian series (backward and cross products), the
 * QR of A_0 and the staged solve run at prec_solve limbs (MD_DD or MD_QD,
 * at most L).  Since b carries all of x's accuracy, repeated steps converge
 * to the same solution as md_newton_step; each step reduces the error by
 * about the solve precision times the condition of A_0, so a few more steps
 * are needed than in the plain iteration.  The Ls-limb truncations of x, cff
 * and b are their leading limb planes (limb-major storage), so no copies are
 * made.  Arguments, workspace (md_workspace_size of the plan), status and
 * norms as md_newton_step; prec_solve == L is md_newton_step.  MD_EINVAL for
 * a prec_solve that is not a precision or exceeds the plan's. */
int md_newton_step_mixed(const md_plan *plan, int prec_solve, const double *cff, const double *cst, double *x,
                         int32_t *dev_status, double *dev_norms, void *ws, size_t ws_bytes, hipStream_t stream);

/* One step of the staggered method (Section 4) on a window of the series.
 * The problem is truncated at order hi: b = -p(x) and A = p'(x) are computed
 * for the coefficients 0..hi-1 only (x's coefficients from hi on are not
 * read and not changed).  Once x_k is correct, b_k vanishes and dx_k need
 * not be computed, so only the stages lo..hi-1 are solved, with dx_k = 0
 * below lo:  A_0 dx_k = b_k - sum_{j=1..k-lo} A_j dx_{k-j},  lo <= k < hi;
 * x_k := x_k + dx_k for lo <= k < hi.  keep_factorization = 1 skips the QR
 * of A_0 and uses the factorization (as M = A_0^{-1}) that the last step
 * without it left in ws, computed at that step's x (Section 5.3: the QR is
 * done once, in the first stage); this makes a chord step.  It is the
 * caller's to ensure that such a step has run on the same plan, ws and
 * prec_solve; the result is undefined otherwise.  prec_solve as for
 * md_newton_step_mixed (the plan's precision: a plain step).  Status and
 * workspace as md_newton_step; dev_norms [2][D]: max |b_k| for k < hi, max
 * |dx_k| for lo <= k < hi, zero elsewhere.  lo = 0, hi = D,
 * keep_factorization = 0 is md_newton_step_mixed.  MD_EINVAL unless
 * 0 <= lo < hi <= D. */
int md_newton_step_window(const md_plan *plan, int prec_solve, int lo, int hi, int keep_factorization,
                          const double *cff, const double *cst, double *x, int32_t *dev_status, double *dev_norms,
                          void *ws, size_t ws_bytes, hipStream_t stream);

/* The order schedule of the staggered method (Section 4): the next order
 * after d, d + 1 + d/2 (integer division), capped at D.  Host only. */
int md_stagger_next_order(int d, int D);

/* Result of md_newton_staggered. */
typedef struct md_stagger_report {
  int32_t steps;          /* steps taken */
  int32_t converged;      /* 1: every coefficient met the tolerance */
  int32_t lo, hi;         /* window of the last step */
  int32_t factorizations; /* QR factorizations of A_0 computed */
} md_stagger_report;

/* Newton's method with the staggered progression of the order (Section 4),
 * driven from the host: the first step solves for x_0 alone (order 1; x_0
 * should carry about half the working precision, as the paper assumes), each
 * following step raises the order hi by md_stagger_next_order, and the stages
 * below lo are dropped once their residuals vanish: after each step, lo is
 * the number of leading coefficients k with |b_{i,k}| <= tol * s_{i,k} for
 * every equation i, where s_{i,k} = |c_{i,0,k}| + sum_m max_j |f_{m,j,k}| is
 * the size of the terms whose rounding errors reach b_{i,k}: the constant and,
 * per monomial, the largest coefficient k of the products f_j along its
 * forward chain (leading limbs; tol = 0 drops only exactly zero residuals),
 * or whose relative residual max_i |b_{i,k}| / s_{i,k} did not halve since
 * the previous step while below 2^(-40 L) (a Newton or chord step reduces it
 * far more, so it has reached the level of the rounding errors; the ceiling
 * keeps a slowly contracting chord iteration from freezing a coefficient far
 * above that level).  refactor_every_step = 0 factors
 * A_0 once, at the first step (Section 5.3), and makes every later step a
 * chord step; 1 factors at every step (Newton's method).  Stops when hi = D
 * and every coefficient meets the tolerance (converged = 1) or after
 * max_steps steps (converged = 0).  windows (host, nullable): [max_steps][2]
 * gets (lo, hi) of every step; rel (host, nullable) [D] gets the last step's
 * max_i |b_{i,k}| / s_{i,k} for k < hi (zero above).  The host waits for the stream after every
 * step (a few doubles are read back).  Arguments and workspace as
 * md_newton_step_window; dev_norms [2][D] is required.  A step whose status
 * is not MD_OK ends the run with that code. */
int md_newton_staggered(const md_plan *plan, int prec_solve, int refactor_every_step, int max_steps, double tol,
                        const double *cff, const double *cst, double *x, int32_t *windows, double *rel,
                        md_stagger_report *report, int32_t *dev_status, double *dev_norms, void *ws,
                        size_t ws_bytes, hipStream_t stream);

/* Residual of the lower triangular block Toeplitz system of Section 2 (what
 * the Newton loop of Section 2 reports; the residual kernels of Section 5.4
 * and Table 4), in multiple-double precision:
 *   r_{q,k} = b_{i,k} - sum_{j=0..k} sum_v A_j(i,v) dx_{v,k-j},  i = rows[q],
 * for q < nrows and k < D = d + 1.  rows (device int32, nrows entries)
 * selects the equations (Section 7.2 suggests a few random ones instead of
 * all, as the full residual costs about as much as the staged updates); NULL
 * takes every row in order (nrows must then be n).  A [L][n][n][D] as
 * md_eval_diff writes it, b and dx [L][n][D], r [L][nrows][D]; all device
 * arrays, precision prec = L.  norm1 (device, nullable) [D]: norm1[k] =
 * sum_q |r_{q,k}| on leading limbs.  A row index outside 0..n-1 sets
 * *dev_status (nullable) to MD_EINVAL and leaves that row of r unwritten. */
int md_linear_residual(int prec, int n, int d, const double *A, const double *b, const double *dx, int nrows,
                       const int32_t *rows, double *r, double *norm1, int32_t *dev_status, hipStream_t stream);

/* Device pointers into ws (the workspace of plan) where the last Newton step
 * run with it (md_newton_step, md_newton_step_mixed, md_newton_step_window)
 * left b = -p(x) at the step's input [L][n][D], the Jacobian series A
 * [L][n][n][D] and dx [L][n][D].  A and dx hold the step's solve precision
 * (their leading limbs); a window step leaves dx only on its window and b, A
 * only below its order.  With md_linear_residual they give the residual of
 * the step's linear system. */
int md_step_arrays(const md_plan *plan, void *ws, size_t ws_bytes, double **b, double **A, double **dx);

/* Complex data (Section 5.2).  Complex multiple-double arrays are
 * [2][L][...]: the real plane, then the imaginary plane, each laid out as the
 * real array (cff [2][L][m], cst and x [2][L][n][D], b [2][L][n][D], A
 * [2][L][n][n][D]).  The evaluation forms the four real products of every
 * complex convolution (the 4M method) side by side on the lanes of a worker.
 * Exponents must be 1 or 2 (MD_EINVAL otherwise).  md_complex_workspace_size
 * gives the bytes of ws for both calls.
 *
 * md_eval_diff_complex: b = -p(x) and A = p'(x) as md_eval_diff.
 * md_newton_step_complex: one Newton step (Section 2) in place on x; the
 * complex block Toeplitz system is solved through its real form of dimension
 * 2n, [[Re A_k, -Im A_k], [Im A_k, Re A_k]], by the real QR and staged solve
 * (2n <= MD_MAX_DIM); *dev_status as md_newton_step; dev_norms [2][D]
 * (nullable): the larger of the real and imaginary parts' max |b_k| and
 * max |dx_k|. */
int md_complex_workspace_size(const md_plan *plan, size_t *bytes);
int md_eval_diff_complex(const md_plan *plan, const double *cff, const double *cst, const double *x, double *b,
                         double *A, void *ws, size_t ws_bytes, hipStream_t stream);
int md_newton_step_complex(const md_plan *plan, const double *cff, const double *cst, double *x, int32_t *dev_status,
                           double *dev_norms, void *ws, size_t ws_bytes, hipStream_t stream);

/* Batches of independent systems ("paths"; the paper tracks many solution
 * paths of a homotopy, Section 1), one Newton step of every path per call,
 * in one persistent launch.  A path p has n_p (1..128) variables and
 * polynomials, truncation degree d_p (D_p = d_p + 1 <= MD_MAX_COEFFS) and
 * m_p monomials with exponents 1 or 2; precision double or quad double.
 *
 * md_batch_create: poly_ptr, mon_ptr, var and exp are the tables of
 * md_plan_create for each path, concatenated in path order (poly_ptr: n_p + 1
 * entries per path, each starting at 0; mon_ptr: m_p + 1 entries per path,
 * each starting at 0; var, exp: mon_ptr_p[m_p] entries per path, variable
 * indices local to the path).  Host pointers, copied.  MD_EINVAL on any
 * inconsistency.
 *
 * Packed device arrays: x and cst are [L][X] with path p's series block
 * [n_p][D_p] at element x_off[p] of each limb plane (X = x_total); cff is
 * [L][C] with path p's coefficients at cff_off[p] (C = cff_total), all from
 * md_batch_offsets.
 *
 * md_batch_newton_step: x := x + dx for every path, as md_newton_step
 * (prec_solve below the batch's precision: md_newton_step_mixed).
 * dev_status[p] is the path's status (MD_OK, MD_ESINGULAR, MD_ENONFINITE),
 * dev_norms[2p] = max |b| and dev_norms[2p+1] = max |dx| over the path's
 * series (leading limbs).  The workspace (md_batch_workspace_size) holds a
 * queue counter and one slot of intermediates per concurrent workgroup.
 * The call is asynchronous; it captures its launches in a graph on the
 * second call with the same arguments and replays the graph afterwards.
 * Not thread safe per batch.
 *
 * md_batch_autotune: for every size bucket of (n, D) present, times the
 * batched step of that bucket's paths with reduction teams of 4, 8 and 16
 * lanes on a scratch copy of x (x_scratch, [L][X]) and keeps the fastest;
 * chosen[9] (optional) receives the choice per bucket.  md_batch_set_tiles
 * sets them directly. */
typedef struct md_batch md_batch;
int md_batch_create(int prec, int npaths, const int32_t *n, const int32_t *d, const int32_t *m,
                    const int32_t *poly_ptr, const int32_t *mon_ptr, const int32_t *var, const int32_t *exp,
                    md_batch **out);
int md_batch_destroy(md_batch *batch);
int md_batch_offsets(const md_batch *batch, int64_t *x_off, int64_t *cff_off, int64_t *x_total, int64_t *cff_total);
int md_batch_workspace_size(const md_batch *batch, size_t *bytes);
int md_batch_newton_step(md_batch *batch, int prec_solve, const double *cff, const double *cst, double *x,
                         int32_t *dev_status, double *dev_norms, void *ws, size_t ws_bytes, hipStream_t stream);
int md_batch_autotune(md_batch *batch, int prec_solve, const double *cff, const double *cst, const double *x,
                      double *x_scratch, int32_t *dev_status, double *dev_norms, void *ws, size_t ws_bytes,
                      hipStream_t stream, int32_t *chosen);
int md_batch_set_tiles(md_batch *batch, const int32_t *tiles);

/* Elementwise multiple-double arithmetic on device arrays of count elements
 * (limb-major [L][count]): op 0 add, 1 sub, 2 mul, 3 div, 4 sqrt (of a),
 * 5 fused c := c + a*b; op 6 is the dot product c[0] = sum_q a[q] b[q]
 * (c is [L][1], summed in a fixed order).  b is not read for sqrt.
 * (Section 1.2 and Section 6: the inlined arithmetic, exposed for testing,
 * losses and callers.) */
int md_arith(int prec, int op, int64_t count, const double *a, const double *b, double *c, hipStream_t stream);

/* Adjoint of the Newton fixed point (for gradients of Taylor coefficients
 * with respect to the monomial coefficients).  With T the block Toeplitz
 * operator of Section 2 (A_0 on the diagonal, A_k on the k-th block
 * subdiagonal), solve T^T lambda = g, i.e. by blocks from the last
 * coefficient down:
 *   A_0^T lambda_j = g_j - sum_{i=1..d-j} A_i^T lambda_{j+i},  j = d..0,
 * with M = A_0^{-1} from the QR factors of md_qr (qr, tau) and the same
 * staged kernels as md_series_solve applied to M^T and A_k^T.
 * A [L][n][n][D]; g_lambda [L][n][D] holds g on entry and lambda on return. */
int md_adjoint_workspace_size(int prec, int n, int d, size_t *bytes);
int md_adjoint_solve(int prec, int n, int d, const double *qr, const double *tau, const double *A, double *g_lambda,
                     void *ws, size_t ws_bytes, hipStream_t stream, int32_t *dev_status);

/* grad_cff [L][m]: dL/dc_m = -sum_k lambda_{i(m),k} [x^{a_m}]_k, the gradient of
 * a loss L(x) at a solution x of p(x; c) = 0 given lambda from
 * md_adjoint_solve (dp_i/dc_m = x^{a_m} for the monomials of row i).  The
 * monomial values are evaluated by the convolution kernel with unit
 * coefficients.  Workspace as md_workspace_size. */
int md_coef_grad(const md_plan *plan, const double *x, const double *lambda, double *grad_cff, void *ws,
                 size_t ws_bytes, hipStream_t stream);

/* Per-kernel-class timing (the paper measures the time of each kernel type,
 * Section 7, Table 4).  While enabled, the library brackets each class of
 * launches of md_eval_diff, md_series_solve and md_newton_step with HIP events
 * on the caller's stream.  md_timing_read synchronizes those events, returns
 * the accumulated milliseconds and bracket counts per class in
 * ms[MD_NCLASSES] and launches[MD_NCLASSES], and resets them.  Not thread
 * safe: one timing client at a time. */
#define MD_CLASS_CONVOLUTIONS 0 /* power table and monomial eval/diff (convolutions) */
#define MD_CLASS_ASSEMBLY 1     /* sums into b(t) and A(t) */
#define MD_CLASS_QR 2           /* Householder QR of A_0 */
#define MD_CLASS_QHB_BS 3       /* Q^T and back substitution applied to unit vectors: M */
#define MD_CLASS_GEMM 4         /* N = M A_1 */
#define MD_CLASS_UPDATES 5      /* staged right-hand-side updates and stage solves */
#define MD_CLASS_X_UPDATE 6     /* x := x + dx and the norms */
#define MD_NCLASSES 7
int md_timing_enable(int on);
int md_timing_read(double *ms, int64_t *launches);

/* Message for the last host-side error of this thread. */
const char *md_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
