/*
 * Oracle for one Newton step on truncated power series (TEST INFRASTRUCTURE).
 *
 * A plain, slow, arbitrary-precision CPU implementation written from the
 * paper's definitions.  Only the tests, the smoke check and the CPU baseline
 * of the benchmark load it; the GPU library never does, and the two share no
 * code.  Every value is an MPFR number at ORA bits (four times the working
 * precision of the multiple doubles under test, unless the caller asks for
 * more).
 *
 * What it computes (Section 2, linearized series and Newton's method):
 *   b(t)  = -p(x(t)) mod t^D,
 *   A(t)  = dp/dx (x(t)) mod t^D,  A(t) = A_0 + A_1 t + ... + A_d t^d,
 *   the lower triangular block Toeplitz system with A_0 on the diagonal and
 *   A_k on the k-th block subdiagonal, solved by block forward substitution:
 *     dx_0 = A_0^{-1} b_0,  dx_k = A_0^{-1} (b_k - sum_{j=1..k} A_j dx_{k-j}),
 *   and the update x + dx.
 * The system is p_i(x) = c_{i,0}(t) + sum_m c_{i,m} x^{a_{i,m}}.
 *
 * Deliberate independence from any fast method:
 *   - every monomial value is the plain left-to-right truncated product of its
 *     coefficient and each factor repeated by its exponent (no reverse mode);
 *   - every derivative uses the product rule d/dx_j x^a = a_j x^{a - e_j},
 *     each as a product of its own;
 *   - A_0 is factored by Gaussian elimination with partial pivoting (the GPU
 *     uses Householder QR, Sections 1.1 and 5.3);
 *   - a truncated series product is the textbook sum c_s = sum_{i<=s} a_i b_{s-i}
 *     (Section 5.1, without the zero padding the paper uses on the GPU).
 *
 * Multiple-double inputs are limb-major arrays [L][...]; the value of one
 * multiple double is the exact sum of its limbs (Section 1.2: an unevaluated
 * sum of doubles).  Outputs are "expansions" of K doubles obtained by
 * repeated round-to-nearest of the remainder, so K*53 bits of the MPFR value
 * survive the export.
 */
#include <mpfr.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define ORA_OK 0
#define ORA_EINVAL (-1)
#define ORA_ESINGULAR (-2)
#define ORA_ENOMEM (-5)

static int g_inexact = 0; /* counts md inputs whose limb sum was not exact */
static int g_threads = 0;

int ora_set_threads(int t) { g_threads = t; return 0; }
int ora_get_threads(void) { return g_threads > 0 ? g_threads : omp_get_max_threads(); }
int ora_inexact_count(void) { return g_inexact; }

typedef struct {
  int n, D, m;
  const int32_t *pp, *mp, *var, *ex;
} sys_t;

static mpfr_t *vnew(size_t cnt, mpfr_prec_t p) {
  mpfr_t *v = (mpfr_t *)malloc((cnt ? cnt : 1) * sizeof(mpfr_t));
  if (!v) return NULL;
  for (size_t i = 0; i < cnt; ++i) {
    mpfr_init2(v[i], p);
    mpfr_set_zero(v[i], 1);
  }
  return v;
}

static void vfree(mpfr_t *v, size_t cnt) {
  if (!v) return;
  for (size_t i = 0; i < cnt; ++i) mpfr_clear(v[i]);
  free(v);
}

/* Exact value of one multiple double: the sum of its L limbs. */
static void md_get(mpfr_t r, const double *limbs, size_t stride, int L) {
  int inexact = mpfr_set_d(r, limbs[0], MPFR_RNDN);
  for (int l = 1; l < L; ++l) inexact |= mpfr_add_d(r, r, limbs[(size_t)l * stride], MPFR_RNDN);
  if (inexact) {
#pragma omp atomic
    g_inexact++;
  }
}

/* Export v as K doubles: each is the round-to-nearest of what remains. */
static void exp_put(double *out, size_t stride, int K, mpfr_t v, mpfr_t tmp) {
  mpfr_set(tmp, v, MPFR_RNDN);
  for (int l = 0; l < K; ++l) {
    double d = mpfr_get_d(tmp, MPFR_RNDN);
    out[(size_t)l * stride] = d;
    mpfr_sub_d(tmp, tmp, d, MPFR_RNDN);
  }
}

/* Truncated product c = a*b mod t^D: c_s = sum_{i=0..s} a_i b_{s-i}.
 * c must not alias a or b. */
static void ser_mul(mpfr_t *c, mpfr_t *a, mpfr_t *b, int D, mpfr_t t) {
  for (int s = 0; s < D; ++s) {
    mpfr_set_zero(c[s], 1);
    for (int i = 0; i <= s; ++i) {
      mpfr_mul(t, a[i], b[s - i], MPFR_RNDN);
      mpfr_add(c[s], c[s], t, MPFR_RNDN);
    }
  }
}

/* out = coef * prod_l x_{var_l}^{e_l} mod t^D, where entry `skip` (if >= 0)
 * has its exponent lowered by one.  Left to right over the support, each
 * variable repeated by its exponent.  tmp is a scratch series. */
static void mono_series(mpfr_t *out, mpfr_t coef, const int32_t *vars, const int32_t *exps, int k,
                        int skip, mpfr_t *const *X, int D, mpfr_t *tmp, mpfr_t t) {
  for (int s = 0; s < D; ++s) mpfr_set_zero(out[s], 1);
  mpfr_set(out[0], coef, MPFR_RNDN);
  for (int l = 0; l < k; ++l) {
    int e = exps[l] - (l == skip ? 1 : 0);
    for (int r = 0; r < e; ++r) {
      ser_mul(tmp, out, X[vars[l]], D, t);
      for (int s = 0; s < D; ++s) mpfr_swap(out[s], tmp[s]);
    }
  }
}

/* Evaluate rows [r0, r1): b = -(c_0 + sum_m value_m), A_k[i][j] = sum_m (d/dx_j value_m)_k.
 * b is [rows][D], A is [D][rows][n] (row-major per matrix), scale[rows] gets
 * max_s (|c_{i,0,s}| + sum_m |value_{m,s}|); terms (NULL to skip) gets each
 * |c_{i,0,s}| + sum_m |value_{m,s}| itself, [rows][D]. */
static void eval_rows_terms(const sys_t *S, mpfr_t *const *X, mpfr_t *const *C, mpfr_t *cff, int r0,
                            int r1, mpfr_t *b, mpfr_t *A, mpfr_t *scale, mpfr_t *terms, mpfr_prec_t prec) {
  const int D = S->D, n = S->n, rows = r1 - r0;
  for (size_t q = 0; q < (size_t)D * rows * n; ++q) mpfr_set_zero(A[q], 1);
#pragma omp parallel num_threads(ora_get_threads())
  {
    mpfr_t *val = vnew(D, prec), *tmp = vnew(D, prec), *absacc = vnew(D, prec);
    mpfr_t t, c2;
    mpfr_init2(t, prec);
    mpfr_init2(c2, prec);
#pragma omp for schedule(dynamic, 1)
    for (int i = r0; i < r1; ++i) {
      int ri = i - r0;
      for (int s = 0; s < D; ++s) {
        mpfr_set(b[(size_t)ri * D + s], C[i][s], MPFR_RNDN);
        mpfr_abs(absacc[s], C[i][s], MPFR_RNDN);
      }
      for (int mj = S->pp[i]; mj < S->pp[i + 1]; ++mj) {
        const int32_t *vs = S->var + S->mp[mj], *es = S->ex + S->mp[mj];
        int k = S->mp[mj + 1] - S->mp[mj];
        mono_series(val, cff[mj], vs, es, k, -1, X, D, tmp, t);
        for (int s = 0; s < D; ++s) {
          mpfr_add(b[(size_t)ri * D + s], b[(size_t)ri * D + s], val[s], MPFR_RNDN);
          mpfr_abs(t, val[s], MPFR_RNDN);
          mpfr_add(absacc[s], absacc[s], t, MPFR_RNDN);
        }
        /* product rule: d/dx_j (c x^a) = c a_j x^{a - e_j} */
        for (int l = 0; l < k; ++l) {
          mpfr_mul_si(c2, cff[mj], es[l], MPFR_RNDN);
          mono_series(val, c2, vs, es, k, l, X, D, tmp, t);
          for (int s = 0; s < D; ++s) {
            mpfr_t *a = &A[((size_t)s * rows + ri) * n + vs[l]];
            mpfr_add(*a, *a, val[s], MPFR_RNDN);
          }
        }
      }
      for (int s = 0; s < D; ++s) mpfr_neg(b[(size_t)ri * D + s], b[(size_t)ri * D + s], MPFR_RNDN);
      mpfr_set_zero(scale[ri], 1);
      for (int s = 0; s < D; ++s) mpfr_max(scale[ri], scale[ri], absacc[s], MPFR_RNDN);
      if (terms)
        for (int s = 0; s < D; ++s) mpfr_set(terms[(size_t)ri * D + s], absacc[s], MPFR_RNDN);
    }
    vfree(val, D);
    vfree(tmp, D);
    vfree(absacc, D);
    mpfr_clear(t);
    mpfr_clear(c2);
  }
}

static void eval_rows(const sys_t *S, mpfr_t *const *X, mpfr_t *const *C, mpfr_t *cff, int r0,
                      int r1, mpfr_t *b, mpfr_t *A, mpfr_t *scale, mpfr_prec_t prec) {
  eval_rows_terms(S, X, C, cff, r0, r1, b, A, scale, NULL, prec);
}

static int check_sys(const sys_t *S) {
  if (S->n < 1 || S->D < 1 || S->m < 0) return ORA_EINVAL;
  if (S->pp[0] != 0 || S->pp[S->n] != S->m || S->mp[0] != 0) return ORA_EINVAL;
  for (int i = 0; i < S->n; ++i)
    if (S->pp[i + 1] < S->pp[i]) return ORA_EINVAL;
  for (int j = 0; j < S->m; ++j) {
    if (S->mp[j + 1] < S->mp[j]) return ORA_EINVAL;
    for (int q = S->mp[j]; q < S->mp[j + 1]; ++q) {
      if (S->var[q] < 0 || S->var[q] >= S->n || S->ex[q] < 1) return ORA_EINVAL;
      if (q > S->mp[j] && S->var[q] <= S->var[q - 1]) return ORA_EINVAL;
    }
  }
  return ORA_OK;
}

/* Load limb-major inputs: x[L][n][D], cst[L][n][D], cff[L][m]. */
static void load_inputs(const sys_t *S, int L, const double *cff, const double *cst, const double *x,
                        mpfr_t ***Xo, mpfr_t ***Co, mpfr_t **Fo, mpfr_prec_t prec) {
  const int n = S->n, D = S->D, m = S->m;
  const size_t nD = (size_t)n * D;
  mpfr_t **X = (mpfr_t **)malloc(n * sizeof(mpfr_t *));
  mpfr_t **C = (mpfr_t **)malloc(n * sizeof(mpfr_t *));
  for (int i = 0; i < n; ++i) {
    X[i] = vnew(D, prec);
    C[i] = vnew(D, prec);
    for (int s = 0; s < D; ++s) {
      md_get(X[i][s], x + (size_t)i * D + s, nD, L);
      if (cst) md_get(C[i][s], cst + (size_t)i * D + s, nD, L);
    }
  }
  mpfr_t *F = vnew(m, prec);
  for (int j = 0; j < m; ++j) md_get(F[j], cff + j, m, L);
  *Xo = X;
  *Co = C;
  *Fo = F;
}

static void free_inputs(const sys_t *S, mpfr_t **X, mpfr_t **C, mpfr_t *F) {
  for (int i = 0; i < S->n; ++i) {
    vfree(X[i], S->D);
    vfree(C[i], S->D);
  }
  free(X);
  free(C);
  vfree(F, S->m);
}

/* ----- Gaussian elimination with partial pivoting on an n x n matrix ----- */

/* In place: M (row-major n x n) becomes L\U, perm records the row order.
 * Returns ORA_ESINGULAR on an exactly zero pivot. */
static int lu_factor(mpfr_t *M, int n, int *perm, mpfr_prec_t prec) {
  mpfr_t t, best;
  mpfr_init2(t, prec);
  mpfr_init2(best, prec);
  int rc = ORA_OK;
  for (int i = 0; i < n; ++i) perm[i] = i;
  for (int c = 0; c < n; ++c) {
    int p = c;
    mpfr_abs(best, M[(size_t)c * n + c], MPFR_RNDN);
    for (int r = c + 1; r < n; ++r) {
      mpfr_abs(t, M[(size_t)r * n + c], MPFR_RNDN);
      if (mpfr_cmp(t, best) > 0) {
        mpfr_set(best, t, MPFR_RNDN);
        p = r;
      }
    }
    if (mpfr_zero_p(best)) {
      rc = ORA_ESINGULAR;
      break;
    }
    if (p != c) {
      for (int j = 0; j < n; ++j) mpfr_swap(M[(size_t)c * n + j], M[(size_t)p * n + j]);
      int q = perm[c];
      perm[c] = perm[p];
      perm[p] = q;
    }
    for (int r = c + 1; r < n; ++r) {
      mpfr_t *l = &M[(size_t)r * n + c];
      mpfr_div(*l, *l, M[(size_t)c * n + c], MPFR_RNDN);
      for (int j = c + 1; j < n; ++j) {
        mpfr_mul(t, *l, M[(size_t)c * n + j], MPFR_RNDN);
        mpfr_sub(M[(size_t)r * n + j], M[(size_t)r * n + j], t, MPFR_RNDN);
      }
    }
  }
  mpfr_clear(t);
  mpfr_clear(best);
  return rc;
}

/* Solve (L U) y = P r in place in y (r given in y). */
static void lu_solve(mpfr_t *LU, int n, const int *perm, mpfr_t *y, mpfr_t *w, mpfr_t t) {
  for (int i = 0; i < n; ++i) mpfr_set(w[i], y[perm[i]], MPFR_RNDN);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < i; ++j) {
      mpfr_mul(t, LU[(size_t)i * n + j], w[j], MPFR_RNDN);
      mpfr_sub(w[i], w[i], t, MPFR_RNDN);
    }
  for (int i = n - 1; i >= 0; --i) {
    for (int j = i + 1; j < n; ++j) {
      mpfr_mul(t, LU[(size_t)i * n + j], w[j], MPFR_RNDN);
      mpfr_sub(w[i], w[i], t, MPFR_RNDN);
    }
    mpfr_div(w[i], w[i], LU[(size_t)i * n + i], MPFR_RNDN);
  }
  for (int i = 0; i < n; ++i) mpfr_set(y[i], w[i], MPFR_RNDN);
}

/* Block forward substitution on the lower triangular block Toeplitz system
 * (Section 2): dx_k = A_0^{-1} (b_k - sum_{j=1..k} A_j dx_{k-j}).
 * A is [D][n][n] row-major, b and dx are [n][D].  The diagonal block is A0:
 * A itself for Newton's method, or the leading matrix taken at an earlier
 * point when the factorization of the first stage is kept (Section 5.3, a
 * chord step).  Stages below lo are not solved: dx_k = 0 for k < lo
 * (Section 4, a coefficient whose residual vanishes gets no update); the
 * sums still run over every j, with those zeros. */
static int toeplitz_solve_window(mpfr_t *A, mpfr_t *A0, mpfr_t *b, mpfr_t *dx, int n, int D, int lo,
                                 mpfr_prec_t prec) {
  mpfr_t *LU = vnew((size_t)n * n, prec);
  int *perm = (int *)malloc(n * sizeof(int));
  for (size_t q = 0; q < (size_t)n * n; ++q) mpfr_set(LU[q], A0[q], MPFR_RNDN);
  int rc = lu_factor(LU, n, perm, prec);
  if (rc == ORA_OK) {
    mpfr_t *r = vnew(n, prec), *w = vnew(n, prec);
    mpfr_t t;
    mpfr_init2(t, prec);
    for (int k = 0; k < lo && k < D; ++k)
      for (int i = 0; i < n; ++i) mpfr_set_zero(dx[(size_t)i * D + k], 1);
    for (int k = lo; k < D; ++k) {
#pragma omp parallel for schedule(static) num_threads(ora_get_threads())
      for (int i = 0; i < n; ++i) {
        mpfr_t u;
        mpfr_init2(u, prec);
        mpfr_set(r[i], b[(size_t)i * D + k], MPFR_RNDN);
        for (int j = 1; j <= k; ++j)
          for (int v = 0; v < n; ++v) {
            mpfr_mul(u, A[((size_t)j * n + i) * n + v], dx[(size_t)v * D + (k - j)], MPFR_RNDN);
            mpfr_sub(r[i], r[i], u, MPFR_RNDN);
          }
        mpfr_clear(u);
      }
      lu_solve(LU, n, perm, r, w, t);
      for (int i = 0; i < n; ++i) mpfr_set(dx[(size_t)i * D + k], r[i], MPFR_RNDN);
    }
    vfree(r, n);
    vfree(w, n);
    mpfr_clear(t);
  }
  vfree(LU, (size_t)n * n);
  free(perm);
  return rc;
}

static int toeplitz_solve(mpfr_t *A, mpfr_t *b, mpfr_t *dx, int n, int D, mpfr_prec_t prec) {
  return toeplitz_solve_window(A, A, b, dx, n, D, 0, prec);
}

/* ---------------------------- exported API ------------------------------ */

/* Evaluate and differentiate rows [r0, r1) of the system at x.
 * Inputs: L-limb multiple doubles cff[L][m], cst[L][n][D], x[L][n][D].
 * Outputs (K-double expansions): b[K][rows][D], A[K][D][rows][n], scale[rows]
 * (a double: max_s |c_{i,0,s}| + sum_m |value_{m,s}|). */
int ora_eval(int prec_bits, int n, int D, int m, const int32_t *pp, const int32_t *mp,
             const int32_t *var, const int32_t *ex, int L, const double *cff, const double *cst,
             const double *x, int r0, int r1, int K, double *b_out, double *A_out,
             double *scale_out) {
  sys_t S = {n, D, m, pp, mp, var, ex};
  if (check_sys(&S) || r0 < 0 || r1 > n || r0 >= r1 || K < 1 || L < 1) return ORA_EINVAL;
  mpfr_prec_t prec = prec_bits;
  mpfr_t **X, **C, *F;
  load_inputs(&S, L, cff, cst, x, &X, &C, &F, prec);
  int rows = r1 - r0;
  mpfr_t *b = vnew((size_t)rows * D, prec), *A = vnew((size_t)D * rows * n, prec);
  mpfr_t *sc = vnew(rows, prec);
  eval_rows(&S, X, C, F, r0, r1, b, A, sc, prec);
  mpfr_t tmp;
  mpfr_init2(tmp, prec);
  for (size_t q = 0; q < (size_t)rows * D; ++q) exp_put(b_out + q, (size_t)rows * D, K, b[q], tmp);
  if (A_out)
    for (size_t q = 0; q < (size_t)D * rows * n; ++q)
      exp_put(A_out + q, (size_t)D * rows * n, K, A[q], tmp);
  for (int r = 0; r < rows; ++r) scale_out[r] = mpfr_get_d(sc[r], MPFR_RNDN);
  mpfr_clear(tmp);
  vfree(b, (size_t)rows * D);
  vfree(A, (size_t)D * rows * n);
  vfree(sc, rows);
  free_inputs(&S, X, C, F);
  return ORA_OK;
}

/* One Newton step from x (Section 2): x_new = x + dx with dx the solution of
 * the block Toeplitz system built from b = -p(x), A = p'(x).
 * Outputs (K-double expansions, NULL to skip): x_new[K][n][D], dx[K][n][D],
 * b[K][n][D], A[K][D][n][n]. */
int ora_newton_step(int prec_bits, int n, int D, int m, const int32_t *pp, const int32_t *mp,
                    const int32_t *var, const int32_t *ex, int L, const double *cff,
                    const double *cst, const double *x, int K, double *x_out, double *dx_out,
                    double *b_out, double *A_out) {
  sys_t S = {n, D, m, pp, mp, var, ex};
  if (check_sys(&S) || K < 1 || L < 1) return ORA_EINVAL;
  mpfr_prec_t prec = prec_bits;
  mpfr_t **X, **C, *F;
  load_inputs(&S, L, cff, cst, x, &X, &C, &F, prec);
  mpfr_t *b = vnew((size_t)n * D, prec), *A = vnew((size_t)D * n * n, prec), *sc = vnew(n, prec);
  mpfr_t *dx = vnew((size_t)n * D, prec);
  eval_rows(&S, X, C, F, 0, n, b, A, sc, prec);
  int rc = toeplitz_solve(A, b, dx, n, D, prec);
  if (rc == ORA_OK) {
    mpfr_t tmp, xn;
    mpfr_init2(tmp, prec);
    mpfr_init2(xn, prec);
    const size_t nD = (size_t)n * D;
    for (int i = 0; i < n; ++i)
      for (int s = 0; s < D; ++s) {
        size_t q = (size_t)i * D + s;
        mpfr_add(xn, X[i][s], dx[q], MPFR_RNDN);
        if (x_out) exp_put(x_out + q, nD, K, xn, tmp);
        if (dx_out) exp_put(dx_out + q, nD, K, dx[q], tmp);
        if (b_out) exp_put(b_out + q, nD, K, b[q], tmp);
      }
    if (A_out)
      for (size_t q = 0; q < (size_t)D * n * n; ++q) exp_put(A_out + q, (size_t)D * n * n, K, A[q], tmp);
    mpfr_clear(tmp);
    mpfr_clear(xn);
  }
  vfree(b, (size_t)n * D);
  vfree(A, (size_t)D * n * n);
  vfree(sc, n);
  vfree(dx, (size_t)n * D);
  free_inputs(&S, X, C, F);
  return rc;
}

/* One step of the staggered method (Sections 4 and 5.3).  The caller passes
 * series truncated at the step's order, D coefficients (x, cst [L][n][D]), so
 * b = -p(x) mod t^D and A = p'(x) mod t^D.  The diagonal block of the solve
 * is A_0 taken at the leading coefficients xs0 [L][n] (the point where the
 * factorization was computed; NULL: x's own, Newton's method); stages below
 * lo get no update.  Outputs (K-double expansions, NULL to skip): x + dx,
 * dx, b as [K][n][D]; scale[D] (doubles) gets max_i (|c_{i,0,k}| +
 * sum_m |value_{m,k}|), the size of the terms that cancel in b_k. */
int ora_window_step(int prec_bits, int n, int D, int m, const int32_t *pp, const int32_t *mp,
                    const int32_t *var, const int32_t *ex, int L, const double *cff,
                    const double *cst, const double *x, const double *xs0, int lo, int K,
                    double *x_out, double *dx_out, double *b_out, double *scale_out) {
  sys_t S = {n, D, m, pp, mp, var, ex};
  if (check_sys(&S) || K < 1 || L < 1 || lo < 0 || lo >= D) return ORA_EINVAL;
  mpfr_prec_t prec = prec_bits;
  mpfr_t **X, **C, *F;
  load_inputs(&S, L, cff, cst, x, &X, &C, &F, prec);
  const size_t nD = (size_t)n * D, nn = (size_t)n * n;
  mpfr_t *b = vnew(nD, prec), *A = vnew((size_t)D * nn, prec), *sc = vnew(n, prec);
  mpfr_t *terms = vnew(nD, prec), *dx = vnew(nD, prec);
  eval_rows_terms(&S, X, C, F, 0, n, b, A, sc, terms, prec);
  mpfr_t *A0 = A;
  mpfr_t *As = NULL, *bs = NULL, *scs = NULL;
  if (xs0) {  /* A_0 at the kept point: the Jacobian of the order-1 truncation there */
    sys_t S1 = {n, 1, m, pp, mp, var, ex};
    mpfr_t **X1, **C1, *F1;
    load_inputs(&S1, L, cff, NULL, xs0, &X1, &C1, &F1, prec);
    As = vnew(nn, prec);
    bs = vnew(n, prec);
    scs = vnew(n, prec);
    eval_rows(&S1, X1, C1, F1, 0, n, bs, As, scs, prec);
    free_inputs(&S1, X1, C1, F1);
    A0 = As;
  }
  int rc = toeplitz_solve_window(A, A0, b, dx, n, D, lo, prec);
  if (rc == ORA_OK) {
    mpfr_t tmp, xn, mx;
    mpfr_init2(tmp, prec);
    mpfr_init2(xn, prec);
    mpfr_init2(mx, prec);
    for (int i = 0; i < n; ++i)
      for (int s2 = 0; s2 < D; ++s2) {
        size_t q = (size_t)i * D + s2;
        mpfr_add(xn, X[i][s2], dx[q], MPFR_RNDN);
        if (x_out) exp_put(x_out + q, nD, K, xn, tmp);
        if (dx_out) exp_put(dx_out + q, nD, K, dx[q], tmp);
        if (b_out) exp_put(b_out + q, nD, K, b[q], tmp);
      }
    if (scale_out)
      for (int s2 = 0; s2 < D; ++s2) {
        mpfr_set_zero(mx, 1);
        for (int i = 0; i < n; ++i) mpfr_max(mx, mx, terms[(size_t)i * D + s2], MPFR_RNDN);
        scale_out[s2] = mpfr_get_d(mx, MPFR_RNDN);
      }
    mpfr_clear(tmp);
    mpfr_clear(xn);
    mpfr_clear(mx);
  }
  if (As) {
    vfree(As, nn);
    vfree(bs, n);
    vfree(scs, n);
  }
  vfree(b, nD);
  vfree(A, (size_t)D * nn);
  vfree(sc, n);
  vfree(terms, nD);
  vfree(dx, nD);
  free_inputs(&S, X, C, F);
  return rc;
}

/* Residual of the block Toeplitz system (the quantity Newton's loop of
 * Section 2 monitors; the residual kernels of Section 5.4 and Table 4):
 *   r_{i,k} = b_{i,k} - sum_{j=0..k} sum_v A_j(i,v) dx_{v,k-j}
 * for the rows listed in rows[nrows] (every row when rows is NULL).
 * A is [L][D][n][n] row-major per coefficient, b and dx are [L][n][D].
 * Outputs: r_out[K][nrows][D] (expansions), scale_out[nrows][D] (doubles):
 * |b_{i,k}| + sum_j sum_v |A_j(i,v)| |dx_{v,k-j}|, the size of the terms. */
int ora_linear_residual(int prec_bits, int n, int D, int L, const double *A, const double *b, const double *dx,
                        int nrows, const int32_t *rows, int K, double *r_out, double *scale_out) {
  if (n < 1 || D < 1 || K < 1 || L < 1 || nrows < 1) return ORA_EINVAL;
  for (int q = 0; rows && q < nrows; ++q)
    if (rows[q] < 0 || rows[q] >= n) return ORA_EINVAL;
  mpfr_prec_t prec = prec_bits;
  const size_t nn = (size_t)n * n, tot = (size_t)D * nn, nD = (size_t)n * D, rD = (size_t)nrows * D;
  mpfr_t *Am = vnew(tot, prec), *bm = vnew(nD, prec), *xm = vnew(nD, prec);
  for (size_t q = 0; q < tot; ++q) md_get(Am[q], A + q, tot, L);
  for (size_t q = 0; q < nD; ++q) {
    md_get(bm[q], b + q, nD, L);
    md_get(xm[q], dx + q, nD, L);
  }
#pragma omp parallel for schedule(dynamic, 1) num_threads(ora_get_threads())
  for (int ri = 0; ri < nrows; ++ri) {
    const int i = rows ? rows[ri] : ri;
    mpfr_t r, t, sc, at;
    mpfr_init2(r, prec);
    mpfr_init2(t, prec);
    mpfr_init2(sc, prec);
    mpfr_init2(at, prec);
    for (int k = 0; k < D; ++k) {
      mpfr_set(r, bm[(size_t)i * D + k], MPFR_RNDN);
      mpfr_abs(sc, r, MPFR_RNDN);
      for (int j = 0; j <= k; ++j)
        for (int v = 0; v < n; ++v) {
          mpfr_mul(t, Am[(size_t)j * nn + (size_t)i * n + v], xm[(size_t)v * D + (k - j)], MPFR_RNDN);
          mpfr_sub(r, r, t, MPFR_RNDN);
          mpfr_abs(at, t, MPFR_RNDN);
          mpfr_add(sc, sc, at, MPFR_RNDN);
        }
      exp_put(r_out + (size_t)ri * D + k, rD, K, r, t);
      scale_out[(size_t)ri * D + k] = mpfr_get_d(sc, MPFR_RNDN);
    }
    mpfr_clear(r);
    mpfr_clear(t);
    mpfr_clear(sc);
    mpfr_clear(at);
  }
  vfree(Am, tot);
  vfree(bm, nD);
  vfree(xm, nD);
  return ORA_OK;
}

/* ------------------ complex data (Section 5.2: complex series) ------------
 * A complex number is a pair of MPFR numbers, a complex array a pair of
 * arrays.  Inputs are [2][L][...]: the real plane, then the imaginary plane;
 * outputs [2][K][...].  The product is the textbook one,
 * (a + ib)(c + id) = (ac - bd) + i(ad + bc). */

/* r = a * b (r must not alias a or b). */
static void cmul(mpfr_t rr, mpfr_t ri, mpfr_t ar, mpfr_t ai, mpfr_t br, mpfr_t bi, mpfr_t t1, mpfr_t t2) {
  mpfr_mul(t1, ar, br, MPFR_RNDN);
  mpfr_mul(t2, ai, bi, MPFR_RNDN);
  mpfr_sub(rr, t1, t2, MPFR_RNDN);
  mpfr_mul(t1, ar, bi, MPFR_RNDN);
  mpfr_mul(t2, ai, br, MPFR_RNDN);
  mpfr_add(ri, t1, t2, MPFR_RNDN);
}

/* Truncated complex product c = a * b mod t^D (c must not alias a or b). */
static void cser_mul(mpfr_t *cr, mpfr_t *ci, mpfr_t *ar, mpfr_t *ai, mpfr_t *br, mpfr_t *bi, int D, mpfr_t *w) {
  for (int s = 0; s < D; ++s) {
    mpfr_set_zero(cr[s], 1);
    mpfr_set_zero(ci[s], 1);
    for (int i = 0; i <= s; ++i) {
      cmul(w[0], w[1], ar[i], ai[i], br[s - i], bi[s - i], w[2], w[3]);
      mpfr_add(cr[s], cr[s], w[0], MPFR_RNDN);
      mpfr_add(ci[s], ci[s], w[1], MPFR_RNDN);
    }
  }
}

/* out = coef * prod_l x_{var_l}^{e_l} mod t^D with entry `skip` (if >= 0)
 * lowered by one; tmp a scratch pair of series, w four scratch numbers. */
static void cmono_series(mpfr_t *outr, mpfr_t *outi, mpfr_t cr, mpfr_t ci, const int32_t *vars, const int32_t *exps,
                         int k, int skip, mpfr_t *const *Xr, mpfr_t *const *Xi, int D, mpfr_t *tr, mpfr_t *ti,
                         mpfr_t *w) {
  for (int s = 0; s < D; ++s) {
    mpfr_set_zero(outr[s], 1);
    mpfr_set_zero(outi[s], 1);
  }
  mpfr_set(outr[0], cr, MPFR_RNDN);
  mpfr_set(outi[0], ci, MPFR_RNDN);
  for (int l = 0; l < k; ++l) {
    int e = exps[l] - (l == skip ? 1 : 0);
    for (int r = 0; r < e; ++r) {
      cser_mul(tr, ti, outr, outi, Xr[vars[l]], Xi[vars[l]], D, w);
      for (int s = 0; s < D; ++s) {
        mpfr_swap(outr[s], tr[s]);
        mpfr_swap(outi[s], ti[s]);
      }
    }
  }
}

/* b = -(c_0 + sum_m value_m) and A_k[i][j] = sum_m (d/dx_j value_m)_k on every
 * row; b [2][n][D], A [2][D][n][n]. */
static void ceval_rows(const sys_t *S, mpfr_t *const *Xr, mpfr_t *const *Xi, mpfr_t *const *Cr, mpfr_t *const *Ci,
                       mpfr_t *Fr, mpfr_t *Fi, mpfr_t *br, mpfr_t *bi, mpfr_t *Ar, mpfr_t *Ai, mpfr_prec_t prec) {
  const int D = S->D, n = S->n;
  for (size_t q = 0; q < (size_t)D * n * n; ++q) {
    mpfr_set_zero(Ar[q], 1);
    mpfr_set_zero(Ai[q], 1);
  }
#pragma omp parallel num_threads(ora_get_threads())
  {
    mpfr_t *vr = vnew(D, prec), *vi = vnew(D, prec), *tr = vnew(D, prec), *ti = vnew(D, prec), *w = vnew(4, prec);
    mpfr_t c2r, c2i;
    mpfr_init2(c2r, prec);
    mpfr_init2(c2i, prec);
#pragma omp for schedule(dynamic, 1)
    for (int i = 0; i < n; ++i) {
      for (int s = 0; s < D; ++s) {
        mpfr_set(br[(size_t)i * D + s], Cr[i][s], MPFR_RNDN);
        mpfr_set(bi[(size_t)i * D + s], Ci[i][s], MPFR_RNDN);
      }
      for (int mj = S->pp[i]; mj < S->pp[i + 1]; ++mj) {
        const int32_t *vs = S->var + S->mp[mj], *es = S->ex + S->mp[mj];
        int k = S->mp[mj + 1] - S->mp[mj];
        cmono_series(vr, vi, Fr[mj], Fi[mj], vs, es, k, -1, Xr, Xi, D, tr, ti, w);
        for (int s = 0; s < D; ++s) {
          mpfr_add(br[(size_t)i * D + s], br[(size_t)i * D + s], vr[s], MPFR_RNDN);
          mpfr_add(bi[(size_t)i * D + s], bi[(size_t)i * D + s], vi[s], MPFR_RNDN);
        }
        for (int l = 0; l < k; ++l) {  /* d/dx_j (c x^a) = c a_j x^{a - e_j} */
          mpfr_mul_si(c2r, Fr[mj], es[l], MPFR_RNDN);
          mpfr_mul_si(c2i, Fi[mj], es[l], MPFR_RNDN);
          cmono_series(vr, vi, c2r, c2i, vs, es, k, l, Xr, Xi, D, tr, ti, w);
          for (int s = 0; s < D; ++s) {
            size_t q = ((size_t)s * n + i) * n + vs[l];
            mpfr_add(Ar[q], Ar[q], vr[s], MPFR_RNDN);
            mpfr_add(Ai[q], Ai[q], vi[s], MPFR_RNDN);
          }
        }
      }
      for (int s = 0; s < D; ++s) {
        mpfr_neg(br[(size_t)i * D + s], br[(size_t)i * D + s], MPFR_RNDN);
        mpfr_neg(bi[(size_t)i * D + s], bi[(size_t)i * D + s], MPFR_RNDN);
      }
    }
    vfree(vr, D);
    vfree(vi, D);
    vfree(tr, D);
    vfree(ti, D);
    vfree(w, 4);
    mpfr_clear(c2r);
    mpfr_clear(c2i);
  }
}

/* Complex Gaussian elimination with partial pivoting (largest |re| + |im|)
 * on an n x n row-major pair; returns ORA_ESINGULAR on a zero pivot. */
static int clu_factor(mpfr_t *Mr, mpfr_t *Mi, int n, int *perm, mpfr_prec_t prec) {
  mpfr_t t, best, den, qr, qi, w[4];
  mpfr_inits2(prec, t, best, den, qr, qi, w[0], w[1], w[2], w[3], (mpfr_ptr)0);
  int rc = ORA_OK;
  for (int i = 0; i < n; ++i) perm[i] = i;
  for (int c = 0; c < n && rc == ORA_OK; ++c) {
    int piv = c;
    mpfr_set_zero(best, 1);
    for (int r = c; r < n; ++r) {
      mpfr_abs(t, Mr[(size_t)r * n + c], MPFR_RNDN);
      mpfr_abs(den, Mi[(size_t)r * n + c], MPFR_RNDN);
      mpfr_add(t, t, den, MPFR_RNDN);
      if (mpfr_cmp(t, best) > 0) {
        mpfr_set(best, t, MPFR_RNDN);
        piv = r;
      }
    }
    if (mpfr_zero_p(best)) {
      rc = ORA_ESINGULAR;
      break;
    }
    if (piv != c) {
      for (int j = 0; j < n; ++j) {
        mpfr_swap(Mr[(size_t)c * n + j], Mr[(size_t)piv * n + j]);
        mpfr_swap(Mi[(size_t)c * n + j], Mi[(size_t)piv * n + j]);
      }
      int tp = perm[c];
      perm[c] = perm[piv];
      perm[piv] = tp;
    }
    mpfr_t *pr = &Mr[(size_t)c * n + c], *pi = &Mi[(size_t)c * n + c];
    mpfr_sqr(den, *pr, MPFR_RNDN);
    mpfr_sqr(t, *pi, MPFR_RNDN);
    mpfr_add(den, den, t, MPFR_RNDN);
    for (int r = c + 1; r < n; ++r) {
      /* l = M[r][c] / p = a conj(p) / |p|^2, a conj(p) = (ar pr + ai pi) + i (ai pr - ar pi) */
      mpfr_mul(w[0], Mr[(size_t)r * n + c], *pr, MPFR_RNDN);
      mpfr_mul(w[1], Mi[(size_t)r * n + c], *pi, MPFR_RNDN);
      mpfr_add(qr, w[0], w[1], MPFR_RNDN);
      mpfr_mul(w[0], Mi[(size_t)r * n + c], *pr, MPFR_RNDN);
      mpfr_mul(w[1], Mr[(size_t)r * n + c], *pi, MPFR_RNDN);
      mpfr_sub(qi, w[0], w[1], MPFR_RNDN);
      mpfr_div(qr, qr, den, MPFR_RNDN);
      mpfr_div(qi, qi, den, MPFR_RNDN);
      mpfr_set(Mr[(size_t)r * n + c], qr, MPFR_RNDN);
      mpfr_set(Mi[(size_t)r * n + c], qi, MPFR_RNDN);
      for (int j = c + 1; j < n; ++j) {
        cmul(w[2], w[3], qr, qi, Mr[(size_t)c * n + j], Mi[(size_t)c * n + j], w[0], w[1]);
        mpfr_sub(Mr[(size_t)r * n + j], Mr[(size_t)r * n + j], w[2], MPFR_RNDN);
        mpfr_sub(Mi[(size_t)r * n + j], Mi[(size_t)r * n + j], w[3], MPFR_RNDN);
      }
    }
  }
  mpfr_clears(t, best, den, qr, qi, w[0], w[1], w[2], w[3], (mpfr_ptr)0);
  return rc;
}

/* Solve (LU) y = rhs in place (y [n] pairs), with the row order of perm. */
static void clu_solve(mpfr_t *LUr, mpfr_t *LUi, int n, const int *perm, mpfr_t *yr, mpfr_t *yi, mpfr_prec_t prec) {
  mpfr_t *zr = vnew(n, prec), *zi = vnew(n, prec), *w = vnew(6, prec);
  for (int i = 0; i < n; ++i) {
    mpfr_set(zr[i], yr[perm[i]], MPFR_RNDN);
    mpfr_set(zi[i], yi[perm[i]], MPFR_RNDN);
  }
  for (int i = 0; i < n; ++i) /* forward, unit lower */
    for (int j = 0; j < i; ++j) {
      cmul(w[0], w[1], LUr[(size_t)i * n + j], LUi[(size_t)i * n + j], zr[j], zi[j], w[2], w[3]);
      mpfr_sub(zr[i], zr[i], w[0], MPFR_RNDN);
      mpfr_sub(zi[i], zi[i], w[1], MPFR_RNDN);
    }
  for (int i = n - 1; i >= 0; --i) { /* backward */
    for (int j = i + 1; j < n; ++j) {
      cmul(w[0], w[1], LUr[(size_t)i * n + j], LUi[(size_t)i * n + j], zr[j], zi[j], w[2], w[3]);
      mpfr_sub(zr[i], zr[i], w[0], MPFR_RNDN);
      mpfr_sub(zi[i], zi[i], w[1], MPFR_RNDN);
    }
    /* z_i / U_ii = z_i conj(u) / |u|^2 */
    mpfr_t *ur = &LUr[(size_t)i * n + i], *ui = &LUi[(size_t)i * n + i];
    mpfr_sqr(w[4], *ur, MPFR_RNDN);
    mpfr_sqr(w[5], *ui, MPFR_RNDN);
    mpfr_add(w[4], w[4], w[5], MPFR_RNDN);
    mpfr_mul(w[0], zr[i], *ur, MPFR_RNDN);
    mpfr_mul(w[1], zi[i], *ui, MPFR_RNDN);
    mpfr_add(w[2], w[0], w[1], MPFR_RNDN);
    mpfr_mul(w[0], zi[i], *ur, MPFR_RNDN);
    mpfr_mul(w[1], zr[i], *ui, MPFR_RNDN);
    mpfr_sub(w[3], w[0], w[1], MPFR_RNDN);
    mpfr_div(zr[i], w[2], w[4], MPFR_RNDN);
    mpfr_div(zi[i], w[3], w[4], MPFR_RNDN);
  }
  for (int i = 0; i < n; ++i) {
    mpfr_set(yr[i], zr[i], MPFR_RNDN);
    mpfr_set(yi[i], zi[i], MPFR_RNDN);
  }
  vfree(zr, n);
  vfree(zi, n);
  vfree(w, 6);
}

/* Block forward substitution on the complex block Toeplitz system (Section
 * 2): dx_k = A_0^{-1} (b_k - sum_{j=1..k} A_j dx_{k-j}). */
static int ctoeplitz_solve(mpfr_t *Ar, mpfr_t *Ai, mpfr_t *br, mpfr_t *bi, mpfr_t *xr, mpfr_t *xi, int n, int D,
                           mpfr_prec_t prec) {
  const size_t nn = (size_t)n * n;
  mpfr_t *LUr = vnew(nn, prec), *LUi = vnew(nn, prec), *rr = vnew(n, prec), *ri = vnew(n, prec), *w = vnew(4, prec);
  int *perm = (int *)malloc(n * sizeof(int));
  for (size_t q = 0; q < nn; ++q) {
    mpfr_set(LUr[q], Ar[q], MPFR_RNDN);
    mpfr_set(LUi[q], Ai[q], MPFR_RNDN);
  }
  int rc = clu_factor(LUr, LUi, n, perm, prec);
  for (int k = 0; k < D && rc == ORA_OK; ++k) {
    for (int i = 0; i < n; ++i) {
      mpfr_set(rr[i], br[(size_t)i * D + k], MPFR_RNDN);
      mpfr_set(ri[i], bi[(size_t)i * D + k], MPFR_RNDN);
      for (int j = 1; j <= k; ++j)
        for (int v = 0; v < n; ++v) {
          size_t a = (size_t)j * nn + (size_t)i * n + v, x = (size_t)v * D + (k - j);
          cmul(w[0], w[1], Ar[a], Ai[a], xr[x], xi[x], w[2], w[3]);
          mpfr_sub(rr[i], rr[i], w[0], MPFR_RNDN);
          mpfr_sub(ri[i], ri[i], w[1], MPFR_RNDN);
        }
    }
    clu_solve(LUr, LUi, n, perm, rr, ri, prec);
    for (int i = 0; i < n; ++i) {
      mpfr_set(xr[(size_t)i * D + k], rr[i], MPFR_RNDN);
      mpfr_set(xi[(size_t)i * D + k], ri[i], MPFR_RNDN);
    }
  }
  vfree(LUr, nn);
  vfree(LUi, nn);
  vfree(rr, n);
  vfree(ri, n);
  vfree(w, 4);
  free(perm);
  return rc;
}

/* Complex evaluation, differentiation and (optionally) one Newton step.
 * Inputs [2][L][...]: cff [m], cst and x [n][D].  Outputs (NULL to skip) as
 * [2][K][...] expansions: b [n][D], A [D][n][n], x + dx and dx [n][D]. */
int ora_complex_step(int prec_bits, int n, int D, int m, const int32_t *pp, const int32_t *mp, const int32_t *var,
                     const int32_t *ex, int L, const double *cff, const double *cst, const double *x, int K,
                     double *b_out, double *A_out, double *x_out, double *dx_out) {
  sys_t S = {n, D, m, pp, mp, var, ex};
  if (check_sys(&S) || K < 1 || L < 1) return ORA_EINVAL;
  mpfr_prec_t prec = prec_bits;
  const size_t nD = (size_t)n * D, nn = (size_t)n * n, DA = (size_t)D * nn;
  mpfr_t **Xr, **Cr, *Fr, **Xi, **Ci, *Fi;
  load_inputs(&S, L, cff, cst, x, &Xr, &Cr, &Fr, prec);
  load_inputs(&S, L, cff + (size_t)L * m, cst + (size_t)L * nD, x + (size_t)L * nD, &Xi, &Ci, &Fi, prec);
  mpfr_t *br = vnew(nD, prec), *bi = vnew(nD, prec), *Ar = vnew(DA, prec), *Ai = vnew(DA, prec);
  ceval_rows(&S, Xr, Xi, Cr, Ci, Fr, Fi, br, bi, Ar, Ai, prec);
  mpfr_t tmp;
  mpfr_init2(tmp, prec);
  int rc = ORA_OK;
  for (size_t q = 0; b_out && q < nD; ++q) {
    exp_put(b_out + q, nD, K, br[q], tmp);
    exp_put(b_out + (size_t)K * nD + q, nD, K, bi[q], tmp);
  }
  for (size_t q = 0; A_out && q < DA; ++q) {
    exp_put(A_out + q, DA, K, Ar[q], tmp);
    exp_put(A_out + (size_t)K * DA + q, DA, K, Ai[q], tmp);
  }
  if (x_out || dx_out) {
    mpfr_t *dxr = vnew(nD, prec), *dxi = vnew(nD, prec), xn;
    mpfr_init2(xn, prec);
    rc = ctoeplitz_solve(Ar, Ai, br, bi, dxr, dxi, n, D, prec);
    for (int i = 0; i < n && rc == ORA_OK; ++i)
      for (int s2 = 0; s2 < D; ++s2) {
        size_t q = (size_t)i * D + s2;
        if (x_out) {
          mpfr_add(xn, Xr[i][s2], dxr[q], MPFR_RNDN);
          exp_put(x_out + q, nD, K, xn, tmp);
          mpfr_add(xn, Xi[i][s2], dxi[q], MPFR_RNDN);
          exp_put(x_out + (size_t)K * nD + q, nD, K, xn, tmp);
        }
        if (dx_out) {
          exp_put(dx_out + q, nD, K, dxr[q], tmp);
          exp_put(dx_out + (size_t)K * nD + q, nD, K, dxi[q], tmp);
        }
      }
    vfree(dxr, nD);
    vfree(dxi, nD);
    mpfr_clear(xn);
  }
  mpfr_clear(tmp);
  vfree(br, nD);
  vfree(bi, nD);
  vfree(Ar, DA);
  vfree(Ai, DA);
  free_inputs(&S, Xr, Cr, Fr);
  free_inputs(&S, Xi, Ci, Fi);
  return rc;
}

/* Solve the block Toeplitz system for given A[L][D][n][n] (row-major) and
 * rhs[L][n][D]; dx[K][n][D].  Used for the standalone series solve. */
int ora_toeplitz_solve(int prec_bits, int n, int D, int L, const double *A, const double *rhs, int K,
                       double *dx_out) {
  if (n < 1 || D < 1 || K < 1 || L < 1) return ORA_EINVAL;
  mpfr_prec_t prec = prec_bits;
  const size_t nn = (size_t)n * n, tot = (size_t)D * nn, nD = (size_t)n * D;
  mpfr_t *Am = vnew(tot, prec), *b = vnew(nD, prec), *dx = vnew(nD, prec);
  for (size_t q = 0; q < tot; ++q) md_get(Am[q], A + q, tot, L);
  for (size_t q = 0; q < nD; ++q) md_get(b[q], rhs + q, nD, L);
  int rc = toeplitz_solve(Am, b, dx, n, D, prec);
  if (rc == ORA_OK) {
    mpfr_t tmp;
    mpfr_init2(tmp, prec);
    for (size_t q = 0; q < nD; ++q) exp_put(dx_out + q, nD, K, dx[q], tmp);
    mpfr_clear(tmp);
  }
  vfree(Am, tot);
  vfree(b, nD);
  vfree(dx, nD);
  return rc;
}

/* Manufactured right-hand side: c_{i,0}(t) = -sum_m c_m x*(t)^{a_m} mod t^D,
 * rounded to Lout limbs (round-to-nearest of each remainder), so that x* is a
 * solution of the rounded system up to that rounding.  cst_out[Lout][n][D]. */
int ora_manufacture(int prec_bits, int n, int D, int m, const int32_t *pp, const int32_t *mp,
                    const int32_t *var, const int32_t *ex, int L, const double *cff,
                    const double *xstar, int Lout, double *cst_out) {
  sys_t S = {n, D, m, pp, mp, var, ex};
  if (check_sys(&S)) return ORA_EINVAL;
  mpfr_prec_t prec = prec_bits;
  mpfr_t **X, **C, *F;
  load_inputs(&S, L, cff, NULL, xstar, &X, &C, &F, prec);
  const size_t nD = (size_t)n * D;
#pragma omp parallel num_threads(ora_get_threads())
  {
    mpfr_t *val = vnew(D, prec), *tmp = vnew(D, prec), *acc = vnew(D, prec);
    mpfr_t t;
    mpfr_init2(t, prec);
#pragma omp for schedule(dynamic, 1)
    for (int i = 0; i < n; ++i) {
      for (int s = 0; s < D; ++s) mpfr_set_zero(acc[s], 1);
      for (int mj = pp[i]; mj < pp[i + 1]; ++mj) {
        mono_series(val, F[mj], var + mp[mj], ex + mp[mj], mp[mj + 1] - mp[mj], -1, X, D, tmp, t);
        for (int s = 0; s < D; ++s) mpfr_add(acc[s], acc[s], val[s], MPFR_RNDN);
      }
      for (int s = 0; s < D; ++s) {
        mpfr_neg(acc[s], acc[s], MPFR_RNDN);
        exp_put(cst_out + (size_t)i * D + s, nD, Lout, acc[s], t);
      }
    }
    vfree(val, D);
    vfree(tmp, D);
    vfree(acc, D);
    mpfr_clear(t);
  }
  free_inputs(&S, X, C, F);
  return ORA_OK;
}

/* Round K-double expansions to Lout limbs (round-to-nearest of each
 * remainder); in[K][count], out[Lout][count]. */
int ora_round(int prec_bits, int K, const double *in, int count, int Lout, double *out) {
  mpfr_t v, t;
  mpfr_init2(v, prec_bits);
  mpfr_init2(t, prec_bits);
  for (int q = 0; q < count; ++q) {
    md_get(v, in + q, count, K);
    exp_put(out + q, count, Lout, v, t);
  }
  mpfr_clear(v);
  mpfr_clear(t);
  return ORA_OK;
}

/* |u - w| for two expansions u[Lu][count], w[Lw][count], rounded to double. */
int ora_absdiff(int prec_bits, int Lu, const double *u, int Lw, const double *w, int count,
                double *out) {
#pragma omp parallel num_threads(ora_get_threads())
  {
    mpfr_t a, c;
    mpfr_init2(a, prec_bits);
    mpfr_init2(c, prec_bits);
#pragma omp for schedule(static)
    for (int q = 0; q < count; ++q) {
      md_get(a, u + q, count, Lu);
      md_get(c, w + q, count, Lw);
      mpfr_sub(a, a, c, MPFR_RNDN);
      out[q] = fabs(mpfr_get_d(a, MPFR_RNDN));
    }
    mpfr_clear(a);
    mpfr_clear(c);
  }
  return ORA_OK;
}

/* Check a compact Householder QR of A0 (row-major n x n in every limb) given
 * as qr[L][n][n] row-major (R on and above the diagonal, the reflector
 * vectors below it with an implicit unit leading entry) and tau[L][n]:
 * Q = H_0 H_1 ... H_{n-1}, H_c = I - tau_c v_c v_c^T.
 * out[0] = max|QR - A0| / max|A0|, out[1] = max|Q^T Q - I|. */
int ora_qr_check(int prec_bits, int n, int L, const double *A0, const double *qr, const double *tau,
                 double *out) {
  mpfr_prec_t prec = prec_bits;
  const size_t nn = (size_t)n * n;
  mpfr_t *Q = vnew(nn, prec), *F = vnew(nn, prec), *A = vnew(nn, prec), *T = vnew(n, prec);
  mpfr_t *v = vnew(n, prec), *w = vnew(n, prec);
  mpfr_t t, mx, ma;
  mpfr_init2(t, prec);
  mpfr_init2(mx, prec);
  mpfr_init2(ma, prec);
  for (size_t q = 0; q < nn; ++q) {
    md_get(F[q], qr + q, nn, L);
    md_get(A[q], A0 + q, nn, L);
  }
  for (int c = 0; c < n; ++c) md_get(T[c], tau + c, n, L);
  for (int i = 0; i < n; ++i) mpfr_set_si(Q[(size_t)i * n + i], 1, MPFR_RNDN);
  /* Q := H_c Q for c = n-1 down to 0 */
  for (int c = n - 1; c >= 0; --c) {
    for (int i = 0; i < n; ++i) {
      if (i < c) mpfr_set_zero(v[i], 1);
      else if (i == c) mpfr_set_si(v[i], 1, MPFR_RNDN);
      else mpfr_set(v[i], F[(size_t)i * n + c], MPFR_RNDN);
    }
    for (int j = 0; j < n; ++j) {
      mpfr_set_zero(w[j], 1);
      for (int i = c; i < n; ++i) {
        mpfr_mul(t, v[i], Q[(size_t)i * n + j], MPFR_RNDN);
        mpfr_add(w[j], w[j], t, MPFR_RNDN);
      }
      mpfr_mul(w[j], w[j], T[c], MPFR_RNDN);
    }
    for (int i = c; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        mpfr_mul(t, v[i], w[j], MPFR_RNDN);
        mpfr_sub(Q[(size_t)i * n + j], Q[(size_t)i * n + j], t, MPFR_RNDN);
      }
  }
  mpfr_set_zero(ma, 1);
  for (size_t q = 0; q < nn; ++q) {
    mpfr_abs(t, A[q], MPFR_RNDN);
    mpfr_max(ma, ma, t, MPFR_RNDN);
  }
  mpfr_set_zero(mx, 1);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      mpfr_t s;
      mpfr_init2(s, prec);
      mpfr_neg(s, A[(size_t)i * n + j], MPFR_RNDN);
      for (int k = 0; k <= j; ++k) {
        mpfr_mul(t, Q[(size_t)i * n + k], F[(size_t)k * n + j], MPFR_RNDN);
        mpfr_add(s, s, t, MPFR_RNDN);
      }
      mpfr_abs(s, s, MPFR_RNDN);
      mpfr_max(mx, mx, s, MPFR_RNDN);
      mpfr_clear(s);
    }
  mpfr_div(mx, mx, ma, MPFR_RNDN);
  out[0] = mpfr_get_d(mx, MPFR_RNDN);
  mpfr_set_zero(mx, 1);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      mpfr_t s;
      mpfr_init2(s, prec);
      mpfr_set_si(s, i == j ? -1 : 0, MPFR_RNDN);
      for (int k = 0; k < n; ++k) {
        mpfr_mul(t, Q[(size_t)k * n + i], Q[(size_t)k * n + j], MPFR_RNDN);
        mpfr_add(s, s, t, MPFR_RNDN);
      }
      mpfr_abs(s, s, MPFR_RNDN);
      mpfr_max(mx, mx, s, MPFR_RNDN);
      mpfr_clear(s);
    }
  out[1] = mpfr_get_d(mx, MPFR_RNDN);
  mpfr_clear(t);
  mpfr_clear(mx);
  mpfr_clear(ma);
  vfree(Q, nn);
  vfree(F, nn);
  vfree(A, nn);
  vfree(T, n);
  vfree(v, n);
  vfree(w, n);
  return ORA_OK;
}

/* |R_ii| of any QR factorization of A0 (unique): the diagonal of the
 * Cholesky factor of A0^T A0.  A0[L][n][n] row-major; out[K][n]. */
int ora_rdiag(int prec_bits, int n, int L, const double *A0, int K, double *out) {
  mpfr_prec_t prec = prec_bits;
  const size_t nn = (size_t)n * n;
  mpfr_t *A = vnew(nn, prec), *G = vnew(nn, prec);
  mpfr_t t;
  mpfr_init2(t, prec);
  for (size_t q = 0; q < nn; ++q) md_get(A[q], A0 + q, nn, L);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      for (int k = 0; k < n; ++k) {
        mpfr_mul(t, A[(size_t)k * n + i], A[(size_t)k * n + j], MPFR_RNDN);
        mpfr_add(G[(size_t)i * n + j], G[(size_t)i * n + j], t, MPFR_RNDN);
      }
  int rc = ORA_OK;
  /* Cholesky G = R^T R, R upper triangular, stored in the upper triangle of G */
  for (int i = 0; i < n && rc == ORA_OK; ++i) {
    for (int k = 0; k < i; ++k) {
      mpfr_sqr(t, G[(size_t)k * n + i], MPFR_RNDN);
      mpfr_sub(G[(size_t)i * n + i], G[(size_t)i * n + i], t, MPFR_RNDN);
    }
    if (mpfr_sgn(G[(size_t)i * n + i]) <= 0) {
      rc = ORA_ESINGULAR;
      break;
    }
    mpfr_sqrt(G[(size_t)i * n + i], G[(size_t)i * n + i], MPFR_RNDN);
    for (int j = i + 1; j < n; ++j) {
      for (int k = 0; k < i; ++k) {
        mpfr_mul(t, G[(size_t)k * n + i], G[(size_t)k * n + j], MPFR_RNDN);
        mpfr_sub(G[(size_t)i * n + j], G[(size_t)i * n + j], t, MPFR_RNDN);
      }
      mpfr_div(G[(size_t)i * n + j], G[(size_t)i * n + j], G[(size_t)i * n + i], MPFR_RNDN);
    }
  }
  if (rc == ORA_OK)
    for (int i = 0; i < n; ++i) exp_put(out + i, n, K, G[(size_t)i * n + i], t);
  mpfr_clear(t);
  vfree(A, nn);
  vfree(G, nn);
  return rc;
}

/* Elementwise reference arithmetic on multiple doubles: op 0 a+b, 1 a-b,
 * 2 a*b, 3 a/b, 4 sqrt(a), 5 c + a*b; inputs [L][count], out[K][count]. */
int ora_arith(int prec_bits, int op, int L, const double *a, const double *b, const double *c, int count, int K,
              double *out) {
  if (op < 0 || op > 5 || L < 1 || K < 1) return ORA_EINVAL;
#pragma omp parallel num_threads(ora_get_threads())
  {
    mpfr_t x, y, z, t;
    mpfr_init2(x, prec_bits);
    mpfr_init2(y, prec_bits);
    mpfr_init2(z, prec_bits);
    mpfr_init2(t, prec_bits);
#pragma omp for schedule(static)
    for (int q = 0; q < count; ++q) {
      md_get(x, a + q, count, L);
      if (op != 4) md_get(y, b + q, count, L);
      switch (op) {
        case 0: mpfr_add(z, x, y, MPFR_RNDN); break;
        case 1: mpfr_sub(z, x, y, MPFR_RNDN); break;
        case 2: mpfr_mul(z, x, y, MPFR_RNDN); break;
        case 3: mpfr_div(z, x, y, MPFR_RNDN); break;
        case 4: mpfr_sqrt(z, x, MPFR_RNDN); break;
        default:
          md_get(z, c + q, count, L);
          mpfr_fma(z, x, y, z, MPFR_RNDN);
          break;
      }
      exp_put(out + q, count, K, z, t);
    }
    mpfr_clear(x);
    mpfr_clear(y);
    mpfr_clear(z);
    mpfr_clear(t);
  }
  return ORA_OK;
}

/* ------------------------------ adjoint ------------------------------- */

/* Solve the transposed block Toeplitz system T^T lambda = g (T has A_0 on the
 * diagonal and A_k on the k-th block subdiagonal, Section 2), by block back
 * substitution: A_0^T lambda_j = g_j - sum_{i=1..D-1-j} A_i^T lambda_{j+i},
 * j = D-1 .. 0.  A [L][D][n][n] row-major per matrix, g [L][n][D], out [K][n][D]. */
int ora_adjoint_solve(int prec_bits, int n, int D, int L, const double *A, const double *g, int K,
                      double *lam_out) {
  if (n < 1 || D < 1 || K < 1 || L < 1) return ORA_EINVAL;
  mpfr_prec_t prec = prec_bits;
  const size_t nn = (size_t)n * n, tot = (size_t)D * nn, nD = (size_t)n * D;
  mpfr_t *Am = vnew(tot, prec), *gv = vnew(nD, prec), *lam = vnew(nD, prec), *LU = vnew(nn, prec);
  for (size_t q = 0; q < tot; ++q) md_get(Am[q], A + q, tot, L);
  for (size_t q = 0; q < nD; ++q) md_get(gv[q], g + q, nD, L);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) mpfr_set(LU[(size_t)i * n + j], Am[(size_t)j * n + i], MPFR_RNDN);  /* A_0^T */
  int *perm = (int *)malloc(n * sizeof(int));
  int rc = lu_factor(LU, n, perm, prec);
  if (rc == ORA_OK) {
    mpfr_t *r = vnew(n, prec), *w = vnew(n, prec);
    mpfr_t t;
    mpfr_init2(t, prec);
    for (int j = D - 1; j >= 0; --j) {
#pragma omp parallel for schedule(static) num_threads(ora_get_threads())
      for (int v = 0; v < n; ++v) {
        mpfr_t u;
        mpfr_init2(u, prec);
        mpfr_set(r[v], gv[(size_t)v * D + j], MPFR_RNDN);
        for (int i = 1; j + i < D; ++i)
          for (int q = 0; q < n; ++q) {  /* (A_i^T lambda_{j+i})_v = sum_q A_i[q][v] lambda_{j+i}[q] */
            mpfr_mul(u, Am[(size_t)i * nn + (size_t)q * n + v], lam[(size_t)q * D + j + i], MPFR_RNDN);
            mpfr_sub(r[v], r[v], u, MPFR_RNDN);
          }
        mpfr_clear(u);
      }
      lu_solve(LU, n, perm, r, w, t);
      for (int v = 0; v < n; ++v) mpfr_set(lam[(size_t)v * D + j], r[v], MPFR_RNDN);
    }
    for (size_t q = 0; q < nD; ++q) exp_put(lam_out + q, nD, K, lam[q], t);
    vfree(r, n);
    vfree(w, n);
    mpfr_clear(t);
  }
  free(perm);
  vfree(Am, tot);
  vfree(gv, nD);
  vfree(lam, nD);
  vfree(LU, nn);
  return rc;
}

/* Gradient of a loss with respect to the monomial coefficients, given the
 * adjoint lambda of the converged system: p_i = c_{i,0} + sum_m c_m x^{a_m}
 * gives dp_i/dc_m = x^{a_m}, so dL/dc_m = -sum_k lambda_{i(m),k} [x^{a_m}]_k.
 * x [L][n][D], lambda [Ll][n][D] (any number of limbs), out [K][m]. */
int ora_coef_grad(int prec_bits, int n, int D, int m, const int32_t *pp, const int32_t *mp, const int32_t *var,
                  const int32_t *ex, int L, const double *x, int Ll, const double *lambda, int K, double *out) {
  sys_t S = {n, D, m, pp, mp, var, ex};
  if (check_sys(&S) || K < 1) return ORA_EINVAL;
  mpfr_prec_t prec = prec_bits;
  const size_t nD = (size_t)n * D;
  mpfr_t **X = (mpfr_t **)malloc(n * sizeof(mpfr_t *));
  mpfr_t *lam = vnew(nD, prec);
  for (int i = 0; i < n; ++i) {
    X[i] = vnew(D, prec);
    for (int s = 0; s < D; ++s) md_get(X[i][s], x + (size_t)i * D + s, nD, L);
  }
  for (size_t q = 0; q < nD; ++q) md_get(lam[q], lambda + q, nD, Ll);
#pragma omp parallel num_threads(ora_get_threads())
  {
    mpfr_t *val = vnew(D, prec), *tmp = vnew(D, prec);
    mpfr_t t, one, acc;
    mpfr_init2(t, prec);
    mpfr_init2(one, prec);
    mpfr_init2(acc, prec);
    mpfr_set_si(one, 1, MPFR_RNDN);
#pragma omp for schedule(dynamic, 1)
    for (int i = 0; i < n; ++i)
      for (int mj = pp[i]; mj < pp[i + 1]; ++mj) {
        mono_series(val, one, var + mp[mj], ex + mp[mj], mp[mj + 1] - mp[mj], -1, X, D, tmp, t);
        mpfr_set_zero(acc, 1);
        for (int s = 0; s < D; ++s) {
          mpfr_mul(t, lam[(size_t)i * D + s], val[s], MPFR_RNDN);
          mpfr_add(acc, acc, t, MPFR_RNDN);
        }
        mpfr_neg(acc, acc, MPFR_RNDN);
        exp_put(out + mj, m, K, acc, t);
      }
    vfree(val, D);
    vfree(tmp, D);
    mpfr_clear(t);
    mpfr_clear(one);
    mpfr_clear(acc);
  }
  for (int i = 0; i < n; ++i) vfree(X[i], D);
  free(X);
  vfree(lam, nD);
  return ORA_OK;
}
