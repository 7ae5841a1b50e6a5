"""Pins of the oracle against things other than itself (CPU only).

Each test checks the oracle against the mathematics or the paper:
exact rational brute force with sympy, the paper's exponential-series worked
example (Section 3) and its two-column variant, binomial series, classical
Newton at D=1 with a hand-written Jacobian, one-step convergence on linear
systems, quadratic convergence in t-order, the stopping invariant of
Section 4, the printed 1/k! values of Table 1, and LAPACK's Householder QR
for the QR checker.  A plausible slip in the oracle (dropped convolution
term, wrong sign of b, transposed Jacobian, wrong block index in the forward
substitution, wrong exponent handling, pivoting error) fails at least one.
"""
from __future__ import annotations

import math
import os
from fractions import Fraction

import mpmath
import numpy as np
import pytest
import sympy

import mdinputs
import oracle
from oracle_helpers import make, md_value, series_md, to_md

HERE = os.path.dirname(os.path.abspath(__file__))


def exact(e):
    """Exact values of expansions e[K, ...] as a Fraction array."""
    K = e.shape[0]
    flat = e.reshape(K, -1)
    return np.array([md_value(flat[:, q]) for q in range(flat.shape[1])], dtype=object).reshape(e.shape[1:])


def newton_run(sys, cst, x, steps):
    for _ in range(steps):
        x = oracle.newton_step(sys, sys.cff, cst, x)["x"]
    return x


# --------------------------------------------------------------------------
# 1. brute force: exact rational arithmetic with sympy on tiny systems
# --------------------------------------------------------------------------

def _sympy_step(sys, cst, x):
    """Exact b, A, and Newton step with sympy: expand p(x(t)), differentiate
    symbolically, solve the full (nD x nD) block system by exact LU."""
    t = sympy.Symbol("t")
    n, D, L = sys.n, sys.D, sys.L
    X = sympy.symbols(f"y0:{n}")
    cfv = [md_value(sys.cff[:, j]) for j in range(sys.m)]
    xs = [sum(sympy.Rational(md_value(x[:, i, s])) * t ** s for s in range(D)) for i in range(n)]
    cs = [sum(sympy.Rational(md_value(cst[:, i, s])) * t ** s for s in range(D)) for i in range(n)]
    P = []
    for i in range(n):
        expr = 0
        for mj in range(sys.poly_ptr[i], sys.poly_ptr[i + 1]):
            term = sympy.Rational(cfv[mj])
            for q in range(sys.mon_ptr[mj], sys.mon_ptr[mj + 1]):
                term *= X[sys.var[q]] ** int(sys.exp[q])
            expr += term
        P.append(expr)

    def trunc(e):
        poly = sympy.Poly(sympy.expand(e), t)
        return [poly.coeff_monomial(t ** s) for s in range(D)]

    sub = dict(zip(X, xs))
    b = [[-c for c in trunc(cs[i] + P[i].subs(sub))] for i in range(n)]
    A = [[trunc(sympy.diff(P[i], X[j]).subs(sub)) for j in range(n)] for i in range(n)]
    # full block lower-triangular Toeplitz matrix, unknowns ordered (k, i)
    T = sympy.zeros(n * D, n * D)
    rhs = sympy.zeros(n * D, 1)
    for k in range(D):
        for i in range(n):
            rhs[k * n + i] = b[i][k]
            for j in range(k + 1):
                for v in range(n):
                    T[k * n + i, j * n + v] = A[i][v][k - j]
    sol = T.LUsolve(rhs)
    dx = [[sol[k * n + i] for k in range(D)] for i in range(n)]
    xn = [[sympy.Rational(md_value(x[:, i, s])) + dx[i][s] for s in range(D)] for i in range(n)]
    return b, A, xn


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_brute_force_sympy(seed):
    sys = mdinputs.tiny(2, 3, 3, mons=2, kmin=1, kmax=3, exps=(1, 2), seed=seed)
    x = mdinputs.random_point(sys, seed)
    cst = mdinputs.random_constant(sys, seed)
    b, A, xn = _sympy_step(sys, cst, x)
    ob, oA, _ = oracle.eval_diff(sys, sys.cff, cst, x, prec=700, K=16)
    out = oracle.newton_step(sys, sys.cff, cst, x, prec=700, K=16)
    eb, eA, ex = exact(ob), exact(oA), exact(out["x"])
    tol = Fraction(1, 2 ** 600)
    for i in range(sys.n):
        for s in range(sys.D):
            assert abs(eb[i, s] - Fraction(str(b[i][s]))) <= tol * (1 + abs(eb[i, s]))
            assert abs(ex[i, s] - Fraction(str(xn[i][s]))) <= tol * (1 + abs(ex[i, s]))
            for j in range(sys.n):
                assert abs(eA[s, i, j] - Fraction(str(A[i][j][s]))) <= tol * (1 + abs(eA[s, i, j]))


# --------------------------------------------------------------------------
# 2. the paper's worked example: x^E = b(t) with exponential solutions
# --------------------------------------------------------------------------

def _exp_coefs(alpha: Fraction, D: int):
    return [alpha ** k / math.factorial(k) for k in range(D)]


def test_exp_one_column_closed_form():
    """Section 3: E lower triangular of ones, b_i(t) = exp((a_1+..+a_i) t);
    the unique solution is x_k(t) = exp(a_k t)."""
    L, n, d = 2, 4, 15
    D = d + 1
    alphas = [Fraction(3, 4), Fraction(-7, 8), Fraction(1, 1), Fraction(-5, 8)]
    polys = [[(1, [(j, 1) for j in range(i + 1)])] for i in range(n)]
    sys = make(L, n, d, polys)
    sums = np.cumsum(np.array(alphas, dtype=object))
    cst = series_md([[-c for c in _exp_coefs(sums[i], D)] for i in range(n)], L)
    x = np.zeros((L, n, D))
    x[0, :, 0] = 1.0
    x = newton_run(sys, cst, x, 6)
    ex = exact(x)
    for i in range(n):
        ref = _exp_coefs(alphas[i], D)
        err = max(abs(ex[i, k] - ref[k]) for k in range(D))
        assert err < 1e-29, (i, float(err))


def test_exp_two_columns_closed_form():
    """Section 3: c1 x^{E1} + c2 x^{E2} = b(t), E1 lower and E2 upper
    triangular ones; with b manufactured from x_k = exp(a_k t) exactly."""
    L, n, d = 2, 3, 11
    D = d + 1
    alphas = [Fraction(1, 2), Fraction(-3, 4), Fraction(7, 8)]
    c1 = [Fraction(5, 4), Fraction(-3, 2), Fraction(7, 4)]
    c2 = [Fraction(-1, 2), Fraction(3, 4), Fraction(1, 4)]
    polys = []
    csts = []
    for i in range(n):
        low = list(range(i + 1))
        up = list(range(n - i))
        polys.append([(c1[i], [(j, 1) for j in low]), (c2[i], [(j, 1) for j in up])])
        s1 = sum(alphas[j] for j in low)
        s2 = sum(alphas[j] for j in up)
        e1, e2 = _exp_coefs(s1, D), _exp_coefs(s2, D)
        csts.append([-(c1[i] * e1[k] + c2[i] * e2[k]) for k in range(D)])
    sys = make(L, n, d, polys)
    cst = series_md(csts, L)
    x = np.zeros((L, n, D))
    x[0, :, 0] = 1.0
    x = newton_run(sys, cst, x, 6)
    ex = exact(x)
    for i in range(n):
        ref = _exp_coefs(alphas[i], D)
        assert max(abs(ex[i, k] - ref[k]) for k in range(D)) < 1e-28


# --------------------------------------------------------------------------
# 3. binomial series
# --------------------------------------------------------------------------

def _binom(r: Fraction, k: int) -> Fraction:
    out = Fraction(1)
    for j in range(k):
        out = out * (r - j) / (j + 1)
    return out


@pytest.mark.parametrize("e", [2, 3])
def test_root_binomial_series(e):
    """n = 1, x^e = 1 + t: the series of (1+t)^(1/e) has coefficients binom(1/e, k)."""
    L, d = 4, 23
    D = d + 1
    sys = make(L, 1, d, [[(1, [(0, e)])]])
    cst = series_md([[-1, -1] + [0] * (D - 2)], L)
    x = np.zeros((L, 1, D))
    x[0, 0, 0] = 1.0
    x = newton_run(sys, cst, x, 6)
    ex = exact(x)
    for k in range(D):
        assert abs(ex[0, k] - _binom(Fraction(1, e), k)) < 1e-60


def test_eval_at_one_plus_t_binomials():
    """All x_j = 1 + t: c x^a = c (1+t)^deg and d/dx_j = c a_j (1+t)^(deg-1)."""
    L, n, d = 2, 3, 9
    D = d + 1
    polys = [[(Fraction(3, 2), [(0, 2), (1, 1), (2, 3)])], [(Fraction(-1, 4), [(1, 1), (2, 1)])],
             [(Fraction(1), [(0, 1)])]]
    sys = make(L, n, d, polys)
    x = np.zeros((L, n, D))
    x[0, :, 0] = 1.0
    x[0, :, 1] = 1.0
    cst = np.zeros((L, n, D))
    b, A, _ = oracle.eval_diff(sys, sys.cff, cst, x)
    eb, eA = exact(b), exact(A)
    degs = [6, 2, 1]
    coefs = [Fraction(3, 2), Fraction(-1, 4), Fraction(1)]
    for i in range(n):
        for k in range(D):
            assert eb[i, k] == -coefs[i] * math.comb(degs[i], k)
    # d p_0 / d x_2 = 3/2 * 3 * (1+t)^5
    for k in range(D):
        assert eA[k, 0, 2] == Fraction(9, 2) * math.comb(5, k)
        assert eA[k, 0, 0] == 3 * math.comb(5, k)
        assert eA[k, 1, 0] == 0
        assert eA[k, 2, 0] == (1 if k == 0 else 0)


# --------------------------------------------------------------------------
# 4. D = 1 is classical Newton (hand-written Jacobian, library solve)
# --------------------------------------------------------------------------

def test_classical_newton_d0():
    """p1 = x0^2 x1 - 3/4 x1 + 2, p2 = 5/2 x0 x1^2 - x0 - 1/8; one Newton step at
    a point equals x - J^{-1} p with J written out by hand (non-symmetric)."""
    L = 4
    polys = [[(1, [(0, 2), (1, 1)]), (Fraction(-3, 4), [(1, 1)])],
             [(Fraction(5, 2), [(0, 1), (1, 2)]), (-1, [(0, 1)])]]
    sys = make(L, 2, 0, polys)
    cst = series_md([[2], [Fraction(-1, 8)]], L)
    x0, x1 = Fraction(5, 4), Fraction(-3, 8)
    x = series_md([[x0], [x1]], L)
    out = oracle.newton_step(sys, sys.cff, cst, x)
    mpmath.mp.prec = 600
    X0, X1 = mpmath.mpf(x0.numerator) / x0.denominator, mpmath.mpf(x1.numerator) / x1.denominator
    p = mpmath.matrix([X0 ** 2 * X1 - mpmath.mpf(3) / 4 * X1 + 2,
                       mpmath.mpf(5) / 2 * X0 * X1 ** 2 - X0 - mpmath.mpf(1) / 8])
    J = mpmath.matrix([[2 * X0 * X1, X0 ** 2 - mpmath.mpf(3) / 4],
                       [mpmath.mpf(5) / 2 * X1 ** 2 - 1, 5 * X0 * X1]])
    step = mpmath.lu_solve(J, -p)
    ex = exact(out["x"])
    for i, xi in enumerate((X0, X1)):
        ref = xi + step[i]
        assert abs(mpmath.mpf(ex[i, 0].numerator) / ex[i, 0].denominator - ref) < mpmath.mpf(2) ** -400


def test_linear_system_one_step():
    """p(x) = M x + c(t): Newton converges in one step from any start to
    x_k = -M^{-1} c_k for every coefficient k (textbook LU via mpmath)."""
    rng = np.random.default_rng(11)
    L, n, d = 4, 5, 4
    D = d + 1
    M = [[Fraction(int(v), 8) for v in row] for row in rng.integers(-16, 17, size=(n, n))]
    for i in range(n):
        M[i][i] += 20
    polys = [[(M[i][j], [(j, 1)]) for j in range(n) if M[i][j] != 0] for i in range(n)]
    sys = make(L, n, d, polys)
    c = [[Fraction(int(v), 16) for v in row] for row in rng.integers(-32, 33, size=(n, D))]
    cst = series_md(c, L)
    x = mdinputs.random_point(sys, 3)
    out = oracle.newton_step(sys, sys.cff, cst, x)
    ex = exact(out["x"])
    mpmath.mp.prec = 900
    Mm = mpmath.matrix([[mpmath.mpf(v.numerator) / v.denominator for v in row] for row in M])
    for k in range(D):
        ck = mpmath.matrix([-mpmath.mpf(c[i][k].numerator) / c[i][k].denominator for i in range(n)])
        sol = mpmath.lu_solve(Mm, ck)
        for i in range(n):
            got = mpmath.mpf(ex[i, k].numerator) / ex[i, k].denominator
            assert abs(got - sol[i]) < mpmath.mpf(2) ** -800


# --------------------------------------------------------------------------
# 5. quadratic convergence in t-order and the stopping invariant (Section 4)
# --------------------------------------------------------------------------

def _exact_data_system(L, n, d, seed, mons=4, kmax=3):
    """Random supports with short dyadic data: x*_k = m/16 * 4^-k, c = j/8, and
    a diagonal boost.  Every series product is then exact in L limbs, so the
    manufactured c_{i,0} is exact and x* solves the rounded system exactly."""
    rng = np.random.default_rng(seed)
    D = d + 1
    polys = []
    for i in range(n):
        row = [(Fraction(int(rng.integers(-8, 9)) or 1, 8),
                [(int(v), int(rng.integers(1, 3))) for v in rng.choice(n, size=int(rng.integers(1, kmax + 1)), replace=False)])
               for _ in range(mons)]
        row.append((Fraction(16), [(i, 1)]))
        polys.append(row)
    sys = make(L, n, d, polys)
    xs = [[Fraction(int(rng.integers(8, 25)), 16) / 4 ** k for k in range(D)] for _ in range(n)]
    sys.xstar = series_md(xs, L)
    return sys


def test_quadratic_convergence_order_doubles():
    """From x*(0), after s Newton steps exactly the coefficients 0..2^s-1 are
    correct and coefficient 2^s is not: Newton on series doubles the number of
    correct coefficients (Section 4 grows the order by d := d + 1 + d/2 at
    best).  The data are exact, so "correct" means equal to the oracle's own
    rounding at 424 bits."""
    L, n, d = 2, 4, 15
    sys = _exact_data_system(L, n, d, seed=7)
    cst = oracle.manufacture(sys, Lout=L)
    b, _, _ = oracle.eval_diff(sys, sys.cff, cst, sys.xstar)
    assert np.abs(b).max() == 0.0  # x* is an exact root of the stored system
    x = sys.start()
    for s in range(1, 5):
        x = oracle.newton_step(sys, sys.cff, cst, x)["x"]
        err = oracle.absdiff(x, sys.xstar).max(axis=0)  # per coefficient
        good = 2 ** s
        assert err[:min(good, sys.D)].max() < 1e-110
        if good < sys.D:
            assert err[good] > 1e-20 * 4.0 ** -good


def test_zero_residual_gives_zero_update():
    """Section 4: once b_k = 0 the update dx_k = 0.  With exactly representable
    data the residual of the first k coefficients is exactly zero."""
    L, n, d = 2, 3, 7
    D = d + 1
    polys = [[(1, [(0, 1), (1, 1)]), (2, [(2, 1)])], [(1, [(1, 2)]), (-1, [(0, 1)])],
             [(1, [(2, 1)]), (1, [(0, 1), (2, 1)])]]
    sys = make(L, n, d, polys)
    xs = [[Fraction(1 + i, 2) if s == 0 else Fraction((-1) ** s * (s + i), 8) for s in range(D)]
          for i in range(n)]
    sys.xstar = series_md(xs, L)
    cst = oracle.manufacture(sys, Lout=L)
    k = 3
    x = sys.xstar.copy()
    x[:, :, k:] = 0.0
    out = oracle.newton_step(sys, sys.cff, cst, x)
    eb, edx = exact(out["b"]), exact(out["dx"])
    for i in range(n):
        for s in range(k):
            assert eb[i, s] == 0 and edx[i, s] == 0
    assert any(edx[i, k] != 0 for i in range(n))


# --------------------------------------------------------------------------
# 6. Table 1: printed values of 1/k!
# --------------------------------------------------------------------------

def test_table1_inverse_factorials():
    """Table 1 prints 1/k! for k up to 127.  The oracle's Newton on
    x0 = e^t, x0 x1 = e^{2t} (Section 3, alpha = 1) at D = 128 gives x1_k = 1/k!;
    compare with the printed two-digit values: each must be within half a unit
    of its last printed digit, widened to 0.06 units because the paper prints
    7.7e-13 for 1/15! = 7.647e-13."""
    rows = []
    with open(os.path.join(HERE, "golden", "table1_inverse_factorials.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                k, v = line.split()[:2]
                rows.append((int(k), float(v)))
    L, n, d = 8, 2, 127
    D = d + 1
    sys = make(L, n, d, [[(1, [(0, 1)])], [(1, [(0, 1), (1, 1)])]])
    cst = series_md([[-c for c in _exp_coefs(Fraction(1), D)], [-c for c in _exp_coefs(Fraction(2), D)]], L)
    x = np.zeros((L, n, D))
    x[0, :, 0] = 1.0
    x = newton_run(sys, cst, x, 8)
    ex = exact(x)
    for k, printed in rows:
        got = float(ex[1, k])
        unit = 10.0 ** (math.floor(math.log10(printed)) - 1)
        assert abs(got - printed) <= 0.6 * unit, (k, got, printed)
        assert abs(ex[1, k] - Fraction(1, math.factorial(k))) < Fraction(1, 10 ** 125)


# --------------------------------------------------------------------------
# 7. the QR checker and |R_ii| against LAPACK's Householder QR
# --------------------------------------------------------------------------

def test_qr_check_and_rdiag_against_lapack():
    rng = np.random.default_rng(5)
    n = 7
    A = rng.uniform(-1, 1, size=(n, n)) + 3 * np.eye(n)
    h, tau = np.linalg.qr(A, mode="raw")   # LAPACK geqrf, column-major
    F = h.T.copy()                           # row-major: R above, v below the diagonal
    res, orth = oracle.qr_check(A[None], F[None], tau[None])
    assert res < 1e-14 and orth < 1e-14
    rd = oracle.rdiag(A[None])
    assert np.allclose(rd[0], np.abs(np.diag(F)), rtol=1e-13)
    # a planted error in one reflector is seen
    F2 = F.copy()
    F2[3, 1] += 1e-6
    res2, orth2 = oracle.qr_check(A[None], F2[None], tau[None])
    assert res2 > 1e-8


# --------------------------------------------------------------------------
# 8. conversions
# --------------------------------------------------------------------------

def test_round_and_absdiff_exact():
    rng = np.random.default_rng(3)
    vals = [Fraction(int(rng.integers(1, 2 ** 62))) / 2 ** 61 + Fraction(int(rng.integers(1, 2 ** 62)), 2 ** 170)
            for _ in range(20)]
    e = to_md(vals, 6)
    for L in (2, 4):
        r = oracle.round_md(e, L)
        for q in range(len(vals)):
            v = md_value(r[:, q])
            assert abs(v - vals[q]) <= abs(vals[q]) * Fraction(1, 2 ** (53 * L - 1))
            for l in range(L - 1):  # nonoverlapping limbs
                assert r[l + 1, q] == 0 or abs(r[l + 1, q]) <= 0.5 * np.spacing(abs(r[l, q]))
    d = oracle.absdiff(e, to_md(vals[::-1], 6))
    for q in range(len(vals)):
        assert d[q] == float(abs(vals[q] - vals[::-1][q]))


def test_manufactured_solution_is_a_root():
    sys = mdinputs.tiny(4, 4, 7, mons=3, seed=3)
    cst = oracle.manufacture(sys)
    b, _, scale = oracle.eval_diff(sys, sys.cff, cst, sys.xstar)
    # only the rounding of c_{i,0} to four limbs remains
    assert np.max(np.abs(b[0]).max(axis=1) / scale) < 2.0 ** -205
    assert oracle.inexact_inputs() == 0


# --------------------------------------------------------------------------
# 9. the adjoint: transposed block solve and coefficient gradients
# --------------------------------------------------------------------------

def _dot_exact(a, b):
    ea, eb = exact(a), exact(b)
    return sum((ea.flat[q] * eb.flat[q] for q in range(ea.size)), Fraction(0))


def test_adjoint_dot_product_identity():
    """<T^{-1} u, v> = <u, T^{-T} v> for the block Toeplitz T (two different
    solves: forward block substitution with LU of A_0, backward with LU of A_0^T)."""
    rng = np.random.default_rng(21)
    L, n, D = 4, 4, 6
    A = mdinputs.random_md(rng, L, (D, n, n), -1.0, 1.0)
    A[0, 0] += 4 * np.eye(n)
    u = mdinputs.random_md(rng, L, (n, D), -1.0, 1.0)
    v = mdinputs.random_md(rng, L, (n, D), -1.0, 1.0)
    K = 16
    x = oracle.toeplitz_solve(A, u, K=K, prec=900)
    y = oracle.adjoint_solve(A, v, K=K, prec=900)
    lhs, rhs = _dot_exact(x, np.concatenate([v, np.zeros((K - L, n, D))])), \
        _dot_exact(np.concatenate([u, np.zeros((K - L, n, D))]), y)
    assert abs(lhs - rhs) <= abs(lhs) * Fraction(1, 2 ** 800)
    # and a transposition slip would be seen
    At = np.ascontiguousarray(np.swapaxes(A, 2, 3))
    y2 = oracle.adjoint_solve(At, v, K=K, prec=900)
    assert abs(_dot_exact(np.concatenate([u, np.zeros((K - L, n, D))]), y2) - lhs) > abs(lhs) * Fraction(1, 2 ** 40)


def test_adjoint_gradient_closed_form():
    """c x^2 = 1 + t: x = sqrt((1+t)/c), dx/dc = -x/(2c), so for L = sum_{k>=2} x_k^2
    dL/dc = -sum_{k>=2} x_k^2 / c."""
    L, d = 4, 7
    D = d + 1
    c = Fraction(5, 4)
    sys = make(L, 1, d, [[(c, [(0, 2)])]])
    cst = series_md([[-1, -1] + [0] * (D - 2)], L)
    x0 = np.zeros((L, 1, D))
    x0[0, 0, 0] = 0.9
    x = oracle.converge(sys, sys.cff, cst, x0, 7, K=18)
    xr = oracle.round_md(x, L)
    g = oracle.loss_top_grad(x, 2)
    out = oracle.newton_step(sys, sys.cff, cst, xr, want_A=True, K=18)
    lam = oracle.adjoint_solve(oracle.round_md(out["A"], L), oracle.round_md(g, L), K=18)
    grad = oracle.coef_grad(sys, xr, lam, K=18)
    ex = exact(x)
    ref = -sum((ex[0, k] ** 2 for k in range(2, D)), Fraction(0)) / c
    assert abs(exact(grad)[0] - ref) <= abs(ref) * Fraction(1, 10 ** 55)


def test_adjoint_gradient_matches_finite_differences():
    """Central differences of L(c) = sum_{k>=ktop} x_{i,k}(c)^2 at 1000 bits with
    h = 2^-150, Newton carried to convergence in the oracle, against the adjoint."""
    sys = mdinputs.tiny(4, 3, 5, mons=2, kmin=1, kmax=3, exps=(1, 2), seed=4)
    cst = oracle.manufacture(sys)
    K, prec, ktop = 24, 1200, 3
    x = oracle.converge(sys, sys.cff, cst, sys.start(), 6, K=K, prec=prec)
    out = oracle.newton_step(sys, sys.cff, cst, x, want_A=True, K=K, prec=prec)
    g = oracle.loss_top_grad(x, ktop)
    lam = oracle.adjoint_solve(out["A"], g, K=K, prec=prec)
    grad = exact(oracle.coef_grad(sys, x, lam, K=K, prec=prec))
    h = Fraction(1, 2 ** 150)
    for mj in (0, 2, sys.m - 1):
        vals = []
        for sgn in (1, -1):
            cf = np.concatenate([sys.cff, np.zeros((K - sys.L, sys.m))])
            cf[sys.L, mj] = float(sgn * h)  # c_m +- h as an extra limb, exact
            cs = np.concatenate([cst, np.zeros((K - sys.L, sys.n, sys.D))])
            xp = oracle.converge(sys, cf, cs, sys.start(), 7, K=K, prec=prec)
            ex = exact(xp)
            vals.append(sum((ex[i, k] ** 2 for i in range(sys.n) for k in range(ktop, sys.D)), Fraction(0)))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - grad[mj]) <= abs(grad[mj]) * Fraction(1, 10 ** 70) + Fraction(1, 10 ** 80), mj


# --------------------------------------------------------------------------
# 10. the staggered step: order truncation, stage window, kept factorization
#     (Sections 4 and 5.3)
# --------------------------------------------------------------------------

def _sympy_window(sys, cst, x, lo, hi, x_kept=None):
    """Exact window step with sympy: b and A of the order-hi truncation, the
    block system over stages lo..hi-1 only (dx_k = 0 below lo), its diagonal
    block the Jacobian at x_kept's leading coefficients (x's own if None)."""
    t = sympy.Symbol("t")
    n = sys.n
    X = sympy.symbols(f"y0:{n}")
    cfv = [md_value(sys.cff[:, j]) for j in range(sys.m)]
    xs = [sum(sympy.Rational(md_value(x[:, i, s])) * t ** s for s in range(hi)) for i in range(n)]
    cs = [sum(sympy.Rational(md_value(cst[:, i, s])) * t ** s for s in range(hi)) for i in range(n)]
    P = []
    for i in range(n):
        expr = 0
        for mj in range(sys.poly_ptr[i], sys.poly_ptr[i + 1]):
            term = sympy.Rational(cfv[mj])
            for q in range(sys.mon_ptr[mj], sys.mon_ptr[mj + 1]):
                term *= X[sys.var[q]] ** int(sys.exp[q])
            expr += term
        P.append(expr)

    def trunc(e):
        poly = sympy.Poly(sympy.expand(e), t)
        return [poly.coeff_monomial(t ** s) for s in range(hi)]

    sub = dict(zip(X, xs))
    b = [[-c for c in trunc(cs[i] + P[i].subs(sub))] for i in range(n)]
    A = [[trunc(sympy.diff(P[i], X[j]).subs(sub)) for j in range(n)] for i in range(n)]
    if x_kept is None:
        A0 = [[A[i][j][0] for j in range(n)] for i in range(n)]
    else:
        sub0 = {X[v]: sympy.Rational(md_value(x_kept[:, v, 0])) for v in range(n)}
        A0 = [[sympy.diff(P[i], X[j]).subs(sub0) for j in range(n)] for i in range(n)]
    W = hi - lo
    T = sympy.zeros(n * W, n * W)
    rhs = sympy.zeros(n * W, 1)
    for kk in range(W):
        for i in range(n):
            rhs[kk * n + i] = b[i][lo + kk]
            for jj in range(kk + 1):
                for v in range(n):
                    T[kk * n + i, jj * n + v] = A0[i][v] if jj == kk else A[i][v][kk - jj]
    sol = T.LUsolve(rhs)
    dx = [[sol[(s - lo) * n + i] if lo <= s < hi else 0 for s in range(sys.D)] for i in range(n)]
    return b, dx


@pytest.mark.parametrize("lo,hi,kept", [(0, 4, False), (1, 3, False), (2, 4, False), (0, 2, True), (1, 4, True),
                                        (3, 4, True)])
def test_window_step_brute_force_sympy(lo, hi, kept):
    sys = mdinputs.tiny(2, 3, 3, mons=2, kmin=1, kmax=3, exps=(1, 2), seed=4)
    x = mdinputs.random_point(sys, 4)
    cst = mdinputs.random_constant(sys, 4)
    xk = mdinputs.random_point(sys, 5) if kept else None
    b, dx = _sympy_window(sys, cst, x, lo, hi, xk)
    out = oracle.window_step(sys, sys.cff, cst, x, lo, hi, x_kept=xk, prec=700, K=16)
    eb, edx, ex = exact(out["b"]), exact(out["dx"]), exact(out["x"])
    tol = Fraction(1, 2 ** 600)
    for i in range(sys.n):
        for s in range(sys.D):
            want_dx = Fraction(str(dx[i][s]))
            assert abs(edx[i, s] - want_dx) <= tol * (1 + abs(want_dx))
            want_x = md_value(x[:, i, s]) + want_dx
            assert abs(ex[i, s] - want_x) <= tol * (1 + abs(want_x))
            if s < hi:
                want_b = Fraction(str(b[i][s]))
                assert abs(eb[i, s] - want_b) <= tol * (1 + abs(want_b))
            else:
                assert eb[i, s] == 0 and ex[i, s] == md_value(x[:, i, s])


def test_window_step_truncation_is_the_leading_part_of_newton():
    """Coefficient k of the Newton update depends on the coefficients 0..k
    only, so the step of the order-hi truncation is the leading part of the
    full step; exact data make every residual product exact."""
    L, n, d = 2, 4, 11
    sys = _exact_data_system(L, n, d, seed=3)
    cst = oracle.manufacture(sys, Lout=L)
    x = sys.start()
    x[:, :, 1:4] = sys.xstar[:, :, 1:4] * 0.5
    full = oracle.newton_step(sys, sys.cff, cst, x)
    for hi in (1, 5, 12):
        w = oracle.window_step(sys, sys.cff, cst, x, 0, hi)
        assert np.array_equal(exact(w["dx"])[:, :hi], exact(full["dx"])[:, :hi])
        assert np.array_equal(exact(w["x"])[:, hi:], exact(x[:, :, hi:]))


def test_chord_step_fixed_point_and_zero_window():
    """At an exact root b = 0, so the chord step (any kept A_0) leaves x
    unchanged; with x_k exact below lo, the window from lo is Newton's step
    (Section 4: dx_k = 0 where b_k = 0)."""
    L, n, d = 2, 4, 9
    sys = _exact_data_system(L, n, d, seed=11)
    cst = oracle.manufacture(sys, Lout=L)
    kept = sys.xstar.copy()
    kept[:, :, 0] *= 1.0 + 2.0 ** -20
    w = oracle.window_step(sys, sys.cff, cst, sys.xstar, 0, sys.D, x_kept=kept)
    assert not np.any(w["dx"]) and np.array_equal(exact(w["x"]), exact(sys.xstar))
    lo = 4
    x = sys.xstar.copy()
    x[:, :, lo:] = 0.0
    newton = oracle.newton_step(sys, sys.cff, cst, x)
    win = oracle.window_step(sys, sys.cff, cst, x, lo, sys.D)
    assert np.array_equal(exact(win["dx"]), exact(newton["dx"]))
    assert not np.any(exact(newton["dx"])[:, :lo])


def test_chord_step_contracts_linearly():
    """A chord step (A_0 kept from a point sigma away) reduces an error delta
    to about sigma * delta, where Newton's step reaches delta^2."""
    sys = mdinputs.tiny(4, 4, 5, mons=3, seed=6)
    cst = oracle.manufacture(sys)
    delta, sigma = 1e-12, 1e-4
    rng = np.random.default_rng(0)
    x = sys.xstar.copy()
    x[0] += delta * rng.uniform(0.5, 1.0, size=x.shape[1:])
    kept = sys.xstar.copy()
    kept[0, :, 0] *= 1.0 + sigma
    chord = oracle.absdiff(oracle.window_step(sys, sys.cff, cst, x, 0, sys.D, x_kept=kept)["x"], sys.xstar).max()
    newton = oracle.absdiff(oracle.newton_step(sys, sys.cff, cst, x)["x"], sys.xstar).max()
    assert 1e-3 * sigma * delta < chord < 1e3 * sigma * delta
    assert newton < 1e-3 * chord


# --------------------------------------------------------------------------
# 11. the linear residual b - T dx (Section 5.4, Table 4)
# --------------------------------------------------------------------------

def test_linear_residual_brute_force():
    """Exact rationals: r_{i,k} = b_{i,k} - sum_{j<=k} sum_v A_j(i,v) dx_{v,k-j},
    on all rows and on a sample of rows."""
    rng = np.random.default_rng(3)
    L, n, D = 2, 3, 4
    A = mdinputs.random_md(rng, L, (D, n, n), -1.0, 1.0)
    b = mdinputs.random_md(rng, L, (n, D), -1.0, 1.0)
    dx = mdinputs.random_md(rng, L, (n, D), -1.0, 1.0)
    eA = exact(A)
    eb, edx = exact(b), exact(dx)
    for rows in (None, [2, 0]):
        r, sc = oracle.linear_residual(A, b, dx, rows=rows, prec=700, K=16)
        er = exact(r)
        for q, i in enumerate(range(n) if rows is None else rows):
            for k in range(D):
                want = eb[i, k] - sum(eA[j, i, v] * edx[v, k - j] for j in range(k + 1) for v in range(n))
                assert abs(er[q, k] - want) <= Fraction(1, 2 ** 600) * (1 + abs(want))
                size = abs(eb[i, k]) + sum(abs(eA[j, i, v] * edx[v, k - j]) for j in range(k + 1) for v in range(n))
                assert sc[q, k] == pytest.approx(float(size), rel=1e-15)


def test_linear_residual_of_the_block_solve_vanishes():
    """The residual of the oracle's own block forward substitution (pinned by
    the sympy brute force above) is zero to the working bits."""
    rng = np.random.default_rng(4)
    L, n, D = 4, 5, 7
    A = mdinputs.random_md(rng, L, (D, n, n), -1.0, 1.0)
    A[0, 0] += 4.0 * np.eye(n)  # a well-conditioned A_0 (the added leading limbs keep the limbs nonoverlapping)
    b = mdinputs.random_md(rng, L, (n, D), -1.0, 1.0)
    dx = oracle.toeplitz_solve(A, b)
    r, sc = oracle.linear_residual(A, b, dx)
    assert np.max(oracle.absdiff(r, np.zeros((1,) + r.shape[1:])) / sc) < 2.0 ** -(4 * 53 * L - 20)
    r2, _ = oracle.linear_residual(A, b, np.zeros_like(b))
    assert np.array_equal(exact(r2), exact(b))


# --------------------------------------------------------------------------
# 12. complex data (Section 5.2)
# --------------------------------------------------------------------------

def _cval(a, idx):
    """Exact complex value of entry idx of a complex md array [2, L, ...]."""
    return sympy.Rational(md_value(a[(0, slice(None)) + idx])) + sympy.I * sympy.Rational(md_value(a[(1, slice(None)) + idx]))


def test_complex_step_brute_force_sympy():
    """Exact complex rationals: b = -(c_0 + p(x)), A = p'(x) and one Newton step
    by solving the full block system exactly."""
    s = mdinputs.tiny(2, 2, 2, mons=2, kmin=1, kmax=2, exps=(1, 2), seed=8)
    cff, cst, x = mdinputs.complex_random(s, 8)
    t = sympy.Symbol("t")
    n, D = s.n, s.D
    X = sympy.symbols(f"y0:{n}")
    xs = [sum(_cval(x, (i, k)) * t ** k for k in range(D)) for i in range(n)]
    P = []
    for i in range(n):
        e = sum(_cval(cst, (i, k)) * t ** k for k in range(D))
        for mj in range(s.poly_ptr[i], s.poly_ptr[i + 1]):
            term = _cval(cff, (mj,))
            for q in range(s.mon_ptr[mj], s.mon_ptr[mj + 1]):
                term *= X[s.var[q]] ** int(s.exp[q])
            e += term
        P.append(e)
    sub = dict(zip(X, xs))
    trunc = lambda e: [sympy.expand(e).coeff(t, k) for k in range(D)]
    b = [[-c for c in trunc(P[i].subs(sub))] for i in range(n)]
    A = [[trunc(sympy.diff(P[i], X[j]).subs(sub)) for j in range(n)] for i in range(n)]
    T = sympy.zeros(n * D, n * D)
    rhs = sympy.zeros(n * D, 1)
    for k in range(D):
        for i in range(n):
            rhs[k * n + i] = b[i][k]
            for j in range(k + 1):
                for v in range(n):
                    T[k * n + i, j * n + v] = A[i][v][k - j]
    sol = T.LUsolve(rhs)
    out = oracle.complex_step(s, cff, cst, x, prec=700, K=16)
    tol = Fraction(1, 2 ** 600)
    close = lambda got_re, got_im, want: (abs(got_re - Fraction(str(sympy.re(want)))) <= tol * (1 + abs(got_re)) and
                                          abs(got_im - Fraction(str(sympy.im(want)))) <= tol * (1 + abs(got_im)))
    ebr, ebi = exact(out["b"][0]), exact(out["b"][1])
    eAr, eAi = exact(out["A"][0]), exact(out["A"][1])
    exr, exi = exact(out["x"][0]), exact(out["x"][1])
    for i in range(n):
        for k in range(D):
            assert close(ebr[i, k], ebi[i, k], sympy.nsimplify(b[i][k]))
            assert close(exr[i, k], exi[i, k], sympy.expand(_cval(x, (i, k)) + sol[k * n + i]))
            for j in range(n):
                assert close(eAr[k, i, j], eAi[k, i, j], sympy.expand(A[i][j][k]))


def test_complex_real_case_and_conjugation():
    """With zero imaginary parts the complex oracle is the real one: b and A
    exactly (the same products), the step to the working bits (a complex
    division z conj(u) / |u|^2 rounds otherwise than z / u), with exactly
    zero imaginary outputs; conjugating every input conjugates every output
    exactly."""
    s = mdinputs.tiny(4, 4, 5, mons=3, kmin=1, kmax=3, exps=(1, 2), seed=9)
    cff, cst, x = mdinputs.complex_random(s, 9)
    real = oracle.newton_step(s, cff[0], cst[0], x[0], want_A=True)
    z = lambda a: np.stack([a[0], np.zeros_like(a[0])])
    c = oracle.complex_step(s, z(cff), z(cst), z(x))
    for key in ("b", "A"):
        assert np.array_equal(exact(c[key][0]), exact(real[key])) and not np.any(c[key][1])
    for key in ("x", "dx"):
        assert not np.any(c[key][1])
        assert np.max(oracle.absdiff(c[key][0], real[key])) <= 2.0 ** -(4 * 53 * 4 - 40) * np.abs(real[key][0]).max()
    conj = lambda a: np.stack([a[0], -a[1]])
    o1 = oracle.complex_step(s, cff, cst, x)
    o2 = oracle.complex_step(s, conj(cff), conj(cst), conj(x))
    for key in ("b", "A", "x", "dx"):
        assert np.array_equal(o2[key][0], o1[key][0]) and np.array_equal(o2[key][1], -o1[key][1])


@pytest.mark.parametrize("cols", [1, 2])
def test_complex_column_system_closed_form(cols):
    """The complex column systems (|alpha| = 1, Section 3): the closed-form
    right-hand side vanishes at x* to the rounding of the data, and Newton
    from x*(0) reaches x* with exact data (error at the oracle's working
    bits after log2(D) + 1 steps)."""
    s = mdinputs.complex_column_system(6, 7, 4, cols, seed=2)
    out = oracle.complex_step(s, s.cff, s.cst, s.xstar, step=False)
    b = np.abs(out["b"][:, 0])
    assert b.max() < 2.0 ** -200
    x = s.start()
    for _ in range(4):
        x = oracle.complex_step(s, s.cff, s.cst, x)["x"]
    err = max(oracle.absdiff(x[0], s.xstar[0]).max(), oracle.absdiff(x[1], s.xstar[1]).max())
    assert err < 2.0 ** -200


# --------------------------------------------------------------------------
# 12. reference md arithmetic against exact rational arithmetic
# --------------------------------------------------------------------------

def _arith_inputs(L, cnt, seed):
    """Seeded md operands with every limb drawn, plus exponent gaps and
    leading-limb cancellation, so a swapped operand or op code shows."""
    rng = np.random.default_rng(seed)
    a = mdinputs.random_md(rng, L, (cnt,), -1.0, 1.0)
    b = mdinputs.random_md(rng, L, (cnt,), -1.0, 1.0)
    c = mdinputs.random_md(rng, L, (cnt,), -1.0, 1.0)
    q = cnt // 3
    b[:, :q] *= 2.0 ** rng.integers(-30, 30, size=q)
    b[0, q:2 * q] = -a[0, q:2 * q]           # leading limbs cancel exactly
    return a, b, c


@pytest.mark.parametrize("L", [2, 4, 8])
@pytest.mark.parametrize("op", ["add", "sub", "mul", "div", "sqrt", "fma"])
def test_arith_against_exact_rationals(L, op):
    """oracle.arith(op) is the correctly rounded result at its working
    precision P: |out - exact| <= 2^(1-P) |exact| with the exact value from
    Fraction arithmetic on the limbs (sqrt: the exact root of exact squares,
    and out^2 = a within the same bound for arbitrary a).  fma is c + a*b.
    The export into doubles stops at the subnormal range, so at 8 limbs
    (P = 1696) an absolute floor of 2^-1070 is added to the bound."""
    a, b, c = _arith_inputs(L, 60, 700 + L)
    P = oracle.prec_bits(L)
    if op == "sqrt":
        # exact squares: y = m 2^-e with m an integer of 26 L bits, so y^2
        # has at most 52 L significant bits and fits in L limbs exactly
        rng = np.random.default_rng(710 + L)
        bits = 26 * L
        want = []
        for _ in range(40):
            m = int.from_bytes(rng.bytes(bits // 8 + 1), "little") % (1 << (bits - 1)) + (1 << (bits - 1))
            want.append(Fraction(m, 1 << (bits - 1 + int(rng.integers(-8, 8)))))
        a2 = to_md([w * w for w in want], L)
        assert all(md_value(a2[:, q]) == want[q] ** 2 for q in range(len(want)))
        got = exact(oracle.arith("sqrt", a2))
        assert all(g == w for g, w in zip(got, want))
        pos = a * np.sign(a[0])[None, :]
        got = exact(oracle.arith("sqrt", pos))
        for q in range(pos.shape[1]):
            av = md_value(pos[:, q])
            assert abs(got[q] ** 2 - av) <= Fraction(2) ** (2 - P) * av + Fraction(2) ** -1070
        return
    out = exact(oracle.arith(op, a, b, c))
    for q in range(a.shape[1]):
        x, y, z = md_value(a[:, q]), md_value(b[:, q]), md_value(c[:, q])
        want = {"add": x + y, "sub": x - y, "mul": x * y, "div": x / y, "fma": z + x * y}[op]
        bound = Fraction(2) ** (1 - P) * abs(want) + Fraction(2) ** -1070
        assert abs(out[q] - want) <= bound, (op, L, q)


def test_arith_op_codes_are_distinct():
    """Every op code gives a different result on the same operands (a
    mapping slip such as sub for add, or a*b + c read as a + b*c, shows)."""
    a, b, c = _arith_inputs(4, 12, 9)
    a = a * np.sign(a[0])[None, :]
    res = {op: exact(oracle.arith(op, a, b, c)) for op in ("add", "sub", "mul", "div", "fma")}
    ops = list(res)
    for i in range(len(ops)):
        for j in range(i + 1, len(ops)):
            assert any(u != v for u, v in zip(res[ops[i]], res[ops[j]])), (ops[i], ops[j])
    # fma operand order: c + a*b differs from a + b*c on generic data
    alt = [md_value(a[:, q]) + md_value(b[:, q]) * md_value(c[:, q]) for q in range(a.shape[1])]
    assert all(u != v for u, v in zip(res["fma"], alt))
