"""Oracle for the power-series Newton step (TEST INFRASTRUCTURE ONLY).

A plain, slow, arbitrary-precision CPU implementation in C with MPFR
(``oracle.c``), wrapped here with ctypes.  Only the tests, the smoke check and
the CPU-baseline leg of the benchmark may import it.  It shares no code with
the GPU library: inputs come from the seeded generators in ``mdinputs``.

Working precision of the oracle: four times the bits of the multiple doubles
under test (dd 424, qd 848, od 1696 bits) unless a caller asks for more.

Every function takes and returns limb-major arrays.  Results are returned as
"expansions" of K doubles (default 4L+2) that keep the oracle's full precision;
``absdiff`` measures |gpu - oracle| exactly.

Parity pins (see tests/test_oracle_pins.py): brute-force exact rationals on
tiny systems, the paper's exponential-series worked example (Section 3),
binomial series, classical Newton at D=1, one-step convergence of linear
systems, quadratic convergence from a manufactured solution, the paper's
Table 1 values.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")
_MPFR_INC = "/opt/conda/include"
_LIBS = ["/usr/lib/x86_64-linux-gnu/libmpfr.so.6", "/usr/lib/x86_64-linux-gnu/libgmp.so.10"]

_lib = None


def build() -> str:
    """Compile liboracle.so with gcc (C + MPFR + OpenMP)."""
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-I" + _MPFR_INC, "-o", _SO + ".tmp", _SRC] + _LIBS
    subprocess.run(cmd, check=True)
    os.replace(_SO + ".tmp", _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        i32p = ctypes.POINTER(ctypes.c_int32)
        dp = ctypes.POINTER(ctypes.c_double)
        ci = ctypes.c_int
        L.ora_eval.argtypes = [ci, ci, ci, ci, i32p, i32p, i32p, i32p, ci, dp, dp, dp, ci, ci, ci, dp, dp, dp]
        L.ora_newton_step.argtypes = [ci, ci, ci, ci, i32p, i32p, i32p, i32p, ci, dp, dp, dp, ci, dp, dp, dp, dp]
        L.ora_toeplitz_solve.argtypes = [ci, ci, ci, ci, dp, dp, ci, dp]
        L.ora_manufacture.argtypes = [ci, ci, ci, ci, i32p, i32p, i32p, i32p, ci, dp, dp, ci, dp]
        L.ora_round.argtypes = [ci, ci, dp, ci, ci, dp]
        L.ora_absdiff.argtypes = [ci, ci, dp, ci, dp, ci, dp]
        L.ora_qr_check.argtypes = [ci, ci, ci, dp, dp, dp, dp]
        L.ora_rdiag.argtypes = [ci, ci, ci, dp, ci, dp]
        L.ora_set_threads.argtypes = [ci]
        L.ora_arith.argtypes = [ci, ci, ci, dp, dp, dp, ci, ci, dp]
        L.ora_adjoint_solve.argtypes = [ci, ci, ci, ci, dp, dp, ci, dp]
        L.ora_coef_grad.argtypes = [ci, ci, ci, ci, i32p, i32p, i32p, i32p, ci, dp, ci, dp, ci, dp]
        L.ora_complex_step.argtypes = [ci, ci, ci, ci, i32p, i32p, i32p, i32p, ci, dp, dp, dp, ci, dp, dp, dp, dp]
        L.ora_linear_residual.argtypes = [ci, ci, ci, ci, dp, dp, dp, ci, i32p, ci, dp, dp]
        L.ora_window_step.argtypes = [ci, ci, ci, ci, i32p, i32p, i32p, i32p, ci, dp, dp, dp, dp, ci, ci, dp, dp,
                                      dp, dp]
        _lib = L
    return _lib


def set_threads(t: int) -> None:
    lib().ora_set_threads(int(t))


def threads() -> int:
    return int(lib().ora_get_threads())


def inexact_inputs() -> int:
    """How many multiple-double inputs were not exactly representable (must be 0)."""
    return int(lib().ora_inexact_count())


def prec_bits(L: int) -> int:
    return 4 * 53 * L


def _d(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _i(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _c64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _c32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


class OracleError(RuntimeError):
    pass


def _check(rc: int, what: str):
    if rc == -2:
        raise OracleError(f"{what}: A_0 is singular")
    if rc != 0:
        raise OracleError(f"{what}: error {rc}")


def _pad(a, L):
    """Zero-pad an expansion to L limbs (the value is unchanged)."""
    a = _c64(a)
    if a.shape[0] >= L:
        return a
    return np.concatenate([a, np.zeros((L - a.shape[0],) + a.shape[1:])])


def _common(*arrs):
    L = max(a.shape[0] for a in arrs)
    return L, [_pad(a, L) for a in arrs]


def _sys_args(sys):
    return (_c32(sys.poly_ptr), _c32(sys.mon_ptr), _c32(sys.var), _c32(sys.exp))


def eval_diff(sys, cff, cst, x, rows=None, K=None, prec=None):
    """b = -p(x) and A = p'(x) for rows ``rows=(r0, r1)``.

    Returns b[K, rows, D], A[K, D, rows, n] and the row scale
    max_s (|c_{i,0,s}| + sum_m |value_{m,s}|) used to judge b near a root."""
    L0 = cff.shape[0]  # the system's precision sets the defaults
    L, (cff, cst, x) = _common(cff, cst, x)
    K = K or 4 * L0 + 2
    prec = prec or prec_bits(L0)
    r0, r1 = rows or (0, sys.n)
    R = r1 - r0
    pp, mp, var, ex = _sys_args(sys)
    b = np.zeros((K, R, sys.D))
    A = np.zeros((K, sys.D, R, sys.n))
    sc = np.zeros(R)
    rc = lib().ora_eval(prec, sys.n, sys.D, sys.m, _i(pp), _i(mp), _i(var), _i(ex), L, _d(cff), _d(cst),
                        _d(x), r0, r1, K, _d(b), _d(A), _d(sc))
    _check(rc, "ora_eval")
    return b, A, sc


def newton_step(sys, cff, cst, x, K=None, prec=None, want_A=False):
    """One Newton step from x; returns dict of expansions x, dx, b (and A)."""
    L0 = cff.shape[0]  # the system's precision sets the defaults
    L, (cff, cst, x) = _common(cff, cst, x)
    K = K or 4 * L0 + 2
    prec = prec or prec_bits(L0)
    pp, mp, var, ex = _sys_args(sys)
    out = {k: np.zeros((K, sys.n, sys.D)) for k in ("x", "dx", "b")}
    A = np.zeros((K, sys.D, sys.n, sys.n)) if want_A else None
    rc = lib().ora_newton_step(prec, sys.n, sys.D, sys.m, _i(pp), _i(mp), _i(var), _i(ex), L, _d(cff),
                               _d(cst), _d(x), K, _d(out["x"]), _d(out["dx"]), _d(out["b"]),
                               _d(A) if want_A else ctypes.POINTER(ctypes.c_double)())
    _check(rc, "ora_newton_step")
    if want_A:
        out["A"] = A
    return out


def toeplitz_solve(A, rhs, K=None, prec=None):
    """Solve the block lower-triangular Toeplitz system; A[L, D, n, n], rhs[L, n, D]."""
    L0 = A.shape[0]
    L, (A, rhs) = _common(A, rhs)
    _, D, n, _ = A.shape
    K = K or 4 * L0 + 2
    prec = prec or prec_bits(L0)
    dx = np.zeros((K, n, D))
    rc = lib().ora_toeplitz_solve(prec, n, D, L, _d(A), _d(rhs), K, _d(dx))
    _check(rc, "ora_toeplitz_solve")
    return dx


def linear_residual(A, b, dx, rows=None, K=None, prec=None):
    """r = b - T dx for the block Toeplitz matrix T of A[L, D, n, n] (oracle
    layout), b and dx [L, n, D], on the rows listed (all rows when None).
    Returns (r [K, nrows, D] expansions, scale [nrows, D]: |b| plus the sum of
    the absolute products)."""
    L0 = max(A.shape[0], b.shape[0], dx.shape[0])
    L, (A, b, dx) = _common(A, b, dx)
    _, D, n, _ = A.shape
    K = K or 4 * L0 + 2
    prec = prec or prec_bits(L0)
    rr = np.arange(n, dtype=np.int32) if rows is None else _c32(rows)
    r = np.zeros((K, len(rr), D))
    sc = np.zeros((len(rr), D))
    rc = lib().ora_linear_residual(prec, n, D, L, _d(A), _d(b), _d(dx), len(rr), _i(rr), K, _d(r), _d(sc))
    _check(rc, "ora_linear_residual")
    return r, sc


def complex_step(sys, cff, cst, x, K=None, prec=None, step=True):
    """Complex data (Section 5.2): cff [2, L, m], cst and x [2, L, n, D] (real
    plane, imaginary plane).  Returns a dict of expansions b [2, K, n, D],
    A [2, K, D, n, n] and, with step, x + dx and dx [2, K, n, D] (one Newton
    step by complex LU and block forward substitution)."""
    L0 = cff.shape[1]
    L = max(cff.shape[1], cst.shape[1], x.shape[1])
    pad = lambda a: np.stack([_pad(a[0], L), _pad(a[1], L)])
    cff, cst, x = pad(cff), pad(cst), pad(x)
    K = K or 4 * L0 + 2
    prec = prec or prec_bits(L0)
    n, D = sys.n, sys.D
    pp, mp, var, ex = _sys_args(sys)
    out = {"b": np.zeros((2, K, n, D)), "A": np.zeros((2, K, D, n, n))}
    null = ctypes.POINTER(ctypes.c_double)()
    if step:
        out["x"] = np.zeros((2, K, n, D))
        out["dx"] = np.zeros((2, K, n, D))
    rc = lib().ora_complex_step(prec, n, D, sys.m, _i(pp), _i(mp), _i(var), _i(ex), L, _d(cff), _d(cst), _d(x), K,
                                _d(out["b"]), _d(out["A"]), _d(out["x"]) if step else null,
                                _d(out["dx"]) if step else null)
    _check(rc, "ora_complex_step")
    return out


def manufacture(sys, Lout=None, prec=None):
    """Constant series c_{i,0} = -sum_m c_m x*^{a_m}, rounded to Lout limbs."""
    L = sys.cff.shape[0]
    Lout = Lout or L
    prec = prec or prec_bits(max(L, Lout))
    pp, mp, var, ex = _sys_args(sys)
    cst = np.zeros((Lout, sys.n, sys.D))
    rc = lib().ora_manufacture(prec, sys.n, sys.D, sys.m, _i(pp), _i(mp), _i(var), _i(ex), L,
                               _d(_c64(sys.cff)), _d(_c64(sys.xstar)), Lout, _d(cst))
    _check(rc, "ora_manufacture")
    return cst


def round_md(e: np.ndarray, L: int, prec=None) -> np.ndarray:
    """Round expansions e[K, ...] to L-limb multiple doubles (limb by limb to nearest)."""
    K = e.shape[0]
    shape = e.shape[1:]
    flat = _c64(e.reshape(K, -1))
    cnt = flat.shape[1]
    out = np.zeros((L, cnt))
    lib().ora_round(prec or 4 * 53 * max(K, L), K, _d(flat), cnt, L, _d(out))
    return out.reshape((L,) + shape)


def absdiff(u: np.ndarray, w: np.ndarray, prec=None) -> np.ndarray:
    """|u - w| computed exactly for expansions u[Lu, ...], w[Lw, ...]."""
    Lu, Lw = u.shape[0], w.shape[0]
    assert u.shape[1:] == w.shape[1:]
    shape = u.shape[1:]
    uf, wf = _c64(u.reshape(Lu, -1)), _c64(w.reshape(Lw, -1))
    cnt = uf.shape[1]
    out = np.zeros(cnt)
    lib().ora_absdiff(prec or 53 * (Lu + Lw) + 2200, Lu, _d(uf), Lw, _d(wf), cnt, _d(out))
    return out.reshape(shape)


def qr_check(A0, qr, tau, prec=None):
    """(max|QR - A0|/max|A0|, max|Q^T Q - I|) for a compact Householder QR."""
    L, n, _ = A0.shape
    out = np.zeros(2)
    lib().ora_qr_check(prec or prec_bits(L), n, L, _d(_c64(A0)), _d(_c64(qr)), _d(_c64(tau)), _d(out))
    return float(out[0]), float(out[1])


def rdiag(A0, K=None, prec=None):
    """|R_ii| of the QR factorization of A0[L, n, n] (unique), as expansions [K, n]."""
    L, n, _ = A0.shape
    K = K or 4 * L + 2
    out = np.zeros((K, n))
    rc = lib().ora_rdiag(prec or prec_bits(L), n, L, _d(_c64(A0)), K, _d(out))
    _check(rc, "ora_rdiag")
    return out


def rel_err_series(gpu: np.ndarray, ora: np.ndarray, axis_series=-1) -> np.ndarray:
    """Normwise relative error per series: max_k |gpu-ora| / max_k |ora| (0/0 = 0).

    gpu[L, ..., D] and ora[K, ..., D]; the last axis indexes the coefficients."""
    diff = absdiff(gpu, ora)
    mag = np.abs(ora[0])
    num = diff.max(axis=axis_series)
    den = mag.max(axis=axis_series)
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.where(den > 0, num / np.where(den > 0, den, 1.0), np.where(num > 0, np.inf, 0.0))
    return r


ARITH_OPS = {"add": 0, "sub": 1, "mul": 2, "div": 3, "sqrt": 4, "fma": 5}


def arith(op, a, b=None, c=None, K=None, prec=None):
    """Reference a+b, a-b, a*b, a/b, sqrt(a) or c+a*b for md arrays [L, count]."""
    L, count = a.shape
    K = K or 4 * L + 2
    opc = ARITH_OPS[op]
    z = np.zeros((L, count))
    out = np.zeros((K, count))
    rc = lib().ora_arith(prec or prec_bits(L), opc, L, _d(_c64(a)), _d(_c64(b if b is not None else z)),
                         _d(_c64(c if c is not None else z)), count, K, _d(out))
    _check(rc, "ora_arith")
    return out


def adjoint_solve(A, g, K=None, prec=None):
    """Solve T^T lambda = g for the block Toeplitz T of A[L, D, n, n]; g[L, n, D]."""
    L0 = A.shape[0]
    L, (A, g) = _common(A, g)
    _, D, n, _ = A.shape
    K = K or 4 * L0 + 2
    prec = prec or prec_bits(L0)
    lam = np.zeros((K, n, D))
    rc = lib().ora_adjoint_solve(prec, n, D, L, _d(A), _d(g), K, _d(lam))
    _check(rc, "ora_adjoint_solve")
    return lam


def coef_grad(sys, x, lam, K=None, prec=None):
    """dL/dc_m = -sum_k lambda_{i(m),k} [x^{a_m}]_k for x[L, n, D], lambda[Ll, n, D]."""
    L = x.shape[0]
    K = K or 4 * L + 2
    prec = prec or prec_bits(L)
    pp, mp, var, ex = _sys_args(sys)
    out = np.zeros((K, sys.m))
    rc = lib().ora_coef_grad(prec, sys.n, sys.D, sys.m, _i(pp), _i(mp), _i(var), _i(ex), L, _d(_c64(x)),
                             lam.shape[0], _d(_c64(lam)), K, _d(out))
    _check(rc, "ora_coef_grad")
    return out


def window_step(sys, cff, cst, x, lo, hi, x_kept=None, K=None, prec=None):
    """One step of the staggered method (Sections 4 and 5.3) on the problem
    truncated at order ``hi``: b = -p(x) mod t^hi, A = p'(x) mod t^hi, the
    block solve with dx_k = 0 for k < lo, and x_k + dx_k for k < hi.  With
    ``x_kept`` the diagonal block is A_0 at x_kept's leading coefficients (the
    factorization kept from an earlier step: a chord step), else at x.

    Returns a dict of expansions x, dx, b of shape [K, n, D]: coefficients at
    and above hi are x's own (dx and b zero there), and ``scale`` [D], the
    size max_i (|c_{i,0,k}| + sum_m |value_{m,k}|) of the terms of b_k (zero
    at and above hi)."""
    L0 = cff.shape[0]
    L, (cff, cst, x) = _common(cff, cst, x)
    K = K or 4 * L0 + 2
    prec = prec or prec_bits(L0)
    n, D = sys.n, sys.D
    if not (0 <= lo < hi <= D):
        raise ValueError("need 0 <= lo < hi <= D")
    xt = _c64(x[:, :, :hi])
    ct = _c64(cst[:, :, :hi])
    xs = None
    if x_kept is not None:
        xs = _c64(_pad(x_kept, L)[:L, :, 0])
    pp, mp, var, ex = _sys_args(sys)
    out = {k: np.zeros((K, n, hi)) for k in ("x", "dx", "b")}
    sc = np.zeros(hi)
    null = ctypes.POINTER(ctypes.c_double)()
    rc = lib().ora_window_step(prec, n, hi, sys.m, _i(pp), _i(mp), _i(var), _i(ex), L, _d(cff), _d(ct), _d(xt),
                               _d(xs) if xs is not None else null, lo, K, _d(out["x"]), _d(out["dx"]),
                               _d(out["b"]), _d(sc))
    _check(rc, "ora_window_step")
    res = {}
    for k in ("dx", "b"):
        full = np.zeros((K, n, D))
        full[:, :, :hi] = out[k]
        res[k] = full
    xf = np.zeros((K, n, D))
    xf[:L] = x  # coefficients at and above hi: x itself (an exact expansion)
    xf[:, :, :hi] = out["x"]
    res["x"] = xf
    res["scale"] = np.concatenate([sc, np.zeros(D - hi)])
    return res


def converge(sys, cff, cst, x0, steps, K=None, prec=None):
    """Newton steps carried in full oracle precision (K-double expansions)."""
    x = x0
    for _ in range(steps):
        x = newton_step(sys, cff, cst, x, K=K, prec=prec)["x"]
    return x


def loss_top_grad(x, ktop):
    """Gradient of L = sum_i sum_{k >= ktop} x_{i,k}^2: 2 x_{i,k} for k >= ktop, else 0."""
    g = np.zeros_like(x)
    g[:, :, ktop:] = 2.0 * x[:, :, ktop:]  # exact: doubling every limb
    return g
