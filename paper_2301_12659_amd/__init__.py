"""Python binding of libmdnewton (argument marshalling only).

Every function mirrors a C entry point of include/mdnewton.h and takes
torch.float64 tensors that live on the GPU, limb-major with a leading limb
axis of size L (2, 4 or 8).  Shapes are checked here before any launch; all
arithmetic runs in the HIP kernels of the shared library.  There is no CPU
fallback: if the library is missing, importing this package raises.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmdnewton.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "mdnewton.h")

MD_OK, MD_EINVAL, MD_ESINGULAR, MD_ENONFINITE, MD_EHIP, MD_ENOSPACE = 0, -1, -2, -3, -4, -5
MD_D, MD_DD, MD_QD, MD_OD = 1, 2, 4, 8
OPS = {"add": 0, "sub": 1, "mul": 2, "div": 3, "sqrt": 4, "fma": 5, "dot": 6}
STATUS_NAMES = {0: "ok", -2: "singular", -3: "nonfinite"}

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run paper_2301_12659_amd.build.build() (or __graft_entry__.build())")

# torch first: it carries a HIP runtime of its own, and the library must bind
# to that one (loaded first, it satisfies the library's dependency by its
# soname).  Loaded the other way round, the process holds two HIP runtimes
# and the second one sees no device.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

_vp = ctypes.c_void_p
_i32 = ctypes.c_int
_i32p = ctypes.POINTER(ctypes.c_int32)
_szp = ctypes.POINTER(ctypes.c_size_t)

_lib.md_plan_create.argtypes = [_i32, _i32, _i32, _i32, _i32p, _i32p, _i32p, _i32p, ctypes.POINTER(_vp)]
_lib.md_plan_destroy.argtypes = [_vp]
_lib.md_workspace_size.argtypes = [_vp, _szp]
_lib.md_eval_diff.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]
_lib.md_qr_workspace_size.argtypes = [_i32, _i32, _szp]
_lib.md_qr.argtypes = [_i32, _i32, _vp, _vp, _vp, ctypes.c_size_t, _vp, _vp]
_lib.md_qr_noalloc.argtypes = [_i32, _i32, _vp, _vp, _vp, _vp]
_lib.md_solve_workspace_size.argtypes = [_i32, _i32, _i32, _szp]
_lib.md_series_solve.argtypes = [_i32, _i32, _i32, _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp, _vp]
_lib.md_newton_step.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]
_lib.md_newton_steps.argtypes = [_vp, _i32, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]
_lib.md_newton_step_mixed.argtypes = [_vp, _i32, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]
_lib.md_newton_step_window.argtypes = [_vp, _i32, _i32, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t,
                                       _vp]
_lib.md_stagger_next_order.argtypes = [_i32, _i32]


class StaggerReport(ctypes.Structure):
    """md_stagger_report: steps, converged, lo, hi, factorizations."""
    _fields_ = [("steps", ctypes.c_int32), ("converged", ctypes.c_int32), ("lo", ctypes.c_int32),
                ("hi", ctypes.c_int32), ("factorizations", ctypes.c_int32)]


_lib.md_newton_staggered.argtypes = [_vp, _i32, _i32, _i32, ctypes.c_double, _vp, _vp, _vp, _i32p,
                                     ctypes.POINTER(ctypes.c_double), ctypes.POINTER(StaggerReport), _vp, _vp, _vp,
                                     ctypes.c_size_t, _vp]
_lib.md_linear_residual.argtypes = [_i32, _i32, _i32, _vp, _vp, _vp, _i32, _vp, _vp, _vp, _vp, _vp]
_lib.md_step_arrays.argtypes = [_vp, _vp, ctypes.c_size_t, ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                ctypes.POINTER(_vp)]
_lib.md_complex_workspace_size.argtypes = [_vp, _szp]
_lib.md_eval_diff_complex.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]
_lib.md_newton_step_complex.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]
_lib.md_arith.argtypes = [_i32, _i32, ctypes.c_int64, _vp, _vp, _vp, _vp]
_lib.md_last_error.restype = ctypes.c_char_p
_lib.md_adjoint_workspace_size.argtypes = [_i32, _i32, _i32, _szp]
_lib.md_adjoint_solve.argtypes = [_i32, _i32, _i32, _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp, _vp]
_lib.md_coef_grad.argtypes = [_vp, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]
_lib.md_timing_enable.argtypes = [_i32]
_i64p = ctypes.POINTER(ctypes.c_int64)
_lib.md_batch_create.argtypes = [_i32, _i32, _i32p, _i32p, _i32p, _i32p, _i32p, _i32p, _i32p, ctypes.POINTER(_vp)]
_lib.md_batch_destroy.argtypes = [_vp]
_lib.md_batch_offsets.argtypes = [_vp, _i64p, _i64p, _i64p, _i64p]
_lib.md_batch_workspace_size.argtypes = [_vp, _szp]
_lib.md_batch_newton_step.argtypes = [_vp, _i32, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]
_lib.md_batch_autotune.argtypes = [_vp, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp, _i32p]
_lib.md_batch_set_tiles.argtypes = [_vp, _i32p]
_lib.md_timing_read.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]

# Kernel classes of md_timing_read (the paper's kernel types, Table 4).
TIMING_CLASSES = ["convolutions", "assembly", "qr", "qhb_bs", "gemm", "updates", "x_update"]


def exported_functions():
    """Names of the functions declared in include/mdnewton.h."""
    with open(HEADER) as f:
        text = f.read()
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*(md_\w+)\s*\(", text, re.M)))


class MdError(RuntimeError):
    def __init__(self, code, what):
        msg = _lib.md_last_error().decode()
        super().__init__(f"{what} failed with {code}: {msg}")
        self.code = code


def _check(rc, what):
    if rc != MD_OK:
        raise MdError(rc, what)


def _stream(stream):
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return _vp(s.cuda_stream)


def _ptr(t, shape, name):
    """Device pointer of a contiguous float64/int32 CUDA tensor of the given shape."""
    import torch

    if t is None:
        return _vp(0)
    if not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    if t.dtype not in (torch.float64, torch.int32):
        raise ValueError(f"{name} must be float64 or int32")
    return _vp(t.data_ptr())


def _i32arr(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(_i32p)


class Plan:
    """md_plan: a validated system structure resident on the device."""

    def __init__(self, prec, n, d, poly_ptr, mon_ptr, var, exp):
        self.prec, self.n, self.d = int(prec), int(n), int(d)
        self.D = self.d + 1
        self._keep = [_i32arr(poly_ptr), _i32arr(mon_ptr), _i32arr(var), _i32arr(exp)]
        self.m = int(len(self._keep[1][0]) - 1)
        self.nnz = int(len(self._keep[2][0]))
        h = _vp()
        rc = _lib.md_plan_create(self.prec, self.n, self.d, self.m, self._keep[0][1], self._keep[1][1],
                                 self._keep[2][1], self._keep[3][1], ctypes.byref(h))
        _check(rc, "md_plan_create")
        self._h = h

    @classmethod
    def from_system(cls, sys):
        return cls(sys.L, sys.n, sys.d, sys.poly_ptr, sys.mon_ptr, sys.var, sys.exp)

    def workspace_bytes(self):
        v = ctypes.c_size_t()
        _check(_lib.md_workspace_size(self._h, ctypes.byref(v)), "md_workspace_size")
        return int(v.value)

    def close(self):
        if getattr(self, "_h", None):
            _lib.md_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """md_batch: many independent systems (paths) stepped together.

    `systems` are objects with L, n, d, poly_ptr, mon_ptr, var, exp (the
    mdinputs.System fields); all share the precision `prec`.  Device arrays
    are packed: x and cst [L, x_total], cff [L, cff_total]; pack/unpack
    convert from and to per-path arrays."""

    BUCKETS = 9

    def __init__(self, systems, prec=None):
        self.prec = int(prec if prec is not None else systems[0].L)
        self.P = len(systems)
        n = np.array([s.n for s in systems], dtype=np.int32)
        d = np.array([s.d for s in systems], dtype=np.int32)
        m = np.array([len(s.mon_ptr) - 1 for s in systems], dtype=np.int32)
        cat = lambda f: np.concatenate([np.asarray(getattr(s, f), dtype=np.int32) for s in systems])
        self._keep = [_i32arr(n), _i32arr(d), _i32arr(m), _i32arr(cat("poly_ptr")), _i32arr(cat("mon_ptr")),
                      _i32arr(cat("var")), _i32arr(cat("exp"))]
        h = _vp()
        rc = _lib.md_batch_create(self.prec, self.P, *[k[1] for k in self._keep], ctypes.byref(h))
        _check(rc, "md_batch_create")
        self._h = h
        self.n, self.D, self.m = n.tolist(), (d + 1).tolist(), m.tolist()
        xo = (ctypes.c_int64 * self.P)()
        co = (ctypes.c_int64 * self.P)()
        xt, ct = ctypes.c_int64(), ctypes.c_int64()
        _check(_lib.md_batch_offsets(self._h, xo, co, ctypes.byref(xt), ctypes.byref(ct)), "md_batch_offsets")
        self.x_off, self.cff_off = list(xo), list(co)
        self.x_total, self.cff_total = int(xt.value), int(ct.value)

    def workspace_bytes(self):
        v = ctypes.c_size_t()
        _check(_lib.md_batch_workspace_size(self._h, ctypes.byref(v)), "md_batch_workspace_size")
        return int(v.value)

    def pack_series(self, arrays):
        """[L, n_p, D_p] per path -> [L, x_total] (numpy)."""
        out = np.zeros((self.prec, self.x_total))
        for p, a in enumerate(arrays):
            sz = self.n[p] * self.D[p]
            out[:, self.x_off[p]:self.x_off[p] + sz] = np.asarray(a)[:self.prec].reshape(self.prec, sz)
        return out

    def unpack_series(self, packed):
        packed = np.asarray(packed)
        return [packed[:, self.x_off[p]:self.x_off[p] + self.n[p] * self.D[p]].reshape(-1, self.n[p], self.D[p])
                for p in range(self.P)]

    def pack_cff(self, arrays):
        out = np.zeros((self.prec, self.cff_total))
        for p, a in enumerate(arrays):
            out[:, self.cff_off[p]:self.cff_off[p] + self.m[p]] = np.asarray(a)[:self.prec]
        return out

    def step(self, cff, cst, x, status, norms, ws, prec_solve=None, stream=None):
        L = self.prec
        rc = _lib.md_batch_newton_step(self._h, int(prec_solve or L), _ptr(cff, (L, self.cff_total), "cff"),
                                       _ptr(cst, (L, self.x_total), "cst"), _ptr(x, (L, self.x_total), "x"),
                                       _ptr(status, (self.P,), "status"), _ptr(norms, (2 * self.P,), "norms"),
                                       _ptr(ws, None, "ws"), ws.numel() * 8, _stream(stream))
        _check(rc, "md_batch_newton_step")

    def autotune(self, cff, cst, x, x_scratch, status, norms, ws, prec_solve=None, stream=None):
        L = self.prec
        chosen = (ctypes.c_int32 * self.BUCKETS)()
        rc = _lib.md_batch_autotune(self._h, int(prec_solve or L), _ptr(cff, (L, self.cff_total), "cff"),
                                    _ptr(cst, (L, self.x_total), "cst"), _ptr(x, (L, self.x_total), "x"),
                                    _ptr(x_scratch, (L, self.x_total), "x_scratch"),
                                    _ptr(status, (self.P,), "status"), _ptr(norms, (2 * self.P,), "norms"),
                                    _ptr(ws, None, "ws"), ws.numel() * 8, _stream(stream), chosen)
        _check(rc, "md_batch_autotune")
        return list(chosen)

    def set_tiles(self, tiles):
        arr, ptr = _i32arr(tiles)
        _check(_lib.md_batch_set_tiles(self._h, ptr), "md_batch_set_tiles")

    def close(self):
        if getattr(self, "_h", None):
            _lib.md_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def workspace(nbytes, device="cuda"):
    import torch

    return torch.empty(max(int(nbytes), 8) // 8 + 1, dtype=torch.float64, device=device)


def eval_diff(plan: Plan, cff, cst, x, b, A, ws, stream=None):
    L, n, D, m = plan.prec, plan.n, plan.D, plan.m
    rc = _lib.md_eval_diff(plan._h, _ptr(cff, (L, m), "cff"), _ptr(cst, (L, n, D), "cst"), _ptr(x, (L, n, D), "x"),
                           _ptr(b, (L, n, D), "b"), _ptr(A, (L, n, n, D), "A"), _ptr(ws, None, "ws"),
                           ws.numel() * 8, _stream(stream))
    _check(rc, "md_eval_diff")


def qr_workspace_bytes(prec, n):
    v = ctypes.c_size_t()
    _check(_lib.md_qr_workspace_size(int(prec), int(n), ctypes.byref(v)), "md_qr_workspace_size")
    return int(v.value)


def qr(prec, n, a0, tau, status, ws=None, stream=None):
    L = int(prec)
    if ws is None:
        ws = workspace(qr_workspace_bytes(L, n), a0.device)
    rc = _lib.md_qr(L, int(n), _ptr(a0, (L, n, n), "a0"), _ptr(tau, (L, n), "tau"), _ptr(ws, None, "ws"),
                    ws.numel() * 8, _stream(stream), _ptr(status, (1,), "status"))
    _check(rc, "md_qr")


def qr_noalloc(prec, n, a0, tau, status, stream=None):
    """md_qr without a workspace: the scratch is the library's static device
    array (for callers that cannot allocate)."""
    L = int(prec)
    rc = _lib.md_qr_noalloc(L, int(n), _ptr(a0, (L, n, n), "a0"), _ptr(tau, (L, n), "tau"), _stream(stream),
                            _ptr(status, (1,), "status"))
    _check(rc, "md_qr_noalloc")


def solve_workspace_bytes(prec, n, d):
    v = ctypes.c_size_t()
    _check(_lib.md_solve_workspace_size(int(prec), int(n), int(d), ctypes.byref(v)), "md_solve_workspace_size")
    return int(v.value)


def series_solve(prec, n, d, qr_, tau, A, rhs_dx, ws, status, stream=None):
    L, D = int(prec), int(d) + 1
    rc = _lib.md_series_solve(L, int(n), int(d), _ptr(qr_, (L, n, n), "qr"), _ptr(tau, (L, n), "tau"),
                              _ptr(A, (L, n, n, D), "A"), _ptr(rhs_dx, (L, n, D), "rhs_dx"), _ptr(ws, None, "ws"),
                              ws.numel() * 8, _stream(stream), _ptr(status, (1,), "status"))
    _check(rc, "md_series_solve")


def newton_step(plan: Plan, cff, cst, x, status, norms, ws, stream=None):
    L, n, D, m = plan.prec, plan.n, plan.D, plan.m
    rc = _lib.md_newton_step(plan._h, _ptr(cff, (L, m), "cff"), _ptr(cst, (L, n, D), "cst"),
                             _ptr(x, (L, n, D), "x"), _ptr(status, (1,), "status"),
                             _ptr(norms, (2, D), "norms"), _ptr(ws, None, "ws"), ws.numel() * 8, _stream(stream))
    _check(rc, "md_newton_step")


def newton_steps(plan: Plan, count, cff, cst, x, status, norms, ws, stream=None):
    """md_newton_steps: count plain steps, each factorization beside the previous step."""
    L, n, D, m = plan.prec, plan.n, plan.D, plan.m
    rc = _lib.md_newton_steps(plan._h, int(count), _ptr(cff, (L, m), "cff"), _ptr(cst, (L, n, D), "cst"),
                              _ptr(x, (L, n, D), "x"), _ptr(status, (1,), "status"),
                              _ptr(norms, (2, D), "norms"), _ptr(ws, None, "ws"), ws.numel() * 8, _stream(stream))
    _check(rc, "md_newton_steps")


def newton_step_mixed(plan: Plan, prec_solve, cff, cst, x, status, norms, ws, stream=None):
    L, n, D, m = plan.prec, plan.n, plan.D, plan.m
    rc = _lib.md_newton_step_mixed(plan._h, int(prec_solve), _ptr(cff, (L, m), "cff"), _ptr(cst, (L, n, D), "cst"),
                                   _ptr(x, (L, n, D), "x"), _ptr(status, (1,), "status"),
                                   _ptr(norms, (2, D), "norms"), _ptr(ws, None, "ws"), ws.numel() * 8,
                                   _stream(stream))
    _check(rc, "md_newton_step_mixed")


def newton_step_window(plan: Plan, prec_solve, lo, hi, keep_factorization, cff, cst, x, status, norms, ws,
                       stream=None):
    """md_newton_step_window: one staggered step on the window lo..hi-1."""
    L, n, D, m = plan.prec, plan.n, plan.D, plan.m
    rc = _lib.md_newton_step_window(plan._h, int(prec_solve), int(lo), int(hi), int(bool(keep_factorization)),
                                    _ptr(cff, (L, m), "cff"), _ptr(cst, (L, n, D), "cst"), _ptr(x, (L, n, D), "x"),
                                    _ptr(status, (1,), "status"), _ptr(norms, (2, D), "norms"), _ptr(ws, None, "ws"),
                                    ws.numel() * 8, _stream(stream))
    _check(rc, "md_newton_step_window")


def linear_residual(prec, n, d, A, b, dx, r, rows=None, norm1=None, status=None, stream=None):
    """md_linear_residual: r = b - T dx on the rows listed (all when None).

    A [L, n, n, D], b and dx [L, n, D] (tensors, or raw device addresses from
    step_arrays), r [L, nrows, D]; rows an int32 device tensor; norm1 [D]."""
    L, D = int(prec), int(d) + 1
    nrows = n if rows is None else int(rows.numel())
    raw = lambda t, shape, name: _vp(t) if isinstance(t, int) else _ptr(t, shape, name)
    rc = _lib.md_linear_residual(L, int(n), int(d), raw(A, (L, n, n, D), "A"), raw(b, (L, n, D), "b"),
                                 raw(dx, (L, n, D), "dx"), nrows, _ptr(rows, (nrows,), "rows"),
                                 _ptr(r, (L, nrows, D), "r"), _ptr(norm1, (D,), "norm1"),
                                 _ptr(status, (1,), "status"), _stream(stream))
    _check(rc, "md_linear_residual")


def step_arrays(plan: Plan, ws):
    """Device addresses (b, A, dx) where the last Newton step on ws left its arrays."""
    b, A, dx = _vp(), _vp(), _vp()
    _check(_lib.md_step_arrays(plan._h, _ptr(ws, None, "ws"), ws.numel() * 8, ctypes.byref(b), ctypes.byref(A),
                               ctypes.byref(dx)), "md_step_arrays")
    return int(b.value), int(A.value), int(dx.value)


def complex_workspace_bytes(plan: Plan):
    v = ctypes.c_size_t()
    _check(_lib.md_complex_workspace_size(plan._h, ctypes.byref(v)), "md_complex_workspace_size")
    return int(v.value)


def eval_diff_complex(plan: Plan, cff, cst, x, b, A, ws, stream=None):
    """md_eval_diff_complex: complex arrays [2, L, ...] (real plane, imaginary plane)."""
    L, n, D, m = plan.prec, plan.n, plan.D, plan.m
    rc = _lib.md_eval_diff_complex(plan._h, _ptr(cff, (2, L, m), "cff"), _ptr(cst, (2, L, n, D), "cst"),
                                   _ptr(x, (2, L, n, D), "x"), _ptr(b, (2, L, n, D), "b"),
                                   _ptr(A, (2, L, n, n, D), "A"), _ptr(ws, None, "ws"), ws.numel() * 8,
                                   _stream(stream))
    _check(rc, "md_eval_diff_complex")


def newton_step_complex(plan: Plan, cff, cst, x, status, norms, ws, stream=None):
    """md_newton_step_complex: one Newton step on complex data, x [2, L, n, D] in place."""
    L, n, D, m = plan.prec, plan.n, plan.D, plan.m
    rc = _lib.md_newton_step_complex(plan._h, _ptr(cff, (2, L, m), "cff"), _ptr(cst, (2, L, n, D), "cst"),
                                     _ptr(x, (2, L, n, D), "x"), _ptr(status, (1,), "status"),
                                     _ptr(norms, (2, D), "norms"), _ptr(ws, None, "ws"), ws.numel() * 8,
                                     _stream(stream))
    _check(rc, "md_newton_step_complex")


def stagger_next_order(d, D):
    """The order after d in the staggered schedule, d + 1 + d // 2, capped at D."""
    return int(_lib.md_stagger_next_order(int(d), int(D)))


def newton_staggered(plan: Plan, prec_solve, refactor_every_step, max_steps, tol, cff, cst, x, status, norms, ws,
                     stream=None):
    """md_newton_staggered; returns (StaggerReport, [(lo, hi) per step]); the
    report's `rel` attribute holds the last step's relative residuals [D]."""
    L, n, D, m = plan.prec, plan.n, plan.D, plan.m
    win = (ctypes.c_int32 * (2 * int(max_steps)))()
    rel = (ctypes.c_double * D)()
    rep = StaggerReport()
    rc = _lib.md_newton_staggered(plan._h, int(prec_solve), int(bool(refactor_every_step)), int(max_steps),
                                  float(tol), _ptr(cff, (L, m), "cff"), _ptr(cst, (L, n, D), "cst"),
                                  _ptr(x, (L, n, D), "x"), win, rel, ctypes.byref(rep),
                                  _ptr(status, (1,), "status"), _ptr(norms, (2, D), "norms"), _ptr(ws, None, "ws"),
                                  ws.numel() * 8, _stream(stream))
    _check(rc, "md_newton_staggered")
    rep.rel = np.array(rel[:])
    return rep, [(win[2 * q], win[2 * q + 1]) for q in range(rep.steps)]


def default_stagger_tol(prec, chain=1):
    """Residual tolerance of the staggered driver relative to the size of the
    cancelling terms of each equation: 2^8 units in the last place of the
    multiple double, times the length of the longest product chain (the
    largest monomial support), along which rounding errors add up."""
    return 2.0 ** (8 - 53 * int(prec)) * max(1, int(chain))


def arith(prec, op, a, b, c, stream=None):
    """Elementwise c = a op b on [L, count] md arrays; op "dot" writes sum_q a[q] b[q] to c [L, 1]."""
    L = int(prec)
    opc = OPS[op] if isinstance(op, str) else int(op)
    count = a.shape[1]
    shp = (L, count)
    rc = _lib.md_arith(L, opc, count, _ptr(a, shp, "a"), _ptr(b, shp if opc != 4 else None, "b"),
                       _ptr(c, (L, 1) if opc == 6 else shp, "c"), _stream(stream))
    _check(rc, "md_arith")


def adjoint_workspace_bytes(prec, n, d):
    v = ctypes.c_size_t()
    _check(_lib.md_adjoint_workspace_size(int(prec), int(n), int(d), ctypes.byref(v)), "md_adjoint_workspace_size")
    return int(v.value)


def adjoint_solve(prec, n, d, qr_, tau, A, g_lambda, ws, status, stream=None):
    """Solve T^T lambda = g in place (g_lambda [L, n, D])."""
    L, D = int(prec), int(d) + 1
    rc = _lib.md_adjoint_solve(L, int(n), int(d), _ptr(qr_, (L, n, n), "qr"), _ptr(tau, (L, n), "tau"),
                               _ptr(A, (L, n, n, D), "A"), _ptr(g_lambda, (L, n, D), "g_lambda"),
                               _ptr(ws, None, "ws"), ws.numel() * 8, _stream(stream), _ptr(status, (1,), "status"))
    _check(rc, "md_adjoint_solve")


def coef_grad(plan: Plan, x, lam, grad, ws, stream=None):
    L, n, D, m = plan.prec, plan.n, plan.D, plan.m
    rc = _lib.md_coef_grad(plan._h, _ptr(x, (L, n, D), "x"), _ptr(lam, (L, n, D), "lambda"),
                           _ptr(grad, (L, m), "grad"), _ptr(ws, None, "ws"), ws.numel() * 8, _stream(stream))
    _check(rc, "md_coef_grad")


def timing_enable(on=True):
    _check(_lib.md_timing_enable(1 if on else 0), "md_timing_enable")


def timing_read():
    """{class: (milliseconds, brackets)} accumulated since the last read."""
    k = len(TIMING_CLASSES)
    ms = (ctypes.c_double * k)()
    cnt = (ctypes.c_int64 * k)()
    _check(_lib.md_timing_read(ms, cnt), "md_timing_read")
    return {TIMING_CLASSES[c]: (float(ms[c]), int(cnt[c])) for c in range(k)}


def raw_call(name, *args):
    """Call an entry point with raw ctypes arguments (tests of the host-side checks)."""
    return getattr(_lib, name)(*args)


class Newton:
    """Convenience driver: device copies of a system and its workspace.

    Holds cff, cst and x on the device and runs md_newton_step in place."""

    def __init__(self, sys, cst, x0=None, device="cuda"):
        import torch

        self.sys = sys
        self.plan = Plan.from_system(sys)
        t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=device)
        self.cff = t(sys.cff)
        self.cst = t(cst)
        self.x = t(sys.start() if x0 is None else x0)
        self.ws = workspace(self.plan.workspace_bytes(), device)
        self.status = torch.zeros(1, dtype=torch.int32, device=device)
        self.norms = torch.zeros((2, sys.D), dtype=torch.float64, device=device)

    def step(self, stream=None, prec_solve=None):
        """One Newton step; prec_solve below the system's precision runs the
        mixed-precision step (md_newton_step_mixed)."""
        if prec_solve is None or prec_solve == self.plan.prec:
            newton_step(self.plan, self.cff, self.cst, self.x, self.status, self.norms, self.ws, stream)
        else:
            newton_step_mixed(self.plan, prec_solve, self.cff, self.cst, self.x, self.status, self.norms, self.ws,
                              stream)

    def steps(self, count, stream=None):
        """count plain steps (md_newton_steps): the same iterates as count calls
        of step(), with each factorization computed beside the previous step."""
        newton_steps(self.plan, count, self.cff, self.cst, self.x, self.status, self.norms, self.ws, stream)

    def step_window(self, lo, hi, keep_factorization=False, stream=None, prec_solve=None):
        """One step of the staggered method on the window lo..hi-1 (md_newton_step_window)."""
        ps = self.plan.prec if prec_solve is None else prec_solve
        newton_step_window(self.plan, ps, lo, hi, keep_factorization, self.cff, self.cst, self.x, self.status,
                           self.norms, self.ws, stream)

    def staggered(self, max_steps=40, tol=None, refactor_every_step=False, stream=None, prec_solve=None):
        """Newton's method with the staggered order schedule (md_newton_staggered);
        returns (StaggerReport, [(lo, hi) per step])."""
        ps = self.plan.prec if prec_solve is None else prec_solve
        chain = int(np.max(np.diff(self.sys.mon_ptr))) if self.sys.m > 0 else 1
        tol = default_stagger_tol(ps, chain) if tol is None else tol
        return newton_staggered(self.plan, ps, refactor_every_step, max_steps, tol, self.cff, self.cst, self.x,
                                self.status, self.norms, self.ws, stream)

    def residual(self, rows=None, prec=None, stream=None):
        """Residual b - T dx of the last step's linear system (md_step_arrays +
        md_linear_residual) on the listed rows (all when None), at precision
        prec (default: the plan's; a mixed step solved at fewer limbs).
        Returns (r [prec, nrows, D], norm1 [D])."""
        import torch

        L = self.plan.prec if prec is None else int(prec)
        n, D = self.plan.n, self.plan.D
        rws = None if rows is None else torch.as_tensor(np.asarray(rows, dtype=np.int32), device=self.x.device)
        nrows = n if rws is None else int(rws.numel())
        b, A, dx = step_arrays(self.plan, self.ws)
        r = torch.empty((L, nrows, D), dtype=torch.float64, device=self.x.device)
        norm1 = torch.empty(D, dtype=torch.float64, device=self.x.device)
        linear_residual(L, n, D - 1, A, b, dx, r, rows=rws, norm1=norm1, status=self.status, stream=stream)
        return r, norm1

    def status_code(self):
        return int(self.status.item())


class ComplexNewton:
    """Device copies of a system with complex data (cff [2, L, m], cst and x
    [2, L, n, D]) and its workspace; md_newton_step_complex in place."""

    def __init__(self, sys, cff, cst, x0, device="cuda"):
        import torch

        self.sys = sys
        self.plan = Plan.from_system(sys)
        t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=device)
        self.cff, self.cst, self.x = t(cff), t(cst), t(x0)
        self.ws = workspace(complex_workspace_bytes(self.plan), device)
        self.status = torch.zeros(1, dtype=torch.int32, device=device)
        self.norms = torch.zeros((2, sys.D), dtype=torch.float64, device=device)

    def step(self, stream=None):
        newton_step_complex(self.plan, self.cff, self.cst, self.x, self.status, self.norms, self.ws, stream)

    def eval_diff(self, x=None, stream=None):
        """(b, A) at x (default: the current iterate)."""
        import torch

        L, n, D = self.plan.prec, self.plan.n, self.plan.D
        b = torch.empty((2, L, n, D), dtype=torch.float64, device=self.x.device)
        A = torch.empty((2, L, n, n, D), dtype=torch.float64, device=self.x.device)
        eval_diff_complex(self.plan, self.cff, self.cst, self.x if x is None else x, b, A, self.ws, stream)
        return b, A

    def status_code(self):
        return int(self.status.item())


# ----------------------------------------------------------------- autograd
#
# Multiple-double tensors carry a leading limb axis; torch must never add or
# scale them itself.  The two Functions below are md-aware: their forward and
# backward run in the library, and the backward of a loss has to be seeded
# with the md number 1 ([1, 0, ..., 0]), see md_backward.


def _torch_fns():
    import torch

    class NewtonSolve(torch.autograd.Function):
        """x(cff): `steps` Newton steps from x0 on p(x; cff) = 0; the backward
        gives dL/dcff by the adjoint (md_adjoint_solve, md_coef_grad)."""

        @staticmethod
        def forward(ctx, cff, plan, cst, x0, steps):
            L, n, D = plan.prec, plan.n, plan.D
            ws = workspace(plan.workspace_bytes(), cff.device)
            status = torch.zeros(1, dtype=torch.int32, device=cff.device)
            norms = torch.zeros((2, D), dtype=torch.float64, device=cff.device)
            x = x0.clone().contiguous()
            newton_steps(plan, int(steps), cff.contiguous(), cst, x, status, norms, ws)
            ctx.plan = plan
            ctx.save_for_backward(cff, cst, x)
            return x

        @staticmethod
        def backward(ctx, gx):
            cff, cst, x = ctx.saved_tensors
            plan = ctx.plan
            L, n, d, D = plan.prec, plan.n, plan.d, plan.D
            dev = cff.device
            ws = workspace(plan.workspace_bytes(), dev)
            b = torch.empty((L, n, D), dtype=torch.float64, device=dev)
            A = torch.empty((L, n, n, D), dtype=torch.float64, device=dev)
            eval_diff(plan, cff.contiguous(), cst, x, b, A, ws)
            a0 = A[..., 0].contiguous()
            tau = torch.zeros((L, n), dtype=torch.float64, device=dev)
            status = torch.zeros(1, dtype=torch.int32, device=dev)
            qr(L, n, a0, tau, status)
            lam = gx.contiguous().clone()
            adjoint_solve(L, n, d, a0, tau, A, lam, workspace(adjoint_workspace_bytes(L, n, d), dev), status)
            grad = torch.empty_like(cff)
            coef_grad(plan, x, lam, grad, ws)
            return grad, None, None, None, None

    class TopCoefficientLoss(torch.autograd.Function):
        """L = sum_i sum_{k >= ktop} x_{i,k}^2 as a multiple double [L]."""

        @staticmethod
        def forward(ctx, x, ktop):
            L = x.shape[0]
            sel = x[:, :, ktop:].contiguous().reshape(L, -1)
            out = torch.empty((L, 1), dtype=torch.float64, device=x.device)
            arith(L, "dot", sel, sel, out)
            ctx.ktop = ktop
            ctx.save_for_backward(x)
            return out.reshape(L)

        @staticmethod
        def backward(ctx, gl):
            (x,) = ctx.saved_tensors
            L = x.shape[0]
            g = torch.zeros_like(x)
            g[:, :, ctx.ktop:] = 2.0 * x[:, :, ctx.ktop:]  # exact: every limb doubled
            flat = g.reshape(L, -1).contiguous()
            s = gl.reshape(L, 1).expand(L, flat.shape[1]).contiguous()
            out = torch.empty_like(flat)
            arith(L, "mul", flat, s, out)  # times the incoming multiple-double gradient
            return out.reshape(x.shape), None

    return NewtonSolve, TopCoefficientLoss


def newton_solve(cff, plan, cst, x0, steps):
    """Differentiable Newton solve (see NewtonSolve)."""
    return _torch_fns()[0].apply(cff, plan, cst, x0, steps)


def top_coefficient_loss(x, ktop):
    return _torch_fns()[1].apply(x, ktop)


def md_backward(loss):
    """loss.backward() seeded with the multiple double 1 = [1, 0, ..., 0]."""
    import torch

    seed = torch.zeros_like(loss)
    seed[0] = 1.0
    loss.backward(seed)
