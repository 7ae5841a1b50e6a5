"""Helpers for the GPU parity tests: device transfers and error metrics."""
from __future__ import annotations

import numpy as np

import oracle

# Relative tolerances on well-conditioned inputs: double double, quad double,
# octo double; plain double (one limb) takes about as many units of its last
# place as the double-double tolerance does of its own (1e-28 is about 8 000
# units of 2^-106, 1e-12 about 9 000 units of 2^-53).
TOL = {1: 1e-12, 2: 1e-28, 4: 1e-60, 8: 1e-120}


def dev(a):
    import torch

    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def series_err(gpu, ora):
    """Max over series of max_k |gpu - ora| / max_k |ora| (last axis = coefficients)."""
    return float(np.max(oracle.rel_err_series(gpu, ora)))


def scaled_err(gpu, ora, scale):
    """Max over rows of max_k |gpu - ora| / scale[row]  (gpu, ora: [L|K, rows, D])."""
    d = oracle.absdiff(gpu, ora).max(axis=-1)
    return float(np.max(d / scale))


def matrix_series_err(gpu_A, ora_A):
    """Jacobian series: per entry (i, j), max_k |diff| / max_k |ora|; structural
    zeros must be exact zeros.  gpu_A [L, n, n, D], ora_A [K, D, n, n] (oracle
    layout) -> compare in the GPU layout."""
    ora = np.moveaxis(ora_A, 1, -1)  # [K, n, n, D]
    diff = oracle.absdiff(gpu_A, ora)
    mag = np.abs(ora[0]).max(axis=-1)
    num = diff.max(axis=-1)
    zero = mag == 0
    assert np.all(num[zero] == 0.0), "nonzero where the Jacobian is structurally zero"
    return float(np.max(np.where(zero, 0.0, num / np.where(zero, 1.0, mag))))


def step_err(gpu_out, ora_out, x_in):
    """Error of one Newton step, per series normwise relative to the data the
    step works with: max_k |gpu - ora| / max_k max(|x_in|, |x_out|)."""
    diff = oracle.absdiff(gpu_out, ora_out).max(axis=-1)
    scale = np.maximum(np.abs(x_in[0]).max(axis=-1), np.abs(ora_out[0]).max(axis=-1))
    return float(np.max(diff / scale))


def coef_errs(gpu_out, ora_out, x_in=None):
    """Error of every coefficient k separately: max_i |gpu - ora|_{i,k} divided
    by max_i max(|x_in_{i,k}|, |ora_{i,k}|) (leading limbs), for series
    gpu[L, n, D] and ora[K, n, D].  Damped series have coefficients of very
    different sizes, so a normwise error says little about the late ones; this
    one sees a wrong low limb of any coefficient.  Coefficients that are zero
    on both sides must match exactly (their error is 0 or inf)."""
    diff = oracle.absdiff(gpu_out, ora_out).max(axis=-2)  # [D]
    mag = np.abs(ora_out[0]).max(axis=-2)
    if x_in is not None:
        mag = np.maximum(mag, np.abs(x_in[0]).max(axis=-2))
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(mag > 0, diff / np.where(mag > 0, mag, 1.0), np.where(diff > 0, np.inf, 0.0))


def coef_err(gpu_out, ora_out, x_in=None):
    """Largest per-coefficient error (see coef_errs)."""
    return float(np.max(coef_errs(gpu_out, ora_out, x_in)))


# The per-coefficient bound of a step where rounding errors are amplified by
# the problem itself (late coefficients of an unconverged iterate, or a
# near-singular series problem): the error of the same step computed by the
# oracle at the working precision (53 L bits, every operation correctly
# rounded, LU instead of QR) against the oracle at 4 x 53 L bits, times
# WORKING_FACTOR.  The forward substitution of the block Toeplitz system
# carries the error of every coefficient into the later ones, so the error
# of coefficient k is bounded by the errors of coefficients 0..k, and the
# bound takes the largest working-precision error among them (one sample of
# the oracle's error at a single coefficient can be far below its
# neighbours').  The library's multiple-double operations end a few units
# of the last limb away from the correctly rounded result; measured ratios
# of the two errors are at most 17 on the configurations of the tests.
WORKING_FACTOR = 32.0


def assert_step_per_coefficient(sys, cst, x_in, got, ref, tol):
    """Every coefficient k of a step's output within max(tol, WORKING_FACTOR
    e_k) relative to its size (coef_errs), e_k the largest per-coefficient
    error of the oracle's step at the working precision over coefficients
    0..k."""
    ce = coef_errs(got, ref, x_in)
    if np.max(ce) <= tol:
        return ce
    low = oracle.newton_step(sys, sys.cff, cst, x_in, prec=53 * sys.L)["x"]
    cl = np.maximum.accumulate(coef_errs(low, ref, x_in))
    bound = np.maximum(tol, WORKING_FACTOR * cl)
    bad = np.nonzero(ce > bound)[0]
    assert bad.size == 0, ("coefficients beyond the working-precision bound", bad.tolist(),
                           ce[bad].tolist(), bound[bad].tolist())
    return ce
