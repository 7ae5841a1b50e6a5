"""Helpers for the GPU parity tests: device transfers and error metrics."""
from __future__ import annotations

import numpy as np

import oracle

# Relative tolerances on well-conditioned inputs: double double, quad double,
# octo double.
TOL = {2: 1e-28, 4: 1e-60, 8: 1e-120}


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
