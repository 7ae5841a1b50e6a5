"""The linear residual b - T dx of the block Toeplitz system (GPU), in
multiple-double precision on all or sampled equations (Section 5.4, Table 4),
against the oracle's residual."""
from __future__ import annotations

import numpy as np
import pytest

import mdinputs
import oracle
from gpu_helpers import TOL, dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mdn():
    import paper_2301_12659_amd as mdn

    return mdn


def _gpu_residual(mdn, L, n, d, A, b, dx, rows):
    import torch

    D = d + 1
    rws = None if rows is None else torch.as_tensor(np.asarray(rows, dtype=np.int32), device="cuda")
    nrows = n if rows is None else len(rows)
    r = torch.empty((L, nrows, D), dtype=torch.float64, device="cuda")
    norm1 = torch.empty(D, dtype=torch.float64, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    mdn.linear_residual(L, n, d, dev(A), dev(b), dev(dx), r, rows=rws, norm1=norm1, status=status)
    return host(r), host(norm1), int(status.item())


@pytest.mark.parametrize("L,n,d", [(2, 9, 12), (4, 9, 12), (8, 5, 6), (4, 70, 20), (2, 1, 0)])
def test_residual_matches_oracle(mdn, L, n, d):
    rng = np.random.default_rng(10 * L + n)
    D = d + 1
    A = mdinputs.random_md(rng, L, (n, n, D), -1.0, 1.0)
    b = mdinputs.random_md(rng, L, (n, D), -1.0, 1.0)
    dx = mdinputs.random_md(rng, L, (n, D), -1.0, 1.0)
    for rows in (None, [n - 1, 0, min(3, n - 1), min(3, n - 1)]):
        r, norm1, status = _gpu_residual(mdn, L, n, d, A, b, dx, rows)
        assert status == 0
        ref, scale = oracle.linear_residual(np.moveaxis(A, 3, 1), b, dx, rows=rows)
        assert np.max(oracle.absdiff(r, ref) / scale) <= TOL[L]
        np.testing.assert_allclose(norm1, np.abs(ref[0]).sum(axis=0), rtol=1e-13)


def test_residual_bad_row_sets_status(mdn):
    rng = np.random.default_rng(1)
    L, n, d = 2, 6, 4
    A = mdinputs.random_md(rng, L, (n, n, d + 1), -1.0, 1.0)
    b = mdinputs.random_md(rng, L, (n, d + 1), -1.0, 1.0)
    dx = mdinputs.random_md(rng, L, (n, d + 1), -1.0, 1.0)
    r, _, status = _gpu_residual(mdn, L, n, d, A, b, dx, [2, n])
    assert status == mdn.MD_EINVAL
    ref, scale = oracle.linear_residual(np.moveaxis(A, 3, 1), b, dx, rows=[2])
    assert np.max(oracle.absdiff(r[:, :1], ref) / scale) <= TOL[L]


def _step_arrays(mdn, drv):
    """b, A, dx of the last step, as host arrays (views into the workspace)."""
    L, n, D = drv.plan.prec, drv.plan.n, drv.plan.D
    base = drv.ws.data_ptr()
    bp, Ap, dxp = mdn.step_arrays(drv.plan, drv.ws)
    view = lambda p, cnt, shape: host(drv.ws[(p - base) // 8:(p - base) // 8 + cnt].reshape(shape))
    return (view(bp, L * n * D, (L, n, D)), view(Ap, L * n * n * D, (L, n, n, D)),
            view(dxp, L * n * D, (L, n, D)))


@pytest.mark.parametrize("L", [2, 4, 8])
def test_residual_of_a_newton_step(mdn, L):
    """The residual of a step's own linear system: the kernel against the
    oracle on the step's b, A and dx, and small (the solve's accuracy)."""
    s = mdinputs.tiny(L, 7, 10, mons=3, kmin=1, kmax=3, exps=(1, 2), seed=50 + L)
    cst = oracle.manufacture(s)
    drv = mdn.Newton(s, cst)
    drv.step()
    assert drv.status_code() == 0
    r, norm1 = drv.residual()
    b, A, dx = _step_arrays(mdn, drv)
    ref, scale = oracle.linear_residual(np.moveaxis(A, 3, 1), b, dx)
    assert np.max(oracle.absdiff(host(r), ref) / scale) <= TOL[L]
    assert np.max(np.abs(ref[0]) / scale) < 1e4 * TOL[L]
    rs, _ = drv.residual(rows=[6, 2])
    assert np.array_equal(host(rs), host(r)[:, [6, 2]])


def test_residual_medium_qd_sampled_rows(mdn):
    """Full size (n=64, d=63, qd), three sampled equations after the first
    step, against the oracle on those rows."""
    s = mdinputs.medium_qd()
    cst = oracle.manufacture(s)
    drv = mdn.Newton(s, cst)
    drv.step()
    rows = [5, 17, 63]
    r, norm1 = drv.residual(rows=rows)
    b, A, dx = _step_arrays(mdn, drv)
    ref, scale = oracle.linear_residual(np.moveaxis(A, 3, 1), b, dx, rows=rows)
    assert np.max(oracle.absdiff(host(r), ref) / scale) <= TOL[4]
    # the residual is at rounding level here: the 1-norm is the GPU residual's
    # own, within the residual's tolerance of the exact one
    np.testing.assert_allclose(host(norm1), np.abs(host(r)[0]).sum(axis=0), rtol=1e-14, atol=0)
    assert np.all(np.abs(host(norm1) - np.abs(ref[0]).sum(axis=0)) <= TOL[4] * scale.sum(axis=0))
