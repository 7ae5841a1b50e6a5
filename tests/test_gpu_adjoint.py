"""The adjoint (transposed staged solve and coefficient gradients) against the
oracle and against octo-double finite differences (GPU)."""
from __future__ import annotations

from fractions import Fraction

import numpy as np
import pytest

import mdinputs
import oracle
from gpu_helpers import TOL, dev, host, series_err
from oracle_helpers import md_value

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mdn():
    import paper_2301_12659_amd as mdn

    return mdn


def _random_series_matrix(rng, L, n, D):
    A = mdinputs.random_md(rng, L, (n, n, D), -1.0, 1.0) * (0.25 ** np.arange(D))[None, None, None, :]
    A[0, :, :, 0] += np.diag(np.full(n, float(n)))
    return A


@pytest.mark.parametrize("L,n,d", [(2, 5, 0), (2, 6, 9), (4, 9, 17), (4, 16, 31), (8, 5, 12)])
def test_adjoint_solve_vs_oracle(mdn, L, n, d):
    import torch

    D = d + 1
    rng = np.random.default_rng(3 * n + d)
    A = _random_series_matrix(rng, L, n, D)
    g = mdinputs.random_md(rng, L, (n, D), -1.0, 1.0)
    tA = dev(A)
    a0 = tA[..., 0].contiguous()
    tau = torch.zeros((L, n), dtype=torch.float64, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    mdn.qr(L, n, a0, tau, status)
    lam = dev(g)
    mdn.adjoint_solve(L, n, d, a0, tau, tA, lam, mdn.workspace(mdn.adjoint_workspace_bytes(L, n, d)), status)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    ref = oracle.adjoint_solve(np.ascontiguousarray(np.moveaxis(A, -1, 1)), g)
    assert series_err(host(lam), ref) <= TOL[L]


def _grad_err(gpu, ref):
    diff = oracle.absdiff(gpu, ref)
    return float(diff.max() / np.abs(ref[0]).max())


@pytest.mark.parametrize("L", [2, 4, 8])
def test_coef_grad_vs_oracle(mdn, L):
    """Same converged point for both: the oracle's solution rounded to L limbs."""
    import torch

    sys = mdinputs.tiny(L, 6, 9, mons=3, kmin=1, kmax=3, exps=(1, 2, 3), seed=11)
    cst = oracle.manufacture(sys)
    x = oracle.round_md(oracle.converge(sys, sys.cff, cst, sys.start(), 6), L)
    ktop = 6
    g = oracle.loss_top_grad(x, ktop)
    out = oracle.newton_step(sys, sys.cff, cst, x, want_A=True)
    lam_o = oracle.adjoint_solve(out["A"], g)
    ref = oracle.coef_grad(sys, x, lam_o)
    # GPU: eval at x, QR, adjoint, gradient
    plan = mdn.Plan.from_system(sys)
    ws = mdn.workspace(plan.workspace_bytes())
    b = torch.empty((L, sys.n, sys.D), dtype=torch.float64, device="cuda")
    A = torch.empty((L, sys.n, sys.n, sys.D), dtype=torch.float64, device="cuda")
    tx = dev(x)
    mdn.eval_diff(plan, dev(sys.cff), dev(cst), tx, b, A, ws)
    a0 = A[..., 0].contiguous()
    tau = torch.zeros((L, sys.n), dtype=torch.float64, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    mdn.qr(L, sys.n, a0, tau, status)
    lam = dev(g)
    mdn.adjoint_solve(L, sys.n, sys.d, a0, tau, A, lam,
                      mdn.workspace(mdn.adjoint_workspace_bytes(L, sys.n, sys.d)), status)
    grad = torch.empty((L, sys.m), dtype=torch.float64, device="cuda")
    mdn.coef_grad(plan, tx, lam, grad, ws)
    torch.cuda.synchronize()
    assert _grad_err(host(grad), ref) <= TOL[L]


@pytest.fixture(scope="module")
def adjoint_config():
    s = mdinputs.adjoint_qd()
    cst = oracle.manufacture(s)
    return s, cst


def _autograd_gradient(mdn, s, cst, ktop, steps):
    import torch

    plan = mdn.Plan.from_system(s)
    cff = dev(s.cff).requires_grad_(True)
    x = mdn.newton_solve(cff, plan, dev(cst), dev(s.start()), steps)
    loss = mdn.top_coefficient_loss(x, ktop)
    mdn.md_backward(loss)
    torch.cuda.synchronize()
    return host(cff.grad), host(x), host(loss.detach())


def _tail_tol(x, ktop, L):
    """Tolerance for gradients of a loss on the coefficients k >= ktop.  x is
    known to about TOL relative to its largest coefficient, so the tail the
    loss sees (smaller by the damping) is known only to TOL * max|x| / max|tail|
    relative; two independently converged solutions differ by that much."""
    return TOL[L] * np.abs(x[0]).max() / np.abs(x[0, :, ktop:]).max()


def test_adjoint_config_gradient_at_common_point(mdn, adjoint_config):
    """n=32, d=31, qd, loss = sum of squares of the top 8 coefficients: the
    library's adjoint gradient and the oracle's at the same point (the
    oracle's converged solution rounded to quad double)."""
    import torch

    s, cst = adjoint_config
    ktop = 24
    x = oracle.round_md(oracle.converge(s, s.cff, cst, s.start(), s.steps + 1), 4)
    out = oracle.newton_step(s, s.cff, cst, x, want_A=True)
    g = oracle.loss_top_grad(x, ktop)
    ref = oracle.coef_grad(s, x, oracle.adjoint_solve(out["A"], g))
    plan = mdn.Plan.from_system(s)
    ws = mdn.workspace(plan.workspace_bytes())
    b = torch.empty((4, s.n, s.D), dtype=torch.float64, device="cuda")
    A = torch.empty((4, s.n, s.n, s.D), dtype=torch.float64, device="cuda")
    tx = dev(x)
    mdn.eval_diff(plan, dev(s.cff), dev(cst), tx, b, A, ws)
    a0 = A[..., 0].contiguous()
    tau = torch.zeros((4, s.n), dtype=torch.float64, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    mdn.qr(4, s.n, a0, tau, status)
    lam = dev(g)
    mdn.adjoint_solve(4, s.n, s.d, a0, tau, A, lam, mdn.workspace(mdn.adjoint_workspace_bytes(4, s.n, s.d)), status)
    grad = torch.empty((4, s.m), dtype=torch.float64, device="cuda")
    mdn.coef_grad(plan, tx, lam, grad, ws)
    torch.cuda.synchronize()
    assert _grad_err(host(grad), ref) <= TOL[4]


def test_adjoint_config_gradient_vs_oracle(mdn, adjoint_config):
    """The same loss through autograd (Newton solve, md loss, hand-written
    backward) against the oracle's gradient at its own converged solution."""
    s, cst = adjoint_config
    grad, x, _ = _autograd_gradient(mdn, s, cst, 24, s.steps + 1)
    xo = oracle.round_md(oracle.converge(s, s.cff, cst, s.start(), s.steps + 1), 4)
    assert series_err(x, xo) <= TOL[4]
    out = oracle.newton_step(s, s.cff, cst, xo, want_A=True)
    lam = oracle.adjoint_solve(out["A"], oracle.loss_top_grad(xo, 24))
    ref = oracle.coef_grad(s, xo, lam)
    assert _grad_err(grad, ref) <= _tail_tol(xo, 24, 4)


def test_adjoint_config_gradient_vs_octo_double_fd(mdn, adjoint_config):
    """Central differences in octo double (h = 1e-40) of the same loss on 64
    random coefficients, each from a full od Newton solve."""
    import torch

    s, cst = adjoint_config
    ktop, steps = 24, s.steps + 1
    grad, xg, _ = _autograd_gradient(mdn, s, cst, ktop, steps)
    tol = _tail_tol(xg, ktop, 4)
    pad = lambda a: np.concatenate([a, np.zeros((4,) + a.shape[1:])])
    sod = mdinputs.System("adjoint_od", 8, s.n, s.d, s.poly_ptr, s.mon_ptr, s.var, s.exp, pad(s.cff),
                          pad(s.xstar), s.seed)
    plan = mdn.Plan.from_system(sod)
    ws = mdn.workspace(plan.workspace_bytes())
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    norms = torch.zeros((2, s.D), dtype=torch.float64, device="cuda")
    tcst = dev(pad(cst))
    h = 1e-40
    rng = np.random.default_rng(55)
    idx = rng.choice(s.m, size=64, replace=False)
    scale = np.abs(grad[0]).max()
    for mj in idx:
        vals = []
        for sgn in (1.0, -1.0):
            cf = dev(pad(s.cff))
            hv = torch.zeros((8, 1), dtype=torch.float64, device="cuda")
            hv[0, 0] = sgn * h
            col = cf[:, mj:mj + 1].contiguous()
            out = torch.empty_like(col)
            mdn.arith(8, "add", col, hv, out)
            cf[:, mj] = out[:, 0]
            x = dev(sod.start())
            for _ in range(steps):
                mdn.newton_step(plan, cf, tcst, x, status, norms, ws)
            sel = x[:, :, ktop:].contiguous().reshape(8, -1)
            lv = torch.empty((8, 1), dtype=torch.float64, device="cuda")
            mdn.arith(8, "dot", sel, sel, lv)
            vals.append(md_value(host(lv)[:, 0]))
        fd = (vals[0] - vals[1]) / (2 * Fraction(h))
        ga = md_value(grad[:, mj])
        assert abs(float(fd - ga)) <= tol * scale, (mj, float(fd), float(ga))
