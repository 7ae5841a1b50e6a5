"""Parity at the benchmark's full sizes (GPU), in the launch configuration
bench.py times: the medium quad-double system (n=64, d=63) against full oracle
steps, the large octo-double system (n=128, d=127) on sampled rows of the
evaluation and on the manufactured-solution property."""
from __future__ import annotations

import numpy as np
import pytest

import mdinputs
import oracle
from gpu_helpers import TOL, dev, host, matrix_series_err, scaled_err, series_err, step_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mdn():
    import paper_2301_12659_amd as mdn

    return mdn


@pytest.fixture(scope="module")
def medium():
    s = mdinputs.medium_qd()
    return s, oracle.manufacture(s)


def test_medium_qd_steps_vs_oracle(mdn, medium):
    """Steps 1, 2 and 6 from x*(0), each against the oracle step from the
    same input; after 6 steps x is the manufactured solution."""
    s, cst = medium
    drv = mdn.Newton(s, cst)
    x = s.start()
    for step in range(1, s.steps + 1):
        drv.step()
        got = host(drv.x)
        if step in (1, 2, s.steps):
            ref = oracle.newton_step(s, s.cff, cst, x)["x"]
            assert step_err(got, ref, x) <= TOL[4], (step, step_err(got, ref, x))
        x = got
    assert drv.status_code() == 0
    assert series_err(host(drv.x), s.xstar) <= TOL[4]
    drv.step()  # one more step: its update is at rounding level
    assert host(drv.norms)[1].max() < TOL[4]


def test_medium_qd_eval_sampled_rows(mdn, medium):
    import torch

    s, cst = medium
    x = mdinputs.random_point(s, 9, 0.5, 1.5)
    x = x * (0.25 ** np.arange(s.D))[None, None, :]
    plan = mdn.Plan.from_system(s)
    b = torch.empty((4, s.n, s.D), dtype=torch.float64, device="cuda")
    A = torch.empty((4, s.n, s.n, s.D), dtype=torch.float64, device="cuda")
    ws = mdn.workspace(plan.workspace_bytes())
    mdn.eval_diff(plan, dev(s.cff), dev(cst), dev(x), b, A, ws)
    torch.cuda.synchronize()
    gb, gA = host(b), host(A)
    for r in (0, 31, 63):
        ob, oA, sc = oracle.eval_diff(s, s.cff, cst, x, rows=(r, r + 1))
        assert scaled_err(gb[:, r:r + 1], ob, sc) <= TOL[4]
        assert matrix_series_err(gA[:, r:r + 1], oA) <= TOL[4]


@pytest.fixture(scope="module")
def large():
    return mdinputs.large_od()


def test_large_od_eval_sampled_rows(mdn, large):
    import torch

    s = large
    x = mdinputs.random_point(s, 3) * (0.25 ** np.arange(s.D))[None, None, :]
    cst = mdinputs.random_constant(s, 4)
    plan = mdn.Plan.from_system(s)
    b = torch.empty((8, s.n, s.D), dtype=torch.float64, device="cuda")
    A = torch.empty((8, s.n, s.n, s.D), dtype=torch.float64, device="cuda")
    ws = mdn.workspace(plan.workspace_bytes())
    mdn.eval_diff(plan, dev(s.cff), dev(cst), dev(x), b, A, ws)
    torch.cuda.synchronize()
    gb, gA = host(b), host(A)
    r = 77
    ob, oA, sc = oracle.eval_diff(s, s.cff, cst, x, rows=(r, r + 1))
    assert scaled_err(gb[:, r:r + 1], ob, sc) <= TOL[8]
    assert matrix_series_err(gA[:, r:r + 1], oA) <= TOL[8]


def test_large_od_converges_to_manufactured_solution(mdn, large):
    """8 steps from x*(0) with the right-hand side manufactured by the oracle
    reach x* (property of the method that holds at any size)."""
    s = large
    cst = oracle.manufacture(s)
    drv = mdn.Newton(s, cst)
    for _ in range(s.steps):
        drv.step()
    assert drv.status_code() == 0
    assert series_err(host(drv.x), s.xstar) <= TOL[8]
