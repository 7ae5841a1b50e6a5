"""md_newton_steps (GPU): several plain steps with the factorization of each
step computed beside the previous one give the iterates of as many calls of
md_newton_step, bit for bit, and the oracle's steps."""
from __future__ import annotations

import numpy as np
import pytest

import mdinputs
import oracle
from gpu_helpers import TOL, assert_step_per_coefficient, host, series_err, step_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mdn():
    import paper_2301_12659_amd as mdn

    return mdn


def _compare(mdn, s, cst, counts):
    import torch

    for count in counts:
        print(f"md_newton_steps {s.name} count={count}", flush=True)
        one = mdn.Newton(s, cst)
        for _ in range(count):
            one.step()
        many = mdn.Newton(s, cst)
        many.steps(count)
        torch.cuda.synchronize()
        assert many.status_code() == 0 and one.status_code() == 0
        assert np.array_equal(host(many.x), host(one.x)), (s.name, count)
        assert np.array_equal(host(many.norms), host(one.norms)), (s.name, count)
        # the kept factorization is the last step's: a chord step after both
        one.step_window(0, s.D, keep_factorization=True)
        many.step_window(0, s.D, keep_factorization=True)
        torch.cuda.synchronize()
        assert np.array_equal(host(many.x), host(one.x)), (s.name, count, "chord step after")


def test_steps_medium_qd_bit_identical(mdn):
    s = mdinputs.medium_qd()
    _compare(mdn, s, oracle.manufacture(s), (1, 2, 3, 6))


@pytest.mark.parametrize("L,n,d", [(2, 9, 20), (4, 37, 30), (2, 64, 63)])
def test_steps_small_systems_bit_identical(mdn, L, n, d):
    s = mdinputs.tiny(L, n, d, mons=4, kmin=1, kmax=4, exps=(1, 2), seed=n + d)
    _compare(mdn, s, oracle.manufacture(s), (2, 5))


def test_steps_fallback_plans(mdn):
    """Plans outside the overlapped form (octo doubles; exponent 3, whose A_0
    does not come from the coefficient-0 pre-pass) take ordinary steps."""
    for s in (mdinputs.tiny(8, 7, 9, seed=3), mdinputs.tiny(4, 8, 7, mons=3, kmin=2, kmax=3, exps=(3,), seed=4)):
        _compare(mdn, s, oracle.manufacture(s), (2,))


def test_steps_medium_qd_against_oracle(mdn):
    """Six overlapped steps from x*(0): step 6 against the oracle step from
    the fifth iterate, and the manufactured solution."""
    import torch

    s = mdinputs.medium_qd()
    cst = oracle.manufacture(s)
    drv = mdn.Newton(s, cst)
    drv.steps(5)
    torch.cuda.synchronize()
    x5 = host(drv.x)
    drv.steps(1)
    torch.cuda.synchronize()
    got = host(drv.x)
    ref = oracle.newton_step(s, s.cff, cst, x5)["x"]
    assert step_err(got, ref, x5) <= TOL[4]
    assert_step_per_coefficient(s, cst, x5, got, ref, TOL[4])
    assert series_err(got, s.xstar) <= TOL[4]
