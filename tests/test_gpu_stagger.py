"""The staggered method on the GPU (Sections 4 and 5.3): steps on a window of
the series (order truncated at hi, stages below lo dropped), chord steps with
the factorization of A_0 kept from an earlier step, and the host-driven order
schedule, against the oracle's window step."""
from __future__ import annotations

import numpy as np
import pytest

import mdinputs
import oracle
from gpu_helpers import TOL, dev, host, series_err, step_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mdn():
    import paper_2301_12659_amd as mdn

    return mdn


def rough_point(s, seed, rel=1e-3):
    """x* with every coefficient off by about rel (a residual in every coefficient)."""
    rng = np.random.default_rng(seed)
    x = s.xstar.copy()
    x[0] *= 1.0 + rel * rng.uniform(-1.0, 1.0, x.shape[1:])
    return x


CASES = [  # (L, n, d, lo, hi, keep)
    (2, 6, 11, 0, 12, False), (2, 6, 11, 3, 9, True), (4, 8, 15, 0, 5, False), (4, 8, 15, 5, 16, False),
    (4, 8, 15, 2, 13, True), (4, 8, 15, 15, 16, True), (8, 5, 9, 1, 7, False), (8, 5, 9, 4, 10, True),
]


@pytest.mark.parametrize("L,n,d,lo,hi,keep", CASES)
def test_window_step_matches_oracle(mdn, L, n, d, lo, hi, keep):
    s = mdinputs.tiny(L, n, d, mons=3, kmin=1, kmax=3, exps=(1, 2), seed=20 + L + lo)
    cst = oracle.manufacture(s)
    x = rough_point(s, 1)
    kept = rough_point(s, 2, rel=1e-6) if keep else None
    drv = mdn.Newton(s, cst, kept if keep else x)
    if keep:
        drv.step_window(0, 1)  # factors A_0 at the kept point
        drv.x.copy_(dev(x))
    drv.step_window(lo, hi, keep_factorization=keep)
    assert drv.status_code() == 0
    ref = oracle.window_step(s, s.cff, cst, x, lo, hi, x_kept=kept)
    gx = host(drv.x)
    assert step_err(gx, ref["x"], x) <= TOL[L]
    assert np.array_equal(gx[:, :, hi:], x[:, :, hi:])  # coefficients from hi on are not touched
    nrm = host(drv.norms)
    assert not np.any(nrm[0, hi:]) and not np.any(nrm[1, :lo]) and not np.any(nrm[1, hi:])
    bmax = np.abs(ref["b"][0]).max(axis=0)
    np.testing.assert_allclose(nrm[0, :hi], bmax[:hi], rtol=1e-12, atol=1e-300)


def test_mixed_window_chord_step(mdn):
    """qd system, dd solve, kept factorization: within the dd bound of the
    oracle's exact window step."""
    s = mdinputs.tiny(4, 8, 15, mons=3, kmin=1, kmax=3, exps=(1, 2), seed=31)
    cst = oracle.manufacture(s)
    x, kept = rough_point(s, 3), rough_point(s, 4, rel=1e-6)
    drv = mdn.Newton(s, cst, kept)
    drv.step_window(0, 1, prec_solve=2)
    drv.x.copy_(dev(x))
    drv.step_window(3, 12, keep_factorization=True, prec_solve=2)
    assert drv.status_code() == 0
    ref = oracle.window_step(s, s.cff, cst, x, 3, 12, x_kept=kept)
    assert step_err(host(drv.x), ref["x"], x) <= TOL[2]


def test_window_rejects_bad_windows(mdn):
    s = mdinputs.tiny(2, 4, 7, seed=1)
    drv = mdn.Newton(s, oracle.manufacture(s))
    for lo, hi in [(0, 0), (3, 3), (-1, 4), (2, 9), (5, 4)]:
        with pytest.raises(mdn.MdError):
            drv.step_window(lo, hi)


def _replay(s, cst, x0, windows, kept):
    x = x0
    for lo, hi in windows:
        x = oracle.round_md(oracle.window_step(s, s.cff, cst, x, lo, hi, x_kept=kept)["x"], s.L)
    return x


@pytest.mark.parametrize("L", [2, 4])
def test_driver_replayed_by_the_oracle(mdn, L):
    """The driver's own sequence of windows, replayed by the oracle (each step
    rounded to the working precision, A_0 kept from the start), ends where
    the GPU ended; both are at the manufactured solution."""
    s = mdinputs.tiny(L, 8, 23, mons=3, kmin=1, kmax=3, exps=(1, 2), seed=40 + L)
    cst = oracle.manufacture(s)
    x0 = s.half_precision_start()
    drv = mdn.Newton(s, cst, x0)
    rep, windows = drv.staggered(max_steps=30)
    assert rep.converged == 1 and rep.factorizations == 1, (rep.steps, windows)
    his = [hi for _, hi in windows]
    sched = [1]
    while len(sched) < len(his):
        sched.append(mdn.stagger_next_order(sched[-1], s.D))
    assert his == sched
    los = [lo for lo, _ in windows]
    assert los == sorted(los) and all(lo < hi for lo, hi in windows)
    gx = host(drv.x)
    assert series_err(gx, s.xstar) <= TOL[L]
    ora = _replay(s, cst, x0, windows, x0)
    assert series_err(gx, ora) <= TOL[L]


def test_driver_medium_qd(mdn):
    """n=64, d=63, quad double from a half-precision x_0: one factorization,
    the order schedule 1, 2, 4, ..., 61, 64, convergence to the manufactured
    solution; refactoring at every step converges as well."""
    s = mdinputs.medium_qd()
    cst = oracle.manufacture(s)
    x0 = s.half_precision_start()
    drv = mdn.Newton(s, cst, x0)
    rep, windows = drv.staggered(max_steps=40)
    assert rep.converged == 1 and rep.factorizations == 1, (rep.steps, windows)
    assert [hi for _, hi in windows][:10] == [1, 2, 4, 7, 11, 17, 26, 40, 61, 64]
    assert series_err(host(drv.x), s.xstar) <= TOL[4]
    drv2 = mdn.Newton(s, cst, x0)
    rep2, _ = drv2.staggered(max_steps=40, refactor_every_step=True)
    assert rep2.converged == 1 and rep2.factorizations == rep2.steps
    assert series_err(host(drv2.x), s.xstar) <= TOL[4]


def test_driver_slow_chord_contraction_does_not_freeze(mdn):
    """A start a quarter off in every coefficient of x_0: the chord steps with
    the factorization of that start contract slowly, and a residual that does
    not halve from one step to the next is then far above the rounding level.
    The driver must not take such a coefficient as done: it either reaches
    the manufactured solution or reports no convergence (or a failed step)."""
    s = mdinputs.tiny(4, 8, 15, mons=3, kmin=1, kmax=3, exps=(1, 2), seed=77)
    cst = oracle.manufacture(s)
    x0 = s.start()
    x0[:, :, 0] *= 1.25
    drv = mdn.Newton(s, cst, x0)
    try:
        rep, windows = drv.staggered(max_steps=40)
    except mdn.MdError:
        return  # a failed step (the chord iteration diverged) is reported, not a false convergence
    if rep.converged:
        assert series_err(host(drv.x), s.xstar) <= TOL[4], windows
    else:
        assert rep.steps == 40
