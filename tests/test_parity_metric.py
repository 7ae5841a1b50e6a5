"""The error measures of the GPU parity tests, checked on the CPU: on the
damped manufactured solutions of the full-size configurations a wrong low
limb in the last coefficient is invisible to the normwise error per series and
fails the per-coefficient error by many orders of magnitude."""
from __future__ import annotations

import numpy as np
import pytest

import mdinputs
from gpu_helpers import TOL, coef_err, coef_errs, step_err


@pytest.mark.parametrize("make", [mdinputs.small_dd, mdinputs.medium_qd, mdinputs.large_od])
def test_flipped_low_limb_of_the_last_coefficient(make):
    s = make()
    L, D = s.L, s.D
    ref = s.xstar.copy()
    x_in = s.start()
    bad = ref.copy()
    i = 5
    bad[L - 1, i, D - 1] = -bad[L - 1, i, D - 1]  # the last limb of coefficient d of one series
    assert bad[L - 1, i, D - 1] != 0.0
    assert coef_err(ref, ref, x_in) == 0.0
    assert step_err(bad, ref, x_in) <= TOL[L]            # normwise: passes
    assert coef_err(bad, ref, x_in) > 1e3 * TOL[L]       # per coefficient: fails
    assert np.argmax(coef_errs(bad, ref, x_in)) == D - 1


def test_zero_coefficients_must_match_exactly():
    s = mdinputs.small_dd()
    ref = np.zeros((2, 3, 4))
    got = ref.copy()
    got[1, 2, 3] = 1e-300
    e = coef_errs(got, ref)
    assert np.isinf(e[3]) and np.all(e[:3] == 0.0)
    del s
