"""The seeded workload generators (CPU only)."""
import numpy as np
import pytest

import mdinputs


def test_deterministic_per_seed():
    a, b = mdinputs.small_dd(), mdinputs.small_dd()
    for f in ("poly_ptr", "mon_ptr", "var", "exp", "cff", "xstar"):
        assert np.array_equal(getattr(a, f), getattr(b, f))
    c = mdinputs.small_dd(seed=99)
    assert not np.array_equal(a.cff, c.cff)


@pytest.mark.parametrize("L", [2, 4, 8])
def test_random_md_nonoverlapping_all_limbs(L):
    rng = np.random.default_rng(1)
    x = mdinputs.random_md(rng, L, (1000,), -1.0, 1.0)
    assert np.all(x != 0.0)
    for l in range(L - 1):
        assert np.all(np.abs(x[l + 1]) <= 0.5 * np.spacing(np.abs(x[l])))


def test_small_dd_shape_and_condition():
    s = mdinputs.small_dd()
    assert (s.L, s.n, s.d, s.D) == (2, 8, 15, 16)
    assert s.m == 64 and np.all(np.diff(s.mon_ptr) == 3) and np.all(s.exp == 1)
    J = mdinputs.jacobian0_estimate(s.poly_ptr, s.mon_ptr, s.var, s.exp, s.cff[0], s.xstar[0, :, 0])
    assert np.linalg.cond(J) <= 1e2
    # supports strictly increasing per monomial
    for j in range(s.m):
        v = s.var[s.mon_ptr[j]:s.mon_ptr[j + 1]]
        assert np.all(np.diff(v) > 0)


def test_medium_qd_matches_recipe():
    s = mdinputs.medium_qd()
    assert (s.L, s.n, s.D) == (4, 64, 64)
    per_row = np.diff(s.poly_ptr)
    assert np.all(per_row == 33)  # 32 monomials plus the diagonal boost
    k = np.diff(s.mon_ptr)
    boost = set(s.boost.tolist())
    ks = np.array([k[j] for j in range(s.m) if j not in boost])
    assert ks.min() >= 2 and ks.max() <= 6
    assert set(np.unique(s.exp).tolist()) <= {1, 2}
    x0 = s.xstar[0]
    assert x0.min() >= 0.5 * 0.25 ** (s.D - 1) * 0.99


def test_damping_scales_by_powers_of_two():
    s = mdinputs.make_system("t", 2, 4, 7, 2, 1, 2, (1,), 3, None, boost=False, damping=0.25)
    r = mdinputs.make_system("t", 2, 4, 7, 2, 1, 2, (1,), 3, None, boost=False, damping=1.0)
    for k in range(8):
        assert np.array_equal(s.xstar[:, :, k], r.xstar[:, :, k] * 0.25 ** k)


@pytest.mark.parametrize("L", [2, 4, 8])
def test_half_precision_start(L):
    """The staggered method's start: x*(0) with the trailing half of its limbs
    dropped, off by about half the working precision; zero above coefficient 0."""
    s = mdinputs.tiny(L, 5, 7, seed=3)
    x = s.half_precision_start()
    keep = (L + 1) // 2
    assert np.array_equal(x[:keep, :, 0], s.xstar[:keep, :, 0])
    assert not np.any(x[keep:]) and not np.any(x[:, :, 1:])
    rel = np.abs(s.xstar[keep, :, 0]) / np.abs(s.xstar[0, :, 0])
    assert np.all(rel < 2.0 ** (-53 * keep + 1))


def test_column_system_exponential_coefficients_match_table1():
    """x_j(t) = exp(alpha t): with alpha = 1 the coefficients are the printed
    1/k! of the paper's Table 1 (two significant digits)."""
    import os

    here = os.path.dirname(os.path.abspath(__file__))
    coefs = mdinputs._exp_coefficients(1, 128)
    with open(os.path.join(here, "golden", "table1_inverse_factorials.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, val = line.split()[:2]
            assert float(coefs[int(k)]) == pytest.approx(float(val), rel=0.051)


@pytest.mark.parametrize("L,cols", [(2, 1), (4, 2), (8, 1)])
def test_column_system_solution_is_a_root(L, cols):
    """The closed-form b(t) of the paper's column systems (Section 3) is
    p(x*) for the exponential x*: the oracle's residual at x* is only the
    rounding of c_{i,0} and x* to L limbs."""
    import oracle

    s = mdinputs.column_system(9, 7, L, cols, seed=2)
    assert s.m == cols * s.n and np.all(s.exp == 1)
    rows = [list(s.var[s.mon_ptr[j]:s.mon_ptr[j + 1]]) for j in range(s.m)]
    assert rows[0] == [0] and rows[cols * 8] == list(range(9))
    b, _, scale = oracle.eval_diff(s, s.cff, s.cst, s.xstar)
    assert np.max(np.abs(b[0]).max(axis=1) / scale) < 2.0 ** (-53 * L + 8)
    np.testing.assert_array_equal(s.start()[0, :, 0], np.ones(9))
