"""Seeded synthetic workloads for the power-series Newton step.

This module only draws random numbers and builds index tables. It holds none
of the method's arithmetic (no series products, no Newton step, no linear
algebra of the method); both the oracle and the GPU path take their inputs
from here.

Workload families (the paper's own systems are synthetic monomial systems with
exponential-series solutions, Section 3; the sizes below replace them):

* ``small_dd``   n=8,   degree 15,  double-double, 8 monomials of 3 variables
                 with exponent 1 per polynomial, plus a constant series.
* ``medium_qd``  n=64,  degree 63,  quad-double, 32 monomials of 2..6
                 variables with exponents in {1,2}, plus a diagonal boost.
* ``large_od``   n=128, degree 127, octo-double, 64 monomials of 4..8
                 variables with exponents in {1,2,3}, plus a diagonal boost.
* ``adjoint_qd`` n=32,  degree 31,  quad-double, 32 monomials of 3..5
                 variables with exponents in {1,2}, plus a diagonal boost.
* ``batched``    many independent paths of uneven size (see ``batched_paths``).
* ``column_system``  the paper's own one- and two-column triangular systems
                 with exponential solutions, in closed form (Section 3);
                 ``complex_column_system`` the same with complex data.

Multiple-double numbers are stored limb-major (structure of arrays by limb),
shape ``[L, ...]``, as the paper does to keep memory accesses coalesced
(Section 1.2 and Section 6).  A random multiple double has every limb drawn:
limb ``l+1`` is uniform in ``(-ulp(limb_l)/2, ulp(limb_l)/2)``, so the limbs
never overlap and lower-limb mistakes cannot hide behind zeros.
"""
from __future__ import annotations

import dataclasses
import numpy as np

PRECISIONS = {"dd": 2, "qd": 4, "od": 8}


@dataclasses.dataclass
class System:
    """A polynomial system p_i(x) = c_{i,0}(t) + sum_m c_{i,m} x^{a_{i,m}}.

    Index tables (CSR):
      poly_ptr[n+1]  monomials of polynomial i are mon_ptr range poly_ptr[i]..poly_ptr[i+1]
      mon_ptr[m+1]   support entries of monomial j are mon_ptr[j]..mon_ptr[j+1]
      var[nnz]       variable index of each support entry, strictly increasing per monomial
      exp[nnz]       exponent (>= 1) of each support entry
    Values (limb-major multiple doubles):
      cff[L, m]      scalar coefficient of each monomial
      xstar[L, n, D] the manufactured solution series (D = d + 1 coefficients)
    """

    name: str
    L: int
    n: int
    d: int
    poly_ptr: np.ndarray
    mon_ptr: np.ndarray
    var: np.ndarray
    exp: np.ndarray
    cff: np.ndarray
    xstar: np.ndarray
    seed: int
    steps: int = 1
    boost: np.ndarray | None = None  # index of the boost monomial of each row, or None
    cst: np.ndarray | None = None  # c_{i,0}(t) [L, n, D] when known in closed form, else None

    @property
    def D(self) -> int:
        return self.d + 1

    @property
    def m(self) -> int:
        return int(self.mon_ptr.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.var.shape[0])

    @property
    def is_complex(self) -> bool:
        """Complex data: cff [2, L, m], xstar and cst [2, L, n, D] (real plane, imaginary plane)."""
        return self.xstar.ndim == 4

    def start(self) -> np.ndarray:
        """x*(0) as a series: coefficient 0 of x*, all higher coefficients zero."""
        x = np.zeros_like(self.xstar)
        x[..., 0] = self.xstar[..., 0]
        return x

    def half_precision_start(self) -> np.ndarray:
        """x*(0) with the trailing half of its limbs dropped (the leading
        ceil(L/2) limbs kept: about half the working precision correct, the
        start the staggered method assumes), higher coefficients zero."""
        x = self.start()
        x[(self.L + 1) // 2:, :, 0] = 0.0
        return x


def random_md(rng: np.random.Generator, L: int, shape, lo: float, hi: float) -> np.ndarray:
    """Random multiple doubles with every limb populated, limb-major [L, *shape].

    The leading limb is uniform in [lo, hi]; each lower limb is uniform in
    (-ulp/2, ulp/2) of the limb above, so the expansion is nonoverlapping.
    """
    shape = tuple(np.atleast_1d(shape)) if not isinstance(shape, tuple) else shape
    out = np.zeros((L,) + shape, dtype=np.float64)
    out[0] = rng.uniform(lo, hi, size=shape)
    for l in range(1, L):
        half_ulp = 0.5 * np.spacing(np.abs(out[l - 1]))
        out[l] = rng.uniform(-1.0, 1.0, size=shape) * half_ulp
    return out


def random_series(rng, L, n, D, lo=0.5, hi=1.5, damping: float = 1.0) -> np.ndarray:
    """Random series x[L, n, D] with coefficients uniform in [lo, hi].

    ``damping`` < 1 draws coefficient k in damping^k * [lo, hi] (the paper's
    delta-damping of t, end of Section 3).
    """
    x = random_md(rng, L, (n, D), lo, hi)
    if damping != 1.0:
        scale = damping ** np.arange(D, dtype=np.float64)
        # scale every limb by a power of two close to damping^k keeps limbs exact
        p2 = np.exp2(np.round(np.log2(scale)))
        x = x * p2[None, None, :]
    return x


def _supports(rng, n, n_mon_per_poly, kmin, kmax, exps):
    poly_ptr = [0]
    mon_ptr = [0]
    var, ex = [], []
    for i in range(n):
        nm = n_mon_per_poly(i)
        for _ in range(nm):
            k = int(rng.integers(kmin, kmax + 1))
            k = min(k, n)
            vs = np.sort(rng.choice(n, size=k, replace=False))
            es = rng.choice(np.asarray(exps), size=k)
            var.extend(int(v) for v in vs)
            ex.extend(int(e) for e in es)
            mon_ptr.append(len(var))
        poly_ptr.append(len(mon_ptr) - 1)
    return (np.asarray(poly_ptr, np.int32), np.asarray(mon_ptr, np.int32),
            np.asarray(var, np.int32), np.asarray(ex, np.int32))


def _supports_vectorized(rng, n, mons, kmin, kmax, exps):
    """As _supports with a fixed number of monomials per polynomial, drawn
    with array operations (another random stream; used for large batches)."""
    m = n * mons
    k = np.minimum(rng.integers(kmin, kmax + 1, size=m), n)
    keys = rng.random((m, n))
    pick = np.argsort(keys, axis=1)[:, :kmax]
    es_all = rng.choice(np.asarray(exps), size=(m, kmax))
    mask = np.arange(kmax)[None, :] < k[:, None]
    picked = np.where(mask, pick, n)  # n sorts after every variable
    order = np.argsort(picked, axis=1)
    vs = np.take_along_axis(picked, order, axis=1)
    es = np.take_along_axis(es_all, order, axis=1)
    var = vs[vs < n].astype(np.int32)
    ex = es[vs < n].astype(np.int32)
    mon_ptr = np.concatenate([[0], np.cumsum(k)]).astype(np.int32)
    poly_ptr = (np.arange(n + 1) * mons).astype(np.int32)
    return poly_ptr, mon_ptr, var, ex


def _jacobian0_vectorized(poly_ptr, mon_ptr, var, exp, cff_hi, x0_hi) -> np.ndarray:
    """jacobian0_estimate with array operations, for points without zero
    entries: d/dx_a of c prod x_b^e_b is e_a c prod x_b^e_b / x_a."""
    n = len(poly_ptr) - 1
    m = len(mon_ptr) - 1
    mono = np.repeat(np.arange(m), np.diff(mon_ptr))
    row = np.repeat(np.arange(n), np.diff(poly_ptr))[mono]
    xe = x0_hi[var] ** exp
    logp = np.zeros(m)
    np.add.at(logp, mono, np.log(xe))
    val = cff_hi[mono] * np.exp(logp[mono]) * exp / x0_hi[var]
    J = np.zeros((n, n))
    np.add.at(J, (row, var), val)
    return J


def jacobian0_estimate(poly_ptr, mon_ptr, var, exp, cff_hi, x0_hi) -> np.ndarray:
    """Float64 estimate of the Jacobian at the point x0 (leading limbs only).

    Used only to choose the diagonal boost and to check the condition number
    of a generated system; it is not part of any computed result.
    """
    n = len(poly_ptr) - 1
    J = np.zeros((n, n))
    for i in range(n):
        for mj in range(poly_ptr[i], poly_ptr[i + 1]):
            vs = var[mon_ptr[mj]:mon_ptr[mj + 1]]
            es = exp[mon_ptr[mj]:mon_ptr[mj + 1]]
            for a in range(len(vs)):
                g = cff_hi[mj] * es[a] * x0_hi[vs[a]] ** (es[a] - 1)
                for b in range(len(vs)):
                    if b != a:
                        g *= x0_hi[vs[b]] ** es[b]
                J[i, vs[a]] += g
    return J


def _append_boost(poly_ptr, mon_ptr, var, exp, cff, L, s):
    """Append one linear monomial s_i * x_i at the end of every polynomial."""
    n = len(poly_ptr) - 1
    new_pp, new_mp, new_var, new_exp, new_cff = [0], [0], [], [], []
    boost_idx = np.zeros(n, np.int32)
    for i in range(n):
        for mj in range(poly_ptr[i], poly_ptr[i + 1]):
            new_var.extend(var[mon_ptr[mj]:mon_ptr[mj + 1]].tolist())
            new_exp.extend(exp[mon_ptr[mj]:mon_ptr[mj + 1]].tolist())
            new_mp.append(len(new_var))
            new_cff.append(cff[:, mj])
        new_var.append(i)
        new_exp.append(1)
        new_mp.append(len(new_var))
        c = np.zeros(L)
        c[0] = s[i]
        new_cff.append(c)
        boost_idx[i] = len(new_mp) - 2
        new_pp.append(len(new_mp) - 1)
    return (np.asarray(new_pp, np.int32), np.asarray(new_mp, np.int32),
            np.asarray(new_var, np.int32), np.asarray(new_exp, np.int32),
            np.stack(new_cff, axis=1), boost_idx)


def make_system(name: str, L: int, n: int, d: int, mons_per_poly, kmin: int, kmax: int,
                exps, seed: int, cond_max: float | None, boost: bool, steps: int = 1,
                damping: float = 1.0, max_tries: int = 64, boost_gamma: float = 0.125,
                vectorized: bool = False, cond_min: float | None = None) -> System:
    """Draw a system and its manufactured solution.

    Without ``boost`` the system is redrawn (from a derived seed) until the
    float64 estimate of cond_2(J(x*(0))) is at most ``cond_max``.  With
    ``boost`` one linear monomial s_i x_i is appended to every polynomial;
    s_i starts at 1/8 of the row's absolute sum of the estimated Jacobian and
    is doubled until the condition bound holds.  With ``cond_min`` the boost
    grows by factors of 2^(1/4) instead, s_i = gamma * rowsum_i, and a draw is
    kept only if the first boost that meets ``cond_max`` leaves
    cond_2(J) >= cond_min: a system near the condition bound.
    """
    D = d + 1
    for attempt in range(max_tries):
        rng = np.random.default_rng([seed, attempt])
        if callable(mons_per_poly):
            per = mons_per_poly
        else:
            per = (lambda i, _c=int(mons_per_poly): _c)
        if vectorized:
            pp, mp, var, ex = _supports_vectorized(rng, n, int(mons_per_poly), kmin, kmax, exps)
        else:
            pp, mp, var, ex = _supports(rng, n, lambda i: per(i) if not callable(mons_per_poly) else int(mons_per_poly(rng)), kmin, kmax, exps)
        m = len(mp) - 1
        cff = random_md(rng, L, (m,), -1.0, 1.0)
        xstar = random_series(rng, L, n, D, 0.5, 1.5, damping)
        J = (_jacobian0_vectorized if vectorized else jacobian0_estimate)(pp, mp, var, ex, cff[0], xstar[0, :, 0])
        bidx = None
        if boost:
            rowsum = np.abs(J).sum(axis=1) + 1.0
            gamma = boost_gamma
            sign = np.where(np.diag(J) < 0, -1.0, 1.0)
            for _ in range(40 if cond_min is None else 200):
                if cond_min is None:
                    s = np.exp2(np.ceil(np.log2(gamma * rowsum))) * sign
                else:
                    s = gamma * rowsum * sign
                Jb = J + np.diag(s)
                if cond_max is None or np.linalg.cond(Jb) <= cond_max:
                    break
                gamma *= 2.0 if cond_min is None else 2.0 ** 0.25
            pp, mp, var, ex, cff, bidx = _append_boost(pp, mp, var, ex, cff, L, s)
            J = Jb
        c2 = np.linalg.cond(J)
        if (cond_max is None or c2 <= cond_max) and (cond_min is None or c2 >= cond_min):
            return System(name, L, n, d, pp, mp, var, ex, np.ascontiguousarray(cff), xstar, seed,
                          steps, bidx)
    raise RuntimeError(f"no system with cond <= {cond_max} after {max_tries} draws")


# Damping and boost readings.  The paper recommends decaying coefficients so
# that the series problem is well conditioned (Section 1.3, the ratio theorem
# of Fabry) and damps t by a factor delta (end of Section 3).  Coefficients
# drawn uniform in [0.5, 1.5] for every order make the block Toeplitz solve
# amplify rounding errors by a factor 4 to 65 per coefficient on these
# systems, so every preset draws coefficient k in delta^k * [0.5, 1.5] with
# delta = 1/4 (a power of two: the scaling is exact), and boosted presets
# start the diagonal boost at twice the row's absolute sum (cond(A_0) ~ 4).
# The small system has no boost (it is only redrawn until cond(A_0) <= 1e3)
# and the large one has monomials of degree up to 24: with delta = 1/4 the
# unconverged coefficients of their Newton iterates grow to 1e4 and 1e22 and
# the last step cancels them, so those two use delta = 1/8.
DAMPING = 0.25
DAMPING_STRONG = 0.125
BOOST_GAMMA = 2.0


def small_dd(seed: int = 1) -> System:
    """n=8, d=15, dd; 8 monomials x 3 distinct variables, exponent 1; 4 steps.

    Redrawn until cond(A_0) <= 1e2 (inside the bound 1e3 of the recipe): the
    double-double tolerance 1e-28 is only about 8000 units in the last place,
    and one step amplifies rounding by cond(A_0) times the growth through the
    stages (about 40 here)."""
    return make_system("small_dd", 2, 8, 15, 8, 3, 3, (1,), seed, 1e2, boost=False, steps=4,
                       damping=DAMPING_STRONG)


def medium_qd(seed: int = 2) -> System:
    """n=64, d=63, qd; 32 monomials x 2..6 variables, exponents {1,2}; 6 steps."""
    return make_system("medium_qd", 4, 64, 63, 32, 2, 6, (1, 2), seed, 1e3, boost=True, steps=6,
                       damping=DAMPING, boost_gamma=BOOST_GAMMA)


def medium_qd_near_bound(seed: int = 2, cond_range=(3e2, 1e3)) -> System:
    """The medium quad-double system (n=64, d=63, 32 monomials of 2..6
    variables, exponents {1,2}) with the smallest boost that brings
    cond_2(A_0) at x*(0) under the configuration's bound 1e3, kept when that
    leaves it at least 3e2: the conditioning the configuration allows, instead
    of the well-conditioned default (cond ~ 4)."""
    return make_system("medium_qd_near_bound", 4, 64, 63, 32, 2, 6, (1, 2), seed, cond_range[1], boost=True,
                       steps=6, damping=DAMPING, boost_gamma=1e-3, cond_min=cond_range[0])


def large_od(seed: int = 3) -> System:
    """n=128, d=127, od; 64 monomials x 4..8 variables, exponents {1,2,3}; 8 steps."""
    return make_system("large_od", 8, 128, 127, 64, 4, 8, (1, 2, 3), seed, 1e4, boost=True, steps=8,
                       damping=DAMPING_STRONG, boost_gamma=BOOST_GAMMA)


def adjoint_qd(seed: int = 5) -> System:
    """n=32, d=31, qd; 32 monomials x 3..5 variables, exponents {1,2}."""
    return make_system("adjoint_qd", 4, 32, 31, 32, 3, 5, (1, 2), seed, 1e3, boost=True, steps=6,
                       damping=DAMPING, boost_gamma=BOOST_GAMMA)


def tiny(L: int, n: int, d: int, mons: int = 3, kmin: int = 1, kmax: int = 3, exps=(1, 2),
         seed: int = 0, boost: bool = True, cond_max: float = 1e3, damping: float = DAMPING) -> System:
    """Small systems for parity tests that the oracle finishes in seconds."""
    return make_system(f"tiny_L{L}_n{n}_d{d}", L, n, d, mons, kmin, kmax, exps, seed, cond_max,
                       boost=boost, steps=1, damping=damping, boost_gamma=BOOST_GAMMA)


def batch_paths(count: int = 2048, L: int = 4, seed: int = 7, n_range=(16, 96), d_choices=(15, 31, 63),
                mons_range=(8, 32), k_range=(2, 5), exps=(1,)) -> list:
    """Independent systems of uneven size for the batched step: path j has n
    uniform in n_range, d from d_choices, a per-path number of monomials per
    polynomial uniform in mons_range, monomials of k_range variables with the
    given exponents, a diagonal boost, damped manufactured solutions."""
    rng = np.random.default_rng([seed, 31337])
    out = []
    for j in range(count):
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        d = int(rng.choice(d_choices))
        mons = int(rng.integers(mons_range[0], mons_range[1] + 1))
        out.append(make_system(f"path{j}", L, n, d, mons, k_range[0], k_range[1], exps, seed * 100003 + j, 1e3,
                               boost=True, steps=6, damping=DAMPING, boost_gamma=BOOST_GAMMA, vectorized=True))
    return out


def bucket_paths(L: int = 4, seed: int = 11, ns=(20, 48, 90), ds=(15, 31, 63)) -> list:
    """One path per size class of the batched workload: every n of ``ns``
    with every d of ``ds`` (by default one path in each of the nine (n, D)
    classes n <= 32, <= 64, <= 96 and D <= 16, 32, 64), drawn like
    batch_paths (8..32 monomials per polynomial of 2..5 variables, exponent
    1, boost, damped manufactured solutions)."""
    rng = np.random.default_rng([seed, 4711])
    out = []
    for n in ns:
        for d in ds:
            mons = int(rng.integers(8, 33))
            out.append(make_system(f"bucket_n{n}_d{d}", L, n, d, mons, 2, 5, (1,), seed * 100003 + n * 131 + d,
                                   1e3, boost=True, steps=6, damping=DAMPING, boost_gamma=BOOST_GAMMA,
                                   vectorized=True))
    return out


def small_batch(L: int = 4, seed: int = 9) -> list:
    """A few small paths for parity tests (the oracle finishes each in seconds):
    n in 3..12, d in {0, 3, 7, 15}, several size buckets."""
    return batch_paths(8, L, seed, (3, 12), (0, 3, 7, 15), (2, 5), (1, 3), (1, 2))


PRESETS = {
    "small_dd": small_dd,
    "medium_qd": medium_qd,
    "large_od": large_od,
    "adjoint_qd": adjoint_qd,
}


def _round_limbs(values, L: int) -> np.ndarray:
    """Exact rationals to L-limb multiple doubles, limb by limb to nearest."""
    from fractions import Fraction

    vals = list(values)
    out = np.zeros((L, len(vals)))
    for q, v in enumerate(vals):
        r = Fraction(v)
        for l in range(L):
            f = float(r)
            out[l, q] = f
            r -= Fraction(f)
    return out


def _exp_coefficients(a, D: int):
    """a^k / k! for k < D, exact rationals (a a rational)."""
    from fractions import Fraction

    c = [Fraction(1)]
    for k in range(1, D):
        c.append(c[-1] * a / k)
    return c


def column_system(n: int, d: int, L: int, columns: int = 1, seed: int = 0, delta: float = 0.25) -> System:
    """The paper's test systems (Section 3): x^E = b(t) with E the lower
    triangular matrix of ones (row i is x_0 x_1 ... x_i), or with two columns
    c_1 x^{E_1} + c_2 x^{E_2} = b(t), E_1 lower and E_2 the reversed
    triangle (row i is x_0 ... x_{n-1-i}).  The solution is
    x_j(t) = exp(alpha_j t) with alpha_j in [-1, -1 + delta] or [1 - delta, 1]
    (sign and value random, a multiple of 2^-20 so that every sum is exact),
    so b_i(t) is a sum of c exp(S t) with S a partial sum of the alphas, and
    both x* and c_{i,0} = -b_i are exact rationals rounded to L limbs.
    Two-column coefficients: c_1 in [1.5, 2], c_2 in [0.25, 0.5] (doubles),
    which keeps the 2 x 2 pairs of equations (k, n-1-k) well conditioned."""
    from fractions import Fraction

    if columns not in (1, 2):
        raise ValueError("one or two columns")
    rng = np.random.default_rng([seed, n, d, columns])
    D = d + 1
    sign = np.where(rng.random(n) < 0.5, -1, 1)
    mag = 1.0 - delta * rng.random(n)
    alpha = [Fraction(int(round(float(s * m) * 2 ** 20)), 2 ** 20) for s, m in zip(sign, mag)]
    part = [Fraction(0)]
    for a in alpha:
        part.append(part[-1] + a)  # part[i + 1] = alpha_0 + ... + alpha_i
    poly_ptr, mon_ptr, var, exp, cf = [0], [0], [], [], []
    c1 = rng.uniform(1.5, 2.0, n) if columns == 2 else np.ones(n)
    c2 = rng.uniform(0.25, 0.5, n)
    rhs = []
    for i in range(n):
        sup = [list(range(i + 1))] + ([list(range(n - i))] if columns == 2 else [])
        coef = [float(c1[i])] + ([float(c2[i])] if columns == 2 else [])
        b = [Fraction(0)] * D
        for vs, c in zip(sup, coef):
            var.extend(vs)
            exp.extend([1] * len(vs))
            mon_ptr.append(len(var))
            cf.append(c)
            for k, e in enumerate(_exp_coefficients(part[len(vs)], D)):
                b[k] += Fraction(c) * e
        poly_ptr.append(len(cf))
        rhs.append(b)
    xs = [_exp_coefficients(a, D) for a in alpha]
    xstar = _round_limbs([v for row in xs for v in row], L).reshape(L, n, D)
    cst = _round_limbs([-v for row in rhs for v in row], L).reshape(L, n, D)
    cff = np.zeros((L, len(cf)))
    cff[0] = cf
    return System(f"column{columns}_L{L}_n{n}_d{d}", L, n, d, np.array(poly_ptr, np.int32),
                  np.array(mon_ptr, np.int32), np.array(var, np.int32), np.array(exp, np.int32), cff, xstar, seed,
                  steps=1, cst=cst)


def _cmul(a, b):
    """(a0 + i a1)(b0 + i b1) on pairs of exact rationals."""
    return (a[0] * b[0] - a[1] * b[1], a[0] * b[1] + a[1] * b[0])


def _cexp_coefficients(a, D: int):
    """a^k / k! for k < D, a a pair of exact rationals."""
    from fractions import Fraction

    c = [(Fraction(1), Fraction(0))]
    for k in range(1, D):
        p = _cmul(c[-1], a)
        c.append((p[0] / k, p[1] / k))
    return c


def complex_column_system(n: int, d: int, L: int, columns: int = 1, seed: int = 0) -> System:
    """The paper's column systems with complex data (Sections 3 and 5.2):
    x_j(t) = exp(alpha_j t) with alpha_j = cos(theta_j) + i sin(theta_j),
    |alpha_j| = 1 up to rounding its parts to multiples of 2^-20, theta_j
    uniform; b_i(t) = exp(S_i t) (one column) or c_1 exp(S_i t) + c_2
    exp(S_{n-1-i} t) (two columns, real c as in column_system), S_i the partial
    sums of the alphas; x* and c_{i,0} = -b_i exact complex rationals rounded
    to L limbs per part.  cff [2, L, m], xstar and cst [2, L, n, D]."""
    from fractions import Fraction

    if columns not in (1, 2):
        raise ValueError("one or two columns")
    rng = np.random.default_rng([seed, n, d, columns, 7])
    D = d + 1
    theta = rng.uniform(0.0, 2.0 * np.pi, n)
    q = lambda v: Fraction(int(round(float(v) * 2 ** 20)), 2 ** 20)
    alpha = [(q(np.cos(t)), q(np.sin(t))) for t in theta]
    part = [(Fraction(0), Fraction(0))]
    for a in alpha:
        part.append((part[-1][0] + a[0], part[-1][1] + a[1]))
    poly_ptr, mon_ptr, var, exp, cf = [0], [0], [], [], []
    c1 = rng.uniform(1.5, 2.0, n) if columns == 2 else np.ones(n)
    c2 = rng.uniform(0.25, 0.5, n)
    re_b, im_b = [], []
    for i in range(n):
        sup = [list(range(i + 1))] + ([list(range(n - i))] if columns == 2 else [])
        coef = [float(c1[i])] + ([float(c2[i])] if columns == 2 else [])
        b = [(Fraction(0), Fraction(0)) for _ in range(D)]
        for vs, c in zip(sup, coef):
            var.extend(vs)
            exp.extend([1] * len(vs))
            mon_ptr.append(len(var))
            cf.append(c)
            for k, e in enumerate(_cexp_coefficients(part[len(vs)], D)):
                b[k] = (b[k][0] + Fraction(c) * e[0], b[k][1] + Fraction(c) * e[1])
        poly_ptr.append(len(cf))
        re_b.append([-v[0] for v in b])
        im_b.append([-v[1] for v in b])
    xs = [_cexp_coefficients(a, D) for a in alpha]
    xstar = np.stack([_round_limbs([v[0] for row in xs for v in row], L).reshape(L, n, D),
                      _round_limbs([v[1] for row in xs for v in row], L).reshape(L, n, D)])
    cst = np.stack([_round_limbs([v for row in re_b for v in row], L).reshape(L, n, D),
                    _round_limbs([v for row in im_b for v in row], L).reshape(L, n, D)])
    cff = np.zeros((2, L, len(cf)))
    cff[0, 0] = cf
    return System(f"ccolumn{columns}_L{L}_n{n}_d{d}", L, n, d, np.array(poly_ptr, np.int32),
                  np.array(mon_ptr, np.int32), np.array(var, np.int32), np.array(exp, np.int32), cff, xstar, seed,
                  steps=1, cst=cst)


def complex_random(sys: System, seed: int, lo: float = -1.0, hi: float = 1.0):
    """Random complex data for a system's tables: (cff [2, L, m], cst [2, L, n, D], x [2, L, n, D])."""
    rng = np.random.default_rng([seed, 31337])
    L, n, D, m = sys.L, sys.n, sys.D, sys.m
    cff = np.stack([random_md(rng, L, (m,), lo, hi) for _ in range(2)])
    cst = np.stack([random_md(rng, L, (n, D), lo, hi) for _ in range(2)])
    x = np.stack([random_md(rng, L, (n, D), lo, hi) for _ in range(2)])
    return cff, cst, x


def random_point(sys: System, seed: int, lo: float = 0.5, hi: float = 1.5) -> np.ndarray:
    """A random series point x[L, n, D] for evaluation tests."""
    rng = np.random.default_rng([seed, 7919])
    return random_series(rng, sys.L, sys.n, sys.D, lo, hi)


def random_constant(sys: System, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """A random constant series c_{i,0}(t), shape [L, n, D]."""
    rng = np.random.default_rng([seed, 104729])
    return random_md(rng, sys.L, (sys.n, sys.D), lo, hi)
