"""Accuracy of the precision-doubling Newton sequences of the multiple-double
header, compiled for the host: 1/sqrt(a) and 1/a by the full sequences and by
the shortened ones of the Householder reflector, checked with exact rational
arithmetic on the residuals a y^2 - 1 and a r - 1 (no oracle involved)."""
import math
import os
import shutil
import subprocess
import tempfile
from fractions import Fraction

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def exe():
    if not (os.path.exists(HIPCC) or shutil.which("hipcc")):
        pytest.skip("hipcc not available")
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "md_host_check")
        # host code only: the header's routines are host and device functions
        cmd = [HIPCC, "-x", "hip", "-O2", "-ffp-contract=off", "-fno-fast-math", "--offload-arch=gfx950",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               os.path.join(HERE, "md_host_check.cpp"), "-o", path]
        r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
        assert r.returncode == 0, r.stderr[-2000:]
        yield path


@pytest.fixture(scope="module")
def rows(exe):
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120, check=True).stdout
    res = []
    for line in out.split("\n"):
        if not line.strip():
            continue
        p = line.split()
        L = int(p[0])
        v = [float.fromhex(x) for x in p[1:]]
        a, y, r, y2, r2 = (sum((Fraction(x) for x in v[i * L:(i + 1) * L]), Fraction(0)) for i in range(5))
        res.append((L, a, y, r, y2, r2))
    return res


def _log2(x):
    return math.log2(abs(float(x))) if x != 0 else -math.inf


@pytest.mark.parametrize("L, full_bits, short_bits", [(2, 103, 103), (4, 209, 205), (8, 421, 421)])
def test_doubling_sequences_reach_their_precision(rows, L, full_bits, short_bits):
    """Relative errors |y sqrt(a) - 1| ~ |a y^2 - 1| / 2 and |a r - 1|: the
    full sequences end within a few units of the last limb (2^-(53 L)); the
    shortened ones (full-width corrections, no repair step) within 2^-(53 L - 7)
    for double and quad doubles; octo doubles keep the full sequence."""
    sel = [t for t in rows if t[0] == L]
    assert len(sel) == 200
    worst = {"y_short": -math.inf, "r_short": -math.inf, "y_full": -math.inf, "r_full": -math.inf}
    for _, a, y, r, y2, r2 in sel:
        worst["y_short"] = max(worst["y_short"], _log2((a * y * y - 1) / 2))
        worst["r_short"] = max(worst["r_short"], _log2(a * r - 1))
        worst["y_full"] = max(worst["y_full"], _log2((a * y2 * y2 - 1) / 2))
        worst["r_full"] = max(worst["r_full"], _log2(a * r2 - 1))
    assert worst["y_full"] <= -full_bits and worst["r_full"] <= -full_bits, worst
    assert worst["y_short"] <= -short_bits and worst["r_short"] <= -short_bits, worst


# ------------------------------------------------ accurate addition


def _md(v: Fraction, L: int):
    """Round an exact value to L limbs, each the nearest double to what remains."""
    out = []
    for _ in range(L):
        d = float(v)
        out.append(d)
        v -= Fraction(d)
    return out


def _val(limbs):
    return sum((Fraction(x) for x in limbs), Fraction(0))


def _cancellation_cases(L, count, rng):
    """Operand pairs whose sum cancels at every depth: b = -a plus a
    perturbation below limb k, b = -a (1 + 2^-j), b = -a limb by limb with
    one limb changed, leading limbs cancelling while the tails do not, and
    unrelated operands of any relative size."""
    def rand_md(scale):
        v = Fraction(scale)
        for l in range(1, L + 3):
            v += Fraction(rng.uniform(-1, 1)) * Fraction(scale) * Fraction(2) ** (-53 * l - rng.randint(0, 3))
        return _md(v, L)

    cases = []
    for t in range(count):
        a = rand_md(rng.uniform(0.5, 2.0) * 2.0 ** rng.randint(-5, 5))
        A = _val(a)
        mode = t % 5
        if mode == 0:
            k = rng.randint(0, L)
            b = _md(-A + Fraction(rng.uniform(-1, 1)) * abs(A) * Fraction(2) ** (-53 * k - rng.randint(0, 52)), L)
        elif mode == 1:
            b = _md(-A * (1 + Fraction(rng.randint(1, 8)) * Fraction(2) ** (-rng.randint(1, 53 * L))), L)
        elif mode == 2:
            b = [-x for x in a]
            j = rng.randint(1, L - 1)
            b[j] = -a[j] * (1 + rng.uniform(-1, 1) * 2.0 ** -rng.randint(1, 52))
            for q in range(j + 1, L):
                b[q] = rng.uniform(-1, 1) * abs(b[q - 1]) * 2.0 ** -53
        elif mode == 3:
            b = [-a[0]] + [(-a[q] + a[q] * 2.0 ** -rng.randint(1, 60)) if rng.random() < 0.5
                           else rng.uniform(-1, 1) * abs(a[q]) for q in range(1, L)]
        else:
            b = rand_md(rng.uniform(-2.0, 2.0) * 2.0 ** rng.randint(-60, 5))
        cases.append((a, b))
    return cases


@pytest.mark.parametrize("L", [2, 4, 8])
def test_accurate_add_relative_to_the_result(exe, L):
    """add_acc and sub_acc: |computed - exact| <= 2^(-53 L) |exact| on operands
    whose sum cancels at every depth (exact results as rationals; an exact
    zero must come out as zero).  The level-sum add, which drops the rounding
    errors of its last level, fails this by about 2^50."""
    import random

    rng = random.Random(1000 + L)
    cases = _cancellation_cases(L, 1500, rng)
    inp = "".join(f"{L} " + " ".join(x.hex() for x in a + b) + "\n" for a, b in cases)
    out = subprocess.run([exe, "add"], input=inp, capture_output=True, text=True, timeout=120, check=True).stdout
    lines = [ln for ln in out.split("\n") if ln.strip()]
    assert len(lines) == len(cases)
    worst = -math.inf
    for (a, b), ln in zip(cases, lines):
        v = [float.fromhex(x) for x in ln.split()[1:]]
        for got, ex in ((_val(v[:L]), _val(a) + _val(b)), (_val(v[L:]), _val(a) - _val(b))):
            if ex == 0:
                assert got == 0
                continue
            worst = max(worst, _log2((got - ex) / ex))
    assert worst <= -53 * L, worst
