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
def rows():
    if not (os.path.exists(HIPCC) or shutil.which("hipcc")):
        pytest.skip("hipcc not available")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "md_host_check")
        # host code only: the header's routines are host and device functions
        cmd = [HIPCC, "-x", "hip", "-O2", "-ffp-contract=off", "-fno-fast-math", "--offload-arch=gfx950",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               os.path.join(HERE, "md_host_check.cpp"), "-o", exe]
        r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
        assert r.returncode == 0, r.stderr[-2000:]
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
