"""Test-side helpers: exact conversions and hand-made systems (no method arithmetic)."""
from __future__ import annotations

from fractions import Fraction

import numpy as np

import mdinputs


def to_md(values, L: int) -> np.ndarray:
    """Round exact values (Fraction / int / mpmath mpf) to L-limb multiple doubles.

    Limb by limb: each limb is the nearest double to what remains."""
    vals = list(values)
    out = np.zeros((L, len(vals)))
    for q, v in enumerate(vals):
        r = Fraction(v) if not isinstance(v, Fraction) else v
        for l in range(L):
            d = float(r)
            out[l, q] = d
            r -= Fraction(d)
    return out


def md_value(limbs) -> Fraction:
    """Exact value of one multiple double (sum of limbs)."""
    return sum((Fraction(float(d)) for d in limbs), Fraction(0))


def make(L, n, d, polys, cff_values=None):
    """Build a System from polys = [[(coef, [(var, exp), ...]), ...] per row].

    Coefficients are exact rationals rounded to L limbs."""
    pp, mp, var, ex, cf = [0], [0], [], [], []
    for row in polys:
        for coef, sup in row:
            for v, e in sorted(sup):
                var.append(v)
                ex.append(e)
            mp.append(len(var))
            cf.append(coef)
        pp.append(len(mp) - 1)
    cff = to_md(cf, L)
    D = d + 1
    return mdinputs.System("hand", L, n, d, np.asarray(pp, np.int32), np.asarray(mp, np.int32),
                           np.asarray(var, np.int32), np.asarray(ex, np.int32), cff,
                           np.zeros((L, n, D)), 0)


def series_md(coefs, L):
    """coefs[n][D] exact values -> md array [L, n, D]."""
    n, D = len(coefs), len(coefs[0])
    flat = [c for row in coefs for c in row]
    return to_md(flat, L).reshape(L, n, D)
