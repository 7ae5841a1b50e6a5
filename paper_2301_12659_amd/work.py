"""Algorithmic work of one Newton step, per kernel class.

Counts are the multiple-double operations the method must perform (unpadded
truncated convolutions: D(D+1)/2 multiply-adds per series product, the
paper pads to D^2, Section 5.1), expressed as double flops with the
instruction and flop counts of this library's own generated routines
(csrc/md_counts.json; a fused multiply-add counts as two flops).  A
convolution output is a multiple-double dot product: its multiply-adds are
accumulated as level sums ("fma_lazy") and renormalized once ("renorm").
"""
from __future__ import annotations

import json
import os

import numpy as np

_COUNTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", "md_counts.json")


def md_costs(L: int) -> dict:
    with open(_COUNTS) as f:
        return json.load(f)[str(L)]


def monomial_products(k: int, exps) -> tuple[int, int]:
    """(series-by-series convolutions, scalar-by-series products) of one
    monomial in the reverse-mode scheme with a common factor."""
    if k == 0:
        return 0, 0
    big = [e for e in exps if e >= 2]
    conv = max(len(big) - 1, 0)          # common factor chain
    scal = 1 if big else 0               # f_0 = c * CF
    f0_scalar = not big
    conv += max(k - 2, 0)                # backward products
    for j in range(1, k + 1):
        if j < k:                        # cross product
            if f0_scalar and j == 1:
                scal += 1
            else:
                conv += 1
        if f0_scalar and j == 1:         # forward product
            scal += 1
        else:
            conv += 1
    return conv, scal


def step_work(sys) -> dict:
    """Multiply-add counts per kernel class for one Newton step of a system
    (an mdinputs.System or anything with L, n, D, mon_ptr, exp, poly_ptr)."""
    L, n, D = sys.L, sys.n, sys.D
    conv = scal = 0
    for j in range(len(sys.mon_ptr) - 1):
        e = sys.exp[sys.mon_ptr[j]:sys.mon_ptr[j + 1]]
        c, s = monomial_products(len(e), e)
        conv += c
        scal += s
    maxexp = int(sys.exp.max()) if len(sys.exp) else 1
    if maxexp >= 3:
        conv += n * (maxexp - 2)         # power table
    tri = D * (D + 1) // 2
    w = {}
    w["convolutions"] = {"fma_lazy": conv * tri, "renorm": conv * D, "mul": scal * D, "products": conv,
                         "scalar_products": scal}
    # assembly: additions into b and A
    m = len(sys.mon_ptr) - 1
    nnz = len(sys.var)
    w["assembly"] = {"add": (m + 0) * D + max(nnz - 0, 0) * D}
    qr = sum((n - c) + 2 * (n - c) * (n - c - 1) for c in range(n))
    w["qr"] = {"fma": qr}
    w["qhb_bs"] = {"fma": n * (sum(2 * (n - r) for r in range(n)) + n * (n - 1) // 2)}
    w["gemm"] = {"fma": n * n * n if D > 1 else 0}
    upd = n * n + sum(2 * n * n + (D - k - 1) * n * n for k in range(1, D))
    w["updates"] = {"fma": upd}
    w["x_update"] = {"add": n * D}
    cost = md_costs(L)
    ops = ("fma", "fma_lazy", "renorm", "mul", "add")
    for cls, d in w.items():
        fl = sum(d.get(o, 0) * cost[o]["flops"] for o in ops)
        ins = sum(d.get(o, 0) * cost[o]["instr"] for o in ops)
        d["flops"] = int(fl)
        d["instr"] = int(ins)
    return w


# The paper's convention (Table 2): md multiplications in zero-padded
# convolutions (D^2 per product) times 23 / 336 / 1742 double flops (one for
# a double).
PAPER_MUL_COST = {1: 1, 2: 23, 4: 336, 8: 1742}


def paper_convention_flops(sys) -> int:
    w = step_work(sys)["convolutions"]
    return int(w["products"] * sys.D * sys.D * PAPER_MUL_COST[sys.L])


def convolution_flops(sys, order: int) -> dict:
    """Evaluation and differentiation of the system at series of `order`
    coefficients: this library's flops (unpadded convolutions) and the paper's
    convention (zero-padded order^2 multiplications per product, Table 2)."""
    conv = scal = 0
    for j in range(len(sys.mon_ptr) - 1):
        e = sys.exp[sys.mon_ptr[j]:sys.mon_ptr[j + 1]]
        c, s = monomial_products(len(e), e)
        conv += c
        scal += s
    cost = md_costs(sys.L)
    ours = (conv * order * (order + 1) // 2 * cost["fma_lazy"]["flops"] + conv * order * cost["renorm"]["flops"] +
            scal * order * cost["mul"]["flops"])
    return {"flops": int(ours), "paper_flops": int(conv * order * order * PAPER_MUL_COST[sys.L]), "products": conv}


# ----------------------------------------------------------------- latency
#
# The QR of A_0 and the staged solve are dependent chains: each column of
# the factorization needs the previous reflector, each stage the previous
# dx.  Their bound is not the FP64 issue rate of the chip but the length of
# the chain times the cycles one wavefront needs per dependent instruction
# (measured with clock stamps in one wavefront: about 4.8 cycles per FP64
# instruction of a multiple-double chain at 2.4 GHz), plus what a hand-over
# between workgroups costs (measured: about 0.6 us for a flag).

CYCLES_PER_DEP_INSTR = 4.8
CLOCK_HZ = 2.4e9
HANDOVER_S = 0.6e-6


def _butterfly(c, width=64):
    """A sum of level-sum accumulators over `width` lanes: log2(width)
    add_lazy levels, then one renormalization."""
    levels = int(np.log2(width))
    return levels * c["add_lazy"]["instr"] + c["renorm"]["instr"]


def newton_chain_instr(L: int, kind: str) -> int:
    """FP64 instructions of the shortened 1/sqrt or reciprocal sequences of
    the Householder reflector (md.hpp: rsqrt_short, recip_short; the full
    sequences for octo doubles), counted from their multiple-double
    operations."""
    def c(P):
        return md_costs(P)

    total = 2  # the double start: a square root or a division
    if L == 4:
        # one doubling at two limbs, then the last one with a fused residual
        # at four limbs, two renormalizations and a two-limb correction
        cp, c2, c4 = c(2), c(4), c(4)
        if kind == "rsqrt":
            total += 2 * cp["mul"]["instr"] + cp["sub"]["instr"] + 1 + cp["add"]["instr"]
            total += (c4["mul"]["instr"] + c4["fms"]["instr"] + 2 * c4["renorm"]["instr"] + c2["mul"]["instr"] + 2 +
                      c4["add"]["instr"])
        else:
            total += cp["mul"]["instr"] + cp["sub"]["instr"] + 1 + cp["add"]["instr"]
            total += c4["fms"]["instr"] + 2 * c4["renorm"]["instr"] + c2["mul"]["instr"] + c4["add"]["instr"]
        return int(total)
    if L >= 8:  # full sequence: steps at 2, 4, 8 limbs, then a one-limb-correction step at 8
        steps = [(2, 1), (4, 2), (8, 8), (8, 1)]
    else:
        steps = [(2, 2)]
    for P, H in steps:
        cp = c(P)
        corr = 1 if H == 1 else c(H)["mul"]["instr"]
        if kind == "rsqrt":  # y^2, a y^2, 1 - a y^2, correction, y + c
            total += 2 * cp["mul"]["instr"] + cp["sub"]["instr"] + corr + cp["add"]["instr"]
        else:                # v r, 1 - v r, correction, r + c
            total += cp["mul"]["instr"] + cp["sub"]["instr"] + corr + cp["add"]["instr"]
    return int(total)


def qr_latency_bound(L: int, n: int, with_qt: bool = True) -> dict:
    """Lower bound of the column-by-column Householder QR of A_0 (with Q^T
    on the augmented columns) as the LDS-resident kernel orders it.  The
    dot S of reflector c with the next column is formed from the first part
    of the hand-over while the owner of column c still computes the scalars,
    so the chain of a column is: the finish of column c+1 with tau and
    1/(x_0 - beta) (d = y_c + S/(x_0 - beta), tau d, tau d/(x_0 - beta), the
    multiply-add of the rows), its norm (one lazy multiply-add per lane, a
    64-lane butterfly), beta, the reflector scalars (1/sqrt and a
    reciprocal), x_0 - beta, and one hand-over of the scalars."""
    c = md_costs(L)
    dot = c["fma_lazy"]["instr"] + _butterfly(c)
    per_col = (2 * c["fma"]["instr"] + 3 * c["mul"]["instr"] + dot + newton_chain_instr(L, "rsqrt") +
               newton_chain_instr(L, "recip") + c["sub"]["instr"])
    s = n * (per_col * CYCLES_PER_DEP_INSTR / CLOCK_HZ + HANDOVER_S)
    return {"chain_instr_per_column": int(per_col), "columns": n, "seconds": s}


def stages_latency_bound(L: int, n: int, D: int) -> dict:
    """Lower bound of the persistent staged solve: per stage one lazy
    multiply-add per lane (N dx_{k-1}, the other terms are accumulated off
    the chain), a 64-lane butterfly, the renormalization, and one hand-over
    of dx_k between the solver workgroups."""
    c = md_costs(L)
    per_stage = c["fma_lazy"]["instr"] + _butterfly(c)
    s = D * (per_stage * CYCLES_PER_DEP_INSTR / CLOCK_HZ + HANDOVER_S)
    return {"chain_instr_per_stage": int(per_stage), "stages": D, "seconds": s}
