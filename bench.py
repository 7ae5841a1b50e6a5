#!/usr/bin/env python3
"""Newton steps/s on one MI355X for the medium quad-double system.

Workload: n = 64 polynomials in 64 variables, truncation degree d = 63
(D = 64 coefficients), quad double; 32 monomials of 2..6 variables with
exponents in {1, 2} per polynomial plus a diagonal boost; seeded synthetic
data (mdinputs.medium_qd).  A step is one full md_newton_step: evaluation
and differentiation by convolutions, assembly, Householder QR of A_0, the
staged block Toeplitz solve and the update, on inputs resident on the GPU.

Prints one JSON line.  --gpus above 1 is refused: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6  # MI355X FP64 vector, FMA = 2 flops


# sources the evaluation/differentiation kernel is compiled from; the HBM
# traffic recorded from hardware counters is reported only while they are
# unchanged since the counters were taken
_EVALDIFF_SOURCES = ("evaldiff.hip", "evaldiff_dev.hpp", "evalargs.hpp", "common.hpp", "md.hpp", "md_gen.inc")
_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "evaldiff_pair_kernel_medium_qd_hbm_traffic.md")


def evaldiff_source_sha256():
    import hashlib

    h = hashlib.sha256()
    for f in _EVALDIFF_SOURCES:
        with open(os.path.join(ROOT, "paper_2301_12659_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _recorded_traffic():
    """HBM bytes per evaldiff launch (FETCH_SIZE + WRITE_SIZE, scaled by the
    same counters' reading for a copy of known size), or None when no record
    exists or the kernel's sources changed since it was taken."""
    try:
        with open(_TRAFFIC_FILE) as fh:
            kv = dict(line.strip().split(": ", 1) for line in fh if line.startswith(("source_sha256:", "fetch_bytes_per_launch:", "write_bytes_per_launch:")))
    except OSError:
        return None
    if kv.get("source_sha256") != evaldiff_source_sha256():
        return None
    return int(kv["fetch_bytes_per_launch"]) + int(kv["write_bytes_per_launch"])


_SQ_FILE = os.path.join(ROOT, "profiles", "evaldiff_pair_kernel_medium_qd_sq_counters.md")


def _recorded_sq():
    """FP64 VALU instruction counts per evaldiff launch from the recorded SQ
    counters, or None when no record exists or the kernel's sources changed
    since it was taken."""
    try:
        with open(_SQ_FILE) as fh:
            kv = dict(line.strip().split(": ", 1) for line in fh if ": " in line and line.split(":")[0] in
                      ("source_sha256", "add_f64", "mul_f64", "fma_f64", "trans_f64", "valu"))
    except OSError:
        return None
    if kv.get("source_sha256") != evaldiff_source_sha256():
        return None
    try:
        return {k: float(v) for k, v in kv.items() if k != "source_sha256"}
    except ValueError:
        return None


def _err_vs(mdn, torch, x, ref):
    """Normwise relative error per series, max over series, of x against ref
    (both [L, n, D] device tensors), computed with the library's md subtraction."""
    L = x.shape[0]
    a = x.reshape(L, -1).contiguous()
    b = ref.reshape(L, -1).contiguous()
    d = torch.empty_like(a)
    mdn.arith(L, "sub", a, b, d)
    diff = d[0].abs().reshape(x.shape[1:])
    mag = ref[0].abs().amax(dim=-1)
    return float((diff.amax(dim=-1) / mag).max().item())


def _bench_batch(mdn, torch, np, mdinputs, npaths, steps):
    """The batched workload: npaths independent quad-double paths, n in
    16..96, d in {15, 31, 63}, 8..32 monomials per polynomial of 2..5
    variables with exponent 1, manufactured solutions (constants evaluated on
    the GPU); plain steps and qd residual / dd solve steps, each a graph
    replay of one persistent launch."""
    paths = mdinputs.batch_paths(npaths, 4)
    b = mdn.Batch(paths)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    # c_{i,0} = -p_i(x*) with zero constant, path by path on the GPU
    cst_parts = []
    for s in paths:
        plan = mdn.Plan.from_system(s)
        ws1 = mdn.workspace(plan.workspace_bytes())
        bb = torch.empty((4, s.n, s.D), dtype=torch.float64, device="cuda")
        AA = torch.empty((4, s.n, s.n, s.D), dtype=torch.float64, device="cuda")
        mdn.eval_diff(plan, dev(s.cff), torch.zeros_like(bb), dev(s.xstar), bb, AA, ws1)
        cst_parts.append(bb.cpu().numpy())
        del AA, ws1
        plan.close()
    cff = dev(b.pack_cff([s.cff for s in paths]))
    cst = dev(b.pack_series(cst_parts))
    x0 = dev(b.pack_series([s.start() for s in paths]))
    status = torch.zeros(npaths, dtype=torch.int32, device="cuda")
    norms = torch.zeros(2 * npaths, dtype=torch.float64, device="cuda")
    ws = mdn.workspace(b.workspace_bytes())
    x = x0.clone()
    t0 = time.perf_counter()
    tiles = b.autotune(cff, cst, x, torch.empty_like(x), status, norms, ws)
    tune_s = time.perf_counter() - t0
    res = {"workload": f"{npaths} quad-double paths, n 16..96, d in {{15,31,63}}, 8..32 monomials per polynomial, "
                       "2..5 variables, exponent 1, manufactured solutions, seed 7",
           "paths": npaths, "total_unknown_series": int(sum(s.n for s in paths)),
           "tiles_per_bucket": tiles, "autotune_s": round(tune_s, 2)}
    xs = dev(b.pack_series([s.xstar for s in paths]))
    # per-path relative error against x*: the library's md subtraction, then
    # max |diff| / max |x*| over each path's block (leading limbs)
    bounds = [(int(o), int(o) + s.n * s.D) for o, s in zip(b.x_off, paths)]

    def worst_err():
        d = torch.empty_like(x)
        mdn.arith(4, "sub", x.contiguous(), xs, d)
        dd, xx = d[0].abs().cpu().numpy(), xs[0].abs().cpu().numpy()
        return max(float(dd[a:c].max() / xx[a:c].max()) for a, c in bounds)

    for name, ls in (("plain_qd", 4), ("mixed_qd_dd", 2)):
        x.copy_(x0)
        for _ in range(2):  # eager, then captured
            b.step(cff, cst, x, status, norms, ws, prec_solve=ls)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            b.step(cff, cst, x, status, norms, ws, prec_solve=ls)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        bad = int((status != 0).sum().item())
        # steps from x*(0) until every path is within the quad-double tolerance
        x.copy_(x0)
        k = 0
        while k < 14:
            b.step(cff, cst, x, status, norms, ws, prec_solve=ls)
            k += 1
            if worst_err() <= 1e-60:
                break
        res[name] = {"ms_per_batched_step": round(ms, 3), "path_steps_per_s": round(npaths * 1000.0 / ms, 1),
                     "paths_not_ok": bad, "steps_to_tol": k, "worst_path_err": worst_err(),
                     "ms_to_tol": round(k * ms, 3)}
    res["tol"] = 1e-60
    return res


def _manufactured(mdn, torch, np, s):
    """A Newton driver on the system s with c_{i,0} = -P_i(x*) computed on the
    GPU (the evaluation at x* with a zero constant), at x*(0)."""
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    drv = mdn.Newton(s, np.zeros((s.L, s.n, s.D)), s.xstar)
    b = torch.empty((s.L, s.n, s.D), dtype=torch.float64, device="cuda")
    A = torch.empty((s.L, s.n, s.n, s.D), dtype=torch.float64, device="cuda")
    mdn.eval_diff(drv.plan, drv.cff, drv.cst, drv.x, b, A, drv.ws)
    drv.cst.copy_(b)
    drv.x.copy_(dev(s.start()))
    del A
    torch.cuda.synchronize()
    return drv, dev(s.start()), dev(s.xstar)


TOL = {1: 1e-12, 2: 1e-28, 4: 1e-60, 8: 1e-120}


def _bench_configs(mdn, torch, np, mdinputs, reps):
    """The other configurations: their full runs from x*(0) (small dd: 4
    steps, large od: 8, adjoint qd: 6) by md_newton_steps, steps/s over
    `reps` runs after one untimed run, the error against the manufactured
    solution; for the adjoint configuration also the backward pass of the
    differentiable solve (loss = sum of squares of the top 8 coefficients,
    gradient with respect to every monomial coefficient)."""
    res = {}
    for name, make, runs in (("small_dd", mdinputs.small_dd, reps), ("large_od", mdinputs.large_od, 1),
                             ("adjoint_qd", mdinputs.adjoint_qd, reps)):
        s = make()
        drv, x0, xs = _manufactured(mdn, torch, np, s)
        drv.steps(s.steps)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ms = 0.0
        for _ in range(runs):
            drv.x.copy_(x0)
            e0.record()
            drv.steps(s.steps)
            e1.record()
            torch.cuda.synchronize()
            ms += e0.elapsed_time(e1)
        r = {"n": s.n, "d": s.d, "precision": {2: "dd", 4: "qd", 8: "od"}[s.L], "steps_per_run": s.steps,
             "ms_per_step": round(ms / (runs * s.steps), 4), "steps_per_s": round(runs * s.steps * 1000.0 / ms, 2),
             "err_vs_manufactured": _err_vs(mdn, torch, drv.x, xs), "tol": TOL[s.L], "status": drv.status_code()}
        if name == "adjoint_qd":
            cff = drv.cff.clone().requires_grad_(True)
            times = []
            for q in range(reps + 1):
                x = mdn.newton_solve(cff, drv.plan, drv.cst, x0, s.steps)
                loss = mdn.top_coefficient_loss(x, s.D - 8)
                torch.cuda.synchronize()
                e0.record()
                mdn.md_backward(loss)
                e1.record()
                torch.cuda.synchronize()
                if q:
                    times.append(e0.elapsed_time(e1))
                cff.grad = None
            r["backward_ms"] = round(min(times), 4)
            r["backward"] = ("A(t) at the solution, QR of A_0, the transposed staged solve and the coefficient "
                             "gradients (%d monomial coefficients)" % s.m)
        res[name] = r
        del drv
        torch.cuda.empty_cache()
    return res


def _bench_mixed(mdn, torch, np, drv, x0, xstar, max_steps=12):
    """Time to the quad-double tolerance on the medium system from x*(0):
    plain quad-double steps against steps with a quad-double residual and a
    double-double solve (md_newton_step_mixed), each as many steps as reach
    1e-60 against the manufactured solution, timed back to back."""
    res = {}
    for name, ps in (("plain_qd", None), ("mixed_qd_dd", 2)):
        drv.x.copy_(x0)
        k = 0
        while k < max_steps:
            drv.step(prec_solve=ps)
            k += 1
            if _err_vs(mdn, torch, drv.x, xstar) <= 1e-60:
                break
        err = _err_vs(mdn, torch, drv.x, xstar)
        times = []
        for r in range(4):
            drv.x.copy_(x0)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(k):
                drv.step(prec_solve=ps)
            e1.record()
            torch.cuda.synchronize()
            if r:
                times.append(e0.elapsed_time(e1))
        res[name] = {"steps_to_tol": k, "ms_to_tol": round(min(times), 4), "ms_per_step": round(min(times) / k, 4),
                     "err_vs_manufactured": err}
    res["tol"] = 1e-60
    return res


def _bench_staggered(mdn, torch, np, sysm, cst, xstar, repeats):
    """Time to solution on the medium system from x*(0) with its trailing two
    limbs dropped (about half the working precision, the start the staggered
    method assumes): the staggered driver with A_0 factored once and with a
    factorization at every step, and plain full-order Newton steps, as many
    as it takes to reach the quad-double tolerance (timed back to back)."""
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    x0 = dev(sysm.half_precision_start())
    drv = mdn.Newton(sysm, np.zeros((sysm.L, sysm.n, sysm.D)), sysm.half_precision_start())
    drv.cst.copy_(cst)
    res = {"start": "x*(0) with its two trailing limbs dropped, higher coefficients zero",
           "tol": mdn.default_stagger_tol(sysm.L, int(np.max(np.diff(sysm.mon_ptr))))}
    for name, refac in (("qr_once", False), ("qr_every_step", True)):
        times = []
        for r in range(repeats + 1):  # the first run is not timed
            drv.x.copy_(x0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rep, win = drv.staggered(max_steps=40, refactor_every_step=refac)
            torch.cuda.synchronize()
            if r:
                times.append(time.perf_counter() - t0)
        res[name] = {"ms_to_solution": round(1000 * min(times), 3), "steps": rep.steps,
                     "factorizations": rep.factorizations, "converged": bool(rep.converged),
                     "err_vs_manufactured": _err_vs(mdn, torch, drv.x, xstar),
                     "windows": [list(w) for w in win]}
    drv.x.copy_(x0)
    k = 0
    while k < 20:
        drv.step()
        k += 1
        if _err_vs(mdn, torch, drv.x, xstar) <= 1e-60:
            break
    times = []
    for r in range(repeats + 1):
        drv.x.copy_(x0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(k):
            drv.step()
        torch.cuda.synchronize()
        if r:
            times.append(time.perf_counter() - t0)
    res["plain_newton"] = {"ms_to_solution": round(1000 * min(times), 3), "steps": k,
                           "err_vs_manufactured": _err_vs(mdn, torch, drv.x, xstar)}
    return res


def _bench_complex(mdn, torch, np, mdinputs, sysm):
    """Complex data (Section 5.2) on the medium system's tables: the
    evaluation with the 4M products side by side and the complex Newton step
    (real form of dimension 2n), timed with HIP events; right-hand side
    manufactured on the GPU at a complex x*."""
    from paper_2301_12659_amd import work

    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    cff, _, _ = mdinputs.complex_random(sysm, 70)
    cff[:, :, sysm.boost] = np.stack([4.0 * sysm.cff[:, sysm.boost], np.zeros_like(sysm.cff[:, sysm.boost])])
    xs = np.stack([sysm.xstar, 0.5 * mdinputs.random_series(np.random.default_rng(71), sysm.L, sysm.n, sysm.D,
                                                              damping=mdinputs.DAMPING)])
    drv = mdn.ComplexNewton(sysm, cff, np.zeros_like(xs), xs)
    b, _ = drv.eval_diff()
    drv.cst.copy_(b)
    x0 = dev(np.concatenate([xs[..., :1], np.zeros_like(xs[..., 1:])], axis=-1))
    res = {"workload": "medium_qd tables with complex coefficients and a complex x* (imaginary part damped like "
                       "the real one, boost four times the real system's), seed 70"}
    for name, fn, reps in (("evaluation", lambda: drv.eval_diff(), 20), ("newton_step", lambda: drv.step(), 10)):
        drv.x.copy_(x0)
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        res[name + "_ms"] = round(e0.elapsed_time(e1) / reps, 4)
    f = work.convolution_flops(sysm, sysm.D)["flops"] * 4  # four real products per complex one
    res["evaluation_tflops"] = round(f / (res["evaluation_ms"] * 1e-3) / 1e12, 3)
    drv.x.copy_(x0)
    for _ in range(8):
        drv.step()
    xsd = dev(xs)
    res["err_vs_manufactured_after_8_steps"] = max(_err_vs(mdn, torch, drv.x[0].contiguous(), xsd[0].contiguous()),
                                                   _err_vs(mdn, torch, drv.x[1].contiguous(), xsd[1].contiguous()))
    res["status"] = drv.status_code()
    return res


# The paper's printed figures for its own workloads (context only: other
# hardware).  Table 5: seconds of 24 Newton steps on the V100, octo double,
# n = 1024, order 64, one and two columns of monomials; Table 6: gigaflops of
# the evaluation and differentiation of one column of 1024 monomials in octo
# double by order; Table 7: kernel and wall-clock seconds of 24 steps on one
# column at order 64 on the V100 by precision.
PAPER_T5_V100 = {
    "one_column": {"convolution": 121.386, "householder_qr": 24.451, "qhb": 5.849, "back_substitution": 17.053,
                   "updates": 111.474, "residuals": 125.122, "total_kernel": 405.334, "wall": 1129.794},
    "two_columns": {"convolution": 244.535, "householder_qr": 24.123, "qhb": 6.139, "back_substitution": 17.884,
                    "updates": 124.080, "residuals": 137.963, "total_kernel": 554.723, "wall": 1808.480},
}
PAPER_T6 = {"V100": {1: 28.997, 2: 59.820, 3: 90.003, 5: 149.894, 8: 240.760, 12: 360.816, 18: 540.572,
                     27: 810.645, 41: 1045.032, 62: 1569.347, 64: 1658.382},
            "A100": {1: 39.284, 2: 95.770, 3: 147.440, 5: 252.502, 8: 411.946, 12: 623.255, 18: 938.634,
                     27: 1412.459, 41: 1601.007, 62: 2472.086, 64: 2568.016}}
PAPER_T7_V100 = {2: {"kernel": 22.6, "wall": 475.3}, 4: {"kernel": 146.4, "wall": 834.7},
                 8: {"kernel": 405.3, "wall": 1129.8}}
# Table 8: kernel and wall-clock seconds of 16 steps at n = 512, order 64, on
# the RTX 2080 Max-Q by precision (1: double).
PAPER_T8_RTX2080 = {1: {"kernel": 1.4, "wall": 35.7}, 2: {"kernel": 16.6, "wall": 80.0},
                    4: {"kernel": 122.4, "wall": 225.0}, 8: {"kernel": 380.1, "wall": 474.8}}


def _replay(mdn, torch, np, mdinputs, steps):
    """The paper's own workloads on this GPU: one and two columns of monomials
    with triangular exponent matrices of ones, n = 1024, exponential
    solutions (Section 3), `steps` steps of the staggered method from x*(0)
    (order schedule 1, 2, 4, ..., 64, every coefficient in the window, A_0
    factored once) with per-class kernel times and the residual of all
    equations after every step, the error against the exact solution and its
    bound; the same by precision; the evaluation alone by order; the driver
    with its stopping test, to convergence; and 16 steps at n = 512 in double
    double, quad double and octo double, and in plain double (the "D" of
    Tables 7 and 8; the shape of Tables 8 and 9)."""
    from paper_2301_12659_amd import work

    def growth(s):
        """n max_{i,k} |S_i|^k / k!: the systems' inherent loss of accuracy in
        units of the working precision (S_i the partial sums of the alphas,
        the exponents along the monomial chains)."""
        S = np.cumsum(s.xstar[0, :, 1])
        g, term = 1.0, np.ones_like(S)
        for k in range(1, s.D):
            term = term * np.abs(S) / k
            g = max(g, float(term.max()))
        return s.n * g

    def run(s, steps):
        drv = mdn.Newton(s, s.cst, s.start())
        pb, pA, pdx = mdn.step_arrays(drv.plan, drv.ws)
        r = torch.empty((s.L, s.n, s.D), dtype=torch.float64, device="cuda")
        nr = torch.empty(s.D, dtype=torch.float64, device="cuda")
        r0, r1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        mdn.timing_enable(True)
        mdn.timing_read()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        # `steps` steps of the staggered schedule with every coefficient in
        # the window (no early exit), A_0 factored at the first step only,
        # and after every step the residual of all equations (the paper's
        # loop computes it at every step), timed with its own events
        win, hi, res_ms = [], 1, 0.0
        for q in range(steps):
            drv.step_window(0, hi, keep_factorization=q > 0)
            r0.record()
            mdn.linear_residual(s.L, s.n, s.d, pA, pb, pdx, r, norm1=nr)
            r1.record()
            torch.cuda.synchronize()
            res_ms += r0.elapsed_time(r1)
            win.append((0, hi))
            hi = mdn.stagger_next_order(hi, s.D)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        cls = mdn.timing_read()
        mdn.timing_enable(False)
        ms = {k: v[0] for k, v in cls.items()}
        err = _err_vs(mdn, torch, drv.x, torch.as_tensor(s.xstar, device="cuda"))
        bound = TOL[s.L] * growth(s)
        out = {"steps": steps, "factorizations": 1, "wall_s": round(wall, 3),
               "kernel_s": {"convolution": round((ms["convolutions"] + ms["assembly"]) / 1e3, 4),
                            "householder_qr_and_prepass": round(ms["qr"] / 1e3, 4),
                            "qhb_and_back_substitution": round(ms["qhb_bs"] / 1e3, 4),
                            "updates": round((ms["gemm"] + ms["updates"] + ms["x_update"]) / 1e3, 4),
                            "residuals": round(res_ms / 1e3, 4)},
               "windows": [list(w) for w in win],
               "err_vs_exact": err, "growth_estimate": bound, "within_estimate": bool(err <= bound)}
        out["kernel_s"]["total_kernel"] = round(sum(out["kernel_s"].values()), 4)
        return drv, out

    res = {"workload": "x^E = b(t), E the lower triangular matrix of ones (one column) or with the reversed "
                       "triangle as a second column, n = 1024, order 64, exponential solutions, seed 1",
           "paper_table5_v100_s": PAPER_T5_V100, "paper_table6_gflops": PAPER_T6,
           "paper_table7_v100_s": PAPER_T7_V100}
    for cols, name in ((1, "one_column"), (2, "two_columns")):
        s = mdinputs.column_system(1024, 63, 8, cols, seed=1)
        drv, out = run(s, steps)
        print(f"replay {name}: {out['wall_s']} s", file=sys.stderr, flush=True)
        if cols == 1:
            # Table 6: the evaluation alone at order k (window steps with the
            # factorization kept; the convolution class is the evaluation)
            conv = {}
            for order in sorted(PAPER_T6["V100"]):
                times = []
                for rep_ in range(3):
                    mdn.timing_enable(True)
                    mdn.timing_read()
                    drv.step_window(max(order - 1, 0), order, keep_factorization=True)
                    torch.cuda.synchronize()
                    c = mdn.timing_read()
                    mdn.timing_enable(False)
                    times.append(c["convolutions"][0])
                t = min(times) / 1e3
                f = work.convolution_flops(s, order)
                conv[order] = {"s": round(t, 6), "gflops": round(f["flops"] / t / 1e9, 1),
                               "gflops_paper_convention": round(f["paper_flops"] / t / 1e9, 1)}
            out["evaluation_by_order"] = conv
            # the driver with its own stopping test, to convergence
            drv.x.copy_(torch.as_tensor(s.start(), device="cuda"))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rep, win = drv.staggered(max_steps=64)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            err = _err_vs(mdn, torch, drv.x, torch.as_tensor(s.xstar, device="cuda"))
            out["driver_to_convergence"] = {"steps": rep.steps, "converged": bool(rep.converged),
                                            "factorizations": rep.factorizations, "wall_s": round(wall, 3),
                                            "err_vs_exact": err}
        res[name] = out
        del drv
        torch.cuda.empty_cache()
    by_prec = {}
    for L in (1, 2, 4):
        s = mdinputs.column_system(1024, 63, L, 1, seed=1)
        drv, out = run(s, steps)
        print(f"replay one_column L={L}: {out['wall_s']} s", file=sys.stderr, flush=True)
        by_prec[L] = {"wall_s": out["wall_s"], "total_kernel_s": out["kernel_s"]["total_kernel"],
                      "err_vs_exact": out["err_vs_exact"], "growth_estimate": out["growth_estimate"]}
        del drv
        torch.cuda.empty_cache()
    by_prec[8] = {"wall_s": res["one_column"]["wall_s"], "total_kernel_s": res["one_column"]["kernel_s"]["total_kernel"],
                  "err_vs_exact": res["one_column"]["err_vs_exact"], "growth_estimate": res["one_column"]["growth_estimate"]}
    res["one_column_by_precision"] = by_prec
    # Tables 8 and 9: n = 512, order 64, 16 steps, one column, by precision
    n512 = {}
    for L in (1, 2, 4, 8):
        s = mdinputs.column_system(512, 63, L, 1, seed=2)
        drv, out = run(s, 16)
        ks = out["kernel_s"]
        f = work.convolution_flops(s, s.D)
        out["evaluation_gflops_per_full_order_step"] = round(f["flops"] / 1e9, 2)
        n512[L] = out
        print(f"replay n=512 L={L}: {out['wall_s']} s, err {out['err_vs_exact']:.2e} (estimate {out['growth_estimate']:.2e})",
              file=sys.stderr, flush=True)
        del drv
        torch.cuda.empty_cache()
    res["n512_one_column_16_steps"] = n512
    res["paper_table8_rtx2080_16_steps_s"] = PAPER_T8_RTX2080
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=60)
    ap.add_argument("--warmup", type=int, default=6)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--batch-paths", type=int, default=2048,
                    help="paths of the batched workload (0 skips it)")
    ap.add_argument("--batch-steps", type=int, default=4)
    ap.add_argument("--config-reps", type=int, default=5,
                    help="timed runs of the small dd, large od and adjoint configurations (0: skip)")
    ap.add_argument("--stagger-repeats", type=int, default=3,
                    help="timed runs of each staggered time-to-solution measurement (0: skip)")
    ap.add_argument("--replay", action="store_true",
                    help="only run the paper's own workloads (n = 1024 column systems) and print their JSON line")
    ap.add_argument("--replay-steps", type=int, default=24)
    ap.add_argument("--headline-only", action="store_true",
                    help="only the timed medium quad-double steps and their kernel classes (for profilers)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 256 MiB device-to-device copy (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch

        # an elementwise kernel that reads 256 MiB and writes 256 MiB
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "copy", "bytes_read": src.numel() * 8, "bytes_written": dst.numel() * 8,
                          "launches": 3, "evaldiff_source_sha256": evaldiff_source_sha256()}))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "independent paths would be split across GPUs without communication, which this build does not do.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import mdinputs
    import paper_2301_12659_amd as mdn
    from paper_2301_12659_amd import work

    torch.cuda.set_device(0)
    if args.replay:
        print(json.dumps({"replay": _replay(mdn, torch, np, mdinputs, args.replay_steps)}))
        return
    sysm = mdinputs.medium_qd()
    L, n, D = sysm.L, sysm.n, sysm.D
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")

    # manufactured right-hand side on the GPU: c_{i,0} = -P_i(x*) (eval at x* with zero constant)
    drv = mdn.Newton(sysm, np.zeros((L, n, D)), sysm.xstar)
    b = torch.empty((L, n, D), dtype=torch.float64, device="cuda")
    A = torch.empty((L, n, n, D), dtype=torch.float64, device="cuda")
    mdn.eval_diff(drv.plan, drv.cff, drv.cst, drv.x, b, A, drv.ws)
    drv.cst.copy_(b)
    drv.x.copy_(dev(sysm.start()))
    xstar = dev(sysm.xstar)
    del A
    torch.cuda.synchronize()

    for _ in range(args.warmup):
        drv.step()
    drv.steps(args.warmup)
    torch.cuda.synchronize()

    # timed region 1: K steps by md_newton_steps (each step's factorization
    # beside the previous step; the same iterates as K md_newton_step calls)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()
    drv.steps(args.steps)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = e0.elapsed_time(e1) / args.steps
    status = drv.status_code()
    err_manufactured = _err_vs(mdn, torch, drv.x, xstar)

    # the same number of single md_newton_step calls (QR on the critical path)
    e0.record()
    for _ in range(args.steps):
        drv.step()
    e1.record()
    torch.cuda.synchronize()
    ms_single = e0.elapsed_time(e1) / args.steps

    # timed region 2: the same steps with per-kernel-class HIP events
    mdn.timing_enable(True)
    mdn.timing_read()
    drv.steps(args.steps)
    torch.cuda.synchronize()
    classes = mdn.timing_read()
    mdn.timing_enable(False)

    w = work.step_work(sysm)
    breakdown = {}
    for cls, (ms, cnt) in classes.items():
        per_step = ms / args.steps
        fl = w[cls]["flops"] if cls in w else 0
        breakdown[cls] = {"ms_per_step": round(per_step, 4), "brackets_per_step": round(cnt / args.steps, 2),
                          "tflops": round(fl / (per_step * 1e-3) / 1e12, 3) if per_step > 0 else None}
    # the dominant kernel is the evaluation/differentiation (class
    # "convolutions", one evaldiff launch per step on the caller's stream):
    # it carries most of the arithmetic and, with the factorization beside
    # the previous step, it is on the critical path
    dom = "convolutions"
    dom_ms = classes[dom][0] / max(classes[dom][1], 1)
    achieved = w[dom]["flops"] / (dom_ms * 1e-3) / 1e12
    total_flops = sum(v["flops"] for v in w.values())
    qr_b = work.qr_latency_bound(L, n)
    st_b = work.stages_latency_bound(L, n, D)
    qr_ms = (classes["qr"][0] + classes["qhb_bs"][0]) / args.steps
    st_ms = classes["updates"][0] / args.steps
    latency = {
        "model": "dependent FP64 instructions on the chain x %.1f cycles at %.1f GHz + %.1f us per hand-over"
                 % (work.CYCLES_PER_DEP_INSTR, work.CLOCK_HZ / 1e9, work.HANDOVER_S * 1e6),
        "qr_and_m": {"bound_ms": round(qr_b["seconds"] * 1e3, 4), "chain_instr_per_column": qr_b["chain_instr_per_column"],
                     "measured_ms": round(qr_ms, 4), "frac": round(qr_b["seconds"] * 1e3 / qr_ms, 3)},
        "staged_solve": {"bound_ms": round(st_b["seconds"] * 1e3, 4), "chain_instr_per_stage": st_b["chain_instr_per_stage"],
                         "measured_ms": round(st_ms, 4), "frac": round(st_b["seconds"] * 1e3 / st_ms, 3)},
    }
    sq = _recorded_sq()
    conventions = {"useful_tflops": round(achieved, 3), "useful_frac": round(achieved / PEAK_FP64_TFLOPS, 4)}
    if sq:
        ex = 64.0 * (sq["add_f64"] + sq["mul_f64"] + sq.get("trans_f64", 0.0) + 2.0 * sq["fma_f64"])
        lane_ops = 64.0 * (sq["add_f64"] + sq["mul_f64"] + sq.get("trans_f64", 0.0) + sq["fma_f64"])
        t = dom_ms * 1e-3
        conventions.update({
            "executed_tflops": round(ex / t / 1e12, 3), "executed_frac": round(ex / t / 1e12 / PEAK_FP64_TFLOPS, 4),
            "fp64_pipe_utilization": round(lane_ops / (64.0 * 256 * 2.4e9 * t), 4),
            "counters": "profiles/evaldiff_pair_kernel_medium_qd_sq_counters.md (same kernel sources)"})
    else:
        conventions.update({"executed_tflops": None, "fp64_pipe_utilization": None,
                            "counters": "no SQ counters recorded for the current kernel sources"})

    out = {
        "metric": "Newton steps/s and FP64 GFLOPS (% FP64 vector peak) at n=64,d=63 qd; err vs oracle",
        "value": round(1000.0 / ms_step, 3),
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "medium_qd: n=64, d=63 (D=64), quad double, 64 x (32 + 1 boost) monomials, "
                               "2..6 variables, exponents {1,2}, manufactured solution, seed 2",
                   "n": n, "d": sysm.d, "precision": "qd", "monomials": sysm.m, "support_entries": sysm.nnz},
        "steps_entry_point": "md_newton_steps (each step's QR beside the previous step; iterates identical to "
                             "md_newton_step calls)",
        "single_step_ms": round(ms_single, 4),
        "single_step_per_s": round(1000.0 / ms_single, 3),
        "gflops_step": round(total_flops / (ms_step * 1e-3) / 1e9, 2),
        "pct_fp64_peak_step": round(100 * total_flops / (ms_step * 1e-3) / (PEAK_FP64_TFLOPS * 1e12), 2),
        "roofline": {"bound": "alu", "kernel": "evaldiff_pair_kernel<4> (" + dom + ", two wavefronts per monomial)", "achieved": round(achieved, 3), "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64_TFLOPS, 4), "traffic": _recorded_traffic(),
                     "flops_per_launch": w[dom]["flops"], "launch_ms": round(dom_ms, 4)},
        "evaldiff_conventions": conventions,
        "latency_roofline": latency,
        "kernel_classes": breakdown,
        "paper_convention_conv_gflops": round(work.paper_convention_flops(sysm) /
                                              (classes["convolutions"][0] / max(classes["convolutions"][1], 1) * 1e-3) / 1e9, 1),
        "status": status,
        "err_vs_manufactured": err_manufactured,
        "wall_s_timed": round(wall, 3),
    }

    if args.headline_only:
        print(json.dumps(out))
        return

    # the linear residual of the last step's system (monitoring): every
    # equation, and one sampled equation
    res_t = {}
    pb, pA, pdx = mdn.step_arrays(drv.plan, drv.ws)
    for name, rows in (("all_rows", None), ("one_row", [n // 2])):
        rws = None if rows is None else torch.tensor(rows, dtype=torch.int32, device="cuda")
        rr = torch.empty((L, n if rows is None else len(rows), D), dtype=torch.float64, device="cuda")
        nr = torch.empty(D, dtype=torch.float64, device="cuda")
        call = lambda: mdn.linear_residual(L, n, D - 1, pA, pb, pdx, rr, rows=rws, norm1=nr)
        call()
        torch.cuda.synchronize()
        r0, r1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        r0.record()
        for _ in range(20):
            call()
        r1.record()
        torch.cuda.synchronize()
        res_t[name + "_us"] = round(1000.0 * r0.elapsed_time(r1) / 20, 2)
    out["residual"] = res_t

    out["complex"] = _bench_complex(mdn, torch, np, mdinputs, sysm)

    out["mixed"] = _bench_mixed(mdn, torch, np, drv, dev(sysm.start()), xstar)

    if args.config_reps > 0:
        out["configs"] = _bench_configs(mdn, torch, np, mdinputs, args.config_reps)

    if args.stagger_repeats > 0:
        out["staggered"] = _bench_staggered(mdn, torch, np, sysm, drv.cst, xstar, args.stagger_repeats)

    if args.batch_paths > 0:
        out["batched"] = _bench_batch(mdn, torch, np, mdinputs, args.batch_paths, args.batch_steps)

    if not args.no_cpu_baseline:
        import oracle

        cst_o = oracle.manufacture(sysm)
        d2 = mdn.Newton(sysm, cst_o)
        for _ in range(sysm.steps - 1):
            d2.step()
        torch.cuda.synchronize()
        x_in = d2.x.cpu().numpy()
        d2.step()
        x_gpu = d2.x.cpu().numpy()
        t0 = time.perf_counter()
        nsteps = 0
        ref = None
        while True:
            ref = oracle.newton_step(sysm, sysm.cff, cst_o, x_in)["x"]
            nsteps += 1
            el = time.perf_counter() - t0
            if el >= args.cpu_seconds or nsteps >= 20:
                break
        diff = oracle.absdiff(x_gpu, ref).max(axis=-1)
        scale = np.maximum(np.abs(x_in[0]).max(axis=-1), np.abs(ref[0]).max(axis=-1))
        out["err_vs_oracle"] = float((diff / scale).max())
        out["cpu_baseline"] = {"value": round(nsteps / el, 4), "unit": "steps/s", "cores": oracle.threads(),
                               "kind": "oracle",
                               "sample": f"{nsteps} full oracle Newton steps (MPFR, 848 bits: eval/diff by the "
                                         f"product rule, LU, block forward substitution) on the same system from the "
                                         f"GPU's 5th iterate, {el:.1f} s"}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
