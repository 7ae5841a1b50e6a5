"""Batched Newton steps (GPU): paths of uneven size in one persistent launch
against their solo steps (md_newton_step, md_newton_step_mixed) and the
oracle, graph replays, the autotuner and the host checks."""
from __future__ import annotations

import numpy as np
import pytest

import mdinputs
import oracle
from gpu_helpers import TOL, coef_err, dev, host, series_err, step_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mdn():
    import paper_2301_12659_amd as mdn

    return mdn


def _setup(mdn, paths):
    import torch

    csts = [oracle.manufacture(s) for s in paths]
    b = mdn.Batch(paths)
    P = len(paths)
    cff = dev(b.pack_cff([s.cff for s in paths]))
    cst = dev(b.pack_series(csts))
    x = dev(b.pack_series([s.start() for s in paths]))
    status = torch.zeros(P, dtype=torch.int32, device="cuda")
    norms = torch.zeros(2 * P, dtype=torch.float64, device="cuda")
    ws = mdn.workspace(b.workspace_bytes())
    return b, csts, cff, cst, x, status, norms, ws


@pytest.fixture(scope="module")
def qd_paths():
    return mdinputs.small_batch(4, seed=9)


def test_batch_step_matches_solo_and_oracle(mdn, qd_paths):
    import torch

    paths = qd_paths
    b, csts, cff, cst, x, status, norms, ws = _setup(mdn, paths)
    b.step(cff, cst, x, status, norms, ws)
    torch.cuda.synchronize()
    assert host(status).tolist() == [0] * len(paths)
    got = b.unpack_series(host(x))
    for p, s in enumerate(paths):
        solo = mdn.Newton(s, csts[p])
        solo.step()
        assert step_err(got[p], host(solo.x), s.start()) <= TOL[4], (p, s.n, s.d)
    p = max(range(len(paths)), key=lambda q: paths[q].n * paths[q].D)
    ref = oracle.newton_step(paths[p], paths[p].cff, csts[p], paths[p].start())["x"]
    assert step_err(got[p], ref, paths[p].start()) <= TOL[4]
    nb = host(norms).reshape(-1, 2)
    assert np.all(np.isfinite(nb)) and np.all(nb[:, 1] > 0)


def test_batch_converges_to_manufactured(mdn, qd_paths):
    import torch

    paths = qd_paths
    b, csts, cff, cst, x, status, norms, ws = _setup(mdn, paths)
    for _ in range(7):
        b.step(cff, cst, x, status, norms, ws)
    torch.cuda.synchronize()
    assert host(status).tolist() == [0] * len(paths)
    got = b.unpack_series(host(x))
    for p, s in enumerate(paths):
        assert series_err(got[p], s.xstar) <= TOL[4], (p, s.n, s.d)


def test_batch_mixed_precision(mdn, qd_paths):
    """qd residual, dd solve: one step equals the solo mixed step; repeated
    steps reach the manufactured solutions."""
    import torch

    paths = qd_paths
    b, csts, cff, cst, x, status, norms, ws = _setup(mdn, paths)
    b.step(cff, cst, x, status, norms, ws, prec_solve=2)
    torch.cuda.synchronize()
    got = b.unpack_series(host(x))
    for p, s in enumerate(paths):
        solo = mdn.Newton(s, csts[p])
        solo.step(prec_solve=2)
        assert step_err(got[p], host(solo.x), s.start()) <= TOL[2], (p, s.n, s.d)
    for _ in range(9):
        b.step(cff, cst, x, status, norms, ws, prec_solve=2)
    torch.cuda.synchronize()
    got = b.unpack_series(host(x))
    for p, s in enumerate(paths):
        assert series_err(got[p], s.xstar) <= TOL[4], (p, s.n, s.d)


def test_batch_double_double(mdn):
    import torch

    paths = mdinputs.small_batch(2, seed=4)
    b, csts, cff, cst, x, status, norms, ws = _setup(mdn, paths)
    b.step(cff, cst, x, status, norms, ws)
    torch.cuda.synchronize()
    got = b.unpack_series(host(x))
    for p, s in enumerate(paths):
        solo = mdn.Newton(s, csts[p])
        solo.step()
        assert step_err(got[p], host(solo.x), s.start()) <= TOL[2], (p, s.n, s.d)


def test_batch_graph_replays_match_eager(mdn, qd_paths):
    """The step is captured in a graph on the second call with the same
    arguments and replayed after: every call from the same input gives the
    eager result bit for bit, with eager work and synchronizations between."""
    import torch

    paths = qd_paths
    b, csts, cff, cst, x, status, norms, ws = _setup(mdn, paths)
    x0 = x.clone()
    results = []
    for rep in range(5):
        x.copy_(x0)
        b.step(cff, cst, x, status, norms, ws)
        torch.cuda.synchronize()
        results.append(host(x).copy())
        _ = (x0 * 2.0).sum().item()  # eager work between replays
    for r in results[1:]:
        assert np.array_equal(r, results[0])


def test_batch_autotune_keeps_results(mdn, qd_paths):
    import torch

    paths = qd_paths
    b, csts, cff, cst, x, status, norms, ws = _setup(mdn, paths)
    xs = torch.empty_like(x)
    chosen = b.autotune(cff, cst, x, xs, status, norms, ws)
    assert len(chosen) == 9 and all(t in (4, 8, 16) for t in chosen)
    x0 = host(x).copy()
    b.step(cff, cst, x, status, norms, ws)
    torch.cuda.synchronize()
    got = b.unpack_series(host(x))
    starts = b.unpack_series(x0)
    for p, s in enumerate(paths):
        solo = mdn.Newton(s, csts[p])
        solo.step()
        assert step_err(got[p], host(solo.x), starts[p]) <= TOL[4]
    for t in (4, 16):
        b.set_tiles([t] * 9)
        xx = dev(x0)
        b.step(cff, cst, xx, status, norms, ws)
        torch.cuda.synchronize()
        assert step_err(host(xx), host(x), x0) <= TOL[4]


def test_batch_rejects_bad_paths(mdn):
    s = mdinputs.tiny(4, 5, 3, mons=2, kmin=1, kmax=2, exps=(3,), seed=1)
    with pytest.raises(mdn.MdError):
        mdn.Batch([s])
    big = mdinputs.tiny(4, 130, 1, mons=1, kmin=1, kmax=1, exps=(1,), seed=2, cond_max=None)
    with pytest.raises(mdn.MdError):
        mdn.Batch([big])


@pytest.fixture(scope="module")
def bucket_paths():
    return mdinputs.bucket_paths(4)


@pytest.mark.parametrize("tiles", [4, 16])
@pytest.mark.parametrize("prec_solve", [4, 2])
def test_batch_every_size_class(mdn, bucket_paths, tiles, prec_solve):
    """One path in each (n, D) class of the batched workload (n 20, 48, 90 with
    D 16, 32, 64): the batched step with reduction teams of ``tiles`` lanes
    equals each path's solo step (md_newton_step, or md_newton_step_mixed for
    the quad-double residual with a double-double solve) within the solve
    precision's tolerance, normwise and per coefficient; the largest path
    also against the oracle step (plain quad double)."""
    import torch

    paths = bucket_paths
    b, csts, cff, cst, x, status, norms, ws = _setup(mdn, paths)
    b.set_tiles([tiles] * 9)
    b.step(cff, cst, x, status, norms, ws, prec_solve=prec_solve)
    torch.cuda.synchronize()
    assert host(status).tolist() == [0] * len(paths)
    got = b.unpack_series(host(x))
    tol = TOL[prec_solve]
    for p, s in enumerate(paths):
        solo = mdn.Newton(s, csts[p])
        solo.step(prec_solve=prec_solve)
        sx = host(solo.x)
        assert step_err(got[p], sx, s.start()) <= tol, (p, s.n, s.d)
        assert coef_err(got[p], sx, s.start()) <= tol, (p, s.n, s.d)
    if prec_solve == 4:
        p = max(range(len(paths)), key=lambda q: paths[q].n * paths[q].D)
        s = paths[p]
        ref = oracle.newton_step(s, s.cff, csts[p], s.start())["x"]
        assert step_err(got[p], ref, s.start()) <= TOL[4]
        assert coef_err(got[p], ref, s.start()) <= TOL[4]


def test_batch_every_size_class_converges(mdn, bucket_paths):
    """Steps of the whole batch reach every path's manufactured solution
    (plain quad double, then the quad-double residual with a double-double
    solve from the start again)."""
    import torch

    paths = bucket_paths
    for prec_solve, steps in ((4, 7), (2, 10)):
        b, csts, cff, cst, x, status, norms, ws = _setup(mdn, paths)
        for _ in range(steps):
            b.step(cff, cst, x, status, norms, ws, prec_solve=prec_solve)
        torch.cuda.synchronize()
        assert host(status).tolist() == [0] * len(paths)
        got = b.unpack_series(host(x))
        for p, s in enumerate(paths):
            assert series_err(got[p], s.xstar) <= TOL[4], (prec_solve, p, s.n, s.d)
