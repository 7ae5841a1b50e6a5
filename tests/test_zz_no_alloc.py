"""md_qr_noalloc, the QR entry point that allocates nothing (its scratch is a
static device array), against md_qr with a workspace: the same factors bit for
bit, on two calls in a row with the second one smaller, and within the
tolerance of the precision against the oracle's QR checks."""
from __future__ import annotations

import numpy as np
import pytest

import mdinputs
import oracle
from gpu_helpers import TOL, dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mdn():
    import torch

    assert torch.cuda.is_available()
    import paper_2301_12659_amd as mdn

    return mdn


def _matrix(L, n, seed):
    rng = np.random.default_rng(seed)
    A0 = mdinputs.random_md(rng, L, (n, n), -1.0, 1.0)
    A0[0] += np.diag(np.full(n, 2.0))
    return A0


def _factor(mdn, fn, L, n, A0):
    import torch

    a = dev(A0)
    tau = torch.zeros((L, n), dtype=torch.float64, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")  # md_qr writes it only on a failure
    fn(L, n, a, tau, status)
    torch.cuda.synchronize()
    return host(a), host(tau), int(status.item())


@pytest.mark.parametrize("L,sizes", [(4, (64, 33)), (8, (100, 19)), (2, (200, 8))])
def test_noalloc_matches_workspace_qr(mdn, L, sizes):
    for k, n in enumerate(sizes):
        A0 = _matrix(L, n, 1000 * L + n)
        print(f"md_qr_noalloc L={L} n={n} call {k + 1}", flush=True)
        ra, rt, rs = _factor(mdn, mdn.qr, L, n, A0)
        ga, gt, gs = _factor(mdn, mdn.qr_noalloc, L, n, A0)
        assert rs == 0 and gs == 0, (rs, gs)
        assert np.array_equal(ga, ra) and np.array_equal(gt, rt), "md_qr_noalloc differs from md_qr"
        res, orth = oracle.qr_check(A0, ga, gt)
        assert res <= TOL[L] and orth <= TOL[L], (res, orth)


def test_noalloc_refuses_beyond_static_scratch(mdn):
    import torch

    L, n = 8, 257  # the octo-double board of n = 257 exceeds the static array
    a = torch.zeros((L, n, n), dtype=torch.float64, device="cuda")
    tau = torch.zeros((L, n), dtype=torch.float64, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    with pytest.raises(mdn.MdError) as ex:
        mdn.qr_noalloc(L, n, a, tau, status)
    assert ex.value.code == mdn.MD_ENOSPACE
    assert "static" in str(ex.value)
