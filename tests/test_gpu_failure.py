"""Failure paths of the C ABI on the GPU, forced from the host: iteration
caps small enough to be hit (every kernel still runs its bounded loop to the
end and exits), a workspace cap below what a solve needs, and a repeat solve
on the same handle after each."""

import numpy as np
import pytest

from paper_2508_11467_amd import _lib, inputs

pytestmark = pytest.mark.gpu


def _solve(s, d, e):
    import torch
    sig, U, VT = s.svd(torch.from_numpy(d), torch.from_numpy(e))
    torch.cuda.synchronize()
    info, stats = s.info()
    return sig.cpu().numpy(), info, stats


def test_secular_iteration_cap_reported(gpu):
    """Two evaluations per root (the midpoint and one model step) are too few
    for most roots of a random merge: info counts the capped roots."""
    from paper_2508_11467_amd.api import Solver
    d, e = inputs.uniform(512, 41)
    s = Solver(0, max_secular_iters=2)
    try:
        sig, info, st = _solve(s, d, e)
        print("secular cap 2: info", info, "roots", st["roots"], flush=True)
        assert info > 0
        assert np.all(np.isfinite(sig))
    finally:
        s.close()
    ok = Solver(0)
    try:
        _, info, _ = _solve(ok, d, e)
        assert info == 0
    finally:
        ok.close()


def test_leaf_sweep_cap_reported(gpu):
    """One QR sweep per leaf row is fewer than a random 32-row leaf needs:
    info counts the leaves that stopped at the cap."""
    from paper_2508_11467_amd.api import Solver
    d, e = inputs.uniform(1024, 42)
    s = Solver(0, max_leaf_sweeps=1)
    try:
        sig, info, _ = _solve(s, d, e)
        print("leaf cap 1: info", info, flush=True)
        assert info > 0
        assert np.all(np.isfinite(sig))
    finally:
        s.close()


def test_workspace_cap_gives_nomem(gpu):
    import torch
    from paper_2508_11467_amd.api import Solver
    d, e = inputs.uniform(300, 43)
    s = Solver(0, workspace_cap_bytes=1 << 16)
    try:
        with pytest.raises(_lib.BdcError) as ex:
            s.svd(torch.from_numpy(d), torch.from_numpy(e))
        assert ex.value.code == _lib.BDC_ERR_NOMEM
        # a size whose workspace fits under the cap still solves
        d1, e1 = inputs.uniform(8, 44)
        sig, info, _ = _solve(s, d1, e1)
        assert info == 0
        B = np.diag(d1) + np.diag(e1, 1)
        assert np.max(np.abs(sig - np.linalg.svd(B, compute_uv=False))) <= 1e-14
    finally:
        s.close()
