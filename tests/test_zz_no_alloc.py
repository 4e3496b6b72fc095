"""The allocation-free back-transformation entry point against the one that
allocates its scratch: the same arguments give the same C bit for bit, on two
calls in a row (the second smaller, so it runs over the fixed scratch the
first one left behind), and a problem beyond the fixed scratch is refused on
the host."""

import numpy as np
import pytest
import scipy.linalg.lapack as lapack

pytestmark = pytest.mark.gpu


def _case(m, p, k, seed, rows):
    g = np.random.default_rng(seed)
    A = g.standard_normal((m, k))
    qr, tau, _, info = lapack.dgeqrf(A)
    assert info == 0
    Y = np.tril(qr, -1)
    if rows:  # the same reflectors stored by rows (gebrd's row-reflector layout)
        Y = np.ascontiguousarray(Y.T)
    C = g.standard_normal((m, p))
    return Y, tau, C


def _run(solver, Y, tau, C, trans, offset, rows, block, noalloc):
    import torch
    Yd = torch.from_numpy(Y).cuda()
    td = torch.from_numpy(np.ascontiguousarray(tau)).cuda()
    Cd = torch.from_numpy(np.ascontiguousarray(C.T)).cuda().T
    solver.apply_reflectors(Yd, td, Cd, trans=trans, offset=offset, rows=rows, block=block, noalloc=noalloc)
    torch.cuda.synchronize()
    return Cd.cpu().numpy()


def test_noalloc_matches_allocating_entry_point(gpu):
    from paper_2508_11467_amd.api import Solver
    s = Solver(0)
    try:
        # first call: more columns than one 512-column panel, blocks of 64;
        # second call: smaller, row-stored reflectors with offset 1, Q^T C
        for (m, p, k, seed, trans, offset, rows, block) in ((3000, 2600, 1500, 1, False, 0, False, 0),
                                                            (700, 300, 500, 2, True, 1, True, 32)):
            Y, tau, C = _case(m, p, k, seed, rows)
            print(f"noalloc m={m} p={p} k={k} trans={trans} offset={offset} rows={rows} block={block}", flush=True)
            ref = _run(s, Y, tau, C, trans, offset, rows, block, noalloc=False)
            out = _run(s, Y, tau, C, trans, offset, rows, block, noalloc=True)
            assert np.array_equal(out, ref), float(np.max(np.abs(out - ref)))
            assert not np.array_equal(out, C)
    finally:
        s.close()


def test_noalloc_refuses_problems_beyond_its_scratch(gpu):
    import torch

    from paper_2508_11467_amd import _lib
    from paper_2508_11467_amd.api import Solver
    s = Solver(0)
    try:
        m, p, k = 70000, 8, 64  # 8 (70000 * 64 + 64^2 + 33 * 64 * 64) + 1024 bytes > 32 MiB
        Y = torch.zeros((m, k), dtype=torch.float64, device="cuda")
        tau = torch.zeros(k, dtype=torch.float64, device="cuda")
        C = torch.zeros((p, m), dtype=torch.float64, device="cuda").T
        with pytest.raises(_lib.BdcError) as err:
            s.apply_reflectors(Y, tau, C, noalloc=True)
        assert err.value.code == _lib.BDC_ERR_TOO_LARGE
        # the allocating entry point takes the same problem
        s.apply_reflectors(Y, tau, C)
        torch.cuda.synchronize()
        assert torch.count_nonzero(C).item() == 0
    finally:
        s.close()
