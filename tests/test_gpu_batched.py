"""Batched solves of uneven sizes against single solves and the oracle."""

import numpy as np
import pytest

import oracle
from paper_2508_11467_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def solver(gpu):
    from paper_2508_11467_amd.api import Solver
    s = Solver(0)
    yield s
    s.close()


def unpack(sizes, sig, U, VT):
    out = []
    off = mo = 0
    for n in sizes:
        s = sig[off:off + n]
        u = U[mo:mo + n * n].reshape(n, n).T
        v = VT[mo:mo + n * n].reshape(n, n).T
        out.append((s, u, v))
        off += n
        mo += n * n
    return out


def test_batched_matches_single_solves(solver):
    import torch
    sizes = [1, 2, 33, 5, 0, 64, 200, 31, 300, 65, 7, 129]
    d, e = inputs.batch_uniform(sizes, 77)
    sig, U, VT = solver.svd_batched(sizes, torch.from_numpy(d), torch.from_numpy(e))
    info, st = solver.info()
    assert info == 0
    res = unpack(sizes, sig.cpu().numpy(), U.cpu().numpy(), VT.cpu().numpy())
    off = 0
    for n, (s, u, v) in zip(sizes, res):
        dd = d[off:off + n]
        ee = e[off:off + max(n - 1, 0)]
        off += n
        if n == 0:
            continue
        s1, u1, v1 = solver.svd(torch.from_numpy(dd.copy()), torch.from_numpy(ee.copy()))
        assert np.array_equal(s, s1.cpu().numpy())
        assert np.array_equal(u, u1.cpu().numpy()) and np.array_equal(v, v1.cpu().numpy())
        ref, _, _ = oracle.bdsdc(dd, ee)
        B = oracle.dense(dd, ee)
        assert np.max(np.abs(s - ref)) <= 1e-13 * max(ref[0], 1e-300)
        assert np.linalg.norm(B - (u * s) @ v) <= 1e-12 * max(np.linalg.norm(B), 1e-300)
        assert np.max(np.abs(u.T @ u - np.eye(n))) <= 1e-12
        assert np.max(np.abs(v @ v.T - np.eye(n))) <= 1e-12


def test_batched_config_2000(solver):
    """2000 problems, sizes log-uniform in [32, 2048]: every problem's
    residual and orthogonality on the GPU, and a sample against the oracle."""
    import torch
    sizes = inputs.batch_sizes(2000, 32, 2048, inputs.seed_for(4, 0)).tolist()
    d, e = inputs.batch_uniform(sizes, inputs.seed_for(4, 1))
    dt = torch.from_numpy(d).cuda()
    et = torch.from_numpy(e).cuda()
    sig, U, VT = solver.svd_batched(sizes, dt, et)
    info, st = solver.info()
    assert info == 0
    off = mo = 0
    worst_res = worst_orth = 0.0
    rng = np.random.default_rng(5)
    sample = set(rng.choice(len(sizes), 4, replace=False).tolist())
    for p, n in enumerate(sizes):
        s = sig[off:off + n]
        u = U[mo:mo + n * n].view(n, n).T
        v = VT[mo:mo + n * n].view(n, n).T.contiguous()
        dd = dt[off:off + n]
        ee = et[off:off + n]
        # B V^T^T = U S, row by row: (B V)[i] = d_i V[i] + e_i V[i+1]
        V = v.T
        BV = dd[:, None] * V
        BV[:-1] += ee[:n - 1, None] * V[1:]
        nb = torch.sqrt(torch.sum(dd * dd) + torch.sum(ee[:n - 1] ** 2))
        res = float(torch.linalg.norm(BV - u * s[None, :]) / nb)
        I = torch.eye(n, dtype=torch.float64, device="cuda")
        uc = u.contiguous()
        orth = max(float(torch.max(torch.abs(uc.T.contiguous() @ uc - I))),
                   float(torch.max(torch.abs(v @ v.T.contiguous() - I))))
        worst_res = max(worst_res, res)
        worst_orth = max(worst_orth, orth)
        if p in sample:
            ref, _, _ = oracle.bdsdc(d[off:off + n], e[off:off + n - 1])
            assert np.max(np.abs(s.cpu().numpy() - ref)) <= 1e-13 * ref[0]
        off += n
        mo += n * n
    assert worst_res <= 1e-12 and worst_orth <= 1e-12
