"""Back-transformation of singular vectors (Section 4.3.3) on the GPU against
the oracle's reflector-by-reflector product, and the dense SVD it completes:
A = Q [B; 0] P^T (the oracle's Householder reduction, on the CPU), B's SVD
by the GPU divide and conquer, then U = Q [U_2; 0] and V = P V_2 by the GPU
back-transformation."""

import numpy as np
import pytest
import scipy.linalg.lapack as lapack

from oracle import householder as hh

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def solver(gpu):
    from paper_2508_11467_amd.api import Solver
    s = Solver(0)
    yield s
    s.close()


def _colmajor(C):
    """A (m, p) view of column-major device memory holding C."""
    import torch
    return torch.from_numpy(np.ascontiguousarray(C.T)).cuda().T


def _gpu_apply(solver, Ypacked, tau, C, trans, offset, rows=False, block=0):
    import torch
    Y = torch.from_numpy(np.ascontiguousarray(Ypacked.T if rows else Ypacked)).cuda()
    t = torch.from_numpy(np.ascontiguousarray(tau)).cuda()
    Cd = _colmajor(C)
    solver.apply_reflectors(Y, t, Cd, trans=trans, offset=offset, rows=rows, block=block)
    return Cd.cpu().numpy()


@pytest.mark.parametrize("trans", [False, True])
@pytest.mark.parametrize("m,p,k,block", [(300, 200, 150, 0), (129, 65, 129, 64), (200, 333, 64, 17),
                                         (64, 1, 10, 0), (1, 5, 1, 0), (500, 70, 300, 32)])
def test_apply_reflectors_matches_oracle(solver, trans, m, p, k, block):
    """Reflectors of a QR factorisation (LAPACK's geqrf on a seeded matrix),
    applied to a seeded C: elementwise against the oracle."""
    g = np.random.default_rng(m * 7 + p + k)
    A = g.standard_normal((m, k))
    qr, tau, _, info = lapack.dgeqrf(A)
    assert info == 0
    Yfull = np.tril(qr, -1) + np.eye(m, k)
    C = g.standard_normal((m, p))
    ref = hh.apply_q(Yfull, tau, C, trans=trans)
    out = _gpu_apply(solver, np.tril(qr, -1), tau, C, trans, 0, block=block)
    err = np.max(np.abs(out - ref))
    assert err <= 1e-13 * max(1.0, np.max(np.abs(C))) * np.sqrt(m), err


def test_apply_reflectors_identity_and_offset(solver):
    """tau = 0 reflectors act as identities; offset-1 row-stored reflectors
    (the layout of a bidiagonal reduction's row reflectors)."""
    g = np.random.default_rng(3)
    n = 90
    d, e, Yq, tq, Yp, tp = hh.bidiagonalize(g.standard_normal((n + 10, n)))
    tp = tp.copy()
    tp[[5, 40]] = 0.0
    Yfull = Yp.copy()
    Yfull[:, [5, 40]] = 0.0
    C = g.standard_normal((n, 37))
    for trans in (False, True):
        ref = hh.apply_q(Yfull, tp, C, trans=trans)
        packed = hh.pack_lapack(Yp, 1)
        out_c = _gpu_apply(solver, packed, tp, C, trans, 1)
        out_r = _gpu_apply(solver, packed, tp, C, trans, 1, rows=True)
        assert np.max(np.abs(out_c - ref)) <= 1e-13 * np.sqrt(n)
        assert np.array_equal(out_c, out_r)


@pytest.mark.parametrize("m,n", [(384, 384), (700, 256)])
def test_dense_svd_through_back_transformation(solver, m, n):
    """A = U Sigma V^T for a dense A: the paper's E_svd and the singular
    values against LAPACK's SVD of A."""
    import torch
    g = np.random.default_rng(m + n)
    A = g.standard_normal((m, n))
    d, e, Yq, tq, Yp, tp = hh.bidiagonalize(A)
    sig, U2, VT2 = solver.svd(torch.from_numpy(d), torch.from_numpy(e))
    U2 = U2.cpu().numpy()
    V2 = VT2.cpu().numpy().T
    Ufull = np.zeros((m, n))
    Ufull[:n] = U2
    U = _gpu_apply(solver, hh.pack_lapack(Yq, 0), tq, Ufull, False, 0)
    V = _gpu_apply(solver, hh.pack_lapack(Yp, 1), tp, V2, False, 1)
    s = sig.cpu().numpy()
    e_svd = np.linalg.norm(A - (U * s) @ V.T) / np.linalg.norm(A)
    ref = np.linalg.svd(A, compute_uv=False)
    e_sigma = np.linalg.norm(s - ref) / n
    print(f"dense {m}x{n}: E_svd {e_svd:.2e} E_sigma {e_sigma:.2e}", flush=True)
    assert e_svd <= 1e-12
    assert np.max(np.abs(s - ref)) <= 1e-13 * ref[0]
    assert np.max(np.abs(U.T @ U - np.eye(n))) <= 1e-12
    assert np.max(np.abs(V.T @ V - np.eye(n))) <= 1e-12
    # U against the oracle's product on the same U_2
    assert np.max(np.abs(U - hh.apply_q(Yq, tq, Ufull))) <= 1e-13 * np.sqrt(m)


def test_apply_reflectors_full_size_sampled(solver):
    """n = 16384: 16384 seeded reflectors (LAPACK storage, tau = 2 / y^T y)
    applied to a 16384 x 16384 matrix; 6 columns against the oracle, which
    applies the reflectors to those columns alone."""
    import torch
    n = 16384
    gen = torch.Generator(device="cuda")
    gen.manual_seed(11)
    Y = torch.randn((n, n), dtype=torch.float64, device="cuda", generator=gen) * 0.01
    Y = torch.tril(Y, -1)
    norms = 1.0 + torch.sum(Y * Y, dim=0)
    tau = 2.0 / norms
    C = torch.randn((n, n), dtype=torch.float64, device="cuda", generator=gen)
    cols = [0, 1, 4097, 9999, 16382, 16383]
    C0 = C[:, cols].cpu().numpy()
    Cd = C.T.contiguous().T  # column-major copy
    del C
    solver.apply_reflectors(Y, tau, Cd, trans=False)
    out = Cd[:, cols].cpu().numpy()
    Yh = Y.cpu().numpy()
    Yh[np.diag_indices(n)] = 1.0
    ref = hh.apply_q(Yh, tau.cpu().numpy(), C0)
    err = float(np.max(np.abs(out - ref)))
    print(f"n=16384 back-transformation: max err on 6 columns {err:.2e}", flush=True)
    assert err <= 1e-12 * np.sqrt(n)
