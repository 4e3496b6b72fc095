"""Bidiagonal reduction on the GPU (bdc_gebrd, the merged-rank-(2b) gebrd of
Algorithm 1) against the oracle's unblocked Householder reduction (Section
4.1), and the dense SVD it starts (gebrd, then the bidiagonal
divide-and-conquer, then the back-transformation) against LAPACK's singular
values, all on the GPU."""

import numpy as np
import pytest

from oracle import householder as hh

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def solver(gpu):
    from paper_2508_11467_amd.api import Solver
    s = Solver(0)
    yield s
    s.close()


def _dev(A):
    import torch
    return torch.from_numpy(np.ascontiguousarray(A.T)).cuda().T


def _gpu_gebrd(solver, A, block=0):
    import torch
    Ad = _dev(A)
    d, e, tq, tp = solver.gebrd(Ad, block=block)
    torch.cuda.synchronize()
    return Ad.cpu().numpy(), d.cpu().numpy(), e.cpu().numpy(), tq.cpu().numpy(), tp.cpu().numpy()


def _unpack(F, m, n):
    """Full reflector vectors from gebrd storage: column i of Yq (unit at row
    i), column i of Yp (unit at coordinate i + 1)."""
    Yq = np.tril(F, -1) + np.eye(m, n)
    Yp = np.zeros((n, max(n - 1, 0)))
    for i in range(n - 1):
        Yp[i + 1, i] = 1.0
        Yp[i + 2:, i] = F[i, i + 2:]
    return Yq, Yp


@pytest.mark.parametrize("m,n,block", [(64, 64, 0), (200, 150, 32), (300, 300, 16), (513, 257, 7), (1000, 100, 0),
                                       (33, 33, 32), (40, 1, 0), (1, 1, 0), (2, 2, 0), (97, 96, 5)])
def test_gebrd_matches_oracle(solver, m, n, block):
    g = np.random.default_rng(m * 31 + n)
    A = g.standard_normal((m, n))
    F, d, e, tq, tp = _gpu_gebrd(solver, A, block)
    d0, e0, Yq0, tq0, Yp0, tp0 = hh.bidiagonalize(A)
    scale = np.linalg.norm(A, 2)
    assert np.max(np.abs(d - d0)) <= 1e-12 * scale, np.max(np.abs(d - d0))
    assert np.max(np.abs(e - e0), initial=0.0) <= 1e-12 * scale
    assert np.array_equal(np.diag(F), d) and np.array_equal(np.diag(F, 1)[:n - 1], e)
    # the last reflectors of a square matrix act on a few entries whose
    # values carry the rounding of the whole reduction (blocked here,
    # unblocked in the oracle): tau and y agree to about 1e-12, not 1e-15
    assert np.max(np.abs(tq - tq0)) <= 1e-10
    assert np.max(np.abs(tp[:n - 1] - tp0), initial=0.0) <= 1e-10 and tp[n - 1] == 0.0
    Yq, Yp = _unpack(F, m, n)
    assert np.max(np.abs(Yq - Yq0)) <= 1e-10
    assert np.max(np.abs(Yp - Yp0), initial=0.0) <= 1e-10
    # Q^T A P = [B; 0] from the GPU's own reflectors
    B = np.zeros((m, n))
    B[np.arange(n), np.arange(n)] = d
    B[np.arange(n - 1), np.arange(1, n)] = e
    QtA = hh.apply_q(Yq, tq, A, trans=True)
    # (Q^T A) P = (P^T (Q^T A)^T)^T
    QtAP = hh.apply_q(Yp, tp[:n - 1], QtA.T, trans=True).T if n > 1 else QtA
    assert np.max(np.abs(QtAP - B)) <= 1e-13 * np.sqrt(m) * scale


def test_gebrd_zero_columns(solver):
    """Zero columns: the identity reflector (tau = 0) where nothing is left
    to eliminate, a zero on the diagonal, and the rest as the oracle's."""
    g = np.random.default_rng(8)
    m, n = 150, 60
    A = g.standard_normal((m, n))
    A[:, 0] = 0.0
    F, d, e, tq, tp = _gpu_gebrd(solver, A, 16)
    d0, e0, Yq0, tq0, Yp0, tp0 = hh.bidiagonalize(A)
    assert tq[0] == 0.0 and tq0[0] == 0.0 and d[0] == 0.0
    scale = np.linalg.norm(A, 2)
    assert np.max(np.abs(d - d0)) <= 1e-12 * scale and np.max(np.abs(e - e0)) <= 1e-12 * scale
    assert np.max(np.abs(tq - tq0)) <= 1e-10 and np.max(np.abs(tp[:n - 1] - tp0)) <= 1e-10


def test_gebrd_nearly_rank_deficient(solver):
    """A column scaled to 1e-150 makes A numerically rank deficient: the
    trailing reflectors are then driven by rounding and not determined by A,
    so only what holds for any of them is checked: Q^T A P = [B; 0] and the
    singular values against LAPACK's."""
    g = np.random.default_rng(9)
    m, n = 150, 60
    A = g.standard_normal((m, n))
    A[:, 30] *= 1e-150
    F, d, e, tq, tp = _gpu_gebrd(solver, A, 16)
    Yq, Yp = _unpack(F, m, n)
    B = np.zeros((m, n))
    B[np.arange(n), np.arange(n)] = d
    B[np.arange(n - 1), np.arange(1, n)] = e
    QtAP = hh.apply_q(Yp, tp[:n - 1], hh.apply_q(Yq, tq, A, trans=True).T, trans=True).T
    scale = np.linalg.norm(A, 2)
    assert np.max(np.abs(QtAP - B)) <= 1e-13 * np.sqrt(m) * scale
    s = np.linalg.svd(B[:n], compute_uv=False)
    ref = np.linalg.svd(A, compute_uv=False)
    assert np.max(np.abs(s - ref)) <= 1e-13 * ref[0]


@pytest.mark.parametrize("m,n", [(600, 600), (900, 500)])
def test_dense_svd_on_gpu(solver, m, n):
    """The whole dense SVD on the GPU: gebrd, the bidiagonal SVD, U = Q [U_2;
    0] and V = P V_2 (bdc_apply_reflectors): Section 5.1's E_svd, orthogonality
    and the singular values against LAPACK's."""
    import torch
    g = np.random.default_rng(m + 7 * n)
    A = g.standard_normal((m, n))
    Ad = _dev(A)
    d, e, tq, tp = solver.gebrd(Ad)
    sig, U2, VT2 = solver.svd(d, e)
    U = torch.zeros((n, m), dtype=torch.float64, device="cuda").T  # column-major m x n
    U[:n, :] = U2
    V = VT2.contiguous().clone().T  # column-major n x n holding V_2
    solver.apply_reflectors(Ad, tq, U, trans=False, offset=0)
    solver.apply_reflectors(Ad, tp[:n - 1], V, trans=False, offset=1, rows=True)
    torch.cuda.synchronize()
    U = U.cpu().numpy()
    V = V.cpu().numpy()
    s = sig.cpu().numpy()
    e_svd = np.linalg.norm(A - (U * s) @ V.T) / np.linalg.norm(A)
    ref = np.linalg.svd(A, compute_uv=False)
    print(f"GPU dense SVD {m}x{n}: E_svd {e_svd:.2e} E_sigma {np.linalg.norm(s - ref) / n:.2e}", flush=True)
    assert e_svd <= 1e-12
    assert np.max(np.abs(s - ref)) <= 1e-13 * ref[0]
    assert np.max(np.abs(U.T @ U - np.eye(n))) <= 1e-12
    assert np.max(np.abs(V.T @ V - np.eye(n))) <= 1e-12


def test_gebrd_square_2048_spectrum(solver):
    """n = 2048 (square N(0,1)): the bidiagonal's singular values (by the
    GPU divide and conquer) against LAPACK's SVD of A, and A = Q B P^T on the
    GPU through bdc_apply_reflectors."""
    import torch

    from paper_2508_11467_amd import inputs
    n = 2048
    A = inputs.dense_normal(n, n, inputs.DENSE_SQUARE_SEED)
    Ad = _dev(A)
    d, e, tq, tp = solver.gebrd(Ad)
    sig, _, _ = solver.svd(d, e)
    torch.cuda.synchronize()
    s = sig.cpu().numpy()
    ref = np.linalg.svd(A, compute_uv=False)
    err = float(np.max(np.abs(s - ref)) / ref[0])
    # A = Q B P^T: Z = P B^T (P on the columns of B^T), then Q (Z^T)
    B = torch.diag(d) + torch.diag(e, 1)
    Z = torch.empty((n, n), dtype=torch.float64, device="cuda").T  # column-major
    Z.copy_(B.T)
    solver.apply_reflectors(Ad, tp[:n - 1], Z, trans=False, offset=1, rows=True)
    W = torch.empty((n, n), dtype=torch.float64, device="cuda").T
    W.copy_(Z.T)                                                    # B P^T
    solver.apply_reflectors(Ad, tq, W, trans=False, offset=0)       # Q B P^T
    torch.cuda.synchronize()
    At = torch.from_numpy(A).cuda()
    res = float(torch.linalg.norm(W - At) / torch.linalg.norm(At))
    print(f"gebrd n=2048: sigma err {err:.2e} residual {res:.2e}", flush=True)
    assert err <= 1e-13 and res <= 1e-14 * np.sqrt(n)


def test_gebrd_is_bitwise_reproducible(solver):
    """Partial sums cross workgroups through per-workgroup slots added in a
    fixed order, whichever workgroup arrives last: two runs on the same input
    give bitwise the same reflectors and bidiagonal."""
    g = np.random.default_rng(11)
    A = g.standard_normal((700, 500))
    r1 = _gpu_gebrd(solver, A)
    r2 = _gpu_gebrd(solver, A)
    for x, y in zip(r1, r2):
        assert np.array_equal(x, y)
