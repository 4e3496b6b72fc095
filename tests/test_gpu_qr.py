"""Householder QR of a tall matrix (bdc_geqrf) and its explicit Q
(bdc_orgqr) on the GPU against the oracle's unblocked Householder QR and
reflector-by-reflector product (Section 4.3.1-4.3.2), and at the
tall-and-skinny size of Section 5.1 (m = 20000, n = 1000) against the
oracle's stored R diagonal, tau and first row of R."""

import os

import numpy as np
import pytest

from oracle import householder as hh

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def solver(gpu):
    from paper_2508_11467_amd.api import Solver
    s = Solver(0)
    yield s
    s.close()


def _dev(A):
    """(m, n) column-major device copy."""
    import torch
    return torch.from_numpy(np.ascontiguousarray(A.T)).cuda().T


def _gpu_qr(solver, A, block=0, ncols=None):
    import torch
    Ad = _dev(A)
    tau = solver.geqrf(Ad, block=block)
    Q = solver.orgqr(Ad, tau, ncols=ncols)
    torch.cuda.synchronize()
    return Ad.cpu().numpy(), tau.cpu().numpy(), Q.cpu().numpy()


@pytest.mark.parametrize("m,n,block", [(300, 100, 0), (513, 257, 32), (1000, 64, 64), (64, 64, 16), (2000, 33, 0),
                                       (777, 129, 17), (1, 1, 0), (40, 1, 0)])
def test_geqrf_orgqr_match_oracle(solver, m, n, block):
    g = np.random.default_rng(m * 13 + n)
    A = g.standard_normal((m, n))
    F, tau, Q = _gpu_qr(solver, A, block)
    R0, Y0, tau0 = hh.qr(A)
    scale = np.linalg.norm(A, 2)
    R = np.triu(F[:n, :])
    assert np.max(np.abs(R - R0)) <= 1e-12 * scale, np.max(np.abs(R - R0))
    assert np.max(np.abs(tau - tau0)) <= 1e-12
    Y = np.tril(F, -1) + np.eye(m, n)
    assert np.max(np.abs(Y - Y0)) <= 1e-11, np.max(np.abs(Y - Y0))
    Qref = hh.form_q(Y0, tau0, n)
    assert np.max(np.abs(Q - Qref)) <= 1e-12
    assert np.max(np.abs(Q.T @ Q - np.eye(n))) <= 1e-13 * max(1.0, np.sqrt(m / 100))
    assert np.linalg.norm(Q @ R - A) <= 1e-14 * np.sqrt(m) * np.linalg.norm(A)


def test_orgqr_full_square_q(solver):
    """All m columns of Q (the m x m factor the tall-and-skinny SVD forms)."""
    g = np.random.default_rng(5)
    m, n = 400, 150
    A = g.standard_normal((m, n))
    F, tau, Q = _gpu_qr(solver, A, 32, ncols=m)
    _, Y0, tau0 = hh.qr(A)
    Qref = hh.form_q(Y0, tau0, m)
    assert np.max(np.abs(Q - Qref)) <= 1e-12
    assert np.max(np.abs(Q.T @ Q - np.eye(m))) <= 1e-13


def test_geqrf_degenerate_columns(solver):
    """Zero columns (nothing below the pivot: the reflector is the identity,
    tau = 0, as in the oracle) and a column scaled to 1e-150: R, tau and the
    reflectors as the oracle's."""
    g = np.random.default_rng(6)
    m, n = 200, 40
    A = g.standard_normal((m, n))
    A[:, 3] = 0.0
    A[:, 7] = 0.0
    A[7, 7] = 2.5
    A[:, 20] *= 1e-150
    F, tau, Q = _gpu_qr(solver, A, 16)
    R0, Y0, tau0 = hh.qr(A)
    assert tau[3] == 0.0 and tau0[3] == 0.0
    R = np.triu(F[:n, :])
    scale = np.linalg.norm(A, 2)
    assert np.max(np.abs(R - R0)) <= 1e-12 * scale
    assert np.max(np.abs(tau - tau0)) <= 1e-12
    assert abs(R[20, 20] - R0[20, 20]) <= 1e-12 * abs(R0[20, 20])
    assert np.linalg.norm(Q @ R - A) <= 1e-14 * np.sqrt(m) * np.linalg.norm(A)
    assert np.max(np.abs(Q.T @ Q - np.eye(n))) <= 1e-13


def test_geqrf_rank_deficient(solver):
    """A repeated column: below its pivot only rounding noise is left, so the
    reflector there (and R's later rows) is not determined by A; the
    factorisation still holds (A = QR, Q orthonormal) and R's diagonal entry
    at the repeated column is at rounding level."""
    g = np.random.default_rng(7)
    m, n = 300, 50
    A = g.standard_normal((m, n))
    A[:, 11] = A[:, 10]
    F, tau, Q = _gpu_qr(solver, A, 16)
    R = np.triu(F[:n, :])
    assert abs(R[11, 11]) <= 1e-13 * np.linalg.norm(A, 2)
    assert np.linalg.norm(Q @ R - A) <= 1e-14 * np.sqrt(m) * np.linalg.norm(A)
    assert np.max(np.abs(Q.T @ Q - np.eye(n))) <= 1e-13


def test_geqrf_rejects_more_rows_than_the_resident_grid(solver):
    """A panel whose rows below its top block exceed 160 per workgroup of the
    resident grid is refused on the host before any work is enqueued."""
    import torch

    from paper_2508_11467_amd import _lib
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    m, n = 160 * cus + 64 + 200, 64
    A = torch.zeros((n, m), dtype=torch.float64, device="cuda").T
    with pytest.raises(_lib.BdcError) as err:
        solver.geqrf(A, block=64)
    assert err.value.code == _lib.BDC_ERR_TOO_LARGE


def test_geqrf_tall_skinny_full_size(solver):
    """m = 20000, n = 1000 N(0,1) (the tall-and-skinny size of Section 5.1):
    R's diagonal, tau and R's first row against the oracle's stored values;
    A = Q R and Q^T Q = I on the GPU."""
    import torch

    from paper_2508_11467_amd import inputs
    m, n = 20000, 1000
    A = inputs.dense_normal(m, n, inputs.DENSE_TS_SEED)
    gold = np.load(os.path.join(HERE, "golden", "oracle_qr_ts20000x1000.npy"), allow_pickle=False)
    Ad = _dev(A)
    tau = solver.geqrf(Ad)
    Q = solver.orgqr(Ad, tau)
    torch.cuda.synchronize()
    R = torch.triu(Ad[:n, :])
    diag = torch.diagonal(R).cpu().numpy()
    print(f"QR {m}x{n}: max |diag R - oracle| {np.max(np.abs(diag - gold[0])):.2e}, "
          f"max |tau - oracle| {np.max(np.abs(tau.cpu().numpy() - gold[1])):.2e}", flush=True)
    assert np.max(np.abs(diag - gold[0])) <= 1e-10
    assert np.max(np.abs(tau.cpu().numpy() - gold[1])) <= 1e-13
    assert np.max(np.abs(R[0].cpu().numpy() - gold[2])) <= 1e-10
    Qc = Q.contiguous()
    orth = float(torch.max(torch.abs(Qc.T.contiguous() @ Qc - torch.eye(n, dtype=torch.float64, device="cuda"))))
    At = torch.from_numpy(A).cuda()
    res = float(torch.linalg.norm(Qc @ R.contiguous() - At) / torch.linalg.norm(At))
    print(f"QR {m}x{n}: orth {orth:.2e} residual {res:.2e}", flush=True)
    assert orth <= 1e-13 and res <= 1e-14


@pytest.mark.parametrize("m,n", [(3000, 300), (1000, 1000), (2500, 129)])
def test_tall_skinny_svd_end_to_end(solver, m, n):
    """The tall-and-skinny SVD on the GPU (Section 4.3.1): QR (bdc_geqrf), the
    SVD of R (bdc_gebrd, bdc_svd, bdc_apply_reflectors), the explicit Q
    (bdc_orgqr) and U = Q U_R (the FP64 matrix-core product of
    bdc_step_gemm): the singular values against LAPACK's, E_svd and
    orthogonality."""
    import torch
    g = np.random.default_rng(m + 3 * n)
    A = g.standard_normal((m, n))
    Ad = _dev(A)
    tau = solver.geqrf(Ad)
    R = torch.empty((n, n), dtype=torch.float64, device="cuda").T
    R.copy_(torch.triu(Ad[:n, :]))
    d, e, tq, tp = solver.gebrd(R)
    sig, U2, VT2 = solver.svd(d, e)
    UR = torch.empty((n, n), dtype=torch.float64, device="cuda").T
    UR.copy_(U2)
    V = torch.empty((n, n), dtype=torch.float64, device="cuda").T
    V.copy_(VT2.T)
    solver.apply_reflectors(R, tq, UR, trans=False, offset=0)
    if n > 1:
        solver.apply_reflectors(R, tp[:n - 1], V, trans=False, offset=1, rows=True)
    Q = solver.orgqr(Ad, tau)
    U = torch.empty((n, m), dtype=torch.float64, device="cuda").T
    solver.gemm(Q, UR, U)
    torch.cuda.synchronize()
    s, Un, Vn = sig.cpu().numpy(), U.cpu().numpy(), V.cpu().numpy()
    ref = np.linalg.svd(A, compute_uv=False)
    e_svd = np.linalg.norm(A - (Un * s) @ Vn.T) / np.linalg.norm(A)
    print(f"TS SVD {m}x{n}: E_svd {e_svd:.2e} max sigma err {np.max(np.abs(s - ref)) / ref[0]:.2e}", flush=True)
    assert np.max(np.abs(s - ref)) <= 1e-13 * ref[0]
    assert e_svd <= 1e-13
    assert np.max(np.abs(Un.T @ Un - np.eye(n))) <= 1e-12
    assert np.max(np.abs(Vn.T @ Vn - np.eye(n))) <= 1e-12


def test_geqrf_is_bitwise_reproducible(solver):
    """The panel's grid all-reduce adds the workgroups' partial sums in a
    fixed order: two runs give bitwise the same R, reflectors and tau."""
    g = np.random.default_rng(12)
    A = g.standard_normal((6000, 200))
    F1, t1, Q1 = _gpu_qr(solver, A)
    F2, t2, Q2 = _gpu_qr(solver, A)
    assert np.array_equal(F1, F2) and np.array_equal(t1, t2) and np.array_equal(Q1, Q2)
