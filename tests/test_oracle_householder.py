"""Pins of the Householder oracle (reflectors, bidiagonal reduction, the
back-transformation product) against hand-worked values, invariants and
LAPACK's own QR routines (geqrf / orgqr / ormqr through scipy)."""

import numpy as np
import pytest
import scipy.linalg.lapack as lapack

from oracle import householder as hh


def test_reflector_hand_worked():
    """x = (3, 4): beta = -5, y = (1, 4 / (3 + 5)) = (1, 0.5),
    tau = 2 / (1 + 0.25) = 1.6, and H x = (-5, 0)."""
    y, tau, beta = hh.reflector(np.array([3.0, 4.0]))
    assert beta == -5.0 and tau == 1.6
    assert np.array_equal(y, [1.0, 0.5])
    H = np.eye(2) - tau * np.outer(y, y)
    assert np.allclose(H @ [3.0, 4.0], [-5.0, 0.0], atol=1e-15)


def test_reflector_properties_and_identity_case():
    g = np.random.default_rng(1)
    for n in (1, 2, 7, 50):
        x = g.standard_normal(n)
        y, tau, beta = hh.reflector(x)
        H = np.eye(n) - tau * np.outer(y, y)
        assert np.max(np.abs(H @ H.T - np.eye(n))) <= 1e-15 * n
        hx = H @ x
        assert abs(hx[0] - beta) <= 1e-14 * abs(beta) and np.max(np.abs(hx[1:]), initial=0.0) <= 1e-14 * abs(beta)
        if n > 1:
            assert np.sign(beta) == -np.sign(x[0]) and tau == pytest.approx(2.0 / (y @ y), rel=1e-15)
    y, tau, beta = hh.reflector(np.array([-2.0, 0.0, 0.0]))
    assert tau == 0.0 and beta == -2.0 and np.array_equal(y, [1.0, 0.0, 0.0])


@pytest.mark.parametrize("m,n", [(5, 5), (40, 25), (64, 64), (120, 33)])
def test_bidiagonalize_identity_and_spectrum(m, n):
    g = np.random.default_rng(m + n)
    A = g.standard_normal((m, n))
    d, e, Yq, tq, Yp, tp = hh.bidiagonalize(A)
    Q = hh.apply_q(Yq, tq, np.eye(m))
    P = hh.apply_q(Yp, tp, np.eye(n))
    B = np.diag(d) + np.diag(e, 1)
    assert np.max(np.abs(Q.T @ A @ P - np.vstack([B, np.zeros((m - n, n))]))) <= 1e-13
    assert np.max(np.abs(Q.T @ Q - np.eye(m))) <= 1e-14 and np.max(np.abs(P.T @ P - np.eye(n))) <= 1e-14
    sa = np.linalg.svd(A, compute_uv=False)
    sb = np.linalg.svd(B, compute_uv=False)
    assert np.max(np.abs(sa - sb)) <= 1e-13 * sa[0]
    # reflector structure: unit pivot, zeros above it
    for i in range(n):
        assert Yq[i, i] == 1.0 and np.all(Yq[:i, i] == 0.0)
    for i in range(n - 1):
        assert Yp[i + 1, i] == 1.0 and np.all(Yp[:i + 1, i] == 0.0)


@pytest.mark.parametrize("trans", ["N", "T"])
def test_apply_q_matches_lapack_ormqr(trans):
    g = np.random.default_rng(5)
    A = g.standard_normal((70, 30))
    qr, tau, _, info = lapack.dgeqrf(A)
    assert info == 0
    Y = np.tril(qr, -1) + np.eye(70, 30)
    C = g.standard_normal((70, 11))
    ref, _, info = lapack.dormqr("L", trans, qr, tau, C, lwork=4096)
    assert info == 0
    out = hh.apply_q(Y, tau, C, trans=trans == "T")
    assert np.max(np.abs(out - ref)) <= 1e-14 * np.max(np.abs(C)) * 10
    Q, _, info = lapack.dorgqr(qr, tau)
    assert np.max(np.abs(hh.apply_q(Y, tau, np.eye(70))[:, :30] - Q)) <= 1e-14


def test_cwy_inverse_triangular_factor():
    """eq. inv_t: I - Y T Y^T equals the reflector product when T^{-1} holds
    y_i^T y_j above the diagonal and 1/tau_i on it."""
    g = np.random.default_rng(6)
    A = g.standard_normal((50, 16))
    qr, tau, _, _ = lapack.dgeqrf(A)
    Y = np.tril(qr, -1) + np.eye(50, 16)
    Ti = hh.cwy_t_inverse(Y, tau)
    assert np.array_equal(Ti, np.triu(Ti))
    T = np.linalg.inv(Ti)
    prod = hh.apply_q(Y, tau, np.eye(50))
    assert np.max(np.abs(np.eye(50) - Y @ T @ Y.T - prod)) <= 1e-14
    # the lower-triangular reading would not reproduce the product
    Tl = np.linalg.inv(Ti.T)
    assert np.max(np.abs(np.eye(50) - Y @ Tl @ Y.T - prod)) > 1e-3


def test_pack_lapack_layout():
    g = np.random.default_rng(7)
    d, e, Yq, tq, Yp, tp = hh.bidiagonalize(g.standard_normal((9, 6)))
    Pq = hh.pack_lapack(Yq, 0)
    Pp = hh.pack_lapack(Yp, 1)
    for i in range(6):
        assert np.all(Pq[:i + 1, i] == 0.0) and np.array_equal(Pq[i + 1:, i], Yq[i + 1:, i])
    for i in range(5):
        assert np.all(Pp[:i + 2, i] == 0.0) and np.array_equal(Pp[i + 2:, i], Yp[i + 2:, i])


@pytest.mark.parametrize("m,n", [(1, 1), (7, 3), (60, 60), (300, 40), (129, 65)])
def test_qr_against_lapack_geqrf_orgqr(m, n):
    """The oracle's QR against LAPACK's geqrf (same reflector convention:
    unit pivot, beta = -sign(alpha) ||x||): R, the reflectors and tau agree
    to rounding; Q against orgqr; A = Q R and Q^T Q = I."""
    g = np.random.default_rng(m * 13 + n)
    A = g.standard_normal((m, n))
    R, Y, tau = hh.qr(A)
    qr_l, tau_l, _, info = lapack.dgeqrf(A)
    assert info == 0
    scale = np.max(np.abs(A)) * np.sqrt(m)
    assert np.max(np.abs(R - np.triu(qr_l[:n, :]))) <= 1e-14 * scale
    assert np.max(np.abs(tau - tau_l)) <= 1e-14
    assert np.max(np.abs(np.tril(Y, -1) - np.tril(qr_l, -1)[:, :n])) <= 1e-13 * np.sqrt(m)
    assert np.allclose(np.triu(Y[:n, :]), np.eye(n), atol=0.0)
    Q = hh.form_q(Y, tau, n)
    Q_l, _, info = lapack.dorgqr(qr_l, tau_l)
    assert info == 0
    assert np.max(np.abs(Q - Q_l[:, :n])) <= 1e-14 * np.sqrt(m)
    assert np.max(np.abs(Q @ R - A)) <= 1e-14 * scale
    assert np.max(np.abs(Q.T @ Q - np.eye(n))) <= 1e-14 * np.sqrt(m)


def test_qr_zero_and_reduced_columns():
    """A column that is already zero below its diagonal takes the identity
    (tau = 0), as LAPACK does; a zero matrix gives R = 0 and Q = I."""
    A = np.zeros((6, 3))
    R, Y, tau = hh.qr(A)
    assert np.array_equal(tau, np.zeros(3)) and np.array_equal(R, np.zeros((3, 3)))
    assert np.array_equal(hh.form_q(Y, tau, 3), np.eye(6)[:, :3])
    B = np.triu(np.arange(1.0, 25.0).reshape(6, 4))[:, :4]
    R, Y, tau = hh.qr(B)
    assert np.array_equal(tau, np.zeros(4)) and np.array_equal(R, B[:4])
