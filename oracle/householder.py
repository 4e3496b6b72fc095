"""Householder reflectors, the bidiagonal reduction and the back-transformation
of singular vectors.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The full SVD the paper builds (Section 2 and Section 4.1, 4.3) reduces a
dense A (m >= n) to an upper bidiagonal B = Q^T A P with products of
Householder reflectors, solves B = U_2 Sigma V_2^T (the divide-and-conquer
step), and back-transforms U = U_1 U_2 with U_1 = Q = H_1 ... H_n and
V^T = V_2^T V_1^T with V_1 = P = G_1 ... G_{n-2} (Section 4.3.3).

Every reflector is H = I - tau y y^T with y[i] = 1 at its pivot position,
zeros above it, and tau = 2 / (y^T y), so that H x = beta e_pivot with
beta = -sign(x_pivot) ||x|| (the reflector of Section 4.1).  The product of a
set of reflectors applied to a matrix is computed here by its plain
definition, one reflector at a time, C <- H_i C, with no blocking.  Readings
are stated where they are used.
"""

from __future__ import annotations

import math

import numpy as np


def reflector(x: np.ndarray):
    """(y, tau, beta) with (I - tau y y^T) x = beta e_0, y[0] = 1, beta =
    -sign(x_0) ||x||; tau = 0 and y = e_0 when x[1:] = 0 (the identity: x is
    already a multiple of e_0, beta = x_0)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.zeros_like(x)
    y[0] = 1.0
    sigma = float(np.dot(x[1:], x[1:]))
    if sigma == 0.0:
        return y, 0.0, float(x[0])
    alpha = float(x[0])
    norm = math.sqrt(alpha * alpha + sigma)
    beta = -math.copysign(norm, alpha)
    # y = (x - beta e_0) / (x_0 - beta); x_0 - beta has the sign of x_0 and
    # no cancellation
    y[1:] = x[1:] / (alpha - beta)
    tau = 2.0 / float(np.dot(y, y))
    return y, tau, beta


def bidiagonalize(A: np.ndarray):
    """Unblocked Householder reduction of A (m x n, m >= n) to upper
    bidiagonal form (the column/row reflector pairs of Section 4.1, one pair
    per column, each applied to the whole trailing matrix as it is formed).

    Returns (d, e, Yq, tq, Yp, tp): d (n), e (n-1); Yq (m x n) holds the
    column reflectors as full vectors (column i: zeros above row i, 1 at row
    i), tq (n); Yp (n x (n-1)) the row reflectors as full vectors (column i
    acts on coordinates i+1..n-1: zeros above row i+1, 1 at row i+1; the last
    one is the identity, tau 0), tp (n-1).  With Q = H_0 ... H_{n-1} and
    P = G_0 ... G_{n-2}: Q^T A P = [B; 0].
    """
    A = np.array(A, dtype=np.float64)
    m, n = A.shape
    assert m >= n
    Yq = np.zeros((m, n))
    Yp = np.zeros((n, max(n - 1, 0)))
    tq = np.zeros(n)
    tp = np.zeros(max(n - 1, 0))
    d = np.zeros(n)
    e = np.zeros(max(n - 1, 0))
    for i in range(n):
        y, t, beta = reflector(A[i:, i])
        Yq[i:, i] = y
        tq[i] = t
        A[i:, i:] -= t * np.outer(y, y @ A[i:, i:])  # A <- H_i A
        A[i, i] = beta
        A[i + 1:, i] = 0.0
        d[i] = beta
        if i < n - 1:
            y, t, beta = reflector(A[i, i + 1:])
            Yp[i + 1:, i] = y
            tp[i] = t
            A[i:, i + 1:] -= t * np.outer(A[i:, i + 1:] @ y, y)  # A <- A G_i
            A[i, i + 1] = beta
            A[i, i + 2:] = 0.0
            e[i] = beta
    return d, e, Yq, tq, Yp, tp


def apply_q(Y: np.ndarray, tau: np.ndarray, C: np.ndarray, trans: bool = False) -> np.ndarray:
    """Q C (trans False) or Q^T C (trans True) for Q = H_0 H_1 ... H_{k-1},
    H_i = I - tau_i y_i y_i^T with y_i the columns of Y (full vectors), by
    applying one reflector at a time: Q C = H_0 (H_1 (... (H_{k-1} C))), and
    Q^T C = H_{k-1} (... (H_0 C)) since every H_i is symmetric."""
    C = np.array(C, dtype=np.float64)
    k = Y.shape[1]
    order = range(k) if trans else range(k - 1, -1, -1)
    for i in order:
        y = Y[:, i]
        C -= tau[i] * np.outer(y, y @ C)
    return C


def pack_lapack(Y: np.ndarray, offset: int = 0) -> np.ndarray:
    """The storage the GPU routine reads: column i keeps only the entries
    below its unit pivot (rows > i + offset); the pivot 1 and the zeros above
    are implicit (the layout of LAPACK's geqrf / gebrd outputs)."""
    m, k = Y.shape
    out = np.zeros_like(Y)
    for i in range(k):
        p = i + offset
        if p < m:
            out[p + 1:, i] = Y[p + 1:, i]
    return out


def cwy_t_inverse(Y: np.ndarray, tau: np.ndarray) -> np.ndarray:
    """T^{-1} of the compact WY form H_0 ... H_{b-1} = I - Y T Y^T, built as
    eq. inv_t states it from the inner products of the reflectors: the
    diagonal holds 1/tau_i (= y_i^T y_i / 2 for tau_i = 2 / y_i^T y_i) and
    the off-diagonal entries y_i^T y_j on one side.  Reading: the text's
    "i > j" side is the lower one in its indexing; for the product in the
    order H_0 H_1 ..., T is upper triangular, so its inverse is too:
    T^{-1}(i, j) = y_i^T y_j for i < j."""
    G = Y.T @ Y
    Ti = np.triu(G, 1)
    Ti[np.diag_indices_from(Ti)] = 1.0 / tau
    return Ti


def qr(A: np.ndarray):
    """Unblocked Householder QR of A (m x n, m >= n): the reflector of
    Section 4.1 applied column by column, H_i eliminating below the diagonal
    of column i and updating the trailing columns as soon as it is formed
    (the panel step of LAPACK's geqrf named in Section 4.3.1, with no
    blocking).

    Returns (R, Y, tau): R (n x n upper triangular), Y (m x n) the reflectors
    as full vectors (column i: zeros above row i, 1 at row i), tau (n).
    A = Q [R; 0] with Q = H_0 H_1 ... H_{n-1}, H_i = I - tau_i y_i y_i^T."""
    A = np.array(A, dtype=np.float64)
    m, n = A.shape
    assert m >= n
    Y = np.zeros((m, n))
    tau = np.zeros(n)
    for i in range(n):
        y, t, beta = reflector(A[i:, i])
        Y[i:, i] = y
        tau[i] = t
        A[i:, i:] -= t * np.outer(y, y @ A[i:, i:])  # A <- H_i A
        A[i, i] = beta
        A[i + 1:, i] = 0.0
    return np.triu(A[:n, :]), Y, tau


def form_q(Y: np.ndarray, tau: np.ndarray, ncols: int) -> np.ndarray:
    """The first ncols columns of Q = H_0 ... H_{k-1} (eq. orgqr-q: the
    reflectors applied to the leading columns of the identity)."""
    m = Y.shape[0]
    return apply_q(Y, tau, np.eye(m)[:, :ncols])
