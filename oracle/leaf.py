"""Oracle leaf solver: SVD of a small upper bidiagonal by implicit-shift QR.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper solves the bottom-level subproblems of the divide-and-conquer tree
"by QR iteration" (Section 4.2.1, Algorithm 2 step (1)).  It does not say which
variant; this file uses the Golub-Kahan SVD step with a Wilkinson shift
(Golub & Van Loan, Matrix Computations, Section 8.6), acting on an explicit
dense copy of the leaf so each rotation can be checked by eye.

A leaf is m x (m+s) with s in {0, 1}: rows carry d[0..m-1] on the diagonal and
the superdiagonal entries; with s = 1 the last superdiagonal entry sits in the
extra column m.  The result is (sigma ascending, W (m x m), Q ((m+s) x (m+s)))
with  B = W [diag(sigma) 0] Q^T  and, when s = 1, B @ Q[:, m] = 0.
"""

from __future__ import annotations

import math

import numpy as np

EPS = 2.0 ** -52


def givens(f: float, g: float) -> tuple[float, float, float]:
    """(c, s, r) with c*f + s*g = r and -s*f + c*g = 0, r >= 0."""
    if g == 0.0:
        if f >= 0.0:
            return 1.0, 0.0, f
        return -1.0, 0.0, -f
    r = math.hypot(f, g)
    return f / r, g / r, r


def rot_cols(A: np.ndarray, i: int, j: int, c: float, s: float) -> None:
    """Columns (i, j) <- (c*a_i + s*a_j, -s*a_i + c*a_j)."""
    ai = A[:, i].copy()
    aj = A[:, j].copy()
    A[:, i] = c * ai + s * aj
    A[:, j] = -s * ai + c * aj


def rot_rows(A: np.ndarray, i: int, j: int, c: float, s: float) -> None:
    """Rows (i, j) <- (c*a_i + s*a_j, -s*a_i + c*a_j)."""
    ai = A[i, :].copy()
    aj = A[j, :].copy()
    A[i, :] = c * ai + s * aj
    A[j, :] = -s * ai + c * aj


def dense_bidiagonal(d: np.ndarray, e: np.ndarray, s: int) -> np.ndarray:
    """The m x (m+s) upper bidiagonal with diagonal d and superdiagonal e
    (len(e) = m - 1 + s)."""
    m = len(d)
    B = np.zeros((m, m + s))
    B[np.arange(m), np.arange(m)] = d
    ne = m - 1 + s
    if ne > 0:
        B[np.arange(ne), np.arange(1, ne + 1)] = e[:ne]
    return B


def _wilkinson_shift(B: np.ndarray, lo: int, hi: int) -> float:
    """Eigenvalue of the trailing 2x2 of (B^T B) restricted to rows/cols
    [lo, hi] that is closer to its last diagonal entry."""
    dm = B[hi - 1, hi - 1]
    dn = B[hi, hi]
    fm = B[hi - 1, hi]
    g = B[hi - 2, hi - 1] if hi - 1 > lo else 0.0
    t11 = dm * dm + g * g
    t12 = dm * fm
    t22 = dn * dn + fm * fm
    if t12 == 0.0:
        return t22
    delta = 0.5 * (t11 - t22)
    root = math.hypot(delta, t12)
    denom = delta + (root if delta >= 0.0 else -root)
    return t22 - t12 * t12 / denom


def _gk_step(B, W, Q, lo, hi):
    """One implicit-shift Golub-Kahan sweep over the unreduced block."""
    mu = _wilkinson_shift(B, lo, hi)
    y = B[lo, lo] * B[lo, lo] - mu
    z = B[lo, lo] * B[lo, lo + 1]
    for k in range(lo, hi):
        c, s, r = givens(y, z)
        rot_cols(B, k, k + 1, c, s)
        rot_cols(Q, k, k + 1, c, s)
        if k > lo:
            B[k - 1, k] = r
            B[k - 1, k + 1] = 0.0
        y = B[k, k]
        z = B[k + 1, k]
        c, s, r = givens(y, z)
        rot_rows(B, k, k + 1, c, s)
        rot_cols(W, k, k + 1, c, s)
        B[k, k] = r
        B[k + 1, k] = 0.0
        if k < hi - 1:
            y = B[k, k + 1]
            z = B[k, k + 2]


def leaf_svd(d: np.ndarray, e: np.ndarray, s: int, max_sweeps: int | None = None):
    """SVD of the m x (m+s) leaf; returns (sigma asc, W, Q, sweeps)."""
    d = np.asarray(d, dtype=np.float64)
    e = np.asarray(e, dtype=np.float64)
    m = len(d)
    B = dense_bidiagonal(d, e, s)
    W = np.eye(m)
    Q = np.eye(m + s)
    # Exact scaling by a power of two (not in the paper) so that no square in
    # the shift or the bulge can overflow or underflow; undone on the values.
    bmax = float(np.max(np.abs(B))) if B.size else 0.0
    p = math.ldexp(1.0, math.frexp(bmax)[1]) if 0.0 < bmax < math.inf else 1.0
    B = B / p
    bnorm = bmax / p
    tiny = EPS * bnorm

    # s = 1: rotate the extra column's entry away, bottom row first.  Each
    # right rotation of columns (j, m) zeroes B[j, m] and pushes a fill-in to
    # B[j-1, m]; the last one (j = 0) leaves column m zero, so Q[:, m] spans
    # the null space.
    if s == 1:
        for j in range(m - 1, -1, -1):
            c, sn, r = givens(B[j, j], B[j, m])
            rot_cols(B, j, m, c, sn)
            rot_cols(Q, j, m, c, sn)
            B[j, j] = r
            B[j, m] = 0.0

    if max_sweeps is None:
        max_sweeps = 40 * max(m, 1)
    sweeps = 0
    hi = m - 1
    while hi > 0:
        for i in range(hi):
            if abs(B[i, i + 1]) <= EPS * (abs(B[i, i]) + abs(B[i + 1, i + 1])):
                B[i, i + 1] = 0.0
        if B[hi - 1, hi] == 0.0:
            hi -= 1
            continue
        lo = hi - 1
        while lo > 0 and B[lo - 1, lo] != 0.0:
            lo -= 1
        # zero diagonal inside the unreduced block: chase its row (or, for
        # the last diagonal, its column) so the block splits.
        zero_at = -1
        for i in range(lo, hi + 1):
            if abs(B[i, i]) <= tiny:
                zero_at = i
                break
        if zero_at >= 0:
            i = zero_at
            B[i, i] = 0.0
            if i < hi:
                for j in range(i + 1, hi + 1):
                    c, sn, r = givens(B[j, j], B[i, j])
                    rot_rows(B, j, i, c, sn)
                    rot_cols(W, j, i, c, sn)
                    B[j, j] = r
                    B[i, j] = 0.0
            else:
                for j in range(hi - 1, lo - 1, -1):
                    c, sn, r = givens(B[j, j], B[j, hi])
                    rot_cols(B, j, hi, c, sn)
                    rot_cols(Q, j, hi, c, sn)
                    B[j, j] = r
                    B[j, hi] = 0.0
            continue
        if sweeps >= max_sweeps:
            raise RuntimeError("leaf QR iteration did not converge")
        _gk_step(B, W, Q, lo, hi)
        sweeps += 1

    sig = np.array([B[i, i] for i in range(m)], dtype=np.float64) * p
    neg = sig < 0.0
    sig[neg] = -sig[neg]
    W[:, neg] = -W[:, neg]
    order = np.argsort(sig, kind="stable")
    sig = sig[order]
    W = W[:, order]
    Q[:, :m] = Q[:, order]
    return sig, W, Q, sweeps
