"""Brute-force references used to pin the oracle (independent of it).

* Cyclic Jacobi on the 2n x 2n Golub-Kahan tridiagonal: zero diagonal and
  off-diagonal (d_1, e_1, d_2, e_2, ..., d_n); its eigenvalues are +-sigma_i,
  and the eigenvector of +sigma is (v_1, u_1, v_2, u_2, ...)/sqrt(2), from
  B v = sigma u and B^T u = sigma v.  It runs in x87 extended precision
  (numpy longdouble, 64-bit significand) so that its own rounding stays well
  below the float64 tolerances it is used to check.
"""

import numpy as np

LD = np.longdouble


def golub_kahan(d, e):
    n = len(d)
    off = np.zeros(2 * n - 1, dtype=LD)
    off[0::2] = np.asarray(d, dtype=LD)
    off[1::2] = np.asarray(e, dtype=LD)[: n - 1]
    T = np.diag(off, 1) + np.diag(off, -1)
    return T


def jacobi_eigh(A, max_sweeps=40):
    """Cyclic-by-row Jacobi for a symmetric matrix: returns (w, V)."""
    A = np.array(A, dtype=LD)
    n = A.shape[0]
    V = np.eye(n, dtype=LD)
    one = LD(1)
    eps = np.finfo(LD).eps
    for _ in range(max_sweeps):
        off = np.sqrt(LD(2) * np.sum(np.triu(A, 1) ** 2))
        if off <= eps * np.sqrt(np.sum(A * A)):
            break
        for p in range(n - 1):
            for q in range(p + 1, n):
                apq = A[p, q]
                if apq == 0:
                    continue
                app, aqq = A[p, p], A[q, q]
                theta = (aqq - app) / (2 * apq)
                if abs(theta) > LD(1e300):
                    t = LD(0.5) / theta
                else:
                    sgn = one if theta >= 0 else -one
                    t = sgn / (abs(theta) + np.sqrt(theta * theta + one))
                c = one / np.sqrt(t * t + one)
                s = t * c
                ap = A[:, p].copy()
                aq = A[:, q].copy()
                A[:, p] = c * ap - s * aq
                A[:, q] = s * ap + c * aq
                ap = A[p, :].copy()
                aq = A[q, :].copy()
                A[p, :] = c * ap - s * aq
                A[q, :] = s * ap + c * aq
                vp = V[:, p].copy()
                vq = V[:, q].copy()
                V[:, p] = c * vp - s * vq
                V[:, q] = s * vp + c * vq
    return np.diag(A).copy(), V


def gk_singular_values(d, e):
    """Singular values (descending, float64) of the bidiagonal via Jacobi on
    its Golub-Kahan tridiagonal."""
    w, _ = jacobi_eigh(golub_kahan(d, e))
    w = np.sort(w)[::-1]
    return w[: len(d)].astype(np.float64)


def sturm_count(d, e, x):
    """Number of singular values of the bidiagonal (d, e) below x >= 0, from
    the LDL^T inertia of the Golub-Kahan tridiagonal T - x I (T has zero
    diagonal and off-diagonal d_1, e_1, d_2, ...): eigenvalues of T below x
    number n + (singular values below x)."""
    n = len(d)
    off = np.empty(2 * n - 1)
    off[0::2] = d
    off[1::2] = np.asarray(e)[: n - 1]
    neg = 0
    tiny = 1e-300
    q = -x
    if q == 0.0:
        q = -tiny  # a zero pivot counts as negative, consistently
    if q < 0:
        neg += 1
    for b in off:
        q = -x - (b * b) / q
        if q == 0.0:
            q = -tiny
        if q < 0:
            neg += 1
    return neg - n


def singular_value_by_bisection(d, e, i, iters=100):
    """The i-th largest singular value (0-based) by bisection on sturm_count."""
    n = len(d)
    hi = float(np.max(np.abs(d)) + np.max(np.abs(np.asarray(e)[: n - 1]), initial=0.0)) * 2.0 + 1e-300
    lo = 0.0
    target = n - i  # number of values <= sigma_i from below
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if mid == lo or mid == hi:
            break
        if sturm_count(d, e, mid) >= target:
            hi = mid
        else:
            lo = mid
    return 0.5 * (lo + hi)
