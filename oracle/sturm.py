"""All singular values of an upper bidiagonal by Sturm-count bisection.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

A second route to the spectrum, independent of the divide-and-conquer steps
and cheap in memory (O(n) per value), used where the dense oracle does not
fit (n = 32768) and to cross-check it at full size.  Plain definition: the
singular values of B are the non-negative eigenvalues of the 2n x 2n
Golub-Kahan tridiagonal T (zero diagonal, off-diagonal d_1, e_1, d_2, ...,
d_n), whose spectrum is {+sigma_i, -sigma_i}.  The number of eigenvalues of
T below x equals the number of negative pivots of the LDL^T factorisation of
T - x I (Sylvester's law of inertia); for x > 0 that count minus n is the
number of singular values below x.  Bisection on that count isolates every
singular value; all n bisections advance together, one pivot recurrence per
step over the vector of midpoints.
"""

from __future__ import annotations

import numpy as np

_TINY = 1e-300


def sturm_counts(d: np.ndarray, e: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Number of singular values of (d, e) below each x >= 0.

    The pivots of T - xI are q_1 = -x, q_{i+1} = -x - b_i^2 / q_i with b the
    off-diagonal; a zero pivot is replaced by -tiny (counted as negative),
    the usual convention that keeps the count monotone in x.
    """
    d = np.asarray(d, dtype=np.float64)
    n = d.shape[0]
    off = np.empty(2 * n - 1)
    off[0::2] = d
    off[1::2] = np.asarray(e, dtype=np.float64)[: n - 1]
    b2 = off * off
    x = np.asarray(x, dtype=np.float64)
    negx = -x
    q = negx.copy()
    q[q == 0.0] = -_TINY
    neg = (q < 0.0).astype(np.int64)
    t = np.empty_like(q)
    mask = np.empty(q.shape, dtype=bool)
    for b in b2:
        np.divide(b, q, out=t)
        np.subtract(negx, t, out=q)
        np.equal(q, 0.0, out=mask)
        if mask.any():
            q[mask] = -_TINY
        np.less(q, 0.0, out=mask)
        neg += mask
    return neg - n


def singular_values(d, e, max_iter: int = 80, index=None) -> np.ndarray:
    """All singular values of the bidiagonal, descending, by bisection
    (or only the 0-based positions ``index`` of the descending order).

    The i-th largest value (0-based) is the point where the count of values
    below x reaches n - i; the bracket starts at [0, 2 max(|d|, |e|)] (a
    Gershgorin bound of T) and is halved until its ends are adjacent doubles
    or ``max_iter`` halvings are done.  Returns the bracket midpoints.
    """
    d = np.asarray(d, dtype=np.float64)
    e = np.asarray(e, dtype=np.float64)
    n = d.shape[0]
    index = np.arange(n) if index is None else np.asarray(index, dtype=np.int64)
    if n == 0:
        return np.zeros(0)
    bound = 2.0 * max(float(np.max(np.abs(d))), float(np.max(np.abs(e[: n - 1]), initial=0.0)))
    if bound == 0.0:
        return np.zeros(index.shape[0])
    bound = bound * (1.0 + 1e-12) + _TINY
    target = n - index
    lo = np.zeros(index.shape[0])
    hi = np.full(index.shape[0], bound)
    for _ in range(max_iter):
        mid = 0.5 * (lo + hi)
        live = (mid > lo) & (mid < hi)
        if not live.any():
            break
        idx = np.nonzero(live)[0]
        c = sturm_counts(d, e, mid[idx])
        up = c >= target[idx]
        hi[idx[up]] = mid[idx[up]]
        lo[idx[~up]] = mid[idx[~up]]
    return 0.5 * (lo + hi)
