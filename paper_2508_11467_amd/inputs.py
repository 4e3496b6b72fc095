"""Seeded synthetic upper-bidiagonal workloads.

This module draws random numbers and nothing else: it holds none of the
divide-and-conquer arithmetic, so both the GPU path and the CPU oracle may use
it to obtain identical inputs.

The paper measures its bidiagonal solver on bidiagonals produced by reducing
dense test matrices (four generator types, Section 3); that generator and the
dense front end are not part of this solver, so seeded bidiagonals with the
spectra below stand in for them.

Every generator returns ``(d, e)`` as float64 NumPy arrays: ``d`` the diagonal
(length n) and ``e`` the superdiagonal (length n-1) of B.
"""

from __future__ import annotations

import numpy as np

BASE_SEED = 2508_11467


def seed_for(config: int, spectrum: int = 0) -> int:
    """Seed of a configuration: base + 100*config + spectrum index."""
    return BASE_SEED + 100 * config + spectrum


def split_seed(config: int, spectrum: int, split: str, k: int) -> int:
    """Seed of the k-th problem of a training ("train") or held-out ("valid")
    set drawn like a configuration; never equal to a configuration's own
    seed."""
    base = {"train": 1_000_000, "valid": 500_000_000}[split]
    return BASE_SEED + 100 * config + spectrum + base * (k + 1)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform(n: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """d_i, e_i iid Uniform(-1, 1); d drawn first, then e."""
    g = _rng(seed)
    d = g.uniform(-1.0, 1.0, n)
    e = g.uniform(-1.0, 1.0, max(n - 1, 0))
    return d, e


def normal(n: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """d_i, e_i iid N(0, 1); d drawn first, then e."""
    g = _rng(seed)
    d = g.standard_normal(n)
    e = g.standard_normal(max(n - 1, 0))
    return d, e


def graded(n: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """d_i = 10^(-8 i / n) * u_i with u_i ~ U(0.5, 1); e_i = 1e-3 * U(-1, 1)."""
    g = _rng(seed)
    u = g.uniform(0.5, 1.0, n)
    i = np.arange(n, dtype=np.float64)
    d = 10.0 ** (-8.0 * i / n) * u
    e = 1e-3 * g.uniform(-1.0, 1.0, max(n - 1, 0))
    return d, e


def clustered(n: int, seed: int, centres: int = 16, jitter: float = 1e-14,
              zero_frac: float = 0.3) -> tuple[np.ndarray, np.ndarray]:
    """Heavy-deflation spectrum.

    ``centres`` values c ~ U(-1, 1) are drawn once; d_i = c_kappa(i) * (1 +
    jitter * U(-1, 1)) with kappa(i) uniform over the centres; e_i = 0 with
    probability ``zero_frac``, otherwise U(-1, 1).
    """
    g = _rng(seed)
    c = g.uniform(-1.0, 1.0, centres)
    kappa = g.integers(0, centres, n)
    d = c[kappa] * (1.0 + jitter * g.uniform(-1.0, 1.0, n))
    ne = max(n - 1, 0)
    zero = g.uniform(0.0, 1.0, ne) < zero_frac
    e = g.uniform(-1.0, 1.0, ne)
    e[zero] = 0.0
    return d, e


def ones(n: int) -> tuple[np.ndarray, np.ndarray]:
    """d = e = 1 (closed-form spectrum sigma_k = 2 cos(k pi / (2n + 1)))."""
    return np.ones(n), np.ones(max(n - 1, 0))


def near_ones(n: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """d, e iid 1 + 0.1 U(-1,1): a perturbed d = e = 1, which keeps most
    values at every merge (large update products)."""
    g = _rng(seed)
    d = 1.0 + 0.1 * g.uniform(-1.0, 1.0, n)
    e = 1.0 + 0.1 * g.uniform(-1.0, 1.0, max(n - 1, 0))
    return d, e


def batch_sizes(count: int, lo: int, hi: int, seed: int) -> np.ndarray:
    """Sizes n_i = round(exp(U(ln lo, ln hi))), as int64."""
    g = _rng(seed)
    return np.rint(np.exp(g.uniform(np.log(lo), np.log(hi), count))).astype(np.int64)


def batch_uniform(sizes, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """Packed batch: problem i occupies d[off_i : off_i + n_i] and the same
    offsets in e (its last slot unused), with off_i = sum_{j<i} n_j."""
    g = _rng(seed)
    total = int(np.sum(sizes))
    d = g.uniform(-1.0, 1.0, total)
    e = g.uniform(-1.0, 1.0, total)
    off = 0
    for n in sizes:
        e[off + int(n) - 1] = 0.0
        off += int(n)
    return d, e


def sigma_law(n: int, law: str, theta: float, seed: int | None = None) -> np.ndarray:
    """Singular values of the paper's test-matrix types (Section 3), in
    descending order, with condition number theta:

    * ``logrand``: log sigma_i iid uniform over (log(1/theta), log 1), seeded;
    * ``arith``: sigma_i = 1 - (i-1)/(n-1) (1 - 1/theta);
    * ``geo``: sigma_i = theta^(-(i-1)/(n-1)).
    """
    if n == 1:
        return np.ones(1)
    i = np.arange(n, dtype=np.float64)
    if law == "arith":
        s = 1.0 - i / (n - 1) * (1.0 - 1.0 / theta)
    elif law == "geo":
        s = theta ** (-i / (n - 1))
    elif law == "logrand":
        s = np.exp(_rng(seed).uniform(np.log(1.0 / theta), 0.0, n))
    else:
        raise KeyError(law)
    return np.sort(s)[::-1].copy()


def gkl_bidiagonal(sigma: np.ndarray, seed: int) -> tuple[np.ndarray, np.ndarray, float]:
    """Upper bidiagonal B with singular values sigma: Golub-Kahan-Lanczos
    bidiagonalisation of A = diag(sigma) from a seeded random unit start
    vector, with full reorthogonalisation (twice) of both Lanczos bases, so
    that A V = U B with U and V orthogonal to working precision.

    Returns (d, e, delta), where delta bounds |sigma_k(B) - sigma_k| for every
    k (Weyl): delta = ||A V - U B||_2 + ||A||_2 max(||U^T U - I||_2,
    ||V^T V - I||_2) computed in FP64, with a factor 2 of headroom for the
    rounding of that evaluation itself.
    """
    n = len(sigma)
    g = _rng(seed)
    U = np.zeros((n, n))
    V = np.zeros((n, n))
    d = np.zeros(n)
    e = np.zeros(max(n - 1, 0))
    v = g.standard_normal(n)
    V[:, 0] = v / np.linalg.norm(v)
    for k in range(n):
        u = sigma * V[:, k]
        if k > 0:
            u -= e[k - 1] * U[:, k - 1]
        for _ in range(2):
            u -= U[:, :k] @ (U[:, :k].T @ u)
        d[k] = np.linalg.norm(u)
        U[:, k] = u / d[k]
        if k + 1 < n:
            v = sigma * U[:, k] - d[k] * V[:, k]
            for _ in range(2):
                v -= V[:, :k + 1] @ (V[:, :k + 1].T @ v)
            e[k] = np.linalg.norm(v)
            V[:, k + 1] = v / e[k]
    B = np.diag(d) + np.diag(e, 1)
    I = np.eye(n)
    res = np.linalg.norm(sigma[:, None] * V - U @ B, 2)
    orth = max(np.linalg.norm(U.T @ U - I, 2), np.linalg.norm(V.T @ V - I, 2))
    delta = 2.0 * (res + float(np.max(sigma)) * orth)
    return d, e, delta


def dense_normal(m: int, n: int, seed: int) -> np.ndarray:
    """A dense m x n matrix with iid N(0, 1) entries, drawn in row-major
    order (the inputs of the dense routines that surround the bidiagonal
    solver: QR of a tall matrix, bidiagonal reduction)."""
    return _rng(seed).standard_normal((m, n))


# Seeds of the dense workloads: the tall-and-skinny matrix of Section 5.1
# (m = 20000, n = 1000) and the square matrices of the reduction.
DENSE_TS_SEED = BASE_SEED + 700
DENSE_SQUARE_SEED = BASE_SEED + 800


# Named workloads (sizes and spectra of the measured configurations).
def workload(name: str) -> tuple[np.ndarray, np.ndarray]:
    if name == "n256_uniform":
        return uniform(256, seed_for(1))
    if name == "n4096_uniform":
        return uniform(4096, seed_for(2, 0))
    if name == "n4096_graded":
        return graded(4096, seed_for(2, 1))
    if name == "n4096_clustered":
        return clustered(4096, seed_for(2, 2))
    if name == "n16384_normal":
        return normal(16384, seed_for(3))
    if name == "n32768_normal":
        return normal(32768, seed_for(5))
    if name == "n16384_ones":
        return ones(16384)
    raise KeyError(name)
