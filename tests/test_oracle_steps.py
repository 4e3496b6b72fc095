"""Pins of each oracle step against references independent of it (CPU)."""

import math
import os

import numpy as np
import pytest

import oracle
from oracle import bdc as obdc
from paper_2508_11467_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- tree
@pytest.mark.parametrize("n,leaf", [(1, 32), (32, 32), (33, 32), (64, 32), (65, 32),
                                    (256, 32), (1000, 32), (4096, 32), (100, 4), (37, 5)])
def test_tree_sizes(n, leaf):
    root = oracle.build_tree(n, leaf)
    nodes = oracle.tree_nodes(root)
    leaves = [x for x in nodes if x.is_leaf]
    merges = [x for x in nodes if not x.is_leaf]
    # every row of B is a leaf row or the middle row of exactly one merge
    assert sum(x.m for x in leaves) + len(merges) == n
    for x in merges:
        assert x.m == x.left.m + 1 + x.right.m
        assert x.m + x.s == (x.left.m + x.left.s) + (x.right.m + x.right.s)
        assert x.left.s == 1 and x.right.s == x.s
        assert x.k == x.m // 2
    for x in leaves:
        assert 1 <= x.m <= leaf
    rows = sorted(sum([list(range(x.r0, x.r0 + x.m)) for x in leaves], []) +
                  [x.r0 + x.k - 1 for x in merges])
    assert rows == list(range(n))


# ---------------------------------------------------------------- leaf
def _leaf_input(m, s, seed):
    g = np.random.default_rng(seed)
    return g.uniform(-1, 1, m), g.uniform(-1, 1, m - 1 + s)


@pytest.mark.parametrize("m", [1, 2, 3, 7, 31, 32])
@pytest.mark.parametrize("s", [0, 1])
def test_leaf_against_numpy_svd(m, s):
    d, e = _leaf_input(m, s, 100 * m + s)
    B = obdc.dense_bidiagonal(d, e, s)
    sig, W, Q, _ = oracle.leaf_svd(d, e, s)
    ref = np.sort(np.linalg.svd(B, compute_uv=False))
    scale = max(ref[-1], 1e-300)
    assert np.all(np.diff(sig) >= 0)
    assert np.max(np.abs(sig - ref)) <= 1e-14 * scale
    S = np.zeros((m, m + s))
    S[np.arange(m), np.arange(m)] = sig
    assert np.linalg.norm(B - W @ S @ Q.T) <= 1e-14 * np.linalg.norm(B)
    assert np.max(np.abs(W.T @ W - np.eye(m))) <= 1e-14
    assert np.max(np.abs(Q.T @ Q - np.eye(m + s))) <= 1e-14
    if s == 1:
        assert np.linalg.norm(B @ Q[:, m]) <= 1e-14 * np.linalg.norm(B)


@pytest.mark.parametrize("case", ["zero_diag_mid", "zero_diag_last", "zero_e", "all_zero", "graded", "huge", "tiny"])
def test_leaf_special(case):
    m, s = 12, 1
    d, e = _leaf_input(m, s, 7)
    if case == "zero_diag_mid":
        d[4] = 0.0
    elif case == "zero_diag_last":
        d[m - 1] = 0.0
        s = 0
        e = e[: m - 1]
    elif case == "zero_e":
        e[3] = 0.0
        e[7] = 0.0
    elif case == "all_zero":
        d[:] = 0.0
        e[:] = 0.0
    elif case == "graded":
        d = d * 10.0 ** (-np.arange(m))
    elif case == "huge":
        d = d * 1e300
        e = e * 1e300
    elif case == "tiny":
        d = d * 1e-300
        e = e * 1e-300
    B = obdc.dense_bidiagonal(d, e, s)
    sig, W, Q, _ = oracle.leaf_svd(d, e, s)
    # compare in units of the largest entry (numpy's SVD is scale-safe)
    unit = max(float(np.max(np.abs(B))), 1e-320)
    ref = np.sort(np.linalg.svd(B / unit, compute_uv=False))
    Bn = B / unit
    nb = max(np.linalg.norm(Bn), 1e-300)
    assert np.max(np.abs(sig / unit - ref)) <= 1e-14 * max(ref[-1], 1e-300) + 1e-300
    S = np.zeros((m, m + s))
    S[np.arange(m), np.arange(m)] = sig / unit
    assert np.linalg.norm(Bn - W @ S @ Q.T) <= 1e-14 * nb
    assert np.max(np.abs(W.T @ W - np.eye(m))) <= 1e-14
    assert np.max(np.abs(Q.T @ Q - np.eye(m + s))) <= 1e-14


# ---------------------------------------------------------------- z and bases
def _child_svd(d, e, r0, m, s):
    """Children's SVD from numpy (independent of the oracle): values
    ascending, W (m x m), [Q q] ((m+s) x (m+s)), null column last."""
    B = obdc.dense_bidiagonal(d[r0:r0 + m], e[r0:r0 + m - 1 + s], s)
    u, sv, vt = np.linalg.svd(B, full_matrices=True)
    order = np.argsort(sv)
    W = u[:, order]
    Q = np.empty((m + s, m + s))
    Q[:, :m] = vt[order, :].T
    if s == 1:
        Q[:, m] = vt[m, :]
    return sv[order], W, Q


@pytest.mark.parametrize("n,s,seed", [(9, 0, 1), (10, 1, 2), (65, 0, 3), (256, 0, 4), (131, 1, 5)])
def test_z_and_bases_reproduce_M(n, s, seed):
    """Lbas^T B_node Rbas = [M | 0], M = e_1 z^T + diag(d) (eqs. bdc-B,
    diag-one-side-M): checks z, (c0, s0) and the placement of x1 and y."""
    g = np.random.default_rng(seed)
    d = g.uniform(-1, 1, n)
    e = g.uniform(-1, 1, n - 1 + s)
    k = n // 2
    m2 = n - k
    sig1, W1, Q1 = _child_svd(d, e, 0, k - 1, 1)
    sig2, W2, Q2 = _child_svd(d, e, k, m2, s)
    pr = oracle.merge_prep(sig1, sig2, Q1[k - 1, :], Q2[0, :], d[k - 1], e[k - 1], s)
    Bn = obdc.dense_bidiagonal(d, e, s) / pr.scale
    L = np.zeros((n, n))
    L[:k - 1, :k - 1] = W1
    L[k - 1, k - 1] = 1.0
    L[k:, k:] = W2
    R = np.zeros((n + s, n + s))
    R[:k, :k - 1] = Q1[:, :k - 1]
    R[k:, k:n] = Q2[:, :m2]
    q1 = np.zeros(n + s)
    q1[:k] = Q1[:, k - 1]
    q2 = np.zeros(n + s)
    if s:
        q2[k:] = Q2[:, m2]
    R[:, k - 1] = pr.c0 * q1 + pr.s0 * q2
    if s:
        R[:, n] = -pr.s0 * q1 + pr.c0 * q2
    M = np.diag(pr.d_local)
    M[k - 1, :] += pr.z_local
    got = L.T @ Bn @ R
    want = np.zeros((n, n + s))
    want[:, :n] = M
    assert np.max(np.abs(got - want)) <= 1e-14 * max(1.0, np.max(np.abs(Bn)))
    assert pr.z_local[k - 1] >= 0.0
    assert abs(pr.c0 ** 2 + pr.s0 ** 2 - 1.0) <= 4e-16


def test_scale_is_power_of_two():
    for v in [1.0, 0.75, 3.0, 1e-300, 1e300, 2.0 ** -1074]:
        p = oracle.scale_of([v, -v / 3])
        assert math.frexp(p)[0] == 0.5
        assert 0.5 <= v / p < 1.0
    assert oracle.scale_of([0.0, 0.0]) == 1.0


# ---------------------------------------------------------------- sort
@pytest.mark.parametrize("seed", range(5))
def test_merge_sort_matches_stable_argsort(seed):
    g = np.random.default_rng(seed)
    k = int(g.integers(2, 40))
    m2 = int(g.integers(1, 40))
    pool = np.round(g.uniform(0, 1, 8), 2)          # force many ties
    left = np.sort(g.choice(pool, k - 1))
    right = np.sort(g.choice(pool, m2))
    dloc = np.concatenate([left, [0.0], right])
    perm = oracle.merge_sort_order(dloc, k)
    cols = np.concatenate([np.arange(k - 1), np.arange(k, k + m2)])
    ref = cols[np.argsort(dloc[cols], kind="stable")]
    assert perm[0] == k - 1
    assert np.array_equal(perm[1:], ref)


# ---------------------------------------------------------------- deflation
def _golden_deflation():
    rows = []
    with open(os.path.join(GOLDEN, "deflation_n3.txt")) as f:
        for line in f:
            if line.startswith("#"):
                continue
            parts = [p.strip() for p in line.split("|")]
            name = parts[0]
            vals = [np.array([float(x) for x in p.split()]) for p in parts[1:5]]
            st = np.array([int(x) for x in parts[5].split()])
            rows.append((name, *vals, st))
    return rows


@pytest.mark.parametrize("row", _golden_deflation(), ids=lambda r: r[0])
def test_deflation_paper_examples(row):
    name, d, z, ed, ez, est = row
    d = d.copy()
    z = z.copy()
    tol, status, rots = oracle.deflate(d, z)
    assert tol == 2.0 ** -50
    assert np.array_equal(status[1:], est[1:])
    assert np.array_equal(d, ed)
    assert np.max(np.abs(z - ez)) <= 2.0 ** -53 * np.max(np.abs(ez))


def _dense_M(d, z):
    M = np.diag(np.asarray(d, dtype=np.float64))
    M[0, :] += z
    return M


@pytest.mark.parametrize("seed", range(6))
def test_deflation_PMQ(seed):
    """P M Q = diag(M_1, D) + O(tol): applying the recorded rotations to the
    original M gives the deflated M up to a few tol per deflation."""
    g = np.random.default_rng(seed)
    N = 40
    base = np.sort(g.uniform(0, 1, N - 1))
    d = np.concatenate([[0.0], base])
    # plant close pairs, near-zero values and tiny z
    d[5] = d[4] + 1e-18
    d[17] = d[16]
    d[1] = 1e-19
    d = np.sort(d)
    d[0] = 0.0
    z = g.uniform(-1, 1, N)
    z[9] = 1e-20
    z[25] = -3e-19
    d0, z0 = d.copy(), z.copy()
    tol, status, rots = oracle.deflate(d, z)
    assert np.sum(status == oracle.DEFL_CLOSE) >= 2
    assert np.sum(status == oracle.DEFL_ZERO_D) >= 1
    assert np.sum(status == oracle.DEFL_SMALL_Z) >= 2
    M = _dense_M(d0, z0)
    Gl = np.eye(N)
    Gr = np.eye(N)
    for kind, p, j, c, s in rots:
        G = np.eye(N)
        G[p, p] = c
        G[p, j] = s
        G[j, p] = -s
        G[j, j] = c
        Gr = G @ Gr
        if kind == oracle.DEFL_CLOSE:
            Gl = G @ Gl
    got = Gl @ M @ Gr.T
    want = _dense_M(d, z)
    ndefl = int(np.sum(status != 0)) + 1
    assert np.max(np.abs(got - want)) <= 4 * tol * ndefl
    # survivors satisfy eq. M-condition
    sv = np.array([0] + [j for j in range(1, N) if status[j] == 0])
    assert np.all(np.diff(d[sv]) >= tol)
    assert np.all(np.abs(z[sv]) >= tol)


# ---------------------------------------------------------------- secular
def _random_arrow(N, seed, spread=1.0):
    g = np.random.default_rng(seed)
    d = np.concatenate([[0.0], np.sort(g.uniform(0.01, 1.0, N - 1) * spread)])
    d[1:] = np.maximum.accumulate(d[1:] + np.arange(N - 1) * 1e-9)
    z = g.uniform(-1, 1, N) * 0.3
    z[0] = abs(z[0]) + 1e-3
    return d, z


@pytest.mark.parametrize("N,seed", [(1, 0), (2, 1), (3, 2), (17, 3), (64, 4), (200, 5)])
def test_secular_against_eigvalsh(N, seed):
    d, z = _random_arrow(N, seed)
    o, tau, it = oracle.secular_roots(d, z)
    omega = d[o] + tau
    ref = np.sqrt(np.linalg.eigvalsh(np.diag(d * d) + np.outer(z, z)))
    assert np.max(np.abs(omega - ref)) <= 1e-14 * ref[-1]
    # interlacing and origin = a bounding pole
    assert np.all(omega[:-1] > d[:-1]) and np.all(omega[:-1] < d[1:])
    assert omega[-1] > d[-1]
    assert np.all((o == np.arange(N)) | (o == np.minimum(np.arange(N) + 1, N - 1)))
    assert np.all(it <= 64)


@pytest.mark.parametrize("seed", range(3))
def test_secular_sign_change(seed):
    """f changes sign within a few ulps of tau around each computed root."""
    d, z = _random_arrow(30, seed)
    o, tau, _ = oracle.secular_roots(d, z)

    def f(i, t):
        dd = (d - d[o[i]] - t) * (d + d[o[i]] + t)
        return 1.0 + np.sum(z * z / dd)

    for i in range(len(d)):
        t = tau[i]
        h = 16 * np.spacing(abs(t))
        assert f(i, t - h) <= 1e-13 * 30 and f(i, t + h) >= -1e-13 * 30


# ---------------------------------------------------------------- Loewner + vectors
@pytest.mark.parametrize("N,seed", [(2, 0), (5, 1), (50, 2), (180, 3)])
def test_lowner_exactness(N, seed):
    """The computed roots are the exact singular values of M~ built from z~
    (eq. bdc-zi), and z~ is close to z."""
    d, z = _random_arrow(N, seed)
    o, tau, _ = oracle.secular_roots(d, z)
    omega = d[o] + tau
    zt = oracle.lowner_z(d, z, o, tau)
    Mt = _dense_M(d, zt)
    sv = np.sort(np.linalg.svd(Mt, compute_uv=False))
    # numpy's dense SVD is accurate to a few eps * ||M~|| (absolute)
    assert np.max(np.abs(sv - omega)) <= 2e-15 * omega[-1]
    assert np.linalg.norm(zt - z) <= 1e-13 * np.linalg.norm(z)
    assert np.all(np.sign(zt) == np.sign(z))


@pytest.mark.parametrize("N,seed", [(1, 0), (2, 1), (7, 2), (120, 3)])
def test_vectors_orthogonal_and_singular(N, seed):
    d, z = _random_arrow(N, seed)
    o, tau, _ = oracle.secular_roots(d, z)
    omega = d[o] + tau
    zt = oracle.lowner_z(d, z, o, tau)
    U, V = oracle.vectors(d, zt, o, tau)
    assert np.max(np.abs(U.T @ U - np.eye(N))) <= 1e-14
    assert np.max(np.abs(V.T @ V - np.eye(N))) <= 1e-14
    Mt = _dense_M(d, zt)
    assert np.max(np.abs(Mt @ V - U * omega[None, :])) <= 1e-14 * omega[-1]


def test_merge_values_is_stable_merge():
    g = np.random.default_rng(3)
    pool = np.arange(10) / 10
    om = np.sort(g.choice(pool, 15))
    dv = np.sort(g.choice(pool, 9))
    dr, dd = oracle.merge_values(om, dv)
    allv = np.concatenate([om, dv])
    grp = np.concatenate([np.zeros(15), np.ones(9)])
    order = np.lexsort((np.arange(24), grp, allv))
    dest = np.empty(24, dtype=np.int64)
    dest[order] = np.arange(24)
    assert np.array_equal(dr, dest[:15]) and np.array_equal(dd, dest[15:])
