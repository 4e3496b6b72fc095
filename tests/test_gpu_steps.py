"""Each merge stage on the GPU against the oracle on identical inputs."""

import numpy as np
import pytest

import oracle
from oracle import bdc as obdc

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def solver(gpu):
    from paper_2508_11467_amd.api import Solver
    s = Solver(0)
    yield s
    s.close()


# ---------------------------------------------------------------- GEMM
@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (16, 16, 4), (64, 64, 16), (100, 37, 53), (130, 200, 70),
                                   (5, 300, 1), (257, 3, 129)])
def test_gemm_matches_numpy(solver, M, N, K):
    import torch
    g = np.random.default_rng(M * 1000 + N * 10 + K)
    A = g.standard_normal((M, K))
    B = g.standard_normal((K, N))
    C = solver.step_gemm(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()).cpu().numpy()
    ref = A @ B
    scale = np.abs(A) @ np.abs(B)
    assert np.all(np.abs(C - ref) <= 4 * K * 2.0 ** -53 * scale + 1e-300)


# ---------------------------------------------------------------- leaf
@pytest.mark.parametrize("m", [1, 2, 3, 8, 17, 31, 32])
@pytest.mark.parametrize("s", [0, 1])
def test_leaf_matches_oracle(solver, m, s):
    g = np.random.default_rng(10 * m + s)
    d = g.uniform(-1, 1, m)
    e = g.uniform(-1, 1, m - 1 + s)
    sig, W, Q = solver.step_leaf(d, e, s)
    sig, W, Q = sig.cpu().numpy(), W.cpu().numpy(), Q.cpu().numpy()
    ref, _, _, _ = oracle.leaf_svd(d, e, s)
    B = obdc.dense_bidiagonal(d, e, s)
    assert np.all(np.diff(sig) >= 0)
    assert np.max(np.abs(sig - ref)) <= 1e-14 * max(ref[-1], 1e-300)
    S = np.zeros((m, m + s))
    S[np.arange(m), np.arange(m)] = sig
    assert np.linalg.norm(B - W @ S @ Q.T) <= 1e-14 * np.linalg.norm(B)
    assert np.max(np.abs(W.T @ W - np.eye(m))) <= 1e-14
    assert np.max(np.abs(Q.T @ Q - np.eye(m + s))) <= 1e-14


@pytest.mark.parametrize("case", ["zero_diag_mid", "zero_diag_last", "zero_e", "all_zero", "graded", "huge", "tiny"])
def test_leaf_special(solver, case):
    m, s = 20, 1
    g = np.random.default_rng(7)
    d = g.uniform(-1, 1, m)
    e = g.uniform(-1, 1, m)
    if case == "zero_diag_mid":
        d[4] = 0.0
    elif case == "zero_diag_last":
        d[m - 1] = 0.0
        s = 0
        e = e[: m - 1]
    elif case == "zero_e":
        e[3] = e[11] = 0.0
    elif case == "all_zero":
        d[:] = 0.0
        e[:] = 0.0
    elif case == "graded":
        d = d * 10.0 ** (-np.arange(m) / 2)
    elif case == "huge":
        d *= 1e300
        e *= 1e300
    elif case == "tiny":
        d *= 1e-300
        e *= 1e-300
    sig, W, Q = solver.step_leaf(d, e, s)
    sig, W, Q = sig.cpu().numpy(), W.cpu().numpy(), Q.cpu().numpy()
    ref, _, _, _ = oracle.leaf_svd(d, e, s)
    B = obdc.dense_bidiagonal(d, e, s)
    unit = max(float(np.max(np.abs(B))), 1e-320)
    assert np.max(np.abs(sig - ref) / unit) <= 1e-14 * max(ref[-1] / unit, 1e-300) + 1e-300
    assert np.max(np.abs(W.T @ W - np.eye(m))) <= 1e-14
    assert np.max(np.abs(Q.T @ Q - np.eye(m + s))) <= 1e-14
    Bn = B / unit
    S = np.zeros((m, m + s))
    S[np.arange(m), np.arange(m)] = sig / unit
    assert np.linalg.norm(Bn - W @ S @ Q.T) <= 1e-14 * max(np.linalg.norm(Bn), 1e-300)


# ---------------------------------------------------------------- deflation (bit exact)
def _children(n, s, seed, kind="uniform"):
    """Inputs of one merge from numpy SVDs of the children of a bidiagonal."""
    g = np.random.default_rng(seed)
    if kind == "uniform":
        d = g.uniform(-1, 1, n)
        e = g.uniform(-1, 1, n - 1 + s)
    elif kind == "ones":
        d = np.ones(n)
        e = np.ones(n - 1 + s)
    elif kind == "mirror":
        # n = 2k, s = 0: the right child is the left child over a zero row,
        # so the two children share k-1 values (close-pair deflation)
        k = n // 2
        d = np.zeros(n)
        e = np.zeros(n - 1)
        d[: k - 1] = g.uniform(-1, 1, k - 1)
        e[: k - 2] = g.uniform(-1, 1, k - 2)
        e[k - 2] = 0.35
        d[k - 1] = 0.7
        e[k - 1] = -0.4
        d[k: 2 * k - 1] = d[: k - 1]
        e[k: 2 * k - 2] = e[: k - 2]
        e[2 * k - 2] = 0.35
    elif kind == "zeros":
        d = g.uniform(-1, 1, n)
        e = g.uniform(-1, 1, n - 1 + s)
        d[3::7] = 0.0
        e[5::11] = 0.0
    k = n // 2
    m2 = n - k
    B = obdc.dense_bidiagonal(d, e, s)
    B1 = B[: k - 1, : k]
    B2 = B[k:, k:]
    u1, s1, v1 = np.linalg.svd(B1, full_matrices=True)
    u2, s2, v2 = np.linalg.svd(B2, full_matrices=True)
    o1 = np.argsort(s1, kind="stable")
    o2 = np.argsort(s2, kind="stable")
    Q1 = np.empty((k, k))
    Q1[:, : k - 1] = v1[o1, :].T
    Q1[:, k - 1] = v1[k - 1, :]
    Q2 = np.empty((m2 + s, m2 + s))
    Q2[:, :m2] = v2[o2, :].T
    if s:
        Q2[:, m2] = v2[m2, :]
    sig1 = s1[o1]
    sig2 = s2[o2]
    return sig1, sig2, Q1[k - 1, :].copy(), Q2[0, :].copy(), d[k - 1], e[k - 1]


@pytest.mark.parametrize("n,s,seed,kind", [
    (9, 0, 1, "uniform"), (10, 1, 2, "uniform"), (65, 0, 3, "uniform"), (256, 0, 4, "uniform"),
    (131, 1, 5, "uniform"), (1000, 0, 6, "uniform"), (3001, 1, 7, "uniform"),
    (64, 0, 8, "ones"), (101, 1, 9, "ones"), (40, 0, 10, "mirror"), (80, 0, 11, "mirror"),
    (300, 0, 12, "zeros"), (301, 1, 13, "zeros"),
    # merges of at least 2048 rows take the 1024-thread deflation kernel
    (2500, 0, 14, "zeros"), (2048, 1, 15, "ones"), (2400, 0, 16, "mirror"),
])
def test_deflation_bit_exact(solver, n, s, seed, kind):
    sig1, sig2, q1, q2, alpha, beta = _children(n, s, seed, kind)
    k = n // 2
    pr = oracle.merge_prep(sig1, sig2, q1, q2, alpha, beta, s)
    sig = np.concatenate([sig1, [0.0], sig2])
    got = solver.step_deflate(n, s, sig, q1, q2, alpha, beta)
    assert got["scale"] == pr.scale
    assert got["tol"] == pr.tol
    assert got["c0"] == pr.c0 and got["s0"] == pr.s0
    assert np.array_equal(got["perm"], pr.perm)
    assert np.array_equal(got["d"], pr.d)
    assert np.array_equal(got["z"], pr.z)
    st = got["status"].copy()
    st[0] = 0
    assert np.array_equal(st, pr.status)
    assert got["N"] == len(pr.survivors)
    assert got["counts"] == pr.counts
    assert got["rot_pos"].shape[0] == len(pr.rots)
    for (kind_, p, j, c, sn), pos, cs in zip(pr.rots, got["rot_pos"], got["rot_cs"]):
        assert (p, j) == (pos[0], pos[1])
        assert (kind_ == oracle.DEFL_ZERO_D) == (pos[0] == 0)
        assert (c, sn) == (cs[0], cs[1])


def _synthetic_children(n, s, seed):
    """Merge inputs drawn directly (no child SVDs, so any size is cheap): a
    fifth of the right child's values copied from the left child (close
    pairs), values at the rounding level (d ~ 0), a quarter of each child's
    null-vector entries scaled by 1e-17 (small z)."""
    g = np.random.default_rng(seed)
    k = n // 2
    m2 = n - k
    sig1 = np.sort(g.uniform(0, 2, k - 1))
    sig2 = g.uniform(0, 2, m2)
    shared = g.choice(m2, size=min(m2, k - 1) // 5, replace=False)
    sig2[shared] = sig1[g.choice(k - 1, size=shared.size, replace=False)]
    sig1[:3] = [0.0, 1e-18, 3e-17]
    sig2[:2] = [0.0, 2e-17]
    sig1 = np.sort(sig1)
    sig2 = np.sort(sig2)
    q1 = g.normal(size=k)
    q1 /= np.linalg.norm(q1)
    q2 = g.normal(size=m2 + s)
    q2 /= np.linalg.norm(q2)
    q1[g.choice(k - 1, size=k // 4, replace=False)] *= 1e-17
    q2[g.choice(m2, size=m2 // 4, replace=False)] *= 1e-17
    return sig1, sig2, q1, q2, g.uniform(-1, 1), g.uniform(-1, 1)


# sizes through every launch shape of the deflation kernel: one wavefront
# (up to 64, 128, 256 values), 4 wavefronts, 16 wavefronts with 4, 8 and 16
# steps per lane, and beyond 16384 values
@pytest.mark.parametrize("n,s,seed", [
    (40, 0, 21), (100, 1, 22), (250, 0, 23), (700, 1, 24), (1900, 0, 25), (3500, 1, 26),
    (6000, 0, 27), (12000, 1, 28), (16384, 0, 29), (20000, 0, 30),
])
def test_deflation_bit_exact_synthetic(solver, n, s, seed):
    sig1, sig2, q1, q2, alpha, beta = _synthetic_children(n, s, seed)
    pr = oracle.merge_prep(sig1, sig2, q1, q2, alpha, beta, s)
    assert set(np.unique(pr.status[1:]).tolist()) == {0, 1, 2, 3}
    sig = np.concatenate([sig1, [0.0], sig2])
    got = solver.step_deflate(n, s, sig, q1, q2, alpha, beta)
    assert got["tol"] == pr.tol
    assert np.array_equal(got["perm"], pr.perm)
    assert np.array_equal(got["d"], pr.d)
    assert np.array_equal(got["z"], pr.z)
    st = got["status"].copy()
    st[0] = 0
    assert np.array_equal(st, pr.status)
    assert got["N"] == len(pr.survivors)
    assert got["counts"] == pr.counts
    assert got["rot_pos"].shape[0] == len(pr.rots)
    pos = np.array([(p, j) for _, p, j, _, _ in pr.rots])
    cs = np.array([(c, sn) for _, _, _, c, sn in pr.rots])
    assert np.array_equal(got["rot_pos"], pos)
    assert np.array_equal(got["rot_cs"], cs)


def test_deflation_exercises_all_cases(solver):
    """The bit-exact cases above cover every deflation branch."""
    seen = set()
    for n, s, seed, kind in [(40, 0, 10, "mirror"), (300, 0, 12, "zeros"), (1000, 0, 6, "uniform")]:
        sig1, sig2, q1, q2, alpha, beta = _children(n, s, seed, kind)
        pr = oracle.merge_prep(sig1, sig2, q1, q2, alpha, beta, s)
        seen |= set(np.unique(pr.status[1:]).tolist())
    assert seen == {0, 1, 2, 3}


# ---------------------------------------------------------------- secular
def _arrow(N, seed):
    g = np.random.default_rng(seed)
    d = np.concatenate([[0.0], np.sort(g.uniform(0.01, 1.0, N - 1))])
    z = g.uniform(-1, 1, N) * 0.3
    z[0] = abs(z[0]) + 1e-3
    return d, z


def _secular_residual(d, z, o, tau):
    LD = np.longdouble
    dl = d.astype(LD)
    zl = z.astype(LD)
    f = np.empty(len(d), dtype=LD)
    E = np.empty(len(d), dtype=LD)
    for i in range(len(d)):
        do = dl[o[i]]
        t = LD(tau[i])
        delta = (dl - do - t) * (dl + do + t)
        terms = zl * zl / delta
        f[i] = 1 + np.sum(terms)
        E[i] = 1 + np.sum(np.abs(terms))
    return f.astype(np.float64), E.astype(np.float64)


def test_secular_residual_pins_oracle():
    d, z = _arrow(500, 5)
    o, tau, _ = oracle.secular_roots(d, z)
    f, E = _secular_residual(d, z, o, tau)
    assert np.all(np.abs(f) <= 32 * 2.0 ** -52 * E)


@pytest.fixture(scope="module")
def solver_lanes(gpu):
    """A handle whose secular problems of up to 256 roots take the
    lanes-per-root kernel (8 lanes up to 64 values, else 16)."""
    from paper_2508_11467_amd.api import Solver
    s = Solver(0)
    s.set_tuning(small_n=96, flat=0, grid64=1024, grid128=512, sec_small_n=256)
    yield s
    s.close()


@pytest.mark.parametrize("kernel", ["wide", "lanes"])
@pytest.mark.parametrize("N,seed", [(1, 0), (2, 1), (3, 2), (9, 7), (33, 8), (64, 3), (65, 4), (130, 9),
                                    (256, 10), (257, 11), (500, 5), (3000, 6)])
def test_secular_matches_oracle(solver, solver_lanes, kernel, N, seed):
    d, z = _arrow(N, seed)
    s = solver if kernel == "wide" else solver_lanes
    keep = s.tuning()
    s.set_tuning(small_n=96, flat=0, grid64=1024, grid128=512, sec_small_n=0 if kernel == "wide" else 256)
    try:
        o, tau, it = s.step_secular(d, z)
    finally:
        s.set_tuning(**{k: keep[k] for k in ("small_n", "flat", "grid64", "grid128", "sec_small_n")})
    o, tau, it = o.cpu().numpy(), tau.cpu().numpy(), it.cpu().numpy()
    ro, rt, rit = oracle.secular_roots(d, z)
    w = d[o] + tau
    rw = d[ro] + rt
    assert np.max(np.abs(w - rw)) <= 1e-14 * rw[-1]
    same = o == ro
    assert np.mean(same) >= 0.99
    # each GPU root solves the secular equation to the stopping rule's
    # accuracy, f evaluated in extended precision at (o, tau)
    f, E = _secular_residual(d, z, o, tau)
    assert np.all(np.abs(f) <= 32 * 2.0 ** -52 * E)
    assert np.all(it <= 64)
    if N > 1:
        assert abs(np.mean(it) - np.mean(rit)) <= 0.5


# ---------------------------------------------------------------- Loewner + vectors
@pytest.mark.parametrize("N,seed", [(1, 0), (2, 1), (7, 2), (200, 3), (1500, 4)])
def test_vectors_match_oracle(solver, N, seed):
    d, z = _arrow(N, seed)
    o, tau, _ = oracle.secular_roots(d, z)
    zt_ref = oracle.lowner_z(d, z, o, tau)
    U_ref, V_ref = oracle.vectors(d, zt_ref, o, tau)
    zt, U, V = solver.step_vectors(d, z, o, tau)
    zt, U, V = zt.cpu().numpy(), U.cpu().numpy(), V.cpu().numpy()
    assert np.all(np.abs(zt - zt_ref) <= 1e-13 * np.abs(zt_ref))
    assert np.max(np.abs(U - U_ref)) <= 1e-12
    assert np.max(np.abs(V - V_ref)) <= 1e-12
    assert np.max(np.abs(U.T @ U - np.eye(N))) <= 1e-13
    assert np.max(np.abs(V.T @ V - np.eye(N))) <= 1e-13
