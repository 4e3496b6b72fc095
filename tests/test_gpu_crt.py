"""Split-precision products on the int8 matrix cores (Chinese remainder
theorem over int8 residues) against exact arithmetic."""

import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

MODULI = [255, 253, 251, 247, 241, 239, 233, 229, 227, 223, 217, 211, 199, 197, 193, 191]
EPS = 2.0 ** -53


@pytest.fixture(scope="module")
def solver(gpu):
    from paper_2508_11467_amd.api import Solver
    s = Solver(0)
    yield s
    s.close()


def beta(L, K):
    """Largest beta <= 55 with P 2^(2 beta) <= (M - 1) / 2, P = K rounded up
    to 64, M the product of the first L moduli (the exactness condition of
    the rebuilt integer product; 55 keeps the scaled operands within the
    seven bytes the residues are taken from)."""
    P = max(64, -(-K // 64) * 64)
    lg = sum(math.log2(m) for m in MODULI[:L])
    return min(55, math.floor((lg - 1.0 - math.ceil(math.log2(P)) - 1e-9) / 2.0))


def bound(A, B, L):
    """Each entry of A is rounded at half a unit of 2^(e_i + 1 - beta), e_i the
    exponent of row i's largest |entry| (likewise the columns of B), so
    |C - AB| <= 2^-beta (2 max_i sum_k |B_kj| + 2 max_j sum_k |A_ik|), plus the
    rounding of the rebuilt integer's Horner sum and of the result."""
    K = A.shape[1]
    b = beta(L, K)
    ra = np.max(np.abs(A), axis=1)
    cb = np.max(np.abs(B), axis=0)
    t = 2.0 ** -b * (np.outer(ra, np.sum(np.abs(B), axis=0)) + np.outer(np.sum(np.abs(A), axis=1), cb))
    return 1.01 * t + 32 * EPS * (np.abs(A) @ np.abs(B)) + 1e-300


def exact(A, B):
    return (A.astype(np.longdouble) @ B.astype(np.longdouble)).astype(np.float64)


@pytest.mark.parametrize("L", [13, 14, 15, 16])
@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (37, 29, 61), (128, 128, 64), (300, 200, 777), (129, 257, 1000),
                                   (64, 700, 130)])
def test_gemm_crt_bound(solver, L, M, N, K):
    import torch
    g = np.random.default_rng(M * 1000 + N + K + L)
    A = g.standard_normal((M, K)) * 10.0 ** g.uniform(-3, 3, (M, 1))
    B = g.standard_normal((K, N)) * 10.0 ** g.uniform(-3, 3, (1, N))
    A[g.uniform(size=A.shape) < 0.1] = 0.0
    C = solver.step_gemm_crt(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(), L).cpu().numpy()
    err = np.abs(C - exact(A, B))
    bd = bound(A, B, L)
    assert np.all(err <= bd), float(np.max(err / bd))


def test_gemm_crt_integers_exact(solver):
    """Integer operands whose products and sums are exact in FP64: the result
    is the exact integer product, bit for bit, for every number of moduli."""
    import torch
    g = np.random.default_rng(9)
    A = g.integers(-1000, 1001, (150, 333)).astype(np.float64)
    B = g.integers(-1000, 1001, (333, 141)).astype(np.float64)
    ref = A @ B  # |entries| < 333 * 10^6 < 2^53: exact in FP64
    At, Bt = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    for L in (13, 14, 15, 16):
        C = solver.step_gemm_crt(At, Bt, L).cpu().numpy()
        assert np.array_equal(C, ref), L


def test_gemm_crt_extreme_scales_and_zero_rows(solver):
    """Rows and columns spanning 10^-200 .. 10^200, an all-zero row and an
    all-zero column: the power-of-two scales keep each one's relative
    accuracy."""
    import torch
    g = np.random.default_rng(10)
    M, N, K = 96, 80, 300
    A = g.standard_normal((M, K)) * 10.0 ** np.linspace(-200, 200, M)[:, None]
    B = g.standard_normal((K, N)) * 10.0 ** np.linspace(100, -100, N)[None, :]
    A[5] = 0.0
    B[:, 7] = 0.0
    C = solver.step_gemm_crt(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(), 16).cpu().numpy()
    ref = exact(A, B)
    assert np.all(C[5] == 0.0) and np.all(C[:, 7] == 0.0)
    rel = np.abs(C - ref) / (np.abs(A) @ np.abs(B) + 1e-300)
    assert np.max(rel) <= 1e-14


def test_gemm_crt_more_accurate_than_fp64(solver):
    """With 16 moduli the rounding is at about 2^-54 of each row's largest
    entry: the error is below the FP64 matrix-core product's."""
    import torch
    g = np.random.default_rng(4)
    A = g.standard_normal((512, 4096))
    B = g.standard_normal((4096, 300))
    At, Bt = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    C = solver.step_gemm_crt(At, Bt, 16).cpu().numpy()
    C64 = solver.step_gemm(At, Bt).cpu().numpy()
    ref = exact(A, B)
    scale = np.abs(A) @ np.abs(B)
    e_crt = np.max(np.abs(C - ref) / scale)
    e_64 = np.max(np.abs(C64 - ref) / scale)
    print(f"crt {e_crt:.2e} fp64 {e_64:.2e}", flush=True)
    assert e_crt <= e_64, (e_crt, e_64)


# ---------------------------------------------------------------- whole solves
def _checks(d, e, sig, U, VT):
    import oracle
    ref, _, _ = oracle.bdsdc(d, e)
    B = oracle.dense(d, e)
    n = len(d)
    es = np.max(np.abs(sig - ref)) / ref[0]
    res = np.linalg.norm(B - (U * sig) @ VT) / np.linalg.norm(B)
    ou = np.max(np.abs(U.T @ U - np.eye(n)))
    ov = np.max(np.abs(VT @ VT.T - np.eye(n)))
    return es, res, ou, ov


@pytest.mark.parametrize("L", [14, 16])
@pytest.mark.parametrize("name", ["uniform", "ones", "near_ones"])
def test_solve_with_crt_meets_tolerances(gpu, name, L):
    """Whole solves with the int8 residue products on every merge that keeps
    at least 128 values, against the oracle at the FP64 tolerances (the
    uniform spectrum keeps at most 98 values per merge at this size, so there
    the split products never run and the solve is the FP64 one)."""
    import torch

    from paper_2508_11467_amd import inputs
    from paper_2508_11467_amd.api import Solver
    n = 2000
    d, e = {"uniform": lambda: inputs.uniform(n, 3), "ones": lambda: inputs.ones(n),
            "near_ones": lambda: inputs.near_ones(n, 5)}[name]()
    s = Solver(0, gemm="crt", ozaki_min_n=128, crt_moduli=L)
    try:
        sig, U, VT = s.svd(torch.from_numpy(d), torch.from_numpy(e))
        info, st = s.info()
        assert info == 0
        es, res, ou, ov = _checks(d, e, sig.cpu().numpy(), U.cpu().numpy(), VT.cpu().numpy())
        print(f"{name} L={L}: split merges {st['split_merges']} sigma {es:.2e} residual {res:.2e} "
              f"orth {ou:.2e} {ov:.2e}", flush=True)
        if name != "uniform":
            assert st["split_merges"] > 0
        assert es <= 1e-13 and res <= 1e-12 and ou <= 1e-12 and ov <= 1e-12
    finally:
        s.close()


def test_crt_full_size_ones(gpu):
    """n = 16384, d = e = 1 (no deflation: every product is large): all 16384
    singular values against the closed form, residual and orthogonality."""
    import torch

    from paper_2508_11467_amd import inputs
    from paper_2508_11467_amd.api import Solver
    n = 16384
    d, e = inputs.ones(n)
    s = Solver(0, gemm="crt")
    try:
        sig, U, VT = s.svd(torch.from_numpy(d), torch.from_numpy(e))
        info, st = s.info()
        assert info == 0 and st["split_merges"] > 0
        ref = 2.0 * np.cos(np.arange(1, n + 1) * math.pi / (2 * n + 1))
        err = float(np.max(np.abs(sig.cpu().numpy() - ref)) / ref[0])
        I = torch.eye(n, dtype=torch.float64, device="cuda")
        Uc = U.contiguous()
        ou = float(torch.max(torch.abs(Uc.T.contiguous() @ Uc - I)))
        Vc = VT.contiguous()
        ov = float(torch.max(torch.abs(Vc @ Vc.T.contiguous() - I)))
        dt = torch.from_numpy(d).cuda()
        et = torch.from_numpy(np.concatenate([e, [0.0]])).cuda()
        V = VT.T
        BV = dt[:, None] * V
        BV[:-1] += et[:-1, None] * V[1:]
        res = float(torch.linalg.norm(BV - U * sig[None, :])) / math.sqrt(2 * n - 1)
        print(f"crt n=16384 ones: split merges {st['split_merges']} sigma {err:.2e} orth {ou:.2e} {ov:.2e} "
              f"residual {res:.2e}", flush=True)
        assert err <= 1e-13 and ou <= 1e-12 and ov <= 1e-12 and res <= 1e-12
    finally:
        s.close()
