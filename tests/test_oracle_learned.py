"""Pins of the learned-start oracle: the gradient against finite differences,
bfloat16 rounding against torch's conversion, features on a worked example
and their invariances, and the learned-start iteration against the
eigenvalues of the arrow matrix and the plain start."""

import math

import numpy as np
import pytest

from oracle import learned as L
from oracle import secular_roots


def test_parameter_count():
    assert L.NPARAMS == 19 * 64 + 64 + 64 * 64 + 64 + 64 * 64 + 64 + 64 + 1 == 9665
    p = L.mlp_init(3)
    assert np.array_equal(L.flatten(L.unflatten(p)), p)


def test_gelu_special_values():
    assert L.gelu(np.array(0.0)) == 0.0
    assert L.gelu_grad(np.array(0.0)) == 0.5
    big = np.array([30.0, -30.0])
    assert np.allclose(L.gelu(big), [30.0, 0.0], atol=1e-12)
    # odd part: gelu(x) - gelu(-x) = x
    x = np.linspace(-5, 5, 41)
    assert np.allclose(L.gelu(x) - L.gelu(-x), x, atol=1e-15)


def test_gradient_finite_differences():
    """The analytic backward pass against central differences of the loss."""
    g = np.random.default_rng(11)
    p = L.mlp_init(5) + 0.05 * g.standard_normal(L.NPARAMS)
    X = g.uniform(-2, 2, (37, L.NFEAT))
    y = g.uniform(0, 1, 37)
    loss, grad = L.mlp_loss_grad(p, X, y)
    idx = np.concatenate([g.choice(1088, 12, replace=False),            # W1
                          1088 + g.choice(64, 4, replace=False),         # b1
                          1152 + g.choice(4096, 12, replace=False),      # W2
                          5312 + g.choice(4096, 12, replace=False),      # W3
                          9408 + g.choice(64, 4, replace=False),         # b3
                          9472 + g.choice(64, 6, replace=False), [9536]])
    for k in idx:
        h = 1e-6 * max(1.0, abs(p[k]))
        pp, pm = p.copy(), p.copy()
        pp[k] += h
        pm[k] -= h
        fd = (L.mlp_loss_grad(pp, X, y)[0] - L.mlp_loss_grad(pm, X, y)[0]) / (2 * h)
        assert abs(fd - grad[k]) <= 1e-6 * max(1e-3, np.max(np.abs(grad))), (k, fd, grad[k])


def test_bf16_round_against_torch():
    torch = pytest.importorskip("torch")
    g = np.random.default_rng(2)
    x = np.concatenate([g.standard_normal(20000) * 10.0 ** g.uniform(-30, 30, 20000),
                        [0.0, -0.0, 1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 65504.0, 3.4e38, 1e-40]])
    x32 = x.astype(np.float32)
    ref = torch.from_numpy(x32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(L.bf16_round(x32), ref)
    # ties go to the even neighbour
    assert L.bf16_round(np.float32(1.0 + 2 ** -8)) == 1.0
    assert L.bf16_round(np.float32(1.0 + 3 * 2 ** -8)) == 1.0 + 2 ** -6


def test_bf16_network_close_to_f64():
    """Rounding every product operand to bfloat16 (unit roundoff 2^-9) moves
    the output and the gradient by a few of those units per layer."""
    g = np.random.default_rng(4)
    p = L.mlp_init(7)
    X = g.uniform(-2, 2, (200, L.NFEAT))
    y = g.uniform(0, 1, 200)
    x64, _ = L.mlp_forward(p, X, "f64")
    x16, _ = L.mlp_forward(p, X, "bf16")
    assert np.max(np.abs(x64 - x16)) < 0.05
    _, g64 = L.mlp_loss_grad(p, X, y, "f64")
    _, g16 = L.mlp_loss_grad(p, X, y, "bf16")
    assert np.linalg.norm(g64 - g16) <= 0.05 * np.linalg.norm(g64)


FAR1 = math.asinh(1.0) / 8  # far field of a problem with no far poles: v = 1, s = 0


def test_features_worked_example():
    """N = 3, d = (0, 1, 3), z = (1, 2, 2): rho = 9, computed by hand."""
    d = np.array([0.0, 1.0, 3.0])
    z = np.array([1.0, 2.0, 2.0])
    F = L.features(d, z)
    # root 0: lo = 0, hi = 1, h = 1, w2 = 1
    exp0 = [0.0, 0.0, -4, -2, -4, -2, -4, -2,
            1.0, 2 / 32, 3.0, 2 / 32, 5, -2, 5, -2,
            math.log2(9) / 32, FAR1, 0.0]
    assert np.allclose(F[0], exp0, rtol=0, atol=1e-15)
    # root 1: lo = 1, hi = 3, h = 2, w2 = 8
    exp1 = [0.0, math.log2(4 / 8) / 32, -0.5, math.log2(1 / 8) / 32, -4, -2, -4, -2,
            1.0, math.log2(4 / 8) / 32, 5, -2, 5, -2, 5, -2,
            math.log2(9 / 8) / 32, FAR1, 0.0]
    assert np.allclose(F[1], exp1, rtol=0, atol=1e-15)
    # root 2 (last): lo = 3, hi = sqrt(18), h = 9 / (3 + sqrt(18)), w2 = rho = 9
    h = 9 / (3 + math.sqrt(18))
    exp2 = [0.0, math.log2(4 / 9) / 32, -2 / h, math.log2(4 / 9) / 32, -3 / h, math.log2(1 / 9) / 32, -4, -2,
            5, -2, 5, -2, 5, -2, 5, -2, 0.0, FAR1, 0.0]
    assert np.allclose(F[2], exp2, rtol=0, atol=1e-15)


def test_features_invariances():
    g = np.random.default_rng(9)
    N = 50
    d = np.concatenate([[0.0], np.sort(g.uniform(0.01, 2, N - 1))])
    z = g.standard_normal(N)
    F = L.features(d, z)
    # power-of-two scaling of the whole problem changes no feature
    assert np.array_equal(L.features(d * 2.0 ** 40, z * 2.0 ** 40), F)
    # the sign of z does not enter
    assert np.array_equal(L.features(d, -z), F)
    assert np.all(F[:, 0:8:2] <= 0) and np.all(F[:, 0:8:2] >= -4)
    assert np.all(F[:, 8:16:2] >= 1) and np.all(F[:, 8:16:2] <= 5)
    assert np.all(np.abs(F[:, 1:16:2]) <= 2)
    # tiny and huge strengths saturate instead of overflowing
    z2 = z.copy()
    z2[5] = 1e-300
    F2 = L.features(d, z2)
    assert F2[5, 1] == -2.0 and np.all(np.isfinite(F2))


def test_far_field_small_problems_are_exact():
    """With one block every far pole is summed term by term: the far field is
    f at the midpoint minus the 8 nearest terms, by direct summation."""
    g = np.random.default_rng(12)
    N = 16
    assert L.far_block(N) == 4
    d = np.concatenate([[0.0], np.sort(g.uniform(0.01, 2, N - 1))])
    z = g.standard_normal(N)
    rho = float(np.sum(z * z))
    F = L.features(d, z)
    B = L.far_block(N)
    for i in range(N):
        lo, hi, h, w2 = L.interval(d, rho, i)
        lam = lo * lo + 0.5 * w2
        far = [j for j in range(N) if not (i - 3 <= j <= i + 4)]
        blocks_near = {j // B for j in range(max(0, i - 3), min(N, i + 5))}
        if all(j // B in blocks_near for j in far):
            v = 1.0 + sum(z[j] ** 2 / (d[j] ** 2 - lam) for j in far)
            s = sum(z[j] ** 2 / (d[j] ** 2 - lam) ** 2 for j in far)
            assert abs(F[i, 17] - math.asinh(v) / 8) <= 1e-13
            assert abs(F[i, 18] - math.asinh(s * w2) / 8) <= 1e-13


def test_far_field_monopoles_approximate_the_sum():
    """For a large problem the block monopoles stay close to the exact far
    field (they are exact for one-pole blocks and accurate for distant ones)."""
    g = np.random.default_rng(13)
    N = 2000
    d = np.concatenate([[0.0], np.sort(g.uniform(0.0, 3.0, N - 1))])
    z = g.standard_normal(N) * 0.02
    rho = float(np.sum(z * z))
    B = L.far_block(N)
    assert B == 64
    Zb, Db = L.block_moments(d, z, B)
    errs = []
    for i in range(5, N, 97):
        lo, hi, h, w2 = L.interval(d, rho, i)
        lam = lo * lo + 0.5 * w2
        far = np.array([j for j in range(N) if not (i - 3 <= j <= i + 4)])
        t = z[far] ** 2 / (d[far] ** 2 - lam)
        v_exact = 1.0 + np.sum(t)
        v, _ = L.far_field(d, z, rho, i, B, Zb, Db)
        errs.append(abs(v - v_exact) / (1.0 + np.sum(np.abs(t))))
    # relative to the sum of |terms|: crude only next to a block boundary
    assert max(errs) < 0.1 and np.median(errs) < 0.02


def _arrow_roots(d, z):
    """Singular values of M = e_1 z^T + diag(d) from LAPACK's dense SVD
    (absolute accuracy about eps ||M||, independent of the secular iteration)."""
    M = np.diag(d)
    M[0, :] = z
    return np.sort(np.linalg.svd(M, compute_uv=False))


def _problem(g, N, spread="uniform"):
    if spread == "uniform":
        dd = np.sort(g.uniform(0.0, 1.0, N - 1))
    else:
        dd = np.sort(10.0 ** g.uniform(-6, 0, N - 1))
    d = np.concatenate([[0.0], dd])
    z = g.standard_normal(N) * 10.0 ** g.uniform(-3, 0, N)
    return d, z


@pytest.mark.parametrize("how", ["exact", "random", "zeros", "ones"])
def test_learned_roots_converge_to_the_roots(how):
    g = np.random.default_rng(21)
    for N, spread in [(2, "uniform"), (7, "graded"), (60, "uniform"), (90, "graded")]:
        d, z = _problem(g, N, spread)
        o0, t0, it0 = secular_roots(d, z)
        x = {"exact": lambda: L.labels(d, z, o0, t0), "random": lambda: g.uniform(0, 1, N),
             "zeros": lambda: np.zeros(N), "ones": lambda: np.ones(N)}[how]()
        o, t, it = L.learned_roots(d, z, x)
        om = d[o] + t
        ref = _arrow_roots(d, z)
        assert np.max(np.abs(om - ref)) <= 1e-13 * ref[-1]
        # each root in its interval, against the pole it is nearer to in omega^2
        for i in range(N):
            assert (d[i] < om[i] < d[i + 1]) if i < N - 1 else (om[i] > d[-1])
            if i < N - 1:
                mid2 = 0.5 * (d[i] ** 2 + d[i + 1] ** 2)
                if abs(om[i] ** 2 - mid2) > 1e-10 * mid2:
                    assert o[i] == (i if om[i] ** 2 < mid2 else i + 1)
            else:
                assert o[i] == N - 1
        # same roots as the plain start: tau to high relative accuracy where
        # the origins agree (they differ only next to the midpoint)
        same = o == o0
        assert np.mean(same) >= 0.9
        assert np.all(np.abs(t[same] - t0[same]) <= 1e-13 * np.abs(t0[same]))
        assert np.all(it >= 1) and np.all(it <= L.MAX_ITERS)
        if how == "exact" and N > 2:
            assert it.mean() < it0.mean()


def test_learned_roots_relative_accuracy_near_poles():
    """Roots a tiny distance from a pole keep their distance to full relative
    accuracy even when the proposal puts them in the wrong half."""
    d = np.array([0.0, 1.0, 2.0, 3.0])
    z = np.array([1e-9, 1e-9, 1e-9, 1e-9])
    o0, t0, _ = secular_roots(d, z)
    o, t, _ = L.learned_roots(d, z, np.array([0.9, 0.9, 0.9, 0.9]))
    assert np.array_equal(o, o0)
    assert np.allclose(t, t0, rtol=1e-14, atol=0)


def test_shipped_network_cuts_oracle_iterations():
    """The network shipped with the package, run through the oracle's
    bfloat16 forward pass, starts the oracle's iteration on a held-out
    N(0,1) bidiagonal: same singular values, fewer evaluations per root."""
    import os
    import oracle
    from paper_2508_11467_amd import inputs
    path = os.path.join(os.path.dirname(__file__), "..", "paper_2508_11467_amd", "data", "start_mlp.npy")
    p = np.load(path, allow_pickle=False).astype(np.float64)
    assert p.shape == (L.NPARAMS,)
    d, e = inputs.normal(600, inputs.split_seed(3, 0, "valid", 5))
    s0, _, _, st0 = oracle.bdsdc(d, e, return_stats=True)
    s1, _, _, st1 = oracle.bdsdc(d, e, return_stats=True,
                                 start=lambda dd, zz: L.mlp_forward(p, L.features(dd, zz), "bf16")[0])
    assert np.max(np.abs(s1 - s0)) <= 1e-14 * s0[0]
    ip = sum(m.iters.sum() for m in st0) / sum(m.N for m in st0)
    il = sum(m.iters.sum() for m in st1) / sum(m.N for m in st1)
    assert il <= 0.9 * ip, (ip, il)
