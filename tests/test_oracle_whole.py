"""Pins of the whole oracle SVD against closed forms, brute force and library
routines (CPU)."""

import math
import os

import numpy as np
import pytest

import oracle
from paper_2508_11467_amd import inputs

from _bruteforce import gk_singular_values

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def check_svd(d, e, sigma, U, VT, tol_sig=None, ref=None, rtol=1e-12):
    n = len(d)
    B = oracle.dense(d, e)
    nb = np.linalg.norm(B)
    assert sigma.shape == (n,)
    assert np.all(sigma >= 0.0)
    assert np.all(np.diff(sigma) <= 0.0)
    if n == 0:
        return
    if nb > 0:
        assert np.linalg.norm(B - (U * sigma[None, :]) @ VT) <= rtol * nb
    assert np.max(np.abs(U.T @ U - np.eye(n))) <= rtol
    assert np.max(np.abs(VT @ VT.T - np.eye(n))) <= rtol
    if ref is not None:
        assert np.max(np.abs(sigma - ref)) <= (tol_sig or 1e-13) * max(ref[0], 1e-300)


def _golden_ones(n):
    with open(os.path.join(GOLDEN, f"ones_n{n}.txt")) as f:
        return np.array([float(x) for x in f if not x.startswith("#")])


@pytest.mark.parametrize("n,leaf", [(1, 32), (2, 32), (5, 32), (5, 4), (40, 32), (40, 6), (100, 32), (100, 8)])
def test_ones_closed_form(n, leaf):
    d, e = inputs.ones(n)
    sigma, U, VT = oracle.bdsdc(d, e, leaf=leaf)
    check_svd(d, e, sigma, U, VT, ref=_golden_ones(n), tol_sig=1e-14)


@pytest.mark.parametrize("n", [257, 1000])
def test_ones_closed_form_formula(n):
    d, e = inputs.ones(n)
    sigma, U, VT = oracle.bdsdc(d, e)
    ref = 2.0 * np.cos(np.arange(1, n + 1) * math.pi / (2 * n + 1))
    check_svd(d, e, sigma, U, VT, ref=ref, tol_sig=1e-14)


@pytest.mark.parametrize("n", [1, 7, 64, 300])
def test_diagonal_closed_form(n):
    g = np.random.default_rng(n)
    d = g.uniform(-1, 1, n)
    e = np.zeros(max(n - 1, 0))
    sigma, U, VT = oracle.bdsdc(d, e, leaf=8)
    check_svd(d, e, sigma, U, VT, ref=np.sort(np.abs(d))[::-1], tol_sig=0.0)


@pytest.mark.parametrize("n,leaf,seed", [(33, 32, 0), (64, 32, 1), (48, 5, 2), (60, 4, 3), (17, 4, 4)])
def test_against_jacobi_golub_kahan(n, leaf, seed):
    d, e = inputs.uniform(n, 1000 + seed)
    sigma, U, VT = oracle.bdsdc(d, e, leaf=leaf)
    ref = gk_singular_values(d, e)
    check_svd(d, e, sigma, U, VT, ref=ref, tol_sig=1e-14)


@pytest.mark.parametrize("name,n,gen", [
    ("uniform", 256, lambda n: inputs.workload("n256_uniform")),
    ("normal", 700, lambda n: inputs.normal(n, 5)),
    ("graded", 600, lambda n: inputs.graded(n, 6)),
    ("clustered", 600, lambda n: inputs.clustered(n, 7)),
    ("ones_odd", 333, lambda n: inputs.ones(n)),
])
def test_against_numpy_svd(name, n, gen):
    d, e = gen(n)
    sigma, U, VT, stats = oracle.bdsdc(d, e, return_stats=True)
    ref = np.linalg.svd(oracle.dense(d, e), compute_uv=False)
    check_svd(d, e, sigma, U, VT, ref=ref)
    B = oracle.dense(d, e)
    assert abs(np.sum(sigma ** 2) - np.linalg.norm(B) ** 2) <= 1e-13 * np.linalg.norm(B) ** 2


def mirrored(k, seed):
    """n = 2k bidiagonal whose two children at the root split share k-1
    values: the left child is L ((k-1) x k), the right child is L over a zero
    row (k x k), so its values are those of L and 0."""
    g = np.random.default_rng(seed)
    n = 2 * k
    d = np.empty(n)
    e = np.empty(n - 1)
    d[: k - 1] = g.uniform(-1, 1, k - 1)
    e[: k - 2] = g.uniform(-1, 1, k - 2)
    e[k - 2] = 0.35                    # the left child's extra column
    d[k - 1] = 0.7                     # alpha
    e[k - 1] = -0.4                    # beta
    d[k: 2 * k - 1] = d[: k - 1]
    e[k: 2 * k - 2] = e[: k - 2]
    e[2 * k - 2] = 0.35
    d[2 * k - 1] = 0.0
    return d, e


@pytest.mark.parametrize("k,leaf", [(20, 32), (40, 32), (50, 8)])
def test_close_pair_deflation_case(k, leaf):
    d, e = mirrored(k, 21)
    sigma, U, VT, stats = oracle.bdsdc(d, e, leaf=leaf, return_stats=True)
    assert sum(s.n_close for s in stats) > 0
    assert any(s.counts[1] > 0 for s in stats)          # mixed (type 2) columns
    check_svd(d, e, sigma, U, VT, ref=np.linalg.svd(oracle.dense(d, e), compute_uv=False))


def test_zero_d_deflation_case():
    # zero diagonal entries make the children singular: their zero values
    # sit within tol of d_1 = 0 and deflate by the right-side rotation
    d, e = inputs.uniform(200, 11)
    d[10::17] = 0.0
    sigma, U, VT, stats = oracle.bdsdc(d, e, return_stats=True)
    assert sum(s.n_zero_d for s in stats) > 0
    check_svd(d, e, sigma, U, VT, ref=np.linalg.svd(oracle.dense(d, e), compute_uv=False))


def test_scaling_equivariance_bitwise():
    d, e = inputs.uniform(300, 12)
    s1, U1, V1 = oracle.bdsdc(d, e)
    for p in (2.0 ** 40, 2.0 ** -37):
        s2, U2, V2 = oracle.bdsdc(d * p, e * p)
        assert np.array_equal(s2, s1 * p)
        assert np.array_equal(U2, U1) and np.array_equal(V2, V1)


def test_log_det_wellconditioned():
    g = np.random.default_rng(13)
    n = 400
    d = g.uniform(2, 3, n)
    e = g.uniform(-1, 1, n - 1)
    sigma, _, _ = oracle.bdsdc(d, e)
    assert abs(np.sum(np.log(sigma)) - np.sum(np.log(np.abs(d)))) <= 1e-12 * n


def test_edge_sizes():
    s, U, VT = oracle.bdsdc(np.zeros(0), np.zeros(0))
    assert s.shape == (0,)
    s, U, VT = oracle.bdsdc(np.array([-3.0]), np.zeros(0))
    assert s[0] == 3.0 and U[0, 0] * VT[0, 0] == -1.0
    d = np.array([0.0, 0.0, 1.0])
    e = np.array([0.0, 0.0])
    s, U, VT = oracle.bdsdc(d, e)
    check_svd(d, e, s, U, VT, ref=np.array([1.0, 0.0, 0.0]), tol_sig=0.0)
    d = np.zeros(70)
    e = np.zeros(69)
    s, U, VT = oracle.bdsdc(d, e)
    check_svd(d, e, s, U, VT, ref=np.zeros(70), tol_sig=0.0)


def test_secular_iterations_reported():
    d, e = inputs.workload("n256_uniform")
    _, _, _, stats = oracle.bdsdc(d, e, return_stats=True)
    it = np.concatenate([s.iters for s in stats])
    assert it.min() >= 1 and it.max() <= 64
    assert 2.0 <= it.mean() <= 12.0
