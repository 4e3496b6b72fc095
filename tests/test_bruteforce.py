"""The brute-force references used by the tests, checked against closed forms."""

import math

import numpy as np

from _bruteforce import gk_singular_values, singular_value_by_bisection, sturm_count


def test_sturm_bisection_ones_closed_form():
    n = 2000
    d, e = np.ones(n), np.ones(n - 1)
    for i in (0, 1, 666, n // 2, n - 1):
        ref = 2.0 * math.cos((i + 1) * math.pi / (2 * n + 1))
        assert abs(singular_value_by_bisection(d, e, i) - ref) <= 4e-16 * 2.0
    # counts at exact points of the spectrum's range, including x = 1 where a
    # zero pivot appears
    assert sturm_count(d, e, 1.0) == sum(2.0 * math.cos(k * math.pi / (2 * n + 1)) < 1.0 for k in range(1, n + 1))
    assert sturm_count(d, e, 2.0) == n and sturm_count(d, e, 0.0) == 0


def test_sturm_bisection_diagonal():
    g = np.random.default_rng(1)
    d = g.uniform(-1, 1, 50)
    e = np.zeros(49)
    ref = np.sort(np.abs(d))[::-1]
    for i in (0, 10, 49):
        assert abs(singular_value_by_bisection(d, e, i) - ref[i]) <= 1e-15


def test_jacobi_ones_closed_form():
    n = 20
    ref = 2.0 * np.cos(np.arange(1, n + 1) * math.pi / (2 * n + 1))
    assert np.max(np.abs(gk_singular_values(np.ones(n), np.ones(n - 1)) - ref)) <= 1e-15
