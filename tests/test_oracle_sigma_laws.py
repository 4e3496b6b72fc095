"""The paper's singular-value laws (Section 3: logrand, arith, geo with
condition number theta) as bidiagonals of exactly known spectrum, built by
Golub-Kahan-Lanczos on diag(sigma); the generator and the oracle pinned to
that spectrum (CPU).

The generator reports delta, a Weyl bound on how far B's singular values can
lie from the law's (from its own residual and loss of orthogonality), so a
solver is held to |sigma_k - law_k| <= 1e-13 sigma_1 + delta."""

import numpy as np
import pytest

import oracle
from paper_2508_11467_amd import inputs

LAWS = [("logrand", 1e6), ("arith", 1e6), ("geo", 1e6), ("geo", 1e12), ("logrand", 1e12)]


def test_laws_by_their_definitions():
    n = 9
    a = inputs.sigma_law(n, "arith", 1e3)
    assert a[0] == 1.0 and abs(a[-1] - 1e-3) <= 1e-18
    assert np.allclose(np.diff(a), -(1.0 - 1e-3) / (n - 1), rtol=0, atol=1e-15)
    g = inputs.sigma_law(n, "geo", 1e8)
    assert g[0] == 1.0 and abs(g[-1] / 1e-8 - 1.0) <= 1e-14
    assert np.allclose(g[1:] / g[:-1], 1e-1, rtol=1e-14)
    r = inputs.sigma_law(1000, "logrand", 1e4, seed=3)
    assert np.all(np.diff(r) <= 0) and r[0] <= 1.0 and r[-1] >= 1e-4
    # log sigma uniform over (log 1e-4, 0): mean -ln(1e4)/2
    assert abs(np.mean(np.log(r)) + 0.5 * np.log(1e4)) < 0.2


@pytest.mark.parametrize("law,theta", LAWS)
def test_gkl_bidiagonal_has_the_law_spectrum(law, theta):
    s = inputs.sigma_law(96, law, theta, seed=11)
    d, e, delta = inputs.gkl_bidiagonal(s, 12)
    assert np.all(d > 0) and np.all(e > 0)
    assert delta <= 1e-13 * s[0]
    sv = np.linalg.svd(oracle.dense(d, e), compute_uv=False)
    assert np.max(np.abs(sv - s)) <= delta + 1e-14 * s[0]


@pytest.mark.parametrize("law,theta", LAWS)
@pytest.mark.parametrize("n,leaf", [(150, 32), (150, 8)])
def test_oracle_recovers_the_law(law, theta, n, leaf):
    s = inputs.sigma_law(n, law, theta, seed=21)
    d, e, delta = inputs.gkl_bidiagonal(s, 22)
    sigma, U, VT = oracle.bdsdc(d, e, leaf=leaf)
    assert np.max(np.abs(sigma - s)) <= 1e-13 * s[0] + delta
    B = oracle.dense(d, e)
    assert np.linalg.norm(B - (U * sigma) @ VT) <= 1e-12 * np.linalg.norm(B)
    assert np.max(np.abs(U.T @ U - np.eye(n))) <= 1e-12
    assert np.max(np.abs(VT @ VT.T - np.eye(n))) <= 1e-12
