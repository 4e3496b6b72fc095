"""The HIP path on bidiagonals with the paper's singular-value laws
(logrand, arith, geo; Section 3) and exactly known spectrum, against the law
and against the oracle."""

import numpy as np
import pytest

import oracle
from paper_2508_11467_amd import inputs

pytestmark = pytest.mark.gpu

LAWS = [("logrand", 1e6), ("arith", 1e6), ("geo", 1e6), ("geo", 1e12), ("logrand", 1e12)]


@pytest.fixture(scope="module")
def solver(gpu):
    from paper_2508_11467_amd.api import Solver
    s = Solver(0)
    yield s
    s.close()


@pytest.mark.parametrize("law,theta", LAWS)
def test_law_spectrum_n1024(solver, law, theta):
    import torch
    n = 1024
    s = inputs.sigma_law(n, law, theta, seed=31)
    d, e, delta = inputs.gkl_bidiagonal(s, 32)
    print(f"law={law} theta={theta:g} n={n}", flush=True)
    sig, U, VT = solver.svd(torch.from_numpy(d), torch.from_numpy(e))
    info, _ = solver.info()
    assert info == 0
    sg = sig.cpu().numpy()
    assert np.max(np.abs(sg - s)) <= 1e-13 * s[0] + delta
    B = torch.from_numpy(oracle.dense(d, e)).cuda()
    I = torch.eye(n, dtype=torch.float64, device="cuda")
    Uc, Vc = U.contiguous(), VT.contiguous()
    assert float(torch.linalg.norm(B - (Uc * sig[None, :]) @ Vc) / torch.linalg.norm(B)) <= 1e-12
    assert float(torch.max(torch.abs(Uc.T.contiguous() @ Uc - I))) <= 1e-12
    assert float(torch.max(torch.abs(Vc @ Vc.T.contiguous() - I))) <= 1e-12


@pytest.mark.parametrize("law,theta", LAWS[:3])
def test_law_against_oracle_n300(solver, law, theta):
    import torch
    n = 300
    s = inputs.sigma_law(n, law, theta, seed=41)
    d, e, delta = inputs.gkl_bidiagonal(s, 42)
    sig, _, _ = solver.svd(torch.from_numpy(d), torch.from_numpy(e))
    ref, _, _ = oracle.bdsdc(d, e)
    assert np.max(np.abs(sig.cpu().numpy() - ref)) <= 1e-13 * ref[0]
