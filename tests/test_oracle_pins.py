"""Pins of the oracle parts behind the reported iteration counts and the
learned start, each against something other than the oracle itself:

* the secular evaluation count is the number of O(N) evaluations of f the
  solver actually performs (counted by instrumenting the one routine that
  evaluates f), and for N = 2, where the two-pole model of R.-C. Li's
  iteration is the secular function itself, one model step lands on the
  closed-form root;
* the network's forward pass and gradient equal torch's float64 modules
  (nn.Linear layers, GELU in its tanh form, the logistic function, autograd);
* the root labels place lo + x h at the root omega = d[o] + tau.
"""

import math

import numpy as np
import pytest

import oracle
from oracle import learned, secular


class _CountingEvaluate:
    """Wraps the secular-function evaluation and counts evaluated roots."""

    def __init__(self, fn):
        self.fn = fn
        self.rows = 0

    def __call__(self, d, zsq, o_val, tau, lp):
        self.rows += int(np.asarray(o_val).shape[0])
        return self.fn(d, zsq, o_val, tau, lp)


def _random_merge(g, N):
    d = np.concatenate([[0.0], np.sort(g.uniform(0.0, 1.0, N - 1))])
    z = g.uniform(0.05, 1.0, N) * np.where(g.uniform(size=N) < 0.5, -1.0, 1.0)
    return d, z


@pytest.mark.parametrize("N", [2, 3, 17, 200])
def test_plain_iteration_count_is_evaluations_performed(monkeypatch, N):
    g = np.random.default_rng(100 + N)
    d, z = _random_merge(g, N)
    spy = _CountingEvaluate(secular._evaluate)
    monkeypatch.setattr(secular, "_evaluate", spy)
    o, tau, iters = oracle.secular_roots(d, z)
    assert spy.rows == int(np.sum(iters))
    assert np.all(iters >= 1)


@pytest.mark.parametrize("N", [2, 9, 60])
def test_learned_iteration_count_is_evaluations_performed(monkeypatch, N):
    g = np.random.default_rng(300 + N)
    d, z = _random_merge(g, N)
    spy = _CountingEvaluate(secular._evaluate)
    monkeypatch.setattr(learned, "_evaluate", spy)
    xhat = g.uniform(0.0, 1.0, N)
    o, tau, iters = learned.learned_roots(d, z, xhat)
    assert spy.rows == int(np.sum(iters))
    assert np.all(iters >= 1)


def test_single_pole_needs_no_evaluation(monkeypatch):
    spy = _CountingEvaluate(secular._evaluate)
    monkeypatch.setattr(secular, "_evaluate", spy)
    o, tau, iters = oracle.secular_roots(np.array([0.0]), np.array([-0.75]))
    assert spy.rows == 0 and iters[0] == 0 and tau[0] == 0.75


def _closed_form_n2(d2, z1, z2):
    """Roots of 1 - z1^2/w^2 + z2^2/(d2^2 - w^2) = 0: w^2 solves
    x^2 - (d2^2 + rho) x + z1^2 d2^2 = 0 (clearing denominators), in
    extended precision."""
    L = np.longdouble
    d2, z1, z2 = L(d2), L(z1), L(z2)
    b = d2 * d2 + z1 * z1 + z2 * z2
    c = z1 * z1 * d2 * d2
    disc = np.sqrt(b * b - 4 * c)
    x_small = 2 * c / (b + disc)
    x_large = (b + disc) / 2
    return np.sqrt(x_small), np.sqrt(x_large)


def test_two_poles_one_model_step():
    """N = 2: psi and phi are one term each, so the two-pole model is exact
    and the first model step from the midpoint lands on the root: two
    evaluations (midpoint + the root), a third only when rounding keeps |f|
    just above the stopping threshold there."""
    g = np.random.default_rng(7)
    counts = []
    for _ in range(400):
        d2 = g.uniform(0.05, 1.0)
        z1, z2 = g.uniform(0.05, 1.0, 2) * np.where(g.uniform(size=2) < 0.5, -1.0, 1.0)
        o, tau, iters = oracle.secular_roots(np.array([0.0, d2]), np.array([z1, z2]))
        w = np.array([0.0, d2])[o] + tau
        ref = np.array(_closed_form_n2(d2, z1, z2), dtype=np.float64)
        assert np.all(np.abs(w - ref) <= 16 * 2.0 ** -52 * ref[1])
        counts.extend(iters.tolist())
    counts = np.array(counts)
    assert set(counts.tolist()) <= {2, 3}
    assert np.mean(counts == 2) >= 0.9


def test_root_at_midpoint_takes_one_evaluation():
    """d = (0, 2), z = (1.5, 0.5): z1^2 - z2^2 = d2^2 / 2 puts the first root
    at the interval's midpoint in omega^2 (w^2 = 2), so the midpoint
    evaluation already meets the stopping rule; the second root (w^2 = 4.5
    from the quadratic) needs the usual model step."""
    o, tau, iters = oracle.secular_roots(np.array([0.0, 2.0]), np.array([1.5, 0.5]))
    w = np.array([0.0, 2.0])[o] + tau
    assert abs(w[0] - math.sqrt(2.0)) <= 4e-16 * 2
    assert abs(w[1] - math.sqrt(4.5)) <= 4e-16 * 4
    assert iters[0] == 1 and iters[1] >= 2


def _torch_mlp(p):
    import torch
    P = learned.unflatten(p)
    layers = []
    for l, (fi, fo) in enumerate(learned.LAYERS):
        lin = torch.nn.Linear(fi, fo, dtype=torch.float64)
        with torch.no_grad():
            lin.weight.copy_(torch.from_numpy(P[2 * l].T.copy()))
            lin.bias.copy_(torch.from_numpy(P[2 * l + 1].copy()))
        layers.append(lin)
        if l < 3:
            layers.append(torch.nn.GELU(approximate="tanh"))
    return torch.nn.Sequential(*layers)


def test_mlp_forward_matches_torch_float64():
    import torch
    g = np.random.default_rng(11)
    p = learned.mlp_init(5) + 0.05 * g.standard_normal(learned.NPARAMS)
    X = g.standard_normal((257, learned.NFEAT))
    xhat, _ = learned.mlp_forward(p, X, precision="f64")
    net = _torch_mlp(p)
    with torch.no_grad():
        ref = torch.sigmoid(net(torch.from_numpy(X))[:, 0]).numpy()
    assert np.max(np.abs(xhat - ref)) <= 1e-14


def test_gelu_matches_torch_tanh_form():
    import torch
    x = np.linspace(-8.0, 8.0, 4001)
    ref = torch.nn.functional.gelu(torch.from_numpy(x), approximate="tanh").numpy()
    assert np.max(np.abs(learned.gelu(x) - ref)) <= 1e-15 * 8
    xt = torch.from_numpy(x).requires_grad_(True)
    torch.nn.functional.gelu(xt, approximate="tanh").sum().backward()
    assert np.max(np.abs(learned.gelu_grad(x) - xt.grad.numpy())) <= 1e-14


def test_mlp_gradient_matches_torch_autograd():
    import torch
    g = np.random.default_rng(12)
    p = learned.mlp_init(6) + 0.05 * g.standard_normal(learned.NPARAMS)
    X = g.standard_normal((96, learned.NFEAT))
    y = g.uniform(0.0, 1.0, 96)
    loss, grad = learned.mlp_loss_grad(p, X, y, precision="f64")
    net = _torch_mlp(p)
    out = torch.sigmoid(net(torch.from_numpy(X))[:, 0])
    tl = torch.mean((out - torch.from_numpy(y)) ** 2)
    tl.backward()
    tg = []
    for mod in net:
        if isinstance(mod, torch.nn.Linear):
            tg.append(mod.weight.grad.numpy().T.ravel())
            tg.append(mod.bias.grad.numpy().ravel())
    tg = np.concatenate(tg)
    assert abs(loss - float(tl)) <= 1e-15
    assert np.max(np.abs(grad - tg)) <= 1e-13 * max(1.0, np.max(np.abs(tg)))


def test_labels_place_the_root():
    """lo + x h reproduces omega = d[o] + tau for every root, with x in
    [0, 1], on a merge solved by the oracle."""
    g = np.random.default_rng(13)
    for N in (2, 5, 40, 300):
        d, z = _random_merge(g, N)
        o, tau, _ = oracle.secular_roots(d, z)
        rho = float(np.sum(z * z))
        x = learned.labels(d, z, o, tau)
        w = d[o] + tau
        for i in range(N):
            lo = d[i]
            hi = d[i + 1] if i < N - 1 else math.sqrt(d[i] ** 2 + rho)
            assert 0.0 <= x[i] <= 1.0
            assert abs(lo + x[i] * (hi - lo) - w[i]) <= 4e-16 * 4 * max(hi, 1e-300) + 1e-300
