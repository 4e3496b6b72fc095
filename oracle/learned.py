"""Oracle of the learned secular start.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

A small MLP proposes, for every root of the secular equation (eq.
M-svd-val), its fractional position x in the root's interval; the
safeguarded iteration then starts there instead of at the interval's
midpoint.  The iteration, its safeguards and its stopping rule are those of
``secular.py``, so a proposal only changes how many evaluations a root needs,
never the tolerance it converges to.  The paper has no such component; the
definitions below are this implementation's and the GPU kernels follow them.

Interval of root i (0-based, poles 0 = d_0 < d_1 < ... < d_{N-1}):
  interior  lo = d_i, hi = d_{i+1}, h = hi - lo, w2 = h (hi + lo) = hi^2 - lo^2
  last      lo = d_{N-1}, hi = sqrt(lo^2 + rho), h = rho / (lo + hi), w2 = rho
with rho = sum z_j^2.

Features (19 per root):
  for q = 0..3, left pole j = i - q:  F[2q]   = max((d_j - lo) / h, -4)
                                      F[2q+1] = clip(log2(z_j^2 / w2) / 32, -2, 2)
  for q = 0..3, right pole j = i+1+q: F[8+2q] = min((d_j - lo) / h, 5)
                                      F[9+2q] = clip(log2(z_j^2 / w2) / 32, -2, 2)
  a missing pole (beyond either end) has gap -4 (left) or 5 (right) and
  strength -2;  F[16] = clip(log2(rho / w2) / 32, -2, 2);
  F[17], F[18]: the far field -- the rest of f without the 8 poles above --
  at the interval's midpoint lam = lo^2 + w2/2 in omega^2: its value
  v = 1 + sum_far z_j^2 / (d_j^2 - lam) and slope s = sum_far z_j^2 /
  (d_j^2 - lam)^2, as asinh(v)/8 and asinh(s w2)/8 (clamped to [-4, 4]).
  The far sum is approximate and costs O(sqrt N) per root instead of N:
  the poles are cut into blocks of B (the least power of two >= 4 with
  B^2 >= N and 512 B >= N); blocks that hold root i or one of its 8 poles are
  summed term by term (ascending j, skipping the 8 poles), every other block
  by one monopole term Z_k / (D_k - lam) with Z_k = sum z_j^2 and D_k =
  (sum z_j^2 d_j^2) / Z_k over the block (ascending j; skipped when Z_k = 0).
z_j^2 / w2 is the strength of pole j relative to the interval: near the
interval f is about 1 + sum_j c_j / (g_j - x) with g_j the gap and c_j that
ratio, and with a logistic output the dominant two-pole relation
logit(x) ~ log c_lo - log c_hi is linear in the log features.  Which of the
two poles a root sits next to is decided by the sign of the far field, which
the 8 nearest poles alone do not determine.

Label: x = (omega - lo) / h of the computed root, in [0, 1].

Network: 19 -> 64 -> 64 -> 64 -> 1, GELU (tanh form) after the hidden
layers, logistic output; loss = mean squared error of x_hat.  Parameters are
one flat FP32 vector: W1 (19 x 64, row-major, in x out), b1 (64), W2 (64 x
64), b2, W3 (64 x 64), b3, W4 (64), b4 (1): 9665 numbers.

Precision.  ``precision="f64"`` is the exact network in FP64.
``precision="bf16"`` takes the rounding points of the MFMA kernels: every
operand of a matrix product (the inputs, the weights, the hidden activations,
and in the backward pass the back-propagated gradients) is rounded to
bfloat16 (round to nearest, ties to even); products, biases, GELU, the
logistic and all bias gradients stay in high precision.
"""

from __future__ import annotations

import math

import numpy as np

from .secular import EPS, MAX_ITERS, _evaluate

NFEAT = 19
HIDDEN = 64
GAP_LEFT = -4.0
GAP_RIGHT = 5.0
STRENGTH_MIN = -2.0
STRENGTH_MAX = 2.0
LOG_SCALE = 32.0
X_CLAMP = 2.0 ** -20  # a proposal is kept this far inside (0, 1)
LAYERS = [(NFEAT, HIDDEN), (HIDDEN, HIDDEN), (HIDDEN, HIDDEN), (HIDDEN, 1)]
NPARAMS = sum(fi * fo + fo for fi, fo in LAYERS)


# ---------------------------------------------------------------- features
def interval(d, rho, i):
    """(lo, hi, h, w2) of root i's interval."""
    N = d.shape[0]
    lo = float(d[i])
    if i < N - 1:
        hi = float(d[i + 1])
        h = hi - lo
        return lo, hi, h, h * (hi + lo)
    hi = math.sqrt(lo * lo + rho)
    return lo, hi, rho / (lo + hi), rho


def _strength(zj, w2):
    c = (zj * zj) / w2
    if c == 0.0:
        return STRENGTH_MIN
    if math.isinf(c):
        return STRENGTH_MAX
    return min(max(math.log2(c) / LOG_SCALE, STRENGTH_MIN), STRENGTH_MAX)


def far_block(N):
    """Block size of the far-field sum."""
    B = 4
    while B * B < N or 512 * B < N:
        B *= 2
    return B


def far_field(d, z, rho, i, B, Zb, Db):
    """(v, s) of the far field of root i at its interval's midpoint."""
    N = d.shape[0]
    lo, hi, h, w2 = interval(d, rho, i)
    lam = lo * lo + 0.5 * w2
    v, s = 1.0, 0.0
    home = i // B
    nb = (N + B - 1) // B
    for k in range(nb):
        j0, j1 = k * B, min(N, (k + 1) * B)
        if k == home or (j1 > i - 3 and j0 <= i + 4):
            for j in range(j0, j1):
                if i - 3 <= j <= i + 4:
                    continue
                den = d[j] * d[j] - lam
                t = (z[j] * z[j]) / den
                v += t
                s += t / den
        elif Zb[k] > 0.0:
            den = Db[k] - lam
            t = Zb[k] / den
            v += t
            s += t / den
    return v, s


def block_moments(d, z, B):
    """Z_k and D_k of the far-field blocks (sequential sums)."""
    N = d.shape[0]
    nb = (N + B - 1) // B
    Zb = np.zeros(nb)
    Db = np.zeros(nb)
    for k in range(nb):
        zs, ms = 0.0, 0.0
        for j in range(k * B, min(N, (k + 1) * B)):
            zz = z[j] * z[j]
            zs += zz
            ms += zz * (d[j] * d[j])
        Zb[k] = zs
        Db[k] = ms / zs if zs > 0.0 else 0.0
    return Zb, Db


def _asinh8(x):
    return min(max(math.asinh(x) / 8.0, -4.0), 4.0)


def features(d, z, rho=None):
    """(N, 19) inputs of the proposal network (FP64)."""
    d = np.asarray(d, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    N = d.shape[0]
    if rho is None:
        rho = float(np.sum(z * z))
    F = np.empty((N, NFEAT))
    B = far_block(N)
    Zb, Db = block_moments(d, z, B)
    for i in range(N):
        lo, hi, h, w2 = interval(d, rho, i)
        for q in range(4):
            j = i - q
            if j >= 0:
                F[i, 2 * q] = max((d[j] - lo) / h, GAP_LEFT)
                F[i, 2 * q + 1] = _strength(z[j], w2)
            else:
                F[i, 2 * q] = GAP_LEFT
                F[i, 2 * q + 1] = STRENGTH_MIN
            j = i + 1 + q
            if j < N:
                F[i, 8 + 2 * q] = min((d[j] - lo) / h, GAP_RIGHT)
                F[i, 9 + 2 * q] = _strength(z[j], w2)
            else:
                F[i, 8 + 2 * q] = GAP_RIGHT
                F[i, 9 + 2 * q] = STRENGTH_MIN
        F[i, 16] = min(max(math.log2(rho / w2) / LOG_SCALE, STRENGTH_MIN), STRENGTH_MAX)
        v, sl = far_field(d, z, rho, i, B, Zb, Db)
        F[i, 17] = _asinh8(v)
        F[i, 18] = _asinh8(sl * w2)
    return F


def labels(d, z, o, tau, rho=None):
    """Fractional position x = (omega - lo) / h of each root (o, tau)."""
    d = np.asarray(d, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    N = d.shape[0]
    if rho is None:
        rho = float(np.sum(z * z))
    x = np.empty(N)
    for i in range(N):
        lo, hi, h, w2 = interval(d, rho, i)
        # omega - lo without cancellation: tau when the origin is lo's pole
        x[i] = tau[i] / h if o[i] == i else 1.0 + tau[i] / h
    return np.clip(x, 0.0, 1.0)


# ---------------------------------------------------------------- bfloat16
def bf16_round(x):
    """Round to bfloat16 (nearest, ties to even), returned as float64.  The
    value is first rounded to float32, as the kernels hold it."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    b = a.view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    r = ((b + 0x7FFF + lsb) >> 16) << 16
    nan = np.isnan(a)
    out = (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32).astype(np.float64)
    if np.any(nan):
        out = np.where(nan, np.nan, out)
    return out.reshape(np.shape(x))


# ---------------------------------------------------------------- the MLP
def unflatten(p):
    p = np.asarray(p, dtype=np.float64)
    assert p.shape == (NPARAMS,)
    out, off = [], 0
    for fi, fo in LAYERS:
        out.append(p[off:off + fi * fo].reshape(fi, fo))
        off += fi * fo
        out.append(p[off:off + fo])
        off += fo
    return out


def flatten(params):
    return np.concatenate([np.asarray(x, dtype=np.float64).ravel() for x in params])


def mlp_init(seed: int = 0):
    """He-style initial parameters (flat vector)."""
    g = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for fi, fo in LAYERS:
        parts.append(g.standard_normal(fi * fo) * math.sqrt(2.0 / fi))
        parts.append(np.zeros(fo))
    return np.concatenate(parts)


_C = math.sqrt(2.0 / math.pi)
_A = 0.044715


def gelu(x):
    return 0.5 * x * (1.0 + np.tanh(_C * (x + _A * x ** 3)))


def gelu_grad(x):
    t = np.tanh(_C * (x + _A * x ** 3))
    return 0.5 * (1.0 + t) + 0.5 * x * (1.0 - t * t) * _C * (1.0 + 3.0 * _A * x * x)


def _rounder(precision):
    if precision == "f64":
        return lambda v: np.asarray(v, dtype=np.float64)
    if precision == "bf16":
        return bf16_round
    raise ValueError(precision)


def mlp_forward(p, X, precision="f64"):
    """x_hat (B,) and the cache (pre-activations, product operands)."""
    rnd = _rounder(precision)
    P = unflatten(p)
    a = rnd(X)
    ops = [a]
    pres = []
    for l in range(4):
        W, b = rnd(P[2 * l]), P[2 * l + 1]
        pre = a @ W + b
        pres.append(pre)
        if l < 3:
            a = rnd(gelu(pre))
            ops.append(a)
    out = pres[3][:, 0]
    xhat = 1.0 / (1.0 + np.exp(-out))
    return xhat, (ops, pres)


def mlp_loss_grad(p, X, y, precision="f64"):
    """Mean squared error of x_hat against y, and its gradient (flat)."""
    rnd = _rounder(precision)
    P = unflatten(p)
    xhat, (ops, pres) = mlp_forward(p, X, precision)
    B = xhat.shape[0]
    diff = xhat - np.asarray(y, dtype=np.float64)
    loss = float(np.mean(diff * diff))
    g = ((2.0 / B) * diff * xhat * (1.0 - xhat))[:, None]  # d loss / d out
    grads = [None] * 8
    for l in range(3, -1, -1):
        gr = rnd(g)
        grads[2 * l] = ops[l].T @ gr
        grads[2 * l + 1] = np.sum(g, axis=0)
        if l > 0:
            g = (gr @ rnd(P[2 * l]).T) * gelu_grad(pres[l - 1])
    return loss, flatten(grads)


# ---------------------------------------------------------------- learned start
def learned_roots(d, z, xhat):
    """Secular roots started from proposed positions x_hat (one per root).

    The first evaluation is at the proposed point.  Its half of the interval
    (split at the midpoint in omega^2, the plain start's origin test) gives
    the origin pole, and tau starts as x h from the left pole or (x - 1) h
    from the right one.  When an iterate crosses the midpoint the root is
    re-referenced to the other pole (tau and the bracket shifted by h), and
    a step that ends in a frame it has just entered is not accepted as
    converged, so a root is always finished against the pole it is stored
    with.  Model, safeguard and stopping rules are the plain iteration's.
    Returns (o, tau, iters).
    """
    d = np.asarray(d, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    N = d.shape[0]
    o = np.zeros(N, dtype=np.int64)
    tau = np.zeros(N)
    iters = np.zeros(N, dtype=np.int64)
    if N == 0:
        return o, tau, iters
    if N == 1:
        tau[0] = abs(z[0])
        return o, tau, iters
    zsq = z * z
    rho = float(np.sum(zsq))
    x = np.clip(np.asarray(xhat, dtype=np.float64), X_CLAMP, 1.0 - X_CLAMP)
    for i in range(N):
        o[i], tau[i], iters[i] = _learned_one(d, zsq, rho, i, float(x[i]))
    return o, tau, iters


def _learned_one(d, zsq, rho, i, x):
    N = d.shape[0]
    last = i == N - 1
    lp = N - 2 if last else i
    rp = lp + 1
    dl, dr = float(d[lp]), float(d[rp])
    if last:
        h = rho / (dr + math.sqrt(dr * dr + rho))
        o, tau, lo, hi = rp, x * h, 0.0, h
        mu = 0.0
    else:
        h = dr - dl
        mu = 0.5 * (dr - dl) * (dr + dl)  # midpoint in omega^2, offset from dl^2
        t0 = x * h
        if t0 * (2.0 * dl + t0) > mu:
            o, tau, lo, hi = rp, (x - 1.0) * h, -h, 0.0
        else:
            o, tau, lo, hi = lp, t0, 0.0, h
    it = 0
    lpa = np.array([lp])
    while True:
        ov = float(d[o])
        f, psi, dpsi, phi, dphi, E, delta = _evaluate(d, zsq, np.array([ov]), np.array([tau]), lpa)
        f, dpsi, dphi, E = float(f[0]), float(dpsi[0]), float(dphi[0]), float(E[0])
        it += 1
        if f < 0.0:
            lo = tau
        else:
            hi = tau
        if abs(f) <= 8.0 * EPS * E or it >= MAX_ITERS:
            return o, tau, it
        Dl = float(delta[0, lp])
        Dr = float(delta[0, rp])
        c = f - Dl * dpsi - Dr * dphi
        a = (Dl + Dr) * f - Dl * Dr * (dpsi + dphi)
        b = Dl * Dr * f
        disc = math.sqrt(abs(a * a - 4.0 * b * c))
        with np.errstate(divide="ignore", invalid="ignore"):
            if c == 0.0:
                eta = np.float64(b) / np.float64(a)
            elif last:
                eta = (np.float64(a) + disc) / (2.0 * c) if a >= 0.0 else 2.0 * np.float64(b) / (a - disc)
            else:
                eta = (np.float64(a) - disc) / (2.0 * c) if a <= 0.0 else 2.0 * np.float64(b) / (a + disc)
            om = ov + tau
            tn = tau + eta / (om + np.sqrt(np.float64(om * om) + eta))
        tn = float(tn)
        if not (lo < tn < hi):  # also catches NaN
            tn = 0.5 * (lo + hi)
        small = abs(tn - tau) <= 2.0 * EPS * abs(tn)
        tau = tn
        if not last:
            if o == lp and tau * (2.0 * dl + tau) > mu:
                o, tau, lo, hi = rp, tau - h, lo - h, hi - h
                small = False
            elif o == rp and tau * (2.0 * dr + tau) < -mu:
                o, tau, lo, hi = lp, tau + h, lo + h, hi + h
                small = False
        if small:
            return o, tau, it
