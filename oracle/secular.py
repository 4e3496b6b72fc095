"""Oracle secular-equation solver, Loewner recomputation and vectors of M.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

M = e_1 z^T + diag(d) with 0 = d_1 < d_2 < ... < d_N (the deflated "broken
arrow" of Section 4.2.1, eq. diag-one-side-M).  Its singular values omega_i are
the roots of the secular equation (eq. M-svd-val)

    f(omega) = 1 + sum_j z_j^2 / (d_j^2 - omega^2) = 0,

one in each interval (d_i, d_{i+1}) and the last in (d_N, sqrt(d_N^2 + |z|^2)).

The paper calls LAPACK's ``lasd4`` for the roots and names no method.  The
reading used here (the same one the GPU kernel implements independently):

* each root is stored as omega = d[o] + tau with o the index of the nearer pole,
  so that every difference d_j^2 - omega^2 is formed as
  ((d_j - d_o) - tau) * (d_j + d_o + tau) without cancellation;
* the origin is chosen by the sign of f at the midpoint (in omega^2) of the
  interval: f >= 0 -> left pole, else right pole; the last root always takes
  the last pole;
* iteration on omega^2 with R.-C. Li's "middle way" two-pole rational model
  (LAPACK Working Note 89): the sums over poles left of the interval (psi) and
  right of it (phi) are each replaced by a + b / (delta - x) matched in value
  and slope at the current point, and the resulting quadratic is solved;
* safeguard: the root stays bracketed; a step that leaves the bracket or is
  not finite is replaced by bisection of the bracket;
* stop when |f| <= 8 eps (1 + sum_j |z_j^2 / (d_j^2 - omega^2)|), or when the
  step changes tau by no more than 2 eps |tau| (that step is accepted without
  evaluating f again), or after 64 evaluations.  One "iteration" is one O(N)
  evaluation of f, the midpoint one included.

The summation order is fixed: terms of poles left of the interval are added
from the first pole upwards, terms right of it from the last pole downwards,
i.e. from far to near.
"""

from __future__ import annotations

import numpy as np

EPS = 2.0 ** -52
MAX_ITERS = 64


def _evaluate(d, zsq, o_val, tau, lp):
    """f and its pieces at omega = o_val + tau for a block of roots.

    d, zsq: (N,), o_val, tau: (R,), lp: (R,) index of the left model pole.
    Returns f, psi, dpsi, phi, dphi, E, delta (R x N) with
    delta[r, j] = d_j^2 - omega_r^2.
    """
    N = d.shape[0]
    delta = (d[None, :] - o_val[:, None] - tau[:, None]) * (d[None, :] + o_val[:, None] + tau[:, None])
    t = zsq[None, :] / delta
    dt = t / delta
    j = np.arange(N)[None, :]
    left = j <= lp[:, None]
    # psi: left poles summed far-to-near (ascending j); phi: right poles
    # summed far-to-near (descending j).  np.cumsum is sequential, so the
    # order is the one stated.
    tl = np.where(left, t, 0.0)
    dl = np.where(left, dt, 0.0)
    tr = np.where(left, 0.0, t)[:, ::-1]
    dr = np.where(left, 0.0, dt)[:, ::-1]
    psi = np.cumsum(tl, axis=1)[:, -1]
    dpsi = np.cumsum(dl, axis=1)[:, -1]
    phi = np.cumsum(tr, axis=1)[:, -1]
    dphi = np.cumsum(dr, axis=1)[:, -1]
    f = 1.0 + psi + phi
    E = 1.0 + np.sum(np.abs(t), axis=1)
    return f, psi, dpsi, phi, dphi, E, delta


def secular_roots(d, z, chunk: int = 256):
    """Roots of the secular equation.

    d: (N,) strictly increasing with d[0] = 0; z: (N,) with no zero entry.
    Returns (o int64 (N,), tau (N,), iters int64 (N,)), omega_i = d[o_i] + tau_i.
    """
    d = np.asarray(d, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    N = d.shape[0]
    o = np.zeros(N, dtype=np.int64)
    tau = np.zeros(N)
    iters = np.zeros(N, dtype=np.int64)
    if N == 0:
        return o, tau, iters
    zsq = z * z
    rho = float(np.sum(zsq))
    if N == 1:
        # single pole at 0: f = 1 - z^2/omega^2, so omega = |z| exactly.
        tau[0] = abs(z[0])
        return o, tau, iters
    for start in range(0, N, chunk):
        idx = np.arange(start, min(N, start + chunk))
        oo, tt, it = _solve_block(d, zsq, rho, idx)
        o[idx] = oo
        tau[idx] = tt
        iters[idx] = it
    return o, tau, iters


def _solve_block(d, zsq, rho, idx):
    N = d.shape[0]
    R = idx.shape[0]
    last = idx == N - 1
    lp = np.where(last, N - 2, idx)          # left model pole
    rp = lp + 1                               # right model pole
    dl = d[lp]
    dr = d[rp]

    # ---- midpoint evaluation (counts as the first iteration) ----
    # interior: omega_mid^2 = (d_i^2 + d_{i+1}^2)/2, offset mu from d_i^2
    # last:     omega_mid^2 = d_N^2 + rho/2, offset mu from d_N^2
    base = np.where(last, dr, dl)
    mu = np.where(last, 0.5 * rho, 0.5 * (dr - dl) * (dr + dl))
    tau_mid = mu / (base + np.sqrt(base * base + mu))
    f, psi, dpsi, phi, dphi, E, delta = _evaluate(d, zsq, base, tau_mid, lp)
    iters = np.ones(R, dtype=np.int64)

    # origin: interior roots take the left pole if f(mid) >= 0, else the right
    go_right = (~last) & (f < 0.0)
    o = np.where(last | go_right, rp, lp)
    ov = d[o]
    # tau of the midpoint relative to the chosen origin
    omega_mid = base + tau_mid
    tau = np.where(go_right, -mu / (dr + omega_mid), tau_mid)
    # bracket (in tau relative to the origin)
    lo = np.where(last, 0.0, np.where(go_right, tau, 0.0))
    hi = np.where(last, rho / (dr + np.sqrt(dr * dr + rho)), np.where(go_right, 0.0, tau))
    # for the last root the midpoint already tightened one side
    lo = np.where(last & (f < 0.0), tau, lo)
    hi = np.where(last & (f >= 0.0), tau, hi)

    done = np.abs(f) <= 8.0 * EPS * E
    while True:
        active = ~done
        if not np.any(active):
            break
        a_idx = np.nonzero(active)[0]
        # model step from the current evaluation
        Dl = delta[a_idx, lp[a_idx]]
        Dr = delta[a_idx, rp[a_idx]]
        fa = f[a_idx]
        c = fa - Dl * dpsi[a_idx] - Dr * dphi[a_idx]
        a = (Dl + Dr) * fa - Dl * Dr * (dpsi[a_idx] + dphi[a_idx])
        b = Dl * Dr * fa
        disc = np.sqrt(np.abs(a * a - 4.0 * b * c))
        is_last = last[a_idx]
        with np.errstate(divide="ignore", invalid="ignore"):
            eta_in = np.where(a <= 0.0, (a - disc) / (2.0 * c), 2.0 * b / (a + disc))
            eta_la = np.where(a >= 0.0, (a + disc) / (2.0 * c), 2.0 * b / (a - disc))
            eta = np.where(is_last, eta_la, eta_in)
            eta = np.where(c == 0.0, b / a, eta)
            om = ov[a_idx] + tau[a_idx]
            om_new = np.sqrt(om * om + eta)
            tau_new = tau[a_idx] + eta / (om + om_new)
        bad = ~np.isfinite(tau_new) | (tau_new <= lo[a_idx]) | (tau_new >= hi[a_idx])
        tau_new = np.where(bad, 0.5 * (lo[a_idx] + hi[a_idx]), tau_new)
        small_step = np.abs(tau_new - tau[a_idx]) <= 2.0 * EPS * np.abs(tau_new)
        tau[a_idx] = tau_new
        # a step at the rounding level is accepted as it is; elsewhere f is
        # evaluated at the new point
        done[a_idx[small_step]] = True
        e_idx = a_idx[~small_step]
        if e_idx.size == 0:
            continue
        fn, psin, dpsin, phin, dphin, En, deltan = _evaluate(d, zsq, ov[e_idx], tau[e_idx], lp[e_idx])
        iters[e_idx] += 1
        f[e_idx] = fn
        psi[e_idx] = psin
        dpsi[e_idx] = dpsin
        phi[e_idx] = phin
        dphi[e_idx] = dphin
        E[e_idx] = En
        delta[e_idx] = deltan
        neg = fn < 0.0
        lo[e_idx] = np.where(neg, tau[e_idx], lo[e_idx])
        hi[e_idx] = np.where(neg, hi[e_idx], tau[e_idx])
        conv = (np.abs(fn) <= 8.0 * EPS * En) | (iters[e_idx] >= MAX_ITERS)
        done[e_idx] = conv
    return o, tau, iters


def lowner_z(d, z, o, tau, chunk: int = 512):
    """Gu-Eisenstat recomputation of z (eq. bdc-zi), sign taken from z.

    |zt_i|^2 = (w_N^2 - d_i^2) prod_{k<i} (w_k^2 - d_i^2)/(d_k^2 - d_i^2)
                               prod_{i<=k<N-1} (w_k^2 - d_i^2)/(d_{k+1}^2 - d_i^2)
    with every w_k^2 - d_i^2 formed as (d_{o_k} - d_i + tau_k)(d_{o_k} + d_i + tau_k).
    By interlacing every ratio lies in (0, 1), so the product cannot overflow
    and it cannot underflow below its own (final) value.
    """
    d = np.asarray(d, dtype=np.float64)
    N = d.shape[0]
    ov = d[o]
    zt = np.empty(N)
    kk = np.arange(N - 1)
    for start in range(0, N, chunk):
        i = np.arange(start, min(N, start + chunk))
        di = d[i][:, None]
        num = (ov[None, :] - di + tau[None, :]) * (ov[None, :] + di + tau[None, :])
        # denominator pole for ratio k: d_k if k < i, d_{k+1} if k >= i
        pole = np.where(kk[None, :] < i[:, None], d[kk][None, :], d[kk + 1][None, :])
        ratios = num[:, :N - 1] / ((pole - di) * (pole + di))
        prod = num[:, N - 1] * np.prod(ratios, axis=1)
        zt[i] = np.copysign(np.sqrt(prod), z[i])
    return zt


def vectors(d, zt, o, tau, chunk: int = 2048):
    """Singular vectors of M~ = e_1 zt^T + diag(d) (eq. M-svd-vec).

    Column i: v = [zt_j / (d_j^2 - w_i^2)]_j normalised; u = [-1, d_j v_j]_{j>=2}
    (built from the unnormalised v) normalised, with
    d_j^2 - w_i^2 = ((d_j - d_{o_i}) - tau_i)(d_j + d_{o_i} + tau_i).
    Returns (U_M, V_M), both N x N, columns in root order.
    """
    d = np.asarray(d, dtype=np.float64)
    N = d.shape[0]
    if N == 1:
        # M~ = [zt_1] with omega = |zt_1| >= 0: u = [-1] and v = zt/(0 - omega^2)
        # normalised = [-1] (also the limit when omega = 0)
        return -np.ones((1, 1)), -np.ones((1, 1))
    ov = d[o]
    U = np.empty((N, N))
    V = np.empty((N, N))
    for start in range(0, N, chunk):
        c = slice(start, min(N, start + chunk))
        delta = (d[:, None] - ov[None, c] - tau[None, c]) * (d[:, None] + ov[None, c] + tau[None, c])
        v = zt[:, None] / delta
        u = d[:, None] * v
        u[0, :] = -1.0
        V[:, c] = v / np.sqrt(np.sum(v * v, axis=0))[None, :]
        U[:, c] = u / np.sqrt(np.sum(u * u, axis=0))[None, :]
    return U, V
