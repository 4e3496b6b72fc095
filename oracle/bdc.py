"""Oracle bidiagonal divide-and-conquer SVD (B = U Sigma V^T, full vectors).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Follows Section 4.2.1 of the paper (Algorithm 2): split the bidiagonal at
row k = floor(m/2), solve the bottom subproblems by QR iteration, then merge
bottom-up -- each merge forms z, sorts, deflates (``lasd2``), solves the
secular equation, recomputes z (Gu-Eisenstat), forms the singular vectors of
M and multiplies them into the children's bases (``lasd3``) -- and finally
sorts the values.  Every step is written in the plain form of the paper's
equations: the bases of a merge are assembled as explicit dense matrices and
the vector update is one dense product per side (eq. bdc-B-svd), so a reader
can check each line against the paper.  Readings of points the paper leaves
open are stated where they are used.

Notation for a node: it owns rows [r0, r0+m) and columns [r0, r0+m+s) of B,
s in {0, 1}.  The root is (0, n, 0).  A node with m > leaf splits at
k = floor(m/2): left child (r0, k-1, 1), right child (r0+k, m-k, s), and the
middle row r0+k-1 carries alpha = d[r0+k-1] (in the left child's last column)
and beta = e[r0+k-1] (in the right child's first column).
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from .leaf import leaf_svd, dense_bidiagonal
from .learned import learned_roots
from .secular import secular_roots, lowner_z, vectors

EPS = 2.0 ** -52
LEAF_DEFAULT = 32

# deflation status codes of a sorted position
SURVIVOR = 0
DEFL_SMALL_Z = 1     # |z_j| < tol
DEFL_ZERO_D = 2      # d_j < tol: rotated into z_1, value 0
DEFL_CLOSE = 3       # d_j - d_p < tol: rotated into the previous survivor


@dataclass
class Node:
    r0: int
    m: int
    s: int
    k: int = 0
    left: "Node | None" = None
    right: "Node | None" = None
    height: int = 0

    @property
    def is_leaf(self) -> bool:
        return self.left is None


def build_tree(n: int, leaf: int = LEAF_DEFAULT, r0: int = 0, s: int = 0) -> Node:
    """Recursive split at k = floor(m/2) until m <= leaf (Section 4.2.1)."""
    node = Node(r0=r0, m=n, s=s)
    if n > leaf:
        k = n // 2
        node.k = k
        node.left = build_tree(k - 1, leaf, r0, 1)
        node.right = build_tree(n - k, leaf, r0 + k, s)
        node.height = 1 + max(node.left.height, node.right.height)
    return node


def tree_nodes(root: Node) -> list[Node]:
    out = []
    stack = [root]
    while stack:
        x = stack.pop()
        out.append(x)
        if not x.is_leaf:
            stack.append(x.left)
            stack.append(x.right)
    return out


def scale_of(values) -> float:
    """Power of two p with max|v| / p in [0.5, 1) (1.0 when all are zero)."""
    vmax = 0.0
    for v in values:
        vmax = max(vmax, abs(float(v)))
    if vmax == 0.0 or not math.isfinite(vmax):
        return 1.0
    return math.ldexp(1.0, math.frexp(vmax)[1])


def merge_sort_order(dloc: np.ndarray, k: int) -> np.ndarray:
    """Sorted order of a merge's positions (Algorithm 3, sort step).

    Position k-1 (the new d = 0) comes first; then the left child's columns
    0..k-2 and the right child's columns k..m-1, each already ascending, are
    merged by value; equal values take the left child first.  Returns perm with
    perm[sorted position] = local column.
    """
    m = dloc.shape[0]
    out = [k - 1]
    i, j = 0, k
    while i < k - 1 and j < m:
        if dloc[j] < dloc[i]:
            out.append(j)
            j += 1
        else:
            out.append(i)
            i += 1
    out.extend(range(i, k - 1))
    out.extend(range(j, m))
    return np.array(out, dtype=np.int64)


def deflate(d: np.ndarray, z: np.ndarray, support: np.ndarray | None = None):
    """Deflation of M = e_1 z^T + diag(d) in place (``lasd2``).

    d (sorted ascending, d[0] = 0) and z are modified in place; returns
    (tol, status per position, rotations in scan order).  Follows eq.
    M-condition and the four cases listed after it.  Readings:
    eps*||M|| -> tol = 8 * 2^-52 * max(max d, max |z|) with strict "<"; the
    scan runs over positions 2..N in order and compares each with the last
    position that survived; in the close-value case the earlier position keeps
    the combined z and takes the later value (the worked example with
    i = 3, j = 2), and the later one is zeroed; a value within tol of d_1 = 0
    is set to 0; the floor on z_1 is applied after the scan.  An exactly zero
    z_j (or an exact tie) deflates even when tol is 0, which happens only
    when the whole merge is zero.  ``support``
    (1 = left child, 3 = right child, 2 = both) is updated when a close-value
    rotation mixes the two children.
    """
    m = d.shape[0]
    tol = 8.0 * EPS * max(float(np.max(d)), float(np.max(np.abs(z))))
    status = np.zeros(m, dtype=np.int64)
    rots = []
    last = -1
    for j in range(1, m):
        if abs(z[j]) < tol or z[j] == 0.0:
            # small z component: z_j -> 0, d_j is a singular value as it is
            z[j] = 0.0
            status[j] = DEFL_SMALL_Z
            continue
        if d[j] < tol or d[j] == 0.0:
            # |d_j - d_1| < tol: rotate z_j into z_1 from the right (M G^T),
            # the right basis only; d_j is set to 0
            r = math.sqrt(z[0] * z[0] + z[j] * z[j])
            c = z[0] / r
            sn = z[j] / r
            rots.append((DEFL_ZERO_D, 0, j, c, sn))
            z[0] = r
            z[j] = 0.0
            d[j] = 0.0
            status[j] = DEFL_ZERO_D
            continue
        if last >= 0 and (d[j] - d[last] < tol or d[j] == d[last]):
            # close values: G M G^T on both bases; the earlier position keeps
            # the combined z and takes the later value, the later is zeroed
            r = math.sqrt(z[last] * z[last] + z[j] * z[j])
            c = z[last] / r
            sn = z[j] / r
            rots.append((DEFL_CLOSE, last, j, c, sn))
            z[last] = r
            z[j] = 0.0
            d[last] = d[j]
            if support is not None and support[last] != support[j]:
                support[last] = 2
                support[j] = 2
            status[j] = DEFL_CLOSE
            continue
        last = j
    # small z_1: raised to tol (first case of the small-z deflation)
    if z[0] < tol:
        z[0] = tol
    return tol, status, rots


@dataclass
class Prep:
    """Everything the z / sort / deflation stage (``lasd2``) decides."""
    scale: float
    c0: float
    s0: float
    tol: float
    perm: np.ndarray          # sorted position -> local column
    d: np.ndarray             # values at sorted positions after deflation (scaled)
    z: np.ndarray             # z at sorted positions after deflation (scaled)
    status: np.ndarray        # per sorted position
    rots: list = field(default_factory=list)   # (kind, p, j, c, s), sorted positions
    survivors: np.ndarray = None               # sorted positions, ascending (0 first)
    deflated: np.ndarray = None                # sorted positions, in value order
    support: np.ndarray = None                 # per sorted position: 1 left, 3 right, 2 both, 0 middle
    group: np.ndarray = None                   # group order of the vector update (sorted positions)
    counts: tuple = (0, 0, 0)                  # (n1, n2, n3)
    d_local: np.ndarray = None                 # values before sorting, local column order
    z_local: np.ndarray = None                 # z before deflation, local column order


def merge_prep(sig1, sig2, qrow1, qrow2, alpha, beta, s) -> Prep:
    """z formation, scaling, sort and deflation of one merge.

    sig1 (k-1,), sig2 (m2,): children's values, ascending.
    qrow1 (k,): last row of the left child's right basis [Q1 q1]; qrow1[k-1]
      is the last entry lambda_1 of its null vector q1.
    qrow2 (m2+s,): first row of the right child's right basis; with s = 1,
      qrow2[m2] = phi_2 is the first entry of its null vector q2.
    alpha, beta: the middle row's entries (Section 4.2.1 divide step).
    """
    sig1 = np.asarray(sig1, dtype=np.float64)
    sig2 = np.asarray(sig2, dtype=np.float64)
    k = sig1.shape[0] + 1
    m2 = sig2.shape[0]
    m = k + m2

    # Scaling by a power of two (not in the paper; exact, so it changes no
    # decision): every value of the merge lies in [0, 1) afterwards.
    p = scale_of([alpha, beta] + list(sig1) + list(sig2))
    a_s = alpha / p
    b_s = beta / p

    # z (Algorithm 3 first step).  Row k of B_node times the children's right
    # bases: alpha * last row of [Q1 q1] and beta * first row of [Q2 q2].
    # The two null-vector entries combine into one rotation (c0, s0):
    # x1 = c0 [q1; 0] + s0 [0; q2] carries z_1 = r0 and
    # y = -s0 [q1; 0] + c0 [0; q2] becomes the node's null vector.
    lam1 = float(qrow1[k - 1])
    phi2 = float(qrow2[m2]) if s == 1 else 0.0
    a = a_s * lam1
    b = b_s * phi2
    r0 = math.sqrt(a * a + b * b)
    if r0 == 0.0:
        c0, s0 = 1.0, 0.0
    else:
        c0, s0 = a / r0, b / r0

    dloc = np.empty(m)
    zloc = np.empty(m)
    dloc[:k - 1] = sig1 / p
    dloc[k - 1] = 0.0
    dloc[k:] = sig2 / p
    zloc[:k - 1] = a_s * np.asarray(qrow1[:k - 1], dtype=np.float64)
    zloc[k - 1] = r0
    zloc[k:] = b_s * np.asarray(qrow2[:m2], dtype=np.float64)

    perm = merge_sort_order(dloc, k)
    d = dloc[perm].copy()
    z = zloc[perm].copy()
    support = np.where(perm < k - 1, 1, np.where(perm >= k, 3, 0)).astype(np.int64)

    tol, status, rots = deflate(d, z, support)

    survivors = np.array([0] + [j for j in range(1, m) if status[j] == SURVIVOR], dtype=np.int64)
    # deflated values in ascending order: the zeros of case DEFL_ZERO_D first,
    # then the others in scan order (their d are the sorted, untouched values)
    zero_d = [j for j in range(1, m) if status[j] == DEFL_ZERO_D]
    other = [j for j in range(1, m) if status[j] in (DEFL_SMALL_Z, DEFL_CLOSE)]
    deflated = np.array(zero_d + other, dtype=np.int64)
    sup = support[survivors]
    t1 = survivors[sup == 1]
    t2 = survivors[sup == 2]
    t3 = survivors[sup == 3]
    group = np.concatenate([t1, [0], t2, t3, deflated]).astype(np.int64)
    return Prep(scale=p, c0=c0, s0=s0, tol=tol, perm=perm, d=d, z=z, status=status,
                rots=rots, survivors=survivors, deflated=deflated, support=support,
                group=group, counts=(len(t1), len(t2), len(t3)),
                d_local=dloc, z_local=zloc)


def merge_values(omega: np.ndarray, defl: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Merge ascending roots with ascending deflated values; ties put roots
    first.  Returns (dest of each root, dest of each deflated value)."""
    N = omega.shape[0]
    D = defl.shape[0]
    dest_r = np.empty(N, dtype=np.int64)
    dest_d = np.empty(D, dtype=np.int64)
    i = j = pos = 0
    while i < N or j < D:
        if j >= D or (i < N and omega[i] <= defl[j]):
            dest_r[i] = pos
            i += 1
        else:
            dest_d[j] = pos
            j += 1
        pos += 1
    return dest_r, dest_d


@dataclass
class MergeStats:
    r0: int
    m: int
    s: int
    N: int
    n_small_z: int
    n_zero_d: int
    n_close: int
    counts: tuple
    iters: np.ndarray
    # the merge's secular problem and its roots (kept values ascending)
    dS: np.ndarray | None = None
    zS: np.ndarray | None = None
    o: np.ndarray | None = None
    tau: np.ndarray | None = None


def merge(node: Node, left, right, d, e, stats: list | None = None, start=None):
    """Conquer one node from its children's SVDs (Algorithm 2 step (2)).

    start: None for the plain secular start, else a callable (d, z) -> x_hat
    proposing each root's position in its interval (learned start).
    """
    sig1, W1, Q1 = left
    sig2, W2, Q2 = right
    r0, m, s, k = node.r0, node.m, node.s, node.k
    m2 = m - k
    alpha = float(d[r0 + k - 1])
    beta = float(e[r0 + k - 1])
    pr = merge_prep(sig1, sig2, Q1[k - 1, :], Q2[0, :], alpha, beta, s)

    # Bases of eq. bdc-B: left columns in local column order
    # [W1 columns | e_{k-1} (middle row) | W2 columns]; right columns
    # [Q1 columns | x1 | Q2 columns | y (s = 1)].
    L = np.zeros((m, m))
    L[:k - 1, :k - 1] = W1
    L[k - 1, k - 1] = 1.0
    L[k:, k:] = W2
    R = np.zeros((m + s, m + s))
    R[:k, :k - 1] = Q1[:, :k - 1]
    R[k:, k:m] = Q2[:, :m2]
    q1 = np.zeros(m + s)
    q1[:k] = Q1[:, k - 1]
    q2 = np.zeros(m + s)
    if s == 1:
        q2[k:] = Q2[:, m2]
    R[:, k - 1] = pr.c0 * q1 + pr.s0 * q2
    if s == 1:
        R[:, m] = -pr.s0 * q1 + pr.c0 * q2

    # columns in sorted order, then the deflation rotations in scan order
    Ls = L[:, pr.perm].copy()
    Rs = R[:, pr.perm].copy()
    for kind, pp, j, c, sn in pr.rots:
        if kind == DEFL_CLOSE:
            lp_, lj = Ls[:, pp].copy(), Ls[:, j].copy()
            Ls[:, pp] = c * lp_ + sn * lj
            Ls[:, j] = -sn * lp_ + c * lj
        rp_, rj = Rs[:, pp].copy(), Rs[:, j].copy()
        Rs[:, pp] = c * rp_ + sn * rj
        Rs[:, j] = -sn * rp_ + c * rj

    surv = pr.survivors
    dS = pr.d[surv]
    zS = pr.z[surv]
    if start is None:
        o, tau, iters = secular_roots(dS, zS)
    else:
        o, tau, iters = learned_roots(dS, zS, start(dS, zS))
    zt = lowner_z(dS, zS, o, tau)
    UM, VM = vectors(dS, zt, o, tau)
    omega = dS[o] + tau

    # eq. bdc-B-svd: new vectors = (non-deflated basis columns) x (vectors of M)
    Wr = Ls[:, surv] @ UM
    Qr = Rs[:, surv] @ VM

    dv = pr.d[pr.deflated]
    dest_r, dest_d = merge_values(omega, dv)
    sig = np.empty(m)
    W = np.empty((m, m))
    Q = np.empty((m + s, m + s))
    sig[dest_r] = omega * pr.scale
    sig[dest_d] = dv * pr.scale
    W[:, dest_r] = Wr
    W[:, dest_d] = Ls[:, pr.deflated]
    Q[:, dest_r] = Qr
    Q[:, dest_d] = Rs[:, pr.deflated]
    if s == 1:
        Q[:, m] = R[:, m]
    if stats is not None:
        st = pr.status
        stats.append(MergeStats(r0=r0, m=m, s=s, N=int(surv.shape[0]),
                                n_small_z=int(np.sum(st == DEFL_SMALL_Z)),
                                n_zero_d=int(np.sum(st == DEFL_ZERO_D)),
                                n_close=int(np.sum(st == DEFL_CLOSE)),
                                counts=pr.counts, iters=iters,
                                dS=dS, zS=zS, o=o, tau=tau))
    return sig, W, Q


def solve_node(node: Node, d, e, stats=None, start=None):
    """SVD of the node's m x (m+s) block: (sigma asc, W, Q)."""
    if node.is_leaf:
        r0, m, s = node.r0, node.m, node.s
        dd = d[r0:r0 + m]
        ee = e[r0:r0 + m - 1 + s]
        sig, W, Q, _ = leaf_svd(dd, ee, s)
        return sig, W, Q
    left = solve_node(node.left, d, e, stats, start)
    right = solve_node(node.right, d, e, stats, start)
    return merge(node, left, right, d, e, stats, start)


def bdsdc(d, e, leaf: int = LEAF_DEFAULT, return_stats: bool = False, start=None):
    """B = U diag(sigma) VT for the n x n upper bidiagonal (d, e).

    Returns (sigma descending, U, VT[, stats]).  Algorithm 2 step (3): the
    root's ascending order is reversed.
    """
    d = np.asarray(d, dtype=np.float64)
    e = np.asarray(e, dtype=np.float64)
    n = d.shape[0]
    stats: list = []
    if n == 0:
        res = (np.zeros(0), np.zeros((0, 0)), np.zeros((0, 0)))
        return res + (stats,) if return_stats else res
    ee = np.zeros(n)
    ee[:n - 1] = e[:n - 1]
    root = build_tree(n, leaf)
    sig, W, Q = solve_node(root, d, ee, stats, start)
    sigma = sig[::-1].copy()
    U = W[:, ::-1].copy()
    VT = Q[:, ::-1].T.copy()
    if return_stats:
        return sigma, U, VT, stats
    return sigma, U, VT


def dense(d, e) -> np.ndarray:
    """Dense n x n upper bidiagonal."""
    d = np.asarray(d, dtype=np.float64)
    return dense_bidiagonal(d, np.asarray(e, dtype=np.float64)[: max(len(d) - 1, 0)], 0)
