"""Writes the full-size expected singular values in this folder.

Every value here comes from ``oracle/`` alone, on the seeded inputs of
``paper_2508_11467_amd.inputs`` (a module that only draws random numbers):

* ``oracle_sigma_n16384_normal.npy`` -- oracle.bdsdc (the CPU divide-and-
  conquer) on the n = 16384 N(0,1) bidiagonal; needs about 20 GB of RAM.
* ``sturm_sigma_n16384_normal.npy`` -- oracle.sturm bisection on the same
  input: an independent route to the same spectrum (the CPU tests compare
  the two).
* ``sturm_sigma_n32768_normal.npy`` -- oracle.sturm on the n = 32768 N(0,1)
  bidiagonal (the dense oracle would need more than 50 GB there).
* ``oracle_sigma_batch2000_sample.npz``-style pair: ``batch2000_sample_idx.npy``
  (100 problem indices of the 2000-problem batch, 10 from each of 10 size
  strata of equal width in log n) and ``oracle_sigma_batch2000_sample.npy``
  (their oracle.bdsdc values, concatenated in index order).

Arrays are float64 / int64 .npy files (read with numpy.load, no pickle).
Usage: python tests/golden/make_oracle_sigma.py [n16384|sturm16384|n32768|batch]...
"""

from __future__ import annotations

import os
import sys
import time
from multiprocessing import Pool

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle import sturm  # noqa: E402
from paper_2508_11467_amd import inputs  # noqa: E402

WORKERS = int(os.environ.get("GOLDEN_WORKERS", "8"))


def _sturm_chunk(args):
    d, e, idx = args
    return sturm.singular_values(d, e, index=idx)


def sturm_all(d, e):
    n = len(d)
    chunks = np.array_split(np.arange(n), WORKERS * 4)
    with Pool(WORKERS) as p:
        parts = p.map(_sturm_chunk, [(d, e, c) for c in chunks])
    return np.concatenate(parts)


def batch_sample():
    """10 problems from each of 10 strata of equal width in log n over
    [32, 2048], drawn with a fixed seed; sorted problem indices."""
    sizes = inputs.batch_sizes(2000, 32, 2048, inputs.seed_for(4, 0))
    edges = np.exp(np.linspace(np.log(32), np.log(2048), 11))
    edges[-1] += 1
    g = np.random.default_rng(4_2000)
    pick = []
    for a, b in zip(edges[:-1], edges[1:]):
        members = np.nonzero((sizes >= a) & (sizes < b))[0]
        pick.extend(g.choice(members, min(10, len(members)), replace=False).tolist())
    return np.array(sorted(pick), dtype=np.int64)


def _oracle_problem(args):
    d, e = args
    s, _, _ = oracle.bdsdc(d, e)
    return s


def main(what):
    t0 = time.time()
    if "n16384" in what:
        d, e = inputs.workload("n16384_normal")
        s, _, _ = oracle.bdsdc(d, e)
        np.save(os.path.join(HERE, "oracle_sigma_n16384_normal.npy"), s)
        print(f"oracle n16384_normal done {time.time() - t0:.0f}s", flush=True)
    if "sturm16384" in what:
        d, e = inputs.workload("n16384_normal")
        np.save(os.path.join(HERE, "sturm_sigma_n16384_normal.npy"), sturm_all(d, e))
        print(f"sturm n16384_normal done {time.time() - t0:.0f}s", flush=True)
    if "n32768" in what:
        d, e = inputs.workload("n32768_normal")
        np.save(os.path.join(HERE, "sturm_sigma_n32768_normal.npy"), sturm_all(d, e))
        print(f"sturm n32768_normal done {time.time() - t0:.0f}s", flush=True)
    if "batch" in what:
        sizes = inputs.batch_sizes(2000, 32, 2048, inputs.seed_for(4, 0))
        d, e = inputs.batch_uniform(sizes.tolist(), inputs.seed_for(4, 1))
        off = np.concatenate([[0], np.cumsum(sizes)])
        idx = batch_sample()
        jobs = [(d[off[i]:off[i + 1]], e[off[i]:off[i + 1] - 1]) for i in idx]
        with Pool(WORKERS) as p:
            parts = p.map(_oracle_problem, jobs)
        np.save(os.path.join(HERE, "batch2000_sample_idx.npy"), idx)
        np.save(os.path.join(HERE, "oracle_sigma_batch2000_sample.npy"), np.concatenate(parts))
        print(f"batch sample done {time.time() - t0:.0f}s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["n16384", "sturm16384", "n32768", "batch"])
