"""Writes the expected values of the tall-and-skinny QR in this folder, from
``oracle/`` alone on the seeded input of ``paper_2508_11467_amd.inputs``
(a module that only draws random numbers):

* ``oracle_qr_ts20000x1000.npy`` -- float64 array of shape (3, 1000): the
  diagonal of R, tau, and the first row of R, from oracle.householder.qr on
  the m = 20000, n = 1000 N(0,1) matrix (the tall-and-skinny size of the
  paper's accuracy experiments, Section 5.1).

Read with numpy.load (no pickle).  Usage: python tests/golden/make_oracle_qr.py
"""

from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import householder as hh  # noqa: E402
from paper_2508_11467_amd import inputs  # noqa: E402


def main() -> None:
    m, n = 20000, 1000
    A = inputs.dense_normal(m, n, inputs.DENSE_TS_SEED)
    t0 = time.perf_counter()
    R, _, tau = hh.qr(A)
    print(f"oracle QR {m}x{n}: {time.perf_counter() - t0:.1f} s", flush=True)
    out = np.stack([np.diag(R).copy(), tau, R[0].copy()])
    np.save(os.path.join(HERE, "oracle_qr_ts20000x1000.npy"), out, allow_pickle=False)


if __name__ == "__main__":
    main()
