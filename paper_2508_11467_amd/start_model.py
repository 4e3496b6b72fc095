"""Parameters of the learned secular start shipped with the package.

The network (19 features -> 64 -> 64 -> 64 -> 1) is trained by
``train_start.py`` on the GPU with the library's own kernels and stored as a
flat float32 vector in ``data/start_mlp.npy``.
"""

from __future__ import annotations

import os

import numpy as np

from ._lib import MLP_PARAMS

HERE = os.path.dirname(os.path.abspath(__file__))
PARAMS_PATH = os.path.join(HERE, "data", "start_mlp.npy")


def load_params(path: str | None = None) -> np.ndarray:
    p = path or PARAMS_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"{p} not found: train the start network with "
                           "python -m paper_2508_11467_amd.train_start")
    a = np.load(p, allow_pickle=False)
    if a.dtype != np.float32 or a.shape != (MLP_PARAMS,):
        raise ValueError(f"{p}: expected {MLP_PARAMS} float32 parameters")
    return a


def init_params(seed: int = 0) -> np.ndarray:
    """He-style initial parameters (flat float32): W ~ N(0, 2/fan_in), b = 0."""
    g = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for fi, fo in [(19, 64), (64, 64), (64, 64), (64, 1)]:
        parts.append(g.standard_normal(fi * fo) * np.sqrt(2.0 / fi))
        parts.append(np.zeros(fo))
    return np.concatenate(parts).astype(np.float32)
