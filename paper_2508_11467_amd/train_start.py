"""Train the learned secular start on the GPU.

    python -m paper_2508_11467_amd.train_start [--roots 1000000] [--epochs 12]

1. Harvest: plain solves of seeded bidiagonals drawn like the n = 256 uniform
   configuration, the three n = 4096 spectra (uniform, graded, heavy
   deflation), d = e = 1 perturbed by 10% and by 1e-6 (little deflation:
   large merges that keep most values; the second with the evenly spread
   spectrum of d = e = 1), with training seeds distinct from every measured
   configuration's seed, until at least ``--roots`` secular roots have been
   collected; each root contributes its 19 features and the position of the
   computed root in its interval.  A held-out set is drawn the same way from
   validation seeds.
2. Train: Adam on the mean squared error of the proposed position, in the
   library's forward/backward kernels (bfloat16 matrix cores, FP32
   accumulation), shuffled mini-batches, learning rate decayed by a cosine
   over the epochs.
3. Evaluate: held-out loss, and the mean secular evaluations per root of
   plain and learned solves of held-out problems (overall and per problem).
4. Write the parameters (float32) to ``data/start_mlp.npy`` and print one
   JSON line.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np
import torch

from . import inputs
from .api import Solver
from .start_model import PARAMS_PATH, init_params

def ones_jitter(n: int, seed: int) -> tuple:
    """d, e iid 1 + 1e-6 U(-1, 1): d = e = 1 up to a jitter far below the
    spacing of its spectrum."""
    g = np.random.Generator(np.random.PCG64(seed))
    d = 1.0 + 1e-6 * g.uniform(-1.0, 1.0, n)
    e = 1.0 + 1e-6 * g.uniform(-1.0, 1.0, max(n - 1, 0))
    return d, e


# (generator, n, config, spectrum) of the harvest mix, one round
MIX = [(inputs.uniform, 256, 1, 0)] * 8 + [
    (inputs.uniform, 4096, 2, 0),
    (inputs.graded, 4096, 2, 1),
    (inputs.clustered, 4096, 2, 2),
    (inputs.near_ones, 4096, 2, 3),
    (ones_jitter, 2048, 2, 4),
    (ones_jitter, 3072, 2, 5),
    (ones_jitter, 4096, 2, 6),
]


def harvest(solver: Solver, split: str, target: int, capacity: int, log) -> tuple:
    X, y, tag, count = solver.harvest(capacity)
    k = 0
    problems = 0
    while True:
        for gen, n, cfg, spec in MIX:
            d, e = gen(n, inputs.split_seed(cfg, spec, split, k))
            solver.svd(d, e)
            problems += 1
        k += 1
        got = int(count.item())
        if got >= target or got >= capacity:
            break
    solver.stop_harvest()
    rows = min(int(count.item()), capacity)
    log(f"harvest {split}: {rows} roots from {problems} solves")
    return X[:rows], y[:rows]


def evaluate_iters(params: np.ndarray, problems) -> dict:
    """Mean evaluations per root of plain and learned (every merge) solves,
    over all problems and per problem (name -> (d, e))."""
    out = {}
    for start in ("plain", "learned"):
        s = Solver(0, start=start, mlp_params=params if start == "learned" else None, use_graph=False,
                   learned_min_n=0)
        ev = roots = 0
        per = {}
        for name, (d, e) in problems.items():
            s.svd(d, e)
            info, st = s.info()
            assert info == 0, info
            ev += st["secular_evals"]
            roots += st["roots"]
            per[name] = st["secular_evals"] / max(st["roots"], 1)
        s.close()
        out[start] = ev / max(roots, 1)
        out[start + "_per_problem"] = per
    return out


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--roots", type=int, default=1_000_000)
    ap.add_argument("--valid-roots", type=int, default=100_000)
    ap.add_argument("--epochs", type=int, default=12)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=PARAMS_PATH)
    args = ap.parse_args(argv)

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    t0 = time.time()
    solver = Solver(0, use_graph=False)
    Xt, yt = harvest(solver, "train", args.roots, args.roots + 200_000, log)
    Xv, yv = harvest(solver, "valid", args.valid_roots, args.valid_roots + 100_000, log)
    solver.mlp_set(init_params(args.seed))
    rows = Xt.shape[0]
    g = torch.Generator(device="cuda")
    g.manual_seed(args.seed)
    steps_per_epoch = rows // args.batch
    hist = []
    for ep in range(args.epochs):
        lr = 1e-4 + 0.5 * (args.lr - 1e-4) * (1.0 + math.cos(math.pi * ep / max(args.epochs, 1)))
        idx = torch.randperm(rows, generator=g, device="cuda").to(torch.int32)
        losses = solver.mlp_train(Xt, yt, idx[: steps_per_epoch * args.batch], args.batch, lr)
        vloss, _ = solver.mlp_grad(Xv, yv)
        hist.append((float(losses.mean().item()), vloss))
        log(f"epoch {ep}: lr {lr:.2e} train {hist[-1][0]:.5f} valid {vloss:.5f}")
    params = solver.mlp_get()
    solver.close()
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    np.save(args.out, params.astype(np.float32))
    # held-out problems for the iteration count: the n = 4096 spectra, one
    # N(0,1) bidiagonal of n = 8192 (a spectrum the network was not trained
    # on) and d = e = 1 at n = 4096
    probs = {f"{gen.__name__}_{n}": gen(n, inputs.split_seed(cfg, spec, "valid", 10_000))
             for gen, n, cfg, spec in MIX[8:]}
    probs["normal_8192"] = inputs.normal(8192, inputs.split_seed(3, 0, "valid", 10_000))
    probs["ones_4096"] = inputs.ones(4096)
    iters = evaluate_iters(params, probs)
    print(json.dumps({
        "train_roots": rows, "valid_roots": int(Xv.shape[0]), "epochs": args.epochs, "batch": args.batch,
        "steps": steps_per_epoch * args.epochs, "final_train_loss": hist[-1][0], "final_valid_loss": hist[-1][1],
        "valid_label_variance": float(torch.var(yv).item()),
        "iters_per_root_plain": iters["plain"], "iters_per_root_learned": iters["learned"],
        "iters_per_root_plain_per_problem": iters["plain_per_problem"],
        "iters_per_root_learned_per_problem": iters["learned_per_problem"],
        "seconds": time.time() - t0, "out": os.path.relpath(args.out),
    }), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
