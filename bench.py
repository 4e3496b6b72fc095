"""Benchmark: bidiagonal divide-and-conquer SVD with full vectors, FP64, one
MI355X.

Default workload: n = 16384 upper bidiagonal with d, e iid N(0, 1) (fixed
seed), sigma + full U and V^T.  A step is one whole solve with the inputs
already resident in HBM.  Prints one JSON line.

  value     nominal GFLOP/s = (8/3) n^3 / time  (the paper's convention,
            Section 4.2.2; deflation removes most of that work, so the
            executed vector-update flops are reported beside it)
  roofline  the kernel kind with the largest share of the timed region,
            measured with HIP events on the solve's stream, against its
            bound (MFMA FP64 peak, HBM bandwidth, or FP64 vector ALU)
  cpu_baseline  the CPU oracle timed on a bounded sample of the same
            workload family on this host
  learned   the same workload with the learned secular start (the MLP's
            proposal as each root's first point): time and secular
            evaluations per root next to the plain start's; config5 repeats
            the comparison at n = 32768 (d, e iid N(0,1))
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP64_MFMA = 78.6e12     # dense FP64 matrix, FLOP/s
PEAK_FP64_VALU = 78.6e12     # FP64 vector, FLOP/s
PEAK_HBM = 8.0e12            # bytes/s
METRIC = "bidiag SVD+vectors time & GFLOP/s at n=16384 FP64; secular iters/root, learned vs plain"

WORKLOADS = {
    "n16384_normal": ("n = 16384, d, e iid N(0,1), seed 250811767", 16384),
    "n32768_normal": ("n = 32768, d, e iid N(0,1), seed 250811967", 32768),
    "n16384_ones": ("n = 16384, d = e = 1 (no deflation, update-GEMM bound)", 16384),
    "n4096_uniform": ("n = 4096, d, e iid U(-1,1)", 4096),
    "batch2000": ("2000 bidiagonals, sizes round(exp(U(ln 32, ln 2048))), d, e iid U(-1,1)", 0),
    "sigma_laws": ("n = 1024 bidiagonals with the paper's singular-value laws (logrand, arith, geo at "
                   "theta = 1e6 and 1e12), built by Golub-Kahan-Lanczos on diag(sigma)", 1024),
}
SIGMA_LAWS = [("logrand", 1e6), ("arith", 1e6), ("geo", 1e6), ("geo", 1e12), ("logrand", 1e12)]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="n16384_normal", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-n", type=int, default=4096, help="size of the CPU oracle sample")
    ap.add_argument("--no-config5", action="store_true", help="skip the n = 32768 plain/learned comparison")
    ap.add_argument("--no-ozaki", action="store_true", help="skip the split-precision comparison")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-start comparison")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="bytes of one device-to-device copy issued first (calibrates HBM counters)")
    return ap.parse_args()


def kernel_work(kind: str, stats: dict, n2: float, launches: int):
    """(bound, algorithmic units per launch, unit, peak) of a kernel kind;
    n2 = sum of n^2 over the problems of a solve."""
    if kind == "update_gemm":
        return "mfma", stats["update_flops"] / max(launches, 1), "TFLOP/s", PEAK_FP64_MFMA
    if kind == "final":
        # write U and V^T in full; read each column's support once
        byts = 8.0 * (2.0 * n2 + stats["final_read_elems"])
        return "hbm", byts / max(launches, 1), "GB/s", PEAK_HBM
    if kind == "gather":
        return "hbm", stats["gather_bytes"] / max(launches, 1), "GB/s", PEAK_HBM
    if kind == "secular":
        # ~12 FP64 flops per pole term per evaluation
        return "alu", 12.0 * stats["secular_terms"] / max(launches, 1), "TFLOP/s", PEAK_FP64_VALU
    if kind == "leaf":
        return "alu", stats["leaf_flops"] / max(launches, 1), "TFLOP/s", PEAK_FP64_VALU
    return "hbm", 0.0, "GB/s", PEAK_HBM


# the kernels a timed kind consists of (single-problem solves; the final
# pass of a size that is not a multiple of 4096 is k_final_u + k_final_vt)
KIND_KERNELS = {
    "final": ["k_final_meta", "k_final_u_chunks", "k_final_vt_chunks"],
    "deflate": ["k_zsort", "k_prep_w", "k_prep"],
    "secular": ["k_secular"],
    "update_gemm": ["k_update"],
}


def measured_traffic(workload: str, kind: str):
    """HBM bytes per launch of a kernel kind from the committed counter
    summary (profiles/traffic_<workload>_<kind>.json), or None when there is
    none or it was taken from other kernel sources than the ones built."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}_{kind}.json")
    if not os.path.exists(path):
        return None
    from paper_2508_11467_amd.build import source_hash
    t = json.load(open(path))
    if t.get("source_hash") != source_hash():
        return None
    return t.get("traffic_bytes_per_launch")


def time_solver(solver, dt, et, out, steps: int, warmup: int) -> float:
    import torch
    for _ in range(warmup):
        solver.svd(dt, et, out=out)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        solver.svd(dt, et, out=out)
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


def accuracy(d, e, sig, U, VT) -> dict:
    """Residual ||B V - U S||_F / ||B||_F and orthogonality of U and V, on the
    GPU in FP64."""
    import numpy as np
    import torch
    n = len(d)
    dev = sig.device
    dt = torch.from_numpy(d).to(dev)
    et = torch.from_numpy(np.concatenate([e, [0.0]])).to(dev)
    V = VT.T
    BV = dt[:, None] * V
    BV[:-1] += et[:-1, None] * V[1:]
    nb = math.sqrt(float(np.sum(d * d) + np.sum(e * e)))
    res = float(torch.linalg.norm(BV - U * sig[None, :])) / nb
    del BV
    Uc = U.contiguous()
    G = Uc.T.contiguous() @ Uc
    G.diagonal().sub_(1.0)
    ou = float(torch.max(torch.abs(G)))
    del G, Uc
    Vc = VT.contiguous()
    G = Vc @ Vc.T.contiguous()
    G.diagonal().sub_(1.0)
    ov = float(torch.max(torch.abs(G)))
    del G, Vc
    torch.cuda.empty_cache()
    return {"residual": res, "orth_U": ou, "orth_V": ov}


def plain_vs_learned(d, e, steps: int, warmup: int, tuning=None) -> dict:
    """ms per solve and secular evaluations per root with each start."""
    import torch

    from paper_2508_11467_amd.api import Solver
    n = len(d)
    dev = torch.device("cuda:0")
    dt = torch.from_numpy(d).to(dev)
    et = torch.from_numpy(e).to(dev)
    out = (torch.empty(n, dtype=torch.float64, device=dev), torch.empty((n, n), dtype=torch.float64, device=dev),
           torch.empty((n, n), dtype=torch.float64, device=dev))
    res = {}
    for start in ("plain", "learned"):
        s = Solver(0, start=start)
        if tuning:
            s.set_tuning(**tuning)
        ms = time_solver(s, dt, et, out, steps, warmup)
        info, st = s.info()
        s.close()
        res[start] = {"ms_per_step": ms, "secular_iters_per_root": st["secular_evals"] / max(st["roots"], 1),
                      "roots": st["roots"], "info": info}
    del out
    torch.cuda.empty_cache()
    return res


def batch_checks(sizes, d, e, sig, U, VT) -> dict:
    """Worst residual and orthogonality over the problems of a batch (GPU)."""
    import numpy as np
    import torch
    dev = sig.device
    dt = torch.from_numpy(d).to(dev)
    et = torch.from_numpy(e).to(dev)
    off = mo = 0
    wr = wo = 0.0
    for n in sizes:
        s = sig[off:off + n]
        u = U[mo:mo + n * n].view(n, n).T
        v = VT[mo:mo + n * n].view(n, n).T
        V = v.T
        BV = dt[off:off + n, None] * V
        BV[:-1] += et[off:off + n - 1, None] * V[1:]
        nb = torch.sqrt(torch.sum(dt[off:off + n] ** 2) + torch.sum(et[off:off + n - 1] ** 2))
        wr = max(wr, float(torch.linalg.norm(BV - u * s[None, :]) / nb))
        uc = u.contiguous()
        I = torch.eye(n, dtype=torch.float64, device=dev)
        wo = max(wo, float(torch.max(torch.abs(uc.T.contiguous() @ uc - I))),
                 float(torch.max(torch.abs(V.contiguous() @ V.T.contiguous() - I))))
        off += n
        mo += n * n
    return {"worst_residual": wr, "worst_orth": wo}


def bench_batched(args, desc):
    import numpy as np
    import torch

    from paper_2508_11467_amd import inputs
    from paper_2508_11467_amd.api import Solver
    sizes = inputs.batch_sizes(2000, 32, 2048, inputs.seed_for(4, 0)).tolist()
    d, e = inputs.batch_uniform(sizes, inputs.seed_for(4, 1))
    dev = torch.device("cuda:0")
    dt = torch.from_numpy(d).to(dev)
    et = torch.from_numpy(e).to(dev)
    tot = sum(sizes)
    tot2 = sum(x * x for x in sizes)
    out = (torch.empty(tot, dtype=torch.float64, device=dev), torch.empty(tot2, dtype=torch.float64, device=dev),
           torch.empty(tot2, dtype=torch.float64, device=dev))
    nominal = sum((8.0 / 3.0) * x ** 3 for x in sizes)

    def run(solver, steps, warmup):
        for _ in range(warmup):
            solver.svd_batched(sizes, dt, et, out=out)
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(steps):
            solver.svd_batched(sizes, dt, et, out=out)
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / steps

    solver = Solver(0)
    ms_default = run(solver, args.steps, args.warmup)
    t0 = time.perf_counter()
    tuned = solver.autotune(sizes, dt, et, out=out, repeats=2)
    tune_s = time.perf_counter() - t0
    ms = run(solver, args.steps, args.warmup)
    info, stats = solver.info()
    solver.close()
    ts = Solver(0, timing=True)
    ts.set_tuning(**tuned)
    run(ts, 1, 1)
    ts.clear_timing()
    ms_events = run(ts, args.steps, 0)
    timing = ts.timing()
    ts.close()
    kinds = {k: v for k, v in timing.items() if v[1] > 0}
    dom = max(kinds, key=lambda k: kinds[k][0])
    tot_ms, launches = kinds[dom]
    bound, work, unit, peak = kernel_work(dom, stats, float(tot2), launches / args.steps)
    avg_s = tot_ms * 1e-3 / launches
    scale = 1e9 if unit == "GB/s" else 1e12
    line = {
        "metric": METRIC, "value": nominal / (ms * 1e-3) / 1e9, "unit": "GFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": desc, "problems": len(sizes), "sum_n": tot, "leaf_size": 32},
        "autotuned": {"tuning": tuned, "ms_per_step_default": ms_default, "tuning_seconds": tune_s},
        "nominal_flops": nominal, "update_flops": stats["update_flops"], "roots": stats["roots"],
        "secular_iters_per_root": stats["secular_evals"] / max(stats["roots"], 1), "info": info,
        "kernel_ms_per_step": {k: v[0] / args.steps for k, v in sorted(kinds.items())},
        "ms_per_step_kernel_by_kernel": ms_events,
        "roofline": {"bound": bound, "kernel": dom, "achieved": work / avg_s / scale, "peak": peak / scale,
                     "unit": unit, "frac": work / avg_s / peak, "traffic": None, "avg_launch_ms": avg_s * 1e3,
                     "share_of_step": tot_ms / args.steps / ms_events},
        "checks": batch_checks(sizes, d, e, *out),
    }
    print(json.dumps(line), flush=True)


def bench_sigma_laws(args, desc, n):
    """Each law: time per solve (autotuned), the largest |sigma_k - law_k|
    relative to sigma_1 beside the generator's own bound delta, residual and
    orthogonality."""
    import numpy as np
    import torch

    from paper_2508_11467_amd import inputs
    from paper_2508_11467_amd.api import Solver
    dev = torch.device("cuda:0")
    out = (torch.empty(n, dtype=torch.float64, device=dev), torch.empty((n, n), dtype=torch.float64, device=dev),
           torch.empty((n, n), dtype=torch.float64, device=dev))
    per = {}
    total_ms = 0.0
    for k, (law, theta) in enumerate(SIGMA_LAWS):
        s = inputs.sigma_law(n, law, theta, seed=inputs.seed_for(6, k))
        d, e, delta = inputs.gkl_bidiagonal(s, inputs.seed_for(6, 10 + k))
        dt, et = torch.from_numpy(d).to(dev), torch.from_numpy(e).to(dev)
        solver = Solver(0)
        solver.autotune([n], dt, et, out=out, repeats=2)
        ms = time_solver(solver, dt, et, out, args.steps, args.warmup)
        info, _ = solver.info()
        solver.close()
        sig, ub, vb = out
        U, VT = ub.T, vb.T
        B = torch.diag(dt) + torch.diag(et, 1)
        I = torch.eye(n, dtype=torch.float64, device=dev)
        per[f"{law}({theta:g})"] = {
            "ms_per_step": ms,
            "sigma_err_rel": float(np.max(np.abs(sig.cpu().numpy() - s)) / s[0]),
            "generator_delta_rel": delta / s[0],
            "residual": float(torch.linalg.norm(B - (U * sig[None, :]) @ VT) / torch.linalg.norm(B)),
            "orth": max(float(torch.max(torch.abs(U.T @ U - I))), float(torch.max(torch.abs(VT @ VT.T - I)))),
            "info": info,
        }
        total_ms += ms
    nominal = len(SIGMA_LAWS) * (8.0 / 3.0) * n ** 3
    line = {
        "metric": METRIC, "value": nominal / (total_ms * 1e-3) / 1e9, "unit": "GFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": total_ms / len(SIGMA_LAWS),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": desc, "n": n}, "laws": per,
    }
    print(json.dumps(line), flush=True)


def cpu_baseline(n: int):
    import numpy as np  # noqa: F401

    import oracle
    from paper_2508_11467_amd import inputs

    d, e = inputs.normal(n, inputs.seed_for(3))
    t0 = time.perf_counter()
    oracle.bdsdc(d, e)
    t = time.perf_counter() - t0
    cores = len(os.sched_getaffinity(0))
    return {
        "value": (8.0 / 3.0) * n ** 3 / t / 1e9,
        "unit": "GFLOP/s",
        "cores": cores,
        "kind": "oracle",
        "sample": f"one n={n} N(0,1) bidiagonal (same generator) solved by the NumPy oracle in {t:.2f} s; "
                  f"nominal (8/3)n^3 flops",
        "seconds": t,
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (--gpus {args.gpus} requested); "
              "this solver has no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2508_11467_amd import inputs
    from paper_2508_11467_amd.api import Solver

    if args.copy_calibration > 0:
        src = torch.ones(args.copy_calibration // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    desc, n = WORKLOADS[args.workload]
    if args.workload == "batch2000":
        return bench_batched(args, desc)
    if args.workload == "sigma_laws":
        return bench_sigma_laws(args, desc, n)
    d, e = inputs.workload(args.workload)
    dev = torch.device("cuda:0")
    dt = torch.from_numpy(d).to(dev)
    et = torch.from_numpy(e).to(dev)
    sig = torch.empty(n, dtype=torch.float64, device=dev)
    ub = torch.empty((n, n), dtype=torch.float64, device=dev)
    vb = torch.empty((n, n), dtype=torch.float64, device=dev)
    # timed region 1: the solve as a caller runs it (graph replay), with the
    # default options and after the library's autotuner has picked the leaf
    # size and launch shapes for this workload (outside the timed region)
    solver = Solver(0)
    ms_default = time_solver(solver, dt, et, (sig, ub, vb), args.steps, args.warmup)
    tuned = solver.autotune([n], dt, et, out=(sig, ub, vb), repeats=2)
    tuning = {k: v for k, v in tuned.items() if k != "ms"}
    ms = time_solver(solver, dt, et, (sig, ub, vb), args.steps, args.warmup)
    info, stats = solver.info()
    solver.close()

    def tuned_solver(**kw):
        s = Solver(0, **kw)
        s.set_tuning(**tuning)
        return s

    # timed region 2: the same steps launched kernel by kernel, each launch
    # bracketed by HIP events on the solve's stream (per-kernel durations)
    tsolver = tuned_solver(timing=True)
    tsolver.svd(dt, et, out=(sig, ub, vb))
    torch.cuda.synchronize()
    tsolver.clear_timing()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(args.steps):
        tsolver.svd(dt, et, out=(sig, ub, vb))
    stop.record()
    torch.cuda.synchronize()
    ms_events = start.elapsed_time(stop) / args.steps
    timing = tsolver.timing()
    tsolver.close()

    sig_fp64 = sig.clone()
    acc_fp64 = accuracy(d, e, sig, ub.T, vb.T)

    # the same solves with split-precision update products
    ozaki = None
    if not args.no_ozaki:
        osv = tuned_solver(gemm="ozaki")
        ms_oz = time_solver(osv, dt, et, (sig, ub, vb), args.steps, args.warmup)
        info_o, _ = osv.info()
        osv.close()
        ozaki = {"ms_per_step": ms_oz, "value": (8.0 / 3.0) * n ** 3 / (ms_oz * 1e-3) / 1e9, "slices": int(osv.options.ozaki_slices),
                 "min_kept_values": 256, "info": info_o,
                 "sigma_max_rel_diff_vs_fp64": float(torch.max(torch.abs(sig - sig_fp64)) / sig_fp64[0]),
                 **accuracy(d, e, sig, ub.T, vb.T)}

    # the same solves with the learned start
    if not args.no_learned:
        ls = tuned_solver(start="learned")
        ms_learned = time_solver(ls, dt, et, (sig, ub, vb), args.steps, args.warmup)
        info_l, stats_l = ls.info()
        ls.close()

    nominal = (8.0 / 3.0) * n ** 3
    value = nominal / (ms * 1e-3) / 1e9

    # dominant kernel kind over the timed region
    kinds = {k: v for k, v in timing.items() if v[1] > 0}
    dom = max(kinds, key=lambda k: kinds[k][0])
    tot_ms, launches = kinds[dom]
    per_launch_launches = launches / args.steps
    bound, work, unit, peak = kernel_work(dom, stats, float(n) * n, per_launch_launches)
    avg_s = tot_ms * 1e-3 / launches
    achieved = work / avg_s
    scale = 1e9 if unit == "GB/s" else 1e12
    traffic = measured_traffic(args.workload, dom)
    roofline = {
        "bound": bound,
        "kernel": dom,
        "kernels": KIND_KERNELS.get(dom, []) if (dom != "final" or n % 4096 == 0) else ["k_final_u", "k_final_vt"],
        "achieved": achieved / scale,
        "peak": peak / scale,
        "unit": unit,
        "frac": achieved / peak,
        "traffic": traffic,
        "avg_launch_ms": avg_s * 1e3,
        "share_of_step": tot_ms / args.steps / ms_events,
    }
    iters_per_root = stats["secular_evals"] / max(stats["roots"], 1)
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": desc, "n": n, "leaf_size": tuning["leaf_size"], "secular_start": "plain",
                   "tuning": tuning},
        "ms_per_step_default_options": ms_default,
        "executed_update_gflops": stats["update_flops"] / (ms * 1e-3) / 1e9,
        "update_flops": stats["update_flops"],
        "nominal_flops": nominal,
        "secular_iters_per_root": iters_per_root,
        "root_N": stats["root_N"],
        "roots": stats["roots"],
        "info": info,
        "kernel_ms_per_step": {k: v[0] / args.steps for k, v in sorted(kinds.items())},
        "ms_per_step_kernel_by_kernel": ms_events,
        "roofline": roofline,
    }
    line["accuracy"] = acc_fp64
    if ozaki is not None:
        line["ozaki"] = ozaki
    if not args.no_learned:
        line["learned"] = {
            "ms_per_step": ms_learned,
            "value": nominal / (ms_learned * 1e-3) / 1e9,
            "secular_iters_per_root": stats_l["secular_evals"] / max(stats_l["roots"], 1),
            "secular_iters_per_root_plain": iters_per_root,
            "roots": stats_l["roots"],
            "info": info_l,
        }
    if not args.no_config5 and args.workload == "n16384_normal":
        del sig, ub, vb
        torch.cuda.empty_cache()
        d5, e5 = inputs.workload("n32768_normal")
        line["config5"] = {"workload": WORKLOADS["n32768_normal"][0],
                           **plain_vs_learned(d5, e5, max(2, args.steps // 3), 1, tuning)}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.cpu_n)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
