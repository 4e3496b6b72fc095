"""Batched solves of uneven sizes against single solves and the oracle."""

import os

import numpy as np
import pytest

import oracle
from paper_2508_11467_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def solver(gpu):
    from paper_2508_11467_amd.api import Solver
    s = Solver(0)
    yield s
    s.close()


def unpack(sizes, sig, U, VT):
    out = []
    off = mo = 0
    for n in sizes:
        s = sig[off:off + n]
        u = U[mo:mo + n * n].reshape(n, n).T
        v = VT[mo:mo + n * n].reshape(n, n).T
        out.append((s, u, v))
        off += n
        mo += n * n
    return out


def test_batched_matches_single_solves(solver):
    import torch
    sizes = [1, 2, 33, 5, 0, 64, 200, 31, 300, 65, 7, 129]
    d, e = inputs.batch_uniform(sizes, 77)
    sig, U, VT = solver.svd_batched(sizes, torch.from_numpy(d), torch.from_numpy(e))
    info, st = solver.info()
    assert info == 0
    res = unpack(sizes, sig.cpu().numpy(), U.cpu().numpy(), VT.cpu().numpy())
    off = 0
    for n, (s, u, v) in zip(sizes, res):
        dd = d[off:off + n]
        ee = e[off:off + max(n - 1, 0)]
        off += n
        if n == 0:
            continue
        s1, u1, v1 = solver.svd(torch.from_numpy(dd.copy()), torch.from_numpy(ee.copy()))
        assert np.array_equal(s, s1.cpu().numpy())
        assert np.array_equal(u, u1.cpu().numpy()) and np.array_equal(v, v1.cpu().numpy())
        ref, _, _ = oracle.bdsdc(dd, ee)
        B = oracle.dense(dd, ee)
        assert np.max(np.abs(s - ref)) <= 1e-13 * max(ref[0], 1e-300)
        assert np.linalg.norm(B - (u * s) @ v) <= 1e-12 * max(np.linalg.norm(B), 1e-300)
        assert np.max(np.abs(u.T @ u - np.eye(n))) <= 1e-12
        assert np.max(np.abs(v @ v.T - np.eye(n))) <= 1e-12


def test_batched_config_2000(solver):
    """2000 problems, sizes log-uniform in [32, 2048]: every problem's
    residual and orthogonality on the GPU, and every singular value of 100
    problems (10 from each of 10 size strata, equal width in log n) against
    the oracle's values written by tests/golden/make_oracle_sigma.py."""
    import torch
    sizes = inputs.batch_sizes(2000, 32, 2048, inputs.seed_for(4, 0)).tolist()
    d, e = inputs.batch_uniform(sizes, inputs.seed_for(4, 1))
    dt = torch.from_numpy(d).cuda()
    et = torch.from_numpy(e).cuda()
    sig, U, VT = solver.svd_batched(sizes, dt, et)
    info, st = solver.info()
    assert info == 0
    gdir = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    sample = np.load(os.path.join(gdir, "batch2000_sample_idx.npy"), allow_pickle=False).tolist()
    ref_all = np.load(os.path.join(gdir, "oracle_sigma_batch2000_sample.npy"), allow_pickle=False)
    assert len(sample) >= 100 and ref_all.shape[0] == sum(sizes[i] for i in sample)
    ref_at = {}
    ro = 0
    for i in sample:
        ref_at[i] = ref_all[ro:ro + sizes[i]]
        ro += sizes[i]
    sig_h = sig.cpu().numpy()
    off = mo = 0
    worst_res = worst_orth = worst_sig = 0.0
    for p, n in enumerate(sizes):
        s = sig[off:off + n]
        u = U[mo:mo + n * n].view(n, n).T
        v = VT[mo:mo + n * n].view(n, n).T.contiguous()
        dd = dt[off:off + n]
        ee = et[off:off + n]
        # B V^T^T = U S, row by row: (B V)[i] = d_i V[i] + e_i V[i+1]
        V = v.T
        BV = dd[:, None] * V
        BV[:-1] += ee[:n - 1, None] * V[1:]
        nb = torch.sqrt(torch.sum(dd * dd) + torch.sum(ee[:n - 1] ** 2))
        res = float(torch.linalg.norm(BV - u * s[None, :]) / nb)
        I = torch.eye(n, dtype=torch.float64, device="cuda")
        uc = u.contiguous()
        orth = max(float(torch.max(torch.abs(uc.T.contiguous() @ uc - I))),
                   float(torch.max(torch.abs(v @ v.T.contiguous() - I))))
        worst_res = max(worst_res, res)
        worst_orth = max(worst_orth, orth)
        if p in ref_at:
            ref = ref_at[p]
            err = float(np.max(np.abs(sig_h[off:off + n] - ref)) / ref[0])
            worst_sig = max(worst_sig, err)
            assert err <= 1e-13, (p, n, err)
        off += n
        mo += n * n
    print(f"batch2000: worst residual {worst_res:.2e}, orthogonality {worst_orth:.2e}, "
          f"sigma vs oracle (100 problems) {worst_sig:.2e}", flush=True)
    assert worst_res <= 1e-12 and worst_orth <= 1e-12


def test_flat_schedule_and_tile_classes_match(gpu):
    """The persistent flattened schedule and other tile-class thresholds give
    the same results as the default launch shapes."""
    import torch
    from paper_2508_11467_amd.api import Solver
    sizes = [40, 900, 33, 260, 1200, 75, 31, 500]
    d, e = inputs.batch_uniform(sizes, 91)
    dt, et = torch.from_numpy(d).cuda(), torch.from_numpy(e).cuda()
    ref = Solver(0)
    alt = Solver(0)
    try:
        r = [x.clone() for x in ref.svd_batched(sizes, dt, et)]
        for tune in ({"small_n": 96, "flat": 1, "grid64": 512, "grid128": 256},
                     {"small_n": 192, "flat": 1, "grid64": 2048, "grid128": 1024},
                     {"small_n": 64, "flat": 0, "grid64": 1024, "grid128": 512},
                     {"small_n": 96, "flat": 0, "grid64": 1024, "grid128": 512, "sec_small_n": 64},
                     {"small_n": 96, "flat": 0, "grid64": 1024, "grid128": 512, "sec_small_n": 256},
                     {"small_n": 96, "flat": 0, "grid64": 1024, "grid128": 512, "sec_small_n": 0},
                     {"small_n": 1 << 20, "flat": 0, "grid64": 1024, "grid128": 512},
                     {"small_n": 1 << 20, "flat": 1, "grid64": 2048, "grid128": 1024}):
            alt.set_tuning(**tune)
            a = alt.svd_batched(sizes, dt, et)
            info, _ = alt.info()
            assert info == 0
            # the flat schedule changes no arithmetic: bitwise equal whenever
            # the tile class and the secular kernels are the reference's
            if tune["small_n"] == 96 and tune.get("sec_small_n", 256) == ref.tuning()["sec_small_n"]:
                for x, y in zip(r, a):
                    assert torch.equal(x, y)
            else:
                assert torch.max(torch.abs(r[0] - a[0])) <= 1e-14 * torch.max(r[0])
        # single-problem solves take the same tunings
        d1, e1 = inputs.normal(3000, 12)
        s0 = ref.svd(d1, e1)[0].clone()
        alt.set_tuning(small_n=96, flat=1, grid64=1024, grid128=512, sec_small_n=ref.tuning()["sec_small_n"])
        s1 = alt.svd(d1, e1)[0]
        assert torch.equal(s0, s1)
    finally:
        ref.close()
        alt.close()


@pytest.mark.parametrize("flat", [0, 1])
def test_second_stream_gives_the_same_results(gpu, flat):
    """Rotations and gathers on a second stream beside the secular solve,
    Löwner z and vectors (streams = 2): bitwise the same sigma, U and V^T as
    one stream, on a batch and on single problems (n a multiple of 4096 takes
    the chunked final pass), over replays of the captured solve."""
    import torch
    from paper_2508_11467_amd.api import Solver
    sizes = [40, 900, 33, 260, 1200, 75, 31, 500, 2048, 64]
    d, e = inputs.batch_uniform(sizes, 92)
    dt, et = torch.from_numpy(d).cuda(), torch.from_numpy(e).cuda()
    one = Solver(0)
    two = Solver(0)
    try:
        tune = {"small_n": 96, "flat": flat, "grid64": 1024, "grid128": 512}
        one.set_tuning(**tune, streams=1)
        two.set_tuning(**tune, streams=2)
        assert two.tuning()["streams"] == 2
        r = [x.clone() for x in one.svd_batched(sizes, dt, et)]
        for _ in range(3):
            a = two.svd_batched(sizes, dt, et)
            torch.cuda.synchronize()
            for x, y in zip(r, a):
                assert torch.equal(x, y)
        assert one.info()[0] == 0 and two.info()[0] == 0
        for n, seed in ((4096, 13), (3000, 14)):
            d1, e1 = inputs.normal(n, seed)
            r1 = [x.clone() for x in one.svd(d1, e1)]
            for _ in range(2):
                a1 = two.svd(d1, e1)
                torch.cuda.synchronize()
                for x, y in zip(r1, a1):
                    assert torch.equal(x, y)
        with pytest.raises(Exception):
            two.set_tuning(**tune, streams=3)
    finally:
        one.close()
        two.close()


def test_autotune_picks_a_valid_tuning(gpu):
    import torch
    from paper_2508_11467_amd.api import Solver
    sizes = inputs.batch_sizes(60, 32, 600, 5).tolist()
    d, e = inputs.batch_uniform(sizes, 6)
    s = Solver(0)
    try:
        best = s.autotune(sizes, d, e, repeats=1)
        assert best["ms"] > 0 and best["flat"] in (0, 1) and best["small_n"] in (64, 96, 192, 1 << 20)
        assert best["leaf_size"] in (8, 12, 16, 20, 24, 32)
        assert best["tile128"] in (0, 1) and best["streams"] in (1, 2)
        assert s.tuning() == {k: best[k] for k in ("small_n", "flat", "grid64", "grid128", "sec_small_n",
                                                    "leaf_size", "tile128", "streams")}
        sig, U, VT = s.svd_batched(sizes, torch.from_numpy(d), torch.from_numpy(e))
        info, _ = s.info()
        assert info == 0
        res = unpack(sizes, sig.cpu().numpy(), U.cpu().numpy(), VT.cpu().numpy())
        off = 0
        for n, (sg, u, v) in zip(sizes, res):
            B = oracle.dense(d[off:off + n], e[off:off + n - 1])
            off += n
            assert np.linalg.norm(B - (u * sg) @ v) <= 1e-12 * np.linalg.norm(B)
            assert np.max(np.abs(u.T @ u - np.eye(n))) <= 1e-12
    finally:
        s.close()


@pytest.mark.parametrize("n", [2048, 4096, 8192])
def test_single_problem_final_pass_matches_batched(solver, n):
    """A single problem whose size is a multiple of 4096 writes its outputs in
    XCD-aligned 4 KB chunks; the same problem inside a batch takes the
    per-column work items (as a single problem of another size does).  The
    final pass only moves data, so both must agree bit for bit."""
    import torch
    d, e = inputs.uniform(n, 300 + n)
    s1, u1, v1 = [x.clone() for x in solver.svd(torch.from_numpy(d), torch.from_numpy(e))]
    sizes = [n, 7]
    d2 = np.concatenate([d, inputs.uniform(7, 5)[0]])
    e2 = np.concatenate([e, [0.0], inputs.uniform(7, 5)[1], [0.0]])
    sig, U, VT = solver.svd_batched(sizes, torch.from_numpy(d2), torch.from_numpy(e2))
    info, _ = solver.info()
    assert info == 0
    res = unpack(sizes, sig.cpu().numpy(), U.cpu().numpy(), VT.cpu().numpy())
    s, u, v = res[0]
    assert np.array_equal(s, s1.cpu().numpy())
    assert np.array_equal(u, u1.cpu().numpy())
    assert np.array_equal(v, v1.cpu().numpy())


def test_batched_outputs_at_8_byte_alignment(solver):
    """Output buffers that are only 8-byte aligned (a caller's views one
    double into an allocation) get the same bits as aligned ones; the sizes
    make 4 KB chunks span several problems and end on odd element counts."""
    import torch
    sizes = [3, 1, 0, 7, 40, 2, 129, 1, 5]
    d, e = inputs.batch_uniform(sizes, 123)
    dt, et = torch.from_numpy(d).cuda(), torch.from_numpy(e).cuda()
    ref = [x.clone() for x in solver.svd_batched(sizes, dt, et)]
    tot, tot2 = sum(sizes), sum(n * n for n in sizes)
    bufs = [torch.full((t + 1,), float("nan"), dtype=torch.float64, device="cuda") for t in (tot, tot2, tot2)]
    out = [b[1:] for b in bufs]
    assert out[1].data_ptr() % 16 == 8
    got = solver.svd_batched(sizes, dt, et, out=out)
    info, _ = solver.info()
    assert info == 0
    for x, y in zip(ref, got):
        assert torch.equal(x, y)
    # the element before each view is untouched
    assert all(torch.isnan(b[0]) for b in bufs)
