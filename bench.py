#!/usr/bin/env python3
"""Benchmark of the five-point Jacobi hot path on one MI355X.

One step = one call of the plain FP64 method on the 4096x4096 grid
(N(0,1), seed 0) with T sweeps (default 100): ring setup, T sweep kernels with
the ping-pong swap, result in `out`. Inputs are resident in HBM before the
timed region. The printed value is the whole-job effective bandwidth,
16 B per interior point per sweep (8 B read + 8 B written, compulsory),
divided by the wall time of the timed steps.

Also reported on the same JSON line:
  roofline      the sweep kernel's algorithmic bytes per launch divided by its
                average launch duration (HIP events on the launch stream),
                against the 8 TB/s HBM peak; `traffic` from rocprofv3 counters
                when a committed measurement of the current kernel source exists
  cpu_baseline  the CPU oracle (C + OpenMP twin) timed on the host's cores on
                a bounded sample of the same workload
  extensions    the other forms of the hot path (when built)

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--sweeps T]
"""

from __future__ import annotations

import argparse
import hashlib
import re
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "hot-path GB/s or FLOP/s and % roofline, plain FP64 vs mixed/batched at stated tol"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sweep_f64_4096_traffic.json")
SWEEP_SRC = os.path.join(ROOT, "paper_2512_19851_amd", "csrc", "sweep.hip")
TB_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sweep_stream_f64_4096_traffic.json")
TB_SRC = [os.path.join(ROOT, "paper_2512_19851_amd", "csrc", "temporal.hip"),
          os.path.join(ROOT, "paper_2512_19851_amd", "csrc", "stream_common.hpp")]
PRESSURE_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pressure_stream_f64_16384_traffic.json")
PRESSURE_SRC = [os.path.join(ROOT, "paper_2512_19851_amd", "csrc", "pressure.hip"),
                os.path.join(ROOT, "paper_2512_19851_amd", "csrc", "stream_common.hpp")]
TB_CAP = 12     # most sweeps per launch of the built-in FP64 schedule
TB_LEVELS = 11  # sweeps per launch of the dominant kernel: 100 sweeps run as one launch of 12 and eight of 11
PREWARM_S = 0.25  # seconds of untimed steps before the timed region


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def source_sha(paths) -> str:
    """Hash of a kernel's code: in each file (one path or a list), the region between the BEGIN/END
    KERNEL SOURCE markers with `//` comments, trailing blanks and blank lines removed, so that only a
    change of code invalidates counters taken on it."""
    if isinstance(paths, str):
        paths = [paths]
    parts = []
    for path in paths:
        with open(os.path.join(ROOT, path) if not os.path.isabs(path) else path, encoding="utf-8") as f:
            text = f.read()
        a = text.find("BEGIN KERNEL SOURCE")
        b = text.find("END KERNEL SOURCE")
        if a >= 0 and b > a:
            text = text[a:b]
        lines = [re.sub(r"//.*$", "", ln).rstrip() for ln in text.splitlines()]
        parts.append("\n".join(ln for ln in lines if ln.strip()))
    return hashlib.sha256("\n".join(parts).encode()).hexdigest()[:16]


def load_traffic(path: str, src: str):
    """HBM bytes per launch from committed rocprofv3 counters, if they match the kernel source."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_sha") != source_sha(src):
        return None
    return rec.get("bytes_per_launch")


def time_kernel_launches(ops, a, b, reps: int) -> float:
    """Average duration (ms) of one sweep launch over `reps` back-to-back launches.

    One HIP event pair on the launch stream brackets the launches, so the
    figure is kernel time plus the (small) dispatch gaps between them.
    """
    import torch

    stream = torch.cuda.current_stream()
    for _ in range(3):
        ops.sweep(a, b)
        a, b = b, a
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        ops.sweep(a, b)
        a, b = b, a
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def cpu_baseline(u0_np, T_step: int, budget_s: float):
    """Time the CPU oracle (C + OpenMP) on a bounded number of sweeps of the same grid."""
    from oracle import cref

    nthreads = int(os.environ.get("OMP_NUM_THREADS", "0")) or min(16, os.cpu_count() or 1)
    used = cref.threads(nthreads)
    H, W = u0_np.shape
    cref.jacobi5(u0_np, 1, nthreads=nthreads)  # first touch, thread start-up
    t0 = time.perf_counter()
    cref.jacobi5(u0_np, 5, nthreads=nthreads)
    t5 = time.perf_counter() - t0
    t0 = time.perf_counter()
    cref.jacobi5(u0_np, 45, nthreads=nthreads)
    t45 = time.perf_counter() - t0
    per = max((t45 - t5) / 40, 1e-5)  # per-sweep cost without the fixed set-up of a call
    # calls of about 2 s each until the budget is spent (the estimate above runs high once the
    # threads are warm, so a single call sized from it would stop well short of the budget)
    chunk = int(max(10, min(20 * T_step, 2.0 / per)))
    sweeps, dt = 0, 0.0
    while dt < budget_s and sweeps < 200 * T_step:
        t0 = time.perf_counter()
        cref.jacobi5(u0_np, chunk, nthreads=nthreads)
        dt += time.perf_counter() - t0
        sweeps += chunk
    gbs = 16.0 * (H - 2) * (W - 2) * sweeps / dt / 1e9
    return {
        "value": round(gbs, 3),
        "unit": "GB/s",
        "cores": used,
        "kind": "oracle",
        "sample": f"{H}x{W} FP64 N(0,1) seed 0, {sweeps} sweeps in {dt:.1f} s, calls of {chunk} sweeps "
                  f"(C + OpenMP oracle, {used} threads); same 16 B/point/sweep accounting",
    }


def bench_mixed(ops, n: int, T: int, args, plain_sec_per_step: float, default_sec_per_step: float) -> dict:
    """The hi/lo form on the mixed-magnitude n x n workload: encode, T sweeps, decode per step.

    Compared with plain FP64 at the same schedule (one pass over HBM per sweep), where the hi/lo form's
    12 B per point beat 16 B, and with the plain calls' default temporally blocked schedule, where the
    work is no longer HBM-bound and FP64's full-rate arithmetic wins."""
    import torch

    from workloads import mixed_f64

    log("[bench] mixed hi/lo form")
    u0 = torch.from_numpy(mixed_f64(0, n)).to("cuda:0")
    out = torch.empty_like(u0)
    work = torch.empty(ops.hilo_work_bytes(n, n), dtype=torch.uint8, device=u0.device)
    for _ in range(max(1, args.warmup)):
        ops.jacobi5_hilo(u0, T, out=out, work=work)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ops.jacobi5_hilo(u0, T, out=out, work=work)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / args.steps
    # per-launch time of the encoded sweep kernel: R back-to-back sweeps on encoded grids
    g = ops.hilo_encode(u0)
    dst = ops.hilo_empty(n, n, n, u0.device)
    wk = ops.hilo_empty(n, n, n, u0.device)
    ops.jacobi5_hilo_encoded(g, 4, dst=dst, work=wk)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    ops.jacobi5_hilo_encoded(g, args.kernel_reps, dst=dst, work=wk)
    e1.record()
    torch.cuda.synchronize()
    per_sweep = e0.elapsed_time(e1) / args.kernel_reps * 1e-3
    interior = (n - 2) * (n - 2)
    return {
        "workload": f"{n}x{n} FP64 z*10**U(-3,3) seed 0, encode + {T} hi/lo sweeps + decode per step",
        "ms_per_step": round(sec * 1e3, 4),
        "fp64_equivalent_GBps": round(16.0 * interior * T / sec / 1e9, 1),
        "speedup_vs_plain_fp64_single_sweep": round(plain_sec_per_step / sec, 3),
        "speedup_vs_plain_fp64_default_schedule": round(default_sec_per_step / sec, 3),
        "sweep_kernel_us": round(per_sweep * 1e6, 2),
        "sweep_kernel_GBps_at_12B": round(12.0 * interior / per_sweep / 1e9, 1),
        "sweep_kernel_hbm_frac": round(12.0 * interior / per_sweep / 1e9 / HBM_PEAK_GBS, 4),
        "tolerance": "componentwise |y - y64| <= 1e-10 (|J||u0|) at T=100; bit-exact with the "
                     "hi/lo model (parity tests)",
    }


def bench_paper_shape(ops, args, n: int = 16384, T: int = 1000) -> dict:
    """The paper's per-GPU Laplace configuration (Section V: 16k x 16k per GPU, 1,000 iterations) from the
    listing's initial state (unit ring, zero interior), under the default and the one-sweep schedules."""
    import torch

    from workloads import unit_ring_grid

    log(f"[bench] paper shape {n}x{n}, T={T}")
    u0 = torch.from_numpy(unit_ring_grid(n, n)).to("cuda:0")
    out = torch.empty_like(u0)
    work = torch.empty_like(u0)
    res = {"workload": f"{n}x{n} FP64, unit ring and zero interior, {T} sweeps (one solve)"}
    interior = (n - 2) ** 2
    for name, sched in (("default_schedule", 0), ("single_sweep_schedule", 1)):
        ops.set_schedule(sched)
        ops.jacobi5(u0, 10, out=out, work=work)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ops.jacobi5(u0, T, out=out, work=work)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        res[name] = {"s_per_solve": round(sec, 4), "ms_per_sweep": round(sec / T * 1e3, 4),
                     "effective_GBps_at_16B": round(16.0 * interior * T / sec / 1e9, 1)}
    ops.set_schedule(0)
    res["center_value"] = float(out[n // 2, n // 2].item())
    del u0, out, work
    torch.cuda.empty_cache()
    return res


def bench_hbm_check(ops, args, n: int = 8192, T: int = 100) -> dict:
    """The plain step at 8192^2 FP64: a ping-pong pair of 2 x 512 MiB does not fit the 256 MB Infinity
    Cache (MALL), so HBM serves every byte; at 4096^2 (2 x 128 MiB) part of the traffic is MALL-served.
    A device copy of the same size gives the practical ceiling at this size."""
    import torch

    from workloads import large_f64

    log(f"[bench] HBM check {n}x{n}")
    u0 = torch.from_numpy(large_f64(0, n)).to("cuda:0")
    out = torch.empty_like(u0)
    work = torch.empty_like(u0)
    interior = (n - 2) ** 2
    res = {"workload": f"{n}x{n} FP64 N(0,1) seed 0, {T} sweeps per step"}

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps * 1e-3

    sec = timed(lambda: out.copy_(u0), 10)
    res["device_copy_GBps"] = round(2 * 8 * n * n / sec / 1e9, 1)
    for name, sched in (("default_schedule", 0), ("single_sweep_schedule", 1)):
        ops.set_schedule(sched)
        sec = timed(lambda: ops.jacobi5(u0, T, out=out, work=work), 3)
        res[name] = {"ms_per_step": round(sec * 1e3, 3), "us_per_sweep": round(sec / T * 1e6, 2),
                     "effective_GBps_at_16B": round(16.0 * interior * T / sec / 1e9, 1)}
    ops.set_schedule(0)
    del u0, out, work
    torch.cuda.empty_cache()
    return res


def bench_batch(ops, T: int, args) -> dict:
    """1024 FP32 grids (point counts log-uniform in [2^8, 2^16], seed 0), T sweeps each,
    in one persistent launch replayed from a HIP graph; launch configuration autotuned."""
    import tempfile

    import torch

    from workloads import batch_f32

    log("[bench] batched form")
    u0s = [torch.from_numpy(u).to("cuda:0") for u in batch_f32(0)]
    interior = sum((u.shape[0] - 2) * (u.shape[1] - 2) for u in u0s)
    points = sum(u.numel() for u in u0s)
    with tempfile.TemporaryDirectory() as td:
        cache = os.path.join(td, "batch_tune.txt")
        plan = ops.BatchPlan(u0s, T)
        tuned_us = plan.autotune(cache, reps=3)
        plan = ops.BatchPlan(u0s, T, outs=plan.outs, works=plan.works, tune_cache=cache)
    info = plan.info()
    plan.run()
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        plan.run()
    for _ in range(max(1, args.warmup)):
        g.replay()
    torch.cuda.synchronize()
    reps = max(5, args.steps)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(reps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / reps
    ev_sec = e0.elapsed_time(e1) * 1e-3 / reps
    # the plain path on the same grids: one call (T sweep launches) per grid
    outs = [torch.empty_like(u) for u in u0s]
    works = [torch.empty_like(u) for u in u0s]
    for u, o, w in zip(u0s, outs, works):
        ops.jacobi5(u, T, out=o, work=w)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for u, o, w in zip(u0s, outs, works):
        ops.jacobi5(u, T, out=o, work=w)
    torch.cuda.synchronize()
    plain_sec = time.perf_counter() - t0
    same = all(torch.equal(a, b) for a, b in zip(outs, plan.outs))
    pts = interior * T
    lds_cap = (info["lds_bytes"] - 64) // 4
    lds_pts = sum((u.shape[0] - 2) * (u.shape[1] - 2) for u in u0s
                  if u.shape[0] >= 3 and u.shape[1] >= 3 and 2 * u.numel() <= lds_cap)
    return {
        "workload": f"1024 FP32 grids N(0,1) seed 0, sizes log-uniform in [2^8, 2^16] points "
                    f"({points} points, {interior} interior), {T} sweeps each, one persistent launch "
                    f"replayed from a HIP graph",
        "ms_per_batch": round(sec * 1e3, 4),
        "ms_per_batch_events": round(ev_sec * 1e3, 4),
        "batches_per_s": round(1.0 / sec, 2),
        "grids_per_s": round(len(u0s) / sec, 1),
        "point_sweeps_per_s": round(pts / sec, 1),
        "effective_GBps_at_8B": round(8.0 * pts / sec / 1e9, 1),
        "hbm_frac_at_8B": round(8.0 * pts / sec / 1e9 / HBM_PEAK_GBS, 4),
        "config": info,
        "autotuned_us": round(tuned_us, 1),
        "plain_per_grid_ms": round(plain_sec * 1e3, 2),
        "speedup_vs_plain_launches": round(plain_sec / sec, 1),
        "bit_identical_to_plain": bool(same),
        "interior_points_in_lds_frac": round(lds_pts / interior, 4),
    }


def bench_tiled(ops, n: int, T: int, args, plain_sec_per_step: float, blocked_sec_per_step: float) -> dict:
    """The plain FP64 step on the same grid split into tiles with ghost exchange (one GPU): depth-1 ghosts
    (one exchange and one kernel per tile per sweep) and deep ghosts (one exchange and one blocked launch
    over all tiles per chunk of up to g sweeps)."""
    import torch

    from workloads import large_f64

    log("[bench] tiled execution")
    u0 = torch.from_numpy(large_f64(0, n)).to("cuda:0")
    want = ops.jacobi5(u0, T)
    comm = torch.cuda.Stream()
    res = {}
    cases = ((2, 2, 1, "packed", True), (4, 4, 1, "packed", True), (2, 2, 12, "packed", True),
             (2, 2, 12, "packed", False), (2, 2, 12, "direct", False), (4, 4, 12, "direct", False),
             (8, 8, 12, "direct", False))
    for pr, pc, g, mode, two_streams in cases:
        t = ops.TiledGrid(n, n, pr, pc, comm_stream=comm if two_streams else None, ghost=g, exchange=mode)
        t.scatter(u0)
        t.run(T)
        same = bool(torch.equal(t.gather(), want))
        t.run(2)
        torch.cuda.synchronize()
        before = t.stats()
        reps = max(3, args.steps // 4)
        t0 = time.perf_counter()
        for _ in range(reps):
            t.run(T)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / reps
        st = t.stats()
        res[f"{pr}x{pc}_ghost{g}_{mode}_{'2' if two_streams else '1'}stream"] = {
            "ms_per_step": round(sec * 1e3, 4),
            "effective_GBps": round(16.0 * (n - 2) ** 2 * T / sec / 1e9, 1),
            "vs_single_grid_single_sweep": round(sec / plain_sec_per_step, 3),
            "vs_single_grid_default_schedule": round(sec / blocked_sec_per_step, 3),
            "exchanges_per_step": (st["exchanges"] - before["exchanges"]) // reps,
            "sweep_launches_per_step": (st["sweep_launches"] - before["sweep_launches"]) // reps,
            "bit_identical_to_single_grid": same,
        }
    res["workload"] = (f"{n}x{n} FP64 N(0,1) seed 0, {T} sweeps per step; pr x pc tiles with ghost frames of "
                       "depth g; exchange packed (pack + unpack kernels through send buffers) or direct (one "
                       "copy kernel), on a second stream (2stream) or the compute stream (1stream); g = 1: one "
                       "exchange and one sweep kernel per tile per sweep; g > 1: one exchange and one blocked "
                       "launch over all tiles (per 32 tiles) per chunk of up to g sweeps, the sweeps split "
                       "evenly over the chunks")
    return res


def bench_temporal(ops, n: int, T: int, args, plain_sec_per_step: float) -> dict:
    """The plain step with temporal blocking: `levels` sweeps per HBM pass, same bits, for both
    blocked kernels (register tile, streaming) and both precisions."""
    import torch

    from workloads import large_f64

    log("[bench] temporal blocking")
    u64 = torch.from_numpy(large_f64(0, n)).to("cuda:0")
    res = {"workload": f"{n}x{n} N(0,1) seed 0, {T} sweeps per step, bit-identical to the plain step"}
    cases = [("block", 1, torch.float64, (2, 4, 6)), ("stream", 2, torch.float64, (2, 4, 6, 8, 10, 12)),
             ("stream", 2, torch.float32, (4, 8, 10, 12))]
    for name, variant, dt, levels_list in cases:
        u0 = u64.to(dt)
        out = torch.empty_like(u0)
        work = torch.empty_like(u0)
        bpp = 2 * u0.element_size()
        ops.set_tb(variant, 0, 0)
        for levels in levels_list:
            ops.jacobi5_tb(u0, T, levels=levels, out=out, work=work)
            torch.cuda.synchronize()
            reps = max(3, args.steps // 2)
            t0 = time.perf_counter()
            for _ in range(reps):
                ops.jacobi5_tb(u0, T, levels=levels, out=out, work=work)
            torch.cuda.synchronize()
            sec = (time.perf_counter() - t0) / reps
            launches = -(-T // levels)
            key = f"{name}_{'f64' if dt == torch.float64 else 'f32'}_levels_{levels}"
            res[key] = {
                "ms_per_step": round(sec * 1e3, 4),
                "us_per_sweep": round(sec / T * 1e6, 3),
                f"effective_GBps_at_{bpp}B": round(bpp * (n - 2) ** 2 * T / sec / 1e9, 1),
                "us_per_launch": round(sec / launches * 1e6, 2),
            }
            if dt == torch.float64:
                res[key]["speedup_vs_single_sweep"] = round(plain_sec_per_step / sec, 3)
    ops.set_tb(0, 0, 0)
    return res


def bench_frontend(ops, args) -> dict:
    """One-GPU analog of the pipelining experiment (Section V): the listing program through the
    lazy frontend, runtime against the maximum DAG depth, next to one direct call (no Python per node)."""
    import torch

    from paper_2512_19851_amd import frontend

    log("[bench] frontend pipelining")
    n, T = 4096, 200
    u = torch.zeros((n, n), dtype=torch.float64, device="cuda:0")
    u[0, :] = u[-1, :] = u[:, 0] = u[:, -1] = 1
    ideal = []
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ops.jacobi5(u, T)
        torch.cuda.synchronize()
        ideal.append(time.perf_counter() - t0)
    res = {"workload": f"listing program, {n}x{n} FP64 unit ring, {T} iterations; per DAG depth the best "
                       f"of 3 runs (the first loads the kernels a chain plan needs)",
           "ideal_ms": round(min(ideal) * 1e3, 2)}
    for depth in (1, 10, 100, 1000):
        best = None
        for _ in range(3):
            ctx = frontend.Context(max_depth=depth)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            u1 = ctx.create_array((n, n))
            u2 = ctx.create_array((n, n))
            u1[0, :] = u1[-1, :] = u1[:, 0] = u1[:, -1] = 1
            u2[0, :] = u2[-1, :] = u2[:, 0] = u2[:, -1] = 1
            for _ in range(T):
                u2[1:-1, 1:-1] = 0.25 * (u1[:-2, 1:-1] + u1[2:, 1:-1] + u1[1:-1, :-2] + u1[1:-1, 2:])
                u1, u2 = u2, u1
            ctx.sync()
            sec = time.perf_counter() - t0
            best = sec if best is None else min(best, sec)
        res[f"depth_{depth}_ms"] = round(best * 1e3, 2)
        res[f"depth_{depth}_chained_nodes"] = ctx.stats["chained_nodes"]
        del ctx, u1, u2
    return res


def bench_cavity(args, n: int = 16384, nit: int = 50, steps: int = 2) -> dict:
    """The paper's second application (Section V): lid-driven cavity flow, 16k x 16k per GPU, written
    as slice assignments on the frontend; most nodes run as generated kernels, the u and v updates fused.
    Two pressure solves: the blocked library call (default) and one frontend node per iteration."""
    import torch

    from paper_2512_19851_amd import frontend
    from paper_2512_19851_amd.cavity import CavityFlow

    interior = (n - 2) ** 2
    # algorithmic bytes per step: source (read u, v; write b), nit pressure iterations (read p, b;
    # write p), velocities (read u, v, p; write u, v); walls are O(n)
    step_bytes = interior * (24 + 24 * nit + 40)
    res = {
        "workload": f"{n}x{n} FP64, rest start, lid u = 1, nu = 0.1, dt = 0.001, {nit} pressure iterations per "
                    f"step, {steps} timed steps after one warm-up step",
        "algorithmic_bytes_per_step": step_bytes,
        "parity": "bit-identical to the NumPy oracle on 3x130 ... 257x513, both pressure solves "
                  "(tests/test_gpu_cavity.py, tests/test_gpu_pressure.py)",
    }
    fields = {}
    for blocked in (True, False):
        log(f"[bench] cavity flow {n}x{n}, {nit} pressure iterations per step, blocked pressure {blocked}")
        ctx = frontend.Context(max_depth=64)
        flow = CavityFlow(ctx, n, n, nit=nit, blocked_pressure=blocked)
        t0 = time.perf_counter()
        flow.run(1)  # warm-up: compiles the generated kernels (hiprtc) once per process
        ctx.sync()
        warm = time.perf_counter() - t0
        t0 = time.perf_counter()
        flow.run(steps)
        ctx.sync()
        sec = (time.perf_counter() - t0) / steps
        u, v, p = flow.fields()
        fields[blocked] = (u.clone(), v.clone(), p.clone())
        finite = bool(torch.isfinite(u).all() and torch.isfinite(v).all() and torch.isfinite(p).all())
        res["blocked_pressure" if blocked else "per_node_pressure"] = {
            "ms_per_step": round(sec * 1e3, 2),
            "effective_GBps": round(step_bytes / sec / 1e9, 1),
            "warmup_step_s_incl_compile": round(warm, 2),
            "fields_finite": finite,
        }
        del flow, ctx, u, v, p
    res["blocked_bit_identical_to_per_node"] = all(torch.equal(a, b) for a, b in zip(fields[True], fields[False]))
    passes = bench_pressure_passes(n, 5)
    traffic = load_traffic(PRESSURE_TRAFFIC_FILE, PRESSURE_SRC) if n == 16384 else None
    passes["traffic"] = traffic
    passes["hbm_use_frac"] = (round(traffic / (passes["avg_us_per_call"] * 1e-6) / (HBM_PEAK_GBS * 1e9), 4)
                              if traffic else None)
    res["pressure_pass"] = passes
    res["speedup_blocked_vs_per_node"] = round(res["per_node_pressure"]["ms_per_step"] /
                                               res["blocked_pressure"]["ms_per_step"], 2)
    del fields
    torch.cuda.empty_cache()
    return res


def bench_pressure_passes(n: int, reps: int, levels: int = 8) -> dict:
    """`reps` launches of the blocked pressure kernel, each one pass of `levels` cavity pressure iterations
    on an n x n FP64 grid (N(0,1) p and b, seed 0), timed with HIP events on the launch stream."""
    import torch

    from oracle.cavity import CavityParams
    from paper_2512_19851_amd import ops
    from workloads import normal_grid

    prm = CavityParams(n, n)
    p0 = torch.from_numpy(normal_grid(n, n, seed=0)).to("cuda:0")
    b = torch.from_numpy(normal_grid(n, n, seed=1)).to("cuda:0")
    out = torch.empty_like(p0)
    for _ in range(3):
        ops.cavity_pressure(p0, b, levels, prm.cw, prm.cn, prm.cb, levels=levels, out=out)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        ops.cavity_pressure(p0, b, levels, prm.cw, prm.cn, prm.cb, levels=levels, out=out)
    e1.record(stream)
    torch.cuda.synchronize()
    per_ms = e0.elapsed_time(e1) / reps
    interior = (n - 2) ** 2
    return {"mode": "pressure", "grid": [n, n], "levels": levels, "launches": reps,
            "avg_us_per_call": round(per_ms * 1e3, 2),
            "note": "a call is the lid fill kernel plus one blocked launch",
            "algorithmic_bytes_per_launch": 24.0 * interior * levels,
            "pass_floor_bytes": 24.0 * interior,
            "pass_floor_frac": round(24.0 * interior / (per_ms * 1e-3) / (HBM_PEAK_GBS * 1e9), 4)}


def bench_adjoint(T: int, args) -> dict:
    """Gradient workload: 1024x1024 FP32, L = sum(w * u_T), dL/du0 and dL/dc through autograd."""
    import torch

    from paper_2512_19851_amd import autograd
    from workloads import adjoint_f32

    log("[bench] adjoint")
    u0_np, w_np, _ = adjoint_f32(0)
    u0 = torch.from_numpy(u0_np).to("cuda:0")
    w = torch.from_numpy(w_np.astype("float32")).to("cuda:0")
    c = torch.tensor(0.25, dtype=torch.float32, device="cuda:0", requires_grad=True)
    H, W = u0.shape

    def step():
        x = u0.detach().requires_grad_(True)
        y = autograd.jacobi5_autograd(x, T, c)
        L = (y * w).sum()
        return torch.autograd.grad(L, (x, c))

    for _ in range(max(1, args.warmup)):
        step()
    torch.cuda.synchronize()
    reps = max(5, args.steps)
    t0 = time.perf_counter()
    for _ in range(reps):
        step()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / reps
    # transposed-sweep kernel alone: R steps without states
    g = torch.randn_like(u0)
    R = args.kernel_reps
    autograd.adjoint(g, 2, 0.25)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    autograd.adjoint(g, R, 0.25)
    e1.record()
    torch.cuda.synchronize()
    per = e0.elapsed_time(e1) * 1e-3 / R
    return {
        "workload": f"{H}x{W} FP32 u0 N(0,1), w N(0,1) seed 0, T={T}: forward with recorded states + "
                    f"reverse pass (dL/du0 and dL/dc) per step",
        "ms_per_step": round(sec * 1e3, 4),
        "adjoint_sweep_us": round(per * 1e6, 2),
        "adjoint_sweep_GBps_at_8B": round(8.0 * H * W / per / 1e9, 1),
        "tolerance": "dL/du0 within the FP32 bound of the FP64 oracle gradient and of central FD "
                     "(h=1e-6) at 64 coordinates; dL/dc within its bound (parity tests)",
    }


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--sweeps", type=int, default=100, help="sweeps T per step")
    ap.add_argument("--n", type=int, default=4096, help="grid side")
    ap.add_argument("--kernel-reps", type=int, default=100)
    ap.add_argument("--cpu-budget", type=float, default=16.0, help="seconds of CPU oracle work")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extensions", action="store_true")
    ap.add_argument("--mode", choices=["step", "sweep", "copy", "hilo", "tb", "cavity", "pressure", "batch"],
                    default="step",
                    help="step: the benchmark; sweep: only --kernel-reps sweep launches; "
                         "copy: only --kernel-reps plain grid copies (counter calibration); "
                         "hilo: only --kernel-reps hi/lo sweeps on encoded grids; "
                         "tb: only --kernel-reps temporally blocked launches; "
                         "cavity: only the cavity-flow extension (--n grid side); "
                         "pressure: only --kernel-reps blocked passes of 8 cavity pressure iterations (--n); "
                         "batch: only the batched extension (--sweeps, --steps graph replays)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path; "
              "run with --gpus 1", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_2512_19851_amd import ops
    from workloads import large_f64

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.mode == "cavity":
        print(json.dumps({"mode": "cavity", **bench_cavity(args, n=args.n)}), flush=True)
        return 0
    if args.mode == "pressure":
        print(json.dumps(bench_pressure_passes(args.n, args.kernel_reps)), flush=True)
        return 0
    if args.mode == "batch":
        from paper_2512_19851_amd import ops

        print(json.dumps({"mode": "batch", **bench_batch(ops, args.sweeps, args)}), flush=True)
        return 0
    n, T = args.n, args.sweeps
    log(f"[bench] generating {n}x{n} FP64 N(0,1) seed 0")
    u0_np = large_f64(0, n)
    u0 = torch.from_numpy(u0_np).to(dev)
    out = torch.empty_like(u0)
    work = torch.empty_like(u0)
    interior = (n - 2) * (n - 2)
    launch_bytes = 16.0 * interior
    step_bytes = launch_bytes * T

    if args.mode == "hilo":
        from workloads import mixed_f64

        m = torch.from_numpy(mixed_f64(0, n)).to(dev)
        g = ops.hilo_encode(m)
        d1 = ops.hilo_empty(n, n, n, dev)
        d2 = ops.hilo_empty(n, n, n, dev)
        ops.jacobi5_hilo_encoded(g, 2, dst=d1, work=d2)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        ops.jacobi5_hilo_encoded(g, args.kernel_reps, dst=d1, work=d2)
        e1.record()
        torch.cuda.synchronize()
        per = e0.elapsed_time(e1) / args.kernel_reps
        print(json.dumps({"mode": "hilo", "launches": args.kernel_reps, "avg_us": round(per * 1e3, 2),
                          "algorithmic_bytes_per_launch": 12.0 * interior,
                          "GBps": round(12.0 * interior / (per * 1e-3) / 1e9, 1)}), flush=True)
        return 0

    if args.mode != "step":
        # short runs for rocprofv3 counter passes: no CPU work, no extensions
        a = u0.clone()
        b = u0.clone()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.kernel_reps):
            if args.mode == "sweep":
                ops.sweep(a, b)
            elif args.mode == "tb":
                ops.jacobi5_tb(a, TB_LEVELS, levels=TB_LEVELS, out=b)  # one blocked launch
            else:
                ops.jacobi5(a, 0, out=b)  # T = 0: one plain copy of the grid
            a, b = b, a
        e1.record()
        torch.cuda.synchronize()
        per = e0.elapsed_time(e1) / args.kernel_reps
        moved = {"sweep": launch_bytes, "tb": TB_LEVELS * launch_bytes}.get(args.mode, 16.0 * n * n)
        print(json.dumps({"mode": args.mode, "launches": args.kernel_reps, "avg_us": round(per * 1e3, 2),
                          "algorithmic_bytes_per_launch": moved,
                          "GBps": round(moved / (per * 1e-3) / 1e9, 1)}), flush=True)
        return 0

    log(f"[bench] warmup {args.warmup} steps of T={T}, then the same step until {PREWARM_S} s have passed")
    for _ in range(args.warmup):
        ops.jacobi5(u0, T, out=out, work=work)
    torch.cuda.synchronize()
    # Clocks ramp up over the first tens of milliseconds of sustained work (a cold start ran the first
    # steps about 15% slower); run the untimed step until the GPU has been busy for PREWARM_S seconds.
    t_warm = time.perf_counter()
    while time.perf_counter() - t_warm < PREWARM_S:
        ops.jacobi5(u0, T, out=out, work=work)
        torch.cuda.synchronize()

    log(f"[bench] timing {args.steps} steps")
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        ops.jacobi5(u0, T, out=out, work=work)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = ev0.elapsed_time(ev1)
    sec_per_step = wall / args.steps
    value = step_bytes / sec_per_step / 1e9
    log(f"[bench] {sec_per_step * 1e3:.3f} ms/step, {value:.1f} GB/s (events: {ev_ms / args.steps:.3f} ms/step)")

    log("[bench] the same step with one sweep per launch (the paper's schedule)")
    ops.set_schedule(1)
    ops.jacobi5(u0, T, out=out, work=work)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ops.jacobi5(u0, T, out=out, work=work)
    torch.cuda.synchronize()
    single_sec_per_step = (time.perf_counter() - t0) / args.steps
    ops.set_schedule(0)

    log(f"[bench] per-launch kernel timing, {args.kernel_reps} launches")
    a = out.clone()
    b = work
    b.copy_(a)
    # The step's launches, timed live: the HIP events that bracket the timed steps on the launch stream,
    # divided by the blocked launches per step (the step's kernels are these launches plus a ring copy of
    # a few microseconds). T sweeps run as ceil(T / TB_CAP) launches, the sweeps split evenly.
    launches = -(-T // TB_CAP)
    base, extra = divmod(T, launches)
    mix = ([f"sweep_stream_kernel<double,2,{base + 1},4> x{extra}"] if extra else []) + \
        [f"sweep_stream_kernel<double,2,{base},4> x{launches - extra}"]
    step_launch_ms = ev_ms / args.steps / launches
    step_launch_bytes = T * launch_bytes / launches
    tb_achieved = step_launch_bytes / (step_launch_ms * 1e-3) / 1e9
    traffic = load_traffic(TB_TRAFFIC_FILE, TB_SRC)
    roofline = {
        "bound": "hbm",
        "achieved": round(tb_achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(tb_achieved / HBM_PEAK_GBS, 4),
        "traffic": traffic,
        "kernel": f"the step's blocked launches: {' + '.join(mix)} ({T} sweeps of the {n}x{n} FP64 grid in "
                  f"{launches} launches)",
        "algorithmic_bytes_per_launch": step_launch_bytes,
        "avg_launch_us": round(step_launch_ms * 1e3, 2),
        "step_us_per_sweep": round(sec_per_step / T * 1e6, 2),
        "hbm_floor_us_per_launch": round(launch_bytes / (HBM_PEAK_GBS * 1e9) * 1e6, 2),
        "launch_floor_frac": round(launch_bytes / (HBM_PEAK_GBS * 1e9) / (step_launch_ms * 1e-3), 4),
        "hbm_use_frac": round(traffic / (step_launch_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if traffic else None,
        "note": "algorithmic bytes count 16 B per interior point per sweep, as for one sweep per launch; a "
                f"launch applies {base} or {base + 1} sweeps while reading and writing the grid about once, so "
                "achieved exceeds the HBM peak. avg_launch_us: HIP events over the timed steps divided by the "
                "launches per step. traffic is the measured HBM bytes of one launch of the dominant kernel "
                f"(sweep_stream_kernel<double,2,{TB_LEVELS},4>, about one grid read plus one write); hbm_use_frac "
                "= traffic / launch time / peak; launch_floor_frac = (one grid read plus write at peak) / "
                "launch time (the arithmetic floor, 4 FP64 ops per point per sweep at the 39.3 Tops/s "
                "add/multiply rate, is lower)",
    }
    # The ALU view of the same launches: 4 FP64 adds/multiplies per interior point per sweep against the
    # chip's FP64 add/multiply issue rate (256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3 Tops/s; FMA counts
    # twice in the 78.6 TFLOP/s figure). A launch also issues 2 DPP lane shifts per point per level and
    # recomputes the halo rows and columns its bands and strips share (measured tile: 1.25 x the rows,
    # 128/104 x the columns), so the VALU issues about 4 x 1.5 x 1.54 = 9.2 lane-operations per useful point
    # and level.
    alu_peak = 256 * 4 * 16 * 2.4e9 / 1e12
    alu_achieved = 4.0 * interior * T / (step_launch_ms * 1e-3 * launches) / 1e12
    roofline["alu_view"] = {
        "bound": "alu",
        "achieved": round(alu_achieved, 2),
        "peak": round(alu_peak, 2),
        "unit": "Tops/s",
        "frac": round(alu_achieved / alu_peak, 4),
        "valu_issue_frac_estimate": round(alu_achieved * 9.24 / 4.0 / alu_peak, 3),
        "note": "4 FP64 operations per interior point per sweep (3 adds, 1 multiply) over the step's launch "
                "time; valu_issue_frac_estimate adds the DPP lane shifts and the halo recomputation "
                "(9.2 VALU lane-operations per useful point and level)",
    }
    # the dominant kernel alone (every launch TB_LEVELS sweeps), as the traffic counters see it
    w2 = torch.empty_like(u0)
    ops.set_schedule(TB_LEVELS)
    ops.jacobi5(a, TB_LEVELS * 2, out=b, work=w2)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    ops.jacobi5(a, TB_LEVELS * args.kernel_reps, out=b, work=w2)  # kernel_reps blocked launches + ring copy
    e1.record(stream)
    torch.cuda.synchronize()
    ops.set_schedule(0)
    alone_ms = e0.elapsed_time(e1) / args.kernel_reps
    roofline["dominant_kernel_alone"] = {
        "kernel": f"sweep_stream_kernel<double,2,{TB_LEVELS},4>",
        "launches": args.kernel_reps,
        "avg_launch_us": round(alone_ms * 1e3, 2),
        "algorithmic_bytes_per_launch": TB_LEVELS * launch_bytes,
        "achieved": round(TB_LEVELS * launch_bytes / (alone_ms * 1e-3) / 1e9, 1),
    }
    # the single-sweep kernel (one sweep per launch, the paper's schedule) for reference
    avg_ms = time_kernel_launches(ops, a, b, args.kernel_reps)
    achieved = launch_bytes / (avg_ms * 1e-3) / 1e9
    single = {
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": load_traffic(TRAFFIC_FILE, SWEEP_SRC),
        "kernel": "sweep_kernel<double,2,4> (one sweep of the 4096x4096 FP64 grid)",
        "algorithmic_bytes_per_launch": launch_bytes,
        "avg_launch_us": round(avg_ms * 1e3, 2),
        "ms_per_step_single_sweep_schedule": round(single_sec_per_step * 1e3, 4),
        "GBps_single_sweep_schedule": round(step_bytes / single_sec_per_step / 1e9, 1),
    }

    rec = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(sec_per_step * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"plain FP64 five-point Jacobi, {n}x{n} grid N(0,1) seed 0, {T} sweeps per step",
            "grid": [n, n],
            "sweeps_per_step": T,
            "schedule": f"temporal blocking, up to {TB_CAP} sweeps per launch, the {T} sweeps split evenly over "
                        f"{-(-T // TB_CAP)} launches (bit-identical to one sweep per launch)",
            "bytes_per_point_per_sweep": 16,
            "parallelism": "single GPU",
        },
        "roofline": roofline,
        "single_sweep_roofline": single,
    }

    if not args.no_extensions:
        rec["extensions"] = {
            "mixed_hilo": bench_mixed(ops, n, T, args, single_sec_per_step, sec_per_step),
            "paper_shape": bench_paper_shape(ops, args),
            "hbm_check": bench_hbm_check(ops, args),
            "batched": bench_batch(ops, T, args),
            "tiled": bench_tiled(ops, n, T, args, single_sec_per_step, sec_per_step),
            "temporal_blocking": bench_temporal(ops, n, T, args, single_sec_per_step),
            "frontend": bench_frontend(ops, args),
            "adjoint": bench_adjoint(10, args),
            "cavity_flow": bench_cavity(args),
        }

    if not args.no_cpu:
        log("[bench] CPU oracle baseline")
        rec["cpu_baseline"] = cpu_baseline(u0_np, T, args.cpu_budget)
    else:
        rec["cpu_baseline"] = None

    print(json.dumps(rec), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
