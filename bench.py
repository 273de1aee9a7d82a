#!/usr/bin/env python3
"""Benchmark of the five-point Jacobi hot path on one MI355X.

One step = one call of the plain FP64 method on the 4096x4096 grid
(N(0,1), seed 0) with T sweeps (default 100): ring setup, T sweeps with the
ping-pong swap (temporally blocked: several sweeps per launch), result in
`out`. Inputs are resident in HBM before the timed region. The printed value
is the whole-job arithmetic rate, 4 FP64 operations per interior point per
sweep (3 adds and 1 multiply, the method's own count), divided by the wall
time of the timed steps; the effective bandwidth at 16 B per point per sweep
is reported beside it.

Also reported on the same JSON line:
  roofline      the step's blocked launches against the bound that binds
                them, the FP64 vector ALU (78.6 TFLOP/s): 4 flop per interior
                point per sweep over the average launch duration (HIP events
                on the launch stream over the timed steps), with the HBM view
                (measured traffic from rocprofv3 counters, when a committed
                measurement of the current kernel source exists) beside it
  single_sweep_roofline  one sweep per launch (the paper's schedule), which is
                HBM-bound, against 8 TB/s and a measured 16-byte-vector copy
  cpu_baseline  the CPU oracle (C + OpenMP twin) timed on all host cores on a
                bounded sample of the same workload
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
FP64_PEAK_TFLOPS = 78.6    # MI355X FP64 vector, an FMA counted as two operations
FP32_PEAK_TFLOPS = 157.3   # MI355X FP32 vector (packed FMA counted as four operations)
# Add or multiply issue rate of the vector ALUs without fused or packed operations (the method's
# adds and multiplies are separate roundings, and packed FP32 is not generated): 256 CUs x 4 SIMDs x
# 16 lanes x 2.4 GHz, the same for FP64 and FP32 on this chip.
ADD_MUL_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
FLOP_PER_POINT = 4.0       # 3 adds + 1 multiply per interior point per sweep
METRIC = "hot-path GB/s or FLOP/s and % roofline, plain FP64 vs mixed/batched at stated tol"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sweep_f64_4096_traffic.json")
SWEEP_SRC = os.path.join(ROOT, "paper_2512_19851_amd", "csrc", "sweep.hip")
TB_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sweep_stream_f64_4096_traffic.json")
TB_SRC = [os.path.join(ROOT, "paper_2512_19851_amd", "csrc", "temporal.hip"),
          os.path.join(ROOT, "paper_2512_19851_amd", "csrc", "stream_common.hpp")]
PRESSURE_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pressure_stream_f64_16384_traffic.json")
PRESSURE_SRC = [os.path.join(ROOT, "paper_2512_19851_amd", "csrc", "pressure.hip"),
                os.path.join(ROOT, "paper_2512_19851_amd", "csrc", "stream_common.hpp")]
TB_CAP = 12     # most sweeps per launch of the built-in FP64 schedule while one grid is at most 128 MiB
TB_CAP_DEEP = 14  # ... and above that (the pair of buffers no longer fits the 256 MiB Infinity Cache)
TB_LEVELS = 11  # sweeps per launch of the dominant kernel: 100 sweeps run as one launch of 12 and eight of 11
PREWARM_S = 0.25  # seconds of untimed steps before the timed region
PRESSURE_MAX_LEVELS = 12  # most cavity pressure iterations per blocked pass (the library's default)
CAVITY_NIT = 50           # pressure iterations per cavity time step


def tb_cap(n: int) -> int:
    """Most sweeps per launch of the library's built-in FP64 schedule for an n x n grid."""
    return TB_CAP if n * n * 8 <= (128 << 20) else TB_CAP_DEEP


def pressure_pass_levels(nit: int) -> int:
    """Iterations in the longest pass when the library splits nit pressure iterations at its default:
    ceil(nit / 12) passes, as even as they go (50 -> 5 passes of 10)."""
    passes = -(-nit // PRESSURE_MAX_LEVELS)
    return -(-nit // passes)


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


def load_traffic(path: str, src: str, **expect):
    """HBM bytes per launch from committed rocprofv3 counters, if they match the kernel source (and each
    `expect` key, e.g. the levels per launch the counters were taken at)."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_sha") != source_sha(src) or any(rec.get(k) != v for k, v in expect.items()):
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


def host_cores() -> int:
    """The host's core count as `nproc` reports it: the CPUs this process may run on."""
    try:
        return len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        return os.cpu_count() or 1


def time_copy(ops, a, b, reps: int) -> float:
    """Average duration (ms) of the library's contiguous 16-byte vector copy of grid a into b (the plain
    call with T = 0), over `reps` back-to-back calls bracketed by one HIP event pair."""
    import torch

    stream = torch.cuda.current_stream()
    for _ in range(3):
        ops.jacobi5(a, 0, out=b)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        ops.jacobi5(a, 0, out=b)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def cpu_baseline(u0_np, T_step: int, budget_s: float):
    """Time the CPU oracle (C + OpenMP) on a bounded number of sweeps of the same grid, one thread per
    host core."""
    from oracle import cref

    nthreads = host_cores()
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
    pts = (H - 2) * (W - 2) * sweeps
    return {
        "value": round(FLOP_PER_POINT * pts / dt / 1e9, 3),
        "unit": "GFLOP/s",
        "cores": used,
        "kind": "oracle",
        "sample": f"{H}x{W} FP64 N(0,1) seed 0, {sweeps} sweeps in {dt:.1f} s, calls of {chunk} sweeps "
                  f"(C + OpenMP oracle, {used} threads, one per core nproc reports; os.cpu_count() = "
                  f"{os.cpu_count()}); same 4 flop/point/sweep accounting",
        "effective_GBps_at_16B": round(16.0 * pts / dt / 1e9, 3),
    }


def hilo_errors(ops, u0, y, T: int) -> dict:
    """Measured error of a hi/lo result y against the plain FP64 method on the GPU (bit-identical to the
    FP64 oracle, as the parity tests check): componentwise |y - y64| / (|J| |u0|), normwise
    max|y - y64| / max|y64|, and plain relative |y - y64| / |y64| over outputs with |y64| >= 1e-3 max|y64|.
    |J| |u0| is the plain method run on |u0| (the sweep's weights are non-negative)."""
    import torch

    y64 = ops.jacobi5(u0, T)
    ja = ops.jacobi5(u0.abs(), T)
    d = (y - y64).abs()
    comp = torch.where(ja > 0, d / ja, torch.where(d > 0, torch.full_like(d, float("inf")), torch.zeros_like(d)))
    big = y64.abs() >= 1e-3 * y64.abs().max()
    rel = (d[big] / y64.abs()[big]).max() if bool(big.any()) else torch.zeros((), dtype=d.dtype)
    return {
        "componentwise_max": float(comp.max()),
        "normwise": float(d.max() / y64.abs().max()),
        "relative_max_where_large": float(rel),
        "target": 1e-10,
        "normalisation": "componentwise: |y - y64|_i / (|J| |u0|)_i with J the T-sweep map; relative: over "
                         "outputs with |y64| >= 1e-3 max|y64| (componentwise relative error is ill-posed where "
                         "outputs cancel toward 0; FP64 itself does not meet it there)",
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
    errors = hilo_errors(ops, u0, out, T)
    interior = (n - 2) * (n - 2)
    res = {
        "workload": f"{n}x{n} FP64 z*10**U(-3,3) seed 0, encode + {T} hi/lo sweeps + decode per step",
        "ms_per_step": round(sec * 1e3, 4),
        "GFLOPs_fp64_equivalent": round(FLOP_PER_POINT * interior * T / sec / 1e9, 1),
        "fp64_equivalent_GBps": round(16.0 * interior * T / sec / 1e9, 1),
        "speedup_vs_plain_fp64_single_sweep": round(plain_sec_per_step / sec, 3),
        "speedup_vs_plain_fp64_default_schedule": round(default_sec_per_step / sec, 3),
        "error_vs_fp64": errors,
    }
    del out, work
    # Per-launch time of the encoded sweep against plain FP64 at one sweep per launch, at this size and
    # at 8192^2, where the Infinity Cache cannot hold the ping-pong pair and HBM serves every byte.
    res["one_pass_per_sweep"] = {}
    for m in (n, 8192):
        um = u0 if m == n else torch.from_numpy(mixed_f64(0, m)).to("cuda:0")
        g = ops.hilo_encode(um)
        dst = ops.hilo_empty(m, m, m, um.device)
        wk = ops.hilo_empty(m, m, m, um.device)
        ops.jacobi5_hilo_encoded(g, 4, dst=dst, work=wk)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        ops.jacobi5_hilo_encoded(g, args.kernel_reps, dst=dst, work=wk)
        e1.record()
        torch.cuda.synchronize()
        hilo_us = e0.elapsed_time(e1) / args.kernel_reps * 1e3
        a, b = um.clone(), um.clone()
        plain_us = time_kernel_launches(ops, a, b, args.kernel_reps) * 1e3
        # encode and decode of the whole grid, timed alone
        e0.record()
        for _ in range(10):
            ops.hilo_encode(um, out=g)
        e1.record()
        torch.cuda.synchronize()
        enc_us = e0.elapsed_time(e1) / 10 * 1e3
        e0.record()
        for _ in range(10):
            ops.hilo_decode(g, out=a)
        e1.record()
        torch.cuda.synchronize()
        dec_us = e0.elapsed_time(e1) / 10 * 1e3
        pts = (m - 2) * (m - 2)
        res["one_pass_per_sweep"][f"{m}x{m}"] = {
            "hilo_sweep_us": round(hilo_us, 2),
            "hilo_sweep_hbm_frac_at_12B": round(12.0 * pts / (hilo_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
            "plain_fp64_sweep_us": round(plain_us, 2),
            "plain_fp64_hbm_frac_at_16B": round(16.0 * pts / (plain_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
            "speedup_hilo_vs_plain": round(plain_us / hilo_us, 3),
            "speedup_ceiling": round(16.0 / 12.0, 3),
            "encode_us": round(enc_us, 2),
            "encode_hbm_frac_at_14B": round(14.0 * m * m / (enc_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
            "decode_us": round(dec_us, 2),
            "decode_hbm_frac_at_14B": round(14.0 * m * m / (dec_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
        }
        del g, dst, wk, a, b
        if m != n:
            del um
        torch.cuda.empty_cache()
    res["verdict"] = (
        "At one sweep per launch, where the sweep is HBM-bound, the hi/lo form moves 12 B per point instead "
        "of 16 B and beats plain FP64 (speedup_hilo_vs_plain, ceiling 1.33x). It loses to the plain calls' "
        "default temporally blocked schedule: there the launches are bound by vector ALU issue, not bytes, "
        "and a hi/lo sweep costs several times the plain sweep's 4 operations per point (TwoSum chains, "
        "renormalisation, re-quantisation), while FP32 vector operations issue at the same rate as FP64 "
        "ones on this chip when packed FP32 is not used.")
    return res


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


def bench_hbm_check(ops, args, sizes=(8192, 16384), T: int = 100) -> dict:
    """The plain step where HBM serves every byte: at 8192^2 FP64 a ping-pong pair is 2 x 512 MiB and at
    16384^2 (the paper's per-GPU tile) 2 x 2 GiB, both past the 256 MB Infinity Cache (MALL); at 4096^2
    (2 x 128 MiB) part of the traffic is MALL-served. The library's 16-byte vector copy of the same grid
    (the plain call with T = 0) gives the practical HBM ceiling at each size; torch's copy_ is shown
    beside it."""
    import torch

    from workloads import large_f64

    res = {}

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

    for n in sizes:
        log(f"[bench] HBM check {n}x{n}")
        u0 = torch.from_numpy(large_f64(0, n)).to("cuda:0")
        out = torch.empty_like(u0)
        work = torch.empty_like(u0)
        interior = (n - 2) ** 2
        r = {"workload": f"{n}x{n} FP64 N(0,1) seed 0, {T} sweeps per step"}
        copy_sec = timed(lambda: ops.jacobi5(u0, 0, out=out), 10)
        copy_gbs = 2 * 8 * n * n / copy_sec / 1e9
        r["copy16_GBps"] = round(copy_gbs, 1)
        r["copy16_hbm_frac"] = round(copy_gbs / HBM_PEAK_GBS, 4)
        r["torch_copy_GBps"] = round(2 * 8 * n * n / timed(lambda: out.copy_(u0), 10) / 1e9, 1)
        for name, sched in (("default_schedule", 0), ("single_sweep_schedule", 1)):
            ops.set_schedule(sched)
            sec = timed(lambda: ops.jacobi5(u0, T, out=out, work=work), 3 if n <= 8192 else 1)
            gbs = 16.0 * interior * T / sec / 1e9
            r[name] = {"ms_per_step": round(sec * 1e3, 3), "us_per_sweep": round(sec / T * 1e6, 2),
                       "GFLOPs": round(FLOP_PER_POINT * interior * T / sec / 1e9, 1),
                       "effective_GBps_at_16B": round(gbs, 1)}
            if sched == 1:
                r[name]["hbm_frac"] = round(gbs / HBM_PEAK_GBS, 4)
                r[name]["frac_of_copy16"] = round(gbs / copy_gbs, 4)
        ops.set_schedule(0)
        res[f"{n}x{n}"] = r
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
    return {
        "workload": f"1024 FP32 grids N(0,1) seed 0, sizes log-uniform in [2^8, 2^16] points "
                    f"({points} points, {interior} interior), {T} sweeps each, one persistent launch "
                    f"replayed from a HIP graph",
        "ms_per_batch": round(sec * 1e3, 4),
        "ms_per_batch_events": round(ev_sec * 1e3, 4),
        "batches_per_s": round(1.0 / sec, 2),
        "grids_per_s": round(len(u0s) / sec, 1),
        "point_sweeps_per_s": round(pts / sec, 1),
        "roofline": {
            "bound": "alu",
            "achieved": round(FLOP_PER_POINT * pts / ev_sec / 1e12, 3),
            "peak": FP32_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(FLOP_PER_POINT * pts / ev_sec / 1e12 / FP32_PEAK_TFLOPS, 4),
            "add_mul_rate_frac": round(FLOP_PER_POINT * pts / ev_sec / 1e12 / ADD_MUL_PEAK_TOPS, 4),
            "note": "4 FP32 operations per interior point per sweep over the batch's event time, against the "
                    "FP32 vector peak and against the add/multiply issue rate without packed or fused "
                    "operations (39.3 Tops/s); grids in register mode never leave registers between sweeps, "
                    "so neither HBM nor LDS bandwidth binds them (LDS carries only each wave's edge rows)",
        },
        "effective_GBps_at_8B": round(8.0 * pts / sec / 1e9, 1),
        "config": info,
        "autotuned_us": round(tuned_us, 1),
        "plain_per_grid_ms": round(plain_sec * 1e3, 2),
        "speedup_vs_plain_launches": round(plain_sec / sec, 1),
        "bit_identical_to_plain": bool(same),
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
    cases = ((2, 2, 1, "packed", True), (4, 4, 1, "packed", True), (2, 2, 1, "direct", False),
             (4, 4, 1, "direct", False), (2, 2, 12, "packed", True), (2, 2, 12, "packed", False),
             (2, 2, 12, "direct", False), (4, 4, 12, "direct", False), (8, 8, 12, "direct", False))
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
                       "copy kernel), on a second stream (2stream, the paper's overlap scheme, with an event "
                       "each way per exchange) or the compute stream (1stream); g = 1: one exchange and one "
                       "sweep launch over all tiles (per 32 tiles) per sweep; g > 1: one exchange and one "
                       "blocked launch over all tiles (per 32 tiles) per chunk of up to g sweeps, the sweeps "
                       "split evenly over the chunks")
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


def _frontend_listing(ops, n: int, T: int, depths) -> dict:
    """The listing program on an n x n unit-ring grid through the lazy frontend, T iterations, for each
    maximum DAG depth (best of 3 runs), next to one direct call."""
    import torch

    from paper_2512_19851_amd import frontend

    u = torch.zeros((n, n), dtype=torch.float64, device="cuda:0")
    u[0, :] = u[-1, :] = u[:, 0] = u[:, -1] = 1
    ideal = []
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ops.jacobi5(u, T)
        torch.cuda.synchronize()
        ideal.append(time.perf_counter() - t0)
    del u
    res = {"workload": f"listing program, {n}x{n} FP64 unit ring, {T} iterations; per DAG depth the best "
                       f"of 3 runs (the first loads the kernels a chain plan needs)",
           "ideal_ms": round(min(ideal) * 1e3, 2)}
    for depth in depths:
        best = None
        host = None
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
            ctx.flush()
            t_host = time.perf_counter() - t0
            ctx.sync()
            sec = time.perf_counter() - t0
            if best is None or sec < best:
                best, host = sec, t_host
            del u1, u2
        res[f"depth_{depth}_ms"] = round(best * 1e3, 2)
        res[f"depth_{depth}_host_ms"] = round(host * 1e3, 2)
        res[f"depth_{depth}_chained_nodes"] = ctx.stats["chained_nodes"]
        del ctx
    torch.cuda.empty_cache()
    return res


def bench_frontend(ops, args) -> dict:
    """One-GPU analog of the pipelining experiment (Section V): the listing program through the
    lazy frontend, runtime against the maximum DAG depth, next to one direct call (no Python per node).
    At 4096^2 a chained node carries less GPU work than its Python cost, so the host bounds the run;
    at the paper's 16384^2 per GPU the GPU does, and the host's recording of later nodes overlaps the
    kernels of earlier flushes (depth_*_host_ms: time until the last flush returned)."""
    log("[bench] frontend pipelining")
    res = _frontend_listing(ops, 4096, 200, (1, 10, 100, 1000))
    res["paper_size"] = _frontend_listing(ops, 16384, 200, (1, 10, 100, 1000))
    return res


def bench_cavity(args, n: int = 16384, nit: int = CAVITY_NIT, steps: int = 2) -> dict:
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
    passes = bench_pressure_passes(n, 5, pressure_pass_levels(nit))
    traffic = load_traffic(PRESSURE_TRAFFIC_FILE, PRESSURE_SRC, levels=passes["levels"]) if n == 16384 else None
    passes["traffic"] = traffic
    passes["hbm_use_frac"] = (round(traffic / (passes["avg_us_per_call"] * 1e-6) / (HBM_PEAK_GBS * 1e9), 4)
                              if traffic else None)
    res["pressure_pass"] = passes
    res["speedup_blocked_vs_per_node"] = round(res["per_node_pressure"]["ms_per_step"] /
                                               res["blocked_pressure"]["ms_per_step"], 2)
    del fields
    torch.cuda.empty_cache()
    return res


def bench_pressure_passes(n: int, reps: int, levels: int = 0) -> dict:
    """`reps` launches of the blocked pressure kernel, each one pass of `levels` cavity pressure iterations
    (0: the pass of the cavity step's 50, i.e. 10, the LDS-ring kernel) on an n x n FP64 grid (N(0,1) p and
    b, seed 0), timed with HIP events on the launch stream."""
    levels = levels or pressure_pass_levels(CAVITY_NIT)
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
    """Gradient workload: 1024x1024 FP32, L = sum(w * u_T), dL/du0 and dL/dc through autograd; the forward
    pass with recorded states and the reverse pass timed on the GPU; the transposed sweep per point against
    the forward FP32 method at the same size and schedule kind."""
    import torch

    from paper_2512_19851_amd import _lib, autograd, ops
    from workloads import adjoint_f32

    log("[bench] adjoint")
    u0_np, w_np, _ = adjoint_f32(0)
    u0 = torch.from_numpy(u0_np).to("cuda:0")
    w = torch.from_numpy(w_np.astype("float32")).to("cuda:0")
    c = torch.tensor(0.25, dtype=torch.float32, device="cuda:0", requires_grad=True)
    H, W = u0.shape
    stream = torch.cuda.current_stream()

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

    def timed(fn, r):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(r):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / r * 1e-3

    # the two passes of the step on the GPU: forward recording u_0..u_T, reverse with dL/dc
    states = torch.empty((T + 1, H, W), dtype=torch.float32, device=u0.device)
    gin = torch.empty_like(u0)
    work = torch.empty_like(u0)
    parts = torch.empty(int(_lib.load().sten_adjoint_partials_len(H, W)), dtype=torch.float64, device=u0.device)
    dc = torch.empty(1, dtype=torch.float64, device=u0.device)
    sp = stream.cuda_stream
    fwd_sec = timed(lambda: _lib.call("sten_jacobi5_f32_states", u0.data_ptr(), states.data_ptr(), H, W, W, T, 0.25,
                                      sp), 20)

    def reverse():
        _lib.call("sten_jacobi5_adjoint_f32_seg", w.data_ptr(), states.data_ptr(), T, gin.data_ptr(),
                  work.data_ptr(), parts.data_ptr(), 1, H, W, W, 0.25, sp)
        _lib.call("sten_reduce_f64", parts.data_ptr(), parts.numel(), dc.data_ptr(), sp)

    rev_sec = timed(reverse, 20)
    # the transposed sweep without states (several per launch) against the forward FP32 method, per sweep
    R = args.kernel_reps
    g = torch.randn_like(u0)
    adj_sec = timed(lambda: autograd.adjoint(g, R, 0.25), 3) / R
    fo, fw = torch.empty_like(u0), torch.empty_like(u0)
    fwd_sweep_sec = timed(lambda: ops.jacobi5(u0, R, out=fo, work=fw), 3) / R
    return {
        "workload": f"{H}x{W} FP32 u0 N(0,1), w N(0,1) seed 0, T={T}: forward with recorded states + "
                    f"reverse pass (dL/du0 and dL/dc) per step",
        "ms_per_step": round(sec * 1e3, 4),
        "forward_with_states_us": round(fwd_sec * 1e6, 2),
        "reverse_with_dc_us": round(rev_sec * 1e6, 2),
        "reverse_vs_forward": round(rev_sec / fwd_sec, 3),
        "adjoint_sweep_us": round(adj_sec * 1e6, 3),
        "forward_fp32_sweep_us": round(fwd_sweep_sec * 1e6, 3),
        "adjoint_vs_forward_per_point": round(adj_sec / fwd_sweep_sec, 3),
        "adjoint_sweep_GBps_at_8B": round(8.0 * H * W / adj_sec / 1e9, 1),
        "note": "ms_per_step: wall time of autograd forward + backward (Python and allocations included); "
                "forward_with_states_us / reverse_with_dc_us: HIP events around the library calls alone; "
                f"adjoint_sweep_us and forward_fp32_sweep_us: {R} sweeps in one call each (several sweeps "
                "per launch in both), divided by the sweeps",
        "tolerance": "dL/du0 within the FP32 bound of the FP64 oracle gradient and of central FD "
                     "(h=1e-6) at 64 coordinates; dL/dc within its bound (parity tests)",
    }


def graph_replay_step(ops, u0, T: int, out, work, steps: int, eager_sec: float) -> dict:
    """The plain step (ring copy + blocked launches) captured once in a HIP graph and replayed: wall time per
    replay, and the replays' result against the eager step's bits (the output is cleared between replays)."""
    import torch

    ref = out.clone()
    ops.jacobi5(u0, T, out=ref, work=work)
    gs = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=gs):
        ops.jacobi5(u0, T, out=out, work=work)
    same = True
    for _ in range(3):
        out.zero_()
        g.replay()
        torch.cuda.synchronize()
        same = same and bool(torch.equal(out, ref))
    t0 = time.perf_counter()
    for _ in range(steps):
        g.replay()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    same = same and bool(torch.equal(out, ref))
    del g
    return {"ms_per_step": round(sec * 1e3, 4), "vs_eager_calls": round(eager_sec / sec, 3),
            "bit_identical_to_eager": same,
            "note": "one step (ring copy + the blocked launches) captured with torch.cuda.graph and replayed; "
                    "the headline value is the eager calls"}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--sweeps", type=int, default=100, help="sweeps T per step")
    ap.add_argument("--n", type=int, default=4096, help="grid side")
    ap.add_argument("--kernel-reps", type=int, default=100)
    ap.add_argument("--levels", type=int, default=TB_LEVELS, help="sweeps per launch in --mode tb")
    ap.add_argument("--pressure-levels", type=int, default=0,
                    help="iterations per pass in --mode pressure (1..12; 0: the cavity step's pass, 10)")
    ap.add_argument("--cpu-budget", type=float, default=16.0, help="seconds of CPU oracle work")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extensions", action="store_true")
    ap.add_argument("--mode", choices=["step", "sweep", "copy", "hilo", "tb", "cavity", "pressure", "batch", "adjoint",
                                       "tiled", "mixed", "frontend"],
                    default="step",
                    help="step: the benchmark; sweep: only --kernel-reps sweep launches; "
                         "copy: only --kernel-reps plain grid copies (counter calibration); "
                         "hilo: only --kernel-reps hi/lo sweeps on encoded grids; "
                         "tb: only --kernel-reps temporally blocked launches of --levels sweeps; "
                         "cavity: only the cavity-flow extension (--n grid side); "
                         "pressure: only --kernel-reps blocked passes of --pressure-levels cavity pressure "
                         "iterations (--n); "
                         "batch: only the batched extension (--sweeps, --steps graph replays); "
                         "adjoint: only the gradient extension (1024^2, T = 10); "
                         "tiled: only the tiled extension (--n, --sweeps); "
                         "mixed: only the hi/lo extension (--n, --sweeps; timed against one sweep per launch); "
                         "frontend: only the lazy-frontend pipelining runs (4096^2 and 16384^2)")
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
        print(json.dumps(bench_pressure_passes(args.n, args.kernel_reps, args.pressure_levels)), flush=True)
        return 0
    if args.mode == "batch":
        from paper_2512_19851_amd import ops

        print(json.dumps({"mode": "batch", **bench_batch(ops, args.sweeps, args)}), flush=True)
        return 0
    if args.mode == "adjoint":
        print(json.dumps({"mode": "adjoint", **bench_adjoint(10, args)}), flush=True)
        return 0
    if args.mode == "frontend":
        print(json.dumps({"mode": "frontend", **bench_frontend(ops, args)}), flush=True)
        return 0
    if args.mode in ("tiled", "mixed"):
        n, T = args.n, args.sweeps
        u0 = torch.from_numpy(large_f64(0, n)).to(dev)
        o, w = torch.empty_like(u0), torch.empty_like(u0)
        ops.jacobi5(u0, T, out=o, work=w)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ops.jacobi5(u0, T, out=o, work=w)
        torch.cuda.synchronize()
        blocked = time.perf_counter() - t0
        ops.set_schedule(1)
        ops.jacobi5(u0, T, out=o, work=w)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ops.jacobi5(u0, T, out=o, work=w)
        torch.cuda.synchronize()
        single = time.perf_counter() - t0
        ops.set_schedule(0)
        del u0, o, w
        if args.mode == "tiled":
            res = bench_tiled(ops, n, T, args, single, blocked)
        else:
            res = bench_mixed(ops, n, T, args, single, blocked)
        print(json.dumps({"mode": args.mode, **res}), flush=True)
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
                ops.jacobi5_tb(a, args.levels, levels=args.levels, out=b)  # one blocked launch
            else:
                ops.jacobi5(a, 0, out=b)  # T = 0: one plain copy of the grid
            a, b = b, a
        e1.record()
        torch.cuda.synchronize()
        per = e0.elapsed_time(e1) / args.kernel_reps
        moved = {"sweep": launch_bytes, "tb": args.levels * launch_bytes}.get(args.mode, 16.0 * n * n)
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

    log("[bench] the same step captured in a HIP graph and replayed")
    try:
        graph_replay = graph_replay_step(ops, u0, T, out, work, args.steps, sec_per_step)
    except Exception as e:  # reported, never fatal to the benchmark line
        torch.cuda.synchronize()
        graph_replay = {"error": f"{type(e).__name__}: {e}"}

    log(f"[bench] per-launch kernel timing, {args.kernel_reps} launches")
    a = out.clone()
    b = work
    b.copy_(a)
    # The step's launches, timed live: the HIP events that bracket the timed steps on the launch stream,
    # divided by the blocked launches per step (the step's kernels are these launches plus a ring copy of
    # a few microseconds). T sweeps run as ceil(T / cap) launches, the sweeps split evenly.
    cap = tb_cap(n)
    launches = -(-T // cap)
    base, extra = divmod(T, launches)
    def kname(lev: int) -> str:
        return f"sweep_stream_deep_kernel<{lev}>" if lev > TB_CAP else f"sweep_stream_kernel<double,2,{lev},4>"

    mix = ([f"{kname(base + 1)} x{extra}"] if extra else []) + [f"{kname(base)} x{launches - extra}"]
    step_launch_ms = ev_ms / args.steps / launches
    step_launch_flop = FLOP_PER_POINT * interior * T / launches
    tflops = step_launch_flop / (step_launch_ms * 1e-3) / 1e12
    traffic = load_traffic(TB_TRAFFIC_FILE, TB_SRC)
    roofline = {
        "bound": "alu",
        "achieved": round(tflops, 3),
        "peak": FP64_PEAK_TFLOPS,
        "unit": "TFLOP/s",
        "frac": round(tflops / FP64_PEAK_TFLOPS, 4),
        "traffic": traffic,
        "kernel": f"the step's blocked launches: {' + '.join(mix)} ({T} sweeps of the {n}x{n} FP64 grid in "
                  f"{launches} launches)",
        "algorithmic_flop_per_launch": step_launch_flop,
        "avg_launch_us": round(step_launch_ms * 1e3, 2),
        "step_us_per_sweep": round(sec_per_step / T * 1e6, 2),
        "note": "achieved = 4 FP64 operations (3 adds, 1 multiply) per interior point per sweep, "
                f"{T / launches:.2f} sweeps per launch on average, over avg_launch_us (HIP events over the "
                "timed steps on the launch stream, divided by the launches per step; includes the step's "
                "ring copy and dispatch gaps). The launches read and write the grid about once for all "
                "their sweeps, so they are bound by vector ALU issue, not HBM; traffic is the measured HBM "
                f"bytes of one launch of the dominant kernel (sweep_stream_kernel<double,2,{TB_LEVELS},4>, "
                "rocprofv3 FETCH_SIZE + WRITE_SIZE, scaled by a plain copy's counters), null when the "
                "kernel source changed since it was measured",
    }
    # Sub-views of the same launches against the other ceilings.
    roofline["add_mul_rate_view"] = {
        "achieved": round(tflops, 3),
        "peak": round(ADD_MUL_PEAK_TOPS, 2),
        "unit": "Tops/s",
        "frac": round(tflops / ADD_MUL_PEAK_TOPS, 4),
        "note": "the same operations against the vector ALUs' add/multiply issue rate without fused "
                "multiply-add (256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz); the sweep's operations are separate "
                "roundings, so this is the arithmetic ceiling; the launches also issue lane shifts and "
                "recompute the halo of each band and strip (VALU issue counters: profiles/)",
    }
    roofline["hbm_view"] = {
        "grid_bytes_per_launch": 16.0 * interior,
        "hbm_floor_us_per_launch": round(launch_bytes / (HBM_PEAK_GBS * 1e9) * 1e6, 2),
        "launch_floor_frac": round(launch_bytes / (HBM_PEAK_GBS * 1e9) / (step_launch_ms * 1e-3), 4),
        "measured_traffic_bytes_per_launch": traffic,
        "hbm_use_frac": round(traffic / (step_launch_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if traffic else None,
        "effective_GBps_at_16B_per_point_per_sweep": round(16.0 * interior * T / launches /
                                                           (step_launch_ms * 1e-3) / 1e9, 1),
        "note": "launch_floor_frac = one read and one write of the grid at 8 TB/s over the launch time; "
                "hbm_use_frac = measured traffic over the launch time against 8 TB/s; the effective figure "
                "counts 16 B per point per sweep as for one sweep per launch, so it exceeds the HBM peak",
    }
    # the dominant kernel alone (every launch TB_LEVELS sweeps), as the profiler's trace sees it
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
    alone_tflops = FLOP_PER_POINT * interior * TB_LEVELS / (alone_ms * 1e-3) / 1e12
    roofline["dominant_kernel_alone"] = {
        "kernel": f"sweep_stream_kernel<double,2,{TB_LEVELS},4>",
        "launches": args.kernel_reps,
        "avg_launch_us": round(alone_ms * 1e3, 2),
        "algorithmic_flop_per_launch": FLOP_PER_POINT * interior * TB_LEVELS,
        "achieved_TFLOPs": round(alone_tflops, 3),
        "frac_of_fp64_peak": round(alone_tflops / FP64_PEAK_TFLOPS, 4),
        "hbm_use_frac": round(traffic / (alone_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if traffic else None,
    }
    # the single-sweep kernel (one sweep per launch, the paper's schedule), HBM-bound
    avg_ms = time_kernel_launches(ops, a, b, args.kernel_reps)
    achieved = launch_bytes / (avg_ms * 1e-3) / 1e9
    copy_ms = time_copy(ops, a, b, args.kernel_reps)
    copy_gbs = 16.0 * n * n / (copy_ms * 1e-3) / 1e9
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
        "copy16_GBps": round(copy_gbs, 1),
        "frac_of_copy16": round(achieved / copy_gbs, 4),
        "ms_per_step_single_sweep_schedule": round(single_sec_per_step * 1e3, 4),
        "GBps_single_sweep_schedule": round(step_bytes / single_sec_per_step / 1e9, 1),
        "note": "at 4096^2 the 2 x 128 MiB pair is about the size of the 256 MiB Infinity Cache, which "
                "serves part of the traffic; extensions.hbm_check repeats the single-sweep schedule and the "
                "copy at 8192^2 and 16384^2, where HBM serves every byte. copy16: the library's 16-byte "
                "vector copy of the same grid (read + write)",
    }

    rec = {
        "metric": METRIC,
        "value": round(FLOP_PER_POINT * interior * T / sec_per_step / 1e9, 1),
        "unit": "GFLOP/s",
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
            "schedule": f"temporal blocking, up to {tb_cap(n)} sweeps per launch, the {T} sweeps split evenly over "
                        f"{-(-T // tb_cap(n))} launches (bit-identical to one sweep per launch)",
            "flop_per_point_per_sweep": FLOP_PER_POINT,
            "bytes_per_point_per_sweep": 16,
            "parallelism": "single GPU",
        },
        "effective_GBps_at_16B": round(value, 1),
        "point_sweeps_per_s": round(interior * T / sec_per_step, 1),
        "roofline": roofline,
        "single_sweep_roofline": single,
        "graph_replay": graph_replay,
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
