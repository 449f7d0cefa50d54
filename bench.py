"""Benchmark of the LOD diffusion-decay step with cell sources on one MI355X.

    python bench.py [--steps K] [--warmup W] [--config single|tumour|batched|plain]

A step is one full LOD step (x, y, z line solves with Dirichlet projection and
decay folded in, then the cell sources) over every simulation of the
workload.  The default workload is the single large simulation (200^3 voxels
x 4 substrates, 1e5 cells, FP32 storage and sweeps); the plain FP64 path is
timed on the same grid for the speedup.  Inputs are resident in HBM before
the timed region; setup (binding, coefficients, cell binning) is excluded.

Prints one JSON line: whole-job voxel-substrate updates/s, per-kernel
roofline of the dominant kernel (algorithmic bytes / average duration from
HIP events recorded on the library's stream) and the FP64 CPU oracle timed on
a bounded sample of the same workload on the host's cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
METRIC = "voxel-substrate updates/s per LOD step (FP32/batched vs FP64) + % HBM peak"
UNIT = "voxel-substrate updates/s"


def make_workload(name: str):
    from paper_2110_13368_amd import workloads as W
    if name == "single":
        return W.single_large("f32")
    if name == "tumour":
        return W.tumour_scale()
    if name == "batched":
        return W.batched()
    if name == "plain":
        return W.plain_fp64()
    raise SystemExit(f"unknown config {name!r}")


def time_steps(ctx, steps: int, warmup: int):
    """Wall time of `steps` graph-replayed steps, synchronised on both sides."""
    import torch
    ctx.step(warmup)
    ctx.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(steps)
    ctx.sync()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def kernel_profile(ctx, steps: int):
    """Per-kernel totals over `steps` directly launched steps, from HIP events
    recorded on the library's stream around every launch."""
    ctx.set_profiling(True)
    ctx.step(steps)
    stats = ctx.kernel_stats()
    ctx.set_profiling(False)
    return stats


def copy_reference(nbytes: int, reps: int = 20):
    """Device-to-device copy of nbytes with a plain elementwise kernel: the
    practical bandwidth ceiling, and the kernel of known traffic (nbytes read,
    nbytes written per launch) that scales the FETCH_SIZE / WRITE_SIZE
    counters."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / reps
    del src, dst
    torch.cuda.empty_cache()
    return {"bytes": nbytes, "GBps_read_plus_write": round(2 * nbytes / t / 1e9, 1)}


def cpu_baseline(wl, budget_s: float):
    """The FP64 oracle on the host cores: whole steps of the same workload
    (for a batch: its first simulations), as many as fit the time budget."""
    import oracle
    threads = oracle.get_threads()
    sims = wl.sims if len(wl.sims) == 1 else wl.sims[:8]
    objs = [oracle.from_spec(s) for s in sims]
    updates = sum(s.n_vox * s.n_sub for s in sims)
    steps, t = 0, 0.0
    while t < budget_s and steps < 1000:
        t0 = time.perf_counter()
        for o in objs:
            o.step(1)
        t += time.perf_counter() - t0
        steps += 1
    sample = (f"{steps} step(s) of {len(sims)} simulation(s) "
              f"({'x'.join(map(str, sims[0].shape))} x {sims[0].n_sub}"
              f"{', first of the batch' if len(sims) > 1 else ''})")
    return {"value": updates * steps / t, "unit": UNIT, "cores": threads, "kind": "oracle",
            "sample": sample, "seconds": round(t, 3)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--config", default="single")
    ap.add_argument("--fp64-steps", type=int, default=None)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-copy-reference", action="store_true")
    ap.add_argument("--mode", default="tuned", choices=["tuned", "launches", "persistent"])
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "batched simulations shard by simulation and a single grid by z-slabs, "
              "neither is built here.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2110_13368_amd import binding as vb

    wl = make_workload(args.config)
    E = wl.voxel_substrates
    print(f"bench: {wl.name}: {len(wl.sims)} sim(s), {E} voxel-substrates", file=sys.stderr, flush=True)

    precision = vb.VL_F64 if wl.dtype == "f64" else vb.VL_F32
    ctx = vb.Context(wl.sims, precision=precision)
    if args.mode == "tuned":
        ctx.tune(None)  # times the step modes on these buffers; setup, not timed
    else:
        ctx.set_option(vb.VL_OPT_STEP_MODE,
                       vb.VL_MODE_PERSISTENT if args.mode == "persistent" else vb.VL_MODE_LAUNCHES)
    mode = "persistent" if ctx.get_option(vb.VL_OPT_STEP_MODE) == vb.VL_MODE_PERSISTENT else "launches"
    for k, s in enumerate(wl.sims):
        ctx.set_field(k, s.rho0)
    elapsed = time_steps(ctx, args.steps, args.warmup)
    value = E * args.steps / elapsed
    esize = 8 if precision == vb.VL_F64 else 4
    b_alg = 3 * 2 * esize  # bytes per voxel-substrate-step: three sweeps, read + write
    print(f"bench: {args.steps} steps in {elapsed:.4f} s", file=sys.stderr, flush=True)

    stats = kernel_profile(ctx, args.steps)
    ctx.close()
    del ctx
    torch.cuda.empty_cache()
    kinds = {k: v for k, v in stats.items() if v[0] > 0}
    dom = max(kinds, key=lambda k: kinds[k][1])
    launches, total_ms = kinds[dom]
    per_step_ms = total_ms / args.steps
    launches_per_step = launches / args.steps
    if dom.startswith("sweep"):
        alg_bytes = 2 * esize * E  # every element read once and written once per sweep
    elif dom == "step":
        alg_bytes = b_alg * E  # the one-launch step: three sweeps
    else:
        alg_bytes = None
    roofline = {
        "kernel": dom,
        "bound": "hbm",
        "achieved": round(alg_bytes / (per_step_ms * 1e-3) / 1e9, 1) if alg_bytes else None,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(alg_bytes / (per_step_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if alg_bytes else None,
        "traffic": None,
        "avg_ms": round(per_step_ms / launches_per_step, 5),
        "launches_per_step": launches_per_step,
        "bytes_per_launch": alg_bytes / launches_per_step if alg_bytes else None,
    }
    kernels = {k: {"launches": v[0], "avg_ms": round(v[1] / max(v[0], 1), 5)} for k, v in kinds.items()}

    extra = {}
    if precision == vb.VL_F32 and len(wl.sims) == 1:
        # plain FP64 path on the same grid: the speedup denominator
        from paper_2110_13368_amd import workloads as W
        s64 = [W.SimSpec(s.shape, s.h, s.lo, s.D, s.lam, s.dt, s.bc_kind, s.bc_value,
                         s.rho0.astype(np.float64), s.cells) for s in wl.sims]
        n64 = args.fp64_steps or max(10, args.steps // 5)
        c64 = vb.Context(s64, precision=vb.VL_F64)
        t64 = time_steps(c64, n64, min(args.warmup, 5))
        c64.close()
        v64 = E * n64 / t64
        extra["fp64_plain"] = {"value": v64, "ms_per_step": 1e3 * t64 / n64, "steps": n64,
                               "speedup_fp32_over_fp64": value / v64}

    line = {
        "metric": METRIC,
        "value": value,
        "unit": UNIT,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": wl.dtype,
        "data": "synthetic (seeded generators shaped like the paper's tumour workloads)",
        "config": {"workload": wl.name, "sims": len(wl.sims), "voxel_substrates": E,
                   "grid": list(wl.sims[0].shape) if len(wl.sims) == 1 else "ragged",
                   "n_sub": wl.sims[0].n_sub, "cells": int(sum(s.cells.n for s in wl.sims)),
                   "dt": wl.sims[0].dt, "parallelism": "single-gpu", "step_mode": mode},
        "hbm_effective": {"bytes_per_update": b_alg,
                          "GBps": round(b_alg * value / 1e9, 1),
                          "frac_of_peak": round(b_alg * value / 1e9 / HBM_PEAK_GBS, 4)},
        "roofline": roofline,
        "kernels": kernels,
    }
    line.update(extra)
    if not args.no_copy_reference:
        line["copy_reference"] = [copy_reference(128 << 20), copy_reference(2 << 30, reps=5)]
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
