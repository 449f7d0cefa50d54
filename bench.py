"""Benchmark of the LOD diffusion-decay step with cell sources on one MI355X.

    python bench.py [--steps K] [--warmup W] [--config tumour|single|batched|planar|plain|adjoint]

A step is one full LOD step (x, y, z line solves with Dirichlet projection and
decay folded in, then the cell sources) over every simulation of the
workload.  The default workload is the tumour-scale simulation (400^3 voxels
x 8 substrates, 1e6 cells, FP32 storage and sweeps): the largest
configuration, and the one whose 2 GB field cannot sit in the 256 MB
Infinity Cache, so its bandwidth is HBM bandwidth.  The plain FP64 path is
timed on the same grid for the speedup, and the batch of 256 ragged
simulations is timed after it as an extra line (``batched``).  Inputs are
resident in HBM before the timed region; setup (binding, coefficients, cell
binning, tuning) is excluded.

Prints one JSON line: whole-job voxel-substrate updates/s, per-kernel
roofline of the dominant kernel (algorithmic bytes / average duration from
HIP events recorded on the library's stream) and the FP64 CPU oracle timed on
a bounded sample of the same workload on the host's cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
INFINITY_CACHE_BYTES = 256 << 20  # MI355X last-level (memory-side) cache
METRIC = "voxel-substrate updates/s per LOD step (FP32/batched vs FP64) + % HBM peak"
UNIT = "voxel-substrate updates/s"


LDS_PER_WORKGROUP = 160 * 1024  # gfx950
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_mi355x.json")


def source_digest(files) -> str:
    """sha256 over the named kernel sources (paper_2110_13368_amd/csrc)."""
    h = hashlib.sha256()
    for name in sorted(files):
        h.update(name.encode())
        with open(os.path.join(ROOT, "paper_2110_13368_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(workload: str, kernel: str, launch: dict | None = None):
    """HBM bytes of a sweep kind per step (its launches in one step, the basis
    of the roofline's achieved rate) from the committed FETCH_SIZE /
    WRITE_SIZE measurements (scaled by the copy-kernel calibration), or None
    when there is none for this workload and launch configuration, or the
    kernel's sources changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            table = json.load(f)
    except (OSError, ValueError):
        return None
    for e in table.get("entries", []):
        if e.get("workload") == workload and e.get("kernel") == kernel:
            if launch is not None and e.get("launch") != launch:
                continue
            if e.get("sources_sha256") != source_digest(e.get("sources", [])):
                return None
            return int(e["bytes_read"] + e["bytes_written"])
    return None


def plane_fits(nx: int, ny: int) -> bool:
    """Whether a z-plane of nx x ny is solved by the x+y plane kernel (its LDS
    need: both pivot tables, the exchange slots, rows padded to odd length)."""
    cbx, cby = nx - 1 - (nx - 1) // 2, ny - 1 - (ny - 1) // 2
    return (cbx + cby) * 16 + 256 * 8 + ny * (nx | 1) * 4 <= LDS_PER_WORKGROUP


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
    if name == "planar":
        return W.planar()
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


def time_snapshots(ctx, wl, steps: int, every: int):
    """Steps with a snapshot of every simulation's field to pinned host memory
    every `every` steps (vl_snapshot: a staging copy on the library's stream,
    the transfer on its copy stream while the next steps run), all waited for
    at the end.  Returns (seconds, snapshots, seconds for one snapshot of
    every simulation taken alone, bytes per snapshot of all simulations)."""
    torch = ctx.torch
    outs = [torch.empty(tuple(s.field_shape), dtype=ctx.dtype, pin_memory=True) for s in wl.sims]
    nbytes = sum(o.numel() * o.element_size() for o in outs)
    for rep in range(2):  # the first call also creates the copy stream
        ctx.sync()
        t0 = time.perf_counter()
        for k in range(len(wl.sims)):
            ctx.snapshot(k, outs[k])
        ctx.snapshot_wait()
        t_alone = time.perf_counter() - t0
    ctx.sync()
    t0 = time.perf_counter()
    done = n = 0
    while done < steps:
        take = min(every, steps - done)
        ctx.step(take)
        done += take
        if take == every:
            for k in range(len(wl.sims)):
                ctx.snapshot(k, outs[k])
            n += 1
    ctx.sync()
    ctx.snapshot_wait()
    return time.perf_counter() - t0, n, t_alone, nbytes


def time_moving_cells(ctx, wl, steps: int, every: int):
    """Steps with the cells of every simulation moved and re-binned from device
    arrays every `every` steps (vl_upload_cells_dev: voxel index, sort,
    composites; the positions are prepared on the device beforehand, a small
    random walk per move; no count of cells off the grid is asked for, so an
    upload waits for the stream only to check the arrays; a forward run, so
    the uploads skip the per-cell tables only the adjoint reads).  Returns
    (seconds, uploads, host seconds in the upload calls, which include waiting
    for the steps queued before them)."""
    import torch
    from paper_2110_13368_amd import binding as vb
    n_moves = max(steps // every, 1)
    g = torch.Generator(device=ctx.device).manual_seed(211013368 + 50)
    dev = []
    for s in wl.sims:
        c = s.cells
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(ctx.device)
        pos0 = t(c.pos)
        walk = torch.randn((n_moves,) + tuple(pos0.shape), generator=g, device=ctx.device,
                           dtype=torch.float64) * (0.5 * s.h[0])
        dev.append((pos0 + torch.cumsum(walk, 0), t(c.V), t(c.S), t(c.U), t(c.rho_star)))
    ctx.set_option(vb.VL_OPT_ADJOINT_TABLES, 0)
    torch.cuda.synchronize()
    t_up = 0.0
    t0 = time.perf_counter()
    done = 0
    for m in range(n_moves):
        u0 = time.perf_counter()
        for k, (pos, V, S, U, rs) in enumerate(dev):
            ctx.upload_cells_device(k, pos[m], V, S, U, rs, count_out=False)
        t_up += time.perf_counter() - u0
        take = min(every, steps - done)
        ctx.step(take)
        done += take
    ctx.sync()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ctx.set_option(vb.VL_OPT_ADJOINT_TABLES, 1)
    return elapsed, n_moves, t_up


def kernel_profile(ctx, steps: int):
    """Per-kernel totals over `steps` directly launched steps, from HIP events
    recorded on the library's stream around every launch."""
    ctx.set_profiling(True)
    ctx.step(steps)
    stats = ctx.kernel_stats()
    ctx.set_profiling(False)
    return stats


def copy_reference(nbytes: int, reps: int = 20):
    """Device-to-device copies of nbytes: torch's elementwise copy and the
    library's copy probe (vl_copy_probe) with 4- and 16-byte accesses per
    lane, ordinary or non-temporal loads and stores, between two buffers and
    in place, and in 64 KiB tiles loaded whole before they are stored.  The fastest is the
    practical bandwidth ceiling for a sweep (which reads and writes every
    element once); each is a kernel of known traffic (nbytes read, nbytes
    written per launch) that scales the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    from paper_2110_13368_amd import binding as vb
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream().cuda_stream

    def rate(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return round(2 * nbytes / ((time.perf_counter() - t0) / reps) / 1e9, 1)

    out = {"bytes": nbytes, "GBps_read_plus_write": rate(lambda: dst.copy_(src))}
    probe = {}
    for width in (4, 16):
        for nt in (0, 3):
            probe[f"width{width}_nt{nt}"] = rate(
                lambda: vb.vl_copy_probe(dst.data_ptr(), src.data_ptr(), nbytes, width, nt, stream))
    # in place (source = destination), the way a sweep moves its field
    for width in (4, 16):
        for nt in (0, 3):
            probe[f"in_place_width{width}_nt{nt}"] = rate(
                lambda: vb.vl_copy_probe(dst.data_ptr(), dst.data_ptr(), nbytes, width, nt, stream))
    # 64 KiB tiles, each loaded whole before it is stored (a sweep tile's shape)
    probe["tile64k"] = rate(lambda: vb.vl_copy_probe(dst.data_ptr(), src.data_ptr(), nbytes, 16, 4, stream))
    probe["tile64k_in_place"] = rate(lambda: vb.vl_copy_probe(dst.data_ptr(), dst.data_ptr(), nbytes, 16, 4, stream))
    if not torch.equal(dst, src):
        raise RuntimeError("vl_copy_probe: destination differs from source")
    out["vl_copy_probe_GBps"] = probe
    del src, dst
    torch.cuda.empty_cache()
    return out


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


def adjoint_cpu_baseline(wl, grads, budget_s: float):
    """The FP64 oracle's adjoint (forward with checkpoints, reverse) on the
    host cores, over as many steps of the same workload as fit the budget."""
    import oracle
    spec = wl.sims[0]
    n, t = 2, 0.0
    while True:
        sim = oracle.from_spec(spec)
        t0 = time.perf_counter()
        sim.adjoint(n, grads[0])
        t = time.perf_counter() - t0
        sim.close()
        if t > budget_s / 3 or n >= wl.steps:
            break
        n = min(wl.steps, 2 * n)
    return {"value": spec.n_vox * spec.n_sub * n / t, "unit": "voxel-substrate steps reversed/s",
            "cores": oracle.get_threads(), "kind": "oracle",
            "sample": f"adjoint of {n} steps of {'x'.join(map(str, spec.shape))} x {spec.n_sub} "
                      f"with {spec.cells.n} cells", "seconds": round(t, 3)}


def apply_launch_options(ctx, args, vb):
    """The launch configuration of an FP32 context: the tuner's choice on the
    bound buffers (setup, not timed) unless --mode launches, then every option
    given on the command line on top."""
    if args.mode == "tuned":
        ctx.tune(None)
    else:
        ctx.set_option(vb.VL_OPT_STEP_MODE,
                       vb.VL_MODE_PERSISTENT if args.mode == "persistent" else vb.VL_MODE_LAUNCHES)
    if args.x_lanes != "auto":
        ctx.set_option(vb.VL_OPT_X_LANES, int(args.x_lanes))
    if args.x_lane_lines != "auto":
        ctx.set_option(vb.VL_OPT_X_LANE_LINES, int(args.x_lane_lines))
    if args.sources != "auto":
        ctx.set_option(vb.VL_OPT_FUSE_SOURCES, int(args.sources))
    if args.xy != "auto":
        ctx.set_option(vb.VL_OPT_FUSE_XY, int(args.xy))


def launch_config(ctx, vb) -> dict:
    """The launch options a run used (what its kernel names follow from)."""
    return {"x_lanes": ctx.get_option(vb.VL_OPT_X_LANES), "x_lines_per_wave": ctx.get_option(vb.VL_OPT_X_LANE_LINES),
            "xy_per_plane": ctx.get_option(vb.VL_OPT_FUSE_XY), "sources": ctx.get_option(vb.VL_OPT_FUSE_SOURCES),
            "xcd_order": ctx.get_option(vb.VL_OPT_XCD_ORDER)}


def run_adjoint(args):
    """Reverse-mode gradient of the differentiation workload: one vl_adjoint
    call over --steps steps (default 200) with a checkpoint every 20 steps,
    timed whole (its checkpointed forward, the segment replays and the reverse
    steps).  value = voxel-substrate steps reversed per second."""
    import torch
    from paper_2110_13368_amd import binding as vb
    from paper_2110_13368_amd import workloads as W
    wl = W.differentiation()
    n_steps = args.steps if args.steps_given else wl.steps
    ckpt = args.ckpt_every
    E = wl.voxel_substrates
    print(f"bench: adjoint of {wl.name}: {E} voxel-substrates, {n_steps} steps, checkpoint every {ckpt}",
          file=sys.stderr, flush=True)
    ctx = vb.Context(wl.sims)
    apply_launch_options(ctx, args, vb)  # tuned, then any option forced on the command line
    for k, s in enumerate(wl.sims):
        ctx.set_field(k, s.rho0)
    rng = np.random.default_rng(211013368 + 40)
    grads = [rng.normal(size=s.field_shape) for s in wl.sims]
    g = ctx.to_field_layout([a.astype(np.float32) for a in grads])
    g0 = torch.zeros_like(g)
    ncs = max(sum(s.cells.n * s.n_sub for s in wl.sims), 1)
    dS = torch.zeros(ncs, dtype=torch.float64, device=ctx.device)
    dU = torch.zeros(ncs, dtype=torch.float64, device=ctx.device)
    nvol = sum(s.n_sub for s in wl.sims)

    def call(n):
        nb = vb.vl_adjoint_workspace(ctx.h, n, ckpt)
        ws = call.ws if getattr(call, "ws", None) is not None and call.ws.numel() >= nb else \
            torch.empty(max(nb, 256), dtype=torch.uint8, device=ctx.device)
        call.ws = ws
        torch.cuda.synchronize()
        return vb.vl_adjoint(ctx.h, n, ckpt, ws.data_ptr(), g.data_ptr(), g0.data_ptr(), nvol,
                             dS.data_ptr(), dU.data_ptr())

    # The tuner times forward steps, but the reverse x solve follows the
    # forward's x option and is faster with lanes along the line.  Unless an
    # option was given, the adjoint takes whichever of the tuner's choice and
    # the lanes solve for lines of 65+ voxels (without per-plane x+y) reverses
    # faster, each timed once after a warm-up call (setup, not timed).
    if args.mode == "tuned" and all(getattr(args, a) == "auto" for a in ("x_lanes", "x_lane_lines", "sources", "xy")):
        cands = [{vb.VL_OPT_X_LANES: ctx.get_option(vb.VL_OPT_X_LANES),
                  vb.VL_OPT_FUSE_XY: ctx.get_option(vb.VL_OPT_FUSE_XY)},
                 {vb.VL_OPT_X_LANES: 2, vb.VL_OPT_FUSE_XY: 0}]
        best = None
        for cand in cands:
            for o, v in cand.items():
                ctx.set_option(o, v)
            call(n_steps)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            call(n_steps)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            if best is None or t < best[0]:
                best = (t, cand)
        for o, v in best[1].items():
            ctx.set_option(o, v)
    x_lanes_opt = ctx.get_option(vb.VL_OPT_X_LANES)
    launch = launch_config(ctx, vb)

    call(n_steps)  # allocates the workspace; warm-up
    for _ in range(max(args.warmup, 0) // 20):
        call(n_steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dD, dl = call(n_steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    value = E * n_steps / elapsed
    print(f"bench: adjoint of {n_steps} steps in {elapsed:.4f} s", file=sys.stderr, flush=True)

    ctx.set_profiling(True)
    call(n_steps)
    stats = ctx.kernel_stats()
    ctx.set_profiling(False)
    kinds = {k: v for k, v in stats.items() if v[0] > 0}
    # algorithmic bytes per element and launch: a forward solve reads and
    # writes the field; a replay also writes its raw output; a reverse solve
    # reads the adjoint and the raw output and writes the adjoint; a copy
    # reads and writes one field
    per_elem = {"sweep_x": 8, "sweep_y": 8, "sweep_z": 8, "replay_x": 12, "replay_y": 12, "replay_z": 12,
                "adjoint_x": 12, "adjoint_y": 12, "adjoint_z": 12, "adjoint_copy": 8}
    dom = max((k for k in kinds if k in per_elem), key=lambda k: kinds[k][1])
    launches, total_ms = kinds[dom]
    avg_ms = total_ms / launches
    alg = per_elem[dom] * E
    roofline = {"kernel": dom, "bound": "hbm", "achieved": round(alg / (avg_ms * 1e-3) / 1e9, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(alg / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), "traffic": None,
                "avg_ms": round(avg_ms, 5), "launches": launches, "bytes_per_launch": alg}
    kernels = {k: {"launches": v[0], "avg_ms": round(v[1] / max(v[0], 1), 5), "total_ms": round(v[1], 3)}
               for k, v in kinds.items()}
    ctx.close()
    line = {
        "metric": "adjoint: voxel-substrate steps reversed/s (checkpointed, FP32 with FP64 sums)",
        "value": value, "unit": "voxel-substrate steps reversed/s", "n_gpus": 1, "steps": n_steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / n_steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded generators shaped like the paper's tumour workloads)",
        "config": {"workload": wl.name, "voxel_substrates": E, "grid": list(wl.sims[0].shape),
                   "n_sub": wl.sims[0].n_sub, "cells": int(wl.sims[0].cells.n), "ckpt_every": ckpt,
                   "parallelism": "single-gpu", "x_lanes_min_line": {0: None, 1: 129, 2: 65}[x_lanes_opt],
                   "launch": launch},
        "gradients": {"dD": [float(x) for x in dD], "dlambda": [float(x) for x in dl]},
        "roofline": roofline, "kernels": kernels,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = adjoint_cpu_baseline(wl, grads, args.cpu_seconds)
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--config", default="tumour")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the extra line for the batch of 256 ragged simulations")
    ap.add_argument("--fp64-steps", type=int, default=None)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-copy-reference", action="store_true")
    ap.add_argument("--mode", default="tuned", choices=["tuned", "launches", "persistent"])
    ap.add_argument("--ckpt-every", type=int, default=20)
    ap.add_argument("--x-lanes", default="auto", choices=["auto", "0", "1", "2"],
                    help="force the x solve (after tuning): lanes along lines of 129+ (1) or 65+ (2) voxels, "
                         "0 split solve")
    ap.add_argument("--x-lane-lines", default="auto", choices=["auto", "1", "2", "4", "8", "16"],
                    help="force the x-lines per wave of the lanes-along-the-line solve (after tuning)")
    ap.add_argument("--snapshot-every", type=int, default=0,
                    help="also time the steps with a snapshot of the field to pinned host memory every N steps")
    ap.add_argument("--move-cells-every", type=int, default=0,
                    help="also time steps with the cells moved and re-binned on the device every N steps")
    ap.add_argument("--xy", default="auto", choices=["auto", "0", "1"],
                    help="force x and y solved per z-plane where planes fit in LDS (1) or not (0), after tuning")
    ap.add_argument("--sources", default="auto", choices=["auto", "0", "1", "2"],
                    help="force where cell sources are applied (after tuning): 0 own kernel, 1 in the z sweep, "
                         "2 carried into the next x solve")
    args = ap.parse_args()
    args.steps_given = any(a == "--steps" or a.startswith("--steps=") for a in sys.argv[1:])
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "batched simulations shard by simulation and a single grid by z-slabs, "
              "neither is built here.", file=sys.stderr)
        sys.exit(2)

    if args.config == "adjoint":
        return run_adjoint(args)

    line = run_workload(args, args.config, cpu=not args.no_cpu_baseline, copy_ref=not args.no_copy_reference)
    if args.config == "tumour" and not args.no_batched:
        line["batched"] = run_workload(args, "batched", cpu=False, copy_ref=False, fp64=False)
    print(json.dumps(line), flush=True)


def run_workload(args, config: str, cpu: bool, copy_ref: bool, fp64: bool = True) -> dict:
    """Times one workload (setup untimed, then --steps graph-replayed steps)
    and returns its JSON record."""
    import torch
    from paper_2110_13368_amd import binding as vb

    wl = make_workload(config)
    E = wl.voxel_substrates
    print(f"bench: {wl.name}: {len(wl.sims)} sim(s), {E} voxel-substrates", file=sys.stderr, flush=True)

    precision = vb.VL_F64 if wl.dtype == "f64" else vb.VL_F32
    ctx = vb.Context(wl.sims, precision=precision)
    if precision == vb.VL_F32:
        apply_launch_options(ctx, args, vb)
    mode = "persistent" if ctx.get_option(vb.VL_OPT_STEP_MODE) == vb.VL_MODE_PERSISTENT else "launches"
    fuse_src = {0: "own kernel", 1: "in the z sweep", 2: "carried into the next x solve"}[
        ctx.get_option(vb.VL_OPT_FUSE_SOURCES)] if precision == vb.VL_F32 else "own kernel"
    xcd_ord = bool(ctx.get_option(vb.VL_OPT_XCD_ORDER))
    x_lanes_opt = ctx.get_option(vb.VL_OPT_X_LANES) if precision == vb.VL_F32 else 0
    x_lanes = bool(x_lanes_opt)
    x_lane_lines = ctx.get_option(vb.VL_OPT_X_LANE_LINES) if x_lanes else None
    # what the per-kernel traffic measurements are keyed by, besides the workload
    launch_cfg = {"cell_sources": fuse_src, "x_lanes_along_line": x_lanes, "x_lines_per_wave": x_lane_lines,
                  "xcd_order": xcd_ord}
    for k, s in enumerate(wl.sims):
        ctx.set_field(k, s.rho0)
    elapsed = time_steps(ctx, args.steps, args.warmup)
    value = E * args.steps / elapsed
    esize = 8 if precision == vb.VL_F64 else 4
    field_bytes = E * esize  # a field that fits the Infinity Cache is not an HBM measurement
    # grids one voxel thick (2-D) take two sweeps: their z solve is the identity
    e_thin = sum(sp.n_vox * sp.n_sub for sp in wl.sims if sp.shape[2] == 1) if precision == vb.VL_F32 else 0
    b_alg = 2 * esize * (3 * E - e_thin) / E  # bytes per voxel-substrate-step: the sweeps' read + write
    print(f"bench: {args.steps} steps in {elapsed:.4f} s", file=sys.stderr, flush=True)

    stats = kernel_profile(ctx, args.steps)
    moving = None
    if args.move_cells_every > 0 and precision == vb.VL_F32 and any(s.cells.n > 0 for s in wl.sims):
        t_mv, n_up, t_up = time_moving_cells(ctx, wl, args.steps, args.move_cells_every)
        moving = {"every_steps": args.move_cells_every, "steps": args.steps, "uploads": n_up,
                  "value": E * args.steps / t_mv, "unit": "voxel-substrate updates/s",
                  "ms_per_rebinning": round(1e3 * (t_mv - elapsed) / n_up, 3),
                  "adjoint_tables": False,
                  "note": "cells moved on the device and re-binned (vl_upload_cells_dev) every every_steps steps, "
                          "inside the timed loop; value counts the diffusion updates only; ms_per_rebinning is the "
                          "loop's time beyond the same steps with fixed cells, per upload"}
    snaps = None
    if args.snapshot_every > 0:
        t_sn, n_sn, t_alone, sn_bytes = time_snapshots(ctx, wl, args.steps, args.snapshot_every)
        snaps = {"every_steps": args.snapshot_every, "steps": args.steps, "snapshots": n_sn,
                 "value": E * args.steps / t_sn, "unit": "voxel-substrate updates/s",
                 "bytes_per_snapshot": sn_bytes,
                 "ms_per_snapshot_beyond_steps": round(1e3 * (t_sn - elapsed) / max(n_sn, 1), 3),
                 "transfer_alone_ms": round(1e3 * t_alone, 3),
                 "transfer_alone_GBps": round(sn_bytes / t_alone / 1e9, 1),
                 "note": "every simulation's field copied to pinned host memory every every_steps steps inside "
                         "the timed loop (vl_snapshot); ms_per_snapshot_beyond_steps is the loop's time beyond "
                         "the same steps without snapshots; transfer_alone is one snapshot with nothing to overlap"}
    ctx.close()
    del ctx
    torch.cuda.empty_cache()
    kinds = {k: v for k, v in stats.items() if v[0] > 0}
    dom = max(kinds, key=lambda k: kinds[k][1])
    launches, total_ms = kinds[dom]
    per_step_ms = total_ms / args.steps
    launches_per_step = launches / args.steps
    fused_xy = kinds.get("sweep_xy", (0, 0))[0] > 0
    e_plane = sum(sp.n_vox * sp.n_sub for sp in wl.sims if plane_fits(sp.shape[0], sp.shape[1]))
    if dom == "sweep_xy":
        alg_bytes = 2 * esize * e_plane  # x and y of those volumes: one read and one write
    elif dom in ("sweep_x", "sweep_y") and fused_xy:
        alg_bytes = 2 * esize * (E - e_plane)  # the volumes whose planes do not fit
    elif dom == "sweep_z":
        alg_bytes = 2 * esize * (E - e_thin)  # the volumes more than one voxel thick
    elif dom.startswith("sweep"):
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
        "traffic": measured_traffic(wl.name, dom, launch_cfg),
        "avg_ms": round(per_step_ms / launches_per_step, 5),
        "launches_per_step": launches_per_step,
        "bytes_per_launch": alg_bytes / launches_per_step if alg_bytes else None,
    }
    kernels = {k: {"launches": v[0], "avg_ms": round(v[1] / max(v[0], 1), 5)} for k, v in kinds.items()}

    extra = {}
    if fp64 and precision == vb.VL_F32 and len(wl.sims) == 1:
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
                   "grid": (list(wl.sims[0].shape) if len({sp.shape for sp in wl.sims}) == 1 else "ragged"),
                   "n_sub": wl.sims[0].n_sub, "cells": int(sum(s.cells.n for s in wl.sims)),
                   "dt": wl.sims[0].dt, "parallelism": "single-gpu", "step_mode": mode,
                   "xy_per_plane": fused_xy, "cell_sources": fuse_src, "xcd_order": xcd_ord,
                   "x_lanes_along_line": x_lanes, "x_lanes_min_line": {0: None, 1: 129, 2: 65}[x_lanes_opt],
                   "x_lines_per_wave": x_lane_lines},
        "hbm_effective": {"basis": "B_alg: three sweeps (two on grids one voxel thick) x (read + write) per "
                                   "voxel-substrate-step; with x and y solved per z-plane the step moves less "
                                   "than B_alg",
                          "field_bytes": field_bytes,
                          "fits_infinity_cache": field_bytes <= INFINITY_CACHE_BYTES,
                          "bytes_per_update": b_alg,
                          "bytes_moved_per_update": (b_alg - 2 * esize * e_plane / E) if fused_xy else b_alg,
                          "GBps": round(b_alg * value / 1e9, 1),
                          "frac_of_peak": round(b_alg * value / 1e9 / HBM_PEAK_GBS, 4)},
        "roofline": roofline,
        "kernels": kernels,
    }
    line.update(extra)
    if moving is not None:
        line["moving_cells"] = moving
    if snaps is not None:
        line["snapshots"] = snaps
    if copy_ref:
        line["copy_reference"] = [copy_reference(128 << 20), copy_reference(2 << 30, reps=5)]
    if cpu:
        line["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds)
    return line


if __name__ == "__main__":
    main()
