"""FP32 parity at the configurations' full sizes and step counts, in the launch
configuration the benchmark times (the autotuner's choice on the same
buffers, as ``bench.py`` runs it), against the FP64 oracle.

The paper's Method 2 (section "Methods of Validation for Data Integrity") is
exactly this check: the whole GPU field against the CPU field, voxel by
voxel.  Per substrate the bound is 1e-5 on both the max-norm error
max|x - y| / max|y| and the L2 error ||x - y|| / ||y||; the pointwise relative
error max |x - y| / |y| over voxels with |y| > 1e-6 max|y| is reported beside
them.  Substrates do not interact, so the oracle runs on the substrates a test
names (``subset``) while the GPU runs the whole configuration.

  * single large simulation, 200^3 x 4, 1e5 cells: 100 steps, every substrate,
    once tuned and once with the lanes-along-the-line x solve and the sources
    carried into the next x solve forced; and its full 1000 steps on the
    substrates with the smallest and the largest D;
  * tumour scale, 400^3 x 8, 1e6 cells: 100 steps, the substrates with the
    smallest and the largest D and the one with the largest lambda;
  * the batch of 256 ragged simulations x 2: 200 steps, every simulation
    (in eight groups of 32);
  * the differentiation workload lives in test_adjoint_gpu.py.
"""
from __future__ import annotations

import numpy as np
import pytest

from paper_2110_13368_amd import binding as vb
from paper_2110_13368_amd import workloads as W
from tests.gpu_helpers import run_oracle, subset

pytestmark = pytest.mark.gpu

TOL = 1e-5


def errors(got, want):
    """Per substrate: max-norm, L2 and pointwise relative errors."""
    out = []
    for s in range(want.shape[0]):
        d = np.abs(got[s] - want[s])
        ay = np.abs(want[s])
        big = ay > 1e-6 * ay.max()
        out.append({"max": float(d.max() / ay.max()),
                    "l2": float(np.linalg.norm(d) / np.linalg.norm(want[s])),
                    "pointwise": float(np.max(d[big] / ay[big])) if big.any() else 0.0})
    return out


def check(got, want, what):
    errs = errors(got, want)
    for s, e in enumerate(errs):
        print(f"{what} substrate {s}: max {e['max']:.3e}  L2 {e['l2']:.3e}  pointwise {e['pointwise']:.3e}",
              flush=True)
        assert e["max"] <= TOL and e["l2"] <= TOL, (what, s, e)
    return errs


def options(ctx):
    names = {"x_lanes": vb.VL_OPT_X_LANES, "lines_per_wave": vb.VL_OPT_X_LANE_LINES,
             "sources": vb.VL_OPT_FUSE_SOURCES, "xcd_order": vb.VL_OPT_XCD_ORDER, "xy_per_plane": vb.VL_OPT_FUSE_XY,
             "step_mode": vb.VL_OPT_STEP_MODE}
    return {k: ctx.get_option(v) for k, v in names.items()}


def run_bench_shape(specs, steps, force=None):
    """The benchmark's sequence: bind, tune on the bound buffers, set the
    initial field again, then the steps (graph-replayed); returns the fields
    (float64) and the options the run used."""
    ctx = vb.Context(specs, device="cuda:0")
    try:
        ctx.tune(None)
        for opt, val in (force or {}).items():
            ctx.set_option(opt, val)
        for k, s in enumerate(specs):
            ctx.set_field(k, s.rho0)
        ctx.step(steps)
        ctx.sync()
        opts = options(ctx)
        print(f"launch configuration: {opts}", flush=True)
        return [ctx.get_field(k) for k in range(len(specs))], opts
    finally:
        ctx.close()


# --------------------------------------------------------------------------
# single large simulation: 200^3 x 4, 100 steps, every substrate

@pytest.fixture(scope="module")
def single_large():
    wl = W.single_large()
    spec = wl.sims[0]
    return spec, run_oracle(spec, 100)


@pytest.mark.parametrize("forced", ["tuned", "lanes+carried"])
def test_single_large_100_steps_every_substrate(single_large, forced):
    spec, want = single_large
    force = None if forced == "tuned" else {vb.VL_OPT_X_LANES: 1, vb.VL_OPT_FUSE_SOURCES: 2}
    (got,), opts = run_bench_shape([spec], 100, force)
    if force:
        assert opts["x_lanes"] == 1 and opts["sources"] == 2
    check(got.astype(np.float64), want, f"200^3x4 {forced}")


def test_single_large_1000_steps(single_large):
    """The configuration's own run length: 1000 steps of 200^3 x 4, checked on
    the substrates with the smallest and the largest D (the oracle on those
    two only; substrates do not interact)."""
    spec, _ = single_large
    (got,), _ = run_bench_shape([spec], 1000)
    for s in (int(np.argmin(spec.D)), int(np.argmax(spec.D))):
        print(f"200^3x4 1000 steps: substrate {s}, D {spec.D[s]:.4g}, lambda {spec.lam[s]:.4g}", flush=True)
        want = run_oracle(subset(spec, [s]), 1000)
        check(got[s:s + 1].astype(np.float64), want, f"200^3x4 1000 steps substrate {s}")


# --------------------------------------------------------------------------
# tumour scale: 400^3 x 8, 100 steps; GPU once, oracle per sampled substrate

@pytest.fixture(scope="module")
def tumour_gpu():
    wl = W.tumour_scale()
    spec = wl.sims[0]
    (got,), opts = run_bench_shape([spec], 100)
    return spec, got, opts


@pytest.mark.parametrize("which", ["smallest D", "largest D", "largest lambda"])
def test_tumour_scale_100_steps(tumour_gpu, which):
    spec, got, _ = tumour_gpu
    if which == "smallest D":
        s = int(np.argmin(spec.D))
    elif which == "largest D":
        s = int(np.argmax(spec.D))
    else:
        s = int(np.argmax(spec.lam))
    print(f"400^3x8 {which}: substrate {s}, D {spec.D[s]:.4g}, lambda {spec.lam[s]:.4g}", flush=True)
    want = run_oracle(subset(spec, [s]), 100)
    check(got[s:s + 1].astype(np.float64), want, f"400^3x8 substrate {s}")


# --------------------------------------------------------------------------
# the batch: 256 ragged simulations x 2, 200 steps; GPU once, the oracle on
# every simulation in groups

@pytest.fixture(scope="module")
def batch_gpu():
    wl = W.batched()
    fields, opts = run_bench_shape(wl.sims, wl.steps)
    return wl, fields


@pytest.mark.parametrize("group", range(8))
def test_batched_200_steps_every_simulation(batch_gpu, group):
    wl, fields = batch_gpu
    ks = range(32 * group, 32 * group + 32)
    for k in ks:
        spec = wl.sims[k]
        check(fields[k].astype(np.float64), run_oracle(spec, wl.steps), f"batch sim {k} {spec.shape}")


def test_batched_covers_every_class():
    """The groups above cover the smallest and the largest simulation and every
    capacity class of every axis (lines of 32-65 voxels and of 66-128)."""
    wl = W.batched()
    sizes = [int(np.prod(s.shape)) for s in wl.sims]
    assert min(sizes) < 32 ** 3 * 4 and max(sizes) > 120 ** 3 * 0.8
    for axis in range(3):
        edges = {s.shape[axis] for s in wl.sims}
        assert min(edges) <= 65 < max(edges), axis
