"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle on
the same seeded inputs.

Tolerances: the plain FP64 path must agree to 1e-12 relative; the FP32 path
to 1e-5 relative in both the max norm and the L2 norm per substrate, the
accuracy target set for FP32 storage and sweeps over 100 steps.  The paper's
own Method 2 (section "Methods of Validation") is this voxel-by-voxel
cross-check of the GPU field against the CPU field.
"""
import dataclasses

import numpy as np
import pytest

import oracle as O
from paper_2110_13368_amd import binding as vb
from paper_2110_13368_amd import workloads as W
from tests.gpu_helpers import assert_close, rel_errs, run_gpu, run_oracle, subset

pytestmark = pytest.mark.gpu

DECAYS = [(vb.VL_DECAY_ONCE, O.DECAY_ONCE), (vb.VL_DECAY_THIRDS, O.DECAY_THIRDS)]


def _spec(shape, n_sub, bc, n_cells, dtype, seed, layout="uniform", h=(20.0, 20.0, 20.0)):
    rng = np.random.default_rng(W.SEED_BASE + 500 + seed)
    spec = W.make_sim(rng, shape, h, n_sub, dtype=dtype, bc=bc, n_cells=n_cells, cell_layout=layout,
                      sigma=0.25 * min(n * d for n, d in zip(shape, h)))
    if n_cells >= 3:
        spec.cells.pos[1] = spec.cells.pos[0]          # two cells in one voxel
        spec.cells.pos[2] = np.array(spec.lo) - 3.0    # one cell outside the grid
    return spec


# --------------------------------------------------------------------------
# plain FP64 path

def test_fp64_plain_configuration():
    """50^3 voxels, Dirichlet 38 on every face, 1000 uptake-only cells, 100 steps."""
    wl = W.plain_fp64()
    spec = wl.sims[0]
    (got,), _ = run_gpu([spec], wl.steps, precision=vb.VL_F64)
    want = run_oracle(spec, wl.steps)
    assert_close(got, want, 1e-12, "plain 50^3")
    assert np.max(got) <= 38.0 + 1e-9 and np.min(got) > 0.0


@pytest.mark.parametrize("shape", [(5, 4, 3), (1, 1, 6), (6, 1, 1), (1, 5, 1), (2, 3, 4), (1, 1, 1), (9, 8, 7)])
@pytest.mark.parametrize("bc", ["neumann", "dirichlet", "mixed"])
@pytest.mark.parametrize("decay", DECAYS)
def test_fp64_tiny_grids(shape, bc, decay):
    spec = _spec(shape, 2, bc, 9, "f64", hash((shape, bc)) % 1000)
    (got,), n_out = run_gpu([spec], 3, precision=vb.VL_F64, decay=decay[0])
    want = run_oracle(spec, 3, decay[1])
    assert n_out == [1]
    assert_close(got, want, 1e-12, f"fp64 {shape} {bc}")


# --------------------------------------------------------------------------
# FP32 path: line lengths around every split and capacity boundary

LINE_LENGTHS = [1, 2, 3, 4, 5, 63, 64, 65, 66, 127, 128, 129, 130, 131, 193, 194, 199, 200, 201, 202, 203, 257, 258,
                321, 401, 513]
# x solve with lanes along the line: around every voxels-per-lane boundary
X_LANE_LENGTHS = [1, 2, 3, 31, 63, 64, 65, 66, 127, 128, 129, 191, 192, 193, 200, 255, 256, 257,
                  319, 320, 321, 383, 384, 385, 400, 447, 448, 449, 511, 512, 513]


@pytest.mark.parametrize("n", LINE_LENGTHS)
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_fp32_line_lengths(n, axis):
    shape = [3, 5, 2]
    shape[axis] = n
    spec = _spec(tuple(shape), 2, "mixed", 12, "f32", n * 3 + axis)
    (got,), _ = run_gpu([spec], 20)
    want = run_oracle(spec, 20)
    assert_close(got, want, 1e-5, f"fp32 n={n} axis={axis}")


@pytest.mark.parametrize("n", X_LANE_LENGTHS)
@pytest.mark.parametrize("bc", ["mixed", "dirichlet"])
@pytest.mark.parametrize("x_lanes", [1, 2])
def test_fp32_x_lanes_line_lengths(n, bc, x_lanes):
    # x_lanes 1: lanes along lines of 129+ voxels, 2: of 65+ voxels
    spec = _spec((n, 5, 3), 2, bc, 12, "f32", n * 7 + len(bc))
    (got,), _ = run_gpu([spec], 20, x_lanes=x_lanes)
    want = run_oracle(spec, 20)
    assert_close(got, want, 1e-5, f"x lanes {x_lanes} n={n} {bc}")


@pytest.mark.parametrize("x_lanes", [0, 1, 2])
@pytest.mark.parametrize("decay", DECAYS)
@pytest.mark.parametrize("bc", ["neumann", "dirichlet", "mixed"])
def test_fp32_boundary_mixes_and_decay(bc, decay, x_lanes):
    spec = _spec((33, 70, 19), 3, bc, 400, "f32", 11, layout="gaussian")
    (got,), _ = run_gpu([spec], 30, decay=decay[0], x_lanes=x_lanes)
    want = run_oracle(spec, 30, decay[1])
    assert_close(got, want, 1e-5, f"fp32 {bc}")


# --------------------------------------------------------------------------
# two-dimensional grids and unequal voxel edges.  A 2-D simulation is a grid
# one voxel thick with no z faces: its z-lines hold one voxel each, so the z
# solve reduces to the identity (decay once) or to the z share of the decay
# (decay in thirds), and the step is the x and y solves of the 2-D method.

def _planar(shape, bc, n_cells, seed, h=(20.0, 20.0, 20.0)):
    rng = np.random.default_rng(W.SEED_BASE + 700 + seed)
    spec = W.make_sim(rng, shape, h, 2, dtype="f32", bc=bc, n_cells=n_cells, cell_layout="disc",
                      sigma=0.25 * min(shape[0] * h[0], shape[1] * h[1]))
    spec.bc_kind[:, 4:] = 0  # a 2-D grid has no z faces
    spec.bc_value[:, 4:] = 0.0
    if n_cells >= 3:
        spec.cells.pos[1] = spec.cells.pos[0]
        spec.cells.pos[2] = np.array(spec.lo) - 3.0
    return spec


PLANAR = [((300, 250, 1), "mixed"), ((513, 64, 1), "dirichlet"), ((64, 513, 1), "mixed"),
          ((1, 300, 1), "neumann"), ((130, 1, 1), "mixed"), ((200, 199, 1), "neumann")]


@pytest.mark.parametrize("x_lanes", [0, 1, 2])
@pytest.mark.parametrize("decay", DECAYS)
@pytest.mark.parametrize("shape,bc", PLANAR)
def test_fp32_two_dimensional(shape, bc, decay, x_lanes):
    spec = _planar(shape, bc, 200, sum(shape) + len(bc), h=(10.0, 15.0, 10.0))
    (got,), n_out = run_gpu([spec], 50, decay=decay[0], x_lanes=x_lanes)
    assert n_out == [1]
    assert_close(got, run_oracle(spec, 50, decay[1]), 1e-5, f"2-D {shape} {bc}")


@pytest.mark.parametrize("sources_mode", [0, 1, 2])
def test_fp32_two_dimensional_in_a_batch_with_3d(sources_mode):
    """2-D and 3-D simulations in one ragged batch, with every placement of
    the cell sources (own kernel, in the z solve, carried into the next x)."""
    specs = [_planar((260, 180, 1), "mixed", 400, 1), _spec((70, 40, 21), 2, "mixed", 300, "f32", 5),
             _planar((129, 7, 1), "dirichlet", 30, 2), _planar((40, 90, 1), "neumann", 80, 3)]
    fields, _ = run_gpu(specs, 40, x_lanes=1, sources_mode=sources_mode)
    for k, spec in enumerate(specs):
        assert_close(fields[k], run_oracle(spec, 40), 1e-5, f"batch sim {k} {spec.shape}")


@pytest.mark.parametrize("x_lanes", [0, 1, 2])
@pytest.mark.parametrize("decay", DECAYS)
def test_fp32_unequal_voxel_edges(decay, x_lanes):
    """Voxels of 8 x 20 x 35 um: a different coupling dt D / h^2 on each axis."""
    spec = _spec((140, 70, 33), 2, "mixed", 500, "f32", 91, layout="gaussian", h=(8.0, 20.0, 35.0))
    (got,), _ = run_gpu([spec], 40, decay=decay[0], x_lanes=x_lanes)
    assert_close(got, run_oracle(spec, 40, decay[1]), 1e-5, "unequal edges")


@pytest.mark.parametrize("decay", DECAYS)
def test_fp64_two_dimensional_and_unequal_edges(decay):
    specs = [_planar((90, 70, 1), "mixed", 60, 4, h=(10.0, 30.0, 5.0)),
             _spec((20, 15, 12), 2, "dirichlet", 40, "f64", 17, h=(5.0, 12.0, 40.0))]
    specs[0] = dataclasses.replace(specs[0], rho0=specs[0].rho0.astype(np.float64))
    fields, _ = run_gpu(specs, 10, precision=vb.VL_F64, decay=decay[0])
    for k, spec in enumerate(specs):
        assert_close(fields[k], run_oracle(spec, 10, decay[1]), 1e-12, f"fp64 sim {k} {spec.shape}")


@pytest.mark.parametrize("x_lanes", [0, 1, 2])
def test_fp32_single_large_scaled_100_steps(x_lanes):
    """The single large simulation at a quarter of its edge (50^3 x 4, Gaussian
    ball of cells), 100 steps."""
    wl = W.single_large(scale=0.25)
    spec = wl.sims[0]
    (got,), _ = run_gpu([spec], 100, x_lanes=x_lanes)
    want = run_oracle(spec, 100)
    errs = assert_close(got, want, 1e-5, "single-large/4")
    print("single-large/4 errors per substrate (max, L2):", errs)


@pytest.mark.parametrize("x_lanes", [0, 1, 2])
def test_fp32_batched_ragged(x_lanes):
    wl = W.batched(n_sims=6, edge_range=(7, 70), cells_range=(50, 800))
    fields, n_out = run_gpu(wl.sims, 40, x_lanes=x_lanes)
    assert n_out == [0] * 6
    for k, spec in enumerate(wl.sims):
        assert_close(fields[k], run_oracle(spec, 40), 1e-5, f"batch sim {k} {spec.shape}")


def test_fp32_x_lanes_long_lines_100_steps():
    """Long x-lines (400 voxels: eight per lane), 100 steps, Dirichlet and
    zero-flux faces mixed."""
    spec = _spec((400, 9, 7), 2, "mixed", 300, "f32", 4242)
    (got,), _ = run_gpu([spec], 100, x_lanes=1)
    assert_close(got, run_oracle(spec, 100), 1e-5, "x lanes 400")


def test_fp32_x_lanes_lines_per_wave():
    """The x-lines each wave takes (VL_OPT_X_LANE_LINES) change only the
    launch shape: fields are bitwise equal for every value, on a batch whose
    volumes have line counts that leave partial tiles and different voxels
    per lane."""
    specs = [_spec((200, 13, 7), 2, "mixed", 150, "f32", 501),
             _spec((300, 5, 3), 1, "dirichlet", 40, "f32", 502),
             _spec((140, 3, 2), 3, "neumann", 20, "f32", 503)]
    ref, _ = run_gpu(specs, 8, x_lanes=1, x_lane_lines=16)
    for k, spec in enumerate(specs):
        assert_close(ref[k], run_oracle(spec, 8), 1e-5, f"x lanes lpw 16 sim {k}")
    for lpw in (1, 2, 4, 8):
        got, _ = run_gpu(specs, 8, x_lanes=1, x_lane_lines=lpw)
        for k in range(len(specs)):
            assert np.array_equal(got[k], ref[k]), f"lines per wave {lpw}, sim {k}"


def test_fp64_batched_ragged():
    wl = W.batched(n_sims=4, edge_range=(5, 40), cells_range=(20, 300), dtype="f64")
    fields, _ = run_gpu(wl.sims, 10, precision=vb.VL_F64)
    for k, spec in enumerate(wl.sims):
        assert_close(fields[k], run_oracle(spec, 10), 1e-12, f"fp64 batch sim {k}")


def test_fp32_many_cells_in_one_voxel():
    spec = _spec((16, 16, 16), 2, "neumann", 0, "f32", 5)
    n = 300
    rng = np.random.default_rng(9)
    pos = np.tile(np.array([[1.0, 2.0, 3.0]]), (n, 1))
    V, S, U, rs = W.tumour_rates(rng, n, 2)
    spec.cells = W.Cells(pos, V, S, U, rs)
    (got,), _ = run_gpu([spec], 5)
    assert_close(got, run_oracle(spec, 5), 1e-5, "300 cells in one voxel")


@pytest.mark.parametrize("sources_mode", [1, 2])
def test_fp32_over_a_million_cells(sources_mode):
    """1.2e6 cells, about 50 per voxel of a 40 x 30 x 20 grid: the binning's
    radix-sort histograms (16 digits per block of 2048 keys) pass the 8192
    entries that the scan takes per round, so the scan runs more than one
    round; sources in the z sweep and carried into the x solve."""
    spec = _spec((40, 30, 20), 2, "mixed", 1_200_000, "f32", 41)
    (got,), n_out = run_gpu([spec], 3, x_lanes=1, sources_mode=sources_mode)
    assert n_out == [1]  # the one cell placed outside the grid
    assert_close(got, run_oracle(spec, 3), 1e-5, f"1.2e6 cells, sources mode {sources_mode}")


def test_all_cells_outside():
    spec = _spec((8, 8, 8), 1, "mixed", 5, "f32", 6)
    spec.cells.pos[:] = np.array(spec.lo) - 10.0
    (got,), n_out = run_gpu([spec], 4)
    assert n_out == [5]
    assert_close(got, run_oracle(spec, 4), 1e-5, "cells outside")


# --------------------------------------------------------------------------
# determinism, graph replay, diagnostics

def test_bitwise_repeatable_and_graph_equals_direct():
    spec = _spec((40, 37, 29), 2, "mixed", 500, "f32", 21)
    (a,), _ = run_gpu([spec], 25)
    (b,), _ = run_gpu([spec], 25)
    (c,), _ = run_gpu([spec], 25, profiling=True)  # direct launches with events
    assert np.array_equal(a, b)
    assert np.array_equal(a, c)


def test_fused_sources_equal_standalone_kernel():
    """Sources applied inside the z sweep and by the separate kernel give the
    same bits (same FP32 arithmetic, each voxel touched once)."""
    wl = W.batched(n_sims=4, edge_range=(9, 90), cells_range=(200, 3000))
    spec = _spec((61, 47, 83), 3, "mixed", 4000, "f32", 51, layout="gaussian")
    for specs in (wl.sims, [spec]):
        fused, _ = run_gpu(specs, 12)
        alone, _ = run_gpu(specs, 12, fuse=False)
        for a, b in zip(fused, alone):
            assert np.array_equal(a, b)
    assert_close(fused[0], run_oracle(spec, 12), 1e-5, "fused sources")


def _run_mode(specs, steps, mode, grid=0):
    ctx = vb.Context(specs)
    try:
        ctx.set_option(vb.VL_OPT_STEP_MODE, mode)
        ctx.set_option(vb.VL_OPT_PERSISTENT_GRID, grid)
        ctx.step(steps)
        ctx.sync()
        return [ctx.get_field(k) for k in range(len(specs))]
    finally:
        ctx.close()


ONE_LAUNCH_OFF = ("the one-launch step is switched off: its first GPU runs did not finish "
                  "(grid = all resident workgroups), also with every wait bounded in time; "
                  "the cause is not yet shown, so the case stays off the GPU")


@pytest.mark.skip(reason=ONE_LAUNCH_OFF)
@pytest.mark.parametrize("grid", [0, 1, 7, 300])
def test_one_launch_step_equals_per_sweep_launches(grid):
    """The one-launch step (queue over all tiles, per-volume waits) gives the
    same bits as one launch per sweep, for any number of workgroups."""
    wl = W.batched(n_sims=5, edge_range=(9, 75), cells_range=(100, 2000))
    a = _run_mode(wl.sims, 6, vb.VL_MODE_LAUNCHES)
    b = _run_mode(wl.sims, 6, vb.VL_MODE_PERSISTENT, grid)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    assert_close(b[2].astype(np.float64), run_oracle(wl.sims[2], 6), 1e-5, "one-launch batch")


@pytest.mark.skip(reason=ONE_LAUNCH_OFF)
def test_one_launch_step_long_lines():
    spec = _spec((130, 66, 201), 2, "mixed", 2000, "f32", 61, layout="gaussian")
    a = _run_mode([spec], 4, vb.VL_MODE_LAUNCHES)
    b = _run_mode([spec], 4, vb.VL_MODE_PERSISTENT)
    assert np.array_equal(a[0], b[0])


def test_tuner_picks_a_mode_and_caches(tmp_path):
    wl = W.batched(n_sims=8, edge_range=(20, 60), cells_range=(100, 500))
    cache = str(tmp_path / "tune.txt")
    ctx = vb.Context(wl.sims)
    try:
        ctx.tune(cache)
        xcd = ctx.get_option(vb.VL_OPT_XCD_ORDER)
        fuse = ctx.get_option(vb.VL_OPT_FUSE_SOURCES)
        assert ctx.get_option(vb.VL_OPT_STEP_MODE) == vb.VL_MODE_LAUNCHES
        fxy = ctx.get_option(vb.VL_OPT_FUSE_XY)
        xl = ctx.get_option(vb.VL_OPT_X_LANES)
        lpw = ctx.get_option(vb.VL_OPT_X_LANE_LINES)
        words = open(cache).read().split()
        assert len(words) == 8 and int(words[3]) == xcd and int(words[4]) == fuse and int(words[5]) == fxy
        assert int(words[6]) == xl and int(words[7]) == lpw
        # a second context with the same shapes reads the choice back
        ctx2 = vb.Context(wl.sims)
        ctx2.set_option(vb.VL_OPT_XCD_ORDER, 1 - xcd)
        ctx2.set_option(vb.VL_OPT_FUSE_SOURCES, (fuse + 1) % 3)
        ctx2.set_option(vb.VL_OPT_FUSE_XY, 1 - fxy)
        ctx2.set_option(vb.VL_OPT_X_LANE_LINES, 24 - lpw)  # 16 <-> 8
        ctx2.tune(cache)
        assert ctx2.get_option(vb.VL_OPT_XCD_ORDER) == xcd
        assert ctx2.get_option(vb.VL_OPT_FUSE_SOURCES) == fuse
        assert ctx2.get_option(vb.VL_OPT_FUSE_XY) == fxy
        assert ctx2.get_option(vb.VL_OPT_X_LANES) == xl
        assert ctx2.get_option(vb.VL_OPT_X_LANE_LINES) == lpw
        assert len(open(cache).read().split()) == 8
        # the tuned context still computes the step correctly
        for k, s in enumerate(wl.sims):
            ctx2.set_field(k, s.rho0)
        ctx2.step(3)
        assert_close(ctx2.get_field(1).astype(np.float64), run_oracle(wl.sims[1], 3), 1e-5, "tuned")
        ctx2.close()
    finally:
        ctx.close()


@pytest.mark.skip(reason=ONE_LAUNCH_OFF)
def test_one_launch_wait_limit_fails_loudly_not_hangs():
    """With a zero wait limit a tile that has to wait gives up at once: the
    step ends and vl_sync reports it (or nothing had to wait).  The next steps
    with the default limit are correct again."""
    wl = W.batched(n_sims=6, edge_range=(40, 90), cells_range=(100, 500))
    ctx = vb.Context(wl.sims)
    try:
        ctx.set_option(vb.VL_OPT_STEP_MODE, vb.VL_MODE_PERSISTENT)
        ctx.set_option(vb.VL_OPT_WAIT_LIMIT_US, 0)
        ctx.step(3)
        try:
            ctx.sync()
        except vb.VoxlodError as e:
            assert e.code == vb.VL_E_STATE
        ctx.set_option(vb.VL_OPT_WAIT_LIMIT_US, 2000000)
        for k, s in enumerate(wl.sims):
            ctx.set_field(k, s.rho0)
        ctx.step(3)
        ctx.sync()
        assert_close(ctx.get_field(0).astype(np.float64), run_oracle(wl.sims[0], 3), 1e-5, "after limit")
    finally:
        ctx.close()


def test_batch_of_one_equals_single():
    wl = W.batched(n_sims=3, edge_range=(10, 40), cells_range=(50, 200))
    fields, _ = run_gpu(wl.sims, 7)
    (alone,), _ = run_gpu([wl.sims[1]], 7)
    assert np.array_equal(fields[1], alone)


@pytest.mark.parametrize("precision", [vb.VL_F32, vb.VL_F64])
def test_mass_and_nonfinite(precision):
    spec = _spec((30, 20, 10), 3, "neumann", 0, "f32" if precision == vb.VL_F32 else "f64", 31)
    spec.lam[:] = 0.0
    ctx = vb.Context([spec], precision=precision)
    try:
        m0 = ctx.mass(0)
        np.testing.assert_allclose(m0, spec.rho0.astype(np.float64).reshape(3, -1).sum(axis=1), rtol=1e-12)
        ctx.step(50)
        m1 = ctx.mass(0)
        field = ctx.get_field(0).astype(np.float64)
        np.testing.assert_allclose(m1, field.reshape(3, -1).sum(axis=1), rtol=1e-12)
        # zero flux and no decay: mass is conserved up to the storage precision
        tol = 2e-5 if precision == vb.VL_F32 else 1e-12
        np.testing.assert_allclose(m1, m0, rtol=tol)
        assert ctx.check_finite() == 0
        bad = field.copy()
        bad[1, 3, 4, 5] = np.nan
        bad[2, 0, 0, 0] = np.inf
        ctx.set_field(0, bad)
        assert ctx.check_finite() == 2
    finally:
        ctx.close()


def test_device_field_io_and_aos():
    spec = _spec((11, 9, 7), 3, "mixed", 30, "f32", 41)
    ctx = vb.Context([spec])
    try:
        import torch
        view = ctx.field_view(0)
        assert torch.equal(view.cpu(), torch.from_numpy(spec.rho0))
        aos = np.ascontiguousarray(np.moveaxis(spec.rho0, 0, -1))
        out = np.empty_like(aos)
        vb.vl_get_field(ctx.h, 0, out.ctypes.data, False, vb.VL_AOS)
        assert np.array_equal(out, aos)
        dev = torch.from_numpy(aos).cuda()
        ctx.step(2)
        vb.vl_set_field(ctx.h, 0, dev.data_ptr(), True, vb.VL_AOS)
        assert np.array_equal(ctx.get_field(0), spec.rho0)
    finally:
        ctx.close()


# --------------------------------------------------------------------------
# x and y of one z-plane per workgroup (planes that fit in LDS) against the
# separate x and y sweeps: the same operations, so bitwise the same field.

def _run_xy(specs, steps, fuse_xy, decay=vb.VL_DECAY_ONCE):
    ctx = vb.Context(specs, decay_split=decay, device="cuda:0")
    try:
        ctx.set_option(vb.VL_OPT_FUSE_XY, fuse_xy)
        ctx.set_option(vb.VL_OPT_X_LANES, 0)  # the plane kernel's x solve is the split one
        ctx.set_profiling(True)
        ctx.step(steps)
        ctx.sync()
        stats = ctx.kernel_stats()
        return [ctx.get_field(k) for k in range(len(specs))], stats
    finally:
        ctx.close()


@pytest.mark.parametrize("decay", [vb.VL_DECAY_ONCE, vb.VL_DECAY_THIRDS])
@pytest.mark.parametrize("shape,bc", [((199, 199, 5), "mixed"), ((199, 57, 9), "dirichlet"), ((64, 130, 6), "mixed"),
                                      ((1, 40, 7), "mixed"), ((45, 1, 3), "dirichlet"), ((3, 2, 4), "mixed"),
                                      ((2, 3, 1), "dirichlet"), ((129, 65, 2), "neumann")])
def test_xy_plane_kernel_equals_separate_sweeps(shape, bc, decay):
    spec = _spec(shape, 2, bc, 300, "f32", 71 + shape[0])
    a, sa = _run_xy([spec], 3, 1, decay)
    b, sb = _run_xy([spec], 3, 0, decay)
    print(f"{shape} {bc}: plane launches {sa['sweep_xy'][0]}, separate x {sb['sweep_x'][0]}", flush=True)
    assert sa["sweep_xy"][0] == 3 and sa["sweep_x"][0] == 0 and sb["sweep_xy"][0] == 0
    assert np.array_equal(a[0], b[0])


def test_xy_plane_kernel_mixed_batch():
    # planes that fit (several LDS classes) next to one that does not
    specs = [_spec(sh, 1 + k % 2, "mixed", 200, "f32", 90 + k)
             for k, sh in enumerate([(30, 20, 5), (120, 100, 4), (201, 199, 3), (260, 210, 2), (7, 90, 6)])]
    a, sa = _run_xy(specs, 2, 1)
    b, _ = _run_xy(specs, 2, 0)
    assert sa["sweep_xy"][0] > 0 and sa["sweep_x"][0] > 0  # the 260 x 210 plane keeps x and y
    for k in range(len(specs)):
        assert np.array_equal(a[k], b[k]), k
    assert_close(a[2].astype(np.float64), run_oracle(specs[2], 2), 1e-5, "xy batch")
