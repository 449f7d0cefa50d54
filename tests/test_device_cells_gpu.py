"""Cell upload from device arrays (vl_upload_cells_dev): cells that move
between steps are re-binned on the device without a host copy.

The upload runs the same binning as the host entry point (voxel of each cell
in FP64, stable sort by voxel, composites of each occupied voxel in FP64), so
fields after uploads from the host and from the device are bitwise equal;
with the cells moving every few steps both are checked against the FP64
oracle given the same sequence of uploads (Eq. 1 with the agents' positions
changing between diffusion steps, as in the paper's hybrid model).
"""
import numpy as np
import pytest

import oracle as O
from paper_2110_13368_amd import binding as vb
from paper_2110_13368_amd import workloads as W
from tests.gpu_helpers import assert_close

pytestmark = pytest.mark.gpu


def _spec(shape, n_sub, bc, n_cells, seed):
    rng = np.random.default_rng(W.SEED_BASE + 1200 + seed)
    h = (20.0, 20.0, 20.0)
    return W.make_sim(rng, shape, h, n_sub, dtype="f32", bc=bc, n_cells=n_cells, cell_layout="gaussian",
                      sigma=0.25 * min(n * d for n, d in zip(shape, h)))


def _moves(spec, n_moves, seed):
    """Cell positions after each move: a seeded random walk of a few voxels,
    some cells leaving the grid, drawn up front so that every path sees the
    same positions."""
    rng = np.random.default_rng(seed)
    pos = spec.cells.pos.copy()
    out = []
    for _ in range(n_moves):
        pos = pos + rng.normal(scale=1.5 * spec.h[0], size=pos.shape)
        out.append(pos.copy())
    return out


def _device(ctx, a):
    return ctx.torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(ctx.device)


def _run(specs, moves, every, n_steps, from_device, x_lanes, count=True, sources=None):
    ctx = vb.Context(specs, device="cuda:0")
    try:
        ctx.set_option(vb.VL_OPT_X_LANES, x_lanes)
        if sources is not None:
            ctx.set_option(vb.VL_OPT_FUSE_SOURCES, sources)
        for k, s in enumerate(specs):
            ctx.set_field(k, s.rho0)
        outs = []
        done = 0
        for m in range(len(moves[0]) + 1):
            if m > 0:
                for k, s in enumerate(specs):
                    c = s.cells
                    if from_device:
                        n_out = ctx.upload_cells_device(k, _device(ctx, moves[k][m - 1]), _device(ctx, c.V),
                                                        _device(ctx, c.S), _device(ctx, c.U),
                                                        _device(ctx, c.rho_star), count_out=count)
                    else:
                        n_out = ctx.upload_cells(k, W.Cells(pos=moves[k][m - 1], V=c.V, S=c.S, U=c.U,
                                                            rho_star=c.rho_star))
                    outs.append(n_out)
            take = min(every, n_steps - done)
            ctx.step(take)
            done += take
        ctx.sync()
        return [ctx.get_field(k).astype(np.float64) for k in range(len(specs))], outs
    finally:
        ctx.close()


def _oracle(spec, moves, every, n_steps):
    sim = O.from_spec(spec)
    done = 0
    for m in range(len(moves) + 1):
        if m > 0:
            c = spec.cells
            sim.upload_cells(moves[m - 1], c.V, c.S, c.U, c.rho_star)
        take = min(every, n_steps - done)
        sim.step(take)
        done += take
    return sim.get_field()


@pytest.mark.parametrize("x_lanes", [0, 1])
def test_moving_cells_uploaded_from_device(x_lanes):
    specs = [_spec((140, 12, 9), 2, "mixed", 300, 1), _spec((33, 20, 17), 1, "neumann", 150, 2)]
    every, n_moves = 3, 3
    moves = [_moves(s, n_moves, 77 + k) for k, s in enumerate(specs)]
    n_steps = every * (n_moves + 1)
    fd, out_d = _run(specs, moves, every, n_steps, True, x_lanes)
    fh, out_h = _run(specs, moves, every, n_steps, False, x_lanes)
    assert out_d == out_h
    assert any(o > 0 for o in out_d)  # the walk takes some cells off the grid
    for k, spec in enumerate(specs):
        assert np.array_equal(fd[k], fh[k]), f"sim {k}: device and host uploads differ"
        assert_close(fd[k], _oracle(spec, moves[k], every, n_steps), 1e-5, f"moving cells sim {k}")


@pytest.mark.parametrize("sources", [0, 1, 2])
def test_moving_cells_without_reading_counts_back(sources):
    """Uploads that ask for no count of cells off the grid wait for nothing
    after the check of the arrays, and keep the step graphs (the cell counts
    stay the same from move to move): the fields equal those of uploads that
    read the counts back (and rebuild nothing), bitwise, in every source
    placement, and the oracle's."""
    specs = [_spec((150, 12, 9), 2, "mixed", 300, 5), _spec((33, 20, 17), 1, "neumann", 150, 6)]
    every, n_moves = 2, 4
    moves = [_moves(s, n_moves, 91 + k) for k, s in enumerate(specs)]
    n_steps = every * (n_moves + 1)
    fa, out_a = _run(specs, moves, every, n_steps, True, 1, count=False, sources=sources)
    fb, out_b = _run(specs, moves, every, n_steps, True, 1, count=True, sources=sources)
    assert all(o is None for o in out_a) and any(o > 0 for o in out_b)
    for k, spec in enumerate(specs):
        assert np.array_equal(fa[k], fb[k]), f"sim {k}: uploads with and without counts differ"
        assert_close(fa[k], _oracle(spec, moves[k], every, n_steps), 1e-5, f"moving cells sim {k}, mode {sources}")


def test_device_upload_rejects_bad_cells_and_keeps_the_old_ones():
    spec = _spec((20, 10, 8), 2, "neumann", 50, 3)
    ctx = vb.Context([spec], device="cuda:0")
    try:
        ctx.set_field(0, spec.rho0)
        c = spec.cells
        ctx.step(2)
        ref = ctx.get_field(0).copy()
        for bad in ("V", "S", "rho_star"):
            V, S, rs = c.V.copy(), c.S.copy(), c.rho_star.copy()
            if bad == "V":
                V[7] = 0.0
            elif bad == "S":
                S[3, 1] = -1.0
            else:
                rs[5, 0] = np.nan
            with pytest.raises(vb.VoxlodError) as e:
                ctx.upload_cells_device(0, _device(ctx, c.pos), _device(ctx, V), _device(ctx, S),
                                        _device(ctx, c.U), _device(ctx, rs))
            assert e.value.code == vb.VL_E_ARG
        # the cells of the first upload are still in place: stepping on gives
        # the same field as a context that never saw the bad uploads
        ctx.step(2)
        got = ctx.get_field(0)
    finally:
        ctx.close()
    ctx2 = vb.Context([spec], device="cuda:0")
    try:
        ctx2.set_field(0, spec.rho0)
        ctx2.step(4)
        want = ctx2.get_field(0)
    finally:
        ctx2.close()
    assert not np.array_equal(ref, got)
    assert np.array_equal(got, want)


def test_cell_counts_change_by_orders_of_magnitude():
    """Uploads of 3000, 30, 0, 3 and 3000 cells (within the capacity reserved
    at set-up) between steps, from device arrays, in every source placement;
    each stretch checked against the oracle given the same uploads."""
    spec = _spec((150, 16, 11), 2, "mixed", 3000, 4)
    c = spec.cells
    counts = [30, 0, 3, 3000]
    rng = np.random.default_rng(99)
    subsets = [np.sort(rng.choice(c.n, size=m, replace=False)) for m in counts]
    for mode in (0, 1, 2):
        ctx = vb.Context([spec], device="cuda:0")
        sim = O.from_spec(spec)
        try:
            ctx.set_option(vb.VL_OPT_X_LANES, 1)
            ctx.set_option(vb.VL_OPT_FUSE_SOURCES, mode)
            ctx.set_field(0, spec.rho0)
            ctx.step(3)
            sim.step(3)
            for idx in subsets:
                n_out = ctx.upload_cells_device(0, _device(ctx, c.pos[idx].reshape(-1, 3)),
                                                _device(ctx, c.V[idx]), _device(ctx, c.S[idx].reshape(-1, 2)),
                                                _device(ctx, c.U[idx].reshape(-1, 2)),
                                                _device(ctx, c.rho_star[idx].reshape(-1, 2)))
                assert n_out == sim.upload_cells(c.pos[idx].reshape(-1, 3), c.V[idx], c.S[idx].reshape(-1, 2),
                                                  c.U[idx].reshape(-1, 2), c.rho_star[idx].reshape(-1, 2))
                ctx.step(4)
                sim.step(4)
                assert_close(ctx.get_field(0).astype(np.float64), sim.get_field(), 1e-5,
                             f"mode {mode}, {len(idx)} cells")
        finally:
            ctx.close()


@pytest.mark.parametrize("precision,sources", [(vb.VL_F32, 1), (vb.VL_F32, 2), (vb.VL_F64, None)])
def test_capacity_grows_without_refinalising(precision, sources):
    """vl_resize_cells: a simulation set up for 30 cells takes 3000 after a
    resize and a new bind, with no new context.  The field survives the
    rebind bitwise, the other simulation of the batch keeps its cells, and
    the fields before and after match the oracle given the same uploads."""
    import copy
    full = _spec((60, 14, 11), 2, "mixed", 3000, 7)
    other = _spec((33, 20, 17), 1, "neumann", 150, 8)
    c = full.cells
    idx = np.sort(np.random.default_rng(12).choice(c.n, size=30, replace=False))
    few = copy.copy(full)
    few.cells = W.Cells(pos=c.pos[idx], V=c.V[idx], S=c.S[idx], U=c.U[idx], rho_star=c.rho_star[idx])
    if precision == vb.VL_F64:
        for sp in (full, other):
            sp.rho0 = sp.rho0.astype(np.float64)
        few.rho0 = full.rho0
    oa, ob = O.from_spec(few), O.from_spec(other)
    ctx = vb.Context([few, other], precision=precision, device="cuda:0")
    tol = 1e-12 if precision == vb.VL_F64 else 1e-5
    try:
        if sources is not None:
            ctx.set_option(vb.VL_OPT_FUSE_SOURCES, sources)
        ctx.step(3)
        oa.step(3)
        ob.step(3)
        before = [ctx.get_field(k).copy() for k in range(2)]
        with pytest.raises(vb.VoxlodError) as e:
            ctx.upload_cells(0, c)
        assert e.value.code == vb.VL_E_SHAPE
        ctx.resize_cells(0, 3000)
        assert all(np.array_equal(before[k], ctx.get_field(k)) for k in range(2)), "field changed by the rebind"
        assert ctx.n_cells(1) == 150
        if sources is not None:
            assert ctx.get_option(vb.VL_OPT_FUSE_SOURCES) == sources
        n_out = ctx.upload_cells(0, c)
        assert n_out == oa.upload_cells(c.pos, c.V, c.S, c.U, c.rho_star)
        ctx.step(4)
        oa.step(4)
        ob.step(4)
        assert_close(ctx.get_field(0).astype(np.float64), oa.get_field(), tol, f"grown sim, sources {sources}")
        assert_close(ctx.get_field(1).astype(np.float64), ob.get_field(), tol, f"other sim, sources {sources}")
    finally:
        ctx.close()
