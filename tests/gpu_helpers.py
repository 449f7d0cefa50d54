"""Helpers shared by the GPU tests: run the HIP library and the oracle on the
same seeded inputs and compare them."""
from __future__ import annotations

import copy

import numpy as np

import oracle as O
from paper_2110_13368_amd import binding as vb


def run_gpu(specs, steps, precision=vb.VL_F32, decay=vb.VL_DECAY_ONCE, profiling=False, fuse=True, x_lanes=0,
            x_lane_lines=None, sources_mode=None):
    ctx = vb.Context(specs, precision=precision, decay_split=decay, device="cuda:0")
    try:
        if not fuse:
            vb.vl_set_option(ctx.h, vb.VL_OPT_FUSE_SOURCES, 0)
        if sources_mode is not None:
            vb.vl_set_option(ctx.h, vb.VL_OPT_FUSE_SOURCES, sources_mode)
        if precision == vb.VL_F32:
            vb.vl_set_option(ctx.h, vb.VL_OPT_X_LANES, x_lanes)
            if x_lane_lines is not None:
                vb.vl_set_option(ctx.h, vb.VL_OPT_X_LANE_LINES, x_lane_lines)
        if profiling:
            ctx.set_profiling(True)
        ctx.step(steps)
        ctx.sync()
        return [ctx.get_field(k).astype(np.float64) for k in range(len(specs))], ctx.n_out
    finally:
        ctx.close()


def run_oracle(spec, steps, decay=O.DECAY_ONCE):
    sim = O.from_spec(spec, decay_mode=decay)
    sim.step(steps)
    return sim.get_field()


def subset(spec, subs):
    """The same simulation restricted to some substrates (substrates do not
    interact, so each one can be checked on its own)."""
    s = copy.copy(spec)
    subs = list(subs)
    s.D, s.lam = spec.D[subs], spec.lam[subs]
    s.bc_kind, s.bc_value = spec.bc_kind[subs], spec.bc_value[subs]
    s.rho0 = spec.rho0[subs]
    c = copy.copy(spec.cells)
    c.S, c.U, c.rho_star = spec.cells.S[:, subs], spec.cells.U[:, subs], spec.cells.rho_star[:, subs]
    s.cells = c
    return s


def rel_errs(got, want):
    """Per substrate: (max |x - y| / max |y|, ||x - y||_2 / ||y||_2)."""
    out = []
    for s in range(want.shape[0]):
        d = got[s] - want[s]
        out.append((float(np.max(np.abs(d)) / np.max(np.abs(want[s]))),
                    float(np.linalg.norm(d) / np.linalg.norm(want[s]))))
    return out


def assert_close(got, want, tol, what=""):
    errs = rel_errs(got, want)
    for s, (em, e2) in enumerate(errs):
        assert em <= tol and e2 <= tol, f"{what} substrate {s}: max {em:.3e}, L2 {e2:.3e} > {tol}"
    return errs
