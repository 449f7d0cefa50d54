"""ctypes binding of libvoxlod.so.

The ``vl_*`` functions mirror ``include/voxlod.h`` one to one and only marshal
arguments; every step of the computation runs in the library's HIP kernels.
``Context`` is a convenience owner: it allocates the field and the workspace
as torch tensors on the GPU, creates a (default-priority) torch stream and
binds them, because the library itself never allocates device memory.

Loading fails loudly when the library has not been built; there is no
fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvoxlod.so")

VL_OK, VL_E_ARG, VL_E_STATE, VL_E_SHAPE, VL_E_HIP, VL_E_NONFINITE = 0, -1, -2, -3, -4, -5
VL_F32, VL_F64 = 0, 1
VL_DECAY_ONCE, VL_DECAY_THIRDS = 0, 1
VL_NEUMANN, VL_DIRICHLET = 0, 1
VL_SOA, VL_AOS = 0, 1
VL_OPT_FUSE_SOURCES, VL_OPT_STEP_MODE, VL_OPT_PERSISTENT_GRID, VL_OPT_WAIT_LIMIT_US = 1, 2, 3, 4
VL_MODE_LAUNCHES, VL_MODE_PERSISTENT = 0, 1
VL_OPT_XCD_ORDER = 5
VL_OPT_FUSE_XY = 6
VL_OPT_X_LANES = 7
VL_OPT_X_LANE_LINES = 8
VL_OPT_ADJOINT_TABLES = 9
VL_OPT_Z_SOURCES_STORING = 10
VL_K_SWEEP_X, VL_K_SWEEP_Y, VL_K_SWEEP_Z, VL_K_SOURCES, VL_K_DIRICHLET, VL_K_DECAY, VL_K_STEP = range(7)
KERNEL_NAMES = ["sweep_x", "sweep_y", "sweep_z", "sources", "dirichlet", "decay", "step",
                "replay_x", "replay_y", "replay_z", "adjoint_x", "adjoint_y", "adjoint_z",
                "adjoint_sources", "adjoint_reduce", "adjoint_copy", "sweep_xy"]

# exported symbol -> (restype, argtypes)
_vp, _i, _d, _sz = C.c_void_p, C.c_int, C.c_double, C.c_size_t
_dp, _ip = C.POINTER(C.c_double), C.POINTER(C.c_int)
SIGNATURES = {
    "vl_abi_version": (_i, []),
    "vl_last_error": (C.c_char_p, []),
    "vl_create": (_i, [C.POINTER(_vp), _i, _i, _i]),
    "vl_destroy": (_i, [_vp]),
    "vl_set_grid": (_i, [_vp, _i, _i, _i, _i, _d, _d, _d, _d, _d, _d]),
    "vl_set_substrates": (_i, [_vp, _i, _i, _dp, _dp]),
    "vl_set_boundary": (_i, [_vp, _i, _i, _i, _i, _d]),
    "vl_reserve_cells": (_i, [_vp, _i, _i]),
    "vl_resize_cells": (_i, [_vp, _i, _i, C.POINTER(C.c_size_t)]),
    "vl_finalize": (_i, [_vp, _d, C.POINTER(_sz), C.POINTER(_sz)]),
    "vl_bind": (_i, [_vp, _vp, _vp, _vp]),
    "vl_field_offset": (_i, [_vp, _i, C.POINTER(_sz)]),
    "vl_volume_stride": (_i, [_vp, _i, C.POINTER(_sz)]),
    "vl_set_field": (_i, [_vp, _i, _vp, _i, _i]),
    "vl_get_field": (_i, [_vp, _i, _vp, _i, _i]),
    "vl_upload_cells": (_i, [_vp, _i, _i, _dp, _dp, _dp, _dp, _dp, _ip]),
    "vl_upload_cells_dev": (_i, [_vp, _i, _i, _vp, _vp, _vp, _vp, _vp, _ip]),
    "vl_snapshot": (_i, [_vp, _i, _vp, _vp]),
    "vl_snapshot_wait": (_i, [_vp]),
    "vl_step": (_i, [_vp, _i]),
    "vl_sync": (_i, [_vp]),
    "vl_mass": (_i, [_vp, _i, _dp]),
    "vl_check_finite": (_i, [_vp, C.POINTER(C.c_longlong)]),
    "vl_set_option": (_i, [_vp, _i, _i]),
    "vl_get_option": (_i, [_vp, _i, _ip]),
    "vl_tune": (_i, [_vp, C.c_char_p]),
    "vl_update_substrates": (_i, [_vp, _i, _i, _dp, _dp]),
    "vl_adjoint_workspace": (_i, [_vp, _i, _i, C.POINTER(_sz)]),
    "vl_adjoint": (_i, [_vp, _i, _i, _vp, _vp, _vp, _dp, _dp, _vp, _vp]),
    "vl_set_profiling": (_i, [_vp, _i]),
    "vl_kernel_stats": (_i, [_vp, _i, C.POINTER(C.c_longlong), _dp]),
    "vl_copy_probe": (_i, [_vp, _vp, _sz, _i, _i, _vp]),
    "vl_mass_noalloc": (_i, [_vp, _i, C.c_longlong, _i, C.c_longlong, _vp, _vp]),
}

_lib = None


class VoxlodError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where}: status {code}: {msg}")
        self.code = code


def lib():
    """Load libvoxlod.so (raises if it is missing or unloadable)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2110_13368_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc: int, where: str) -> int:
    if rc != VL_OK:
        raise VoxlodError(rc, where, vl_last_error())
    return rc


def _f64(a, n=None) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if n is not None and a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a


def _p(a: np.ndarray):
    return a.ctypes.data_as(_dp)


# ---------------------------------------------------------------------------
# One wrapper per exported function (same names as the C ABI).

def vl_abi_version() -> int:
    return lib().vl_abi_version()


def vl_last_error() -> str:
    return lib().vl_last_error().decode(errors="replace")


def vl_create(n_sims: int, precision: int = VL_F32, decay_split: int = VL_DECAY_ONCE):
    h = _vp()
    _check(lib().vl_create(C.byref(h), int(n_sims), int(precision), int(decay_split)), "vl_create")
    return h


def vl_destroy(ctx) -> None:
    lib().vl_destroy(ctx)


def vl_set_grid(ctx, sim, nx, ny, nz, dx, dy, dz, x0, y0, z0) -> None:
    _check(lib().vl_set_grid(ctx, int(sim), int(nx), int(ny), int(nz), float(dx), float(dy), float(dz),
                             float(x0), float(y0), float(z0)), "vl_set_grid")


def vl_set_substrates(ctx, sim, D, lam) -> None:
    D = _f64(D)
    lam = _f64(lam, D.size)
    _check(lib().vl_set_substrates(ctx, int(sim), D.size, _p(D), _p(lam)), "vl_set_substrates")


def vl_set_boundary(ctx, sim, sub, face, kind, value) -> None:
    _check(lib().vl_set_boundary(ctx, int(sim), int(sub), int(face), int(kind), float(value)),
           "vl_set_boundary")


def vl_reserve_cells(ctx, sim, max_cells) -> None:
    _check(lib().vl_reserve_cells(ctx, int(sim), int(max_cells)), "vl_reserve_cells")


def vl_resize_cells(ctx, sim, max_cells) -> int:
    """New cell capacity after vl_finalize; returns the new workspace size in
    bytes (the context is unbound until vl_bind)."""
    ws = C.c_size_t(0)
    _check(lib().vl_resize_cells(ctx, int(sim), int(max_cells), C.byref(ws)), "vl_resize_cells")
    return int(ws.value)


def vl_finalize(ctx, dt):
    fe, wb = _sz(0), _sz(0)
    _check(lib().vl_finalize(ctx, float(dt), C.byref(fe), C.byref(wb)), "vl_finalize")
    return int(fe.value), int(wb.value)


def vl_bind(ctx, field_ptr: int, workspace_ptr: int, stream_ptr: int) -> None:
    _check(lib().vl_bind(ctx, _vp(field_ptr), _vp(workspace_ptr), _vp(stream_ptr or None)), "vl_bind")


def vl_update_substrates(ctx, sim, D, lam) -> None:
    D = _f64(D)
    lam = _f64(lam, len(D))
    _check(lib().vl_update_substrates(ctx, sim, len(D), _p(D), _p(lam)), "vl_update_substrates")


def vl_field_offset(ctx, sim) -> int:
    o = _sz(0)
    _check(lib().vl_field_offset(ctx, int(sim), C.byref(o)), "vl_field_offset")
    return int(o.value)


def vl_volume_stride(ctx, sim) -> int:
    o = _sz(0)
    _check(lib().vl_volume_stride(ctx, int(sim), C.byref(o)), "vl_volume_stride")
    return int(o.value)


def vl_set_field(ctx, sim, src_ptr: int, src_is_device: bool, layout: int = VL_SOA) -> None:
    _check(lib().vl_set_field(ctx, int(sim), _vp(src_ptr), int(bool(src_is_device)), int(layout)),
           "vl_set_field")


def vl_get_field(ctx, sim, dst_ptr: int, dst_is_device: bool, layout: int = VL_SOA) -> None:
    _check(lib().vl_get_field(ctx, int(sim), _vp(dst_ptr), int(bool(dst_is_device)), int(layout)),
           "vl_get_field")


def vl_snapshot(ctx, sim, stage_ptr: int, host_ptr: int) -> None:
    """Enqueue a snapshot of one simulation's field: device staging buffer and
    host destination, each n_sub*nz*ny*nx elements (raw pointers)."""
    _check(lib().vl_snapshot(ctx, int(sim), _vp(stage_ptr), _vp(host_ptr)), "vl_snapshot")


def vl_snapshot_wait(ctx) -> None:
    _check(lib().vl_snapshot_wait(ctx), "vl_snapshot_wait")


def vl_upload_cells_dev(ctx, sim, n: int, pos_ptr: int, V_ptr: int, S_ptr: int, U_ptr: int, rs_ptr: int,
                        count_out: bool = True):
    """Cell upload from device arrays (raw pointers: pos n x 3, V n, S / U /
    rho_star n x n_sub, float64, contiguous); returns the cells outside the
    grid, or None with count_out=False (then the call does not wait for the
    binning, which reads the arrays on the context's stream)."""
    n_out = C.c_int(0)
    _check(lib().vl_upload_cells_dev(ctx, int(sim), int(n), C.c_void_p(pos_ptr), C.c_void_p(V_ptr),
                                     C.c_void_p(S_ptr), C.c_void_p(U_ptr), C.c_void_p(rs_ptr),
                                     C.byref(n_out) if count_out else None),
           "vl_upload_cells_dev")
    return n_out.value if count_out else None


def vl_upload_cells(ctx, sim, pos, V, S, U, rho_star, n_sub: int) -> int:
    pos = _f64(pos).reshape(-1, 3)
    n = pos.shape[0]
    V = _f64(V, n)
    S = _f64(S, n * n_sub)
    U = _f64(U, n * n_sub)
    rs = _f64(rho_star, n * n_sub)
    n_out = C.c_int(0)
    _check(lib().vl_upload_cells(ctx, int(sim), n, _p(pos), _p(V), _p(S), _p(U), _p(rs), C.byref(n_out)),
           "vl_upload_cells")
    return int(n_out.value)


def vl_step(ctx, n_steps: int) -> None:
    _check(lib().vl_step(ctx, int(n_steps)), "vl_step")


def vl_sync(ctx) -> None:
    _check(lib().vl_sync(ctx), "vl_sync")


def vl_mass(ctx, sim, n_sub: int) -> np.ndarray:
    out = np.empty(n_sub, dtype=np.float64)
    _check(lib().vl_mass(ctx, int(sim), _p(out)), "vl_mass")
    return out


def vl_check_finite(ctx) -> int:
    bad = C.c_longlong(0)
    rc = lib().vl_check_finite(ctx, C.byref(bad))
    if rc not in (VL_OK, VL_E_NONFINITE):
        _check(rc, "vl_check_finite")
    return int(bad.value)


def vl_set_option(ctx, option: int, value: int) -> None:
    _check(lib().vl_set_option(ctx, int(option), int(value)), "vl_set_option")


def vl_get_option(ctx, option: int) -> int:
    v = C.c_int(0)
    _check(lib().vl_get_option(ctx, int(option), C.byref(v)), "vl_get_option")
    return int(v.value)


def vl_tune(ctx, cache_path: Optional[str] = None) -> None:
    _check(lib().vl_tune(ctx, cache_path.encode() if cache_path else None), "vl_tune")


def vl_adjoint_workspace(ctx, n_steps: int, ckpt_every: int) -> int:
    b = _sz(0)
    _check(lib().vl_adjoint_workspace(ctx, int(n_steps), int(ckpt_every), C.byref(b)), "vl_adjoint_workspace")
    return int(b.value)


def vl_adjoint(ctx, n_steps: int, ckpt_every: int, ws_ptr: int, grad_final_ptr: int,
               grad_rho0_ptr: int, n_volumes: int, dS_ptr: int, dU_ptr: int):
    """Returns host arrays (dD, dlambda), one entry per volume."""
    dD = np.zeros(n_volumes)
    dl = np.zeros(n_volumes)
    _check(lib().vl_adjoint(ctx, int(n_steps), int(ckpt_every), _vp(ws_ptr), _vp(grad_final_ptr),
                            _vp(grad_rho0_ptr or None), _p(dD), _p(dl), _vp(dS_ptr or None),
                            _vp(dU_ptr or None)), "vl_adjoint")
    return dD, dl


def vl_set_profiling(ctx, enable: bool) -> None:
    _check(lib().vl_set_profiling(ctx, int(bool(enable))), "vl_set_profiling")


def vl_kernel_stats(ctx, kind: int):
    n, ms = C.c_longlong(0), C.c_double(0)
    _check(lib().vl_kernel_stats(ctx, int(kind), C.byref(n), C.byref(ms)), "vl_kernel_stats")
    return int(n.value), float(ms.value)


def vl_mass_noalloc(field_ptr: int, precision: int, n_vox: int, n_vols: int, vol_stride: int, out_ptr: int,
                    stream_ptr: int = 0) -> None:
    _check(lib().vl_mass_noalloc(field_ptr, int(precision), int(n_vox), int(n_vols), int(vol_stride), out_ptr,
                                 stream_ptr), "vl_mass_noalloc")


def vl_copy_probe(dst_ptr: int, src_ptr: int, nbytes: int, width: int = 16, nontemporal: int = 0,
                  stream_ptr: int = 0) -> None:
    _check(lib().vl_copy_probe(dst_ptr, src_ptr, nbytes, int(width), int(nontemporal), stream_ptr),
           "vl_copy_probe")


# ---------------------------------------------------------------------------

class DeviceCells:
    """Cell arrays of a device upload (torch float64 tensors on the context's
    device, kept by reference): pos (n, 3), V (n,), S / U / rho_star
    (n, n_sub)."""

    def __init__(self, pos, V, S, U, rho_star):
        self.pos, self.V, self.S, self.U, self.rho_star = pos, V, S, U, rho_star

    @property
    def n(self) -> int:
        return int(self.V.numel())


class Context:
    """Owns a library context for a list of simulations (workload ``SimSpec``
    objects or anything with the same attributes), with its field and workspace
    allocated as torch tensors on ``device`` and a torch stream of its own.

    ``cells[k]`` is simulation k's cell set as last uploaded through this
    object (the spec's at construction, then whatever ``upload_cells`` or
    ``upload_cells_device`` was given): the adjoint lays out its per-cell
    gradients by these counts, and autograd re-uploads these positions."""

    def __init__(self, sims: Sequence, dt: Optional[float] = None, precision: int = VL_F32,
                 decay_split: int = VL_DECAY_ONCE, device: str = "cuda:0", set_initial: bool = True,
                 upload_cells: bool = True):
        import torch
        self.torch = torch
        self.sims = list(sims)
        self.precision = precision
        self.dtype = torch.float32 if precision == VL_F32 else torch.float64
        self.np_dtype = np.float32 if precision == VL_F32 else np.float64
        self.device = torch.device(device)
        self.dt = float(dt if dt is not None else self.sims[0].dt)
        self.h = vl_create(len(self.sims), precision, decay_split)
        self.cells = [s.cells if getattr(s, "cells", None) is not None else None for s in self.sims]
        # per simulation its current (D, lambda): the spec's, then whatever update_substrates set
        self.params = [(np.asarray(s.D, np.float64).copy(), np.asarray(s.lam, np.float64).copy()) for s in self.sims]
        try:
            for k, s in enumerate(self.sims):
                vl_set_grid(self.h, k, *s.shape, *s.h, *s.lo)
                vl_set_substrates(self.h, k, s.D, s.lam)
                for q in range(s.n_sub):
                    for f in range(6):
                        if int(s.bc_kind[q, f]) == VL_DIRICHLET:
                            vl_set_boundary(self.h, k, q, f, VL_DIRICHLET, float(s.bc_value[q, f]))
                ncell = s.cells.n if getattr(s, "cells", None) is not None else 0
                vl_reserve_cells(self.h, k, ncell)
            self.field_elems, self.ws_bytes = vl_finalize(self.h, self.dt)
            with torch.cuda.device(self.device):
                self.stream = torch.cuda.Stream(device=self.device)
            self.field = torch.zeros(self.field_elems, dtype=self.dtype, device=self.device)
            self.workspace = torch.zeros(self.ws_bytes, dtype=torch.uint8, device=self.device)
            torch.cuda.synchronize(self.device)
            vl_bind(self.h, self.field.data_ptr(), self.workspace.data_ptr(), self.stream.cuda_stream)
            self.offsets = [vl_field_offset(self.h, k) for k in range(len(self.sims))]
            self.strides = [vl_volume_stride(self.h, k) for k in range(len(self.sims))]
            self._stages = {}      # per simulation: device staging buffer of its snapshots
            self._snap_keep = []   # host buffers of snapshots not yet waited for
            if set_initial:
                for k, s in enumerate(self.sims):
                    self.set_field(k, s.rho0)
            if upload_cells:
                self.n_out = [self.upload_cells(k, s.cells) if s.cells.n > 0 else 0
                              for k, s in enumerate(self.sims)]
            else:
                self.cells = [None] * len(self.sims)
        except Exception:
            vl_destroy(self.h)
            self.h = None
            raise

    def close(self):
        if getattr(self, "h", None):
            vl_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- field I/O --
    def set_field(self, k: int, rho) -> None:
        s = self.sims[k]
        if isinstance(rho, self.torch.Tensor):
            t = rho.to(self.device, self.dtype).contiguous()
            self.torch.cuda.synchronize(self.device)
            vl_set_field(self.h, k, t.data_ptr(), True, VL_SOA)
        else:
            a = np.ascontiguousarray(np.asarray(rho, dtype=self.np_dtype).reshape(s.field_shape))
            vl_set_field(self.h, k, a.ctypes.data, False, VL_SOA)

    def get_field(self, k: int) -> np.ndarray:
        s = self.sims[k]
        out = np.empty(s.field_shape, dtype=self.np_dtype)
        vl_get_field(self.h, k, out.ctypes.data, False, VL_SOA)
        return out

    def snapshot(self, k: int, out=None):
        """Enqueue a copy of simulation k's field to host memory after the
        steps queued so far; steps enqueued afterwards overlap the transfer.
        ``out``: a contiguous CPU tensor of shape (n_sub, nz, ny, nx) and the
        field's dtype, pinned for the transfer to overlap (a pinned one is
        allocated when None).  Its contents are valid after snapshot_wait()."""
        torch = self.torch
        shape = tuple(self.sims[k].field_shape)
        if out is None:
            out = torch.empty(shape, dtype=self.dtype, pin_memory=True)
        elif (tuple(out.shape) != shape or out.dtype != self.dtype or out.device.type != "cpu"
              or not out.is_contiguous()):
            raise ValueError("snapshot buffer must be a contiguous CPU tensor of the field's shape and dtype")
        stage = self._stages.get(k)
        if stage is None:
            stage = self._stages[k] = torch.empty(shape, dtype=self.dtype, device=self.device)
        vl_snapshot(self.h, k, stage.data_ptr(), out.data_ptr())
        self._snap_keep.append(out)
        return out

    def snapshot_wait(self) -> None:
        vl_snapshot_wait(self.h)
        self._snap_keep.clear()

    def field_view(self, k: int):
        """Torch view (n_sub, nz, ny, nx) of one simulation's volumes."""
        s = self.sims[k]
        nx, ny, nz = s.shape
        return self.field.as_strided((s.n_sub, nz, ny, nx), (self.strides[k], nx * ny, nx, 1),
                                     self.offsets[k])

    def update_substrates(self, k: int, D, lam) -> None:
        vl_update_substrates(self.h, k, D, lam)
        self.params[k] = (np.asarray(D, np.float64).copy(), np.asarray(lam, np.float64).copy())

    def n_cells(self, k: int) -> int:
        """Cells of simulation k as last uploaded through this object."""
        c = self.cells[k]
        return 0 if c is None else int(c.n)

    def upload_cells(self, k: int, cells) -> int:
        n_out = vl_upload_cells(self.h, k, cells.pos, cells.V, cells.S, cells.U, cells.rho_star,
                                self.sims[k].n_sub)
        self.cells[k] = cells
        self._autograd_params = None
        return n_out

    def upload_cells_device(self, k: int, pos, V, S, U, rho_star, count_out: bool = True):
        """Cells from torch tensors on this context's device (float64: pos
        (n, 3), V (n,), S / U / rho_star (n, n_sub)).  Returns the cells off
        the grid (the call then waits for the binning), or None with
        count_out=False: the binning is queued on the context's stream and
        reads the tensors there, which this object keeps alive and marks as
        used on that stream; the caller must not write them until the stream
        has passed the upload (e.g. sync())."""
        torch = self.torch
        ts = [t.contiguous() for t in (pos, V, S, U, rho_star)]
        for t in ts:
            if t.device != self.device or t.dtype != torch.float64:
                raise ValueError("cell tensors must be float64 on the context's device")
        n = int(ts[1].numel())
        if tuple(ts[0].shape) != (n, 3) or any(tuple(t.shape) != (n, self.sims[k].n_sub) for t in ts[2:]):
            raise ValueError("cell tensor shapes do not match")
        if self.stream is not None:  # the tensors were written on the caller's stream
            self.stream.wait_stream(torch.cuda.current_stream(self.device))
        n_out = vl_upload_cells_dev(self.h, k, n, *[t.data_ptr() for t in ts], count_out=count_out)
        if not count_out and self.stream is not None:
            for t in ts:  # not handed to other allocations before the stream has read them
                t.record_stream(self.stream)
        self.cells[k] = DeviceCells(*ts)
        self._autograd_params = None
        return n_out

    def resize_cells(self, k: int, max_cells: int) -> None:
        """Change simulation k's cell capacity (vl_resize_cells): a workspace
        of the new size is allocated and bound with the same field, whose
        values stay, and every simulation's current cells are uploaded again
        (the step graphs and any tuned options' graphs are rebuilt)."""
        torch = self.torch
        if self.n_cells(k) > max_cells:
            raise ValueError(f"simulation {k} holds {self.n_cells(k)} cells, more than {max_cells}")
        nb = vl_resize_cells(self.h, k, max_cells)
        ws = torch.zeros(max(nb, 1), dtype=torch.uint8, device=self.device)
        torch.cuda.synchronize(self.device)
        vl_bind(self.h, self.field.data_ptr(), ws.data_ptr(), self.stream.cuda_stream)
        self.workspace, self.ws_bytes = ws, nb
        for j, c in enumerate(self.cells):
            if c is None or c.n == 0:
                continue
            if isinstance(c, DeviceCells):
                vl_upload_cells_dev(self.h, j, c.n, c.pos.data_ptr(), c.V.data_ptr(), c.S.data_ptr(),
                                    c.U.data_ptr(), c.rho_star.data_ptr())
            else:
                vl_upload_cells(self.h, j, c.pos, c.V, c.S, c.U, c.rho_star, self.sims[j].n_sub)

    # -- stepping and diagnostics --
    def step(self, n: int = 1) -> None:
        vl_step(self.h, n)

    def sync(self) -> None:
        vl_sync(self.h)

    def mass(self, k: int) -> np.ndarray:
        return vl_mass(self.h, k, self.sims[k].n_sub)

    def check_finite(self) -> int:
        return vl_check_finite(self.h)

    def set_option(self, option: int, value: int) -> None:
        vl_set_option(self.h, option, value)

    def get_option(self, option: int) -> int:
        return vl_get_option(self.h, option)

    def tune(self, cache_path: Optional[str] = None) -> None:
        """Pick the step mode and launch size by timing (overwrites the field)."""
        vl_tune(self.h, cache_path)

    def to_field_layout(self, arrays):
        """Device tensor of the whole field (padded volumes) from one
        (n_sub, nz, ny, nx) array per simulation."""
        t = self.torch.zeros(self.field_elems, dtype=self.dtype, device=self.device)
        for k, a in enumerate(arrays):
            s = self.sims[k]
            nx, ny, nz = s.shape
            view = t.as_strided((s.n_sub, nz, ny, nx), (self.strides[k], nx * ny, nx, 1), self.offsets[k])
            view.copy_(self.torch.as_tensor(a).to(self.device, self.dtype))
        return t

    def from_field_layout(self, t, k: int):
        s = self.sims[k]
        nx, ny, nz = s.shape
        return t.as_strided((s.n_sub, nz, ny, nx), (self.strides[k], nx * ny, nx, 1), self.offsets[k])

    def adjoint_flat(self, n_steps: int, ckpt_every: int, grad_final):
        """vl_adjoint on flat tensors: grad_final in the field layout; returns
        grad_rho0 (field layout), dD and dlambda (float64, one per volume) and
        dS, dU (float64, per simulation its cells x n_sub, concatenated)."""
        torch = self.torch
        nbytes = vl_adjoint_workspace(self.h, n_steps, ckpt_every)
        ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
        g = grad_final.to(self.device, self.dtype).contiguous()
        if g.numel() != self.field_elems:
            raise ValueError(f"grad_final must hold {self.field_elems} elements")
        g0 = torch.zeros_like(g)
        total = sum(self.n_cells(k) * s.n_sub for k, s in enumerate(self.sims))
        dS = torch.zeros(max(total, 1), dtype=torch.float64, device=self.device)
        dU = torch.zeros(max(total, 1), dtype=torch.float64, device=self.device)
        torch.cuda.synchronize(self.device)
        nvol = sum(s.n_sub for s in self.sims)
        dD, dl = vl_adjoint(self.h, n_steps, ckpt_every, ws.data_ptr(), g.data_ptr(), g0.data_ptr(), nvol,
                            dS.data_ptr(), dU.data_ptr())
        return g0, torch.from_numpy(dD), torch.from_numpy(dl), dS[:total], dU[:total]

    def adjoint(self, n_steps: int, ckpt_every: int, grad_final):
        """Gradients of a loss whose gradient w.r.t. the field after n_steps
        from the current field is grad_final (one array per simulation).
        Returns per simulation: grad_rho0 (device tensor), dD, dlambda (numpy),
        dS, dU (device tensors, cells x n_sub)."""
        g0, dD, dl, dS, dU = self.adjoint_flat(n_steps, ckpt_every, self.to_field_layout(grad_final))
        out, v, c = [], 0, 0
        for k, s in enumerate(self.sims):
            n = self.n_cells(k)
            nc = n * s.n_sub
            out.append({"rho0": self.from_field_layout(g0, k).clone(), "D": dD[v:v + s.n_sub].numpy(),
                        "lambda": dl[v:v + s.n_sub].numpy(),
                        "S": dS[c:c + nc].reshape(n, s.n_sub), "U": dU[c:c + nc].reshape(n, s.n_sub)})
            v += s.n_sub
            c += nc
        return out

    def set_profiling(self, on: bool) -> None:
        vl_set_profiling(self.h, on)

    def kernel_stats(self):
        return {KERNEL_NAMES[k]: vl_kernel_stats(self.h, k) for k in range(len(KERNEL_NAMES))}
