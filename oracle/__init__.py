"""FP64 CPU oracle for the LOD diffusion-decay step with cell sources.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the GPU library ``paper_2110_13368_amd`` and never imports it.

The arithmetic lives in ``oracle.c`` (plain C, IEEE double, no FMA
contraction); this module only loads it and marshals numpy arrays.  The
readings of arXiv:2110.13368 that it implements (Eq. (1), section "Elements of
Parallelism") are listed in ``oracle.h``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# VOXLOD_ORACLE_SANITIZE=1 selects a build with AddressSanitizer and
# UndefinedBehaviorSanitizer (host code only; run the tests with libasan
# preloaded, see run_sanitized_tests.py)
SANITIZE = os.environ.get("VOXLOD_ORACLE_SANITIZE", "") == "1"
LIB_PATH = os.path.join(_HERE, "liboracle_san.so" if SANITIZE else "liboracle.so")
SOURCES = [os.path.join(_HERE, "oracle.c")]
SANITIZE_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"]

NEUMANN, DIRICHLET = 0, 1
DECAY_ONCE, DECAY_THIRDS = 0, 1
LAYOUT_AOS, LAYOUT_SOA = 0, 1

_dp = C.POINTER(C.c_double)
_lib = None


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (OpenMP, IEEE double, no contraction)."""
    if not force and os.path.exists(LIB_PATH):
        return LIB_PATH
    cmd = ["gcc", "-std=c11", "-O3", "-march=x86-64-v2", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-fPIC", "-shared", "-Wall", "-o", LIB_PATH + ".tmp"] + SOURCES + ["-lm"]
    if SANITIZE:
        cmd[1:1] = SANITIZE_FLAGS
    subprocess.run(cmd, check=True)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        build()
    lib = C.CDLL(LIB_PATH)
    i, d, p, vp = C.c_int, C.c_double, _dp, C.c_void_p
    lib.orc_create.restype = vp
    lib.orc_create.argtypes = [i, i, i, d, d, d, d, d, d, i, p, p, d, i]
    lib.orc_destroy.argtypes = [vp]
    lib.orc_set_boundary.argtypes = [vp, i, i, i, d]
    lib.orc_set_field.argtypes = [vp, p, i]
    lib.orc_get_field.argtypes = [vp, p, i]
    lib.orc_upload_cells.argtypes = [vp, i, p, p, p, p, p, C.POINTER(C.c_int)]
    lib.orc_cell_voxels.argtypes = [vp, C.POINTER(C.c_longlong)]
    lib.orc_step.argtypes = [vp, i]
    for f in ("orc_decay", "orc_dirichlet", "orc_sources"):
        getattr(lib, f).argtypes = [vp]
    lib.orc_sweep.argtypes = [vp, i]
    lib.orc_mass.argtypes = [vp, p]
    lib.orc_thomas_line.argtypes = [i, d, d, p, p]
    lib.orc_adjoint.argtypes = [vp, i, p, p, p, p, p, p]
    lib.orc_set_threads.argtypes = [i]
    lib.orc_get_threads.restype = i
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def _f64(a, shape=None) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        a = a.reshape(shape)
    return a


def _check(rc: int, what: str) -> None:
    if rc != 0:
        raise ValueError(f"oracle: {what} rejected its arguments")


def set_threads(n: int) -> None:
    _load().orc_set_threads(int(n))


def get_threads() -> int:
    return int(_load().orc_get_threads())


def thomas_line(c: float, sigma: float, r) -> np.ndarray:
    """Solve tridiag(-c, b, -c) x = r with zero-flux ends (see oracle.h)."""
    r = _f64(r).ravel()
    x = np.empty_like(r)
    _check(_load().orc_thomas_line(r.size, float(c), float(sigma), _ptr(r), _ptr(x)), "thomas_line")
    return x


class OracleSim:
    """One simulation grid held by the C oracle.

    Field arrays use shape (n_sub, nz, ny, nx) (structure-of-arrays, x fastest);
    the oracle stores them internally voxel-major like the paper.
    """

    def __init__(self, shape, h, lo, D, lam, dt, decay_mode=DECAY_ONCE):
        nx, ny, nz = (int(v) for v in shape)
        D = _f64(D).ravel()
        lam = _f64(lam).ravel()
        if D.size != lam.size:
            raise ValueError("D and lambda need one entry per substrate")
        self._lib = _load()
        self.shape = (nx, ny, nz)
        self.n_sub = D.size
        self.D, self.lam = D.copy(), lam.copy()
        self.dt = float(dt)
        self.decay_mode = int(decay_mode)
        self._h = self._lib.orc_create(nx, ny, nz, *(float(v) for v in h), *(float(v) for v in lo),
                                       D.size, _ptr(D), _ptr(lam), float(dt), int(decay_mode))
        if not self._h:
            raise ValueError("oracle: orc_create rejected its arguments")
        self.n_cells = 0

    def close(self):
        if getattr(self, "_h", None):
            self._lib.orc_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    @property
    def field_shape(self):
        nx, ny, nz = self.shape
        return (self.n_sub, nz, ny, nx)

    def set_boundary(self, s: int, face: int, kind: int, value: float = 0.0) -> None:
        _check(self._lib.orc_set_boundary(self._h, int(s), int(face), int(kind), float(value)),
               "set_boundary")

    def set_boundaries(self, kind, value) -> None:
        """kind, value: arrays of shape (n_sub, 6)."""
        kind = np.asarray(kind).reshape(self.n_sub, 6)
        value = np.asarray(value, dtype=np.float64).reshape(self.n_sub, 6)
        for s in range(self.n_sub):
            for f in range(6):
                self.set_boundary(s, f, int(kind[s, f]), float(value[s, f]))

    def set_field(self, rho) -> None:
        rho = _f64(rho, self.field_shape)
        _check(self._lib.orc_set_field(self._h, _ptr(rho), LAYOUT_SOA), "set_field")

    def get_field(self) -> np.ndarray:
        out = np.empty(self.field_shape, dtype=np.float64)
        _check(self._lib.orc_get_field(self._h, _ptr(out), LAYOUT_SOA), "get_field")
        return out

    def upload_cells(self, pos, V, S, U, rho_star) -> int:
        pos = _f64(pos).reshape(-1, 3)
        n = pos.shape[0]
        V = _f64(V).reshape(n)
        S = _f64(S).reshape(n, self.n_sub)
        U = _f64(U).reshape(n, self.n_sub)
        rs = _f64(rho_star).reshape(n, self.n_sub)
        n_out = C.c_int(0)
        _check(self._lib.orc_upload_cells(self._h, n, _ptr(pos), _ptr(V), _ptr(S), _ptr(U), _ptr(rs),
                                          C.byref(n_out)), "upload_cells")
        self.n_cells = n
        return int(n_out.value)

    def cell_voxels(self) -> np.ndarray:
        out = np.empty(max(self.n_cells, 1), dtype=np.int64)
        _check(self._lib.orc_cell_voxels(self._h, out.ctypes.data_as(C.POINTER(C.c_longlong))),
               "cell_voxels")
        return out[: self.n_cells]

    def step(self, n: int = 1) -> None:
        _check(self._lib.orc_step(self._h, int(n)), "step")

    def sweep(self, axis: int) -> None:
        _check(self._lib.orc_sweep(self._h, int(axis)), "sweep")

    def decay(self) -> None:
        _check(self._lib.orc_decay(self._h), "decay")

    def dirichlet(self) -> None:
        _check(self._lib.orc_dirichlet(self._h), "dirichlet")

    def sources(self) -> None:
        _check(self._lib.orc_sources(self._h), "sources")

    def mass(self) -> np.ndarray:
        out = np.empty(self.n_sub, dtype=np.float64)
        _check(self._lib.orc_mass(self._h, _ptr(out)), "mass")
        return out

    def adjoint(self, n_steps: int, g_final):
        """Gradients of a loss whose gradient w.r.t. the field after n_steps is
        g_final, with respect to the current field, D, lambda and per-cell S, U."""
        g = _f64(g_final, self.field_shape)
        g0 = np.empty(self.field_shape, dtype=np.float64)
        dD = np.empty(self.n_sub)
        dl = np.empty(self.n_sub)
        nc = max(self.n_cells, 1)
        dS = np.zeros((nc, self.n_sub))
        dU = np.zeros((nc, self.n_sub))
        _check(self._lib.orc_adjoint(self._h, int(n_steps), _ptr(g), _ptr(g0), _ptr(dD), _ptr(dl),
                                     _ptr(dS), _ptr(dU)), "adjoint")
        return {"rho0": g0, "D": dD, "lambda": dl, "S": dS[: self.n_cells], "U": dU[: self.n_cells]}


def from_spec(spec, decay_mode=DECAY_ONCE, dt=None) -> OracleSim:
    """Build an OracleSim from a workload simulation description (an object with
    shape, h, lo, D, lam, dt, bc_kind, bc_value, rho0 and optional cells)."""
    sim = OracleSim(spec.shape, spec.h, spec.lo, spec.D, spec.lam, spec.dt if dt is None else dt,
                    decay_mode)
    sim.set_boundaries(spec.bc_kind, spec.bc_value)
    sim.set_field(np.asarray(spec.rho0, dtype=np.float64))
    if spec.cells is not None and spec.cells.n > 0:
        c = spec.cells
        sim.upload_cells(c.pos, c.V, c.S, c.U, c.rho_star)
    return sim
