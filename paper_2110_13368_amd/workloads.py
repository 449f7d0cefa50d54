"""Seeded synthetic inputs shaped like the paper's tumour workloads.

This module only draws random numbers: grids, coefficients, boundary
conditions, initial fields and cell agents.  It holds none of the method's
arithmetic, so both the GPU library and the CPU oracle can be fed from it.

The paper's timed inputs (PhysiCell's cancer-immune sample project: a
2000 um cube, oxygen plus an immunostimulatory factor, diffusion time step
about 0.01 min, cells fixed in the long runs -- sections "Profiling",
"Input Datasets" and "GPU-accelerated Long-time Simulations") are not
available, so the five configurations below stand in for them with their
shapes.  Every simulation draws from ``numpy.random.default_rng(211013368 +
10*cfg + sim)``.

Field arrays have shape (n_sub, nz, ny, nx) (x fastest).  Face order is
x-, x+, y-, y+, z-, z+; kind 0 = zero flux (Neumann), 1 = Dirichlet.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence, Tuple

import numpy as np

SEED_BASE = 211013368
NEUMANN, DIRICHLET = 0, 1


@dataclasses.dataclass
class Cells:
    pos: np.ndarray  # (n, 3) float64, um
    V: np.ndarray  # (n,) float64, um^3
    S: np.ndarray  # (n, n_sub) float64, 1/min
    U: np.ndarray  # (n, n_sub) float64, 1/min
    rho_star: np.ndarray  # (n, n_sub) float64

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])

    @staticmethod
    def empty(n_sub: int) -> "Cells":
        z = np.zeros((0, n_sub))
        return Cells(np.zeros((0, 3)), np.zeros(0), z, z.copy(), z.copy())


@dataclasses.dataclass
class SimSpec:
    shape: Tuple[int, int, int]  # (nx, ny, nz)
    h: Tuple[float, float, float]  # voxel edges (dx, dy, dz), um
    lo: Tuple[float, float, float]  # lower corner, um
    D: np.ndarray  # (n_sub,) um^2/min
    lam: np.ndarray  # (n_sub,) 1/min
    dt: float  # min
    bc_kind: np.ndarray  # (n_sub, 6) int32
    bc_value: np.ndarray  # (n_sub, 6) float64
    rho0: np.ndarray  # (n_sub, nz, ny, nx), float32 or float64
    cells: Cells

    @property
    def n_sub(self) -> int:
        return int(self.D.size)

    @property
    def n_vox(self) -> int:
        return int(np.prod(self.shape))

    @property
    def field_shape(self):
        nx, ny, nz = self.shape
        return (self.n_sub, nz, ny, nx)


@dataclasses.dataclass
class Workload:
    name: str
    sims: List[SimSpec]
    steps: int
    dtype: str  # "f32" or "f64": storage and sweep precision on the GPU
    note: str = ""

    @property
    def voxel_substrates(self) -> int:
        return int(sum(s.n_vox * s.n_sub for s in self.sims))


def rng_for(cfg: int, sim: int = 0) -> np.random.Generator:
    return np.random.default_rng(SEED_BASE + 10 * cfg + sim)


def log_uniform(rng, lo, hi, size=None):
    return np.exp(rng.uniform(np.log(lo), np.log(hi), size=size))


def centred_lo(shape, h):
    return tuple(-0.5 * n * d for n, d in zip(shape, h))


def uniform_field(rng, field_shape, lo, hi, dtype) -> np.ndarray:
    """i.i.d. U[lo, hi) per voxel and substrate, drawn directly in dtype."""
    out = rng.random(field_shape, dtype=np.float32 if dtype == "f32" else np.float64)
    out *= np.asarray(hi - lo, dtype=out.dtype)
    out += np.asarray(lo, dtype=out.dtype)
    return out


def _inside(p, lo, hi):
    return np.all((p >= lo) & (p < hi), axis=1)


def uniform_positions(rng, n, lo, hi) -> np.ndarray:
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    p = rng.uniform(lo, hi, size=(n, 3))
    bad = ~_inside(p, lo, hi)
    while bad.any():
        p[bad] = rng.uniform(lo, hi, size=(int(bad.sum()), 3))
        bad = ~_inside(p, lo, hi)
    return p


def gaussian_positions(rng, n, sigma, centre, lo, hi) -> np.ndarray:
    """Gaussian ball, redrawn until every cell is inside the half-open box."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    p = rng.normal(centre, sigma, size=(n, 3))
    bad = ~_inside(p, lo, hi)
    while bad.any():
        p[bad] = rng.normal(centre, sigma, size=(int(bad.sum()), 3))
        bad = ~_inside(p, lo, hi)
    return p


def disc_positions(rng, n, sigma, centre, lo, hi) -> np.ndarray:
    """Gaussian disc in x and y (width sigma about the centre), uniform in z
    through the grid's thickness; redrawn until every cell is inside."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)

    def draw(m):
        q = rng.normal(centre, sigma, size=(m, 3))
        q[:, 2] = rng.uniform(lo[2], hi[2], size=m)
        return q

    p = draw(n)
    bad = ~_inside(p, lo, hi)
    while bad.any():
        p[bad] = draw(int(bad.sum()))
        bad = ~_inside(p, lo, hi)
    return p


def tumour_rates(rng, n, n_sub) -> Tuple[np.ndarray, ...]:
    """Per-cell rates as in the single large simulation: S, U log-uniform in
    [0.1, 10] /min, rho* uniform in [0, 40], V uniform in [1000, 4000] um^3."""
    S = log_uniform(rng, 0.1, 10.0, size=(n, n_sub))
    U = log_uniform(rng, 0.1, 10.0, size=(n, n_sub))
    rs = rng.uniform(0.0, 40.0, size=(n, n_sub))
    V = rng.uniform(1000.0, 4000.0, size=n)
    return V, S, U, rs


def make_sim(rng, shape, h, n_sub, *, D=None, lam=None, dt=0.01, dtype="f32",
             bc="neumann", p_dirichlet=0.5, rho_range=(0.0, 40.0), n_cells=0,
             cell_layout="uniform", sigma=300.0, core_fraction=0.7,
             lo=None) -> SimSpec:
    """General generator used by the named configurations and by the tests.

    bc: "neumann" (all zero flux), "dirichlet" (all faces Dirichlet with a value
    drawn from rho_range), or "mixed" (each (substrate, face) Dirichlet with
    probability p_dirichlet).  cell_layout: "uniform", "gaussian" (ball of
    width sigma about the centre), "core" (core_fraction Gaussian, the rest
    uniform) or "disc" (Gaussian in x and y, uniform in z: for grids one voxel
    thick)."""
    shape = tuple(int(v) for v in shape)
    h = tuple(float(v) for v in h)
    lo = centred_lo(shape, h) if lo is None else tuple(float(v) for v in lo)
    hi = tuple(l + n * d for l, n, d in zip(lo, shape, h))
    D = log_uniform(rng, 1e3, 1e5, size=n_sub) if D is None else np.full(n_sub, 0.0) + np.asarray(D, dtype=np.float64)
    lam = log_uniform(rng, 1e-3, 1.0, size=n_sub) if lam is None else np.full(n_sub, 0.0) + np.asarray(lam, dtype=np.float64)
    bc_kind = np.zeros((n_sub, 6), dtype=np.int32)
    bc_value = np.zeros((n_sub, 6), dtype=np.float64)
    if bc == "dirichlet":
        bc_kind[:] = DIRICHLET
        bc_value[:] = rng.uniform(*rho_range, size=(n_sub, 6))
    elif bc == "mixed":
        bc_kind[:] = (rng.random((n_sub, 6)) < p_dirichlet).astype(np.int32)
        bc_value[:] = rng.uniform(*rho_range, size=(n_sub, 6)) * bc_kind
    elif bc != "neumann":
        raise ValueError(f"unknown boundary mix {bc!r}")
    nx, ny, nz = shape
    rho0 = uniform_field(rng, (n_sub, nz, ny, nx), rho_range[0], rho_range[1], dtype)
    if n_cells > 0:
        centre = tuple(0.5 * (a + b) for a, b in zip(lo, hi))
        if cell_layout == "uniform":
            pos = uniform_positions(rng, n_cells, lo, hi)
        elif cell_layout == "gaussian":
            pos = gaussian_positions(rng, n_cells, sigma, centre, lo, hi)
        elif cell_layout == "disc":
            pos = disc_positions(rng, n_cells, sigma, centre, lo, hi)
        elif cell_layout == "core":
            n_core = int(round(core_fraction * n_cells))
            pos = np.concatenate([gaussian_positions(rng, n_core, sigma, centre, lo, hi),
                                  uniform_positions(rng, n_cells - n_core, lo, hi)])
        else:
            raise ValueError(f"unknown cell layout {cell_layout!r}")
        V, S, U, rs = tumour_rates(rng, n_cells, n_sub)
        cells = Cells(pos, V, S, U, rs)
    else:
        cells = Cells.empty(n_sub)
    return SimSpec(shape, h, lo, D, lam, float(dt), bc_kind, bc_value, rho0, cells)


# --------------------------------------------------------------------------
# The five named configurations.

def plain_fp64(scale: float = 1.0) -> Workload:
    """50^3 voxels of 20 um, one substrate (D = 1e5 um^2/min, lambda = 0.1/min),
    Dirichlet 38 on every face, rho0 = 38, 1000 uptake-only cells (V = 2494,
    U = 10, S = 0, rho* = 0) at uniform positions; dt = 0.01, 100 steps."""
    rng = rng_for(1, 0)
    n = max(1, int(round(50 * scale)))
    shape = (n, n, n)
    h = (20.0, 20.0, 20.0)
    lo = centred_lo(shape, h)
    hi = tuple(l + n * d for l, d in zip(lo, h))
    n_cells = max(1, int(round(1000 * scale ** 3)))
    pos = uniform_positions(rng, n_cells, lo, hi)
    cells = Cells(pos, np.full(n_cells, 2494.0), np.zeros((n_cells, 1)), np.full((n_cells, 1), 10.0),
                  np.zeros((n_cells, 1)))
    spec = SimSpec(shape, h, lo, np.array([1e5]), np.array([0.1]), 0.01,
                   np.full((1, 6), DIRICHLET, dtype=np.int32), np.full((1, 6), 38.0),
                   np.full((1, n, n, n), 38.0, dtype=np.float64), cells)
    return Workload("plain-fp64-50^3x1", [spec], 100, "f64",
                    "uniform 38 field, Dirichlet 38 on all faces, 1000 uptake-only cells")


def single_large(dtype: str = "f32", scale: float = 1.0, n_cells: Optional[int] = None) -> Workload:
    """200^3 voxels of 10 um, 4 substrates (D log-uniform [1e3, 1e5], lambda
    log-uniform [1e-3, 1]), zero-flux faces, rho0 i.i.d. U[0, 40]; 1e5 cells in
    a Gaussian ball (sigma 300 um) about the centre; dt = 0.01, 1000 steps."""
    rng = rng_for(2, 0)
    n = max(1, int(round(200 * scale)))
    nc = int(round(1e5 * scale ** 3)) if n_cells is None else n_cells
    spec = make_sim(rng, (n, n, n), (10.0, 10.0, 10.0), 4, dtype=dtype, bc="neumann",
                    n_cells=nc, cell_layout="gaussian", sigma=300.0 * scale)
    return Workload(f"single-large-{n}^3x4-{dtype}", [spec], 1000, dtype,
                    "Gaussian-ball tumour (sigma 300 um) in a 2000 um cube")


def batched(n_sims: int = 256, edge_range=(32, 128), cells_range=(1000, 20000), dtype="f32") -> Workload:
    """n_sims independent grids, each edge uniform in edge_range, 20 um voxels,
    2 substrates, D and lambda log-uniform, every (substrate, face) Dirichlet
    with probability 1/2 (value U[0, 40]), rho0 i.i.d. U[0, 40], cell count
    uniform in cells_range at uniform positions; dt = 0.01, 200 steps."""
    sims = []
    for k in range(n_sims):
        rng = rng_for(3, k)
        shape = tuple(int(v) for v in rng.integers(edge_range[0], edge_range[1] + 1, size=3))
        nc = int(rng.integers(cells_range[0], cells_range[1] + 1))
        sims.append(make_sim(rng, shape, (20.0, 20.0, 20.0), 2, dtype=dtype, bc="mixed",
                             n_cells=nc, cell_layout="uniform"))
    return Workload(f"batched-{n_sims}x2-{dtype}", sims, 200, dtype,
                    "ragged grids, mixed Dirichlet/zero-flux faces")


def differentiation(scale: float = 1.0, dtype="f32") -> Workload:
    """100^3 voxels of 20 um, 2 substrates, zero-flux faces, 2e4 cells in a
    Gaussian ball (sigma 300 um); 200 steps, checkpoints every 20."""
    rng = rng_for(4, 0)
    n = max(1, int(round(100 * scale)))
    nc = max(1, int(round(2e4 * scale ** 3)))
    spec = make_sim(rng, (n, n, n), (20.0, 20.0, 20.0), 2, dtype=dtype, bc="neumann",
                    n_cells=nc, cell_layout="gaussian", sigma=300.0 * scale)
    return Workload(f"differentiation-{n}^3x2-{dtype}", [spec], 200, dtype,
                    "loss = half squared misfit to a run with perturbed parameters")


def tumour_scale(scale: float = 1.0, dtype="f32") -> Workload:
    """400^3 voxels of 20 um, 8 substrates, zero-flux faces; 1e6 cells, 70% in a
    Gaussian core (sigma 800 um) and 30% uniform; dt = 0.01, 100 steps."""
    rng = rng_for(5, 0)
    n = max(1, int(round(400 * scale)))
    nc = max(1, int(round(1e6 * scale ** 3)))
    spec = make_sim(rng, (n, n, n), (20.0, 20.0, 20.0), 8, dtype=dtype, bc="neumann",
                    n_cells=nc, cell_layout="core", sigma=800.0 * scale, core_fraction=0.7)
    return Workload(f"tumour-scale-{n}^3x8-{dtype}", [spec], 100, dtype,
                    "1e6 cells, 70% Gaussian core + 30% uniform")


def planar(n_sims: int = 32, edge: int = 512, dtype="f32") -> Workload:
    """A batch of n_sims two-dimensional simulations (grids edge x edge x 1 of
    10 um voxels: x and y solves only), 4 substrates each (D log-uniform
    [1e3, 1e5], lambda log-uniform [1e-3, 1]), zero-flux faces, rho0 i.i.d.
    U[0, 40]; 1e4 cells per simulation in a Gaussian disc (sigma 800 um);
    dt = 0.01, 200 steps."""
    sims = []
    for k in range(n_sims):
        rng = rng_for(6, k)
        sims.append(make_sim(rng, (edge, edge, 1), (10.0, 10.0, 10.0), 4, dtype=dtype, bc="neumann",
                             n_cells=10000, cell_layout="disc", sigma=800.0 * edge / 512))
    return Workload(f"planar-{n_sims}x{edge}^2x4-{dtype}", sims, 200, dtype,
                    "two-dimensional tissue sections, Gaussian disc of cells")


CONFIGS = {
    "plain": plain_fp64,
    "single": single_large,
    "batched": batched,
    "adjoint": differentiation,
    "tumour": tumour_scale,
    "planar": planar,
}
