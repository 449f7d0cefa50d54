"""Dense Kronecker reference for tiny grids: a third implementation of one
LOD step, independent of both the C oracle and the GPU library.

Each directional implicit operator is built as a full matrix on the whole grid
(I_z x I_y x T_x, and so on, with x the fastest index), where the zero-flux
second difference is formed as K = -G^T G from the forward-difference matrix G
of the line, and T = (1 + sigma) I - c K.  Its inverse is applied with a dense
LAPACK solve of the full 3-D system, not by line recurrences.  The Dirichlet
projection is a per-voxel mask built from face membership, and the sources are
applied cell by cell.  Only usable for grids of a few hundred voxels.
"""
from __future__ import annotations

import numpy as np

DECAY_ONCE, DECAY_THIRDS = 0, 1


def neumann_second_difference(n: int) -> np.ndarray:
    """K = -G^T G with (G u)_i = u_{i+1} - u_i: the discrete Laplacian whose
    boundary rows carry zero flux through the end faces."""
    if n == 1:
        return np.zeros((1, 1))
    G = np.zeros((n - 1, n))
    idx = np.arange(n - 1)
    G[idx, idx] = -1.0
    G[idx, idx + 1] = 1.0
    return -G.T @ G


def line_matrix(n: int, c: float, sigma: float) -> np.ndarray:
    return (1.0 + sigma) * np.eye(n) - c * neumann_second_difference(n)


def grid_operator(shape, axis: int, M: np.ndarray) -> np.ndarray:
    """M acting along one axis of the flattened field (v = i + nx*(j + ny*k))."""
    nx, ny, nz = shape
    factors = [np.eye(nz), np.eye(ny), np.eye(nx)]
    factors[2 - axis] = M
    return np.kron(factors[0], np.kron(factors[1], factors[2]))


def dirichlet_masks(shape, bc_kind, bc_value):
    """Per substrate: boolean mask of Dirichlet voxels and their values.  A
    voxel on several faces takes the value of the highest-numbered active face
    in the order x-, x+, y-, y+, z-, z+."""
    nx, ny, nz = shape
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    coords = [i.ravel(), j.ravel(), k.ravel()]
    n = (nx, ny, nz)
    masks, values = [], []
    for s in range(bc_kind.shape[0]):
        mask = np.zeros(nx * ny * nz, dtype=bool)
        val = np.zeros(nx * ny * nz)
        best = np.full(nx * ny * nz, -1)
        for face in range(6):
            if bc_kind[s, face] != 1:
                continue
            a, side = divmod(face, 2)
            on = coords[a] == (n[a] - 1 if side else 0)
            upd = on & (face > best)
            best[upd] = face
            val[upd] = bc_value[s, face]
            mask |= on
        masks.append(mask)
        values.append(val)
    return masks, values


def cell_voxel(pos, shape, h, lo) -> int:
    idx = []
    for a in range(3):
        t = np.floor((pos[a] - lo[a]) / h[a])
        if not (0 <= t < shape[a]):
            return -1
        idx.append(int(t))
    return idx[0] + shape[0] * (idx[1] + shape[1] * idx[2])


class DenseLOD:
    """Holds the dense operators of one simulation."""

    def __init__(self, shape, h, lo, D, lam, dt, bc_kind, bc_value, decay_mode=DECAY_ONCE, cells=None):
        self.shape = tuple(int(v) for v in shape)
        self.h = tuple(float(v) for v in h)
        self.lo = tuple(float(v) for v in lo)
        self.D = np.asarray(D, dtype=np.float64)
        self.lam = np.asarray(lam, dtype=np.float64)
        self.dt = float(dt)
        self.decay_mode = decay_mode
        self.ns = self.D.size
        self.N = int(np.prod(self.shape))
        self.ops = []  # ops[s][axis]: full-grid matrix of the axis solve
        for s in range(self.ns):
            sigma = self.lam[s] * self.dt / 3.0 if decay_mode == DECAY_THIRDS else 0.0
            per_axis = []
            for a in range(3):
                c = self.dt * self.D[s] / (self.h[a] * self.h[a])
                per_axis.append(grid_operator(self.shape, a, line_matrix(self.shape[a], c, sigma)))
            self.ops.append(per_axis)
        self.masks, self.values = dirichlet_masks(self.shape, np.asarray(bc_kind), np.asarray(bc_value))
        self.cells = []
        if cells is not None:
            vvox = self.h[0] * self.h[1] * self.h[2]
            for i in range(cells.n):
                v = cell_voxel(cells.pos[i], self.shape, self.h, self.lo)
                k = self.dt * cells.V[i] / vvox
                a = k * cells.S[i] * cells.rho_star[i]
                b = 1.0 + k * (cells.S[i] + cells.U[i])
                self.cells.append((v, a, b))

    def project(self, u, s):
        u = u.copy()
        u[self.masks[s]] = self.values[s][self.masks[s]]
        return u

    def step(self, rho):
        """rho: (n_sub, N) float64 -> new (n_sub, N)."""
        out = np.empty_like(rho)
        for s in range(self.ns):
            u = self.project(rho[s], s)
            u = np.linalg.solve(self.ops[s][0], u)
            if self.decay_mode == DECAY_ONCE:
                u = u / (1.0 + self.lam[s] * self.dt)
            u = self.project(u, s)
            u = np.linalg.solve(self.ops[s][1], u)
            u = self.project(u, s)
            u = np.linalg.solve(self.ops[s][2], u)
            u = self.project(u, s)
            out[s] = u
        for v, a, b in self.cells:
            if v < 0:
                continue
            out[:, v] = (out[:, v] + a) / b
        return out
