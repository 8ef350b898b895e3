"""Seeded synthetic inputs for the orthonormalization-multigrid solve.

This module is the only code shared by the CPU oracle side and the GPU side.
It draws random numbers and describes problem geometry; it holds none of the
solver's arithmetic (no assembly, no basis functions, no multigrid).

Workload recipe (the paper's Poisson benchmark of Sec. 5.1 / Table 2, with the
sizes and coefficient fields of the workloads used here):

* unit cube split into ``nx*ny*nz`` cubes of side ``h = 1/nx`` (cells are cubes,
  so ``ny, nz`` must equal ``nx`` for a unit cube; other boxes are allowed);
* cell index ``i + nx*(j + ny*k)``, x fastest;
* piecewise-constant coefficient per cell: ``nu_in`` for cells whose centre is
  strictly inside a sphere, ``nu_out`` elsewhere (the paper's two-phase
  Poisson problem of Sec. 2 with a spherical interface);
* right-hand sides with iid N(0,1) entries in DOF order from
  ``numpy.random.default_rng(seed)``.
"""
from __future__ import annotations

import dataclasses
import numpy as np


def n_basis(p: int) -> int:
    """Number of total-degree-<=p polynomials in 3D: (p+1)(p+2)(p+3)/6."""
    return (p + 1) * (p + 2) * (p + 3) // 6


def default_levels(nx: int, ny: int, nz: int, max_coarse_cells: int = 512) -> int:
    """Number of agglomeration levels: halve every side while the current grid
    has more than ``max_coarse_cells`` cells and every side is even."""
    lv = 1
    while nx * ny * nz > max_coarse_cells and nx % 2 == 0 and ny % 2 == 0 and nz % 2 == 0:
        nx, ny, nz = nx // 2, ny // 2, nz // 2
        lv += 1
    return lv


@dataclasses.dataclass(frozen=True)
class Problem:
    """A Cartesian SIP-DG Poisson problem description (geometry only)."""
    nx: int
    ny: int
    nz: int
    p: int
    n_levels: int
    h: float
    penalty_c: float = 4.0

    @property
    def n_cells(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def bs(self) -> int:
        return n_basis(self.p)

    @property
    def n_dofs(self) -> int:
        return self.n_cells * self.bs


def make_problem(n: int, p: int, n_levels: int | None = None, ny: int | None = None,
                 nz: int | None = None) -> Problem:
    ny = n if ny is None else ny
    nz = n if nz is None else nz
    if n_levels is None:
        n_levels = default_levels(n, ny, nz)
    return Problem(nx=n, ny=ny, nz=nz, p=p, n_levels=n_levels, h=1.0 / n)


def nu_sphere(nx: int, ny: int, nz: int, h: float, center=(0.5, 0.5, 0.5), radius: float = 0.3,
              nu_in: float = 1.0, nu_out: float = 1000.0) -> np.ndarray:
    """Per-cell coefficient: ``nu_in`` if the cell centre is strictly inside the
    sphere, else ``nu_out``. Returned in cell order (x fastest), float64."""
    i = (np.arange(nx) + 0.5) * h
    j = (np.arange(ny) + 0.5) * h
    k = (np.arange(nz) + 0.5) * h
    zz, yy, xx = np.meshgrid(k, j, i, indexing="ij")
    d2 = (xx - center[0]) ** 2 + (yy - center[1]) ** 2 + (zz - center[2]) ** 2
    nu = np.where(d2 < radius * radius, nu_in, nu_out)
    return np.ascontiguousarray(nu.reshape(-1), dtype=np.float64)


def rhs(n_dofs: int, seed: int = 0) -> np.ndarray:
    """iid N(0,1) vector in DOF order (cell-major, basis index fastest)."""
    return np.random.default_rng(seed).standard_normal(n_dofs)


def multi_rhs(n_dofs: int, nrhs: int, seed: int = 0) -> np.ndarray:
    """``nrhs`` iid N(0,1) right-hand sides. Row j of the draw is right-hand
    side j; returned as an (n_dofs, nrhs) array with the RHS index fastest."""
    B = np.random.default_rng(seed).standard_normal((nrhs, n_dofs))
    return np.ascontiguousarray(B.T)


@dataclasses.dataclass(frozen=True)
class Instance:
    n: int
    radius: float
    center: tuple
    ratio: float
    seed: int


def instances(count: int = 16, seed: int = 2, sizes=(16, 24, 32, 48)) -> list[Instance]:
    """Uneven-size instances: cells per side uniform from ``sizes``, sphere
    radius U[0.15, 0.4], centre U[0.3, 0.7]^3, coefficient ratio 10^U[2, 4].
    Parameters are drawn per instance in that order; instance i's right-hand
    side uses seed 100 + i."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(sizes[int(rng.integers(0, len(sizes)))])
        radius = float(rng.uniform(0.15, 0.4))
        center = tuple(float(c) for c in rng.uniform(0.3, 0.7, size=3))
        ratio = float(10.0 ** rng.uniform(2.0, 4.0))
        out.append(Instance(n=n, radius=radius, center=center, ratio=ratio, seed=100 + i))
    return out


def random_spd_bsr(nx: int, ny: int, nz: int, bs: int, seed: int = 0, shift: float = 0.05):
    """A random symmetric positive definite block matrix on the 7-point cell
    stencil of an ``nx*ny*nz`` grid, in BSR form (sorted columns, diagonal block
    present). Built as a sum of random SPD edge couplings
    ``B_e (x) (e_i - e_j)(e_i - e_j)^T`` plus a random SPD diagonal block per
    cell, so it is SPD by construction. Generic test input, unrelated to the
    SIP discretisation.

    Returns ``(row_ptr int32[n+1], col_idx int32[nnzb], val float64[nnzb,bs,bs])``.
    """
    rng = np.random.default_rng(seed)
    n = nx * ny * nz

    def spd():
        g = rng.standard_normal((bs, bs))
        return g @ g.T / bs + shift * np.eye(bs)

    blocks: dict[tuple[int, int], np.ndarray] = {}

    def add(i, j, m):
        if (i, j) in blocks:
            blocks[(i, j)] += m
        else:
            blocks[(i, j)] = m.copy()

    for c in range(n):
        add(c, c, spd())
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                c = i + nx * (j + ny * k)
                for (di, dj, dk, stride) in ((1, 0, 0, 1), (0, 1, 0, nx), (0, 0, 1, nx * ny)):
                    if i + di < nx and j + dj < ny and k + dk < nz:
                        d = c + stride
                        m = spd()
                        add(c, c, m)
                        add(d, d, m)
                        add(c, d, -m)
                        add(d, c, -m)
    keys = sorted(blocks.keys())
    row_ptr = np.zeros(n + 1, dtype=np.int32)
    for (i, _j) in keys:
        row_ptr[i + 1] += 1
    row_ptr = np.cumsum(row_ptr).astype(np.int32)
    col_idx = np.array([j for (_i, j) in keys], dtype=np.int32)
    val = np.stack([blocks[k] for k in keys]).astype(np.float64)
    return row_ptr, col_idx, np.ascontiguousarray(val)
