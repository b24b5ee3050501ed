"""Seeded synthetic inputs of the three-dimensional projection step.

Input recipes only, as in the package's two-dimensional module: grid sizes,
body parameters and seeded face velocities.  No capacities, operators or
solvers are computed here, so the oracle and the device path can both draw
their inputs from this module.

Layout of every 3-D array: shape (nz+2, ny+2, nx+2) indexed [k, j, i] with one
ghost layer.  Cell (i, j, k) -> [k, j, i] for i in 1..nx (likewise j, k);
x-face (i+1/2, j, k) -> [k, j, i] for i in 0..nx (i = 0 and nx lie on the
walls), and likewise for y- and z-faces.
"""

from __future__ import annotations

import dataclasses
from typing import List

import numpy as np

# Body kinds (the same integer codes are used by the C interface).
SPHERE = 0
ZCYLINDER = 1


@dataclasses.dataclass(frozen=True)
class Grid3:
    """Uniform grid of nx*ny*nz cells covering [x0, x0+lx] x [y0, y0+ly] x
    [z0, z0+lz]."""

    nx: int
    ny: int
    nz: int
    x0: float
    y0: float
    z0: float
    lx: float
    ly: float
    lz: float

    @property
    def hx(self) -> float:
        return self.lx / self.nx

    @property
    def hy(self) -> float:
        return self.ly / self.ny

    @property
    def hz(self) -> float:
        return self.lz / self.nz

    @property
    def shape(self):
        return (self.nz + 2, self.ny + 2, self.nx + 2)

    @property
    def cells(self) -> int:
        return self.nx * self.ny * self.nz


@dataclasses.dataclass(frozen=True)
class Body3:
    """A solid body; fluid lies outside it.

    sphere   : centre (cx, cy, cz), radius r.
    zcylinder: the infinite cylinder of radius r about the line through
               (cx, cy) parallel to z (cz unused).
    Bodies of one case are disjoint."""

    kind: int
    cx: float
    cy: float
    cz: float
    r: float


@dataclasses.dataclass
class Case3:
    """One projection problem: grid, bodies, density, time step, the floor of
    the staggered volumes (a fraction of a cell) and the solver tolerance."""

    name: str
    grid: Grid3
    bodies: List[Body3]
    rho: float = 1.0
    tau: float = 1e-3
    mass_floor: float = 0.05
    tol: float = 1e-12
    seed: int = 0


def sphere_box(n: int = 24, r: float = 0.3, seed: int = 31, mass_floor: float = 0.05) -> Case3:
    """Unit box of n^3 cells with one sphere slightly off the centre."""
    g = Grid3(n, n, n, 0.0, 0.0, 0.0, 1.0, 1.0, 1.0)
    return Case3(f"sphere_{n}", g, [Body3(SPHERE, 0.5031, 0.4987, 0.5013, r)], tau=0.25 / n,
                 mass_floor=mass_floor, seed=seed)


def two_spheres(nx: int = 40, ny: int = 36, nz: int = 28, seed: int = 32, mass_floor: float = 0.05) -> Case3:
    """A ragged box (no dimension a multiple of the device's tile) with two
    spheres of different radii."""
    g = Grid3(nx, ny, nz, 0.0, 0.0, 0.0, 1.0, ny / nx, nz / nx)
    bodies = [Body3(SPHERE, 0.31, 0.42, 0.33, 0.17), Body3(SPHERE, 0.70, 0.47, 0.36, 0.12)]
    return Case3(f"two_spheres_{nx}x{ny}x{nz}", g, bodies, tau=0.25 / nx, mass_floor=mass_floor, seed=seed)


def zcylinder_box(nx: int = 24, ny: int = 20, nz: int = 6, seed: int = 33, mass_floor: float = 0.05) -> Case3:
    """A z-invariant case: a cylinder along z through a box, the third
    dimension of a 2-D circle case."""
    g = Grid3(nx, ny, nz, 0.0, 0.0, 0.0, 1.0, ny / nx, nz / nx)
    return Case3(f"zcylinder_{nx}x{ny}x{nz}", g, [Body3(ZCYLINDER, 0.47, 0.41, 0.0, 0.21)], tau=0.25 / nx,
                 mass_floor=mass_floor, seed=seed)


def tiny_box(seed: int = 34) -> Case3:
    """Fewer cells than one device tile in every direction."""
    g = Grid3(7, 5, 6, 0.0, 0.0, 0.0, 1.0, 5 / 7, 6 / 7)
    return Case3("tiny_7x5x6", g, [Body3(SPHERE, 0.52, 0.37, 0.41, 0.23)], tau=0.25 / 7, seed=seed)


def sphere_box_256(seed: int = 35) -> Case3:
    """The benchmark's size: 256^3 cells (16.8 M) around a sphere of radius
    0.3, one GPU's share of a larger box."""
    return sphere_box(256, 0.3, seed=seed)


def face_velocity(case: Case3):
    """Seeded U* on the three face grids: uniform in [-1, 1] on the interior
    faces, zero on the wall faces (the walls are at rest) and on the ghost
    layer.  Returns (Ux, Uy, Uz)."""
    g = case.grid
    rng = np.random.default_rng(case.seed)
    k, j, i = np.indices(g.shape)
    ci, cj, ck = (i >= 1) & (i <= g.nx), (j >= 1) & (j <= g.ny), (k >= 1) & (k <= g.nz)
    fi, fj, fk = (i >= 1) & (i <= g.nx - 1), (j >= 1) & (j <= g.ny - 1), (k >= 1) & (k <= g.nz - 1)
    interior = (fi & cj & ck, ci & fj & ck, ci & cj & fk)
    return tuple(np.where(m, rng.uniform(-1.0, 1.0, size=g.shape), 0.0) for m in interior)


def random_cells(case: Case3, seed: int) -> np.ndarray:
    """A seeded cell field (uniform in [-1, 1] on the real cells, zero on the
    ghost layer)."""
    g = case.grid
    rng = np.random.default_rng(seed)
    a = np.zeros(g.shape)
    a[1:-1, 1:-1, 1:-1] = rng.uniform(-1.0, 1.0, size=(g.nz, g.ny, g.nx))
    return a


def sample_cells(case: Case3, count: int, seed: int) -> List[tuple]:
    """Seeded sample of real cells (i, j, k) for checks at full size."""
    g = case.grid
    rng = np.random.default_rng(seed)
    return [(int(rng.integers(1, g.nx + 1)), int(rng.integers(1, g.ny + 1)), int(rng.integers(1, g.nz + 1)))
            for _ in range(count)]

