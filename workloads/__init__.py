"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds input recipes only: grid sizes, body parameters, seeded
noise fields and random capacity fields.  It contains none of the cut-cell
method's arithmetic (no capacities, operators or solvers), so that the
oracle and the device path can both draw their inputs from it without
sharing any part of the computation.

Bodies are plain parameter records.  Each side evaluates the level set of a
body with its own code.
"""

from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np


@dataclasses.dataclass(frozen=True)
class GridSpec:
    """Cartesian grid of nx*ny cells covering [x0, x0+lx] x [y0, y0+ly].

    Uniform unless xf / yf give the cell-edge abscissas x_{1/2} .. x_{nx+1/2}
    (nx+1 values, increasing, from x0 to x0+lx) and likewise in y: the
    user-defined abscissas of a rectilinear mesh.  hx, hy are then the
    smallest spacings (the scale of the time step, the small-volume floor and
    the divergence diagnostic)."""

    nx: int
    ny: int
    x0: float
    y0: float
    lx: float
    ly: float
    xf: Optional[tuple] = None
    yf: Optional[tuple] = None

    @property
    def uniform(self) -> bool:
        return self.xf is None and self.yf is None

    @property
    def hx(self) -> float:
        return self.lx / self.nx if self.xf is None else float(np.min(np.diff(self.xf)))

    @property
    def hy(self) -> float:
        return self.ly / self.ny if self.yf is None else float(np.min(np.diff(self.yf)))

    def edges(self, axis: int) -> np.ndarray:
        """Cell edges along x (axis 0) or y (axis 1) with one ghost cell on
        each side (whose width repeats the neighbouring cell's): n+3 values,
        entry i = x_{i-1/2}."""
        n, o, h, f = (self.nx, self.x0, self.lx / self.nx, self.xf) if axis == 0 else \
            (self.ny, self.y0, self.ly / self.ny, self.yf)
        if f is None:
            return o + (np.arange(n + 3) - 1.0) * h
        f = np.asarray(f, dtype=np.float64)
        return np.concatenate([[f[0] - (f[1] - f[0])], f, [f[-1] + (f[-1] - f[-2])]])

    def centres(self, axis: int) -> np.ndarray:
        """Cell centres x_i, i = 0 .. n+2 (ghost cells included; the last one
        lies beyond the ghost cell, one more mirrored width out): n+3 values."""
        n, o, h, f = (self.nx, self.x0, self.lx / self.nx, self.xf) if axis == 0 else \
            (self.ny, self.y0, self.ly / self.ny, self.yf)
        if f is None:
            return o + (np.arange(n + 3) - 0.5) * h
        e = self.edges(axis)
        c = 0.5 * (e[:-1] + e[1:])
        return np.concatenate([c, [e[-1] + 0.5 * (e[-1] - e[-2])]])


def stretched_edges(n: int, x0: float, length: float, amp: float, focus: float = 0.5) -> tuple:
    """n+1 edges of a smoothly stretched mesh on [x0, x0+length]:
    x = x0 + length (s + amp (sin(2 pi (s - c)) + sin(2 pi c)) / (2 pi)),
    s = k/n, so the spacing varies between (1 - amp) and (1 + amp) times the
    uniform one (0 <= amp < 1); the smallest spacing lies at x0 + focus
    length (s = c + 1/2 maps there; c = 0 for focus = 1/2)."""
    s = np.arange(n + 1) / n
    c = 0.0
    if focus != 0.5:
        # s_f - amp sin(2 pi s_f) / (2 pi) = focus, then c = s_f - 1/2
        lo, hi = 0.0, 1.0
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if mid - amp * np.sin(2.0 * np.pi * mid) / (2.0 * np.pi) < focus:
                lo = mid
            else:
                hi = mid
        c = 0.5 * (lo + hi) - 0.5
    if c == 0.0:
        x = x0 + length * (s + amp * np.sin(2.0 * np.pi * s) / (2.0 * np.pi))
    else:
        x = x0 + length * (s + amp * (np.sin(2.0 * np.pi * (s - c)) + np.sin(2.0 * np.pi * c)) / (2.0 * np.pi))
    x[0], x[-1] = x0, x0 + length
    return tuple(float(v) for v in x)


# Body kinds (the same integer codes are used by the C interface).
CIRCLE = 0
ELLIPSE = 1
NACA4 = 2


@dataclasses.dataclass(frozen=True)
class Body:
    """A solid body.  Fluid is where the body's level set is positive.

    circle : centre (cx, cy), radius a.
    ellipse: centre (cx, cy), semi-axes a (along the rotated x axis) and b,
             rotation angle `angle` (radians, counter-clockwise).
    naca4  : symmetric NACA 4-digit profile, leading edge at (cx, cy), chord
             `chord`, thickness ratio `t`, angle of attack `angle` (radians,
             nose-up: the trailing edge sits below the leading edge).
    """

    kind: int
    cx: float
    cy: float
    a: float = 0.0
    b: float = 0.0
    angle: float = 0.0
    chord: float = 0.0
    t: float = 0.0

    def ref_length(self) -> float:
        if self.kind == CIRCLE:
            return 2.0 * self.a
        if self.kind == ELLIPSE:
            return 2.0 * max(self.a, self.b)
        return self.chord

    def bbox(self):
        """Axis-aligned bounding box (xmin, xmax, ymin, ymax)."""
        if self.kind == CIRCLE:
            return (self.cx - self.a, self.cx + self.a, self.cy - self.a, self.cy + self.a)
        if self.kind == ELLIPSE:
            r = max(self.a, self.b)
            return (self.cx - r, self.cx + r, self.cy - r, self.cy + r)
        c, s = math.cos(self.angle), math.sin(self.angle)
        ht = 0.6 * self.t * self.chord
        xs = [self.cx, self.cx + self.chord * c]
        ys = [self.cy, self.cy - self.chord * s]
        return (min(xs) - ht, max(xs) + ht, min(ys) - ht, max(ys) + ht)


@dataclasses.dataclass
class Case:
    """One simulation request: grid, bodies, fluid properties and step count."""

    name: str
    grid: GridSpec
    bodies: List[Body]
    re: float
    u_inf: float = 1.0
    rho: float = 1.0
    cfl: float = 0.5
    steps: int = 10
    pcg_tol: float = 1e-10
    noise: float = 1e-2
    seed: int = 0
    # smallest volume the step divides by, as a fraction of a cell
    mass_floor: float = 0.05
    # walls (letters of "WESN") with a homogeneous Neumann velocity and a zero
    # pressure beyond them; the others hold the Dirichlet data
    outflow: str = ""

    @property
    def ref_length(self) -> float:
        return max(b.ref_length() for b in self.bodies) if self.bodies else 1.0

    @property
    def mu(self) -> float:
        return self.rho * self.u_inf * self.ref_length / self.re

    @property
    def tau(self) -> float:
        return self.cfl * min(self.grid.hx, self.grid.hy) / self.u_inf


# ---------------------------------------------------------------------------
# The named workloads
# ---------------------------------------------------------------------------

def cylinder_64() -> Case:
    """64x64 unit box, circle r=0.15 at the centre, Re=100, 10 steps, FP64."""
    g = GridSpec(64, 64, 0.0, 0.0, 1.0, 1.0)
    return Case("cylinder_64", g, [Body(CIRCLE, 0.5, 0.5, a=0.15)], re=100.0,
                steps=10, pcg_tol=1e-10, noise=1e-2, seed=1)


def channel_cylinder_2048() -> Case:
    """2048x1024 channel [0,20]x[0,10], cylinder D=1 at (5,5), Re=100, 200 steps."""
    g = GridSpec(2048, 1024, 0.0, 0.0, 20.0, 10.0)
    return Case("channel_cylinder_2048x1024", g, [Body(CIRCLE, 5.0, 5.0, a=0.5)],
                re=100.0, steps=200, pcg_tol=1e-10, noise=1e-3, seed=2)


def naca_4096() -> Case:
    """4096x2048 box [0,8]x[0,4], NACA0012 chord 1 at 5 degrees, Re=1000, 100 steps."""
    g = GridSpec(4096, 2048, 0.0, 0.0, 8.0, 4.0)
    body = Body(NACA4, 2.0, 2.0, angle=math.radians(5.0), chord=1.0, t=0.12)
    return Case("naca0012_4096x2048", g, [body], re=1000.0, steps=100,
                pcg_tol=1e-10, noise=1e-3, seed=3)


def flat_top_cylinder(n: int = 64, seed: int = 14, steps: int = 10) -> Case:
    """Unit box, circle of radius 0.3 centred on the line x = 0.5 whose top
    lies 0.02 h below a grid line: over the width of a cell the circle is
    nearly flat there, so the cells and face control volumes just below that
    line keep a fluid strip of 2-4% of a cell (velocity unknowns and pressure
    cells below a small-volume floor of 5%).  Re 100, CFL 0.25."""
    g = GridSpec(n, n, 0.0, 0.0, 1.0, 1.0)
    h = 1.0 / n
    r = 0.3
    top = math.floor((0.5 + r) / h) * h - 0.02 * h
    return Case(f"flat_top_cylinder_{n}", g, [Body(CIRCLE, 0.5, top - r, a=r)], re=100.0, steps=steps,
                cfl=0.25, pcg_tol=1e-10, noise=1e-2, seed=seed)


def ellipses(n: int = 96, seed: int = 12, steps: int = 10) -> Case:
    """Three ellipses in the unit box (the serving trace's body family):
    semi-axes 0.05-0.12, several orientations, at least 4h apart.  Re 200
    on twice the largest semi-axis, CFL 0.25."""
    g = GridSpec(n, n, 0.0, 0.0, 1.0, 1.0)
    bodies = [Body(ELLIPSE, 0.32, 0.33, a=0.12, b=0.06, angle=0.4),
              Body(ELLIPSE, 0.68, 0.40, a=0.09, b=0.05, angle=2.1),
              Body(ELLIPSE, 0.47, 0.70, a=0.10, b=0.07, angle=1.2)]
    return Case(f"ellipses3_{n}", g, bodies, re=200.0, steps=steps, cfl=0.25,
                pcg_tol=1e-10, noise=1e-2, seed=seed)


def pocket(n: int = 64, seed: int = 13, steps: int = 5) -> Case:
    """Four overlapping circles around (0.5, 0.5) that enclose a small fluid
    pocket cut off from the rest of the fluid (its cells are no pressure
    unknowns).  Re 100 on the circles' diameter, CFL 0.25."""
    g = GridSpec(n, n, 0.0, 0.0, 1.0, 1.0)
    d, r = 0.125, 0.1
    bodies = [Body(CIRCLE, 0.5 + d, 0.5, a=r), Body(CIRCLE, 0.5 - d, 0.5, a=r),
              Body(CIRCLE, 0.5, 0.5 + d, a=r), Body(CIRCLE, 0.5, 0.5 - d, a=r)]
    return Case(f"pocket_{n}", g, bodies, re=100.0, steps=steps, cfl=0.25,
                pcg_tol=1e-10, noise=1e-2, seed=seed)


def stretched_cylinder(n: int = 64, amp: float = 0.5, seed: int = 15, steps: int = 10) -> Case:
    """Channel [0,4]x[0,2] of 2n x n cells on a smoothly stretched mesh whose
    spacing is smallest through the middle, where a circle of diameter 0.5
    sits at (2, 1): the cells there are (1 - amp) and at the walls (1 + amp)
    times the uniform size (user-defined abscissas, Sec. 3.1).  Re 100 on
    the diameter, CFL 0.25 on the smallest spacing."""
    g = GridSpec(2 * n, n, 0.0, 0.0, 4.0, 2.0, xf=stretched_edges(2 * n, 0.0, 4.0, amp),
                 yf=stretched_edges(n, 0.0, 2.0, amp))
    return Case(f"stretched_cylinder_{2 * n}x{n}", g, [Body(CIRCLE, 2.0, 1.0, a=0.25)], re=100.0,
                steps=steps, cfl=0.25, pcg_tol=1e-10, noise=1e-2, seed=seed)


def outflow_cylinder(n: int = 48, seed: int = 16, steps: int = 10, outflow: str = "ESN") -> Case:
    """The paper's cylinder set-up on a small grid: channel [0,4]x[0,2] of
    2n x n cells, circle of diameter 0.5 at (1.2, 1), free stream entering
    through the west wall, homogeneous Neumann velocity with a zero pressure
    on the other three (outflow) walls.  Re 100 on the diameter, CFL 0.25."""
    g = GridSpec(2 * n, n, 0.0, 0.0, 4.0, 2.0)
    return Case(f"outflow_cylinder_{2 * n}x{n}", g, [Body(CIRCLE, 1.2, 1.0, a=0.25)], re=100.0, steps=steps,
                cfl=0.25, pcg_tol=1e-10, noise=1e-2, seed=seed, outflow=outflow)


def paper_cylinder(n: int = 1024, seed: int = 17, steps: int = 100) -> Case:
    """The set-up of the paper's cylinder case (Sec. 5), synthetic: box
    [0,16]x[0,8] in diameters, 2n x n cells on a mesh stretched around a
    cylinder of diameter 1 at (4, 4) (spacing 0.4 times the uniform one there,
    up to 1.6 times far from it), free stream entering through the west wall,
    outflow on the other three, Re 100, CFL 0.5 on the smallest spacing."""
    g = GridSpec(2 * n, n, 0.0, 0.0, 16.0, 8.0, xf=stretched_edges(2 * n, 0.0, 16.0, 0.6, focus=0.25),
                 yf=stretched_edges(n, 0.0, 8.0, 0.6, focus=0.5))
    return Case(f"paper_cylinder_{2 * n}x{n}", g, [Body(CIRCLE, 4.0, 4.0, a=0.5)], re=100.0, steps=steps,
                cfl=0.5, pcg_tol=1e-10, noise=1e-3, seed=seed, outflow="ESN")


def scaled_cylinder(nx: int, ny: int, lx: float, ly: float, seed: int = 2,
                    steps: int = 10) -> Case:
    """A smaller member of the channel-cylinder family (same geometry ratios)."""
    g = GridSpec(nx, ny, 0.0, 0.0, lx, ly)
    return Case(f"channel_cylinder_{nx}x{ny}", g,
                [Body(CIRCLE, lx / 4.0, ly / 2.0, a=0.05 * ly)], re=100.0,
                steps=steps, pcg_tol=1e-10, noise=1e-3, seed=seed)


def batched_cylinders(n: int = 256, seed: int = 4, steps: int = 50,
                      sizes=(128, 256, 512, 1024)) -> List[Case]:
    """Ragged batch: N in sizes, r~U[0.05,0.2], centre jittered, Re~U[50,200].
    CFL 0.25 (the paper's airfoil value): the smallest grids at the largest
    Reynolds numbers have cell Reynolds numbers above 10, where the explicit
    convection is unstable at 0.5."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        m = int(rng.choice(sizes))
        r = float(rng.uniform(0.05, 0.2))
        cx, cy = 0.5 + rng.uniform(-0.1, 0.1, size=2)
        re = float(rng.uniform(50.0, 200.0))
        g = GridSpec(m, m, 0.0, 0.0, 1.0, 1.0)
        out.append(Case(f"batch{k}_{m}", g, [Body(CIRCLE, float(cx), float(cy), a=r)],
                        re=re, steps=steps, pcg_tol=1e-10, noise=1e-2, cfl=0.25,
                        seed=seed * 100003 + k))
    return out


@dataclasses.dataclass
class Request:
    """A serving request: a case plus its arrival time (seconds)."""

    case: Case
    arrival: float


def serving_trace(n: int = 400, lam: float = 20.0, seed: int = 5, steps: int = 100,
                  nmin: int = 256, nmax: int = 2048) -> List[Request]:
    """Poisson arrivals; N log-uniform on [nmin, nmax] (multiple of 64);
    1-3 ellipses with semi-axes U[0.03,0.15], Re~U[50,500]; CFL 0.1: between
    close bodies the projected initial field reaches 5 u_inf, so a step set
    from u_inf at CFL 0.25 gives a local Courant number above 1 (a request
    with three ellipses then diverges within 50 steps)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for k in range(n):
        t += float(rng.exponential(1.0 / lam))
        m = int(round(2.0 ** rng.uniform(math.log2(nmin), math.log2(nmax)) / 64.0)) * 64
        m = max(nmin, min(nmax, m))
        h = 1.0 / m
        nb = int(rng.integers(1, 4))
        bodies: List[Body] = []
        tries = 0
        while len(bodies) < nb and tries < 1000:
            tries += 1
            a, b = rng.uniform(0.03, 0.15, size=2)
            ang = float(rng.uniform(0.0, math.pi))
            cx, cy = rng.uniform(0.2, 0.8, size=2)
            r = max(a, b)
            if cx - r < 4 * h or cx + r > 1 - 4 * h or cy - r < 4 * h or cy + r > 1 - 4 * h:
                continue
            ok = all(math.hypot(cx - o.cx, cy - o.cy) > r + max(o.a, o.b) + 4 * h for o in bodies)
            if ok:
                bodies.append(Body(ELLIPSE, float(cx), float(cy), a=float(a), b=float(b), angle=ang))
        re = float(rng.uniform(50.0, 500.0))
        g = GridSpec(m, m, 0.0, 0.0, 1.0, 1.0)
        out.append(Request(Case(f"req{k}_{m}", g, bodies, re=re, steps=steps, cfl=0.1,
                                pcg_tol=1e-10, noise=1e-2, seed=seed * 100003 + k), t))
    return out


# ---------------------------------------------------------------------------
# Seeded fields
# ---------------------------------------------------------------------------

def _near_body_mask(grid: GridSpec, bodies: List[Body], xs, ys, margin: float):
    """True where a point lies inside the margin-inflated bounding region of a body."""
    m = np.zeros(np.broadcast(xs, ys).shape, dtype=bool)
    for b in bodies:
        if b.kind == CIRCLE:
            m |= np.hypot(xs - b.cx, ys - b.cy) < b.a + margin
        else:
            x0, x1, y0, y1 = b.bbox()
            m |= (xs > x0 - margin) & (xs < x1 + margin) & (ys > y0 - margin) & (ys < y1 + margin)
    return m


def stream_noise(case: Case) -> np.ndarray:
    """Seeded stream-function noise on nodes, shape (ny+2, nx+2), node (i+1/2, j+1/2)
    stored at [j, i].  Values are i.i.d. U[-1,1] scaled by noise*u_inf*h and set
    to zero within 3h of the walls and of every body."""
    g = case.grid
    rng = np.random.default_rng(case.seed)
    psi = rng.uniform(-1.0, 1.0, size=(g.ny + 2, g.nx + 2))
    h = min(g.hx, g.hy)
    xs = g.edges(0)[1:]      # node (i+1/2, j+1/2) at [j, i]
    ys = g.edges(1)[1:]
    X, Y = np.meshgrid(xs, ys)
    wall = (X < g.x0 + 3 * h) | (X > g.x0 + g.lx - 3 * h) | (Y < g.y0 + 3 * h) | (Y > g.y0 + g.ly - 3 * h)
    body = _near_body_mask(g, case.bodies, X, Y, 3 * h)
    psi[wall | body] = 0.0
    return psi * (case.noise * case.u_inf * h)


def perturbation(case: Case):
    """Face velocity perturbation (ux', uy') built as the grid curl of the
    stream noise: ux'[j,i] = (psi[j,i]-psi[j-1,i])/dy_j at x-face (i+1/2, j),
    uy'[j,i] = -(psi[j,i]-psi[j,i-1])/dx_i at y-face (i, j+1/2), with the cell
    sizes dx_i, dy_j (hx, hy on a uniform grid).  Arrays (ny+2, nx+2)."""
    g = case.grid
    psi = stream_noise(case)
    ux = np.zeros_like(psi)
    uy = np.zeros_like(psi)
    if g.uniform:
        ux[1:, :] = (psi[1:, :] - psi[:-1, :]) / g.hy
        uy[:, 1:] = -(psi[:, 1:] - psi[:, :-1]) / g.hx
    else:
        dy = np.diff(g.edges(1))[: g.ny + 2]     # cell heights, rows 0 .. ny+1
        dx = np.diff(g.edges(0))[: g.nx + 2]
        ux[1:, :] = (psi[1:, :] - psi[:-1, :]) / dy[1:, None]
        uy[:, 1:] = -(psi[:, 1:] - psi[:, :-1]) / dx[None, 1:]
    return ux, uy


def dirichlet(case: Case):
    """Staggered Dirichlet data (Dx, Dy), arrays (ny+2, nx+2), x-face (i+1/2, j) at
    [j, i] and y-face (i, j+1/2) at [j, i].  Free stream Dx = u_inf, Dy = 0, except
    no-slip (0) on faces whose staggered control volume lies within 2h of a body."""
    g = case.grid
    h = min(g.hx, g.hy)
    # centres of the x-staggered control volumes: (x_{i+1/2}, y_j)
    xu = g.edges(0)[1:]
    yu = g.centres(1)[: g.ny + 2]
    XU, YU = np.meshgrid(xu, yu)
    dx = np.full((g.ny + 2, g.nx + 2), case.u_inf)
    dx[_near_body_mask(g, case.bodies, XU, YU, 2 * h + 0.5 * h)] = 0.0
    dy = np.zeros((g.ny + 2, g.nx + 2))
    return dx, dy


def random_capacities(nx: int, ny: int, seed: int, hx: float = 1.0, hy: float = 1.0,
                      zero_frac: float = 0.0):
    """Random positive capacity-like fields for operator-level tests (not a
    geometry): a dict of (ny+2, nx+2) arrays with values in [0.2h, h] for
    lengths and [0.2hxhy, hxhy] for volumes, and optionally a fraction of entries
    set to zero to mimic empty faces and cells."""
    rng = np.random.default_rng(seed)
    shape = (ny + 2, nx + 2)
    names_len_x = ["Ax", "Bx", "Axx", "Bxx", "Ayx", "Byx"]
    names_len_y = ["Ay", "By", "Ayy", "Byy", "Axy", "Bxy"]
    names_vol = ["V", "Vu", "Vv", "Wx", "Wy", "Wxx", "Wxy", "Wyy", "Wyx"]
    out = {}
    for n in names_len_x:
        out[n] = rng.uniform(0.2, 1.0, size=shape) * hy
    for n in names_len_y:
        out[n] = rng.uniform(0.2, 1.0, size=shape) * hx
    for n in names_vol:
        out[n] = rng.uniform(0.2, 1.0, size=shape) * hx * hy
    if zero_frac > 0.0:
        for n in list(out):
            z = rng.uniform(size=shape) < zero_frac
            out[n][z] = 0.0
    return out


def random_field(shape, seed: int, scale: float = 1.0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=shape) * scale
