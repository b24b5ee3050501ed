"""Pins of the oracle's capacities (Sec. 3.2-3.4) against facts fixed by
geometry: exact areas and moments of circles, the surface conservation law
(eq:approximate) computed from independently found arc end-points, full-cell
values, the box-boundary reading, mirror symmetry, and the agreement of the
two independent integration back-ends."""

import math

import numpy as np
import pytest

import workloads as W
from oracle import geometry


def _grid(n=32, l=1.0):
    return W.GridSpec(n, n, 0.0, 0.0, l, l)


def test_no_body_full_cells_and_box_reading():
    g = W.GridSpec(6, 5, 0.0, 0.0, 1.2, 0.5)
    hx, hy = g.hx, g.hy
    c = geometry.capacities(g, [])
    s = np.s_[1:-1, 1:-1]
    assert np.allclose(c["V"][s], hx * hy, rtol=0, atol=1e-15)
    # pressure-grid wall faces are wetted (they carry the prescribed flux)
    assert np.allclose(c["Ax"][1:-1, 0:g.nx + 1], hy)
    assert np.allclose(c["Ay"][0:g.ny + 1, 1:-1], hx)
    assert np.allclose(c["Bx"][s], hy) and np.allclose(c["By"][s], hx)
    # x-grid: control volumes of the wall-normal faces extend outside (full)
    assert np.allclose(c["Vu"][1:-1, 0:g.nx + 1], hx * hy)
    # node lines on the tangential walls are dry; node volume there is half a cell
    assert np.all(c["Axy"][0, :] == 0.0) and np.all(c["Axy"][g.ny, :] == 0.0)
    assert np.allclose(c["Axy"][1:g.ny, 0:g.nx + 1], hx)
    assert np.allclose(c["Wxy"][0, 0:g.nx + 1], 0.5 * hx * hy)
    assert np.allclose(c["Wxy"][g.ny, 0:g.nx + 1], 0.5 * hx * hy)
    assert np.allclose(c["Wxy"][1:g.ny, 0:g.nx + 1], hx * hy)
    assert np.allclose(c["Wxx"][1:-1, 1:g.nx + 1], hx * hy)
    assert np.allclose(c["Bxx"][1:-1, 0:g.nx + 1], hy)
    assert np.allclose(c["Bxy"][1:-1, 0:g.nx + 1], hx)
    # y-grid mirrors it
    assert np.all(c["Ayx"][:, 0] == 0.0) and np.all(c["Ayx"][:, g.nx] == 0.0)
    assert np.allclose(c["Wyx"][0:g.ny + 1, 0], 0.5 * hx * hy)
    assert np.allclose(c["Wyx"][0:g.ny + 1, 1:g.nx], hx * hy)
    assert np.allclose(c["Vv"][0:g.ny + 1, 1:-1], hx * hy)


@pytest.mark.parametrize("n,r,cx,cy", [(64, 0.15, 0.5, 0.5), (40, 0.2113, 0.4711, 0.5302)])
def test_circle_area_and_moments_exact(n, r, cx, cy):
    g = _grid(n)
    body = W.Body(W.CIRCLE, cx, cy, a=r)
    c = geometry.capacities(g, [body])
    s = np.s_[1:-1, 1:-1]
    area = c["V"][s].sum()
    assert abs(area - (1.0 - math.pi * r * r)) < 1e-12
    # first moments: box moment minus disc moment
    assert abs((c["V"] * c["X"])[s].sum() - (0.5 - math.pi * r * r * cx)) < 1e-12
    assert abs((c["V"] * c["Y"])[s].sum() - (0.5 - math.pi * r * r * cy)) < 1e-12
    # staggered grids cover the box extended by half a cell across their own walls
    au = c["Vu"][1:-1, 0:n + 1].sum()
    assert abs(au - ((1.0 + 1.0 / n) * 1.0 - math.pi * r * r)) < 1e-12
    av = c["Vv"][0:n + 1, 1:-1].sum()
    assert abs(av - ((1.0 + 1.0 / n) * 1.0 - math.pi * r * r)) < 1e-12


def _arc_angles_in_rect(cx, cy, r, xa, xb, ya, yb):
    """Angle intervals of the circle lying inside the rectangle, found from the
    intersections of the circle with the four edge lines."""
    ts = [0.0, 2 * math.pi]
    for x in (xa, xb):
        d = (x - cx) / r
        if abs(d) <= 1:
            a = math.acos(d)
            ts += [a % (2 * math.pi), (-a) % (2 * math.pi)]
    for y in (ya, yb):
        d = (y - cy) / r
        if abs(d) <= 1:
            a = math.asin(d)
            ts += [a % (2 * math.pi), (math.pi - a) % (2 * math.pi)]
    ts = sorted(ts)
    out = []
    for t0, t1 in zip(ts[:-1], ts[1:]):
        tm = 0.5 * (t0 + t1)
        x, y = cx + r * math.cos(tm), cy + r * math.sin(tm)
        if xa < x < xb and ya < y < yb and t1 > t0:
            out.append((t0, t1))
    return out


def test_surface_conservation_law_per_cut_cell():
    """eq:approximate with the exact boundary: A+ - A- = -int_Gamma n ds, where n
    is the fluid's outward normal (pointing into the disc)."""
    n, r, cx, cy = 48, 0.23, 0.517, 0.489
    g = _grid(n)
    c = geometry.capacities(g, [W.Body(W.CIRCLE, cx, cy, a=r)])
    h = 1.0 / n
    checked = 0
    for j in range(1, n + 1):
        for i in range(1, n + 1):
            xa, xb = (i - 1) * h, i * h
            ya, yb = (j - 1) * h, j * h
            arcs = _arc_angles_in_rect(cx, cy, r, xa, xb, ya, yb)
            if not arcs:
                continue
            inx = sum(-r * (math.sin(t1) - math.sin(t0)) for t0, t1 in arcs)
            iny = sum(r * (math.cos(t1) - math.cos(t0)) for t0, t1 in arcs)
            sclx = c["Ax"][j, i] - c["Ax"][j, i - 1] + inx
            scly = c["Ay"][j, i] - c["Ay"][j - 1, i] + iny
            assert abs(sclx) < 1e-13 and abs(scly) < 1e-13
            # divergence theorem for the field (x, 0): V = x+ A+ - x- A- + int x n_x ds
            ixn = sum(-(cx * r * (math.sin(t1) - math.sin(t0))
                        + r * r * (0.5 * (t1 - t0) + 0.25 * (math.sin(2 * t1) - math.sin(2 * t0))))
                      for t0, t1 in arcs)
            vol = xb * c["Ax"][j, i] - xa * c["Ax"][j, i - 1] + ixn
            assert abs(vol - c["V"][j, i]) < 1e-14
            checked += 1
    assert checked > 50


def test_mirror_symmetry_centred_circle():
    n = 30
    g = _grid(n)
    c = geometry.capacities(g, [W.Body(W.CIRCLE, 0.5, 0.5, a=0.27)])
    s = np.s_[1:-1, 1:-1]
    V = c["V"][s]
    assert np.allclose(V, V[:, ::-1], atol=1e-15) and np.allclose(V, V[::-1, :], atol=1e-15)
    assert np.allclose(V, V.T, atol=1e-15)
    # x-face wet lengths mirror about x = 1/2: face i <-> face n - i
    Ax = c["Ax"][1:-1, 0:n + 1]
    assert np.allclose(Ax, Ax[:, ::-1], atol=1e-15)
    # second kind: W^x mirrors like the faces, B^x like the cells
    Wx = c["Wx"][1:-1, 1:n]
    assert np.allclose(Wx, Wx[:, ::-1], atol=1e-15)
    assert np.allclose(c["Bx"][s], c["Bx"][s][:, ::-1], atol=1e-15)


@pytest.mark.slow
def test_generic_quadrature_matches_closed_form():
    """The height-function path and the closed-form disc path are independent;
    on a circle they must agree on every capacity."""
    n = 6
    g = _grid(n)
    body = W.Body(W.CIRCLE, 0.48, 0.53, a=0.29)
    a = geometry.capacities(g, [body], geo=geometry.CircleGeometry([body]))
    b = geometry.capacities(g, [body], geo=geometry.LevelSetGeometry([body], bbox_margin=0.1))
    # second-kind capacities inherit the centroids' rounding through the
    # position of the line or strip they are measured on
    for k in geometry.CAPACITY_KEYS:
        assert np.allclose(a[k], b[k], rtol=0, atol=1e-11 * (1.0 / n)), k
    for k in ("X", "Y", "Xu", "Yu", "Xv", "Yv"):
        assert np.allclose(a[k], b[k], rtol=0, atol=1e-12 * (1.0 / n)), k


def test_mesh_aligned_wall_reproduces_worked_example_capacities():
    """A vertical wall inside a cell gives the capacities listed with the
    worked example of Sec. 2.3: V1 = 2 f hy, A on the dry faces 0, B = hy,
    W_{1/2} = f hy, W_{3/2} = g hy with g the centroid distance."""
    n = 8
    g = W.GridSpec(n, 4, 0.0, 0.0, 1.0, 0.5)
    hx, hy = g.hx, g.hy
    f = 0.3 * hx
    xw = 3 * hx - 2 * f        # wall inside cell 3, fluid to the right
    geo = geometry.LevelSetGeometry(phi=lambda x, y: np.asarray(x, dtype=float) - xw + 0 * np.asarray(y, dtype=float))
    c = geometry.capacities(g, [], geo=geo)
    j = 2
    assert c["V"][j, 2] == 0.0
    assert abs(c["V"][j, 3] - 2 * f * hy) < 1e-15
    assert c["Ax"][j, 1] == 0.0 and c["Ax"][j, 2] == 0.0
    assert abs(c["Ax"][j, 3] - hy) < 1e-15
    assert c["Bx"][j, 2] == 0.0 and abs(c["Bx"][j, 3] - hy) < 1e-15
    assert abs(c["Wx"][j, 2] - f * hy) < 1e-15
    gdist = f + 0.5 * hx
    assert abs(c["Wx"][j, 3] - gdist * hy) < 1e-15
    assert abs(c["Wx"][j, 4] - hx * hy) < 1e-15
