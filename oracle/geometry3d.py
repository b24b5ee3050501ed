"""Capacities of the first kind in three dimensions: cell volumes V, face
areas A^x, A^y, A^z, and the volumes V^x, V^y, V^z of the half-cell shifted
control volumes of the three velocity components.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's definitions carry over to three dimensions by adding an index
(Sec. 2.1, after eq:differentiation):
  V_ijk            fluid volume of cell ijk                (eq:volumefirstkind)
  A^x_{i+1/2,j,k}  wet area of the x-face, a plane section  (eq:surfacefirstkindx)
  A^y, A^z         likewise                                (eq:surfacefirstkindy)
  V^x_{i+1/2,j,k}  fluid volume of the x-shifted cell [x_i, x_{i+1}] x
                   [y_{j-1/2}, y_{j+1/2}] x [z_{k-1/2}, z_{k+1/2}]   (Sec. 3.4)
The paper computes capacities with Vofi or Marching Cubes (Sec. 3.1) and
allows any method that integrates the characteristic function.  Here the
bodies are spheres and z-aligned circular cylinders (disjoint), and the
integrals are taken exactly up to rounding:
  * a plane section of a sphere or cylinder is a disc or a strip, whose
    intersection with a rectangle has a closed form (inclusion-exclusion of
    the disc's area below and to the left of each corner, `_disc_quadrant`);
  * a volume is the integral along z of the section areas, by adaptive
    quadrature (QUADPACK through scipy) split at every z where the section
    circle becomes tangent to an edge or passes a corner of the rectangle,
    to 1e-13 of the box volume or 1e-12 of the piece (the section areas
    carry a rounding noise of about 1e-16 of the disc's area).

Capacities below 1e-12 of the full face or cell (the rounding residue of a
covered face, say) are set to 0, as in two dimensions.

Array layout: (nz+2, ny+2, nx+2) indexed [k, j, i] as in the input module;
V on cells 1..n; A^x on x-faces i = 0..nx (j, k real), and likewise; V^x on
the interior x-faces i = 1..nx-1 (the wall faces carry no unknown; 0 there).
"""

from __future__ import annotations

import math
from typing import Dict, List

import numpy as np
from scipy import integrate

from workloads.three_d import ZCYLINDER, Body3, Grid3

EPS_REL = 1e-12


def _circle_primitive(t, rho, s=None):
    """Integral of sqrt(rho^2 - x^2) from -rho to t (t in [-rho, rho]).  s is
    the height sqrt(rho^2 - t^2) when it is known exactly (at the chord's
    ends): the angle then comes from atan2(t, s), which rounding of t / rho
    near +-1 would spoil by up to its square root."""
    t = min(max(t, -rho), rho)
    if s is None:
        s = math.sqrt(max(rho * rho - t * t, 0.0))
    return 0.5 * (t * s + rho * rho * math.atan2(t, s)) + 0.25 * math.pi * rho * rho


def _disc_quadrant(u, v, rho):
    """Area of the part of the disc of radius rho about the origin with
    x < u and y < v."""
    if rho <= 0.0 or u <= -rho or v <= -rho:
        return 0.0
    if v >= rho:
        return 2.0 * _circle_primitive(u, rho)
    av = abs(v)
    w = math.sqrt(rho * rho - v * v)   # the chord y = v meets the circle at x = +-w (height |v|)
    known = {-rho: 0.0, rho: 0.0, -w: av, w: av}

    def prim(x):
        return _circle_primitive(x, rho, known[x]) if x <= u else _circle_primitive(u, rho)

    def seg(a, b):                     # integral of sqrt(rho^2 - x^2) over [a, min(b, u)]
        return prim(b) - prim(a) if min(b, u) > a else 0.0

    def length(a, b):
        b = min(b, u)
        return b - a if b > a else 0.0

    # |x| < w: the column y in (-s, v); |x| > w: (-s, s) when v >= 0, empty
    # when v < 0
    area = v * length(-w, w) + seg(-w, w)
    if v >= 0.0:
        area += 2.0 * (seg(-rho, -w) + seg(w, rho))
    return area


def disc_rect_area(cx, cy, rho, xa, xb, ya, yb):
    """Area of the disc of centre (cx, cy) and radius rho inside the
    rectangle [xa, xb] x [ya, yb]."""
    if rho <= 0.0 or xb <= cx - rho or xa >= cx + rho or yb <= cy - rho or ya >= cy + rho:
        return 0.0
    q = lambda u, v: _disc_quadrant(u - cx, v - cy, rho)  # noqa: E731
    return q(xb, yb) - q(xa, yb) - q(xb, ya) + q(xa, ya)


def _section_radius(b: Body3, z):
    """Radius of the body's section by the plane at height z."""
    if b.kind == ZCYLINDER:
        return b.r
    d = z - b.cz
    return math.sqrt(b.r * b.r - d * d) if abs(d) < b.r else 0.0


def _breaks(b: Body3, za, zb, xa, xb, ya, yb):
    """Heights in (za, zb) where a sphere's section circle is tangent to a
    line of the rectangle or passes one of its corners, and its poles."""
    out = []
    ds = [abs(xa - b.cx), abs(xb - b.cx), abs(ya - b.cy), abs(yb - b.cy)]
    ds += [math.hypot(x - b.cx, y - b.cy) for x in (xa, xb) for y in (ya, yb)]
    for d in ds + [0.0]:
        if d < b.r:
            h = math.sqrt(b.r * b.r - d * d)
            for z in (b.cz - h, b.cz + h):
                if za < z < zb:
                    out.append(z)
    return sorted(set(out))


def box_fluid_volume(bodies: List[Body3], xa, xb, ya, yb, za, zb):
    """Fluid volume of the box [xa, xb] x [ya, yb] x [za, zb]: the box minus
    the integral over z of the bodies' section areas."""
    vol = (xb - xa) * (yb - ya) * (zb - za)
    solid = 0.0
    for b in bodies:
        if b.kind == ZCYLINDER:
            solid += (zb - za) * disc_rect_area(b.cx, b.cy, b.r, xa, xb, ya, yb)
            continue
        lo, hi = max(za, b.cz - b.r), min(zb, b.cz + b.r)
        if hi <= lo or disc_rect_area(b.cx, b.cy, b.r, xa, xb, ya, yb) == 0.0:
            continue
        pts = [lo] + _breaks(b, lo, hi, xa, xb, ya, yb) + [hi]
        f = lambda z: disc_rect_area(b.cx, b.cy, _section_radius(b, z), xa, xb, ya, yb)  # noqa: E731
        for a, c in zip(pts[:-1], pts[1:]):
            if c - a <= 1e-9 * (zb - za):
                # pieces between break points that differ by rounding: the
                # midpoint rule is exact to far below the tolerance there
                solid += (c - a) * f(0.5 * (a + c))
            else:
                val, _ = integrate.quad(f, a, c, epsabs=1e-13 * vol, epsrel=1e-12, limit=200)
                solid += val
    return vol - solid


def _plane_solid_area(bodies, axis, pos, ua, ub, va, vb):
    """Solid area of the rectangle in the plane {x_axis = pos}: (u, v) are the
    two other coordinates in the order (y, z) for x, (x, z) for y, (x, y)
    for z."""
    area = 0.0
    for b in bodies:
        if b.kind == ZCYLINDER:
            if axis == 2:
                area += disc_rect_area(b.cx, b.cy, b.r, ua, ub, va, vb)
            else:
                # the section by x = pos (or y = pos) is the strip |y - cy| < w
                # (or |x - cx| < w) across all z
                d = pos - (b.cx if axis == 0 else b.cy)
                if abs(d) < b.r:
                    w = math.sqrt(b.r * b.r - d * d)
                    c = b.cy if axis == 0 else b.cx
                    area += max(0.0, min(ub, c + w) - max(ua, c - w)) * (vb - va)
            continue
        centre = (b.cx, b.cy, b.cz)
        d = pos - centre[axis]
        if abs(d) >= b.r:
            continue
        rho = math.sqrt(b.r * b.r - d * d)
        others = [centre[a] for a in range(3) if a != axis]
        area += disc_rect_area(others[0], others[1], rho, ua, ub, va, vb)
    return area


def _near(bodies, xa, xb, ya, yb, za, zb):
    """Bodies whose bounding box meets the box (a cheap filter)."""
    out = []
    for b in bodies:
        zlo, zhi = (-math.inf, math.inf) if b.kind == ZCYLINDER else (b.cz - b.r, b.cz + b.r)
        if b.cx - b.r < xb and b.cx + b.r > xa and b.cy - b.r < yb and b.cy + b.r > ya and zlo < zb and zhi > za:
            out.append(b)
    return out


def capacities(g: Grid3, bodies: List[Body3]) -> Dict[str, np.ndarray]:
    """V, Ax, Ay, Az, Vx, Vy, Vz on the layout of the module docstring."""
    sh = g.shape
    # cell i spans [xe[i], xe[i] + hx] (i = 1..nx); its centre is xc[i]; the
    # x-face i+1/2 lies at xe[i] + hx
    xe = g.x0 + (np.arange(g.nx + 2) - 1.0) * g.hx
    ye = g.y0 + (np.arange(g.ny + 2) - 1.0) * g.hy
    ze = g.z0 + (np.arange(g.nz + 2) - 1.0) * g.hz
    xc, yc, zc = xe + 0.5 * g.hx, ye + 0.5 * g.hy, ze + 0.5 * g.hz
    out = {n: np.zeros(sh) for n in ("V", "Ax", "Ay", "Az", "Vx", "Vy", "Vz")}
    hx, hy, hz = g.hx, g.hy, g.hz
    for k in range(1, g.nz + 1):
        for j in range(1, g.ny + 1):
            for i in range(1, g.nx + 1):
                xa, ya, za = xe[i], ye[j], ze[k]
                xb, yb, zb = xa + hx, ya + hy, za + hz
                near = _near(bodies, xa, xb, ya, yb, za, zb)
                out["V"][k, j, i] = box_fluid_volume(near, xa, xb, ya, yb, za, zb) if near else hx * hy * hz
                # the face of this cell's high side in each direction (and the
                # low walls from cell 1)
                for axis, name in ((0, "Ax"), (1, "Ay"), (2, "Az")):
                    faces = [(i, j, k)]
                    if (i, j, k)[axis] == 1:
                        faces.append(tuple(v - (1 if a == axis else 0) for a, v in enumerate((i, j, k))))
                    for (fi, fj, fk) in faces:
                        if axis == 0:
                            pos, rect = xe[fi] + hx, (ya, yb, za, zb)
                        elif axis == 1:
                            pos, rect = ye[fj] + hy, (xa, xb, za, zb)
                        else:
                            pos, rect = ze[fk] + hz, (xa, xb, ya, yb)
                        full = (rect[1] - rect[0]) * (rect[3] - rect[2])
                        out[name][fk, fj, fi] = full - _plane_solid_area(bodies, axis, pos, *rect)
                # shifted control volumes of the interior faces on this cell's
                # high side
                if i < g.nx:
                    box = (xc[i], xc[i + 1], ya, yb, za, zb)
                    nb = _near(bodies, *box)
                    out["Vx"][k, j, i] = box_fluid_volume(nb, *box) if nb else hx * hy * hz
                if j < g.ny:
                    box = (xa, xb, yc[j], yc[j + 1], za, zb)
                    nb = _near(bodies, *box)
                    out["Vy"][k, j, i] = box_fluid_volume(nb, *box) if nb else hx * hy * hz
                if k < g.nz:
                    box = (xa, xb, ya, yb, zc[k], zc[k + 1])
                    nb = _near(bodies, *box)
                    out["Vz"][k, j, i] = box_fluid_volume(nb, *box) if nb else hx * hy * hz
    full = {"V": hx * hy * hz, "Vx": hx * hy * hz, "Vy": hx * hy * hz, "Vz": hx * hy * hz,
            "Ax": hy * hz, "Ay": hx * hz, "Az": hx * hy}
    for n, f in full.items():
        out[n] = np.where(out[n] > EPS_REL * f, out[n], 0.0)
    return out
