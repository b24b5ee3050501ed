"""Capacities of the first and second kind on the pressure grid and on the two
staggered velocity grids (Sec. 3.2 eq:volumefirstkind, eq:centroid,
eq:surfacefirstkindx/y; Sec. 3.3 eq:volumesecondkindx/y, eq:surfacesecondkindx/y;
Sec. 3.4 for the half-cell shifted grids).

Array layout (shared by every field in this package): arrays of shape
(ny+2, nx+2) indexed [j, i] with one ghost ring.  Cell (i, j) -> [j, i];
x-face (i+1/2, j) -> [j, i]; y-face (i, j+1/2) -> [j, i]; node
(i+1/2, j+1/2) -> [j, i].  Real cells are 1..nx x 1..ny; real x-faces are
i = 0..nx (i = 0 and nx lie on the left and right walls).

Fluid domain of each grid (the reading of the box boundary, which the paper
leaves open):
  pressure grid  : box = [x_1/2, x_nx+1/2] x [y_1/2, y_ny+1/2]
  x-velocity grid: box extended by hx/2 beyond the left and right walls
  y-velocity grid: box extended by hy/2 beyond the bottom and top walls
The characteristic function is 1 where the level set is positive and the
point lies in the open box.  One exception: the pressure-grid faces that lie
on the walls carry the prescribed normal velocity, so their wet length is
taken from the level set alone (the face counts as wetted from inside).
Segments on the boundary of a staggered grid's box (the node lines on the
tangential walls) are therefore dry.  An empty control volume has its
centroid at its geometric centre.

Two integration back-ends:
  CircleGeometry   closed-form integrals for non-overlapping circles (exact up
                   to rounding); used for the circle workloads and as the
                   independent check of the generic path.
  LevelSetGeometry height-function quadrature for any level set: the wet
                   length of vertical lines (roots by sign sampling, a
                   search for root pairs hidden between samples, and
                   bracketing) integrated across the rectangle by adaptive
                   Gauss-Kronrod quadrature, split where the interface meets
                   the rectangle's edges.  Limitation: a body feature thinner
                   than 1/16 of a control volume that crosses no sampled point
                   is missed.
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
from scipy.integrate import quad_vec
from scipy.optimize import brentq

from workloads import CIRCLE, GridSpec

from .levelset import make_phi

# ---------------------------------------------------------------------------
# closed-form disc integrals
# ---------------------------------------------------------------------------

def _disc_branch(cx, cy, r, sgn, x1, x2, ya, yb):
    """Integrals over x in [x1,x2] of g, x*g and g^2/2 with
    g(x) = clip(cy + sgn*s(x), ya, yb), s(x) = sqrt(r^2-(x-cx)^2).

    The free (unclipped) pieces are integrated in the polar angle of the
    circle, x = cx + r cos(t), s = r |sin(t)|, which stays well conditioned at
    the vertical tangents x = cx -+ r (the x-parametrised antiderivative
    involves asin near -+1 there)."""

    def theta(x, kind):
        # angle of the branch point above (sgn>0) or below (sgn<0) x
        if kind == "left":
            return math.pi if sgn > 0 else -math.pi
        if kind == "right":
            return 0.0
        d = x - cx
        w = math.sqrt(max((r - d) * (r + d), 0.0))
        t = math.atan2(w, d)
        return t if sgn > 0 else -t

    def I_s(ta, tb):
        # int s dx between the branch points of angles ta (left) and tb (right)
        # s dx = -r^2 sin^2 t dt (upper) and +r^2 sin^2 t dt (lower)
        F = lambda t: 0.5 * (t - math.sin(t) * math.cos(t))
        return (-sgn) * r * r * (F(tb) - F(ta))

    def I_xs(ta, tb):
        # int (x-cx) s dx = [-s^3/3]
        sa, sb = r * abs(math.sin(ta)), r * abs(math.sin(tb))
        return -(sb ** 3 - sa ** 3) / 3.0

    def Q(x):  # antiderivative of s^2
        return r * r * x - (x - cx) ** 3 / 3.0

    pts = [(x1, "left" if x1 == cx - r else "edge"), (x2, "right" if x2 == cx + r else "edge")]
    for d in (ya - cy, yb - cy):
        if sgn * d >= 0.0 and abs(d) <= r:
            w = math.sqrt(max((r - d) * (r + d), 0.0))
            for xb_ in (cx - w, cx + w):
                if x1 < xb_ < x2:
                    pts.append((xb_, "edge"))
    pts.sort(key=lambda p: p[0])
    a = mx = my = 0.0
    for (p, kp), (q, kq) in zip(pts[:-1], pts[1:]):
        if q <= p:
            continue
        xm = 0.5 * (p + q)
        gm = cy + sgn * math.sqrt(max((r - (xm - cx)) * (r + (xm - cx)), 0.0))
        if gm >= yb or gm <= ya:
            c = yb if gm >= yb else ya
            a += c * (q - p)
            mx += c * 0.5 * (q * q - p * p)
            my += 0.5 * c * c * (q - p)
        else:
            ta, tb = theta(p, kp), theta(q, kq)
            dS = I_s(ta, tb)
            a += cy * (q - p) + sgn * dS
            mx += cy * 0.5 * (q * q - p * p) + sgn * (cx * dS + I_xs(ta, tb))
            my += 0.5 * (cy * cy * (q - p) + 2.0 * cy * sgn * dS + (Q(q) - Q(p)))
    return a, mx, my


def disc_rect_moments(cx, cy, r, xa, xb, ya, yb):
    """Area and first moments of the open disc intersected with a rectangle."""
    x1, x2 = max(xa, cx - r), min(xb, cx + r)
    if x2 <= x1 or yb <= ya or cy + r <= ya or cy - r >= yb:
        return 0.0, 0.0, 0.0
    au, mxu, myu = _disc_branch(cx, cy, r, +1.0, x1, x2, ya, yb)
    al, mxl, myl = _disc_branch(cx, cy, r, -1.0, x1, x2, ya, yb)
    return au - al, mxu - mxl, myu - myl


class CircleGeometry:
    """Fluid = plane minus a set of non-overlapping discs."""

    def __init__(self, bodies):
        for b in bodies:
            if b.kind != CIRCLE:
                raise ValueError("CircleGeometry handles circles only")
        self.discs = [(b.cx, b.cy, b.a) for b in bodies]
        self.phi = make_phi(bodies)

    def rect(self, xa, xb, ya, yb):
        if xb <= xa or yb <= ya:
            return 0.0, 0.0, 0.0
        # moments about the rectangle's centre keep the cancellation between
        # the rectangle and the disc parts at the scale of the rectangle
        xc, yc = 0.5 * (xa + xb), 0.5 * (ya + yb)
        hx, hy = 0.5 * (xb - xa), 0.5 * (yb - ya)
        a = (xb - xa) * (yb - ya)
        mx = my = 0.0
        for cx, cy, r in self.discs:
            da, dmx, dmy = disc_rect_moments(cx - xc, cy - yc, r, -hx, hx, -hy, hy)
            a -= da
            mx -= dmx
            my -= dmy
        a = max(a, 0.0)
        return a, mx + xc * a, my + yc * a

    def vseg(self, x, ya, yb):
        if yb <= ya:
            return 0.0
        L = yb - ya
        for cx, cy, r in self.discs:
            d = x - cx
            if abs(d) < r:
                w = math.sqrt(r * r - d * d)
                L -= max(0.0, min(yb, cy + w) - max(ya, cy - w))
        return max(L, 0.0)

    def hseg(self, y, xa, xb):
        if xb <= xa:
            return 0.0
        L = xb - xa
        for cx, cy, r in self.discs:
            d = y - cy
            if abs(d) < r:
                w = math.sqrt(r * r - d * d)
                L -= max(0.0, min(xb, cx + w) - max(xa, cx - w))
        return max(L, 0.0)

    def needs_work(self, xa, xb, ya, yb):
        """False when the rectangle is certainly uncut (disc-free)."""
        for cx, cy, r in self.discs:
            if xa < cx + r and xb > cx - r and ya < cy + r and yb > cy - r:
                return True
        return False


# ---------------------------------------------------------------------------
# generic level-set quadrature
# ---------------------------------------------------------------------------

def sign_change_roots(f, a, b, n=16):
    """Sorted points in (a, b) where f changes between positive and
    non-positive.  f is vectorised.  Sign changes between samples are
    bracketed; a pair of roots hidden between samples is looked for near
    every local minimum of |f| by repeated zooming (33 samples a level)
    towards the extremum."""
    if b <= a:
        return []
    s = np.linspace(a, b, n + 1)
    v = f(s)
    pos = v > 0.0
    roots = []

    def g(t):
        return float(f(np.array([t]))[0])

    for k in range(n):
        if pos[k] != pos[k + 1]:
            if v[k + 1] == 0.0 and not pos[k + 1]:
                roots.append(float(s[k + 1]))
            else:
                roots.append(brentq(g, s[k], s[k + 1], xtol=1e-16 * max(1.0, abs(b)), rtol=8.9e-16, maxiter=200))
    av = np.abs(v)
    for k in range(n + 1):
        lo, hi = max(k - 1, 0), min(k + 1, n)
        if pos[lo] != pos[k] or pos[hi] != pos[k]:
            continue
        if av[k] > av[lo] or av[k] > av[hi]:
            continue
        if av[k] == av[lo] and av[k] == av[hi]:
            continue            # flat: no dip between the samples to search
        # zoom towards the extremum of f nearest zero on [s_lo, s_hi]: sample
        # 33 points, keep the two sample intervals around the best one, repeat
        sg = 1.0 if pos[k] else -1.0
        xl, xh = float(s[lo]), float(s[hi])
        xm = None
        for _ in range(16):
            t = np.linspace(xl, xh, 33)
            ft = f(t)
            flip = (ft > 0.0) != pos[k]
            if flip.any():
                xm = float(t[int(np.argmax(flip))])
                break
            m = int(np.argmin(sg * ft))
            xl, xh = float(t[max(m - 1, 0)]), float(t[min(m + 1, 32)])
            if xh - xl < 1e-15 * max(1.0, abs(xh)):
                break
        if xm is not None:
            roots.append(brentq(g, float(s[lo]), xm, xtol=1e-16, rtol=8.9e-16, maxiter=200))
            roots.append(brentq(g, xm, float(s[hi]), xtol=1e-16, rtol=8.9e-16, maxiter=200))
    roots = sorted(r for r in roots if a < r < b)
    merged = []
    for r in roots:
        if not merged or r - merged[-1] > 1e-13 * (b - a):
            merged.append(r)
    return merged


def fluid_intervals(f, a, b, n=16):
    """Sub-intervals of [a, b] on which f > 0."""
    if b <= a:
        return []
    pts = [a] + sign_change_roots(f, a, b, n) + [b]
    out = []
    for p, q in zip(pts[:-1], pts[1:]):
        if q > p and f(np.array([0.5 * (p + q)]))[0] > 0.0:
            out.append((p, q))
    return out


class LevelSetGeometry:
    """Height-function quadrature of a generic level set."""

    def __init__(self, bodies=(), bbox_margin=0.0, phi=None):
        """Either a list of workload bodies, or a level-set function `phi`
        (vectorised, positive in the fluid) that is then integrated everywhere."""
        self.bodies = list(bodies)
        self.phi = make_phi(self.bodies) if phi is None else phi
        self.boxes = [b.bbox() for b in self.bodies]
        self.margin = bbox_margin
        self.everywhere = phi is not None

    def needs_work(self, xa, xb, ya, yb):
        if self.everywhere:
            return True
        m = self.margin
        for (x0, x1, y0, y1) in self.boxes:
            if xa < x1 + m and xb > x0 - m and ya < y1 + m and yb > y0 - m:
                return True
        return False

    def vseg(self, x, ya, yb):
        return sum(q - p for p, q in fluid_intervals(lambda y: self.phi(x, y), ya, yb))

    def hseg(self, y, xa, xb):
        return sum(q - p for p, q in fluid_intervals(lambda x: self.phi(x, y), xa, xb))

    def _count(self, x, ya, yb):
        return len(sign_change_roots(lambda y: self.phi(x, y), ya, yb))

    def rect(self, xa, xb, ya, yb):
        if xb <= xa or yb <= ya:
            return 0.0, 0.0, 0.0
        phi = self.phi
        bps = {xa, xb}
        for yy in (ya, yb):
            for r in sign_change_roots(lambda x: phi(x, yy), xa, xb):
                bps.add(r)
        # Vertical tangents change the number of roots on a vertical line:
        # probe that count on a uniform grid and just beside every edge
        # crossing (a tangent can sit closer to a crossing than any
        # quadrature node), and bisect wherever it changes.
        eps = 1e-12 * (xb - xa)
        probe = list(np.linspace(xa, xb, 17))
        for b0 in sorted(bps):
            if b0 - eps > xa:
                probe.append(b0 - eps)
            if b0 + eps < xb:
                probe.append(b0 + eps)
        probe = sorted(probe)
        cnt = [self._count(float(x), ya, yb) for x in probe]
        for k in range(len(probe) - 1):
            lo, hi = float(probe[k]), float(probe[k + 1])
            if cnt[k] == cnt[k + 1] or hi - lo <= 2.5 * eps:
                continue
            clo = cnt[k]
            while hi - lo > 1e-15 * max(1.0, abs(hi)):
                mid = 0.5 * (lo + hi)
                if self._count(mid, ya, yb) == clo:
                    lo = mid
                else:
                    hi = mid
            bps.add(0.5 * (lo + hi))
        pts = sorted(bps)

        def moments(x):
            ivs = fluid_intervals(lambda y: phi(float(x), y), ya, yb)
            L = sum(q - p for p, q in ivs)
            M = sum(0.5 * (q * q - p * p) for p, q in ivs)
            return np.array([L, x * L, M])

        # adaptive Gauss-Kronrod: vertical tangents of the interface that fall
        # between the sampled abscissas are resolved by the error control
        scale = (xb - xa) * (yb - ya)
        val, _ = quad_vec(moments, xa, xb, epsabs=1e-15 * scale, epsrel=1e-13,
                          points=pts[1:-1] or None, limit=4000, norm="max")
        area, mx, my = float(val[0]), float(val[1]), float(val[2])
        return area, mx, my


# ---------------------------------------------------------------------------
# capacities on the three grids
# ---------------------------------------------------------------------------

@dataclass
class GridCaps:
    """First- and second-kind capacities of one grid, in the CV-local naming:
    V, X, Y per control volume; E/N wet lengths of the east/north CV edges;
    Bv/Bh wet lengths of the vertical/horizontal lines through the centroid;
    We/Wn fluid areas between the centroids of a CV and its east/north
    neighbour."""

    V: np.ndarray
    X: np.ndarray
    Y: np.ndarray
    E: np.ndarray
    N: np.ndarray
    Bv: np.ndarray
    Bh: np.ndarray
    We: np.ndarray
    Wn: np.ndarray


def _grid_caps(geo, ex, ey, box, wall_faces_wet, eps_v):
    """Capacities of the control volumes [ex[i], ex[i+1]] x [ey[j], ey[j+1]],
    i = 0..len(ex)-2, j = 0..len(ey)-2, for fluid = {phi > 0} in the open box."""
    bx0, bx1, by0, by1 = box
    ni, nj = len(ex) - 1, len(ey) - 1
    shape = (nj, ni)
    V = np.zeros(shape)
    X = np.zeros(shape)
    Y = np.zeros(shape)
    E = np.zeros(shape)
    N = np.zeros(shape)
    Bv = np.zeros(shape)
    Bh = np.zeros(shape)
    We = np.zeros(shape)
    Wn = np.zeros(shape)

    def clip_rect(xa, xb, ya, yb):
        return max(xa, bx0), min(xb, bx1), max(ya, by0), min(yb, by1)

    def rect(xa, xb, ya, yb):
        xa, xb, ya, yb = clip_rect(xa, xb, ya, yb)
        if xb <= xa or yb <= ya:
            return 0.0, 0.0, 0.0
        if not geo.needs_work(xa, xb, ya, yb):
            return ((xb - xa) * (yb - ya), 0.5 * (xb * xb - xa * xa) * (yb - ya),
                    0.5 * (yb * yb - ya * ya) * (xb - xa))
        return geo.rect(xa, xb, ya, yb)

    def vseg(x, ya, yb, wet_wall=False):
        if not (bx0 < x < bx1) and not (wet_wall and bx0 <= x <= bx1):
            return 0.0
        ya, yb = max(ya, by0), min(yb, by1)
        if yb <= ya:
            return 0.0
        if not geo.needs_work(x, x, ya, yb):
            return yb - ya
        return geo.vseg(x, ya, yb)

    def hseg(y, xa, xb, wet_wall=False):
        if not (by0 < y < by1) and not (wet_wall and by0 <= y <= by1):
            return 0.0
        xa, xb = max(xa, bx0), min(xb, bx1)
        if xb <= xa:
            return 0.0
        if not geo.needs_work(xa, xb, y, y):
            return xb - xa
        return geo.hseg(y, xa, xb)

    # Control volumes and segments away from every body are evaluated in
    # closed form for the whole grid at once (the rectangle clipped to the
    # box); the per-entry integration below then revisits only entries that
    # may meet an interface.
    exa, eya = np.asarray(ex), np.asarray(ey)
    XA, YA = np.meshgrid(np.maximum(exa[:-1], bx0), np.maximum(eya[:-1], by0))
    XB, YB = np.meshgrid(np.minimum(exa[1:], bx1), np.minimum(eya[1:], by1))
    wx_, wy_ = np.clip(XB - XA, 0, None), np.clip(YB - YA, 0, None)
    V[:] = wx_ * wy_
    full = V > eps_v
    Xc, Yc = np.meshgrid(0.5 * (exa[:-1] + exa[1:]), 0.5 * (eya[:-1] + eya[1:]))
    X[:] = np.where(full, 0.5 * (XA + XB), Xc)
    Y[:] = np.where(full, 0.5 * (YA + YB), Yc)
    V[~full] = 0.0

    def seg_len_v(xv, y0v, y1v, wet):
        inside = ((xv > bx0) & (xv < bx1)) | (wet & (xv >= bx0) & (xv <= bx1))
        return np.where(inside, np.clip(np.minimum(y1v, by1) - np.maximum(y0v, by0), 0, None), 0.0)

    def seg_len_h(yv, x0v, x1v, wet):
        inside = ((yv > by0) & (yv < by1)) | (wet & (yv >= by0) & (yv <= by1))
        return np.where(inside, np.clip(np.minimum(x1v, bx1) - np.maximum(x0v, bx0), 0, None), 0.0)

    EX0, EY0 = np.meshgrid(exa[:-1], eya[:-1])
    EX1, EY1 = np.meshgrid(exa[1:], eya[1:])
    E[:] = seg_len_v(EX1, EY0, EY1, wall_faces_wet)
    N[:] = seg_len_h(EY1, EX0, EX1, wall_faces_wet)

    def touched(xa, xb, ya, yb):
        return geo.needs_work(max(xa, bx0), min(xb, bx1), max(ya, by0), min(yb, by1))

    work = np.zeros(shape, dtype=bool)
    for j in range(nj):
        for i in range(ni):
            work[j, i] = touched(ex[i] - 1e-12, ex[i + 1] + 1e-12, ey[j] - 1e-12, ey[j + 1] + 1e-12)
    for j, i in zip(*np.nonzero(work)):
        a, mx, my = rect(ex[i], ex[i + 1], ey[j], ey[j + 1])
        if a > eps_v:
            V[j, i] = a
            X[j, i] = min(max(mx / a, ex[i]), ex[i + 1])
            Y[j, i] = min(max(my / a, ey[j]), ey[j + 1])
        else:
            V[j, i] = 0.0
            X[j, i] = 0.5 * (ex[i] + ex[i + 1])
            Y[j, i] = 0.5 * (ey[j] + ey[j + 1])
        E[j, i] = vseg(ex[i + 1], ey[j], ey[j + 1], wall_faces_wet)
        N[j, i] = hseg(ey[j + 1], ex[i], ex[i + 1], wall_faces_wet)
    Bv[:] = seg_len_v(X, EY0, EY1, False)
    Bh[:] = seg_len_h(Y, EX0, EX1, False)
    We[:, :-1] = np.clip(np.minimum(X[:, 1:], bx1) - np.maximum(X[:, :-1], bx0), 0, None) * wy_[:, :-1]
    Wn[:-1, :] = np.clip(np.minimum(Y[1:, :], by1) - np.maximum(Y[:-1, :], by0), 0, None) * wx_[:-1, :]
    # entries next to a worked control volume can be cut as well
    near = work.copy()
    near[:, :-1] |= work[:, 1:]
    near[:-1, :] |= work[1:, :]
    for j, i in zip(*np.nonzero(near)):
        Bv[j, i] = vseg(X[j, i], ey[j], ey[j + 1])
        Bh[j, i] = hseg(Y[j, i], ex[i], ex[i + 1])
        if i + 1 < ni:
            We[j, i] = rect(X[j, i], X[j, i + 1], ey[j], ey[j + 1])[0]
        if j + 1 < nj:
            Wn[j, i] = rect(ex[i], ex[i + 1], Y[j, i], Y[j + 1, i])[0]
    return GridCaps(V, X, Y, E, N, Bv, Bh, We, Wn)


def _shift_east(a):
    """out[:, i] = a[:, i-1] (zero at i = 0)."""
    out = np.zeros_like(a)
    out[:, 1:] = a[:, :-1]
    return out


def _shift_north(a):
    out = np.zeros_like(a)
    out[1:, :] = a[:-1, :]
    return out


def capacities(grid: GridSpec, bodies, geo=None, eps_rel=1e-12):
    """All capacity arrays of the method, in the global (ny+2, nx+2) layout.

    Keys (paper symbol, location):
      V, X, Y      V_ij and centroid (cells)          eq:volumefirstkind, eq:centroid
      Ax, Ay       A^x_{i+1/2,j}, A^y_{i,j+1/2}         eq:surfacefirstkindx/y
      Bx, By       B^x_ij, B^y_ij (cells)             eq:surfacesecondkindx/y
      Wx, Wy       W^x_{i+1/2,j}, W^y_{i,j+1/2}         eq:volumesecondkindx/y
      Vu, Axx, Axy, Bxx, Bxy, Wxx, Wxy   x-velocity grid (Sec. 3.4):
                   V^x_{i+1/2,j}, A^xx_ij, A^xy_{i+1/2,j+1/2}, B^xx_{i+1/2,j},
                   B^xy_{i+1/2,j}, W^xx_ij, W^xy_{i+1/2,j+1/2}
      Vv, Ayy, Ayx, Byy, Byx, Wyy, Wyx   y-velocity grid:
                   V^y_{i,j+1/2}, A^yy_ij, A^yx_{i+1/2,j+1/2}, B^yy_{i,j+1/2},
                   B^yx_{i,j+1/2}, W^yy_ij, W^yx_{i+1/2,j+1/2}
    Capacities below eps_rel*h (lengths) or eps_rel*hx*hy (volumes) are set to 0.
    """
    bodies = list(bodies)
    if geo is None:
        if all(b.kind == CIRCLE for b in bodies):
            geo = CircleGeometry(bodies)
        else:
            geo = LevelSetGeometry(bodies, bbox_margin=max(grid.hx, grid.hy))
    nx, ny, hx, hy = grid.nx, grid.ny, grid.hx, grid.hy
    # cell-edge abscissas x_{i-1/2}, i = 0..nx+2, and cell centres x_i (one
    # ghost cell each side; on a stretched mesh the user's abscissas, Sec. 3.1)
    xe, ye = grid.edges(0), grid.edges(1)
    xc, yc = grid.centres(0), grid.centres(1)
    x0, x1, y0, y1 = xe[1], xe[nx + 1], ye[1], ye[ny + 1]
    # the velocity grids' boxes reach half a cell across their normal walls:
    # to the centres of the ghost cells
    epsV = eps_rel * hx * hy
    p = _grid_caps(geo, xe, ye, (x0, x1, y0, y1), True, epsV)
    u = _grid_caps(geo, xc, ye, (xc[0], xc[nx + 1], y0, y1), False, epsV)
    v = _grid_caps(geo, xe, yc, (x0, x1, yc[0], yc[ny + 1]), False, epsV)

    c = {
        "V": p.V, "X": p.X, "Y": p.Y,
        "Ax": p.E, "Ay": p.N, "Bx": p.Bv, "By": p.Bh, "Wx": p.We, "Wy": p.Wn,
        "Vu": u.V, "Xu": u.X, "Yu": u.Y,
        "Axx": _shift_east(u.E), "Axy": u.N, "Bxx": u.Bv, "Bxy": u.Bh,
        "Wxx": _shift_east(u.We), "Wxy": u.Wn,
        "Vv": v.V, "Xv": v.X, "Yv": v.Y,
        "Ayy": _shift_north(v.N), "Ayx": v.E, "Byy": v.Bh, "Byx": v.Bv,
        "Wyy": _shift_north(v.Wn), "Wyx": v.We,
    }
    for k in ("V", "Wx", "Wy", "Vu", "Wxx", "Wxy", "Vv", "Wyy", "Wyx"):
        c[k] = np.where(c[k] > epsV, c[k], 0.0)
    for k in ("Ax", "Bx", "Axx", "Bxx", "Ayx", "Byx"):
        c[k] = np.where(c[k] > eps_rel * hy, c[k], 0.0)
    for k in ("Ay", "By", "Ayy", "Byy", "Axy", "Bxy"):
        c[k] = np.where(c[k] > eps_rel * hx, c[k], 0.0)
    return c


CAPACITY_KEYS = ("V", "Ax", "Ay", "Bx", "By", "Wx", "Wy",
                 "Vu", "Axx", "Axy", "Bxx", "Bxy", "Wxx", "Wxy",
                 "Vv", "Ayy", "Ayx", "Byy", "Byx", "Wyy", "Wyx")
