// Capacities of the first and second kind on the device (Sec. 3.2
// eq:volumefirstkind, eq:centroid, eq:surfacefirstkindx/y; Sec. 3.3
// eq:volumesecondkindx/y, eq:surfacesecondkindx/y; Sec. 3.4 for the two
// half-cell shifted velocity grids) for bodies bounded by conics: circles and
// rotated ellipses that do not overlap.
//
// Every capacity is the measure of the fluid part of an axis-aligned
// rectangle or segment.  For a conic that measure has a closed form: a
// vertical line x meets the ellipse in the chord y = cy + m X +- k s(X),
// X = x - cx, s(X) = sqrt(xm^2 - X^2), so the solid part of a rectangle is
// the integral over x of the chord clipped to the rectangle's rows, and the
// pieces between the points where a branch crosses a row boundary are
// integrated in closed form (s, X s and s^2 have elementary antiderivatives;
// the one of s is taken in the angle X = xm cos t, which stays well
// conditioned at the vertical tangents).  First moments give the centroids.
// The readings are those of the host computation: each grid's fluid lies in
// its own box, the pressure grid's wall faces are wet, an empty control
// volume has its centroid at its centre, a centroid is clamped into its
// control volume, a full rectangle or segment has the exact measures of its
// extent, and capacities below 1e-12 h (lengths) or 1e-12 hx hy (volumes)
// are 0.
//
// One thread per control volume; two launches per grid: the rectangle
// moments and the edge segments, then the segments through the centroids and
// the strips between neighbouring centroids (which need the neighbours'
// centroids, kept in the scratch buffer).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "ccns.h"

namespace ccns_caps {

constexpr int MAXB = 16;   // bodies per call
constexpr int CT = 256;    // threads per work-group

// A conic in the form of its vertical and horizontal chords.
struct Conic {
    double cx, cy;
    double m, k, xm;    // vertical line x: y = cy + m X +- k sqrt(xm^2 - X^2)
    double mh, kh, ym;  // horizontal line y: x = cx + mh Y +- kh sqrt(ym^2 - Y^2)
};
struct Conics {
    int n;
    Conic c[MAXB];
};

struct Mom {
    double a, mx, my;
};

// One control-volume grid: edges x0 + (i + ox) hx (i = 0..ni) and
// y0 + (j + oy) hy (j = 0..nj), with ox, oy = -1 (cell edges) or -1/2 (cell
// centres), evaluated in that form so that an edge on a wall is the wall's
// abscissa x0 + nx hx exactly; the grid's box and whether the box walls carry
// wet faces.
struct GridDesc {
    int ni, nj;         // control volumes (nx+2, ny+2)
    double x0, y0, ox, oy, hx, hy;
    double bx0, bx1, by0, by1;
    int wet;
};

__host__ __device__ inline double edge_x(const GridDesc &g, int i) { return g.x0 + ((double)i + g.ox) * g.hx; }
__host__ __device__ inline double edge_y(const GridDesc &g, int j) { return g.y0 + ((double)j + g.oy) * g.hy; }

// A length within 1e-9 relative of the spacing is the spacing (a full
// extent carries no rounding of the node coordinates).
__host__ __device__ inline double snap(double len, double h) { return fabs(len - h) <= 1e-9 * h ? h : len; }

__host__ __device__ inline double sroot(double xm, double X) { return sqrt(fmax((xm - X) * (xm + X), 0.0)); }

// Moments over x in [x1, x2] of g, x g and g^2 / 2, where
// g(x) = clip(cy + m X + sgn k s(X), ya, yb), X = x - cx (coordinates
// relative to the caller's origin).
__host__ __device__ Mom conic_branch(const Conic &c, double sgn, double x1, double x2, double ya, double yb) {
    double pts[6];
    int np = 0;
    pts[np++] = x1;
    // where the branch crosses a row boundary y = cy + d: roots of
    // (k^2 + m^2) X^2 - 2 d m X + d^2 - k^2 xm^2 = 0 (both branches; a root of
    // the other branch only splits a piece)
    const double q = c.k * c.k + c.m * c.m;
    for (int e = 0; e < 2; ++e) {
        const double d = (e == 0 ? ya : yb) - c.cy;
        const double disc = q * c.xm * c.xm - d * d;
        if (disc < 0.0) continue;
        const double r = c.k * sqrt(disc);
        for (int f = 0; f < 2; ++f) {
            const double x = c.cx + (d * c.m + (f == 0 ? -r : r)) / q;
            if (x > x1 && x < x2) pts[np++] = x;
        }
    }
    pts[np++] = x2;
    for (int i = 1; i < np; ++i)  // insertion sort (at most six points)
        for (int j = i; j > 0 && pts[j] < pts[j - 1]; --j) {
            const double t = pts[j];
            pts[j] = pts[j - 1];
            pts[j - 1] = t;
        }
    Mom o{0.0, 0.0, 0.0};
    const double xm2 = c.xm * c.xm;
    for (int i = 0; i + 1 < np; ++i) {
        const double p = pts[i], qq = pts[i + 1];
        if (!(qq > p)) continue;
        const double P = p - c.cx, Q = qq - c.cx, L = Q - P;
        const double Xm = 0.5 * (P + Q);
        const double gm = c.cy + c.m * Xm + sgn * c.k * sroot(c.xm, Xm);
        if (gm >= yb || gm <= ya) {
            const double v = gm >= yb ? yb : ya;
            o.a += v * L;
            o.mx += v * 0.5 * (qq - p) * (qq + p);
            o.my += 0.5 * v * v * L;
            continue;
        }
        const double sP = sroot(c.xm, P), sQ = sroot(c.xm, Q);
        // angles X = xm cos t in [0, pi]; int s dX = xm^2 (F(tP) - F(tQ)),
        // F(t) = (t - sin t cos t) / 2
        const double tP = atan2(sP, P), tQ = atan2(sQ, Q);
        const double FP = 0.5 * (tP - sP * P / xm2), FQ = 0.5 * (tQ - sQ * Q / xm2);
        const double S = xm2 * (FP - FQ);
        const double I1 = 0.5 * L * (Q + P);
        const double I2 = (Q * Q * Q - P * P * P) / 3.0;
        const double IXs = (sP * sP * sP - sQ * sQ * sQ) / 3.0;
        const double Iss = xm2 * L - I2;
        const double sk = sgn * c.k;
        const double a = c.cy * L + c.m * I1 + sk * S;
        o.a += a;
        o.mx += c.cx * a + c.cy * I1 + c.m * I2 + sk * IXs;
        o.my += 0.5 * (c.cy * c.cy * L + c.m * c.m * I2 + c.k * c.k * Iss) + c.cy * c.m * I1 + c.cy * sk * S +
                c.m * sk * IXs;
    }
    return o;
}

// Area and first moments of the open conic region inside [xa,xb] x [ya,yb].
__host__ __device__ Mom conic_rect(const Conic &c, double xa, double xb, double ya, double yb) {
    const double x1 = fmax(xa, c.cx - c.xm), x2 = fmin(xb, c.cx + c.xm);
    if (!(x2 > x1) || c.cy + c.ym <= ya || c.cy - c.ym >= yb) return Mom{0.0, 0.0, 0.0};
    const Mom u = conic_branch(c, 1.0, x1, x2, ya, yb);
    const Mom l = conic_branch(c, -1.0, x1, x2, ya, yb);
    return Mom{u.a - l.a, u.mx - l.mx, u.my - l.my};
}

// True when no conic's bounding box meets the open rectangle.
__host__ __device__ inline bool clear_of(const Conics &b, double xa, double xb, double ya, double yb) {
    for (int q = 0; q < b.n; ++q) {
        const Conic &c = b.c[q];
        if (xa < c.cx + c.xm && xb > c.cx - c.xm && ya < c.cy + c.ym && yb > c.cy - c.ym) return false;
    }
    return true;
}

// Fluid moments of a rectangle clipped to the grid's box (absolute
// coordinates).  The conic parts are integrated about the rectangle's
// centre, so that the cancellation between the rectangle and the conic parts
// happens at the scale of the rectangle.
__host__ __device__ Mom fluid_rect(const Conics &b, const GridDesc &g, double xa, double xb, double ya, double yb) {
    xa = fmax(xa, g.bx0);
    xb = fmin(xb, g.bx1);
    ya = fmax(ya, g.by0);
    yb = fmin(yb, g.by1);
    if (!(xb > xa) || !(yb > ya)) return Mom{0.0, 0.0, 0.0};
    if (!clear_of(b, xa, xb, ya, yb)) {
        const double xc = 0.5 * (xa + xb), yc = 0.5 * (ya + yb);
        const double hw = 0.5 * (xb - xa), hh = 0.5 * (yb - ya);
        double sa = 0.0, smx = 0.0, smy = 0.0;
        for (int q = 0; q < b.n; ++q) {
            Conic c = b.c[q];
            c.cx -= xc;
            c.cy -= yc;
            const Mom d = conic_rect(c, -hw, hw, -hh, hh);
            sa += d.a;
            smx += d.mx;
            smy += d.my;
        }
        if (sa != 0.0) {
            const double a = fmax((xb - xa) * (yb - ya) - sa, 0.0);
            return Mom{a, xc * a - smx, yc * a - smy};
        }
    }
    const double w = snap(xb - xa, g.hx), t = snap(yb - ya, g.hy);
    return Mom{w * t, 0.5 * (xb * xb - xa * xa) * t, 0.5 * (yb * yb - ya * ya) * w};
}

// Wet length of the vertical segment x, [ya, yb] (wet: the box's own walls
// count as inside).
__host__ __device__ double fluid_vseg(const Conics &b, const GridDesc &g, double x, double ya, double yb, bool wet) {
    const bool inside = (x > g.bx0 && x < g.bx1) || (wet && x >= g.bx0 && x <= g.bx1);
    if (!inside) return 0.0;
    ya = fmax(ya, g.by0);
    yb = fmin(yb, g.by1);
    if (!(yb > ya)) return 0.0;
    double cut = 0.0;
    for (int q = 0; q < b.n; ++q) {
        const Conic &c = b.c[q];
        const double X = x - c.cx;
        if (!(fabs(X) < c.xm)) continue;
        const double s = c.k * sroot(c.xm, X), yc = c.cy + c.m * X;
        cut += fmax(0.0, fmin(yb, yc + s) - fmax(ya, yc - s));
    }
    if (cut == 0.0) return snap(yb - ya, g.hy);
    return fmax(yb - ya - cut, 0.0);
}

__host__ __device__ double fluid_hseg(const Conics &b, const GridDesc &g, double y, double xa, double xb, bool wet) {
    const bool inside = (y > g.by0 && y < g.by1) || (wet && y >= g.by0 && y <= g.by1);
    if (!inside) return 0.0;
    xa = fmax(xa, g.bx0);
    xb = fmin(xb, g.bx1);
    if (!(xb > xa)) return 0.0;
    double cut = 0.0;
    for (int q = 0; q < b.n; ++q) {
        const Conic &c = b.c[q];
        const double Y = y - c.cy;
        if (!(fabs(Y) < c.ym)) continue;
        const double s = c.kh * sroot(c.ym, Y), xc = c.cx + c.mh * Y;
        cut += fmax(0.0, fmin(xb, xc + s) - fmax(xa, xc - s));
    }
    if (cut == 0.0) return snap(xb - xa, g.hx);
    return fmax(xb - xa - cut, 0.0);
}

// Output arrays of one grid, in the dense (ny+2) x (nx+2) layout.  The
// shifted ones (the velocity grids' east or north edges and strips, stored
// at the next control volume) are named by what the thread of control volume
// (i, j) writes: the value of control volume i-1 (east) or j-1 (north).
struct GridOut {
    double *V, *E, *N, *Bv, *Bh, *We, *Wn;
    int shiftE, shiftN;    // E and We stored one control volume east; N and Wn one north
    double *X, *Y;         // centroids (scratch)
};

// Control-volume moments and centroid, and the edge segments, of control
// volume k.
__host__ __device__ inline void caps_cv(const Conics &b, const GridDesc &g, const GridOut &o, double epsV, int k) {
    const int j = k / g.ni, i = k - j * g.ni;
    const double xa = edge_x(g, i), xb = edge_x(g, i + 1), ya = edge_y(g, j), yb = edge_y(g, j + 1);
    const Mom m = fluid_rect(b, g, xa, xb, ya, yb);
    double V = 0.0, X = 0.5 * (xa + xb), Y = 0.5 * (ya + yb);
    if (m.a > epsV) {
        V = m.a;
        X = fmin(fmax(m.mx / m.a, xa), xb);
        Y = fmin(fmax(m.my / m.a, ya), yb);
    }
    o.V[k] = V;
    o.X[k] = X;
    o.Y[k] = Y;
    const bool wet = g.wet != 0;
    // the east edge of control volume i (or, shifted, of i-1), the north edge
    // of row j (or of j-1)
    if (o.shiftE)
        o.E[k] = i > 0 ? fluid_vseg(b, g, xa, ya, yb, wet) : 0.0;
    else
        o.E[k] = fluid_vseg(b, g, xb, ya, yb, wet);
    if (o.shiftN)
        o.N[k] = j > 0 ? fluid_hseg(b, g, ya, xa, xb, wet) : 0.0;
    else
        o.N[k] = fluid_hseg(b, g, yb, xa, xb, wet);
}

// Segments through the centroid and the strips between neighbouring
// centroids (Sec. 3.3) of control volume k.
__host__ __device__ inline void caps_strips(const Conics &b, const GridDesc &g, const GridOut &o, int k) {
    const int j = k / g.ni, i = k - j * g.ni;
    const double xa = edge_x(g, i), xb = edge_x(g, i + 1), ya = edge_y(g, j), yb = edge_y(g, j + 1);
    o.Bv[k] = fluid_vseg(b, g, o.X[k], ya, yb, false);
    o.Bh[k] = fluid_hseg(b, g, o.Y[k], xa, xb, false);
    if (o.shiftE)
        o.We[k] = i > 0 ? fluid_rect(b, g, o.X[k - 1], o.X[k], ya, yb).a : 0.0;
    else
        o.We[k] = i + 1 < g.ni ? fluid_rect(b, g, o.X[k], o.X[k + 1], ya, yb).a : 0.0;
    if (o.shiftN)
        o.Wn[k] = j > 0 ? fluid_rect(b, g, xa, xb, o.Y[k - g.ni], o.Y[k]).a : 0.0;
    else
        o.Wn[k] = j + 1 < g.nj ? fluid_rect(b, g, xa, xb, o.Y[k], o.Y[k + g.ni]).a : 0.0;
}

__global__ __launch_bounds__(CT) void k_caps_cv(Conics b, GridDesc g, GridOut o, double epsV) {
    const int k = blockIdx.x * CT + threadIdx.x;
    if (k < g.ni * g.nj) caps_cv(b, g, o, epsV, k);
}

__global__ __launch_bounds__(CT) void k_caps_strips(Conics b, GridDesc g, GridOut o) {
    const int k = blockIdx.x * CT + threadIdx.x;
    if (k < g.ni * g.nj) caps_strips(b, g, o, k);
}

// Capacities below the thresholds are 0: nine volume arrays, then six
// lengths along y (x-faces) and six along x (y-faces), each of n entries.
__global__ __launch_bounds__(CT) void k_caps_threshold(double *caps, size_t n, double epsV, double epsX,
                                                       double epsY) {
    const int vol[] = {CCNS_CAP_V, CCNS_CAP_WX, CCNS_CAP_WY, CCNS_CAP_VU, CCNS_CAP_WXX, CCNS_CAP_WXY,
                       CCNS_CAP_VV, CCNS_CAP_WYY, CCNS_CAP_WYX};
    const int lx[] = {CCNS_CAP_AX, CCNS_CAP_BX, CCNS_CAP_AXX, CCNS_CAP_BXX, CCNS_CAP_AYX, CCNS_CAP_BYX};
    const int ly[] = {CCNS_CAP_AY, CCNS_CAP_BY, CCNS_CAP_AYY, CCNS_CAP_BYY, CCNS_CAP_AXY, CCNS_CAP_BXY};
    for (size_t k = (size_t)blockIdx.x * CT + threadIdx.x; k < n; k += (size_t)gridDim.x * CT) {
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            double *a = caps + (size_t)vol[q] * n;
            if (!(a[k] > epsV)) a[k] = 0.0;
        }
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            double *a = caps + (size_t)lx[q] * n;
            if (!(a[k] > epsX)) a[k] = 0.0;
            double *c = caps + (size_t)ly[q] * n;
            if (!(c[k] > epsY)) c[k] = 0.0;
        }
    }
}

// The conic of a body: vertical and horizontal chord forms of
// (u/a)^2 + (v/b)^2 < 1, u, v the coordinates along the body's axes.
Conic make_conic(const ccns_body &bd) {
    const double a = bd.a, b = bd.kind == CCNS_CIRCLE ? bd.a : bd.b;
    const double th = bd.kind == CCNS_CIRCLE ? 0.0 : bd.angle;
    const double c = std::cos(th), s = std::sin(th);
    Conic o;
    o.cx = bd.cx;
    o.cy = bd.cy;
    const double xm2 = a * a * c * c + b * b * s * s, ym2 = a * a * s * s + b * b * c * c;
    o.xm = std::sqrt(xm2);
    o.ym = std::sqrt(ym2);
    o.m = c * s * (a * a - b * b) / xm2;
    o.k = a * b / xm2;
    o.mh = c * s * (a * a - b * b) / ym2;
    o.kh = a * b / ym2;
    return o;
}

// The conics, the three grids and where their arrays go.
struct CapsPlan {
    Conics cs;
    GridDesc g[3];   // pressure, x-velocity, y-velocity grid
    GridOut o[3];
    size_t n;        // entries per array
    double epsV, epsX, epsY;
};

ccns_status plan_caps(const ccns_grid *grid, const ccns_body *bodies, int nbody, double *cap, double *scr,
                      CapsPlan &pl) {
    // the kernels place the edges at x0 + i hx: uniform grids only
    if (!grid || grid->nx < 2 || grid->ny < 2 || !(grid->hx > 0) || !(grid->hy > 0) || grid->xf || grid->yf ||
        nbody < 0 || nbody > MAXB || (nbody > 0 && !bodies))
        return CCNS_EINVAL;
    Conics &cs = pl.cs;
    cs.n = nbody;
    for (int q = 0; q < nbody; ++q) {
        const ccns_body &bd = bodies[q];
        if (bd.kind == CCNS_CIRCLE) {
            if (!(bd.a > 0)) return CCNS_EINVAL;
        } else if (bd.kind == CCNS_ELLIPSE) {
            if (!(bd.a > 0 && bd.b > 0)) return CCNS_EINVAL;
        } else {
            return CCNS_EINVAL;  // only conics have the closed form
        }
        cs.c[q] = make_conic(bd);
    }
    // the bodies must not overlap: their circumscribed discs are disjoint
    for (int p = 0; p < nbody; ++p)
        for (int q = p + 1; q < nbody; ++q) {
            const ccns_body &u = bodies[p], &v = bodies[q];
            const double ru = u.kind == CCNS_CIRCLE ? u.a : std::max(u.a, u.b);
            const double rv = v.kind == CCNS_CIRCLE ? v.a : std::max(v.a, v.b);
            if (std::hypot(u.cx - v.cx, u.cy - v.cy) <= ru + rv) return CCNS_EINVAL;
        }
    for (int q = nbody; q < MAXB; ++q) cs.c[q] = Conic{};
    const int nx = grid->nx, ny = grid->ny;
    const double hx = grid->hx, hy = grid->hy, x0 = grid->x0, y0 = grid->y0;
    const double x1 = x0 + nx * hx, y1 = y0 + ny * hy;
    const size_t n = (size_t)(nx + 2) * (ny + 2);
    pl.n = n;
    pl.epsV = 1e-12 * hx * hy;
    pl.epsX = 1e-12 * hy;
    pl.epsY = 1e-12 * hx;
    auto at = [&](int c) { return cap + (size_t)c * n; };
    // pressure grid: edges x_{i-1/2}; x-velocity grid: edges at the cell
    // centres, box extended by hx/2 across the left and right walls; the
    // y-velocity grid likewise in y
    pl.g[0] = GridDesc{nx + 2, ny + 2, x0, y0, -1.0, -1.0, hx, hy, x0, x1, y0, y1, 1};
    pl.g[1] = GridDesc{nx + 2, ny + 2, x0, y0, -0.5, -1.0, hx, hy, x0 - 0.5 * hx, x1 + 0.5 * hx, y0, y1, 0};
    pl.g[2] = GridDesc{nx + 2, ny + 2, x0, y0, -1.0, -0.5, hx, hy, x0, x1, y0 - 0.5 * hy, y1 + 0.5 * hy, 0};
    pl.o[0] = GridOut{at(CCNS_CAP_V), at(CCNS_CAP_AX), at(CCNS_CAP_AY), at(CCNS_CAP_BX), at(CCNS_CAP_BY),
                      at(CCNS_CAP_WX), at(CCNS_CAP_WY), 0, 0, scr, scr + n};
    pl.o[1] = GridOut{at(CCNS_CAP_VU), at(CCNS_CAP_AXX), at(CCNS_CAP_AXY), at(CCNS_CAP_BXX), at(CCNS_CAP_BXY),
                      at(CCNS_CAP_WXX), at(CCNS_CAP_WXY), 1, 0, scr + 2 * n, scr + 3 * n};
    pl.o[2] = GridOut{at(CCNS_CAP_VV), at(CCNS_CAP_AYX), at(CCNS_CAP_AYY), at(CCNS_CAP_BYX), at(CCNS_CAP_BYY),
                      at(CCNS_CAP_WYX), at(CCNS_CAP_WYY), 0, 1, scr + 4 * n, scr + 5 * n};
    return CCNS_OK;
}

}  // namespace ccns_caps

using namespace ccns_caps;

extern "C" {

size_t ccns_capacities_scratch_bytes(const ccns_grid *grid) {
    if (!grid || grid->nx < 2 || grid->ny < 2) return 0;
    return 6 * sizeof(double) * (size_t)(grid->nx + 2) * (size_t)(grid->ny + 2);
}

ccns_status ccns_capacities_device(const ccns_grid *grid, const ccns_body *bodies, int nbody, double *caps_dev,
                                   void *dev_scratch, size_t scratch_bytes, void *hip_stream) {
    if (!grid || !caps_dev || !dev_scratch) return CCNS_EINVAL;
    if (scratch_bytes < ccns_capacities_scratch_bytes(grid)) return CCNS_ENOMEM;
    CapsPlan pl;
    const ccns_status s = plan_caps(grid, bodies, nbody, caps_dev, (double *)dev_scratch, pl);
    if (s != CCNS_OK) return s;
    hipStream_t st = (hipStream_t)hip_stream;
    const int nb = (int)((pl.n + CT - 1) / CT);
    for (int q = 0; q < 3; ++q) k_caps_cv<<<nb, CT, 0, st>>>(pl.cs, pl.g[q], pl.o[q], pl.epsV);
    for (int q = 0; q < 3; ++q) k_caps_strips<<<nb, CT, 0, st>>>(pl.cs, pl.g[q], pl.o[q]);
    const int nt = (int)std::min<size_t>((pl.n + CT - 1) / CT, 4096);
    k_caps_threshold<<<nt, CT, 0, st>>>(caps_dev, pl.n, pl.epsV, pl.epsX, pl.epsY);
    if (hipGetLastError() != hipSuccess) return CCNS_EDEVICE;
    return CCNS_OK;
}

}  // extern "C"
