// Host side of the three-dimensional projection: first-kind capacities of
// spheres and z-cylinders (Sec. 3.2 and 3.4 with a third index), and the
// unknowns and coefficient fields the device solve reads.
//
// Plane sections of the bodies are discs (or strips), whose area inside a
// rectangle is the integral over one coordinate of the part of the disc's
// chord inside the other coordinate's range: a sum of closed-form pieces
// split where the chord meets the rectangle's edges.  A volume is the
// integral along x of the sections by planes x = const (adaptive
// Gauss-Kronrod 7/15, split where the section circle is tangent to one of
// the box's lines or passes one of its corners, where the integrand has
// power-law kinks).

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "ccns3d.h"
#include "ccns3d_internal.h"
#include "ccns_internal.h"

namespace ccns {
namespace {

constexpr double kEpsRel = 1e-12;

// Integral of sqrt(rho^2 - t^2) from 0 to t, given the height s =
// sqrt(rho^2 - t^2): the angle comes from atan2(t, s), well conditioned where
// the height is known exactly (at the chord's ends), unlike asin(t / rho)
// near t = +-rho.
double arc_primitive(double t, double s, double rho) { return 0.5 * (t * s + rho * rho * std::atan2(t, s)); }

// Area of the disc of centre (a, b) and radius rho inside [ua, ub] x [va,
// vb]: the integral over u of the chord [b - s, b + s] (s = sqrt(rho^2 -
// (u - a)^2)) clipped to [va, vb], in closed-form pieces between the points
// where the chord's ends cross va or vb.
double disc_rect(double a, double b, double rho, double ua, double ub, double va, double vb) {
    if (!(rho > 0.0)) return 0.0;
    const double m = std::max(va - b, b - vb);  // the chord reaches [va, vb] where s > m
    if (m >= rho) return 0.0;
    const double w0 = m > 0.0 ? std::sqrt(rho * rho - m * m) : rho, s0 = std::max(m, 0.0);
    struct Pt {
        double u, s;  // abscissa and the chord's half-height there
    };
    auto edge = [&](double u) {
        const double t = u - a;
        return Pt{u, std::sqrt(std::max(rho * rho - t * t, 0.0))};
    };
    const Pt lo = a - w0 >= ua ? Pt{a - w0, s0} : edge(ua);
    const Pt hi = a + w0 <= ub ? Pt{a + w0, s0} : edge(ub);
    if (!(hi.u > lo.u)) return 0.0;
    Pt br[6];
    int nb = 0;
    br[nb++] = lo;
    auto add = [&](double d) {  // where s(u) = d: the chord's end crosses v = b +- d
        if (d >= 0.0 && d < rho) {
            const double w = std::sqrt(rho * rho - d * d);
            if (a - w > lo.u && a - w < hi.u) br[nb++] = Pt{a - w, d};
            if (a + w > lo.u && a + w < hi.u) br[nb++] = Pt{a + w, d};
        }
    };
    add(vb - b);
    add(b - va);
    br[nb++] = hi;
    std::sort(br, br + nb, [](const Pt &x, const Pt &y) { return x.u < y.u; });
    double area = 0.0;
    for (int k = 0; k + 1 < nb; ++k) {
        const Pt p = br[k], q = br[k + 1];
        if (!(q.u > p.u)) continue;
        const double mid = 0.5 * (p.u + q.u) - a;
        const double sm = std::sqrt(std::max(rho * rho - mid * mid, 0.0));
        const double len = q.u - p.u, S = arc_primitive(q.u - a, q.s, rho) - arc_primitive(p.u - a, p.s, rho);
        const double top = (b + sm >= vb) ? vb * len : b * len + S;  // integral of min(vb, b + s)
        const double bot = (b - sm <= va) ? va * len : b * len - S;  // integral of max(va, b - s)
        area += top - bot;
    }
    return area;
}

struct Body {
    int kind;
    double cx, cy, cz, r;
};

// One G7K15 panel: the Kronrod value, and |Kronrod - Gauss| h as the error.
template <class F>
double gk15(const F &f, double p, double q, double &err) {
    const double c = 0.5 * (p + q), h = 0.5 * (q - p);
    double k = 0.0, g = 0.0;
    for (int i = 0; i < 8; ++i) {
        const double v = (i == 7) ? f(c) : f(c - h * kXK[i]) + f(c + h * kXK[i]);
        k += kWK[i] * v;
        if (i % 2 == 1) g += kWG[i / 2] * v;
    }
    err = std::fabs(k - g) * h;
    return k * h;
}

// Globally adaptive Gauss-Kronrod on [p, q]: the panel with the largest
// error estimate is halved until the estimates add up to at most tol, or
// the budget of panels is spent (next to a tangency the section area is
// known only to its rounding, about 1e-16 of the disc's area, and no split
// gets below that).
template <class F>
double adapt(const F &f, double p, double q, double tol) {
    struct Pan {
        double p, q, v, e;
    };
    constexpr int MAX_PANELS = 256;
    Pan pan[MAX_PANELS];
    int n = 0;
    double e0;
    const double v0 = gk15(f, p, q, e0);
    pan[n++] = Pan{p, q, v0, e0};
    for (;;) {
        double esum = 0.0;
        int worst = 0;
        for (int k = 0; k < n; ++k) {
            esum += pan[k].e;
            if (pan[k].e > pan[worst].e) worst = k;
        }
        if (esum <= tol || n + 1 >= MAX_PANELS) break;
        const Pan w = pan[worst];
        const double m = 0.5 * (w.p + w.q);
        if (!(m > w.p && m < w.q)) break;
        double e1, e2;
        const double v1 = gk15(f, w.p, m, e1), v2 = gk15(f, m, w.q, e2);
        pan[worst] = Pan{w.p, m, v1, e1};
        pan[n++] = Pan{m, w.q, v2, e2};
    }
    double v = 0.0;
    for (int k = 0; k < n; ++k) v += pan[k].v;
    return v;
}

// Solid volume of a sphere inside a box: the integral along x of the area
// of the section disc (radius sqrt(r^2 - (x - cx)^2), centre (cy, cz))
// inside [ya, yb] x [za, zb].
double sphere_box_solid(const Body &b, double xa, double xb, double ya, double yb, double za, double zb) {
    const double lo = std::max(xa, b.cx - b.r), hi = std::min(xb, b.cx + b.r);
    if (hi <= lo) return 0.0;
    auto f = [&](double x) {
        const double d = x - b.cx, rho2 = b.r * b.r - d * d;
        return rho2 > 0.0 ? disc_rect(b.cy, b.cz, std::sqrt(rho2), ya, yb, za, zb) : 0.0;
    };
    std::vector<double> pts{lo, hi};
    const double dy[2] = {ya - b.cy, yb - b.cy}, dz[2] = {za - b.cz, zb - b.cz};
    std::vector<double> ds;
    for (double v : dy) ds.push_back(std::fabs(v));
    for (double v : dz) ds.push_back(std::fabs(v));
    for (double u : dy)
        for (double v : dz) ds.push_back(std::sqrt(u * u + v * v));
    for (double d : ds)
        if (d < b.r) {
            const double w = std::sqrt(b.r * b.r - d * d);
            for (double x : {b.cx - w, b.cx + w})
                if (x > lo && x < hi) pts.push_back(x);
        }
    std::sort(pts.begin(), pts.end());
    const double tol = 1e-14 * (xb - xa) * (yb - ya) * (zb - za);
    double s = 0.0;
    for (size_t k = 0; k + 1 < pts.size(); ++k) {
        const double p = pts[k], q = pts[k + 1];
        if (q - p <= 1e-10 * (xb - xa)) {
            s += (q - p) * f(0.5 * (p + q));  // pieces between break points equal up to rounding
        } else {
            s += adapt(f, p, q, tol);
        }
    }
    return s;
}

bool box_meets(const Body &b, double xa, double xb, double ya, double yb, double za, double zb) {
    // distance from the axis (cylinder) or centre (sphere) to the box
    auto dist1 = [](double c, double a, double e) { return c < a ? a - c : (c > e ? c - e : 0.0); };
    const double dx = dist1(b.cx, xa, xb), dy = dist1(b.cy, ya, yb);
    const double dz = b.kind == CCNS3_SPHERE ? dist1(b.cz, za, zb) : 0.0;
    return dx * dx + dy * dy + dz * dz < b.r * b.r;
}

double box_fluid(const std::vector<Body> &bodies, double xa, double xb, double ya, double yb, double za, double zb) {
    const double vol = (xb - xa) * (yb - ya) * (zb - za);
    double solid = 0.0;
    for (const Body &b : bodies) {
        if (!box_meets(b, xa, xb, ya, yb, za, zb)) continue;
        if (b.kind == CCNS3_ZCYLINDER)
            solid += (zb - za) * disc_rect(b.cx, b.cy, b.r, xa, xb, ya, yb);
        else
            solid += sphere_box_solid(b, xa, xb, ya, yb, za, zb);
    }
    return vol - solid;
}

// Solid area of the rectangle [ua, ub] x [va, vb] in the plane
// {coordinate `axis` = pos}; (u, v) = (y, z), (x, z) or (x, y).
double plane_solid(const std::vector<Body> &bodies, int axis, double pos, double ua, double ub, double va, double vb) {
    double area = 0.0;
    for (const Body &b : bodies) {
        if (b.kind == CCNS3_ZCYLINDER) {
            if (axis == 2) {
                area += disc_rect(b.cx, b.cy, b.r, ua, ub, va, vb);
            } else {
                const double d = pos - (axis == 0 ? b.cx : b.cy);
                if (std::fabs(d) < b.r) {
                    const double w = std::sqrt(b.r * b.r - d * d), c = axis == 0 ? b.cy : b.cx;
                    area += std::max(0.0, std::min(ub, c + w) - std::max(ua, c - w)) * (vb - va);
                }
            }
            continue;
        }
        const double centre[3] = {b.cx, b.cy, b.cz};
        const double d = pos - centre[axis];
        if (std::fabs(d) >= b.r) continue;
        const double rho = std::sqrt(b.r * b.r - d * d);
        const double cu = axis == 0 ? b.cy : b.cx, cv = axis == 2 ? b.cy : b.cz;
        area += disc_rect(cu, cv, rho, ua, ub, va, vb);
    }
    return area;
}

bool grid_ok(const ccns3_grid *g) {
    return g && g->nx >= 1 && g->ny >= 1 && g->nz >= 1 && g->hx > 0.0 && g->hy > 0.0 && g->hz > 0.0 &&
           std::isfinite(g->x0) && std::isfinite(g->y0) && std::isfinite(g->z0) && std::isfinite(g->hx) &&
           std::isfinite(g->hy) && std::isfinite(g->hz) && (double)(g->nx + 2) * (g->ny + 2) * (g->nz + 2) < 4e9;
}

}  // namespace

bool grid3_valid(const ccns3_grid *g) { return grid_ok(g); }

ccns_status prepare3(const ccns3_grid &g, const ccns3_params &p, const double *caps, HostCoef3 &o, std::string &err) {
    const int X = g.nx + 2, Y = g.ny + 2, Z = g.nz + 2;
    const size_t N = (size_t)X * Y * Z;
    const double *V = caps, *A[3] = {caps + N, caps + 2 * N, caps + 3 * N};
    const double *Vf[3] = {caps + 4 * N, caps + 5 * N, caps + 6 * N};
    for (size_t k = 0; k < 7 * N; ++k)
        if (!(caps[k] >= 0.0) || !std::isfinite(caps[k])) {
            err = "capacity negative or not finite";
            return CCNS_EINVAL;
        }
    const double floor = p.mass_floor * g.hx * g.hy * g.hz;
    const size_t stride[3] = {1, (size_t)X, (size_t)X * Y};
    auto at = [&](int i, int j, int k) { return ((size_t)k * Y + j) * X + i; };
    std::vector<double> c[3], M[3];
    std::vector<char> act[3];
    for (int a = 0; a < 3; ++a) {
        c[a].assign(N, 0.0);
        M[a].assign(N, 0.0);
        act[a].assign(N, 0);
    }
    for (int k = 1; k <= g.nz; ++k)
        for (int j = 1; j <= g.ny; ++j)
            for (int i = 1; i <= g.nx; ++i) {
                const size_t q = at(i, j, k);
                const bool interior[3] = {i <= g.nx - 1, j <= g.ny - 1, k <= g.nz - 1};
                for (int a = 0; a < 3; ++a)
                    if (interior[a] && A[a][q] > 0.0 && Vf[a][q] > 0.0) {
                        act[a][q] = 1;
                        M[a][q] = std::max(Vf[a][q], floor);
                        c[a][q] = A[a][q] * A[a][q] / M[a][q];
                    }
            }
    // pressure unknowns: the largest set of fluid cells connected through
    // faces with c > 0 (breadth-first search, cells in index order)
    std::vector<int> comp(N, -1);
    std::vector<size_t> queue;
    int best = -1;
    size_t best_size = 0;
    int ncomp = 0;
    for (int k = 1; k <= g.nz; ++k)
        for (int j = 1; j <= g.ny; ++j)
            for (int i = 1; i <= g.nx; ++i) {
                const size_t s = at(i, j, k);
                if (!(V[s] > 0.0) || comp[s] >= 0) continue;
                queue.assign(1, s);
                comp[s] = ncomp;
                for (size_t h = 0; h < queue.size(); ++h) {
                    const size_t q = queue[h];
                    for (int a = 0; a < 3; ++a) {
                        // faces on the high side (q) and the low side (q - stride)
                        const size_t up = q + stride[a], dn = q - stride[a];
                        if (c[a][q] > 0.0 && V[up] > 0.0 && comp[up] < 0) {
                            comp[up] = ncomp;
                            queue.push_back(up);
                        }
                        if (c[a][dn] > 0.0 && V[dn] > 0.0 && comp[dn] < 0) {
                            comp[dn] = ncomp;
                            queue.push_back(dn);
                        }
                    }
                }
                if (queue.size() > best_size) {
                    best_size = queue.size();
                    best = ncomp;
                }
                ++ncomp;
            }
    std::vector<char> actp(N, 0);
    for (size_t q = 0; q < N; ++q) actp[q] = (best >= 0 && comp[q] == best) ? 1 : 0;
    for (int a = 0; a < 3; ++a) {
        o.c[a].assign(N, 0.0);
        o.g[a].assign(N, 0.0);
        o.a[a].assign(N, 0.0);
        for (size_t q = 0; q < N; ++q) {
            if (act[a][q]) o.a[a][q] = A[a][q];
            if (c[a][q] > 0.0 && actp[q] && actp[q + stride[a]]) {
                o.c[a][q] = c[a][q];
                o.g[a][q] = A[a][q] / M[a][q];
            }
        }
    }
    o.dinv.assign(N, 0.0);
    o.n_active = 0;
    for (int k = 1; k <= g.nz; ++k)
        for (int j = 1; j <= g.ny; ++j)
            for (int i = 1; i <= g.nx; ++i) {
                const size_t q = at(i, j, k);
                if (!actp[q]) continue;
                double d = 0.0;
                for (int a = 0; a < 3; ++a) d += o.c[a][q] + o.c[a][q - stride[a]];
                if (d > 0.0) {
                    o.dinv[q] = 1.0 / d;
                    ++o.n_active;
                }
            }
    return CCNS_OK;
}

}  // namespace ccns

using namespace ccns;

extern "C" {

size_t ccns3_caps_count(const ccns3_grid *g) {
    if (!grid_ok(g)) return 0;
    return (size_t)7 * (g->nx + 2) * (g->ny + 2) * (g->nz + 2);
}

ccns_status ccns3_capacities(const ccns3_grid *g, const ccns3_body *bodies, int nbodies, double *out) {
    if (!grid_ok(g) || !out || nbodies < 0 || (nbodies > 0 && !bodies)) return CCNS_EINVAL;
    std::vector<Body> bs;
    for (int q = 0; q < nbodies; ++q) {
        const ccns3_body &b = bodies[q];
        if ((b.kind != CCNS3_SPHERE && b.kind != CCNS3_ZCYLINDER) || !(b.r > 0.0) || !std::isfinite(b.r) ||
            !std::isfinite(b.cx) || !std::isfinite(b.cy) || !std::isfinite(b.cz))
            return CCNS_EINVAL;
        bs.push_back(Body{b.kind, b.cx, b.cy, b.cz, b.r});
    }
    const int X = g->nx + 2, Y = g->ny + 2, Z = g->nz + 2;
    const size_t N = (size_t)X * Y * Z;
    std::memset(out, 0, 7 * N * sizeof(double));
    double *V = out, *A[3] = {out + N, out + 2 * N, out + 3 * N}, *Vf[3] = {out + 4 * N, out + 5 * N, out + 6 * N};
    const double hx = g->hx, hy = g->hy, hz = g->hz, cell = hx * hy * hz;
    const double full_a[3] = {hy * hz, hx * hz, hx * hy};
#pragma omp parallel for schedule(dynamic, 1)
    for (int k = 1; k <= g->nz; ++k) {
        for (int j = 1; j <= g->ny; ++j)
            for (int i = 1; i <= g->nx; ++i) {
                const size_t q = ((size_t)k * Y + j) * X + i;
                const double xa = g->x0 + (i - 1) * hx, ya = g->y0 + (j - 1) * hy, za = g->z0 + (k - 1) * hz;
                const double xb = xa + hx, yb = ya + hy, zb = za + hz;
                V[q] = box_fluid(bs, xa, xb, ya, yb, za, zb);
                // the faces on the cell's high sides, and the low walls from the
                // first cells
                const double rect[3][4] = {{ya, yb, za, zb}, {xa, xb, za, zb}, {xa, xb, ya, yb}};
                const double hi[3] = {xb, yb, zb}, lo[3] = {xa, ya, za};
                const int idx[3] = {i, j, k};
                const size_t st[3] = {1, (size_t)X, (size_t)X * Y};
                for (int a = 0; a < 3; ++a) {
                    A[a][q] = full_a[a] - plane_solid(bs, a, hi[a], rect[a][0], rect[a][1], rect[a][2], rect[a][3]);
                    if (idx[a] == 1)
                        A[a][q - st[a]] =
                            full_a[a] - plane_solid(bs, a, lo[a], rect[a][0], rect[a][1], rect[a][2], rect[a][3]);
                }
                // control volumes of the interior faces on the high sides:
                // [x_i, x_{i+1}] etc., x_i the cell centres
                if (i < g->nx) Vf[0][q] = box_fluid(bs, xa + 0.5 * hx, xb + 0.5 * hx, ya, yb, za, zb);
                if (j < g->ny) Vf[1][q] = box_fluid(bs, xa, xb, ya + 0.5 * hy, yb + 0.5 * hy, za, zb);
                if (k < g->nz) Vf[2][q] = box_fluid(bs, xa, xb, ya, yb, za + 0.5 * hz, zb + 0.5 * hz);
            }
    }
    // rounding residues (a covered face, say) below 1e-12 of the full value
    for (size_t q = 0; q < N; ++q) {
        if (!(V[q] > kEpsRel * cell)) V[q] = 0.0;
        for (int a = 0; a < 3; ++a) {
            if (!(A[a][q] > kEpsRel * full_a[a])) A[a][q] = 0.0;
            if (!(Vf[a][q] > kEpsRel * cell)) Vf[a][q] = 0.0;
        }
    }
    return CCNS_OK;
}

}  // extern "C"
