// Host computation of the capacities of the first and second kind
// (Sec. 3.2 eq:volumefirstkind, eq:centroid, eq:surfacefirstkindx/y;
// Sec. 3.3 eq:volumesecondkindx/y, eq:surfacesecondkindx/y; Sec. 3.4 for the
// two half-cell shifted velocity grids) from a level set.
//
// Every capacity is an integral of the fluid characteristic function over an
// axis-aligned rectangle or segment.  Segments: the fluid intervals of a line
// are found from sign changes of the level set on 16 samples, pairs of roots
// hidden between samples are searched for around each local minimum of |phi|
// (by zooming towards the extremum), and roots are refined by bisection.  Rectangles: the wet length of the
// vertical line through x (and its first moment in y) is integrated over x by
// adaptive Gauss-Kronrod (7/15 points) after splitting at the points where
// the interface meets the rectangle's top and bottom edges, below the
// interface's corners (a NACA section's trailing edge) and at vertical
// tangents (located where the number of crossings of a vertical line
// changes).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <queue>
#include <vector>

#include "ccns.h"
#include "ccns_internal.h"

namespace ccns {
namespace {

struct Fluid {
    const ccns_body *bodies;
    int nbody;
    ccns_levelset_fn fn;
    void *user;
    double lip = INFINITY;  // Lipschitz bound of the level set (see lipschitz())

    // A Lipschitz bound of the level set: 1 for circles (a distance), 1/min(a,b)
    // for ellipses (|grad| of sqrt((x/a)^2 + (y/b)^2) - 1), none for NACA
    // sections (the thickness slope is unbounded at the nose) or a user
    // function.  The level set is a minimum over bodies, bounded by the
    // largest of their bounds.
    double lipschitz() const {
        if (fn) return INFINITY;
        double L = 0.0;
        for (int k = 0; k < nbody; ++k) {
            const ccns_body &b = bodies[k];
            if (b.kind == CCNS_CIRCLE) L = std::max(L, 1.0);
            else if (b.kind == CCNS_ELLIPSE) L = std::max(L, 1.0 / std::min(b.a, b.b));
            else return INFINITY;
        }
        return L;
    }

    static double naca_yt(double xi, double t) {
        xi = std::min(std::max(xi, 0.0), 1.0);
        return 5.0 * t * (0.2969 * std::sqrt(xi) - 0.1260 * xi - 0.3516 * xi * xi +
                          0.2843 * xi * xi * xi - 0.1015 * xi * xi * xi * xi);
    }
    static double body(const ccns_body &b, double x, double y) {
        switch (b.kind) {
        case CCNS_CIRCLE:
            return std::hypot(x - b.cx, y - b.cy) - b.a;
        case CCNS_ELLIPSE: {
            double c = std::cos(b.angle), s = std::sin(b.angle);
            double xr = c * (x - b.cx) + s * (y - b.cy);
            double yr = -s * (x - b.cx) + c * (y - b.cy);
            return std::sqrt((xr / b.a) * (xr / b.a) + (yr / b.b) * (yr / b.b)) - 1.0;
        }
        default: {  // NACA 4-digit symmetric
            double c = std::cos(b.angle), s = std::sin(b.angle);
            double dx = x - b.cx, dy = y - b.cy;
            double xi = (dx * c - dy * s) / b.chord;
            double eta = (dx * s + dy * c) / b.chord;
            double f;
            if (xi < 0.0)
                f = std::hypot(xi, eta);
            else if (xi > 1.0)
                f = std::hypot(xi - 1.0, std::max(std::fabs(eta) - naca_yt(1.0, b.t), 0.0)) + 1e-300;
            else
                f = std::fabs(eta) - naca_yt(xi, b.t);
            return f * b.chord;
        }
        }
    }
    double operator()(double x, double y) const {
        double v = 1.0;
        bool any = false;
        for (int k = 0; k < nbody; ++k) {
            double f = body(bodies[k], x, y);
            v = any ? std::min(v, f) : f;
            any = true;
        }
        if (fn) {
            double f = fn(x, y, user);
            v = any ? std::min(v, f) : f;
            any = true;
        }
        return v;
    }
    // Axis-aligned box that contains every interface point of the bodies.
    void body_box(int k, double &x0, double &x1, double &y0, double &y1) const {
        const ccns_body &b = bodies[k];
        if (b.kind == CCNS_CIRCLE) {
            x0 = b.cx - b.a; x1 = b.cx + b.a; y0 = b.cy - b.a; y1 = b.cy + b.a;
        } else if (b.kind == CCNS_ELLIPSE) {
            double r = std::max(b.a, b.b);
            x0 = b.cx - r; x1 = b.cx + r; y0 = b.cy - r; y1 = b.cy + r;
        } else {
            double c = std::cos(b.angle), s = std::sin(b.angle), ht = 0.6 * b.t * b.chord;
            double xa = b.cx, xb = b.cx + b.chord * c, ya = b.cy, yb = b.cy - b.chord * s;
            x0 = std::min(xa, xb) - ht; x1 = std::max(xa, xb) + ht;
            y0 = std::min(ya, yb) - ht; y1 = std::max(ya, yb) + ht;
        }
    }
    // Abscissas of the interface's corners inside [xa, xb] x [ya, yb]: the
    // two ends of a NACA section's blunt trailing edge.  Elsewhere the
    // built-in interfaces are smooth.  (A user level set's corners are not
    // known; adaptive quadrature then has to find them.)
    void corners(double xa, double xb, double ya, double yb, std::vector<double> &xs) const {
        for (int k = 0; k < nbody; ++k) {
            const ccns_body &b = bodies[k];
            if (b.kind != CCNS_NACA4) continue;
            double c = std::cos(b.angle), s = std::sin(b.angle), ht = naca_yt(1.0, b.t);
            for (double eta : {-ht, ht}) {
                double x = b.cx + b.chord * (c + eta * s), y = b.cy + b.chord * (-s + eta * c);
                if (x > xa && x < xb && y >= ya && y <= yb) xs.push_back(x);
            }
        }
    }
    // +1 when the rectangle is certainly all fluid, -1 certainly all solid,
    // 0 when it may contain interface points: first the bodies' boxes, then,
    // with a Lipschitz bound, the level set at the centre against the
    // bound times the half diagonal.
    int classify(double xa, double xb, double ya, double yb, double margin) const {
        if (!maybe_cut(xa, xb, ya, yb, margin)) return 1;
        if (std::isfinite(lip)) {
            const double c = (*this)(0.5 * (xa + xb), 0.5 * (ya + yb));
            const double r = lip * 0.5 * std::hypot(xb - xa, yb - ya);
            if (c > r) return 1;
            if (c < -r) return -1;
        }
        return 0;
    }
    // True when the rectangle may contain interface points.
    bool maybe_cut(double xa, double xb, double ya, double yb, double margin) const {
        if (fn) return true;
        for (int k = 0; k < nbody; ++k) {
            double x0, x1, y0, y1;
            body_box(k, x0, x1, y0, y1);
            if (xa < x1 + margin && xb > x0 - margin && ya < y1 + margin && yb > y0 - margin)
                return true;
        }
        return false;
    }
};

// Fluid sub-intervals of [a, b] for g(s) > 0; returns the count (<= cap).
// lip: a Lipschitz bound of g along the line (INFINITY if unknown); a local
// minimum of |g| larger than lip times the sample spacing cannot hide a root
// pair, and is not searched.
template <class G>
int fluid_intervals(const G &g, double a, double b, double *lo, double *hi, int cap, double lip) {
    if (!(b > a)) return 0;
    const int n = 16;
    double s[n + 1], v[n + 1];
    for (int k = 0; k <= n; ++k) {
        s[k] = (k == n) ? b : a + (b - a) * (double)k / n;
        v[k] = g(s[k]);
    }
    double roots[64];
    int nr = 0;
    // bisection down to 1e-16 relative width, or to adjacent doubles
    auto bisect = [&](double l, double r) {
        bool pl = g(l) > 0.0;
        for (int it = 0; it < 200 && r - l > 1e-16 * std::max(1.0, std::fabs(r)); ++it) {
            double m = 0.5 * (l + r);
            if (!(m > l && m < r)) break;
            if ((g(m) > 0.0) == pl) l = m; else r = m;
        }
        return 0.5 * (l + r);
    };
    for (int k = 0; k < n; ++k)
        if ((v[k] > 0.0) != (v[k + 1] > 0.0) && nr < 62) roots[nr++] = bisect(s[k], s[k + 1]);
    // root pairs hidden between samples: look for a sign flip at local minima of |g|
    for (int k = 0; k <= n; ++k) {
        int l = std::max(k - 1, 0), r = std::min(k + 1, n);
        bool p = v[k] > 0.0;
        if ((v[l] > 0.0) != p || (v[r] > 0.0) != p) continue;
        if (std::fabs(v[k]) > std::fabs(v[l]) || std::fabs(v[k]) > std::fabs(v[r])) continue;
        if (std::fabs(v[k]) == std::fabs(v[l]) && std::fabs(v[k]) == std::fabs(v[r])) continue;  // flat
        if (std::fabs(v[k]) > lip * (b - a) / n) continue;  // every point of [s_l, s_r] is too far
        // zoom towards the extremum of g nearest zero: 33 samples a level,
        // keeping the two sample intervals around the best one (robust when
        // g has several dips or a kink between the coarse samples)
        const double sg = p ? 1.0 : -1.0;
        double xl = s[l], xr = s[r], xm = 0.0;
        bool found = false;
        for (int lev = 0; lev < 16 && !found; ++lev) {
            const int m = 32;
            double best = INFINITY;
            int kb = 0;
            for (int q = 0; q <= m; ++q) {
                const double x = (q == m) ? xr : xl + (xr - xl) * q / m;
                const double gv = g(x);
                if ((gv > 0.0) != p) { xm = x; found = true; break; }
                if (sg * gv < best) { best = sg * gv; kb = q; }
            }
            if (found) break;
            const double nl = xl + (xr - xl) * std::max(kb - 1, 0) / m;
            const double nr = (kb + 1 >= m) ? xr : xl + (xr - xl) * (kb + 1) / m;
            xl = nl;
            xr = nr;
            if (xr - xl < 1e-15 * std::max(1.0, std::fabs(xr))) break;
        }
        if (found && nr < 62) {
            roots[nr++] = bisect(s[l], xm);
            roots[nr++] = bisect(xm, s[r]);
        }
    }
    std::sort(roots, roots + nr);
    double pts[66];
    int np = 0;
    pts[np++] = a;
    for (int k = 0; k < nr; ++k)
        if (roots[k] > a && roots[k] < b && roots[k] - pts[np - 1] > 1e-13 * (b - a)) pts[np++] = roots[k];
    pts[np++] = b;
    int m = 0;
    for (int k = 0; k + 1 < np; ++k) {
        if (pts[k + 1] > pts[k] && g(0.5 * (pts[k] + pts[k + 1])) > 0.0 && m < cap) {
            lo[m] = pts[k];
            hi[m] = pts[k + 1];
            ++m;
        }
    }
    return m;
}

struct Moments {
    double a, mx, my;
};

class Integrator {
  public:
    Integrator(const Fluid &f) : f_(f) {}

    double vseg(double x, double ya, double yb) const {
        double lo[32], hi[32];
        int m = fluid_intervals([&](double y) { return f_(x, y); }, ya, yb, lo, hi, 32, f_.lip);
        double L = 0.0;
        for (int k = 0; k < m; ++k) L += hi[k] - lo[k];
        return L;
    }
    double hseg(double y, double xa, double xb) const {
        double lo[32], hi[32];
        int m = fluid_intervals([&](double x) { return f_(x, y); }, xa, xb, lo, hi, 32, f_.lip);
        double L = 0.0;
        for (int k = 0; k < m; ++k) L += hi[k] - lo[k];
        return L;
    }
    Moments rect(double xa, double xb, double ya, double yb) const {
        Moments out{0, 0, 0};
        if (!(xb > xa) || !(yb > ya)) return out;
        std::vector<double> pts{xa, xb}, tangents;
        for (double yy : {ya, yb}) {
            double lo[32], hi[32];
            int m = fluid_intervals([&](double x) { return f_(x, yy); }, xa, xb, lo, hi, 32, f_.lip);
            for (int k = 0; k < m; ++k) {
                if (lo[k] > xa) pts.push_back(lo[k]);
                if (hi[k] < xb) pts.push_back(hi[k]);
            }
        }
        // the wet length has a kink below each corner of the interface
        f_.corners(xa, xb, ya, yb, pts);
        std::sort(pts.begin(), pts.end());
        // Vertical tangents of the interface change the number of roots on a
        // vertical line.  Probe that count on a uniform grid and just beside
        // every edge crossing (a tangent next to a crossing can be closer to
        // it than any quadrature node), and bisect wherever it changes.
        {
            const double eps = 1e-12 * (xb - xa);
            std::vector<double> probe;
            for (int k = 0; k <= 16; ++k) probe.push_back(xa + (xb - xa) * k / 16.0);
            for (double b : pts) {
                if (b - eps > xa) probe.push_back(b - eps);
                if (b + eps < xb) probe.push_back(b + eps);
            }
            std::sort(probe.begin(), probe.end());
            auto count = [&](double x) {
                double lo[32], hi[32];
                int m = fluid_intervals([&](double y) { return f_(x, y); }, ya, yb, lo, hi, 32, f_.lip);
                int c = 0;
                for (int k = 0; k < m; ++k) c += (lo[k] > ya) + (hi[k] < yb);
                return c;
            };
            std::vector<int> cnt(probe.size());
            for (size_t k = 0; k < probe.size(); ++k) cnt[k] = count(probe[k]);
            std::vector<double> extra;
            for (size_t k = 0; k + 1 < probe.size(); ++k) {
                double l = probe[k], r = probe[k + 1];
                if (cnt[k] == cnt[k + 1] || r - l <= 2.5 * eps) continue;
                int cl = cnt[k];
                while (r - l > 1e-15 * std::max(1.0, std::fabs(r))) {
                    double m = 0.5 * (l + r);
                    if (!(m > l && m < r)) break;
                    if (count(m) == cl) l = m; else r = m;
                }
                extra.push_back(0.5 * (l + r));
            }
            pts.insert(pts.end(), extra.begin(), extra.end());
            std::sort(pts.begin(), pts.end());
            tangents.swap(extra);
        }
        // At a vertical tangent the wet length behaves like the square root of
        // the distance to it: pieces that end there are integrated in
        // u = sqrt(|x - x_t|), where the integrand is smooth.
        auto singular = [&](double x) {
            return std::find(tangents.begin(), tangents.end(), x) != tangents.end();
        };
        const double tol = 1e-14 * (xb - xa) * (yb - ya);
        auto add = [&](const Moments &m) { out.a += m.a; out.mx += m.mx; out.my += m.my; };
        for (size_t k = 0; k + 1 < pts.size(); ++k) {
            const double a = pts[k], b = pts[k + 1];
            if (b <= a) continue;
            const double t = tol * (b - a) / (xb - xa);
            const bool sa = singular(a), sb = singular(b);
            if (!sa && !sb) {
                add(adapt(a, b, ya, yb, t, 0.0, 0));
            } else if (sa && !sb) {
                add(adapt(0.0, std::sqrt(b - a), ya, yb, t, a, 1));
            } else if (!sa && sb) {
                add(adapt(0.0, std::sqrt(b - a), ya, yb, t, b, -1));
            } else {
                const double m = 0.5 * (a + b);
                add(adapt(0.0, std::sqrt(m - a), ya, yb, 0.5 * t, a, 1));
                add(adapt(0.0, std::sqrt(b - m), ya, yb, 0.5 * t, b, -1));
            }
        }
        return out;
    }

  private:
    void column(double x, double ya, double yb, double &L, double &M) const {
        double lo[32], hi[32];
        int m = fluid_intervals([&](double y) { return f_(x, y); }, ya, yb, lo, hi, 32, f_.lip);
        L = 0.0;
        M = 0.0;
        for (int k = 0; k < m; ++k) {
            L += hi[k] - lo[k];
            M += 0.5 * (hi[k] * hi[k] - lo[k] * lo[k]);
        }
    }
    // One G7K15 panel over [p, q] in the integration variable u, with
    // x = u (mode 0) or x = x0 + mode u^2 (mode +-1, Jacobian 2u); returns
    // the Kronrod estimates and the largest error estimate.
    double panel(double p, double q, double ya, double yb, Moments &k, double x0, int mode) const {
        double c = 0.5 * (p + q), h = 0.5 * (q - p);
        double ka = 0, kx = 0, ky = 0, ga = 0, gx = 0, gy = 0;
        for (int i = 0; i < 8; ++i) {
            int nside = (i == 7) ? 1 : 2;
            for (int sgn = 0; sgn < nside; ++sgn) {
                const double u = c + (sgn ? -1.0 : 1.0) * h * kXK[i];
                const double x = mode == 0 ? u : x0 + mode * u * u;
                const double jac = mode == 0 ? 1.0 : 2.0 * u;
                double L, M;
                column(x, ya, yb, L, M);
                L *= jac;
                M *= jac;
                ka += kWK[i] * L; kx += kWK[i] * x * L; ky += kWK[i] * M;
                if (i % 2 == 1) {
                    double w = kWG[i / 2];
                    ga += w * L; gx += w * x * L; gy += w * M;
                }
            }
        }
        k.a = ka * h; k.mx = kx * h; k.my = ky * h;
        const double xs = mode == 0 ? c : x0;
        double e = std::max(std::fabs(ka - ga), std::max(std::fabs(kx - gx) / std::max(1.0, std::fabs(xs)),
                                                         std::fabs(ky - gy) / std::max(1.0, std::fabs(yb))));
        return e * h;
    }
    // Globally adaptive Gauss-Kronrod on [p, q] (in u): the panel with the
    // largest error estimate is halved until the estimates add up to at most
    // tol or the panel budget is spent.  A panel is final when its estimate is
    // below the noise of its integrand (the roots that bound the wet length
    // are known to about 1e-16 max(1, |y|), and the estimate itself carries
    // rounding of about 1e-16 of the integral) or when its x-extent is at the
    // resolution of x.  Next to a vertical tangent the root pair is
    // ill-conditioned and the wet length noisier still; the budget bounds the
    // work spent there, on contributions far below the tolerance.
    static constexpr int MAX_PANELS = 400;
    Moments adapt(double p, double q, double ya, double yb, double tol, double x0, int mode) const {
        struct Pan {
            double p, q, e;
            Moments k;
        };
        auto cmp = [](const Pan &a, const Pan &b) { return a.e < b.e; };
        std::priority_queue<Pan, std::vector<Pan>, decltype(cmp)> open(cmp);
        Moments sum{0, 0, 0};
        double esum = 0.0;
        const double ynoise = 16.0 * 2.2e-16 * std::max(1.0, std::max(std::fabs(ya), std::fabs(yb)));
        const double inoise = 256.0 * 2.2e-16 * (yb - ya);
        auto push = [&](double a, double b) {
            Pan pn{a, b, 0.0, Moments{0, 0, 0}};
            const double e = panel(a, b, ya, yb, pn.k, x0, mode);
            const double wx = mode == 0 ? b - a : b * b - a * a;  // x-extent
            const double xr = mode == 0 ? b : x0;
            if (e <= wx * std::max(ynoise, inoise) || wx < 1e-15 * std::max(1.0, std::fabs(xr))) {
                sum.a += pn.k.a; sum.mx += pn.k.mx; sum.my += pn.k.my;
                return;
            }
            pn.e = e;
            esum += e;
            open.push(pn);
        };
        push(p, q);
        for (int npan = 1; !open.empty() && esum > tol && npan < MAX_PANELS; ++npan) {
            const Pan w = open.top();
            open.pop();
            esum -= w.e;
            const double m = 0.5 * (w.p + w.q);
            push(w.p, m);
            push(m, w.q);
        }
        for (; !open.empty(); open.pop()) {
            sum.a += open.top().k.a; sum.mx += open.top().k.mx; sum.my += open.top().k.my;
        }
        return sum;
    }
    const Fluid &f_;
};

// Capacities of one grid of control volumes [ex[i], ex[i+1]] x [ey[j], ey[j+1]]
// (i = 0..ni-1, j = 0..nj-1) for fluid = {phi > 0} inside the open box.
struct GridOut {
    std::vector<double> V, X, Y, E, N, Bv, Bh, We, Wn;
};

// A rectangle or segment entirely in the fluid has the exact measures of its
// extent.  On a uniform axis extents differ from the mesh spacing only by the
// rounding of the node coordinates; one within 1e-9 relative of hx (hy) is
// taken as hx (hy), so that every full cell, face and strip away from the
// interface carries the same capacities bit for bit (V = hx hy, A = B = h,
// W = hx hy).  A stretched axis passes h = 0: its extents are kept as they are.
inline double snap(double len, double h) { return std::fabs(len - h) <= 1e-9 * h ? h : len; }

// One axis of the three grids: the cell edges e[i] = x_{i-1/2} and centres
// c[i] = x_i, i = 0 .. n+2 (one ghost cell each side), the pressure grid's
// box [lo, hi] and the velocity grid's [clo, chi], which reaches half a cell
// across the walls (to the ghost cells' centres), and the snapping spacing.
struct Axis {
    std::vector<double> e, c;
    double lo, hi, clo, chi, snap_h, hmax;
};

Axis make_axis(int n, double o, double h, const double *f) {
    Axis a;
    a.e.resize(n + 3);
    a.c.resize(n + 3);
    if (!f) {
        for (int i = 0; i < n + 3; ++i) { a.e[i] = o + (i - 1.0) * h; a.c[i] = o + (i - 0.5) * h; }
        a.lo = o; a.hi = o + n * h; a.clo = a.lo - 0.5 * h; a.chi = a.hi + 0.5 * h;
        a.snap_h = h; a.hmax = h;
        return a;
    }
    // user abscissas (Sec. 3.1); the ghost cells repeat the wall cells' widths
    for (int i = 0; i <= n; ++i) a.e[i + 1] = f[i];
    a.e[0] = f[0] - (f[1] - f[0]);
    a.e[n + 2] = f[n] + (f[n] - f[n - 1]);
    for (int i = 0; i < n + 2; ++i) a.c[i] = 0.5 * (a.e[i] + a.e[i + 1]);
    a.c[n + 2] = a.e[n + 2] + 0.5 * (a.e[n + 2] - a.e[n + 1]);
    a.lo = a.e[1]; a.hi = a.e[n + 1]; a.clo = a.c[0]; a.chi = a.c[n + 1];
    a.snap_h = 0.0;
    a.hmax = 0.0;
    for (int i = 0; i < n; ++i) a.hmax = std::max(a.hmax, f[i + 1] - f[i]);
    return a;
}

bool valid_abscissas(const double *f, int n, double o) {
    if (!f) return true;
    if (f[0] != o) return false;
    for (int i = 0; i <= n; ++i)
        if (!std::isfinite(f[i]) || (i > 0 && !(f[i] > f[i - 1]))) return false;
    return true;
}

GridOut grid_caps(const Fluid &fl, const Integrator &in, const std::vector<double> &ex,
                  const std::vector<double> &ey, double bx0, double bx1, double by0, double by1,
                  bool wall_faces_wet, double epsV, double margin, double hx, double hy) {
    const int ni = (int)ex.size() - 1, nj = (int)ey.size() - 1;
    GridOut g;
    size_t n = (size_t)ni * nj;
    for (auto *v : {&g.V, &g.X, &g.Y, &g.E, &g.N, &g.Bv, &g.Bh, &g.We, &g.Wn}) v->assign(n, 0.0);
    auto rect = [&](double xa, double xb, double ya, double yb) -> Moments {
        xa = std::max(xa, bx0); xb = std::min(xb, bx1);
        ya = std::max(ya, by0); yb = std::min(yb, by1);
        if (!(xb > xa) || !(yb > ya)) return Moments{0, 0, 0};
        const int cl = fl.classify(xa, xb, ya, yb, margin);
        if (cl > 0) {
            const double w = snap(xb - xa, hx), t = snap(yb - ya, hy);
            return Moments{w * t, 0.5 * (xb * xb - xa * xa) * t, 0.5 * (yb * yb - ya * ya) * w};
        }
        if (cl < 0) return Moments{0, 0, 0};
        return in.rect(xa, xb, ya, yb);
    };
    auto vseg = [&](double x, double ya, double yb, bool wet) -> double {
        bool inside = (x > bx0 && x < bx1) || (wet && x >= bx0 && x <= bx1);
        if (!inside) return 0.0;
        ya = std::max(ya, by0); yb = std::min(yb, by1);
        if (!(yb > ya)) return 0.0;
        const int cl = fl.classify(x, x, ya, yb, margin);
        if (cl != 0) return cl > 0 ? snap(yb - ya, hy) : 0.0;
        return in.vseg(x, ya, yb);
    };
    auto hseg = [&](double y, double xa, double xb, bool wet) -> double {
        bool inside = (y > by0 && y < by1) || (wet && y >= by0 && y <= by1);
        if (!inside) return 0.0;
        xa = std::max(xa, bx0); xb = std::min(xb, bx1);
        if (!(xb > xa)) return 0.0;
        const int cl = fl.classify(xa, xb, y, y, margin);
        if (cl != 0) return cl > 0 ? snap(xb - xa, hx) : 0.0;
        return in.hseg(y, xa, xb);
    };
#pragma omp parallel for schedule(dynamic, 4)
    for (int j = 0; j < nj; ++j)
        for (int i = 0; i < ni; ++i) {
            size_t k = (size_t)j * ni + i;
            Moments m = rect(ex[i], ex[i + 1], ey[j], ey[j + 1]);
            if (m.a > epsV) {
                g.V[k] = m.a;
                g.X[k] = std::min(std::max(m.mx / m.a, ex[i]), ex[i + 1]);
                g.Y[k] = std::min(std::max(m.my / m.a, ey[j]), ey[j + 1]);
            } else {
                g.V[k] = 0.0;
                g.X[k] = 0.5 * (ex[i] + ex[i + 1]);
                g.Y[k] = 0.5 * (ey[j] + ey[j + 1]);
            }
        }
#pragma omp parallel for schedule(dynamic, 4)
    for (int j = 0; j < nj; ++j)
        for (int i = 0; i < ni; ++i) {
            size_t k = (size_t)j * ni + i;
            g.E[k] = vseg(ex[i + 1], ey[j], ey[j + 1], wall_faces_wet);
            g.N[k] = hseg(ey[j + 1], ex[i], ex[i + 1], wall_faces_wet);
            g.Bv[k] = vseg(g.X[k], ey[j], ey[j + 1], false);
            g.Bh[k] = hseg(g.Y[k], ex[i], ex[i + 1], false);
            if (i + 1 < ni) g.We[k] = rect(g.X[k], g.X[k + 1], ey[j], ey[j + 1]).a;
            if (j + 1 < nj) g.Wn[k] = rect(ex[i], ex[i + 1], g.Y[k], g.Y[k + ni]).a;
        }
    return g;
}

}  // namespace
}  // namespace ccns

using namespace ccns;

extern "C" size_t ccns_caps_count(const ccns_grid *grid) {
    if (!grid || grid->nx < 1 || grid->ny < 1) return 0;
    return (size_t)CCNS_NCAPS * (size_t)(grid->nx + 2) * (size_t)(grid->ny + 2);
}

extern "C" ccns_status ccns_capacities(const ccns_grid *grid, const ccns_body *bodies, int nbody,
                                       ccns_levelset_fn fn, void *user, double *caps) {
    if (!grid || !caps || grid->nx < 2 || grid->ny < 2 || !(grid->hx > 0) || !(grid->hy > 0) ||
        nbody < 0 || (nbody > 0 && !bodies) || !valid_abscissas(grid->xf, grid->nx, grid->x0) ||
        !valid_abscissas(grid->yf, grid->ny, grid->y0))
        return CCNS_EINVAL;
    for (int k = 0; k < nbody; ++k) {
        const ccns_body &b = bodies[k];
        if (b.kind < 0 || b.kind > 2) return CCNS_EINVAL;
        if (b.kind == CCNS_CIRCLE && !(b.a > 0)) return CCNS_EINVAL;
        if (b.kind == CCNS_ELLIPSE && !(b.a > 0 && b.b > 0)) return CCNS_EINVAL;
        if (b.kind == CCNS_NACA4 && !(b.chord > 0 && b.t > 0)) return CCNS_EINVAL;
    }
    const int nx = grid->nx, ny = grid->ny;
    const double hx = grid->hx, hy = grid->hy;
    Fluid fl{bodies, nbody, fn, user};
    fl.lip = fl.lipschitz();
    Integrator in(fl);
    const Axis ax = make_axis(nx, grid->x0, hx, grid->xf), ay = make_axis(ny, grid->y0, hy, grid->yf);
    const double epsV = 1e-12 * hx * hy, margin = 2.0 * std::max(ax.hmax, ay.hmax);
    const double sx = ax.snap_h, sy = ay.snap_h;
    GridOut p = grid_caps(fl, in, ax.e, ay.e, ax.lo, ax.hi, ay.lo, ay.hi, true, epsV, margin, sx, sy);
    GridOut u = grid_caps(fl, in, ax.c, ay.e, ax.clo, ax.chi, ay.lo, ay.hi, false, epsV, margin, sx, sy);
    GridOut v = grid_caps(fl, in, ax.e, ay.c, ax.lo, ax.hi, ay.clo, ay.chi, false, epsV, margin, sx, sy);
    const size_t W = nx + 2, H = ny + 2, n = W * H;
    std::memset(caps, 0, sizeof(double) * n * CCNS_NCAPS);
    auto at = [&](int cap) { return caps + (size_t)cap * n; };
    for (size_t j = 0; j < H; ++j)
        for (size_t i = 0; i < W; ++i) {
            size_t k = j * W + i;
            size_t kw = (i > 0) ? k - 1 : SIZE_MAX;   // west neighbour in the CV grid
            size_t ks = (j > 0) ? k - W : SIZE_MAX;   // south neighbour
            at(CCNS_CAP_V)[k] = p.V[k];
            at(CCNS_CAP_AX)[k] = p.E[k];
            at(CCNS_CAP_AY)[k] = p.N[k];
            at(CCNS_CAP_BX)[k] = p.Bv[k];
            at(CCNS_CAP_BY)[k] = p.Bh[k];
            at(CCNS_CAP_WX)[k] = p.We[k];
            at(CCNS_CAP_WY)[k] = p.Wn[k];
            at(CCNS_CAP_VU)[k] = u.V[k];
            at(CCNS_CAP_AXX)[k] = (kw != SIZE_MAX) ? u.E[kw] : 0.0;
            at(CCNS_CAP_AXY)[k] = u.N[k];
            at(CCNS_CAP_BXX)[k] = u.Bv[k];
            at(CCNS_CAP_BXY)[k] = u.Bh[k];
            at(CCNS_CAP_WXX)[k] = (kw != SIZE_MAX) ? u.We[kw] : 0.0;
            at(CCNS_CAP_WXY)[k] = u.Wn[k];
            at(CCNS_CAP_VV)[k] = v.V[k];
            at(CCNS_CAP_AYY)[k] = (ks != SIZE_MAX) ? v.N[ks] : 0.0;
            at(CCNS_CAP_AYX)[k] = v.E[k];
            at(CCNS_CAP_BYY)[k] = v.Bh[k];
            at(CCNS_CAP_BYX)[k] = v.Bv[k];
            at(CCNS_CAP_WYY)[k] = (ks != SIZE_MAX) ? v.Wn[ks] : 0.0;
            at(CCNS_CAP_WYX)[k] = v.We[k];
        }
    // capacities below the thresholds are zero
    const double epsX = 1e-12 * hy, epsY = 1e-12 * hx;
    const int vol[] = {CCNS_CAP_V, CCNS_CAP_WX, CCNS_CAP_WY, CCNS_CAP_VU, CCNS_CAP_WXX, CCNS_CAP_WXY,
                       CCNS_CAP_VV, CCNS_CAP_WYY, CCNS_CAP_WYX};
    const int lx[] = {CCNS_CAP_AX, CCNS_CAP_BX, CCNS_CAP_AXX, CCNS_CAP_BXX, CCNS_CAP_AYX, CCNS_CAP_BYX};
    const int ly[] = {CCNS_CAP_AY, CCNS_CAP_BY, CCNS_CAP_AYY, CCNS_CAP_BYY, CCNS_CAP_AXY, CCNS_CAP_BXY};
    for (int c : vol) for (size_t k = 0; k < n; ++k) if (!(at(c)[k] > epsV)) at(c)[k] = 0.0;
    for (int c : lx) for (size_t k = 0; k < n; ++k) if (!(at(c)[k] > epsX)) at(c)[k] = 0.0;
    for (int c : ly) for (size_t k = 0; k < n; ++k) if (!(at(c)[k] > epsY)) at(c)[k] = 0.0;
    return CCNS_OK;
}
