// Host preparation of the coefficient fields of one context (setup, once per
// geometry).  Readings of the paper used here:
//  - velocity unknowns: faces interior to the box whose staggered control
//    volume holds fluid; every other face keeps its Dirichlet value (Sec. 4)
//  - Poisson operator cont(M^-1 pres(Phi), 0) (eq:pm_poisson with the mass
//    matrix of Sec. 4.5 explicit): face weight c = A^2/V_f
//  - pressure unknowns: fluid cells of the largest set connected through
//    faces with c > 0 (Phi is known up to a constant on it, end of Sec. 4.6)
//  - node strain weights (eq:offdiag): the printed form uses two node volumes
//    W^xy and W^yx; the symmetric default keeps 1/W^xy for the x rows,
//    1/W^yx for the y rows and 1/sqrt(W^xy W^yx) for the cross coupling.
//  - outflow walls (end of Sec. 4.6): the open faces normal to such a wall
//    are corrected by the projection (mass max(V_f, floor), Poisson weight
//    A^2/M on the diagonal of the cell inside, the pressure beyond the wall
//    held at zero); they are no predictor unknowns and keep U = D out of the
//    constant Dirichlet part of the viscous term, since the step replaces
//    their velocity every time.
#include <algorithm>
#include <cmath>
#include <queue>

#include "ccns_internal.h"

namespace ccns {

Layout make_layout(int nx, int ny) {
    Layout L;
    L.nx = nx;
    L.ny = ny;
    L.rows = ny + 2;
    L.pitch = ((nx + 2 + 63) / 64) * 64;
    L.n = (size_t)L.rows * L.pitch;
    return L;
}

static inline double inv0(double a) { return a != 0.0 ? 1.0 / a : 0.0; }

ccns_status prepare_coefficients(const ccns_grid &g, const ccns_params &prm, const double *caps,
                                 const double *dir, HostCoef &o, std::string &err) {
    const int nx = g.nx, ny = g.ny, W = nx + 2, H = ny + 2;
    const size_t n = (size_t)W * H;
    if (nx < 2 || ny < 2 || !(g.hx > 0) || !(g.hy > 0)) { err = "bad grid"; return CCNS_EINVAL; }
    if (!(prm.rho > 0) || !(prm.mu >= 0) || !(prm.tau > 0)) { err = "rho, tau must be > 0 and mu >= 0"; return CCNS_EINVAL; }
    if (!(prm.mass_floor >= 0.0) || !(prm.mass_floor <= 1.0)) { err = "mass_floor must be in [0, 1]"; return CCNS_EINVAL; }
    if (prm.coef_tables != 0 && prm.coef_tables != 1) { err = "coef_tables must be 0 or 1"; return CCNS_EINVAL; }
    if (prm.outflow < 0 || prm.outflow > 15) { err = "outflow must be a sum of CCNS_WALL_*"; return CCNS_EINVAL; }
    if (prm.visc_form < 0 || prm.visc_form > 2 || prm.poisson_weight < 0 || prm.poisson_weight > 1) {
        err = "bad visc_form or poisson_weight"; return CCNS_EINVAL;
    }
    for (size_t k = 0; k < n * CCNS_NCAPS; ++k)
        if (!(caps[k] >= 0.0) || !std::isfinite(caps[k])) { err = "capacity negative or not finite"; return CCNS_EINVAL; }
    for (size_t k = 0; k < 2 * n; ++k)
        if (!std::isfinite(dir[k])) { err = "Dirichlet data not finite"; return CCNS_EINVAL; }
    auto C = [&](int c) { return caps + (size_t)c * n; };
    const double *V = C(CCNS_CAP_V), *Ax = C(CCNS_CAP_AX), *Ay = C(CCNS_CAP_AY);
    const double *Bx = C(CCNS_CAP_BX), *By = C(CCNS_CAP_BY);
    const double *Vu = C(CCNS_CAP_VU), *Vv = C(CCNS_CAP_VV);
    const double *Axx = C(CCNS_CAP_AXX), *Axy = C(CCNS_CAP_AXY), *Bxx = C(CCNS_CAP_BXX), *Bxy = C(CCNS_CAP_BXY);
    const double *Wxx = C(CCNS_CAP_WXX), *Wxy = C(CCNS_CAP_WXY);
    const double *Ayy = C(CCNS_CAP_AYY), *Ayx = C(CCNS_CAP_AYX), *Byy = C(CCNS_CAP_BYY), *Byx = C(CCNS_CAP_BYX);
    const double *Wyy = C(CCNS_CAP_WYY), *Wyx = C(CCNS_CAP_WYX);
    const double *Dx = dir, *Dy = dir + n;
    auto id = [&](int j, int i) { return (size_t)j * W + i; };

    for (auto *v : {&o.cx, &o.cy, &o.dinv, &o.gx, &o.gy, &o.ax, &o.ay, &o.het, &o.hbx, &o.hby, &o.dx, &o.dy,
                    &o.vu, &o.vv, &o.bxx, &o.bxy, &o.byy, &o.byx, &o.wxx, &o.wyy, &o.nxx, &o.nxy, &o.nyx,
                    &o.nyy, &o.hdx, &o.hdy, &o.vinv, &o.utx, &o.uty, &o.vur, &o.vvr})
        v->assign(n, 0.0);

    std::vector<char> au(n, 0), av(n, 0), fluid(n, 0), act(n, 0), ou(n, 0), ov(n, 0);
    const int of = prm.outflow;
    for (int j = 0; j < H; ++j)
        for (int i = 0; i < W; ++i) {
            size_t k = id(j, i);
            // an unknown needs fluid in its control volume and an open face:
            // a face of zero aperture carries no flux, and keeps the body's
            // (Dirichlet) velocity
            au[k] = (i >= 1 && i <= nx - 1 && j >= 1 && j <= ny && Vu[k] > 0.0 && Ax[k] > 0.0);
            av[k] = (i >= 1 && i <= nx && j >= 1 && j <= ny - 1 && Vv[k] > 0.0 && Ay[k] > 0.0);
            fluid[k] = (i >= 1 && i <= nx && j >= 1 && j <= ny && V[k] > 0.0);
            const bool wu = j >= 1 && j <= ny && (((of & CCNS_WALL_W) && i == 0) || ((of & CCNS_WALL_E) && i == nx));
            const bool wv = i >= 1 && i <= nx && (((of & CCNS_WALL_S) && j == 0) || ((of & CCNS_WALL_N) && j == ny));
            ou[k] = wu && Vu[k] > 0.0 && Ax[k] > 0.0;
            ov[k] = wv && Vv[k] > 0.0 && Ay[k] > 0.0;
        }
    if (of) {
        // the Dirichlet data of an outflow face cancel out of cont, strain and
        // the convective bracket where the first-kind and second-kind
        // capacities next to the wall agree (uncut cells): then the data the
        // step leaves in place act as the zero-gradient data it stands for
        auto same = [](double a, double b) { return std::fabs(a - b) <= 1e-12 * std::max(std::fabs(a), std::fabs(b)); };
        bool ok = true;
        for (int j = 1; j <= ny && ok; ++j) {
            if (of & CCNS_WALL_E)
                ok = same(Ax[id(j, nx)], Bx[id(j, nx)]) && same(Bxx[id(j, nx)], Axx[id(j, nx)]) &&
                     (j == ny || (same(Bxy[id(j, nx)], Axy[id(j, nx)]) && same(Bxy[id(j + 1, nx)], Axy[id(j, nx)])));
            if ((of & CCNS_WALL_W) && ok)
                ok = same(Ax[id(j, 0)], Bx[id(j, 1)]) && same(Bxx[id(j, 0)], Axx[id(j, 1)]) &&
                     (j == ny || (same(Bxy[id(j, 0)], Axy[id(j, 0)]) && same(Bxy[id(j + 1, 0)], Axy[id(j, 0)])));
        }
        for (int i = 1; i <= nx && ok; ++i) {
            if (of & CCNS_WALL_N)
                ok = same(Ay[id(ny, i)], By[id(ny, i)]) && same(Byy[id(ny, i)], Ayy[id(ny, i)]) &&
                     (i == nx || (same(Byx[id(ny, i)], Ayx[id(ny, i)]) && same(Byx[id(ny, i + 1)], Ayx[id(ny, i)])));
            if ((of & CCNS_WALL_S) && ok)
                ok = same(Ay[id(0, i)], By[id(1, i)]) && same(Byy[id(0, i)], Ayy[id(1, i)]) &&
                     (i == nx || (same(Byx[id(0, i)], Ayx[id(0, i)]) && same(Byx[id(0, i + 1)], Ayx[id(0, i)])));
        }
        if (!ok) { err = "a body cuts the cells next to an outflow wall"; return CCNS_EINVAL; }
    }
    // mass matrix of the velocity unknowns and outflow faces (with the floor)
    const double mfloor = prm.mass_floor * g.hx * g.hy;
    std::vector<double> Mu(n, 0.0), Mv(n, 0.0);
    for (size_t k = 0; k < n; ++k) {
        Mu[k] = (au[k] || ou[k]) ? std::max(Vu[k], mfloor) : Vu[k];
        Mv[k] = (av[k] || ov[k]) ? std::max(Vv[k], mfloor) : Vv[k];
    }
    const bool volw = prm.poisson_weight == 0;
    for (size_t k = 0; k < n; ++k) {
        double wu = volw ? inv0(Mu[k]) : 1.0, wv = volw ? inv0(Mv[k]) : 1.0;
        o.cx[k] = (au[k] || ou[k]) ? Ax[k] * Ax[k] * wu : 0.0;
        o.cy[k] = (av[k] || ov[k]) ? Ay[k] * Ay[k] * wv : 0.0;
    }
    // largest set of fluid cells connected through faces with c > 0
    std::vector<int> lab(n, -1);
    int best = -1, bestsz = 0, nl = 0;
    for (int j = 1; j <= ny; ++j)
        for (int i = 1; i <= nx; ++i) {
            size_t s = id(j, i);
            if (!fluid[s] || lab[s] >= 0) continue;
            int sz = 0;
            std::queue<size_t> q;
            q.push(s);
            lab[s] = nl;
            while (!q.empty()) {
                size_t k = q.front();
                q.pop();
                ++sz;
                size_t nb[4] = {k + 1, k - 1, k + W, k - W};
                double cc[4] = {o.cx[k], o.cx[k - 1], o.cy[k], o.cy[k - W]};
                for (int e = 0; e < 4; ++e)
                    if (cc[e] > 0.0 && fluid[nb[e]] && lab[nb[e]] < 0) {
                        lab[nb[e]] = nl;
                        q.push(nb[e]);
                    }
            }
            if (sz > bestsz) { bestsz = sz; best = nl; }
            ++nl;
        }
    o.n_active = 0;
    for (size_t k = 0; k < n; ++k) {
        act[k] = (lab[k] == best && best >= 0);
        o.n_active += act[k];
    }
    o.n_out = 0;
    for (size_t k = 0; k < n; ++k) {
        // an outflow face couples the cell inside to the zero pressure beyond
        const bool ae = (k + 1 < n) && act[k + 1], an = (k + W < n) && act[k + W];
        bool ex = (act[k] && ae) || (ou[k] && (act[k] || ae));
        bool ey = (act[k] && an) || (ov[k] && (act[k] || an));
        if (!ex) o.cx[k] = 0.0;
        if (!ey) o.cy[k] = 0.0;
        o.n_out += (ou[k] && ex) + (ov[k] && ey);
        double wu = volw ? inv0(Mu[k]) : 1.0, wv = volw ? inv0(Mv[k]) : 1.0;
        o.gx[k] = o.cx[k] > 0.0 ? Ax[k] * wu : 0.0;
        o.gy[k] = o.cy[k] > 0.0 ? Ay[k] * wv : 0.0;
    }
    for (int j = 1; j <= ny; ++j)
        for (int i = 1; i <= nx; ++i) {
            size_t k = id(j, i);
            if (!act[k]) continue;
            double d = o.cx[k] + o.cx[k - 1] + o.cy[k] + o.cy[k - W];
            o.dinv[k] = inv0(d);
            o.vinv[k] = inv0(std::max(V[k], mfloor));
        }
    // divergence and convection data
    o.n_uact = o.n_vact = 0;
    for (size_t k = 0; k < n; ++k) {
        o.ax[k] = Ax[k];
        o.ay[k] = Ay[k];
        o.dx[k] = Dx[k];
        o.dy[k] = Dy[k];
        o.vu[k] = au[k] ? Mu[k] : 0.0;
        o.vv[k] = av[k] ? Mv[k] : 0.0;
        o.vur[k] = Vu[k];
        o.vvr[k] = Vv[k];
        o.utx[k] = (au[k] || o.gx[k] != 0.0) ? 0.0 : Dx[k];
        o.uty[k] = (av[k] || o.gy[k] != 0.0) ? 0.0 : Dy[k];
        o.n_uact += au[k];
        o.n_vact += av[k];
    }
    for (int j = 1; j <= ny; ++j)
        for (int i = 1; i <= nx; ++i) {
            size_t k = id(j, i);
            o.het[k] = -Ax[k] * Dx[k] + Ax[k - 1] * Dx[k - 1] + Bx[k] * (Dx[k] - Dx[k - 1]) - Ay[k] * Dy[k] +
                       Ay[k - W] * Dy[k - W] + By[k] * (Dy[k] - Dy[k - W]);
        }
    for (int j = 0; j < H; ++j)
        for (int i = 0; i < W; ++i) {
            size_t k = id(j, i);
            if (i + 1 < W) o.hbx[k] = 0.25 * (o.het[k] + o.het[k + 1]);
            if (j + 1 < H) o.hby[k] = 0.25 * (o.het[k] + o.het[k + W]);
        }
    // viscous weights
    for (size_t k = 0; k < n; ++k) {
        o.bxx[k] = Bxx[k];
        o.bxy[k] = Bxy[k];
        o.byy[k] = Byy[k];
        o.byx[k] = Byx[k];
        o.wxx[k] = inv0(Wxx[k]);
        o.wyy[k] = inv0(Wyy[k]);
        double ixy = inv0(Wxy[k]), iyx = inv0(Wyx[k]);
        switch (prm.visc_form) {
        case 0: {
            double gm = inv0(std::sqrt(Wxy[k] * Wyx[k]));
            o.nxx[k] = ixy; o.nxy[k] = gm; o.nyx[k] = gm; o.nyy[k] = iyx;
            break;
        }
        case 1:
            o.nxx[k] = ixy; o.nxy[k] = iyx; o.nyx[k] = ixy; o.nyy[k] = iyx;
            break;
        default: {
            double m = inv0(0.5 * (Wxy[k] + Wyx[k]));
            o.nxx[k] = o.nxy[k] = o.nyx[k] = o.nyy[k] = m;
        }
        }
    }
    // Jacobi diagonal of H = (rho/tau) V - mu visc(strain(., 0))
    const double rt = prm.rho / prm.tau;
    for (int j = 1; j < H - 1; ++j)
        for (int i = 1; i < W - 1; ++i) {
            size_t k = id(j, i);
            if (au[k]) {
                double kd = Bxx[k] * Bxx[k] * (o.wxx[k] + o.wxx[k + 1]) +
                            0.5 * Bxy[k] * Bxy[k] * (o.nxx[k] + o.nxx[k - W]);
                o.hdx[k] = inv0(rt * Mu[k] + prm.mu * kd);
            }
            if (av[k]) {
                double kd = Byy[k] * Byy[k] * (o.wyy[k] + o.wyy[k + W]) +
                            0.5 * Byx[k] * Byx[k] * (o.nyy[k] + o.nyy[k - 1]);
                o.hdy[k] = inv0(rt * Mv[k] + prm.mu * kd);
            }
        }
    // force on the bodies (the momentum exchanged through the capacities):
    // the cells where A^x, A^y, B^xx or B^yy differ across the cell and the
    // nodes off the box's walls where B^xy or B^yx differ across the node;
    // everywhere else the terms cancel
    o.fcell.clear();
    o.fnode.clear();
    for (int j = 1; j <= ny; ++j)
        for (int i = 1; i <= nx; ++i) {
            const size_t k = id(j, i), kw = k - 1, ks = k - W;
            const double wpx = Ax[kw] - Ax[k], wpy = Ay[ks] - Ay[k];
            const double wvx = Bxx[k] - Bxx[kw], wvy = Byy[k] - Byy[ks];
            if (wpx == 0.0 && wpy == 0.0 && wvx == 0.0 && wvy == 0.0) continue;
            const double row[FORCE_W] = {(double)j, (double)i, wpx, wpy, wvx, wvy, o.wxx[k], Bxx[k], Bxx[kw], Axx[k],
                                         o.wyy[k], Byy[k], Byy[ks], Ayy[k]};
            o.fcell.insert(o.fcell.end(), row, row + FORCE_W);
        }
    for (int j = 0; j <= ny; ++j)
        for (int i = 0; i <= nx; ++i) {
            const size_t k = id(j, i);
            const double wnx = (j >= 1 && j <= ny - 1) ? Bxy[k + W] - Bxy[k] : 0.0;
            const double wny = (i >= 1 && i <= nx - 1) ? Byx[k + 1] - Byx[k] : 0.0;
            if (wnx == 0.0 && wny == 0.0) continue;
            const double row[FORCE_W] = {(double)j, (double)i, wnx, wny, Bxy[k + W], Bxy[k], Axy[k], Byx[k + 1], Byx[k],
                                         Ayx[k], o.nxx[k], o.nxy[k], o.nyx[k], o.nyy[k]};
            o.fnode.insert(o.fnode.end(), row, row + FORCE_W);
        }
    // constant Dirichlet contribution of the viscous term on the unknowns
    host_viscous(g, caps, o, o.utx.data(), o.uty.data(), o.vdx, o.vdy);
    for (size_t k = 0; k < n; ++k) {
        if (!au[k]) o.vdx[k] = 0.0;
        if (!av[k]) o.vdy[k] = 0.0;
    }
    return CCNS_OK;
}

// One multigrid coarsening step (2x2 cell agglomeration) of the Poisson
// weights: the coarse face weight is half the sum of the fine weights of the
// two fine faces it covers; a coarse cell is an unknown when one of its
// children is; faces touching a non-unknown are dropped.
void coarsen_poisson(int nx, int ny, const std::vector<double> &cx, const std::vector<double> &cy,
                     const std::vector<double> &dinv, int nxc, int nyc, std::vector<double> &cxc,
                     std::vector<double> &cyc, std::vector<double> &dinvc) {
    const size_t W = nx + 2, Wc = nxc + 2, nc = (size_t)(nyc + 2) * Wc;
    cxc.assign(nc, 0.0);
    cyc.assign(nc, 0.0);
    dinvc.assign(nc, 0.0);
    std::vector<char> act(nc, 0);
    for (int J = 1; J <= nyc; ++J)
        for (int I = 1; I <= nxc; ++I) {
            bool a = false;
            for (int dj = 0; dj < 2; ++dj)
                for (int di = 0; di < 2; ++di) {
                    int j = 2 * J - 1 + dj, i = 2 * I - 1 + di;
                    if (j <= ny && i <= nx && dinv[(size_t)j * W + i] > 0.0) a = true;
                }
            act[(size_t)J * Wc + I] = a;
        }
    // a face on the box's wall (weights only where the pressure beyond the
    // wall is held, on outflow walls) covers the fine wall faces: the east
    // wall face of the last coarse column is the fine face nx even when that
    // column has one fine column
    for (int J = 1; J <= nyc; ++J)
        for (int I = 0; I <= nxc; ++I) {
            double sum = 0.0;
            const int i = std::min(2 * I, nx);
            for (int dj = 0; dj < 2; ++dj) {
                int j = 2 * J - 1 + dj;
                if (j <= ny) sum += cx[(size_t)j * W + i];
            }
            size_t k = (size_t)J * Wc + I;
            const bool wall = I == 0 || I == nxc;
            cxc[k] = ((wall && (act[k] || act[k + 1])) || (act[k] && act[k + 1])) ? 0.5 * sum : 0.0;
        }
    for (int J = 0; J <= nyc; ++J)
        for (int I = 1; I <= nxc; ++I) {
            double sum = 0.0;
            const int j = std::min(2 * J, ny);
            for (int di = 0; di < 2; ++di) {
                int i = 2 * I - 1 + di;
                if (i <= nx) sum += cy[(size_t)j * W + i];
            }
            size_t k = (size_t)J * Wc + I;
            const bool wall = J == 0 || J == nyc;
            cyc[k] = ((wall && (act[k] || act[k + Wc])) || (act[k] && act[k + Wc])) ? 0.5 * sum : 0.0;
        }
    for (int J = 1; J <= nyc; ++J)
        for (int I = 1; I <= nxc; ++I) {
            size_t k = (size_t)J * Wc + I;
            double d = cxc[k] + cxc[k - 1] + cyc[k] + cyc[k - Wc];
            dinvc[k] = (act[k] && d > 0.0) ? 1.0 / d : 0.0;
        }
}

// Moore-Penrose pseudo-inverse of a small symmetric positive semi-definite
// matrix (row-major n x n) by cyclic Jacobi eigenvalue rotations;
// eigenvalues below 1e-12 of the largest are treated as zero (the constants
// on each connected set of unknowns span the null space).
std::vector<double> pseudo_inverse_spsd(std::vector<double> A, int n) {
    std::vector<double> V((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
    auto a = [&](int i, int j) -> double & { return A[(size_t)i * n + j]; };
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                tot += a(i, j) * a(i, j);
                if (i != j) off += a(i, j) * a(i, j);
            }
        if (off <= 1e-30 * tot) break;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                double apq = a(p, q);
                if (std::fabs(apq) < 1e-300) continue;
                double theta = (a(q, q) - a(p, p)) / (2.0 * apq);
                double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
                for (int k = 0; k < n; ++k) {
                    double akp = a(k, p), akq = a(k, q);
                    a(k, p) = cs * akp - sn * akq;
                    a(k, q) = sn * akp + cs * akq;
                }
                for (int k = 0; k < n; ++k) {
                    double apk = a(p, k), aqk = a(q, k);
                    a(p, k) = cs * apk - sn * aqk;
                    a(q, k) = sn * apk + cs * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    double vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
                    V[(size_t)k * n + p] = cs * vkp - sn * vkq;
                    V[(size_t)k * n + q] = sn * vkp + cs * vkq;
                }
            }
    }
    double lmax = 0.0;
    for (int i = 0; i < n; ++i) lmax = std::max(lmax, std::fabs(a(i, i)));
    std::vector<double> P((size_t)n * n, 0.0);
    for (int e = 0; e < n; ++e) {
        double l = a(e, e);
        if (!(l > 1e-12 * lmax)) continue;
        for (int i = 0; i < n; ++i) {
            double vi = V[(size_t)i * n + e] / l;
            for (int j = 0; j < n; ++j) P[(size_t)i * n + j] += vi * V[(size_t)j * n + e];
        }
    }
    return P;
}

// visc(strain(U, D)) with full Dirichlet terms (eq:diag, eq:offdiag, Sec. 4.3)
// on the host, for the constant boundary contribution of the viscous term.
void host_viscous(const ccns_grid &g, const double *caps, const HostCoef &o, const double *Ux,
                  const double *Uy, std::vector<double> &vx, std::vector<double> &vy) {
    const int nx = g.nx, ny = g.ny, W = nx + 2, H = ny + 2;
    const size_t n = (size_t)W * H;
    auto C = [&](int c) { return caps + (size_t)c * n; };
    const double *Axx = C(CCNS_CAP_AXX), *Axy = C(CCNS_CAP_AXY), *Ayy = C(CCNS_CAP_AYY), *Ayx = C(CCNS_CAP_AYX);
    const double *Dx = o.dx.data(), *Dy = o.dy.data();
    std::vector<double> sxx(n, 0.0), syy(n, 0.0), sx(n, 0.0), sy(n, 0.0);
    for (int j = 1; j <= ny; ++j)
        for (int i = 1; i <= nx; ++i) {
            size_t k = (size_t)j * W + i;
            sxx[k] = o.wxx[k] * (o.bxx[k] * (Ux[k] - Dx[k]) - o.bxx[k - 1] * (Ux[k - 1] - Dx[k - 1]) +
                                 Axx[k] * (Dx[k] - Dx[k - 1]));
            syy[k] = o.wyy[k] * (o.byy[k] * (Uy[k] - Dy[k]) - o.byy[k - W] * (Uy[k - W] - Dy[k - W]) +
                                 Ayy[k] * (Dy[k] - Dy[k - W]));
        }
    for (int j = 0; j <= ny; ++j)
        for (int i = 0; i <= nx; ++i) {
            size_t k = (size_t)j * W + i;
            double gx = o.bxy[k + W] * (Ux[k + W] - Dx[k + W]) - o.bxy[k] * (Ux[k] - Dx[k]) +
                        Axy[k] * (Dx[k + W] - Dx[k]);
            double gy = o.byx[k + 1] * (Uy[k + 1] - Dy[k + 1]) - o.byx[k] * (Uy[k] - Dy[k]) +
                        Ayx[k] * (Dy[k + 1] - Dy[k]);
            sx[k] = 0.5 * (o.nxx[k] * gx + o.nxy[k] * gy);
            sy[k] = 0.5 * (o.nyx[k] * gx + o.nyy[k] * gy);
        }
    vx.assign(n, 0.0);
    vy.assign(n, 0.0);
    for (int j = 1; j <= ny; ++j)
        for (int i = 1; i <= nx; ++i) {
            size_t k = (size_t)j * W + i;
            if (i <= nx - 1)
                vx[k] = o.bxx[k] * (sxx[k + 1] - sxx[k]) + o.bxy[k] * (sx[k] - sx[k - W]);
            if (j <= ny - 1)
                vy[k] = o.byy[k] * (syy[k + W] - syy[k]) + o.byx[k] * (sy[k] - sy[k - 1]);
        }
}

}  // namespace ccns
