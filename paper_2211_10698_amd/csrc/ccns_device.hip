// Device path of libccns: HIP kernels for gfx950 and their host driver.
//
// Every kernel is bandwidth-bound (a variable-coefficient nearest-neighbour
// stencil or a vector update with reductions), so there is no matrix-core
// work.  Design points:
//  - fields live in a padded row-major layout (pitch a multiple of 64
//    doubles), so one wavefront reads 64 consecutive elements of a row;
//  - a work-group is 256 threads (4 wavefronts) and owns a 64 x TY tile;
//    tiles are numbered so that each of the 8 XCDs works on a contiguous
//    band of rows (the L2 of that XCD then serves the halo rows);
//  - stencil neighbours are read straight from global memory (L1/L2 hits);
//  - reductions: wavefront shuffles, one block-level pass, per-block
//    partials, and the last block to finish (atomic counter) reduces the
//    partials in a fixed order and updates the solver scalars on the device.
//    Results are therefore deterministic and the host never computes alpha
//    or beta: it only reads a done flag every few iterations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "ccns.h"
#include "ccns_internal.h"

namespace ccns {

constexpr int NT = 256;  // threads per work-group
constexpr int TX = 64;   // tile width (one wavefront)
constexpr int TR = 2;    // rows per thread
constexpr int TY = 4 * TR;
constexpr int NRED = 8;  // reduction slots per block

struct Dims {
    int nx, ny, rows, pitch;
    int gx, gy, ntile, ncomp;  // tiles per component; components (1 cells, 2 faces)
    int nlaunch;               // launched blocks (multiple of 8)
    size_t n;                  // elements per component array
};

struct CgState {
    double alpha, beta, rz, mean, fnorm2, rnorm2, tol2, pq, mean_b;
    int it, maxit, done, status, zero_mean, n_active;
    unsigned counter;
    int pad;
};

struct DiagState {
    double mass, ke, momx, momy, divmax;
    unsigned counter;
    int pad;
};

// ---------------------------------------------------------------------------
// tile mapping and reductions
// ---------------------------------------------------------------------------

// Physical block b runs on XCD b % 8; give each XCD a contiguous range of
// logical tiles so that vertically adjacent tiles share an L2.
__device__ inline int logical_block(int nlaunch) {
    const int b = blockIdx.x;
    const int per = nlaunch >> 3;
    return (b & 7) * per + (b >> 3);
}

__device__ inline double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}
__device__ inline double wave_max(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
    return v;
}

// Block-level sums (NS slots) and maxima (NM slots); result valid in sh[] for
// every thread after the call.
template <int NS, int NM>
__device__ inline void block_reduce(double (&v)[NS + NM], double *sh) {
    __shared__ double part[NRED][4];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NS + NM; ++k) {
        double s = (k < NS) ? wave_sum(v[k]) : wave_max(v[k]);
        if (lane == 0) part[k][w] = s;
    }
    __syncthreads();
    if (threadIdx.x < NS + NM) {
        const int k = threadIdx.x;
        sh[k] = (k < NS) ? ((part[k][0] + part[k][1]) + (part[k][2] + part[k][3]))
                         : fmax(fmax(part[k][0], part[k][1]), fmax(part[k][2], part[k][3]));
    }
    __syncthreads();
}

// Writes this block's partials; returns true in every thread of the last
// block to arrive, with the grid totals (fixed reduction order) in tot[].
template <int NS, int NM>
__device__ inline bool grid_reduce(double (&v)[NS + NM], double *partials, unsigned *counter, int nlaunch,
                                   double (&tot)[NS + NM]) {
    __shared__ double sh[NRED];
    __shared__ int amlast;
    block_reduce<NS, NM>(v, sh);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NS + NM; ++k) partials[(size_t)blockIdx.x * NRED + k] = sh[k];
        __threadfence();
        unsigned t = atomicAdd(counter, 1u);
        amlast = (t == (unsigned)nlaunch - 1u);
    }
    __syncthreads();
    if (!amlast) return false;
    __threadfence();
    double acc[NS + NM];
#pragma unroll
    for (int k = 0; k < NS + NM; ++k) acc[k] = (k < NS) ? 0.0 : -INFINITY;
    const volatile double *vp = partials;
    for (int b = threadIdx.x; b < nlaunch; b += NT) {
#pragma unroll
        for (int k = 0; k < NS + NM; ++k) {
            double x = vp[(size_t)b * NRED + k];
            acc[k] = (k < NS) ? acc[k] + x : fmax(acc[k], x);
        }
    }
    block_reduce<NS, NM>(acc, sh);
#pragma unroll
    for (int k = 0; k < NS + NM; ++k) tot[k] = sh[k];
    if (threadIdx.x == 0) *counter = 0u;
    return true;
}

// Iterates over the cells (or faces) of this block's tile: f(comp, j, i, k).
template <class F>
__device__ inline void for_tile(const Dims &d, F f) {
    const int L = logical_block(d.nlaunch);
    if (L >= d.ntile * d.ncomp) return;
    const int comp = L / d.ntile, t = L % d.ntile;
    const int c0 = (t % d.gx) * TX, r0 = (t / d.gx) * TY;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int i = c0 + tx;
#pragma unroll
    for (int rr = 0; rr < TR; ++rr) {
        const int j = r0 + ty + 4 * rr;
        if (j < d.rows) f(comp, j, i, (size_t)j * d.pitch + i);
    }
}

// ---------------------------------------------------------------------------
// operator building blocks (index form of Sec. 4; k = j*pitch + i)
// ---------------------------------------------------------------------------

struct ViscCoef {
    const double *bxx, *bxy, *byy, *byx, *wxx, *wyy, *nxx, *nxy, *nyx, *nyy;
};

// visc(strain(p, 0)) at x-face k (eq:diag, eq:offdiag, Sec. 4.3) for a
// face vector given by loaders px(k), py(k).
template <class PX, class PY>
__device__ inline double visc_x(const ViscCoef &c, size_t k, size_t P, PX px, PY py) {
    const double sxx_e = c.wxx[k + 1] * (c.bxx[k + 1] * px(k + 1) - c.bxx[k] * px(k));
    const double sxx_w = c.wxx[k] * (c.bxx[k] * px(k) - c.bxx[k - 1] * px(k - 1));
    const size_t s = k - P;
    const double gxn = c.bxy[k + P] * px(k + P) - c.bxy[k] * px(k);
    const double gyn = c.byx[k + 1] * py(k + 1) - c.byx[k] * py(k);
    const double gxs = c.bxy[k] * px(k) - c.bxy[s] * px(s);
    const double gys = c.byx[s + 1] * py(s + 1) - c.byx[s] * py(s);
    const double sn = 0.5 * (c.nxx[k] * gxn + c.nxy[k] * gyn);
    const double ss = 0.5 * (c.nxx[s] * gxs + c.nxy[s] * gys);
    return c.bxx[k] * (sxx_e - sxx_w) + c.bxy[k] * (sn - ss);
}

template <class PX, class PY>
__device__ inline double visc_y(const ViscCoef &c, size_t k, size_t P, PX px, PY py) {
    const double syy_n = c.wyy[k + P] * (c.byy[k + P] * py(k + P) - c.byy[k] * py(k));
    const double syy_s = c.wyy[k] * (c.byy[k] * py(k) - c.byy[k - P] * py(k - P));
    const size_t w = k - 1;
    const double gxe = c.bxy[k + P] * px(k + P) - c.bxy[k] * px(k);
    const double gye = c.byx[k + 1] * py(k + 1) - c.byx[k] * py(k);
    const double gxw = c.bxy[w + P] * px(w + P) - c.bxy[w] * px(w);
    const double gyw = c.byx[k] * py(k) - c.byx[w] * py(w);
    const double se = 0.5 * (c.nyx[k] * gxe + c.nyy[k] * gye);
    const double sw = 0.5 * (c.nyx[w] * gxw + c.nyy[w] * gyw);
    return c.byy[k] * (syy_n - syy_s) + c.byx[k] * (se - sw);
}

// conv(U, U, D, D) at x-face k and y-face k (eq:convective in index form).
__device__ inline double conv_x(const double *ax, const double *ay, const double *ux, const double *uy,
                                const double *hbx, const double *dx, size_t k, size_t P) {
    auto Fxx = [&](size_t c) { return 0.25 * (ax[c - 1] * ux[c - 1] + ax[c] * ux[c]) * (ux[c - 1] + ux[c]); };
    auto Fxy = [&](size_t nd) { return 0.25 * (ay[nd] * uy[nd] + ay[nd + 1] * uy[nd + 1]) * (ux[nd] + ux[nd + P]); };
    return Fxx(k + 1) - Fxx(k) + Fxy(k) - Fxy(k - P) + hbx[k] * (ux[k] + dx[k]);
}
__device__ inline double conv_y(const double *ax, const double *ay, const double *ux, const double *uy,
                                const double *hby, const double *dy, size_t k, size_t P) {
    auto Fyy = [&](size_t c) { return 0.25 * (ay[c - P] * uy[c - P] + ay[c] * uy[c]) * (uy[c - P] + uy[c]); };
    auto Fyx = [&](size_t nd) { return 0.25 * (ax[nd] * ux[nd] + ax[nd + P] * ux[nd + P]) * (uy[nd] + uy[nd + 1]); };
    return Fyy(k + P) - Fyy(k) + Fyx(k) - Fyx(k - 1) + hby[k] * (uy[k] + dy[k]);
}

// ---------------------------------------------------------------------------
// Poisson PCG kernels (A = -L, SPD on the zero-mean space)
// ---------------------------------------------------------------------------

struct PoisCoef {
    const double *cx, *cy, *dinv;
};

// b = (rho/tau) cont(U*, D) on pressure unknowns; mean of b; resets the solver.
__global__ __launch_bounds__(NT) void k_pois_rhs(Dims d, PoisCoef pc, const double *__restrict__ ax,
                                                 const double *__restrict__ ay, const double *__restrict__ het,
                                                 const double *__restrict__ usx, const double *__restrict__ usy,
                                                 double *__restrict__ b, double scale, CgState *st,
                                                 double *partials) {
    const size_t P = d.pitch;
    double v[1] = {0.0};
    for_tile(d, [&](int, int j, int i, size_t k) {
        if (i < 1 || i > d.nx || j < 1 || j > d.ny) return;
        if (pc.dinv[k] > 0.0) {
            double c = ax[k] * usx[k] - ax[k - 1] * usx[k - 1] + ay[k] * usy[k] - ay[k - P] * usy[k - P] + het[k];
            double bv = scale * c;
            b[k] = bv;
            v[0] += bv;
        }
    });
    double tot[1];
    if (grid_reduce<1, 0>(v, partials, &st->counter, d.nlaunch, tot) && threadIdx.x == 0) {
        st->mean_b = tot[0] / (double)st->n_active;
        st->done = 0;
        st->status = 0;
        st->it = 0;
    }
}

// Sum of b over the unknowns (caller-provided b); resets the solver.
__global__ __launch_bounds__(NT) void k_pois_mean(Dims d, PoisCoef pc, const double *__restrict__ b, CgState *st,
                                                  double *partials) {
    double v[1] = {0.0};
    for_tile(d, [&](int, int j, int i, size_t k) {
        if (pc.dinv[k] > 0.0) v[0] += b[k];
    });
    double tot[1];
    if (grid_reduce<1, 0>(v, partials, &st->counter, d.nlaunch, tot) && threadIdx.x == 0) {
        st->mean_b = tot[0] / (double)st->n_active;
        st->done = 0;
        st->status = 0;
        st->it = 0;
    }
}

// b <- b - mean(b); f = -b; r = f - A x; first preconditioned residual.
__global__ __launch_bounds__(NT) void k_pois_init(Dims d, PoisCoef pc, double *__restrict__ b,
                                                  const double *__restrict__ x, double *__restrict__ r, CgState *st,
                                                  double *partials) {
    const size_t P = d.pitch;
    const double mb = st->mean_b;
    double v[5] = {0, 0, 0, 0, 0};
    for_tile(d, [&](int, int j, int i, size_t k) {
        const double dv = pc.dinv[k];
        if (!(dv > 0.0)) return;
        const double bp = b[k] - mb;
        b[k] = bp;
        const double ce = pc.cx[k], cw = pc.cx[k - 1], cn = pc.cy[k], cs = pc.cy[k - P];
        const double Axv = (ce + cw + cn + cs) * x[k] - ce * x[k + 1] - cw * x[k - 1] - cn * x[k + P] - cs * x[k - P];
        const double rv = -bp - Axv;
        r[k] = rv;
        const double s = dv * rv;
        v[0] += bp * bp;
        v[1] += rv * s;
        v[2] += s;
        v[3] += rv;
        v[4] += rv * rv;
    });
    double tot[5];
    if (grid_reduce<5, 0>(v, partials, &st->counter, d.nlaunch, tot) && threadIdx.x == 0) {
        st->fnorm2 = tot[0];
        const double m = st->zero_mean ? tot[2] / (double)st->n_active : 0.0;
        st->mean = m;
        st->rz = tot[1] - m * tot[3];
        st->rnorm2 = tot[4];
        st->beta = 0.0;
        st->it = 0;
        st->done = (tot[4] <= st->tol2 * tot[0]) ? 1 : 0;
        st->status = 0;
    }
}

// p = (M r) + beta p_old on the stencil; q = A p; partial p.q -> alpha.
__global__ __launch_bounds__(NT) void k_pois_dir_apply(Dims d, PoisCoef pc, const double *__restrict__ r,
                                                       const double *__restrict__ pold, double *__restrict__ pnew,
                                                       double *__restrict__ q, CgState *st, double *partials) {
    if (st->done) return;
    const size_t P = d.pitch;
    const double beta = st->beta, m = st->mean;
    double v[1] = {0.0};
    for_tile(d, [&](int, int j, int i, size_t k) {
        const double dv = pc.dinv[k];
        if (!(dv > 0.0)) return;
        auto pn = [&](size_t kk) {
            const double di = pc.dinv[kk];
            return di > 0.0 ? (di * r[kk] - m) + beta * pold[kk] : 0.0;
        };
        const double pcv = (dv * r[k] - m) + beta * pold[k];
        const double ce = pc.cx[k], cw = pc.cx[k - 1], cn = pc.cy[k], cs = pc.cy[k - P];
        const double qv = (ce + cw + cn + cs) * pcv - ce * pn(k + 1) - cw * pn(k - 1) - cn * pn(k + P) - cs * pn(k - P);
        pnew[k] = pcv;
        q[k] = qv;
        v[0] += pcv * qv;
    });
    double tot[1];
    if (grid_reduce<1, 0>(v, partials, &st->counter, d.nlaunch, tot) && threadIdx.x == 0) {
        st->pq = tot[0];
        if (!(tot[0] > 0.0)) {
            st->done = 1;
            st->status = CCNS_EBREAKDOWN;
        } else {
            st->alpha = st->rz / tot[0];
        }
    }
}

// x += alpha p; r -= alpha q; z = M r statistics -> beta, convergence.
// Flat over ncomp*n elements (inactive entries hold zeros).
__global__ __launch_bounds__(NT) void k_cg_update(size_t ntot, int nlaunch, const double *__restrict__ dinv,
                                                  double *__restrict__ x, double *__restrict__ r,
                                                  const double *__restrict__ p, const double *__restrict__ q,
                                                  CgState *st, double *partials) {
    if (st->done) return;
    const double a = st->alpha;
    double v[4] = {0, 0, 0, 0};
    const size_t stride = (size_t)nlaunch * NT;
    for (size_t k = (size_t)blockIdx.x * NT + threadIdx.x; k < ntot; k += stride) {
        const double dv = dinv[k];
        if (!(dv > 0.0)) continue;
        x[k] += a * p[k];
        const double rv = r[k] - a * q[k];
        r[k] = rv;
        const double s = dv * rv;
        v[0] += rv * s;
        v[1] += s;
        v[2] += rv;
        v[3] += rv * rv;
    }
    double tot[4];
    if (grid_reduce<4, 0>(v, partials, &st->counter, nlaunch, tot) && threadIdx.x == 0) {
        const double m = st->zero_mean ? tot[1] / (double)st->n_active : 0.0;
        const double rz = tot[0] - m * tot[2];
        st->beta = rz / st->rz;
        st->rz = rz;
        st->mean = m;
        st->rnorm2 = tot[3];
        st->it += 1;
        if (tot[3] <= st->tol2 * st->fnorm2) {
            st->done = 1;
            st->status = CCNS_OK;
        } else if (st->it >= st->maxit) {
            st->done = 1;
            st->status = CCNS_ENOTCONV;
        }
    }
}

// ---------------------------------------------------------------------------
// predictor (eq:pm_prediction): H = (rho/tau) V - mu visc(strain(., 0))
// ---------------------------------------------------------------------------

struct PredCoef {
    ViscCoef vc;
    const double *vu, *vv, *hdx, *hdy;
    double rt, mu;
};

// conv^n, the predictor right-hand side, and U* := U^n as the start value.
__global__ __launch_bounds__(NT) void k_pred_rhs(Dims d, PredCoef pc, const double *__restrict__ ax,
                                                 const double *__restrict__ ay, const double *__restrict__ hbx,
                                                 const double *__restrict__ hby, const double *__restrict__ dx,
                                                 const double *__restrict__ dy, const double *__restrict__ ux,
                                                 const double *__restrict__ uy, const double *__restrict__ pr,
                                                 const double *__restrict__ vdx, const double *__restrict__ vdy,
                                                 double *__restrict__ convx, double *__restrict__ convy,
                                                 double *__restrict__ rhs, double *__restrict__ xs, double rho,
                                                 double gxv, double gyv, int conv_valid) {
    const size_t P = d.pitch, n = d.n;
    for_tile(d, [&](int comp, int j, int i, size_t k) {
        auto pxm = [&](size_t kk) { return pc.vu[kk] > 0.0 ? ux[kk] : 0.0; };
        auto pym = [&](size_t kk) { return pc.vv[kk] > 0.0 ? uy[kk] : 0.0; };
        if (comp == 0) {
            xs[k] = ux[k];
            if (!(pc.vu[k] > 0.0)) { rhs[k] = 0.0; return; }
            const double cv = conv_x(ax, ay, ux, uy, hbx, dx, k, P);
            const double cold = conv_valid ? convx[k] : cv;
            convx[k] = cv;
            const double presv = ax[k] * (pr[k + 1] - pr[k]);
            const double kv = visc_x(pc.vc, k, P, pxm, pym);
            rhs[k] = pc.rt * pc.vu[k] * ux[k] - 1.5 * rho * cv + 0.5 * rho * cold - presv +
                     pc.mu * (kv + 2.0 * vdx[k]) + rho * pc.vu[k] * gxv;
        } else {
            xs[n + k] = uy[k];
            if (!(pc.vv[k] > 0.0)) { rhs[n + k] = 0.0; return; }
            const double cv = conv_y(ax, ay, ux, uy, hby, dy, k, P);
            const double cold = conv_valid ? convy[k] : cv;
            convy[k] = cv;
            const double presv = ay[k] * (pr[k + P] - pr[k]);
            const double kv = visc_y(pc.vc, k, P, pxm, pym);
            rhs[n + k] = pc.rt * pc.vv[k] * uy[k] - 1.5 * rho * cv + 0.5 * rho * cold - presv +
                         pc.mu * (kv + 2.0 * vdy[k]) + rho * pc.vv[k] * gyv;
        }
    });
}

// r = rhs - H x0 (x0 masked to the unknowns); solver statistics.
__global__ __launch_bounds__(NT) void k_pred_init(Dims d, PredCoef pc, const double *__restrict__ rhs,
                                                  const double *__restrict__ xs, double *__restrict__ r, CgState *st,
                                                  double *partials) {
    const size_t P = d.pitch, n = d.n;
    const double *xu = xs, *xv = xs + n;
    auto pxm = [&](size_t kk) { return pc.vu[kk] > 0.0 ? xu[kk] : 0.0; };
    auto pym = [&](size_t kk) { return pc.vv[kk] > 0.0 ? xv[kk] : 0.0; };
    double v[5] = {0, 0, 0, 0, 0};
    for_tile(d, [&](int comp, int j, int i, size_t k) {
        double hv, f, dv;
        size_t o;
        if (comp == 0) {
            if (!(pc.vu[k] > 0.0)) return;
            hv = pc.rt * pc.vu[k] * xu[k] - pc.mu * visc_x(pc.vc, k, P, pxm, pym);
            o = k;
            dv = pc.hdx[k];
        } else {
            if (!(pc.vv[k] > 0.0)) return;
            hv = pc.rt * pc.vv[k] * xv[k] - pc.mu * visc_y(pc.vc, k, P, pxm, pym);
            o = n + k;
            dv = pc.hdy[k];
        }
        f = rhs[o];
        const double rv = f - hv;
        r[o] = rv;
        const double s = dv * rv;
        v[0] += f * f;
        v[1] += rv * s;
        v[2] += s;
        v[3] += rv;
        v[4] += rv * rv;
    });
    double tot[5];
    if (grid_reduce<5, 0>(v, partials, &st->counter, d.nlaunch, tot) && threadIdx.x == 0) {
        st->fnorm2 = tot[0];
        st->mean = 0.0;
        st->rz = tot[1];
        st->rnorm2 = tot[4];
        st->beta = 0.0;
        st->it = 0;
        st->done = (tot[4] <= st->tol2 * tot[0]) ? 1 : 0;
        st->status = 0;
    }
}

__global__ __launch_bounds__(NT) void k_pred_dir_apply(Dims d, PredCoef pc, const double *__restrict__ r,
                                                       const double *__restrict__ pold, double *__restrict__ pnew,
                                                       double *__restrict__ q, CgState *st, double *partials) {
    if (st->done) return;
    const size_t P = d.pitch, n = d.n;
    const double beta = st->beta;
    auto pnx = [&](size_t kk) { return pc.hdx[kk] * r[kk] + beta * pold[kk]; };
    auto pny = [&](size_t kk) { return pc.hdy[kk] * r[n + kk] + beta * pold[n + kk]; };
    double v[1] = {0.0};
    for_tile(d, [&](int comp, int j, int i, size_t k) {
        if (comp == 0) {
            if (!(pc.vu[k] > 0.0)) return;
            const double pv = pnx(k);
            const double qv = pc.rt * pc.vu[k] * pv - pc.mu * visc_x(pc.vc, k, P, pnx, pny);
            pnew[k] = pv;
            q[k] = qv;
            v[0] += pv * qv;
        } else {
            if (!(pc.vv[k] > 0.0)) return;
            const double pv = pny(k);
            const double qv = pc.rt * pc.vv[k] * pv - pc.mu * visc_y(pc.vc, k, P, pnx, pny);
            pnew[n + k] = pv;
            q[n + k] = qv;
            v[0] += pv * qv;
        }
    });
    double tot[1];
    if (grid_reduce<1, 0>(v, partials, &st->counter, d.nlaunch, tot) && threadIdx.x == 0) {
        st->pq = tot[0];
        if (!(tot[0] > 0.0)) {
            st->done = 1;
            st->status = CCNS_EBREAKDOWN;
        } else {
            st->alpha = st->rz / tot[0];
        }
    }
}

// ---------------------------------------------------------------------------
// corrector, pressure update and diagnostics
// ---------------------------------------------------------------------------

// U^{n+1} = U* - (tau/rho) (A/V_f) dPhi on pressure-coupled faces (eq:pm_projection).
__global__ __launch_bounds__(NT) void k_correct(Dims d, const double *__restrict__ gx, const double *__restrict__ gy,
                                                const double *__restrict__ usx, const double *__restrict__ usy,
                                                const double *__restrict__ phi, double *__restrict__ ux,
                                                double *__restrict__ uy, double s) {
    const size_t P = d.pitch;
    for_tile(d, [&](int, int j, int i, size_t k) {
        const double g1 = gx[k], g2 = gy[k];
        ux[k] = (g1 != 0.0) ? usx[k] - s * g1 * (phi[k + 1] - phi[k]) : usx[k];
        uy[k] = (g2 != 0.0) ? usy[k] - s * g2 * (phi[k + P] - phi[k]) : usy[k];
    });
}

struct DiagCoef {
    const double *ax, *ay, *het, *dinv, *vur, *vvr, *vu, *vv, *cx, *cy, *vinv;
};

// Divergence max / net flux, kinetic energy and momentum of U; optionally
// P += Phi - (tau mu / 2 rho) V^-1 L Phi (eq:pm_update).
__global__ __launch_bounds__(NT) void k_diag(Dims d, DiagCoef c, const double *__restrict__ ux,
                                             const double *__restrict__ uy, const double *__restrict__ phi,
                                             double *__restrict__ pr, double pcoef, int update_p, double rho,
                                             DiagState *ds, double *partials) {
    const size_t P = d.pitch;
    double v[5] = {0, 0, 0, 0, 0};
    for_tile(d, [&](int, int j, int i, size_t k) {
        v[2] += rho * c.vu[k] * ux[k];
        v[3] += rho * c.vv[k] * uy[k];
        if (i < 1 || i > d.nx || j < 1 || j > d.ny) return;
        const double dv = c.ax[k] * ux[k] - c.ax[k - 1] * ux[k - 1] + c.ay[k] * uy[k] - c.ay[k - P] * uy[k - P] + c.het[k];
        v[0] += dv;
        v[1] += 0.25 * (c.vur[k - 1] * ux[k - 1] * ux[k - 1] + c.vur[k] * ux[k] * ux[k] +
                        c.vvr[k - P] * uy[k - P] * uy[k - P] + c.vvr[k] * uy[k] * uy[k]);
        if (c.dinv[k] > 0.0) {
            v[4] = fmax(v[4], fabs(dv));
            if (update_p) {
                const double ph = phi[k];
                const double lp = c.cx[k] * (phi[k + 1] - ph) - c.cx[k - 1] * (ph - phi[k - 1]) +
                                  c.cy[k] * (phi[k + P] - ph) - c.cy[k - P] * (ph - phi[k - P]);
                pr[k] = pr[k] + ph - pcoef * c.vinv[k] * lp;
            }
        }
    });
    double tot[5];
    if (grid_reduce<4, 1>(v, partials, &ds->counter, d.nlaunch, tot) && threadIdx.x == 0) {
        ds->mass = tot[0];
        ds->ke = tot[1];
        ds->momx = tot[2];
        ds->momy = tot[3];
        ds->divmax = tot[4];
    }
}

// ---------------------------------------------------------------------------
// operator applies (parity entry points)
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(NT) void k_op_cont(Dims d, const double *ax, const double *ay, const double *het,
                                                const double *ux, const double *uy, double *out) {
    const size_t P = d.pitch;
    for_tile(d, [&](int, int j, int i, size_t k) {
        if (i < 1 || i > d.nx || j < 1 || j > d.ny || i >= d.nx + 2) { out[k] = 0.0; return; }
        out[k] = ax[k] * ux[k] - ax[k - 1] * ux[k - 1] + ay[k] * uy[k] - ay[k - P] * uy[k - P] + het[k];
    });
}

__global__ __launch_bounds__(NT) void k_op_pres(Dims d, const double *ax, const double *ay, const double *p,
                                                double *gx, double *gy) {
    const size_t P = d.pitch;
    for_tile(d, [&](int, int j, int i, size_t k) {
        auto pv = [&](int jj, int ii) {
            return (ii >= 1 && ii <= d.nx && jj >= 1 && jj <= d.ny) ? p[(size_t)jj * P + ii] : 0.0;
        };
        gx[k] = (i >= 0 && i <= d.nx && j >= 1 && j <= d.ny) ? ax[k] * (pv(j, i + 1) - pv(j, i)) : 0.0;
        gy[k] = (i >= 1 && i <= d.nx && j >= 0 && j <= d.ny) ? ay[k] * (pv(j + 1, i) - pv(j, i)) : 0.0;
    });
}

// mode 0: visc(strain(U, D)) = K U_unknowns + vD; mode 1: H p (p masked).
__global__ __launch_bounds__(NT) void k_op_visc(Dims d, PredCoef pc, const double *vdx, const double *vdy,
                                                const double *ux, const double *uy, double *ox, double *oy,
                                                int mode) {
    const size_t P = d.pitch;
    auto pxm = [&](size_t kk) { return pc.vu[kk] > 0.0 ? ux[kk] : 0.0; };
    auto pym = [&](size_t kk) { return pc.vv[kk] > 0.0 ? uy[kk] : 0.0; };
    for_tile(d, [&](int, int j, int i, size_t k) {
        double a = 0.0, b = 0.0;
        if (pc.vu[k] > 0.0) {
            const double kv = visc_x(pc.vc, k, P, pxm, pym);
            a = mode == 0 ? kv + vdx[k] : pc.rt * pc.vu[k] * ux[k] - pc.mu * kv;
        }
        if (pc.vv[k] > 0.0) {
            const double kv = visc_y(pc.vc, k, P, pxm, pym);
            b = mode == 0 ? kv + vdy[k] : pc.rt * pc.vv[k] * uy[k] - pc.mu * kv;
        }
        ox[k] = a;
        oy[k] = b;
    });
}

__global__ __launch_bounds__(NT) void k_op_conv(Dims d, const double *ax, const double *ay, const double *hbx,
                                                const double *hby, const double *dx, const double *dy,
                                                const double *ux, const double *uy, double *ox, double *oy) {
    const size_t P = d.pitch;
    for_tile(d, [&](int, int j, int i, size_t k) {
        ox[k] = (i >= 1 && i <= d.nx - 1 && j >= 1 && j <= d.ny) ? conv_x(ax, ay, ux, uy, hbx, dx, k, P) : 0.0;
        oy[k] = (i >= 1 && i <= d.nx && j >= 1 && j <= d.ny - 1) ? conv_y(ax, ay, ux, uy, hby, dy, k, P) : 0.0;
    });
}

__global__ __launch_bounds__(NT) void k_op_lap(Dims d, PoisCoef pc, const double *phi, double *out) {
    const size_t P = d.pitch;
    for_tile(d, [&](int, int j, int i, size_t k) {
        if (!(pc.dinv[k] > 0.0)) { out[k] = 0.0; return; }
        const double ph = phi[k];
        out[k] = pc.cx[k] * (phi[k + 1] - ph) - pc.cx[k - 1] * (ph - phi[k - 1]) + pc.cy[k] * (phi[k + P] - ph) -
                 pc.cy[k - P] * (ph - phi[k - P]);
    });
}

__global__ __launch_bounds__(NT) void k_op_kin(Dims d, const double *vur, const double *vvr, const double *ux,
                                               const double *uy, double *out) {
    const size_t P = d.pitch;
    for_tile(d, [&](int, int j, int i, size_t k) {
        if (i < 1 || i > d.nx || j < 1 || j > d.ny) { out[k] = 0.0; return; }
        out[k] = 0.25 * (vur[k - 1] * ux[k - 1] * ux[k - 1] + vur[k] * ux[k] * ux[k] +
                         vvr[k - P] * uy[k - P] * uy[k - P] + vvr[k] * uy[k] * uy[k]);
    });
}

}  // namespace ccns

// ===========================================================================
// host side
// ===========================================================================

using namespace ccns;

namespace {

// Names of the FP64 workspace arrays, in allocation order.
enum Arr {
    A_CX, A_CY, A_DINV, A_GX, A_GY, A_AX, A_AY, A_HET, A_HBX, A_HBY, A_DX, A_DY, A_VU, A_VV,
    A_BXX, A_BXY, A_BYY, A_BYX, A_WXX, A_WYY, A_NXX, A_NXY, A_NYX, A_NYY,
    A_HDX, A_HDY,  // contiguous pair
    A_VINV, A_VUR, A_VVR, A_VDX, A_VDY,
    A_UX, A_UY, A_P, A_PHI, A_CONVX, A_CONVY,
    A_USX, A_USY,    // predictor x (contiguous pair)
    A_PRX, A_PRY,    // predictor r
    A_PP0X, A_PP0Y,  // predictor p (ping)
    A_PP1X, A_PP1Y,  // predictor p (pong)
    A_PQX, A_PQY,    // predictor q
    A_RHSX, A_RHSY,  // predictor right-hand side
    A_B, A_R, A_P0, A_P1, A_Q,  // Poisson
    A_T0, A_T1, A_T2, A_T3,     // scratch for operator applies
    A_COUNT
};

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct WsPlan {
    Layout L;
    size_t arr_bytes;   // bytes per array
    size_t part_off, part_bytes, state_off, total;
    int nlaunch_max;
};

WsPlan plan(int nx, int ny) {
    WsPlan w;
    w.L = make_layout(nx, ny);
    w.arr_bytes = align_up(w.L.n * sizeof(double), 256);
    int gx = w.L.pitch / TX, gy = (w.L.rows + TY - 1) / TY;
    int ntile2 = 2 * gx * gy;
    w.nlaunch_max = std::max(((ntile2 + 7) / 8) * 8, 2048);
    w.part_off = w.arr_bytes * A_COUNT;
    w.part_bytes = align_up((size_t)w.nlaunch_max * NRED * sizeof(double), 256);
    w.state_off = w.part_off + w.part_bytes;
    w.total = w.state_off + 4096;
    return w;
}

}  // namespace

struct ccns_ctx {
    ccns_grid g;
    ccns_params prm;
    WsPlan w;
    hipStream_t stream;
    char *base;
    double *a[A_COUNT];
    double *partials;
    CgState *st_pred, *st_pois;
    DiagState *diag;
    CgState *h_st;      // pinned host copies
    DiagState *h_diag;
    Dims dc, df;        // cell tiles (1 component) and face tiles (2 components)
    int conv_valid;
    int n_active;
    int last_pois_it, last_pred_it;
    int pbuf_pred, pbuf_pois;
    // optional kernel timing: events around every 4th CG iteration
    int timing;
    std::vector<hipEvent_t> evpool;
    size_t evused;
    double t_ms[4];    // Poisson dir-apply, Poisson update, predictor dir-apply, predictor update
    long t_count[4];
    std::string err;
};

namespace {

ccns_status fail(ccns_ctx *c, ccns_status s, const std::string &msg) {
    if (c) c->err = msg;
    return s;
}

#define HIPCHK(ctx, call)                                                                   \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(ctx, CCNS_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

Dims make_dims(const Layout &L, int ncomp) {
    Dims d;
    d.nx = L.nx;
    d.ny = L.ny;
    d.rows = L.rows;
    d.pitch = L.pitch;
    d.gx = L.pitch / TX;
    d.gy = (L.rows + TY - 1) / TY;
    d.ntile = d.gx * d.gy;
    d.ncomp = ncomp;
    d.nlaunch = ((d.ntile * ncomp + 7) / 8) * 8;
    d.n = L.n;
    return d;
}

PoisCoef pois_coef(ccns_ctx *c) { return PoisCoef{c->a[A_CX], c->a[A_CY], c->a[A_DINV]}; }

PredCoef pred_coef(ccns_ctx *c) {
    PredCoef p;
    p.vc = ViscCoef{c->a[A_BXX], c->a[A_BXY], c->a[A_BYY], c->a[A_BYX], c->a[A_WXX],
                    c->a[A_WYY], c->a[A_NXX], c->a[A_NXY], c->a[A_NYX], c->a[A_NYY]};
    p.vu = c->a[A_VU];
    p.vv = c->a[A_VV];
    p.hdx = c->a[A_HDX];
    p.hdy = c->a[A_HDY];
    p.rt = c->prm.rho / c->prm.tau;
    p.mu = c->prm.mu;
    return p;
}

// dense (ny+2)x(nx+2) <-> padded device array
ccns_status to_dev(ccns_ctx *c, double *dst, const double *src, hipMemcpyKind kind) {
    const size_t W = c->g.nx + 2;
    HIPCHK(c, hipMemcpy2DAsync(dst, c->w.L.pitch * sizeof(double), src, W * sizeof(double), W * sizeof(double),
                               c->g.ny + 2, kind, c->stream));
    return CCNS_OK;
}
ccns_status from_dev(ccns_ctx *c, double *dst, const double *src, hipMemcpyKind kind) {
    const size_t W = c->g.nx + 2;
    HIPCHK(c, hipMemcpy2DAsync(dst, W * sizeof(double), src, c->w.L.pitch * sizeof(double), W * sizeof(double),
                               c->g.ny + 2, kind, c->stream));
    return CCNS_OK;
}

// Blocks of an element-wise kernel over ntot entries (about 8 per thread).
int flat_blocks(size_t ntot) {
    size_t b = (ntot + (size_t)NT * 8 - 1) / ((size_t)NT * 8);
    b = std::min<size_t>(std::max<size_t>(b, 8), 2048);
    return (int)((b + 7) / 8 * 8);
}

// Runs CG iterations until the device flags convergence; reads the state.
hipEvent_t next_event(ccns_ctx *c) {
    if (c->evused == c->evpool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        c->evpool.push_back(e);
    }
    return c->evpool[c->evused++];
}

// Adds the durations of the sampled launches recorded since the last call.
void harvest_events(ccns_ctx *c, int kid) {
    for (size_t k = 0; k + 3 <= c->evused; k += 3) {
        float a = 0.f, b = 0.f;
        if (hipEventElapsedTime(&a, c->evpool[k], c->evpool[k + 1]) == hipSuccess &&
            hipEventElapsedTime(&b, c->evpool[k + 1], c->evpool[k + 2]) == hipSuccess) {
            c->t_ms[kid] += a;
            c->t_ms[kid + 1] += b;
            c->t_count[kid] += 1;
            c->t_count[kid + 1] += 1;
        }
    }
    c->evused = 0;
}

template <class DirApply>
ccns_status cg_loop(ccns_ctx *c, CgState *st, double *x, double *r, double *const pbuf[2], int &par, double *q,
                    const double *dinv, size_t ntot, int &last_it, DirApply dir_apply, ccns_solve_info *info,
                    int kid) {
    int chunk = std::max(8, (int)(0.9 * last_it));
    const int nl = flat_blocks(ntot);
    HIPCHK(c, hipMemcpyAsync(c->h_st, st, sizeof(CgState), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    int issued = 0;
    while (!c->h_st->done) {
        for (int it = 0; it < chunk; ++it, ++issued) {
            // timed launches stop at the predicted count so that no early-exit
            // launch after convergence is sampled
            const bool tm = c->timing && (issued % 4 == 0) && issued < last_it;
            if (tm) (void)hipEventRecord(next_event(c), c->stream);
            dir_apply(pbuf[par], pbuf[par ^ 1]);
            if (tm) (void)hipEventRecord(next_event(c), c->stream);
            k_cg_update<<<nl, NT, 0, c->stream>>>(ntot, nl, dinv, x, r, pbuf[par ^ 1], q, st, c->partials);
            if (tm) (void)hipEventRecord(next_event(c), c->stream);
            par ^= 1;
        }
        HIPCHK(c, hipGetLastError());
        HIPCHK(c, hipMemcpyAsync(c->h_st, st, sizeof(CgState), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        if (c->timing) harvest_events(c, kid);
        chunk = 32;
    }
    last_it = c->h_st->it;
    if (info) {
        info->iterations = c->h_st->it;
        info->outer = 1;
        info->rel_residual = c->h_st->fnorm2 > 0 ? std::sqrt(c->h_st->rnorm2 / c->h_st->fnorm2) : 0.0;
        info->status = c->h_st->status;
    }
    return (ccns_status)c->h_st->status;
}

void set_cg(ccns_ctx *c, CgState *st, double tol, int maxit, int zero_mean, int n_active) {
    CgState h{};
    h.tol2 = tol * tol;
    h.maxit = maxit;
    h.zero_mean = zero_mean;
    h.n_active = std::max(n_active, 1);
    h.done = 1;
    (void)hipMemcpyAsync(st, &h, sizeof(CgState), hipMemcpyHostToDevice, c->stream);
}

ccns_status pressure_solve_dev(ccns_ctx *c, ccns_solve_info *info) {
    // b is in A_B with its mean computed; phi (A_PHI) is the start value
    PoisCoef pc = pois_coef(c);
    k_pois_init<<<c->dc.nlaunch, NT, 0, c->stream>>>(c->dc, pc, c->a[A_B], c->a[A_PHI], c->a[A_R], c->st_pois,
                                                     c->partials);
    double *pb[2] = {c->a[A_P0], c->a[A_P1]};
    auto dir = [&](double *pold, double *pnew) {
        k_pois_dir_apply<<<c->dc.nlaunch, NT, 0, c->stream>>>(c->dc, pc, c->a[A_R], pold, pnew, c->a[A_Q], c->st_pois,
                                                              c->partials);
    };
    return cg_loop(c, c->st_pois, c->a[A_PHI], c->a[A_R], pb, c->pbuf_pois, c->a[A_Q], c->a[A_DINV], c->w.L.n,
                   c->last_pois_it, dir, info, 0);
}

ccns_status predict_dev(ccns_ctx *c, ccns_solve_info *info) {
    PredCoef pc = pred_coef(c);
    k_pred_rhs<<<c->df.nlaunch, NT, 0, c->stream>>>(c->df, pc, c->a[A_AX], c->a[A_AY], c->a[A_HBX], c->a[A_HBY],
                                                    c->a[A_DX], c->a[A_DY], c->a[A_UX], c->a[A_UY], c->a[A_P],
                                                    c->a[A_VDX], c->a[A_VDY], c->a[A_CONVX], c->a[A_CONVY],
                                                    c->a[A_RHSX], c->a[A_USX], c->prm.rho, c->prm.gx, c->prm.gy,
                                                    c->conv_valid);
    c->conv_valid = 1;
    k_pred_init<<<c->df.nlaunch, NT, 0, c->stream>>>(c->df, pc, c->a[A_RHSX], c->a[A_USX], c->a[A_PRX], c->st_pred,
                                                     c->partials);
    double *pb[2] = {c->a[A_PP0X], c->a[A_PP1X]};
    auto dir = [&](double *pold, double *pnew) {
        k_pred_dir_apply<<<c->df.nlaunch, NT, 0, c->stream>>>(c->df, pc, c->a[A_PRX], pold, pnew, c->a[A_PQX],
                                                              c->st_pred, c->partials);
    };
    return cg_loop(c, c->st_pred, c->a[A_USX], c->a[A_PRX], pb, c->pbuf_pred, c->a[A_PQX], c->a[A_HDX],
                   2 * c->w.L.n, c->last_pred_it, dir, info, 2);
}

ccns_status diag_dev(ccns_ctx *c, int update_p, ccns_step_info *info) {
    DiagCoef dc{c->a[A_AX], c->a[A_AY], c->a[A_HET], c->a[A_DINV], c->a[A_VUR], c->a[A_VVR],
                c->a[A_VU], c->a[A_VV], c->a[A_CX], c->a[A_CY], c->a[A_VINV]};
    const double pcoef = c->prm.tau * c->prm.mu / (2.0 * c->prm.rho);
    k_diag<<<c->dc.nlaunch, NT, 0, c->stream>>>(c->dc, dc, c->a[A_UX], c->a[A_UY], c->a[A_PHI], c->a[A_P], pcoef,
                                                update_p, c->prm.rho, c->diag, c->partials);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipMemcpyAsync(c->h_diag, c->diag, sizeof(DiagState), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (info) {
        info->div_max = c->h_diag->divmax > 0 ? c->h_diag->divmax : 0.0;
        info->div_rel = info->div_max / (c->prm.u_ref * std::min(c->g.hx, c->g.hy));
        info->ke = c->h_diag->ke;
        info->mass = c->h_diag->mass;
        info->mom_x = c->h_diag->momx;
        info->mom_y = c->h_diag->momy;
    }
    return CCNS_OK;
}

ccns_status correct_dev(ccns_ctx *c, int update_p, ccns_step_info *info) {
    PoisCoef pc = pois_coef(c);
    k_pois_rhs<<<c->dc.nlaunch, NT, 0, c->stream>>>(c->dc, pc, c->a[A_AX], c->a[A_AY], c->a[A_HET], c->a[A_USX],
                                                    c->a[A_USY], c->a[A_B], c->prm.rho / c->prm.tau, c->st_pois,
                                                    c->partials);
    ccns_solve_info si{};
    ccns_status s = pressure_solve_dev(c, &si);
    if (info) info->poisson = si;
    k_correct<<<c->dc.nlaunch, NT, 0, c->stream>>>(c->dc, c->a[A_GX], c->a[A_GY], c->a[A_USX], c->a[A_USY],
                                                   c->a[A_PHI], c->a[A_UX], c->a[A_UY], c->prm.tau / c->prm.rho);
    ccns_status s2 = diag_dev(c, update_p, info);
    if (s2 != CCNS_OK) return s2;
    return s;
}

}  // namespace

extern "C" {

size_t ccns_workspace_bytes(const ccns_grid *grid, const ccns_params *params) {
    (void)params;
    if (!grid || grid->nx < 2 || grid->ny < 2) return 0;
    return plan(grid->nx, grid->ny).total;
}

const char *ccns_last_error(const ccns_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

ccns_status ccns_ctx_create(const ccns_grid *grid, const ccns_params *params, const double *caps_host,
                            const double *dirichlet_host, void *dev_workspace, size_t ws_bytes, void *hip_stream,
                            ccns_ctx **out) {
    if (!out) return CCNS_EINVAL;
    *out = nullptr;
    if (!grid || !params || !caps_host || !dirichlet_host || !dev_workspace) return CCNS_EINVAL;
    if (params->precision != 0) return CCNS_EINVAL;
    ccns_ctx *c = new (std::nothrow) ccns_ctx();
    if (!c) return CCNS_ENOMEM;
    c->g = *grid;
    c->prm = *params;
    c->w = plan(grid->nx, grid->ny);
    if (ws_bytes < c->w.total) {
        delete c;
        return CCNS_ENOMEM;
    }
    if (((uintptr_t)dev_workspace) % 256 != 0) {
        delete c;
        return CCNS_EINVAL;
    }
    c->stream = (hipStream_t)hip_stream;
    c->base = (char *)dev_workspace;
    for (int k = 0; k < A_COUNT; ++k) c->a[k] = (double *)(c->base + (size_t)k * c->w.arr_bytes);
    c->partials = (double *)(c->base + c->w.part_off);
    c->st_pred = (CgState *)(c->base + c->w.state_off);
    c->st_pois = c->st_pred + 1;
    c->diag = (DiagState *)(c->st_pois + 1);
    c->dc = make_dims(c->w.L, 1);
    c->df = make_dims(c->w.L, 2);
    c->conv_valid = 0;
    c->last_pois_it = c->last_pred_it = 16;
    c->pbuf_pred = c->pbuf_pois = 0;
    c->timing = 0;
    c->evused = 0;
    for (int k = 0; k < 4; ++k) { c->t_ms[k] = 0.0; c->t_count[k] = 0; }

    HostCoef hc;
    std::string err;
    ccns_status s = prepare_coefficients(*grid, *params, caps_host, dirichlet_host, hc, err);
    if (s != CCNS_OK) {
        delete c;
        return s;
    }
    c->n_active = hc.n_active;
    if (hipHostMalloc((void **)&c->h_st, sizeof(CgState)) != hipSuccess ||
        hipHostMalloc((void **)&c->h_diag, sizeof(DiagState)) != hipSuccess) {
        delete c;
        return CCNS_EDEVICE;
    }
    // zero the whole workspace, then upload the coefficient fields
    if (hipMemsetAsync(c->base, 0, c->w.total, c->stream) != hipSuccess) {
        ccns_ctx_destroy(c);
        return CCNS_EDEVICE;
    }
    const std::vector<double> *src[] = {&hc.cx, &hc.cy, &hc.dinv, &hc.gx, &hc.gy, &hc.ax, &hc.ay, &hc.het,
                                        &hc.hbx, &hc.hby, &hc.dx, &hc.dy, &hc.vu, &hc.vv, &hc.bxx, &hc.bxy,
                                        &hc.byy, &hc.byx, &hc.wxx, &hc.wyy, &hc.nxx, &hc.nxy, &hc.nyx, &hc.nyy,
                                        &hc.hdx, &hc.hdy, &hc.vinv, &hc.vur, &hc.vvr, &hc.vdx, &hc.vdy};
    for (int k = 0; k <= A_VDY; ++k) {
        if ((s = to_dev(c, c->a[k], src[k]->data(), hipMemcpyHostToDevice)) != CCNS_OK) {
            ccns_ctx_destroy(c);
            return s;
        }
    }
    // state: U = D everywhere (the caller sets the initial field), P = Phi = 0
    to_dev(c, c->a[A_UX], hc.dx.data(), hipMemcpyHostToDevice);
    to_dev(c, c->a[A_UY], hc.dy.data(), hipMemcpyHostToDevice);
    set_cg(c, c->st_pred, params->pred_tol, params->pred_maxit, 0, hc.n_uact + hc.n_vact);
    set_cg(c, c->st_pois, params->pcg_tol, params->pcg_maxit, 1, hc.n_active);
    if (hipStreamSynchronize(c->stream) != hipSuccess) {
        ccns_ctx_destroy(c);
        return CCNS_EDEVICE;
    }
    *out = c;
    return CCNS_OK;
}

void ccns_ctx_destroy(ccns_ctx *ctx) {
    if (!ctx) return;
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->h_st) (void)hipHostFree(ctx->h_st);
    if (ctx->h_diag) (void)hipHostFree(ctx->h_diag);
    for (hipEvent_t e : ctx->evpool) (void)hipEventDestroy(e);
    delete ctx;
}

static const int kFieldArr[CCNS_NFIELDS] = {A_UX, A_UY, A_P, A_PHI, A_CONVX, A_CONVY, A_USX, A_USY, A_B};

ccns_status ccns_field_set(ccns_ctx *c, int field, const double *src, int is_device) {
    if (!c || !src || field < 0 || field >= CCNS_NFIELDS) return fail(c, CCNS_EINVAL, "bad field");
    ccns_status s = to_dev(c, c->a[kFieldArr[field]], src, is_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice);
    if (s != CCNS_OK) return s;
    if (field == CCNS_F_CONVX || field == CCNS_F_CONVY) c->conv_valid = 1;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return CCNS_OK;
}

ccns_status ccns_field_get(ccns_ctx *c, int field, double *dst, int is_device) {
    if (!c || !dst || field < 0 || field >= CCNS_NFIELDS) return fail(c, CCNS_EINVAL, "bad field");
    ccns_status s = from_dev(c, dst, c->a[kFieldArr[field]], is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost);
    if (s != CCNS_OK) return s;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return CCNS_OK;
}

ccns_status ccns_apply(ccns_ctx *c, int op, const double *const *in, double *const *out) {
    if (!c || !in || !out) return fail(c, CCNS_EINVAL, "null argument");
    ccns_status s;
    double *t0 = c->a[A_T0], *t1 = c->a[A_T1], *t2 = c->a[A_T2], *t3 = c->a[A_T3];
    const hipMemcpyKind D2D = hipMemcpyDeviceToDevice;
    switch (op) {
    case CCNS_OP_CONT:
        if ((s = to_dev(c, t0, in[0], D2D)) || (s = to_dev(c, t1, in[1], D2D))) return s;
        k_op_cont<<<c->dc.nlaunch, NT, 0, c->stream>>>(c->dc, c->a[A_AX], c->a[A_AY], c->a[A_HET], t0, t1, t2);
        if ((s = from_dev(c, out[0], t2, D2D))) return s;
        break;
    case CCNS_OP_PRES:
        if ((s = to_dev(c, t0, in[0], D2D))) return s;
        k_op_pres<<<c->dc.nlaunch, NT, 0, c->stream>>>(c->dc, c->a[A_AX], c->a[A_AY], t0, t1, t2);
        if ((s = from_dev(c, out[0], t1, D2D)) || (s = from_dev(c, out[1], t2, D2D))) return s;
        break;
    case CCNS_OP_VISC:
    case CCNS_OP_H:
        if ((s = to_dev(c, t0, in[0], D2D)) || (s = to_dev(c, t1, in[1], D2D))) return s;
        k_op_visc<<<c->dc.nlaunch, NT, 0, c->stream>>>(c->dc, pred_coef(c), c->a[A_VDX], c->a[A_VDY], t0, t1, t2, t3,
                                                       op == CCNS_OP_VISC ? 0 : 1);
        if ((s = from_dev(c, out[0], t2, D2D)) || (s = from_dev(c, out[1], t3, D2D))) return s;
        break;
    case CCNS_OP_CONV:
        if ((s = to_dev(c, t0, in[0], D2D)) || (s = to_dev(c, t1, in[1], D2D))) return s;
        k_op_conv<<<c->dc.nlaunch, NT, 0, c->stream>>>(c->dc, c->a[A_AX], c->a[A_AY], c->a[A_HBX], c->a[A_HBY],
                                                       c->a[A_DX], c->a[A_DY], t0, t1, t2, t3);
        if ((s = from_dev(c, out[0], t2, D2D)) || (s = from_dev(c, out[1], t3, D2D))) return s;
        break;
    case CCNS_OP_LAP:
        if ((s = to_dev(c, t0, in[0], D2D))) return s;
        k_op_lap<<<c->dc.nlaunch, NT, 0, c->stream>>>(c->dc, pois_coef(c), t0, t1);
        if ((s = from_dev(c, out[0], t1, D2D))) return s;
        break;
    case CCNS_OP_KINETIC:
        if ((s = to_dev(c, t0, in[0], D2D)) || (s = to_dev(c, t1, in[1], D2D))) return s;
        k_op_kin<<<c->dc.nlaunch, NT, 0, c->stream>>>(c->dc, c->a[A_VUR], c->a[A_VVR], t0, t1, t2);
        if ((s = from_dev(c, out[0], t2, D2D))) return s;
        break;
    default:
        return fail(c, CCNS_EINVAL, "unknown operator");
    }
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return CCNS_OK;
}

ccns_status ccns_pressure_solve(ccns_ctx *c, const double *b, double *phi, ccns_solve_info *info) {
    if (!c || !b) return fail(c, CCNS_EINVAL, "null argument");
    ccns_status s = to_dev(c, c->a[A_B], b, hipMemcpyDeviceToDevice);
    if (s != CCNS_OK) return s;
    k_pois_mean<<<c->dc.nlaunch, NT, 0, c->stream>>>(c->dc, pois_coef(c), c->a[A_B], c->st_pois, c->partials);
    s = pressure_solve_dev(c, info);
    if (phi) {
        ccns_status s2 = from_dev(c, phi, c->a[A_PHI], hipMemcpyDeviceToDevice);
        if (s2 != CCNS_OK) return s2;
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    return s;
}

ccns_status ccns_project(ccns_ctx *c, ccns_step_info *info) {
    if (!c) return CCNS_EINVAL;
    // U* := U, then the correction of one step without the pressure update
    HIPCHK(c, hipMemcpyAsync(c->a[A_USX], c->a[A_UX], c->w.L.n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->a[A_USY], c->a[A_UY], c->w.L.n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    ccns_step_info si{};
    ccns_status s = correct_dev(c, 0, &si);
    if (info) *info = si;
    return s;
}

ccns_status ccns_predict(ccns_ctx *c, ccns_solve_info *info) {
    if (!c) return CCNS_EINVAL;
    return predict_dev(c, info);
}

ccns_status ccns_correct(ccns_ctx *c, ccns_step_info *info) {
    if (!c) return CCNS_EINVAL;
    return correct_dev(c, 1, info);
}

ccns_status ccns_step(ccns_ctx *c, int nsteps, ccns_step_info *info) {
    if (!c || nsteps < 0) return fail(c, CCNS_EINVAL, "bad arguments");
    ccns_step_info si{};
    ccns_status worst = CCNS_OK;
    for (int n = 0; n < nsteps; ++n) {
        ccns_status s1 = predict_dev(c, &si.pred);
        if (s1 == CCNS_EDEVICE) return s1;
        ccns_status s2 = correct_dev(c, 1, &si);
        if (s2 == CCNS_EDEVICE) return s2;
        if (s1 != CCNS_OK) worst = s1;
        if (s2 != CCNS_OK) worst = s2;
    }
    if (info) *info = si;
    return worst;
}

ccns_status ccns_timing(ccns_ctx *c, int enable, double *ms, long *count) {
    if (!c) return CCNS_EINVAL;
    if (ms && count)
        for (int k = 0; k < 4; ++k) { ms[k] = c->t_ms[k]; count[k] = c->t_count[k]; }
    if (enable >= 0) {
        c->timing = enable;
        for (int k = 0; k < 4; ++k) { c->t_ms[k] = 0.0; c->t_count[k] = 0; }
    }
    return CCNS_OK;
}

ccns_status ccns_diagnostics(ccns_ctx *c, ccns_step_info *info) {
    if (!c) return CCNS_EINVAL;
    return diag_dev(c, 0, info);
}

}  // extern "C"
