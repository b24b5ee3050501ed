// The projection step in three dimensions (Sec. 4.6 with the operators of
// Sec. 4.1 on 7-point stencils; the paper extends its two-dimensional
// statement by adding an index, Sec. 2.1) on gfx950.
//
// Device layout: every field is (nz+2)(ny+2) rows of `pitch` doubles (pitch
// = nx+2 rounded up to 16), element (i, j, k) at (k (ny+2) + j) pitch + i,
// the same index meaning as the dense host layout.
//
// The Poisson solve is preconditioned CG (Jacobi, or a geometric multigrid
// V-cycle with its fields in FP64 or FP32) with two kernels per iteration
// besides the preconditioner's, all HBM-bound:
//  * k3_stencil<DIR>: p = z + beta p_old on a tile of 64 x 4 columns and its
//    one-cell halo, marching up a slab of 32 cells in z with the planes
//    below and above each cell in registers and the current plane in LDS;
//    q = (-L) p = sum over the six faces of c_f (p_c - p_nb); partial p.q;
//  * k3_update: x += alpha p, r -= alpha q, and with the Jacobi preconditioner
//    z = r / diag and the partials r.z, r.r (the multigrid cycle forms z and
//    the partials after it).
// Each launch reduces the previous launch's per-group partials itself, in a
// fixed order, so alpha, beta and the stopping test are the same in every
// group and the solve runs without host round trips inside a chunk of
// iterations; the host looks at the solver state once per chunk.  Every
// reduction has a fixed order, so results are reproducible bit for bit.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <climits>
#include <cstdint>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "ccns3d.h"
#include "ccns3d_internal.h"
#include "ccns_internal.h"
#include "ccns_kern.h"

namespace ccns {
namespace {

constexpr int T3X = 64;     // tile columns in x (one wavefront)
constexpr int T3Y = 4;      // tile rows in y (the four wavefronts of a group)
constexpr int T3Z = 32;     // cells per column of a tile, marched in z
constexpr int NB3 = 4096;   // at most this many work-groups per kernel
constexpr int HALO3 = 2 * (T3X + 2) + 2 * T3Y;  // halo cells of one plane of a tile

// Solver state in device memory.  stop_it: the iteration whose direction
// launch stopped the solve (INT_MAX while it runs); rz[2]: r.z of the last
// two iterations (alternating slots, written by group 0 of the direction
// launch).
struct Cg3 {
    double bb, tol2, rr_final;
    double rz[2];
    int stop_it, status, it_final, maxit;
};

struct Dims3 {
    int nx, ny, nz, pitch;
    size_t plane, n;       // elements per z-plane and per field
    int gxt, gyt, gzt;     // tiles per direction
    int ntile, tpb, nblk;  // tiles, tiles per group, groups of the stencil kernel
    int nflat;             // groups of the element-wise kernels
};

enum { S_APPLY = 0, S_RESID = 1, S_DIR = 2 };

// The value the stencil acts on at element e: the input (apply), the
// iterate x (residual) or the new direction z + beta p_old.
template <int MODE>
__device__ inline double stencil_value(size_t e, const double *__restrict__ a, const double *__restrict__ b2, double beta,
                                       bool first) {
    if (MODE == S_DIR) return first ? a[e] : fma(beta, b2[e], a[e]);
    return a[e];
}

// (-L) v on tiles of 64 x 4 columns marched through T3Z cells in z.
//  S_APPLY: out = (-L) in.
//  S_RESID: b' = b - mean(b) on the unknowns (mean from the right-hand
//    side kernel's partials), r = b' - (-L) x, z = r / diag, b' stored;
//    partials (r.z, r.r, b'.b').
//  S_DIR: iteration `it` of the CG (see the file comment); partial p.q.
template <int MODE>
__global__ __launch_bounds__(NT) void k3_stencil(Dims3 d, const double *__restrict__ cx, const double *__restrict__ cy,
                                                 const double *__restrict__ cz, const double *__restrict__ dinv,
                                                 const double *__restrict__ va, const double *__restrict__ vb,
                                                 double *__restrict__ out1, double *__restrict__ out2,
                                                 double *__restrict__ bvec, Cg3 *st, int it, const double *pin, int nin,
                                                 int n_active, double *part) {
    double beta = 0.0, mean = 0.0;
    bool first = true;
    if (MODE == S_DIR) {
        if (st->stop_it < it) return;
        double rz, rr, bb;
        if (it == 0) {
            double t[3];
            get_totals<3>(pin, nin, t);
            rz = t[0];
            rr = t[1];
            bb = t[2];
        } else {
            double t[2];
            get_totals<2>(pin, nin, t);
            rz = t[0];
            rr = t[1];
            bb = st->bb;
            first = false;
        }
        // a NaN never counts as converged; a residual that is not finite, or
        // r.z not positive, ends the solve as a breakdown
        const bool conv = rr <= st->tol2 * bb;
        const double rz_old = it == 0 ? 1.0 : st->rz[(it - 1) & 1];
        const bool breakdown = !conv && !(rz > 0.0 && rz < INFINITY && rr < INFINITY);
        beta = it == 0 ? 0.0 : rz / rz_old;
        const bool stop = conv || breakdown || it >= st->maxit;
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            if (it == 0) st->bb = bb;
            st->rz[it & 1] = rz;
            if (stop) {
                st->status = conv ? CCNS_OK : (breakdown ? CCNS_EBREAKDOWN : CCNS_ENOTCONV);
                st->it_final = it;
                st->rr_final = rr;
                st->stop_it = it;
            }
        }
        if (stop) return;
    } else if (MODE == S_RESID) {
        double t[1];
        get_totals<1>(pin, nin, t);
        mean = n_active > 0 ? t[0] / n_active : 0.0;
    }
    // two plane buffers, alternating: one barrier per plane suffices (a
    // buffer is written again only after the barrier of the next plane,
    // which every reader of its last contents has passed)
    __shared__ double s2[2][T3Y + 2][T3X + 2];
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int X = d.pitch;
    const size_t PL = d.plane;
    double acc[3] = {0.0, 0.0, 0.0};
    const int L = logical_group(d.nblk);
    const int t0 = L * d.tpb, t1 = min(t0 + d.tpb, d.ntile);
    int ph = 0;  // the plane buffer: alternates with every plane of every tile
    for (int t = t0; t < t1; ++t) {
        const int txi = t % d.gxt, rest = t / d.gxt, tyj = rest % d.gyt, tz = rest / d.gyt;
        const int i0 = 1 + T3X * txi, j0 = 1 + T3Y * tyj, k0 = 1 + T3Z * tz, k1 = min(k0 + T3Z, d.nz + 1);
        const int i = i0 + tx, j = j0 + ty;
        const bool own = i <= d.nx && j <= d.ny;
        // this thread's halo cell of each plane (threads 0 .. HALO3-1)
        int hx = 0, hy = 0;
        bool hin = false;
        if ((int)threadIdx.x < HALO3) {
            const int e = threadIdx.x;
            if (e < 2 * (T3X + 2)) {
                hy = e < T3X + 2 ? 0 : T3Y + 1;
                hx = e < T3X + 2 ? e : e - (T3X + 2);
            } else {
                const int f = e - 2 * (T3X + 2);
                hy = 1 + (f >> 1);
                hx = (f & 1) ? T3X + 1 : 0;
            }
            // beyond the ghost layer the slot holds 0 (no own cell reads it)
            hin = i0 - 1 + hx <= d.nx + 1 && j0 - 1 + hy <= d.ny + 1;
        }
        const size_t hoff = (size_t)(j0 - 1 + hy) * X + (i0 - 1 + hx);
        const size_t col = (size_t)j * X + i;
        double prev = 0.0, cur = 0.0, czb = 0.0;
        if (own) {
            prev = stencil_value<MODE>((size_t)(k0 - 1) * PL + col, va, vb, beta, first);
            cur = stencil_value<MODE>((size_t)k0 * PL + col, va, vb, beta, first);
            czb = cz[(size_t)(k0 - 1) * PL + col];
        }
        for (int k = k0; k < k1; ++k) {
            double(&s)[T3Y + 2][T3X + 2] = s2[ph];
            ph ^= 1;
            const size_t e = (size_t)k * PL + col;
            double nxt = 0.0, ce = 0.0, cw = 0.0, cn = 0.0, cs = 0.0, ct = 0.0, dv = 0.0, bv = 0.0, hv = 0.0;
            if (own) {
                nxt = stencil_value<MODE>(e + PL, va, vb, beta, first);
                ce = cx[e];
                cw = cx[e - 1];
                cn = cy[e];
                cs = cy[e - X];
                ct = cz[e];
                if (MODE == S_RESID) {
                    dv = dinv[e];
                    bv = bvec[e];
                }
            }
            if ((int)threadIdx.x < HALO3 && hin) hv = stencil_value<MODE>((size_t)k * PL + hoff, va, vb, beta, first);
            s[ty + 1][tx + 1] = cur;
            if ((int)threadIdx.x < HALO3) s[hy][hx] = hin ? hv : 0.0;
            __syncthreads();
            if (own) {
                const double av = ce * (cur - s[ty + 1][tx + 2]) + cw * (cur - s[ty + 1][tx]) +
                                  cn * (cur - s[ty + 2][tx + 1]) + cs * (cur - s[ty][tx + 1]) + ct * (cur - nxt) +
                                  czb * (cur - prev);
                if (MODE == S_APPLY) {
                    out1[e] = av;
                } else if (MODE == S_RESID) {
                    const double bb = dv > 0.0 ? bv - mean : 0.0;
                    const double r = dv > 0.0 ? bb - av : 0.0;
                    const double z = dv * r;
                    out1[e] = r;
                    out2[e] = z;
                    bvec[e] = bb;
                    acc[0] += r * z;
                    acc[1] += r * r;
                    acc[2] += bb * bb;
                } else {
                    out1[e] = cur;
                    out2[e] = av;
                    acc[0] += cur * av;
                }
            }
            czb = ct;
            prev = cur;
            cur = nxt;
        }
    }
    if (MODE == S_RESID) {
        double v[3] = {acc[0], acc[1], acc[2]};
        put_partials<3>(v, part, gridDim.x);
    } else if (MODE == S_DIR) {
        double v[1] = {acc[0]};
        put_partials<1>(v, part, gridDim.x);
    }
}

// x += alpha p, r -= alpha q, z = r / diag over every element (the masks
// keep the entries off the unknowns at zero); partials (r.z, r.r).
template <bool JAC>
__global__ __launch_bounds__(NT) void k3_update(Dims3 d, const double *__restrict__ dinv, const double *__restrict__ p,
                                                const double *__restrict__ q, double *__restrict__ x,
                                                double *__restrict__ r, double *__restrict__ z, Cg3 *st, int it,
                                                const double *pin, int nin, double *part) {
    if (st->stop_it <= it) return;
    double t[1];
    get_totals<1>(pin, nin, t);
    const double pq = t[0];
    if (!(pq > 0.0 && pq < INFINITY)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st->status = CCNS_EBREAKDOWN;
            st->it_final = it;
            st->stop_it = it;
        }
        return;
    }
    const double alpha = st->rz[it & 1] / pq;
    double v[2] = {0.0, 0.0};
    const size_t stride = (size_t)gridDim.x * NT;
    for (size_t e = (size_t)blockIdx.x * NT + threadIdx.x; e < d.n; e += stride) {
        const double pe = p[e], qe = q[e];
        const double xe = x[e], re = r[e];
        x[e] = fma(alpha, pe, xe);
        const double rn = fma(-alpha, qe, re);
        r[e] = rn;
        if constexpr (JAC) {
            const double zn = dinv[e] * rn;
            z[e] = zn;
            v[0] += rn * zn;
            v[1] += rn * rn;
        }
    }
    if constexpr (JAC) put_partials<2>(v, part, gridDim.x);
}

// b = -(rho/tau) cont(U*, 0) on the pressure unknowns (eq:divergence with
// D = 0; A is zero off the velocity unknowns, so U* is masked there);
// partial sum of b.
__global__ __launch_bounds__(NT) void k3_rhs(Dims3 d, const double *__restrict__ ax, const double *__restrict__ ay,
                                             const double *__restrict__ az, const double *__restrict__ ux,
                                             const double *__restrict__ uy, const double *__restrict__ uz,
                                             const double *__restrict__ dinv, double scale, double *__restrict__ b,
                                             double *part) {
    double v[1] = {0.0};
    const size_t stride = (size_t)gridDim.x * NT, X = d.pitch, PL = d.plane;
    for (size_t e = (size_t)blockIdx.x * NT + threadIdx.x; e < d.n; e += stride) {
        double be = 0.0;
        if (dinv[e] > 0.0) {
            const double div = (ax[e] * ux[e] - ax[e - 1] * ux[e - 1]) + (ay[e] * uy[e] - ay[e - X] * uy[e - X]) +
                               (az[e] * uz[e] - az[e - PL] * uz[e - PL]);
            be = -scale * div;
        }
        b[e] = be;
        v[0] += be;
    }
    put_partials<1>(v, part, gridDim.x);
}

// Partial sums of x over the pressure unknowns.
__global__ __launch_bounds__(NT) void k3_sum(Dims3 d, const double *__restrict__ dinv, const double *__restrict__ x,
                                             double *part) {
    double v[1] = {0.0};
    const size_t stride = (size_t)gridDim.x * NT;
    for (size_t e = (size_t)blockIdx.x * NT + threadIdx.x; e < d.n; e += stride)
        if (dinv[e] > 0.0) v[0] += x[e];
    put_partials<1>(v, part, gridDim.x);
}

// eq:pm_projection: U = U* - (tau/rho) (A/M) (Phi_nb - Phi_c) on the faces
// with c > 0 (g = A/M there), U* on the other unknowns (a = A > 0), 0 on
// every other face; the three faces on the high sides of each element.
__global__ __launch_bounds__(NT) void k3_correct(Dims3 d, const double *__restrict__ gx, const double *__restrict__ gy,
                                                 const double *__restrict__ gz, const double *__restrict__ ax,
                                                 const double *__restrict__ ay, const double *__restrict__ az,
                                                 const double *__restrict__ x, double tr, double *__restrict__ ux,
                                                 double *__restrict__ uy, double *__restrict__ uz) {
    const size_t stride = (size_t)gridDim.x * NT, X = d.pitch, PL = d.plane;
    // g > 0 only on faces between two real cells, so the neighbour reads stay
    // in the field
    for (size_t e = (size_t)blockIdx.x * NT + threadIdx.x; e < d.n; e += stride) {
        const double xc = x[e];
        const double g0 = gx[e], g1 = gy[e], g2 = gz[e];
        const double u0 = ux[e], u1 = uy[e], u2 = uz[e];
        const double a0 = ax[e], a1 = ay[e], a2 = az[e];
        ux[e] = g0 > 0.0 ? u0 - tr * g0 * (x[e + 1] - xc) : (a0 > 0.0 ? u0 : 0.0);
        uy[e] = g1 > 0.0 ? u1 - tr * g1 * (x[e + X] - xc) : (a1 > 0.0 ? u1 : 0.0);
        uz[e] = g2 > 0.0 ? u2 - tr * g2 * (x[e + PL] - xc) : (a2 > 0.0 ? u2 : 0.0);
    }
}

// x -= mean(x) on the pressure unknowns (the zero-mean solution), and the
// divergence figures of the corrected velocity: partial maxima of
// |cont(U, 0)| over the unknowns and of the face fluxes |A U|.
__global__ __launch_bounds__(NT) void k3_div_shift(Dims3 d, const double *__restrict__ ax, const double *__restrict__ ay,
                                                   const double *__restrict__ az, const double *__restrict__ ux,
                                                   const double *__restrict__ uy, const double *__restrict__ uz,
                                                   const double *__restrict__ dinv, double *__restrict__ x,
                                                   const double *pin, int nin, int n_active, double *part) {
    double t[1];
    get_totals<1>(pin, nin, t);
    const double mean = n_active > 0 ? t[0] / n_active : 0.0;
    double v[2] = {0.0, 0.0};
    const size_t stride = (size_t)gridDim.x * NT, X = d.pitch, PL = d.plane;
    for (size_t e = (size_t)blockIdx.x * NT + threadIdx.x; e < d.n; e += stride) {
        if (dinv[e] > 0.0) {
            const double f0 = ax[e] * ux[e], f1 = ay[e] * uy[e], f2 = az[e] * uz[e];
            const double div = (f0 - ax[e - 1] * ux[e - 1]) + (f1 - ay[e - X] * uy[e - X]) + (f2 - az[e - PL] * uz[e - PL]);
            v[0] = fmax(v[0], fabs(div));
            x[e] = x[e] - mean;
        }
        if (e + PL < d.n)
            v[1] = fmax(v[1], fmax(fabs(ax[e] * ux[e]), fmax(fabs(ay[e] * uy[e]), fabs(az[e] * uz[e]))));
    }
    put_partials<0, 2>(v, part, gridDim.x);
}

// ---------------------------------------------------------------------------
// Geometric multigrid V-cycle on the Poisson weights, the preconditioner of
// the 3-D CG (the two-dimensional cycle's design with a third index): 2x2x2
// agglomeration, a coarse face weight of half the sum of the four fine faces
// it covers, weighted Jacobi (omega = 0.8) two sweeps down and two up,
// piecewise-constant interpolation and its transpose as restriction, and the
// dense pseudo-inverse on the coarsest grid (at most MG3_MAXC cells).  The
// same sweeps down and up make the cycle a symmetric operator, so the CG
// stays valid.  Each level takes four launches: the two down-sweeps in one
// (the first sweep from x = 0 is omega D^-1 b, formed where the second reads
// it), the restriction of the residual, the first up-sweep with the
// interpolated coarse correction added where it reads its input, and the
// second up-sweep.  The cycle's fields are stored in T (double, or float for
// the FP32 cycle inside the FP64 CG); its arithmetic is FP64 either way.
// ---------------------------------------------------------------------------

constexpr double MG3_W = 0.8;   // Jacobi weight of the sweeps
constexpr int MG3_MAXC = 256;   // cells of the coarsest grid at most

// One level: dense (nz+2)(ny+2) rows of `pitch` elements; b is the level's
// right-hand side, x and xt its two iterates (the cycle's correction ends in
// xt).  On the finest level the right-hand side is the CG's residual r (FP64,
// passed to its kernels apart) and the result goes to the CG's z.  Every
// level has fewer than 2^31 elements.
template <class T>
struct LevT {
    int nx, ny, nz, pitch;
    size_t plane, n;
    const T *cx, *cy, *cz, *dinv;
    T *b, *x, *xt;
};

// (i, j, k) of element e of a level
template <class T>
__device__ inline void ijk3(const LevT<T> &v, unsigned e, int &i, int &j, int &k) {
    const unsigned row = e / (unsigned)v.pitch;
    i = (int)(e - row * (unsigned)v.pitch);
    k = (int)(row / (unsigned)(v.ny + 2));
    j = (int)(row - (unsigned)k * (unsigned)(v.ny + 2));
}
template <class T>
__device__ inline bool interior3(const LevT<T> &v, int i, int j, int k) {
    return i >= 1 && i <= v.nx && j >= 1 && j <= v.ny && k >= 1 && k <= v.nz;
}
// the parent of fine cell (i, j, k) on coarse level c
template <class T>
__device__ inline size_t parent3(const LevT<T> &c, int i, int j, int k) {
    return (size_t)((k + 1) >> 1) * c.plane + (size_t)((j + 1) >> 1) * c.pitch + ((i + 1) >> 1);
}

// The value a coarse-level sweep acts on at element e (cell (i, j, k)):
//  FROM_B: the first sweep's result omega D^-1 b;
//  PRO:    u + the parent's coarse correction;
//  else:   u.
template <bool FROM_B, bool PRO, class T>
__device__ inline double sweep_in(const LevT<T> &v, const T *__restrict__ u, const LevT<T> &c,
                                  const T *__restrict__ xc, size_t e, int i, int j, int k) {
    if (FROM_B) return MG3_W * (double)v.dinv[e] * (double)v.b[e];
    if (PRO) return (double)u[e] + (double)xc[parent3(c, i, j, k)];
    return (double)u[e];
}

// Coarse levels: xout = y + omega D^-1 (b - (-L) y) on the unknowns, 0
// elsewhere, with y given by sweep_in.  Every load of an interior element
// is issued before the test of whether it is an unknown (its loads stay
// inside the ghost layer).
template <bool FROM_B, bool PRO, class T>
__global__ __launch_bounds__(NT) void k3_mg_sweep(LevT<T> v, const T *__restrict__ xin, T *__restrict__ xout,
                                                  LevT<T> c, const T *__restrict__ xc, const Cg3 *st, int it) {
    if (st->stop_it <= it) return;
    const size_t stride = (size_t)gridDim.x * NT, P = v.pitch, PL = v.plane;
    for (size_t e = (size_t)blockIdx.x * NT + threadIdx.x; e < v.n; e += stride) {
        int i, j, k;
        ijk3(v, (unsigned)e, i, j, k);
        double o = 0.0;
        if (interior3(v, i, j, k)) {
            const double be = v.b[e], dv = v.dinv[e];
            const double y = sweep_in<FROM_B, PRO>(v, xin, c, xc, e, i, j, k);
            const double ye = sweep_in<FROM_B, PRO>(v, xin, c, xc, e + 1, i + 1, j, k);
            const double yw = sweep_in<FROM_B, PRO>(v, xin, c, xc, e - 1, i - 1, j, k);
            const double yn = sweep_in<FROM_B, PRO>(v, xin, c, xc, e + P, i, j + 1, k);
            const double ys = sweep_in<FROM_B, PRO>(v, xin, c, xc, e - P, i, j - 1, k);
            const double yt = sweep_in<FROM_B, PRO>(v, xin, c, xc, e + PL, i, j, k + 1);
            const double yb = sweep_in<FROM_B, PRO>(v, xin, c, xc, e - PL, i, j, k - 1);
            const double ax = (double)v.cx[e] * (y - ye) + (double)v.cx[e - 1] * (y - yw) +
                              (double)v.cy[e] * (y - yn) + (double)v.cy[e - P] * (y - ys) +
                              (double)v.cz[e] * (y - yt) + (double)v.cz[e - PL] * (y - yb);
            o = dv > 0.0 ? y + MG3_W * dv * (be - ax) : 0.0;
        }
        xout[e] = (T)o;
    }
}

// coarse b = the sum over the (up to eight) children of the fine residual
// b - (-L) xf on the fine unknowns; 0 on the coarse ghost layer.  A child
// index beyond the fine grid is clamped to the grid (its load repeats its
// sibling's) and contributes nothing.
template <class T>
__global__ __launch_bounds__(NT) void k3_mg_restrict(LevT<T> f, const T *__restrict__ xf, LevT<T> c, const Cg3 *st,
                                                     int it) {
    if (st->stop_it <= it) return;
    const size_t stride = (size_t)gridDim.x * NT, P = f.pitch, PL = f.plane;
    for (size_t ec = (size_t)blockIdx.x * NT + threadIdx.x; ec < c.n; ec += stride) {
        int I, J, K;
        ijk3(c, (unsigned)ec, I, J, K);
        double s = 0.0;
        if (interior3(c, I, J, K)) {
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int i0 = 2 * I - 1 + (q & 1), j0 = 2 * J - 1 + ((q >> 1) & 1), k0 = 2 * K - 1 + (q >> 2);
                const bool in = i0 <= f.nx && j0 <= f.ny && k0 <= f.nz;
                const int i = min(i0, f.nx), j = min(j0, f.ny), k = min(k0, f.nz);
                const size_t e = (size_t)k * PL + (size_t)j * P + i;
                const double y = xf[e];
                const double ax = (double)f.cx[e] * (y - (double)xf[e + 1]) +
                                  (double)f.cx[e - 1] * (y - (double)xf[e - 1]) +
                                  (double)f.cy[e] * (y - (double)xf[e + P]) +
                                  (double)f.cy[e - P] * (y - (double)xf[e - P]) +
                                  (double)f.cz[e] * (y - (double)xf[e + PL]) +
                                  (double)f.cz[e - PL] * (y - (double)xf[e - PL]);
                const double r = (double)f.b[e] - ax;
                s += (in && f.dinv[e] > (T)0) ? r : 0.0;
            }
        }
        c.b[ec] = (T)s;
    }
}

// The finest level's cycle kernels on the tiles of k3_stencil (64 x 4
// columns marched up a slab of 32 cells in z, the current plane and its halo
// in LDS), which read each value about once where element-wise forms re-read
// their plane and row neighbours from beyond L2:
//  T_PRE:   both down-sweeps, xt from y = omega D^-1 r;
//  T_RES:   the residual r - (-L) xt on the unknowns (for the restriction);
//  T_POST1: the first up-sweep from y = xt + the parent's correction;
//  T_POST2: the second up-sweep from y = x, written (in TO) to the CG's z;
//           NS = 2: partials (r.z, r.r); NS = 3: also b'.b' of `bp`.
// v carries the finest level's coefficients (in T); r is the CG's residual.
enum { T_PRE = 0, T_RES = 1, T_POST1 = 2, T_POST2 = 3 };
template <int MODE, class T>
__device__ inline double tile_in(const LevT<T> &v, const double *__restrict__ r, const T *__restrict__ u,
                                 const LevT<T> &c, const T *__restrict__ xc, size_t e, int i, int j, int k) {
    if (MODE == T_PRE) return MG3_W * (double)v.dinv[e] * r[e];
    if (MODE == T_POST1) return (double)u[e] + (double)xc[parent3(c, i, j, k)];
    return (double)u[e];
}
template <int MODE, int NS, class T, class TO>
__global__ __launch_bounds__(NT) void k3_mg_tile(Dims3 d, LevT<T> v, const double *__restrict__ r,
                                                 const T *__restrict__ u, LevT<T> c, const T *__restrict__ xc,
                                                 TO *__restrict__ out, const double *__restrict__ bp, double *part,
                                                 const Cg3 *st, int it) {
    if (st->stop_it <= it) return;
    __shared__ double s2[2][T3Y + 2][T3X + 2];
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int X = d.pitch;
    const size_t PL = d.plane;
    double acc[NS > 0 ? NS : 1] = {};
    const int L = logical_group(d.nblk);
    const int t0 = L * d.tpb, t1 = min(t0 + d.tpb, d.ntile);
    int ph = 0;
    for (int t = t0; t < t1; ++t) {
        const int txi = t % d.gxt, rest = t / d.gxt, tyj = rest % d.gyt, tz = rest / d.gyt;
        const int i0 = 1 + T3X * txi, j0 = 1 + T3Y * tyj, k0 = 1 + T3Z * tz, k1 = min(k0 + T3Z, d.nz + 1);
        const int i = i0 + tx, j = j0 + ty;
        const bool own = i <= d.nx && j <= d.ny;
        int hx = 0, hy = 0;
        bool hin = false;
        const bool hthr = (int)threadIdx.x < HALO3;
        if (hthr) {
            const int e = threadIdx.x;
            if (e < 2 * (T3X + 2)) {
                hy = e < T3X + 2 ? 0 : T3Y + 1;
                hx = e < T3X + 2 ? e : e - (T3X + 2);
            } else {
                const int f = e - 2 * (T3X + 2);
                hy = 1 + (f >> 1);
                hx = (f & 1) ? T3X + 1 : 0;
            }
            hin = i0 - 1 + hx <= d.nx + 1 && j0 - 1 + hy <= d.ny + 1;
        }
        const int hi = i0 - 1 + hx, hj = j0 - 1 + hy;
        const size_t hoff = (size_t)hj * X + hi;
        const size_t col = (size_t)j * X + i;
        double prev = 0.0, cur = 0.0, czb = 0.0;
        if (own) {
            prev = tile_in<MODE>(v, r, u, c, xc, (size_t)(k0 - 1) * PL + col, i, j, k0 - 1);
            cur = tile_in<MODE>(v, r, u, c, xc, (size_t)k0 * PL + col, i, j, k0);
            czb = v.cz[(size_t)(k0 - 1) * PL + col];
        }
        for (int k = k0; k < k1; ++k) {
            double(&s)[T3Y + 2][T3X + 2] = s2[ph];
            ph ^= 1;
            const size_t e = (size_t)k * PL + col;
            double nxt = 0.0, ce = 0.0, cw = 0.0, cn = 0.0, cs = 0.0, ct = 0.0, dv = 0.0, bv = 0.0, hv = 0.0;
            if (own) {
                nxt = tile_in<MODE>(v, r, u, c, xc, e + PL, i, j, k + 1);
                ce = v.cx[e];
                cw = v.cx[e - 1];
                cn = v.cy[e];
                cs = v.cy[e - X];
                ct = v.cz[e];
                dv = v.dinv[e];
                bv = r[e];
            }
            if (hthr && hin) hv = tile_in<MODE>(v, r, u, c, xc, (size_t)k * PL + hoff, hi, hj, k);
            s[ty + 1][tx + 1] = cur;
            if (hthr) s[hy][hx] = hin ? hv : 0.0;
            __syncthreads();
            if (own) {
                const double av = ce * (cur - s[ty + 1][tx + 2]) + cw * (cur - s[ty + 1][tx]) +
                                  cn * (cur - s[ty + 2][tx + 1]) + cs * (cur - s[ty][tx + 1]) + ct * (cur - nxt) +
                                  czb * (cur - prev);
                double o;
                if (MODE == T_RES)
                    o = dv > 0.0 ? bv - av : 0.0;
                else
                    o = dv > 0.0 ? cur + MG3_W * dv * (bv - av) : 0.0;
                out[e] = (TO)o;
                if constexpr (NS >= 2) {
                    acc[0] += bv * o;
                    acc[1] += bv * bv;
                }
                if constexpr (NS >= 3) {
                    const double q = bp[e];
                    acc[2] += q * q;
                }
            }
            czb = ct;
            prev = cur;
            cur = nxt;
        }
    }
    if constexpr (NS > 0) put_partials<NS>(acc, part, gridDim.x);
}

// coarse b = the sum of the fine residual rf over the (up to eight)
// children; 0 on the coarse ghost layer.  rf is 0 off the fine unknowns; a
// child index beyond the fine grid is clamped and contributes nothing.
template <class T>
__global__ __launch_bounds__(NT) void k3_mg_sum8(LevT<T> f, const T *__restrict__ rf, LevT<T> c, const Cg3 *st,
                                                 int it) {
    if (st->stop_it <= it) return;
    const size_t stride = (size_t)gridDim.x * NT;
    for (size_t ec = (size_t)blockIdx.x * NT + threadIdx.x; ec < c.n; ec += stride) {
        int I, J, K;
        ijk3(c, (unsigned)ec, I, J, K);
        double s = 0.0;
        if (interior3(c, I, J, K)) {
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int i0 = 2 * I - 1 + (q & 1), j0 = 2 * J - 1 + ((q >> 1) & 1), k0 = 2 * K - 1 + (q >> 2);
                const bool in = i0 <= f.nx && j0 <= f.ny && k0 <= f.nz;
                const size_t e = (size_t)min(k0, f.nz) * f.plane + (size_t)min(j0, f.ny) * f.pitch + min(i0, f.nx);
                const double rv = rf[e];
                s += in ? rv : 0.0;
            }
        }
        c.b[ec] = (T)s;
    }
}

// coarsest grid: x = A^+ b on its n unknowns (element indices idx), one
// work-group; n <= MG3_MAXC
template <class T>
__global__ __launch_bounds__(NT) void k3_mg_coarsest(int n, const int *__restrict__ idx, const double *__restrict__ pinv,
                                                     const T *__restrict__ b, T *__restrict__ x, const Cg3 *st,
                                                     int it) {
    if (st->stop_it <= it) return;
    __shared__ double sb[MG3_MAXC];
    for (int i = threadIdx.x; i < n; i += NT) sb[i] = b[idx[i]];
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += NT) {
        double acc = 0.0;
        for (int j = 0; j < n; ++j) acc += pinv[(size_t)i * n + j] * sb[j];
        x[idx[i]] = (T)acc;
    }
}

__global__ void k3_zero(size_t n, double *a) {
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) a[e] = 0.0;
}

// Workspace fields.
enum { W_X, W_R, W_Z, W_ZT, W_P0, W_P1, W_Q, W_B, W_DINV, W_CX, W_CY, W_CZ, W_GX, W_GY, W_GZ, W_AX, W_AY, W_AZ, W_UX,
       W_UY, W_UZ, W_COUNT };
// Partial-sum buffers (NB3 groups each): residual (3), direction (1),
// update (2), right-hand side and sums (1), divergence (2), the cycle's
// statistics (3).
constexpr int PART_DOUBLES = NB3 * (3 + 1 + 2 + 1 + 1 + 2 + 3);

Dims3 make_dims(const ccns3_grid &g) {
    Dims3 d{};
    d.nx = g.nx;
    d.ny = g.ny;
    d.nz = g.nz;
    d.pitch = (g.nx + 2 + 15) / 16 * 16;
    d.plane = (size_t)(g.ny + 2) * d.pitch;
    d.n = d.plane * (g.nz + 2);
    d.gxt = (g.nx + T3X - 1) / T3X;
    d.gyt = (g.ny + T3Y - 1) / T3Y;
    d.gzt = (g.nz + T3Z - 1) / T3Z;
    d.ntile = d.gxt * d.gyt * d.gzt;
    int nb = std::min(d.ntile, NB3);
    nb = (nb + 7) / 8 * 8;
    d.tpb = (d.ntile + nb - 1) / nb;
    d.nblk = nb;
    size_t f = (d.n + (size_t)NT * 4 - 1) / ((size_t)NT * 4);
    f = std::min<size_t>(std::max<size_t>(f, 8), NB3);
    d.nflat = (int)((f + 7) / 8 * 8);
    return d;
}

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// The cycle's coarse grids: each halves the one above (rounding up) until one
// has at most MG3_MAXC cells; there is always at least one.
std::vector<std::array<int, 3>> mg3_dims(const ccns3_grid &g) {
    std::vector<std::array<int, 3>> v;
    int nx = g.nx, ny = g.ny, nz = g.nz;
    do {
        nx = (nx + 1) / 2;
        ny = (ny + 1) / 2;
        nz = (nz + 1) / 2;
        v.push_back({nx, ny, nz});
    } while ((long)nx * ny * nz > MG3_MAXC);
    return v;
}
size_t mg3_elems(const std::array<int, 3> &d) { return (size_t)(d[0] + 2) * (d[1] + 2) * (d[2] + 2); }
constexpr int MG3_ARRS = 7;  // cx, cy, cz, dinv, b, x, xt of a coarse level
size_t mg3_bytes(const ccns3_grid &g) {
    size_t b = 0;
    for (const auto &d : mg3_dims(g)) b += MG3_ARRS * align256(mg3_elems(d) * sizeof(double));
    return b + align256((size_t)MG3_MAXC * MG3_MAXC * sizeof(double)) + align256(MG3_MAXC * sizeof(int));
}
// The FP32 cycle's finest-level fields: c^x, c^y, c^z, 1/diag, x, xt and the
// residual of the restriction, in the layout of the FP64 fields.
constexpr int MG3_F32_FIELDS = 7;
size_t mg3_f32_bytes(size_t n) { return MG3_F32_FIELDS * align256(n * sizeof(float)); }

// Coarse Poisson weights of a 2x2x2 agglomeration (dense layouts, one ghost
// layer): the weight of a coarse face is half the sum of the weights of the
// fine faces it covers; the coarse diagonal is the sum of the six.
void coarsen3(int nx, int ny, int nz, const std::vector<double> (&c)[3], int NX, int NY, int NZ,
              std::vector<double> (&cc)[3], std::vector<double> &dinv) {
    const size_t fw = nx + 2, fp = fw * (ny + 2), cw = NX + 2, cp = cw * (NY + 2), n = cp * (NZ + 2);
    auto f = [&](int i, int j, int k) { return (size_t)k * fp + (size_t)j * fw + i; };
    auto C = [&](int i, int j, int k) { return (size_t)k * cp + (size_t)j * cw + i; };
    for (auto &a : cc) a.assign(n, 0.0);
    dinv.assign(n, 0.0);
    for (int K = 1; K <= NZ; ++K)
        for (int J = 1; J <= NY; ++J)
            for (int I = 1; I <= NX; ++I) {
                const int i0 = 2 * I - 1, i1 = std::min(2 * I, nx), j0 = 2 * J - 1, j1 = std::min(2 * J, ny);
                const int k0 = 2 * K - 1, k1 = std::min(2 * K, nz);
                double s = 0.0;
                if (I < NX) {  // the fine faces between columns 2I and 2I+1
                    for (int k = k0; k <= k1; ++k)
                        for (int j = j0; j <= j1; ++j) s += c[0][f(2 * I, j, k)];
                    cc[0][C(I, J, K)] = 0.5 * s;
                }
                if (J < NY) {
                    s = 0.0;
                    for (int k = k0; k <= k1; ++k)
                        for (int i = i0; i <= i1; ++i) s += c[1][f(i, 2 * J, k)];
                    cc[1][C(I, J, K)] = 0.5 * s;
                }
                if (K < NZ) {
                    s = 0.0;
                    for (int j = j0; j <= j1; ++j)
                        for (int i = i0; i <= i1; ++i) s += c[2][f(i, j, 2 * K)];
                    cc[2][C(I, J, K)] = 0.5 * s;
                }
            }
    for (int K = 1; K <= NZ; ++K)
        for (int J = 1; J <= NY; ++J)
            for (int I = 1; I <= NX; ++I) {
                const size_t e = C(I, J, K);
                const double dg = cc[0][e] + cc[0][e - 1] + cc[1][e] + cc[1][e - cw] + cc[2][e] + cc[2][e - cp];
                dinv[e] = dg > 0.0 ? 1.0 / dg : 0.0;
            }
}

// Work-groups of an element-wise kernel over n elements.
int flat3(size_t n) {
    size_t f = (n + (size_t)NT * 4 - 1) / ((size_t)NT * 4);
    f = std::min<size_t>(std::max<size_t>(f, 8), NB3);
    return (int)((f + 7) / 8 * 8);
}

}  // namespace
}  // namespace ccns

using namespace ccns;

struct ccns3_ctx {
    ccns3_grid g{};
    ccns3_params p{};
    Dims3 d{};
    hipStream_t stream = nullptr;
    double *w[W_COUNT] = {};
    double *part = nullptr;
    Cg3 *st = nullptr;
    Cg3 *h_st = nullptr;       // pinned
    double *h_part = nullptr;  // pinned, the divergence partials
    int n_active = 0;
    int last_it = 0;  // iterations of the last solve: the first chunk of the next
    // the multigrid cycle (precond = 1): the finest level and the coarse
    // ones, the coarsest grid's unknowns and pseudo-inverse
    std::vector<LevT<double>> lev;  // precond 1
    std::vector<LevT<float>> lev32; // precond 2
    float *r2_32 = nullptr;         // precond 2: the finest residual of the restriction
    int mg_n = 0;
    int *mg_idx = nullptr;
    double *mg_pinv = nullptr;
    std::string err;
    // optional timing of the CG kernels: an event pair around each launch of
    // a chunk, direction (0) and update (1) kernels, and the finest level's
    // first up-sweep of the multigrid cycle that follows each update (2)
    bool timing = false;
    hipEvent_t ev[3][64][2] = {};
    double t_ms[3] = {0.0, 0.0, 0.0};
    long t_count[3] = {0, 0, 0};
    int tslot = -1;  // the chunk slot of the cycle being enqueued (-1: not timed)
};

namespace {

ccns_status fail3(ccns3_ctx *c, ccns_status s, const std::string &m) {
    if (c) c->err = m;
    return s;
}

#define HIP3(ctx, call)                                                                      \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail3(ctx, CCNS_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

double *part_at(ccns3_ctx *c, int which) {
    // 0 residual (3), 1 direction (1), 2 update (2), 3 rhs/sums (1), 4
    // divergence (2), 5 the cycle's statistics (3)
    static const int off[6] = {0, 3, 4, 6, 7, 9};
    return c->part + (size_t)off[which] * NB3;
}

ccns_status upload(ccns3_ctx *c, double *dst, const double *src, hipMemcpyKind kind) {
    const size_t W = c->g.nx + 2, rows = (size_t)(c->g.ny + 2) * (c->g.nz + 2);
    HIP3(c, hipMemcpy2DAsync(dst, c->d.pitch * sizeof(double), src, W * sizeof(double), W * sizeof(double), rows, kind,
                             c->stream));
    return CCNS_OK;
}
ccns_status download(ccns3_ctx *c, double *dst, const double *src, hipMemcpyKind kind) {
    const size_t W = c->g.nx + 2, rows = (size_t)(c->g.ny + 2) * (c->g.nz + 2);
    HIP3(c, hipMemcpy2DAsync(dst, W * sizeof(double), src, c->d.pitch * sizeof(double), W * sizeof(double), rows, kind,
                             c->stream));
    return CCNS_OK;
}

// Stages host rows for an upload in flight (they stay in `keep` until the
// caller synchronises the stream).
template <class T>
const T *stage(std::vector<std::vector<char>> &keep, const std::vector<double> &v) {
    keep.emplace_back(v.size() * sizeof(T));
    T *h = (T *)keep.back().data();
    for (size_t k = 0; k < v.size(); ++k) h[k] = (T)v[k];
    return h;
}

// The cycle's levels in storage type T.  The finest: in FP64 the context's
// fields (x = ZT, xt = Z), in FP32 copies of the weights and 1/diag and
// fields of its own in `f32`.  The coarse ones from coarsen3 in the
// workspace at `mg`, and the coarsest grid's dense operator on its unknowns
// with its pseudo-inverse (which also handles the null space of the closed
// box).  Host rows stay in `keep` until the caller synchronises the stream.
template <class T>
ccns_status mg3_setup(ccns3_ctx *c, const HostCoef3 &hc, char *mg, char *f32, std::vector<LevT<T>> &lev,
                      std::vector<std::vector<char>> &keep) {
    const Dims3 &d = c->d;
    lev.clear();
    LevT<T> l0{c->g.nx, c->g.ny, c->g.nz, d.pitch, d.plane, d.n, nullptr, nullptr, nullptr, nullptr, nullptr,
               nullptr, nullptr};
    if constexpr (sizeof(T) == sizeof(double)) {
        l0.cx = (const T *)c->w[W_CX];
        l0.cy = (const T *)c->w[W_CY];
        l0.cz = (const T *)c->w[W_CZ];
        l0.dinv = (const T *)c->w[W_DINV];
        l0.x = (T *)c->w[W_ZT];
        l0.xt = (T *)c->w[W_Z];
    } else {
        const size_t fb = align256(d.n * sizeof(float)), W = c->g.nx + 2;
        T *f[MG3_F32_FIELDS];
        for (int k = 0; k < MG3_F32_FIELDS; ++k) f[k] = (T *)(f32 + k * fb);
        const std::vector<double> *src[4] = {&hc.c[0], &hc.c[1], &hc.c[2], &hc.dinv};
        for (int k = 0; k < 4; ++k)
            HIP3(c, hipMemcpy2DAsync(f[k], d.pitch * sizeof(T), stage<T>(keep, *src[k]), W * sizeof(T), W * sizeof(T),
                                     (size_t)(c->g.ny + 2) * (c->g.nz + 2), hipMemcpyHostToDevice, c->stream));
        l0.cx = f[0];
        l0.cy = f[1];
        l0.cz = f[2];
        l0.dinv = f[3];
        l0.x = f[4];
        l0.xt = f[5];
        c->r2_32 = (float *)f[6];
    }
    lev.push_back(l0);
    std::vector<double> cf[3] = {hc.c[0], hc.c[1], hc.c[2]}, dinv;
    int nx = c->g.nx, ny = c->g.ny, nz = c->g.nz;
    size_t off = 0;
    for (const auto &D : mg3_dims(c->g)) {
        std::vector<double> cc[3];
        coarsen3(nx, ny, nz, cf, D[0], D[1], D[2], cc, dinv);
        // slots of FP64 size serve either storage type
        const size_t n = mg3_elems(D), ab = align256(n * sizeof(double));
        T *a[MG3_ARRS];
        for (int k = 0; k < MG3_ARRS; ++k) a[k] = (T *)(mg + off + k * ab);
        off += MG3_ARRS * ab;
        const std::vector<double> *src[4] = {&cc[0], &cc[1], &cc[2], &dinv};
        for (int k = 0; k < 4; ++k)
            HIP3(c, hipMemcpyAsync(a[k], stage<T>(keep, *src[k]), n * sizeof(T), hipMemcpyHostToDevice, c->stream));
        const int pitch = D[0] + 2;
        lev.push_back(LevT<T>{D[0], D[1], D[2], pitch, (size_t)pitch * (D[1] + 2), n, a[0], a[1], a[2], a[3], a[4],
                              a[5], a[6]});
        for (int k = 0; k < 3; ++k) cf[k].swap(cc[k]);
        nx = D[0];
        ny = D[1];
        nz = D[2];
    }
    // the coarsest grid (dinv and cf now hold its fields)
    const size_t cw = nx + 2, cp = cw * (ny + 2);
    std::vector<int> idx, pos(dinv.size(), -1);
    for (size_t e = 0; e < dinv.size(); ++e)
        if (dinv[e] > 0.0) {
            pos[e] = (int)idx.size();
            idx.push_back((int)e);
        }
    const int n = (int)idx.size();
    if (n > MG3_MAXC) return fail3(c, CCNS_EINVAL, "coarsest grid larger than its bound");
    std::vector<double> A((size_t)n * n, 0.0);
    for (int a = 0; a < n; ++a) {
        const size_t e = idx[a];
        A[(size_t)a * n + a] = 1.0 / dinv[e];
        const size_t nb[6] = {e + 1, e - 1, e + cw, e - cw, e + cp, e - cp};
        const double w[6] = {cf[0][e], cf[0][e - 1], cf[1][e], cf[1][e - cw], cf[2][e], cf[2][e - cp]};
        for (int q = 0; q < 6; ++q)
            if (w[q] > 0.0 && pos[nb[q]] >= 0) A[(size_t)a * n + pos[nb[q]]] -= w[q];
    }
    c->mg_pinv = (double *)(mg + off);
    c->mg_idx = (int *)(mg + off + align256((size_t)MG3_MAXC * MG3_MAXC * sizeof(double)));
    c->mg_n = n;
    if (n > 0) {
        const double *pinv = stage<double>(keep, pseudo_inverse_spsd(A, n));
        HIP3(c, hipMemcpyAsync(c->mg_pinv, pinv, (size_t)n * n * sizeof(double), hipMemcpyHostToDevice, c->stream));
        keep.emplace_back((size_t)n * sizeof(int));
        std::memcpy(keep.back().data(), idx.data(), (size_t)n * sizeof(int));
        HIP3(c, hipMemcpyAsync(c->mg_idx, keep.back().data(), (size_t)n * sizeof(int), hipMemcpyHostToDevice,
                               c->stream));
    }
    return CCNS_OK;
}

// One V-cycle, z = M^-1 r, on the context's stream, with the levels `lv`
// stored in T and r2 the finest level's residual field (the finest level on
// the tiles of k3_stencil, with d.nblk work-groups; z is written in FP64).
// ns = 2: the finest level's last sweep writes the partials (r.z, r.r) at
// `part`; ns = 3 also b'.b'.  it: the CG iteration whose update this cycle
// follows (-1 before the first); every kernel returns at once when the
// solve stopped at or before it.
template <class T>
ccns_status vcycle3(ccns3_ctx *c, const std::vector<LevT<T>> &lv, T *r2, int ns, double *part, int it) {
    hipStream_t sm = c->stream;
    const int L = (int)lv.size() - 1;
    const Dims3 &d = c->d;
    const double *r = c->w[W_R];
    double *z = c->w[W_Z];
    for (int l = 0; l < L; ++l) {
        const LevT<T> &v = lv[l];
        // the two down-sweeps from x = 0 in one launch, then the restriction
        // (on the finest level through its stored residual)
        if (l == 0) {
            k3_mg_tile<T_PRE, 0, T, T><<<d.nblk, NT, 0, sm>>>(d, v, r, nullptr, v, nullptr, v.xt, nullptr, nullptr,
                                                              c->st, it);
            k3_mg_tile<T_RES, 0, T, T><<<d.nblk, NT, 0, sm>>>(d, v, r, v.xt, v, nullptr, r2, nullptr, nullptr, c->st,
                                                              it);
            k3_mg_sum8<T><<<flat3(lv[1].n), NT, 0, sm>>>(v, r2, lv[1], c->st, it);
            continue;
        }
        k3_mg_sweep<true, false, T><<<flat3(v.n), NT, 0, sm>>>(v, nullptr, v.xt, v, nullptr, c->st, it);
        k3_mg_restrict<T><<<flat3(lv[l + 1].n), NT, 0, sm>>>(v, v.xt, lv[l + 1], c->st, it);
    }
    k3_mg_coarsest<T><<<1, NT, 0, sm>>>(c->mg_n, c->mg_idx, c->mg_pinv, lv[L].b, lv[L].x, c->st, it);
    for (int l = L - 1; l >= 0; --l) {
        const LevT<T> &v = lv[l];
        const int nb = flat3(v.n);
        // the first up-sweep on xt plus the interpolated coarse correction
        const T *xc = l + 1 == L ? lv[L].x : lv[l + 1].xt;
        if (l > 0) {
            k3_mg_sweep<false, true, T><<<nb, NT, 0, sm>>>(v, v.xt, v.x, lv[l + 1], xc, c->st, it);
            k3_mg_sweep<false, false, T><<<nb, NT, 0, sm>>>(v, v.x, v.xt, v, nullptr, c->st, it);
            continue;
        }
        const bool timed = c->tslot >= 0;
        if (timed) HIP3(c, hipEventRecord(c->ev[2][c->tslot][0], sm));
        k3_mg_tile<T_POST1, 0, T, T><<<d.nblk, NT, 0, sm>>>(d, v, r, v.xt, lv[1], xc, v.x, nullptr, nullptr, c->st,
                                                            it);
        if (timed) HIP3(c, hipEventRecord(c->ev[2][c->tslot][1], sm));
        if (ns == 3)
            k3_mg_tile<T_POST2, 3, T, double><<<d.nblk, NT, 0, sm>>>(d, v, r, v.x, v, nullptr, z, c->w[W_B], part,
                                                                     c->st, it);
        else
            k3_mg_tile<T_POST2, 2, T, double><<<d.nblk, NT, 0, sm>>>(d, v, r, v.x, v, nullptr, z, nullptr, part,
                                                                     c->st, it);
    }
    HIP3(c, hipGetLastError());
    return CCNS_OK;
}

ccns_status vcycle3(ccns3_ctx *c, int ns, double *part, int it) {
    return c->p.precond == 2 ? vcycle3<float>(c, c->lev32, c->r2_32, ns, part, it)
                             : vcycle3<double>(c, c->lev, c->w[W_Q], ns, part, it);
}

bool params_ok(const ccns3_params *p) {
    return p && p->rho > 0.0 && std::isfinite(p->rho) && p->tau > 0.0 && std::isfinite(p->tau) && p->tol >= 0.0 &&
           std::isfinite(p->tol) && p->maxit >= 0 && p->mass_floor >= 0.0 && p->mass_floor <= 1.0 &&
           p->precond >= 0 && p->precond <= 2;
}

}  // namespace

extern "C" {

size_t ccns3_workspace_bytes(const ccns3_grid *g) {
    if (!grid3_valid(g)) return 0;
    const Dims3 d = make_dims(*g);
    if (d.n > (size_t)INT_MAX) return 0;  // the kernels index a field's elements in 32 bits
    return (size_t)W_COUNT * align256(d.n * sizeof(double)) + align256(PART_DOUBLES * sizeof(double)) +
           align256(sizeof(Cg3)) + mg3_bytes(*g) + mg3_f32_bytes(d.n);
}

ccns_status ccns3_ctx_create(const ccns3_grid *grid, const ccns3_params *params, const double *caps_host,
                             void *workspace, size_t workspace_bytes, void *stream, ccns3_ctx **out) {
    if (!out || !grid3_valid(grid) || !params_ok(params) || !caps_host || !workspace) return CCNS_EINVAL;
    *out = nullptr;
    if (((uintptr_t)workspace & 255) != 0) return CCNS_EINVAL;
    if (ccns3_workspace_bytes(grid) == 0) return CCNS_EINVAL;
    if (workspace_bytes < ccns3_workspace_bytes(grid)) return CCNS_ENOMEM;
    ccns3_ctx *c = new (std::nothrow) ccns3_ctx;
    if (!c) return CCNS_ENOMEM;
    c->g = *grid;
    c->p = *params;
    c->d = make_dims(*grid);
    c->stream = (hipStream_t)stream;
    HostCoef3 hc;
    std::string err;
    ccns_status s = prepare3(*grid, *params, caps_host, hc, err);
    if (s != CCNS_OK) {
        delete c;
        return s;
    }
    c->n_active = hc.n_active;
    char *base = (char *)workspace;
    const size_t fb = align256(c->d.n * sizeof(double));
    for (int k = 0; k < W_COUNT; ++k) c->w[k] = (double *)(base + (size_t)k * fb);
    c->part = (double *)(base + (size_t)W_COUNT * fb);
    c->st = (Cg3 *)(base + (size_t)W_COUNT * fb + align256(PART_DOUBLES * sizeof(double)));
    if (hipHostMalloc((void **)&c->h_st, sizeof(Cg3)) != hipSuccess ||
        hipHostMalloc((void **)&c->h_part, 2 * NB3 * sizeof(double)) != hipSuccess) {
        ccns3_ctx_destroy(c);
        return CCNS_EDEVICE;
    }
    const size_t total = ccns3_workspace_bytes(grid) / sizeof(double);
    k3_zero<<<1024, NT, 0, c->stream>>>(total, (double *)workspace);
    const std::vector<double> *src[] = {&hc.dinv, &hc.c[0], &hc.c[1], &hc.c[2], &hc.g[0],
                                        &hc.g[1], &hc.g[2], &hc.a[0], &hc.a[1], &hc.a[2]};
    const int dst[] = {W_DINV, W_CX, W_CY, W_CZ, W_GX, W_GY, W_GZ, W_AX, W_AY, W_AZ};
    for (int k = 0; k < 10; ++k)
        if ((s = upload(c, c->w[dst[k]], src[k]->data(), hipMemcpyHostToDevice)) != CCNS_OK) {
            (void)hipStreamSynchronize(c->stream);
            ccns3_ctx_destroy(c);
            return s;
        }
    std::vector<std::vector<char>> keep;  // host rows of uploads in flight
    char *mg = base + (size_t)W_COUNT * fb + align256(PART_DOUBLES * sizeof(double)) + align256(sizeof(Cg3));
    char *f32 = mg + mg3_bytes(*grid);
    if (c->p.precond == 1)
        s = mg3_setup<double>(c, hc, mg, f32, c->lev, keep);
    else if (c->p.precond == 2)
        s = mg3_setup<float>(c, hc, mg, f32, c->lev32, keep);
    if (s != CCNS_OK) {
        (void)hipStreamSynchronize(c->stream);
        ccns3_ctx_destroy(c);
        return s;
    }
    if (hipStreamSynchronize(c->stream) != hipSuccess || hipGetLastError() != hipSuccess) {
        ccns3_ctx_destroy(c);
        return CCNS_EDEVICE;
    }
    *out = c;
    return CCNS_OK;
}

static void free_events(ccns3_ctx *c) {
    for (auto &kk : c->ev)
        for (auto &k : kk)
            for (auto &e : k)
                if (e) {
                    (void)hipEventDestroy(e);
                    e = nullptr;
                }
}

void ccns3_ctx_destroy(ccns3_ctx *c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    free_events(c);
    if (c->h_st) (void)hipHostFree(c->h_st);
    if (c->h_part) (void)hipHostFree(c->h_part);
    delete c;
}

static const int kField3[CCNS3_NFIELDS] = {W_UX, W_UY, W_UZ, W_X};

ccns_status ccns3_field_set(ccns3_ctx *c, int field, const double *src, int is_device) {
    if (!c || !src || field < 0 || field >= CCNS3_NFIELDS) return fail3(c, CCNS_EINVAL, "bad field");
    ccns_status s = upload(c, c->w[kField3[field]], src, is_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice);
    if (s != CCNS_OK) return s;
    HIP3(c, hipStreamSynchronize(c->stream));
    return CCNS_OK;
}

ccns_status ccns3_field_get(ccns3_ctx *c, int field, double *dst, int is_device) {
    if (!c || !dst || field < 0 || field >= CCNS3_NFIELDS) return fail3(c, CCNS_EINVAL, "bad field");
    ccns_status s = download(c, dst, c->w[kField3[field]], is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost);
    if (s != CCNS_OK) return s;
    HIP3(c, hipStreamSynchronize(c->stream));
    return CCNS_OK;
}

ccns_status ccns3_apply_poisson(ccns3_ctx *c, const double *in_dev, double *out_dev) {
    if (!c || !in_dev || !out_dev) return fail3(c, CCNS_EINVAL, "null argument");
    ccns_status s = upload(c, c->w[W_R], in_dev, hipMemcpyDeviceToDevice);
    if (s != CCNS_OK) return s;
    const Dims3 &d = c->d;
    double **w = c->w;
    k3_stencil<S_APPLY><<<d.nblk, NT, 0, c->stream>>>(d, w[W_CX], w[W_CY], w[W_CZ], w[W_DINV], w[W_R], nullptr,
                                                       w[W_Q], nullptr, nullptr, c->st, 0, nullptr, 0, 0, nullptr);
    HIP3(c, hipGetLastError());
    if ((s = download(c, out_dev, w[W_Q], hipMemcpyDeviceToDevice)) != CCNS_OK) return s;
    HIP3(c, hipStreamSynchronize(c->stream));
    return CCNS_OK;
}

ccns_status ccns3_project(ccns3_ctx *c, ccns3_info *info) {
    if (!c) return CCNS_EINVAL;
    const Dims3 &d = c->d;
    double **w = c->w;
    hipStream_t sm = c->stream;
    double *pr = part_at(c, 0), *pd = part_at(c, 1), *pu = part_at(c, 2), *ps = part_at(c, 3), *pv = part_at(c, 4);
    double *pm = part_at(c, 5);
    const bool mg = c->p.precond >= 1;
    // solver state
    Cg3 h{};
    h.tol2 = c->p.tol * c->p.tol;
    h.stop_it = INT_MAX;
    h.maxit = c->p.maxit;
    h.status = CCNS_ENOTCONV;
    *c->h_st = h;
    HIP3(c, hipMemcpyAsync(c->st, c->h_st, sizeof(Cg3), hipMemcpyHostToDevice, sm));
    // b = -(rho/tau) cont(U*, 0); r = b - mean - (-L) x; z = r / diag
    k3_rhs<<<d.nflat, NT, 0, sm>>>(d, w[W_AX], w[W_AY], w[W_AZ], w[W_UX], w[W_UY], w[W_UZ], w[W_DINV],
                                   c->p.rho / c->p.tau, w[W_B], ps);
    k3_stencil<S_RESID><<<d.nblk, NT, 0, sm>>>(d, w[W_CX], w[W_CY], w[W_CZ], w[W_DINV], w[W_X], nullptr, w[W_R],
                                               w[W_Z], w[W_B], c->st, 0, ps, d.nflat, c->n_active, pr);
    HIP3(c, hipGetLastError());
    // with the multigrid preconditioner z = M^-1 r comes from a cycle, whose
    // last sweep writes (r.z, r.r) (and b'.b' before the first iteration)
    ccns_status s = CCNS_OK;
    if (mg && (s = vcycle3(c, 3, pm, -1)) != CCNS_OK) return s;
    // the first chunk covers the last solve's iterations (one look at the
    // solver state when the count repeats), then chunks double
    int it = 0, chunk = std::min(std::max(8, c->last_it + 1), 64);
    for (;;) {
        const int it0 = it;
        for (int k = 0; k < chunk; ++k, ++it) {
            double *pnew = w[(it & 1) ? W_P1 : W_P0], *pold = w[(it & 1) ? W_P0 : W_P1];
            if (c->timing) HIP3(c, hipEventRecord(c->ev[0][k][0], sm));
            k3_stencil<S_DIR><<<d.nblk, NT, 0, sm>>>(d, w[W_CX], w[W_CY], w[W_CZ], w[W_DINV], w[W_Z], pold, pnew,
                                                     w[W_Q], nullptr, c->st, it, mg ? pm : (it == 0 ? pr : pu),
                                                     (it == 0 || mg) ? d.nblk : d.nflat, c->n_active, pd);
            if (c->timing) {
                HIP3(c, hipEventRecord(c->ev[0][k][1], sm));
                HIP3(c, hipEventRecord(c->ev[1][k][0], sm));
            }
            auto upd = mg ? k3_update<false> : k3_update<true>;
            upd<<<d.nflat, NT, 0, sm>>>(d, w[W_DINV], pnew, w[W_Q], w[W_X], w[W_R], w[W_Z], c->st, it, pd, d.nblk, pu);
            if (c->timing) HIP3(c, hipEventRecord(c->ev[1][k][1], sm));
            c->tslot = c->timing ? k : -1;
            s = mg ? vcycle3(c, 2, pm, it) : CCNS_OK;
            c->tslot = -1;
            if (s != CCNS_OK) return s;
        }
        HIP3(c, hipGetLastError());
        HIP3(c, hipMemcpyAsync(c->h_st, c->st, sizeof(Cg3), hipMemcpyDeviceToHost, sm));
        HIP3(c, hipStreamSynchronize(sm));
        if (c->timing) {
            // launches that did the iteration's work (those at and after the
            // stopping iteration return at once)
            const int stop = c->h_st->stop_it;
            for (int k = 0; k < chunk && it0 + k < stop; ++k)
                for (int q = 0; q < (mg ? 3 : 2); ++q) {
                    float ms = 0.0f;
                    HIP3(c, hipEventElapsedTime(&ms, c->ev[q][k][0], c->ev[q][k][1]));
                    c->t_ms[q] += ms;
                    ++c->t_count[q];
                }
        }
        if (c->h_st->stop_it != INT_MAX || it > c->p.maxit + 1) break;
        chunk = std::min(chunk * 2, 64);
    }
    // the correction (the mean of Phi cancels in its differences), then Phi
    // minus its mean and the divergence figures
    k3_sum<<<d.nflat, NT, 0, sm>>>(d, w[W_DINV], w[W_X], ps);
    k3_correct<<<d.nflat, NT, 0, sm>>>(d, w[W_GX], w[W_GY], w[W_GZ], w[W_AX], w[W_AY], w[W_AZ], w[W_X],
                                       c->p.tau / c->p.rho, w[W_UX], w[W_UY], w[W_UZ]);
    k3_div_shift<<<d.nflat, NT, 0, sm>>>(d, w[W_AX], w[W_AY], w[W_AZ], w[W_UX], w[W_UY], w[W_UZ], w[W_DINV],
                                         w[W_X], ps, d.nflat, c->n_active, pv);
    HIP3(c, hipGetLastError());
    HIP3(c, hipMemcpyAsync(c->h_part, pv, 2 * (size_t)d.nflat * sizeof(double), hipMemcpyDeviceToHost, sm));
    HIP3(c, hipMemcpyAsync(c->h_st, c->st, sizeof(Cg3), hipMemcpyDeviceToHost, sm));
    HIP3(c, hipStreamSynchronize(sm));
    double dmax = 0.0, fmax_ = 0.0;
    for (int b = 0; b < d.nflat; ++b) {
        dmax = std::max(dmax, c->h_part[b]);
        fmax_ = std::max(fmax_, c->h_part[d.nflat + b]);
    }
    const Cg3 &r = *c->h_st;
    const ccns_status status = r.stop_it == INT_MAX ? CCNS_ENOTCONV : (ccns_status)r.status;
    c->last_it = r.stop_it == INT_MAX ? it : r.stop_it;
    if (info) {
        info->iterations = r.stop_it == INT_MAX ? it : r.it_final;
        info->status = status;
        info->rel_residual = r.bb > 0.0 ? std::sqrt(std::max(r.rr_final, 0.0) / r.bb) : 0.0;
        info->div_rel = fmax_ > 0.0 ? dmax / fmax_ : 0.0;
        info->n_active = c->n_active;
    }
    if (status != CCNS_OK) return fail3(c, status, "Poisson solve did not converge");
    return CCNS_OK;
}

ccns_status ccns3_timing(ccns3_ctx *c, int enable, double *ms, long *count) {
    if (!c || enable < -1 || enable > 1) return fail3(c, CCNS_EINVAL, "bad argument");
    for (int q = 0; q < 3; ++q) {
        if (ms) ms[q] = c->t_ms[q];
        if (count) count[q] = c->t_count[q];
    }
    if (enable >= 0)
        for (int q = 0; q < 3; ++q) {
            c->t_ms[q] = 0.0;
            c->t_count[q] = 0;
        }
    if (enable == 1 && !c->timing) {
        for (auto &kk : c->ev)
            for (auto &k : kk)
                for (auto &e : k)
                    if (hipEventCreate(&e) != hipSuccess) {
                        free_events(c);
                        return fail3(c, CCNS_EDEVICE, "hipEventCreate");
                    }
        c->timing = true;
    } else if (enable == 0 && c->timing) {
        (void)hipStreamSynchronize(c->stream);
        free_events(c);
        c->timing = false;
    }
    return CCNS_OK;
}

const char *ccns3_last_error(const ccns3_ctx *c) { return c ? c->err.c_str() : "null context"; }

}  // extern "C"
