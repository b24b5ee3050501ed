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
//  - stencil halos are staged in LDS where a value is reused by several
//    neighbours; all global loads of a thread are issued before the
//    arithmetic that depends on the activity masks;
//  - reductions never use atomics or fences: each work-group writes its
//    partial sums, and the next kernel (or a one-group kernel) reduces them
//    in a fixed order, so results are reproducible bit for bit.  Solver
//    scalars (alpha, beta, convergence) are formed on the device; the host
//    only reads a done flag every few iterations.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <atomic>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <type_traits>
#include <vector>

#include "ccns.h"
#include "ccns_internal.h"
#include "ccns_kern.h"

namespace ccns {

// ---------------------------------------------------------------------------
// solver state on the device
// ---------------------------------------------------------------------------

// Conjugate-gradient bookkeeping.  Scalars that change every iteration live
// in two slots used alternately, so that the work-group that records
// iteration i never overwrites what the other groups of the same kernel are
// still reading (iteration i-1).
struct CgSlot {
    double rz;
    int it;
    int pad;
};
struct CgState {
    double tol2, fnorm2, rnorm2_final;
    int maxit, zero_mean, n_active;
    int done, status, it_final;
    int stop_it;  // predictor CG: the launch that stopped the solve
    CgSlot slot[2];
};

struct DiagState {
    double mass, ke, momx, momy, divmax;
};

// Coefficient sets.  T is the storage and stencil type of a solve: double in
// precision 0 and in the FP64 residuals of precision 1, float in the inner
// iterations of precision 1 (whose dot products are still summed in double).
template <class T>
struct PoisCoefT {
    const T *cx, *cy, *dinv;
};
using PoisCoef = PoisCoefT<double>;

template <class T>
struct ViscCoefT {
    const T *bxx, *bxy, *byy, *byx, *wxx, *wyy, *nxx, *nxy, *nyx, *nyy;
};

template <class T>
struct PredCoefT {
    ViscCoefT<T> vc;
    const T *vu, *vv, *hdx, *hdy;
    double rt, mu;
    const int *cls;  // coefficient classes of the predictor CG (or null)
    const T *tab;
};

// Coefficient classes of the predictor CG.  Away from the bodies and the
// walls the capacities repeat, so every entry k of the face layout can name
// a row of a small table that holds each value the CG kernel reads for it:
// the Jacobi diagonal and face volumes at k, and the capacities and weights
// of the strain stencils at k and its neighbours.  The kernel then reads one
// index per entry instead of twelve coefficient arrays; the values, and so
// the arithmetic, are those of the arrays.
enum PredRow {
    PR_HDX, PR_HDY, PR_VU, PR_VV,
    PR_BXX_W, PR_BXX, PR_BXX_E, PR_WXX, PR_WXX_E,    // B^xx at k-1, k, k+1; 1/W^xx at k, k+1
    PR_BYY_S, PR_BYY, PR_BYY_N, PR_WYY, PR_WYY_N,    // B^yy at k-P, k, k+P; 1/W^yy at k, k+P
    PR_BXY, PR_BYX, PR_BXY_N, PR_BYX_E,              // B^xy at k, k+P; B^yx at k, k+1
    PR_NXX, PR_NYY, PR_NXY, PR_NYX,                  // node weights at k
    PR_COUNT
};
constexpr int PCW = 24;  // row width (PR_COUNT, padded)
static_assert(PR_COUNT <= PCW, "class row too narrow");
struct PredCoef {
    ViscCoef vc;
    const double *vu, *vv, *hdx, *hdy;
    double rt, mu;
};

// Shared decision of every work-group of a direction kernel: given the
// statistics of the current residual (r.z, sum z, sum r, r.r), is the solve
// finished, and if not, what are rz, mean(z) and beta.  Group 0 records.
struct DirStep {
    bool stop;
    double rz, mean, beta;
};
template <class G>
__device__ inline DirStep cg_decide(const G &g, CgState *st, int first, int par, double fnorm2, double rs, double s,
                                    double r, double rr) {
    DirStep o;
    const double m = st->zero_mean ? s / (double)st->n_active : 0.0;
    o.mean = m;
    o.rz = rs - m * r;
    const int it = first ? 0 : st->slot[par ^ 1].it + 1;
    // a residual that is not finite never counts as converged; r.z of an
    // unconverged residual must be positive (the preconditioner is SPD)
    const bool conv = rr <= st->tol2 * fnorm2;
    const bool brk = !conv && !(o.rz > 0.0 && o.rz < INFINITY);
    const bool lim = it >= st->maxit;
    o.stop = conv || lim || brk;
    o.beta = first ? 0.0 : o.rz / st->slot[par ^ 1].rz;
    if (g.b() == 0 && threadIdx.x == 0) {
        if (first) st->fnorm2 = fnorm2;
        if (o.stop) {
            st->done = 1;
            st->status = conv ? 0 : (brk ? CCNS_EBREAKDOWN : CCNS_ENOTCONV);
            st->it_final = it;
            st->rnorm2_final = rr;
        } else {
            st->slot[par].rz = o.rz;
            st->slot[par].it = it;
        }
    }
    return o;
}

// ---------------------------------------------------------------------------
// Poisson PCG kernels (A = -L, symmetric positive semi-definite; the
// preconditioned residual is projected to zero mean, end of Sec. 4.6)
// ---------------------------------------------------------------------------

// b = (rho/tau) cont(U*, D) on the pressure unknowns (eq:pm_poisson); sum b.
template <class G>
__device__ __forceinline__ void pois_rhs_body(const G &g, Dims d, PoisCoef pc, const double *__restrict__ ax,
                                                 const double *__restrict__ ay, const double *__restrict__ het,
                                                 const double *__restrict__ usx, const double *__restrict__ usy,
                                                 double *__restrict__ b, double scale, double *pout) {
    const size_t P = d.pitch;
    double v[1] = {0.0};
    struct In {
        double ae, ue, aw, uw, an, vn, as, vs, h, dv;
    };
    auto load = [&](size_t k) {
        // the west and south neighbours exist for every real cell
        const size_t kw = k >= 1 ? k - 1 : k, ks = k >= P ? k - P : k;
        return In{ax[k], usx[k], ax[kw], usx[kw], ay[k], usy[k], ay[ks], usy[ks], het[k], pc.dinv[k]};
    };
    for_cells_batched<TY / 4>(g, d, load, [&](int, int j, int i, size_t k, const In &q) {
        if (i < 1 || i > d.nx || j < 1 || j > d.ny) return;
        const double c = q.ae * q.ue - q.aw * q.uw + q.an * q.vn - q.as * q.vs + q.h;
        const double bv = q.dv > 0.0 ? scale * c : 0.0;
        b[k] = bv;
        v[0] += bv;
    });
    put_partials<1>(g, v, pout, d.nblk);
}
__global__ __launch_bounds__(NT) void k_pois_rhs(Dims d, PoisCoef pc, const double *__restrict__ ax,
                                                 const double *__restrict__ ay, const double *__restrict__ het,
                                                 const double *__restrict__ usx, const double *__restrict__ usy,
                                                 double *__restrict__ b, double scale, double *pout) {
    pois_rhs_body(SoloGrid{}, d, pc, ax, ay, het, usx, usy, b, scale, pout);
}

// Sum of a caller-provided b over the unknowns.
__global__ __launch_bounds__(NT) void k_pois_sum(Dims d, PoisCoef pc, const double *__restrict__ b, double *pout) {
    double v[1] = {0.0};
    for_cells(d, [&](int, int, int, size_t k) {
        if (pc.dinv[k] > 0.0) v[0] += b[k];
    });
    put_partials<1>(v, pout, d.nblk);
}

// b <- b - mean(b) (when pin is given: the partial sums of b); f = -b;
// r = f - A x in FP64; statistics of r.
//  MIX = false: r is stored; partials (f.f, r.z, z, r, r.r) with z = D^-1 r.
//  MIX = true (precision 1): r is rounded to float into r32 (the right-hand
//  side of the inner solve, whose start value x32 is cleared); partials
//  (r32.r32, r32.z, z, r32, r32.r32 | f.f, r.r | max |r|) with z = D32^-1 r32.
template <bool MIX, class G>
__device__ __forceinline__ void pois_init_body(const G &g, Dims d, PoisCoef pc, double *__restrict__ b,
                                                  const double *__restrict__ x, double *__restrict__ r, CgState *st,
                                                  const double *pin, int nin, double *pout, float *__restrict__ r32,
                                                  float *__restrict__ x32, const float *__restrict__ dinv32) {
    double mb = 0.0;
    if (pin && st->zero_mean) {
        double t[1];
        get_totals<1>(pin, nin, t);
        mb = t[0] / (double)st->n_active;
    }
    const size_t P = d.pitch;
    double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    struct In {
        double dv, bk, ce, cw, cn, cs, x0, xe, xw, xn, xs;
        float d32;
    };
    auto load = [&](size_t k) {
        // the four neighbours exist for every unknown
        const size_t kw = k >= 1 ? k - 1 : k, ks = k >= P ? k - P : k;
        const size_t ke = k + 1 < d.n ? k + 1 : k, kn = k + P < d.n ? k + P : k;
        return In{pc.dinv[k], b[k], pc.cx[k], pc.cx[kw], pc.cy[k], pc.cy[ks], x[k], x[ke], x[kw], x[kn], x[ks],
                  MIX ? dinv32[k] : 0.0f};
    };
    for_cells_batched<TY / 4>(g, d, load, [&](int, int, int, size_t k, const In &q) {
        const double dv = q.dv;
        if (MIX) {
            x32[k] = 0.0f;
            r32[k] = 0.0f;
        }
        if (!(dv > 0.0)) return;
        const double bp = q.bk - mb;
        if (pin) b[k] = bp;
        const double ce = q.ce, cw = q.cw, cn = q.cn, cs = q.cs;
        const double Axv = (ce + cw + cn + cs) * q.x0 - ce * q.xe - cw * q.xw - cn * q.xn - cs * q.xs;
        const double rv = -bp - Axv;
        if (MIX) {
            const float rf = (float)rv;
            r32[k] = rf;
            const float sf = q.d32 * rf;
            const double rd = rf, sd = sf;
            v[0] += rd * rd;
            v[1] += rd * sd;
            v[2] += sd;
            v[3] += rd;
            v[4] += rd * rd;
            v[5] += bp * bp;
            v[6] += rv * rv;
            v[7] = fmax(v[7], fabs(rv));
        } else {
            r[k] = rv;
            const double sv = dv * rv;
            v[0] += bp * bp;
            v[1] += rv * sv;
            v[2] += sv;
            v[3] += rv;
            v[4] += rv * rv;
        }
    });
    if (g.b() == 0 && threadIdx.x == 0) {
        st->done = 0;
        st->status = 0;
        st->it_final = 0;
        st->stop_it = 0x7fffffff;
    }
    if (MIX) {
        put_partials<7, 1>(g, v, pout, d.nblk);
    } else {
        double w[5] = {v[0], v[1], v[2], v[3], v[4]};
        put_partials<5>(g, w, pout, d.nblk);
    }
}
template <bool MIX>
__global__ __launch_bounds__(NT) void k_pois_init(Dims d, PoisCoef pc, double *__restrict__ b,
                                                  const double *__restrict__ x, double *__restrict__ r, CgState *st,
                                                  const double *pin, int nin, double *pout, float *__restrict__ r32,
                                                  float *__restrict__ x32, const float *__restrict__ dinv32) {
    pois_init_body<MIX>(SoloGrid{}, d, pc, b, x, r, st, pin, nin, pout, r32, x32, dinv32);
}

// Tile of the Poisson stencil kernels: 64 columns x 16 rows (4 per thread).
constexpr int PTY = 16;

// Direction and operator: p = (M r) + beta p_old on the tile and a one-cell
// halo staged in LDS; q = A p; partial p.q.  Consumes the residual statistics
// of the previous kernel (init if `first`, else the update).
template <class T>
__global__ __launch_bounds__(NT) void k_pois_dir(Dims d, PoisCoefT<T> pc, const T *__restrict__ r,
                                                 const T *__restrict__ pold, T *__restrict__ pnew,
                                                 T *__restrict__ q, CgState *st, int first, int par,
                                                 const double *pin, int nin, double *pout) {
    if (st->done) return;
    double fn2, rs, sm, rsum, rr;
    if (first) {
        double t[5];
        get_totals<5>(pin, nin, t);
        fn2 = t[0]; rs = t[1]; sm = t[2]; rsum = t[3]; rr = t[4];
    } else {
        double t[4];
        get_totals<4>(pin, nin, t);
        fn2 = st->fnorm2; rs = t[0]; sm = t[1]; rsum = t[2]; rr = t[3];
    }
    const DirStep ds = cg_decide(SoloGrid{}, st, first, par, fn2, rs, sm, rsum, rr);
    if (ds.stop) return;
    const T beta = (T)ds.beta, m = (T)ds.mean;
    __shared__ T sp[PTY + 2][TX + 2];
    const int P = d.pitch;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    double v[1] = {0.0};
    for_tiles(d, [&](int, int c0, int r0) {
        for (int e = threadIdx.x; e < (PTY + 2) * (TX + 2); e += NT) {
            const int ly = e / (TX + 2), lx = e - ly * (TX + 2);
            const int j = r0 - 1 + ly, i = c0 - 1 + lx;
            const bool in = (j >= 0) && (j < d.rows) && (i >= 0) && (i < P);
            const size_t k = in ? (size_t)j * P + i : 0;
            const T di = pc.dinv[k], rv = r[k], po = first ? (T)0 : pold[k];
            sp[ly][lx] = (in && di > (T)0) ? (di * rv - m) + beta * po : (T)0;
        }
        __syncthreads();
        const int i = c0 + tx;
#pragma unroll
        for (int rr2 = 0; rr2 < PTY / 4; ++rr2) {
            const int lj = ty + 4 * rr2;
            const int j = r0 + lj;
            if (j < d.rows) {
                const size_t k = (size_t)j * P + i;
                const size_t kw = i > 0 ? k - 1 : k, ks = j > 0 ? k - P : k;
                const T dv = pc.dinv[k], ce = pc.cx[k], cw = pc.cx[kw], cn = pc.cy[k], cs = pc.cy[ks];
                const T pcv = sp[lj + 1][tx + 1];
                T qv = (ce + cw + cn + cs) * pcv - ce * sp[lj + 1][tx + 2] - cw * sp[lj + 1][tx] -
                       cn * sp[lj + 2][tx + 1] - cs * sp[lj][tx + 1];
                qv = dv > (T)0 ? qv : (T)0;
                pnew[k] = pcv;
                q[k] = qv;
                v[0] += (double)pcv * (double)qv;
            }
        }
        __syncthreads();
    });
    put_partials<1>(v, pout, d.nblk);
}

// x += alpha p; r -= alpha q; with STATS, the statistics of the new
// residual (without: the preconditioner that follows forms them, as the
// multigrid cycle's last kernel does, and dinv is not read).  Flat over ntot
// entries (inactive entries hold zeros); each group works on contiguous
// chunks of UPT*NT entries with every load issued before any arithmetic.
constexpr int UPT = 4;
constexpr int UT = 1024;  // threads per work-group of the update (16 wavefronts)
template <class T, bool STATS, class G>
__device__ __forceinline__ void cg_update_body(const G &g, size_t ntot, int nblk, const T *__restrict__ dinv,
                                                  T *__restrict__ x, T *__restrict__ r,
                                                  const T *__restrict__ p, const T *__restrict__ q,
                                                  CgState *st, int par, const double *pin, int nin, double *pout) {
    if (st->done) return;
    double t[1];
    get_totals<1, 0, UT>(pin, nin, t);
    if (!(t[0] > 0.0)) {
        if (g.b() == 0 && threadIdx.x == 0) {
            st->done = 1;
            st->status = CCNS_EBREAKDOWN;
            st->it_final = st->slot[par].it;
        }
        return;
    }
    const T a = (T)(st->slot[par].rz / t[0]);
    double v[4] = {0, 0, 0, 0};
    const size_t chunk = (size_t)UPT * UT;
    const int L = logical_group(g, nblk);
    for (size_t base = (size_t)L * chunk; base < ntot; base += (size_t)nblk * chunk) {
        T dv[UPT], xv[UPT], pv[UPT], rv[UPT], qv[UPT];
#pragma unroll
        for (int u = 0; u < UPT; ++u) {
            const size_t k0 = base + (size_t)u * UT + threadIdx.x;
            const size_t k = k0 < ntot ? k0 : ntot - 1;
            dv[u] = STATS ? dinv[k] : (T)1;
            xv[u] = x[k];
            pv[u] = p[k];
            rv[u] = r[k];
            qv[u] = q[k];
        }
#pragma unroll
        for (int u = 0; u < UPT; ++u) {
            const size_t k = base + (size_t)u * UT + threadIdx.x;
            // without STATS every entry is written: p and q are 0 where
            // inactive, so x and r keep their values there
            if (k < ntot && dv[u] > (T)0) {
                x[k] = xv[u] + a * pv[u];
                const T rn = rv[u] - a * qv[u];
                r[k] = rn;
                if (STATS) {
                    const T sv = dv[u] * rn;
                    const double rd = rn, sd = sv;
                    v[0] += rd * sd;
                    v[1] += sd;
                    v[2] += rd;
                    v[3] += rd * rd;
                }
            }
        }
    }
    if (STATS) put_partials<4, 0, UT>(g, v, pout, nblk);
}
template <class T, bool STATS = true>
__global__ __launch_bounds__(UT) void k_cg_update(size_t ntot, int nblk, const T *__restrict__ dinv,
                                                  T *__restrict__ x, T *__restrict__ r,
                                                  const T *__restrict__ p, const T *__restrict__ q,
                                                  CgState *st, int par, const double *pin, int nin, double *pout) {
    cg_update_body<T, STATS>(SoloGrid{}, ntot, nblk, dinv, x, r, p, q, st, par, pin, nin, pout);
}

// x += dx (float correction of an inner solve) over ntot entries.
template <class G>
__device__ __forceinline__ void add_correction_body(const G &g, size_t ntot, double *__restrict__ x,
                                                    const float *__restrict__ dx) {
    for (size_t k = (size_t)g.b() * NT + threadIdx.x; k < ntot; k += (size_t)g.n() * NT) x[k] += (double)dx[k];
}
__global__ __launch_bounds__(NT) void k_add_correction(size_t ntot, double *__restrict__ x,
                                                       const float *__restrict__ dx) {
    add_correction_body(SoloGrid{}, ntot, x, dx);
}

// ---------------------------------------------------------------------------
// multigrid V-cycle preconditioner for the Poisson solve.  Each coarse cell
// agglomerates 2x2 cells; the coarse face weight is half the sum of the two
// fine face weights it covers (for uncut cells this is the Laplacian
// rediscretised on the coarse grid); weighted-Jacobi smoothing; interpolation
// copies a coarse value to its active children and restriction is its
// transpose.  With equal numbers of pre- and post-smoothing sweeps the cycle
// is a symmetric positive definite operator, as the conjugate-gradient
// iteration requires.
// ---------------------------------------------------------------------------

// Factor on the interpolated coarse correction.  A constant factor keeps the
// cycle symmetric (pre- and post-smoothing are adjoint and restriction is the
// transpose of interpolation) and positive definite below 2.  Measured on the
// 2048x1024 channel: 1.0 needs 10 iterations per step, 0.9 needs 16 and 1.3
// needs 31 (the coarse operator's half-sum weights already scale the
// correction as a rediscretisation would).
constexpr double MG_CGC = 1.0;

// Weights of the two smoothing sweeps x' = x + w D^-1 (b - A x) on the way
// down (first w1, then w2) and on the way up (the same two).  Both sweeps are
// polynomials in D^-1 A, so they commute and the cycle stays symmetric
// whatever their order.  With w1 = w2 this is weighted Jacobi; two different
// weights are the degree-2 Chebyshev smoother on an interval [lo, 2] of the
// spectrum of D^-1 A (which lies in [0, 2] for these diagonally dominant
// operators): w = 1 / ((2 + lo) / 2 +- (2 - lo) / 2 cos(pi / 4)).  The
// default is weighted Jacobi at 0.8.  Chebyshev on [2/3, 2] takes 15.8
// Poisson iterations per FP64 step on the 4096x2048 NACA 0012 case against 17
// (the same 10 on the 2048x1024 channel), but where a pressure cell holds
// 2.5e-12 of a cell's volume and the mass matrix is not floored, its solve
// stops on r.z <= 0 at a relative residual of 1.3e-12, above the 1e-13 that
// weighted Jacobi reaches there.
#ifndef CCNS_MG_W1
#define CCNS_MG_W1 0.8
#endif
#ifndef CCNS_MG_W2
#define CCNS_MG_W2 0.8
#endif
constexpr double MG_W1 = CCNS_MG_W1, MG_W2 = CCNS_MG_W2;

// Fused cycle kernels.  Tiles cover the real cells, starting at cell (1, 1)
// so that every 2x2 group of children that forms a coarse cell lies inside
// one tile (64 = 32 coarse columns, 16 = 8 coarse rows).  One tile per
// work-group.  Values needed beyond the tile are recomputed on a one-cell
// ring (in LDS) instead of being exchanged through a second kernel.
constexpr int MTY = 16;
// Tile height of the cycle kernels on the coarser levels that would get
// fewer than MG_SMALL_GROUPS tiles of height MTY.
constexpr int MTY_SMALL = 4;
constexpr int MG_SMALL_GROUPS = 256;

// Kernel forms of a cycle level's down- and up-sweep kernels (the values of
// ccns_params.mg_forms): staged first sweep with the ring's operands in
// registers; the same with every operand of the ring in LDS; the first
// sweep formed pointwise on 64 x MTY tiles; the same on 64 x MTY_SMALL tiles;
// the LDS form on 64 x MTY/2 tiles.
enum MgForm {
    MGF_AUTO = 0, MGF_STAGED = 1, MGF_STAGED_LDS = 2, MGF_PLAIN = 3, MGF_PLAIN_SHORT = 4, MGF_STAGED_LDS_HALF = 5
};
constexpr int MG_FORM_BITS = 3, MG_FORM_LEVELS = 10;  // 6 bits (down, up) per level in a 64-bit word

struct MgTile {
    int c0, r0;  // first real cell of the tile
};
template <class G>
__device__ inline MgTile mg_tile(const G &g, int gx, int ty = MTY) {
    const int L = logical_group(g, ((g.n() + 7) / 8) * 8);
    MgTile t;
    t.c0 = 1 + (L % gx) * TX;
    t.r0 = 1 + (L / gx) * ty;
    return t;
}

// Forms of k_mg_down and k_mg_up for a level large enough to be bound by
// HBM bandwidth rather than by latency (the finest): the first sweep's input
// is staged in LDS on a two-cell ring, so each value is loaded once per tile
// instead of being formed at the five points of every stencil.  Same
// arithmetic per cell as the forms below.
constexpr int MH = 2;  // halo width of the staged first sweep
constexpr int MW = TX + 2 * MH, MHt = MTY + 2 * MH;

// Stencil operands of one cell of the tile phase (the residual of k_mg_down,
// the last sweep of k_mg_up): 1/diag, right-hand side and the four face
// weights.  They do not depend on the sweep before, so every thread loads
// its cells' operands at the start of the kernel and the loads overlap the
// first phase.
template <class T, int R>
struct MgCellOps {
    T d[R], b[R], e[R], w[R], n[R], s[R];
};
template <class T, int R>
__device__ inline void mg_load_tile_ops(MgCellOps<T, R> &o, const PoisCoefT<T> &c, const T *b, int nx, int ny, int P,
                                        const MgTile &t) {
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
#pragma unroll
    for (int m = 0; m < R; ++m) {
        const int j = t.r0 + ty + 4 * m, i = t.c0 + tx;
        const bool in = (j <= ny) && (i <= nx);
        const size_t k = in ? (size_t)j * P + i : 0;
        o.d[m] = c.dinv[k];
        o.b[m] = b[k];
        o.e[m] = c.cx[k];
        o.w[m] = c.cx[in ? k - 1 : 0];
        o.n[m] = c.cy[k];
        o.s[m] = c.cy[in ? k - P : 0];
    }
}

// Every phase of these kernels issues all of its thread's loads before the
// first use (the loop over the phase's cells is unrolled into a loop of loads
// and a loop of arithmetic), and the loads of the next phase are issued
// before the barrier that ends this one: a work-group then waits for one
// memory round trip per phase instead of one per cell it handles.
constexpr int MS1 = MHt * MW, MI1 = (MS1 + NT - 1) / NT;                  // 2-ring region
constexpr int MS2 = (MTY + 2) * (TX + 2), MI2 = (MS2 + NT - 1) / NT;      // 1-ring region
template <class T>
struct MgRingOps {
    T d[MI2], b[MI2], e[MI2], w[MI2], n[MI2], s[MI2];
};
// Operands of the 1-ring region's cells (entry q of this thread: cell e =
// threadIdx.x + q NT of the (MTY+2) x (TX+2) region).
template <class T>
__device__ inline void mg_load_ring_ops(MgRingOps<T> &o, const PoisCoefT<T> &c, const T *b, int nx, int ny, int P,
                                        const MgTile &t) {
#pragma unroll
    for (int q = 0; q < MI2; ++q) {
        const int e = threadIdx.x + q * NT;
        const int ly = e / (TX + 2), lx = e - ly * (TX + 2);
        const int j = t.r0 - 1 + ly, i = t.c0 - 1 + lx;
        const bool in = (e < MS2) && (j >= 1) && (j <= ny) && (i >= 1) && (i <= nx);
        const size_t k = in ? (size_t)j * P + i : 0;
        o.d[q] = c.dinv[k];
        o.b[q] = b[k];
        o.e[q] = c.cx[k];
        o.w[q] = c.cx[in ? k - 1 : 0];
        o.n[q] = c.cy[k];
        o.s[q] = c.cy[in ? k - P : 0];
    }
}
// The sweep x' = x + omega D^-1 (b - A x) on the 1-ring region, x read from
// the 2-ring array s1, written to the 1-ring array s2.
template <class T>
__device__ inline void mg_ring_sweep(const MgRingOps<T> &o, const T (*s1)[MW], T (*s2)[TX + 2], int nx, int ny,
                                     const MgTile &t, T omega) {
#pragma unroll
    for (int q = 0; q < MI2; ++q) {
        const int e = threadIdx.x + q * NT;
        if (e < MS2) {
            const int ly = e / (TX + 2), lx = e - ly * (TX + 2);
            const int j = t.r0 - 1 + ly, i = t.c0 - 1 + lx;
            const bool in = (j >= 1) && (j <= ny) && (i >= 1) && (i <= nx);
            const T ce = o.e[q], cw = o.w[q], cn = o.n[q], cs = o.s[q], dv = o.d[q];
            const int y = ly + 1, x = lx + 1;  // position in s1
            const T xv = s1[y][x];
            const T Ax = (ce + cw + cn + cs) * xv - ce * s1[y][x + 1] - cw * s1[y][x - 1] - cn * s1[y + 1][x] -
                         cs * s1[y - 1][x];
            s2[ly][lx] = (in && dv > (T)0) ? xv + omega * dv * (o.b[q] - Ax) : (T)0;
        }
    }
}

// Two weighted-Jacobi sweeps from a zero guess, the residual, and its
// restriction: x2 (written to x2out) and b_coarse.
template <class T, class G>
__device__ __forceinline__ void mg_down_staged_body(const G &g, int nx, int ny, int P, int gx, PoisCoefT<T> c,
                                                const T *__restrict__ b, T *__restrict__ x2out,
                                                int Pc, int nxc, int nyc, const T *__restrict__ dinvc,
                                                T *__restrict__ bc, const int *done) {
    if (*done) return;
    __shared__ T s1[MHt][MW];            // first sweep on the 2-ring region
    __shared__ T s2[MTY + 2][TX + 2];    // second sweep on the 1-ring region
    __shared__ T sr[MTY][TX];            // residual on the tile
    const MgTile t = mg_tile(g, gx);
    if (t.r0 > ny || t.c0 > nx) return;
    {
        T dv[MI1], bv[MI1];
#pragma unroll
        for (int q = 0; q < MI1; ++q) {
            const int e = threadIdx.x + q * NT;
            const int ly = e / MW, lx = e - ly * MW;
            const int j = t.r0 - MH + ly, i = t.c0 - MH + lx;
            const bool in = (e < MS1) && (j >= 0) && (j <= ny + 1) && (i >= 0) && (i <= nx + 1);
            const size_t k = in ? (size_t)j * P + i : 0;
            dv[q] = c.dinv[k];
            bv[q] = b[k];
        }
#pragma unroll
        for (int q = 0; q < MI1; ++q) {
            const int e = threadIdx.x + q * NT;
            if (e < MS1) {
                const int ly = e / MW, lx = e - ly * MW;
                const int j = t.r0 - MH + ly, i = t.c0 - MH + lx;
                const bool in = (j >= 0) && (j <= ny + 1) && (i >= 0) && (i <= nx + 1);
                s1[ly][lx] = (in && dv[q] > (T)0) ? (T)MG_W1 * dv[q] * bv[q] : (T)0;
            }
        }
    }
    MgRingOps<T> ro;
    mg_load_ring_ops<T>(ro, c, b, nx, ny, P, t);
    __syncthreads();
    mg_ring_sweep<T>(ro, s1, s2, nx, ny, t, (T)MG_W2);
    MgCellOps<T, MTY / 4> o;
    mg_load_tile_ops<T, MTY / 4>(o, c, b, nx, ny, P, t);
    // one coarse cell per thread for the restriction: 32 x 8 coarse cells per tile
    const int cxl = threadIdx.x & 31, cyl = threadIdx.x >> 5;
    const int I = (t.c0 + 1) / 2 + cxl, J = (t.r0 + 1) / 2 + cyl;
    const bool cin = (I <= nxc) && (J <= nyc);
    const size_t kc = cin ? (size_t)J * Pc + I : 0;
    const T dcv = dinvc[kc];
    __syncthreads();
    {
        const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
#pragma unroll
        for (int m = 0; m < MTY / 4; ++m) {
            const int ly = ty + 4 * m;
            const int j = t.r0 + ly, i = t.c0 + tx;
            const bool in = (j <= ny) && (i <= nx);
            const int y = ly + 1, x = tx + 1;
            const T xv = s2[y][x];
            const T Ax = (o.e[m] + o.w[m] + o.n[m] + o.s[m]) * xv - o.e[m] * s2[y][x + 1] -
                         o.w[m] * s2[y][x - 1] - o.n[m] * s2[y + 1][x] - o.s[m] * s2[y - 1][x];
            sr[ly][tx] = (in && o.d[m] > (T)0) ? o.b[m] - Ax : (T)0;
            if (in) x2out[(size_t)j * P + i] = xv;
        }
    }
    __syncthreads();
    if (cin) {
        const T sum = (sr[2 * cyl][2 * cxl] + sr[2 * cyl][2 * cxl + 1]) +
                      (sr[2 * cyl + 1][2 * cxl] + sr[2 * cyl + 1][2 * cxl + 1]);
        bc[kc] = dcv > (T)0 ? sum : (T)0;
    }
}
template <class T>
__global__ __launch_bounds__(NT) void k_mg_down_staged(int nx, int ny, int P, int gx, PoisCoefT<T> c,
                                                const T *__restrict__ b, T *__restrict__ x2out,
                                                int Pc, int nxc, int nyc, const T *__restrict__ dinvc,
                                                T *__restrict__ bc, const int *done) {
    mg_down_staged_body<T>(SoloGrid{}, nx, ny, P, gx, c, b, x2out, Pc, nxc, nyc, dinvc, bc, done);
}

// The coarse correction interpolated onto x2, then two weighted-Jacobi
// sweeps: z.  With STATS, partials of (b.z, z, b, b.b).
template <class T, bool STATS, class G>
__device__ __forceinline__ void mg_up_staged_body(const G &g, int nx, int ny, int P, int gx, PoisCoefT<T> c, const T *__restrict__ b,
                                              const T *__restrict__ x2, const T *__restrict__ xc, int Pc,
                                              T *__restrict__ z, double *pout, int nblk, const int *done) {
    if (*done) return;
    __shared__ T s1[MHt][MW];
    __shared__ T s2[MTY + 2][TX + 2];
    const MgTile t = mg_tile(g, gx);
    double v[4] = {0, 0, 0, 0};
    const bool live = !(t.r0 > ny || t.c0 > nx);
    MgCellOps<T, MTY / 4> o;
    if (live) {
        T dv[MI1], xv[MI1], ec[MI1];
#pragma unroll
        for (int q = 0; q < MI1; ++q) {
            const int e = threadIdx.x + q * NT;
            const int ly = e / MW, lx = e - ly * MW;
            const int j = t.r0 - MH + ly, i = t.c0 - MH + lx;
            const bool in = (e < MS1) && (j >= 1) && (j <= ny) && (i >= 1) && (i <= nx);
            const size_t k = in ? (size_t)j * P + i : 0;
            const size_t kc = in ? (size_t)((j + 1) >> 1) * Pc + ((i + 1) >> 1) : 0;
            dv[q] = c.dinv[k];
            xv[q] = x2[k];
            ec[q] = xc[kc];
        }
#pragma unroll
        for (int q = 0; q < MI1; ++q) {
            const int e = threadIdx.x + q * NT;
            if (e < MS1) {
                const int ly = e / MW, lx = e - ly * MW;
                const int j = t.r0 - MH + ly, i = t.c0 - MH + lx;
                const bool in = (j >= 1) && (j <= ny) && (i >= 1) && (i <= nx);
                s1[ly][lx] = (in && dv[q] > (T)0) ? xv[q] + (T)MG_CGC * ec[q] : (T)0;
            }
        }
        MgRingOps<T> ro;
        mg_load_ring_ops<T>(ro, c, b, nx, ny, P, t);
        __syncthreads();
        mg_ring_sweep<T>(ro, s1, s2, nx, ny, t, (T)MG_W1);
        mg_load_tile_ops<T, MTY / 4>(o, c, b, nx, ny, P, t);
    } else {
        __syncthreads();
    }
    __syncthreads();
    if (live) {
        const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
#pragma unroll
        for (int m = 0; m < MTY / 4; ++m) {
            const int ly = ty + 4 * m;
            const int j = t.r0 + ly, i = t.c0 + tx;
            const bool in = (j <= ny) && (i <= nx);
            const int y = ly + 1, x = tx + 1;
            const T xv = s2[y][x];
            const T Ax = (o.e[m] + o.w[m] + o.n[m] + o.s[m]) * xv - o.e[m] * s2[y][x + 1] -
                         o.w[m] * s2[y][x - 1] - o.n[m] * s2[y + 1][x] - o.s[m] * s2[y - 1][x];
            const T zv = (in && o.d[m] > (T)0) ? xv + (T)MG_W2 * o.d[m] * (o.b[m] - Ax) : (T)0;
            if (in) z[(size_t)j * P + i] = zv;
            if (STATS && in) {
                const double bd = o.b[m], zd = zv;
                v[0] += bd * zd;
                v[1] += zd;
                v[2] += bd;
                v[3] += bd * bd;
            }
        }
    }
    if (STATS) put_partials<4>(g, v, pout, nblk);
}
template <class T, bool STATS>
__global__ __launch_bounds__(NT) void k_mg_up_staged(int nx, int ny, int P, int gx, PoisCoefT<T> c, const T *__restrict__ b,
                                              const T *__restrict__ x2, const T *__restrict__ xc, int Pc,
                                              T *__restrict__ z, double *pout, int nblk, const int *done) {
    mg_up_staged_body<T, STATS>(SoloGrid{}, nx, ny, P, gx, c, b, x2, xc, Pc, z, pout, nblk, done);
}

// The staged forms with every operand of the tile's two-cell ring (1/diag,
// b, c^x, c^y) loaded once into LDS: the ring sweep and the tile phase read
// their stencil weights from there instead of loading them again.  Same
// arithmetic, in the same order, as the forms above.  Tiles of 64 x TY
// cells: TY = MTY takes 64 KB of LDS in FP64 (two work-groups per compute
// unit), TY = MTY / 2 about 38 KB (four), with more ring per tile cell.
template <int TY>
struct LdsTile {
    static constexpr int Ht = TY + 2 * MH;                                  // rows of the 2-ring region
    static constexpr int S1 = Ht * MW, I1 = (S1 + NT - 1) / NT;             // 2-ring region
    static constexpr int S2 = (TY + 2) * (TX + 2), I2 = (S2 + NT - 1) / NT;  // 1-ring region
};
template <class T, int TY>
__device__ inline void mg_stage_ops(T (*sd)[MW], T (*sb)[MW], T (*se)[MW], T (*sn)[MW], const PoisCoefT<T> &c,
                                    const T *b, int nx, int ny, int P, const MgTile &t, T dv[LdsTile<TY>::I1], T bv[LdsTile<TY>::I1]) {
    T ev[LdsTile<TY>::I1], nv[LdsTile<TY>::I1];
#pragma unroll
    for (int q = 0; q < LdsTile<TY>::I1; ++q) {
        const int e = threadIdx.x + q * NT;
        const int ly = e / MW, lx = e - ly * MW;
        const int j = t.r0 - MH + ly, i = t.c0 - MH + lx;
        const bool in = (e < LdsTile<TY>::S1) && (j >= 0) && (j <= ny + 1) && (i >= 0) && (i <= nx + 1);
        const size_t k = in ? (size_t)j * P + i : 0;
        dv[q] = c.dinv[k];
        bv[q] = b[k];
        ev[q] = c.cx[k];
        nv[q] = c.cy[k];
    }
#pragma unroll
    for (int q = 0; q < LdsTile<TY>::I1; ++q) {
        const int e = threadIdx.x + q * NT;
        if (e < LdsTile<TY>::S1) {
            const int ly = e / MW, lx = e - ly * MW;
            const int j = t.r0 - MH + ly, i = t.c0 - MH + lx;
            const bool in = (j >= 0) && (j <= ny + 1) && (i >= 0) && (i <= nx + 1);
            sd[ly][lx] = in ? dv[q] : (T)0;
            sb[ly][lx] = in ? bv[q] : (T)0;
            se[ly][lx] = in ? ev[q] : (T)0;
            sn[ly][lx] = in ? nv[q] : (T)0;
        }
    }
}

// The sweep of mg_ring_sweep with the weights read from the staged arrays.
template <class T, int TY>
__device__ inline void mg_ring_sweep_lds(const T (*sd)[MW], const T (*sb)[MW], const T (*se)[MW], const T (*sn)[MW],
                                         const T (*s1)[MW], T (*s2)[TX + 2], int nx, int ny, const MgTile &t,
                                         T omega) {
#pragma unroll
    for (int q = 0; q < LdsTile<TY>::I2; ++q) {
        const int e = threadIdx.x + q * NT;
        if (e < LdsTile<TY>::S2) {
            const int ly = e / (TX + 2), lx = e - ly * (TX + 2);
            const int j = t.r0 - 1 + ly, i = t.c0 - 1 + lx;
            const bool in = (j >= 1) && (j <= ny) && (i >= 1) && (i <= nx);
            const int y = ly + 1, x = lx + 1;  // position in the two-ring arrays
            const T ce = se[y][x], cw = se[y][x - 1], cn = sn[y][x], cs = sn[y - 1][x], dv = sd[y][x];
            const T xv = s1[y][x];
            const T Ax = (ce + cw + cn + cs) * xv - ce * s1[y][x + 1] - cw * s1[y][x - 1] - cn * s1[y + 1][x] -
                         cs * s1[y - 1][x];
            s2[ly][lx] = (in && dv > (T)0) ? xv + omega * dv * (sb[y][x] - Ax) : (T)0;
        }
    }
}

template <class T, int TY, class G>
__device__ __forceinline__ void mg_down_lds_body(const G &g, int nx, int ny, int P, int gx, PoisCoefT<T> c,
                                                    const T *__restrict__ b, T *__restrict__ x2out, int Pc, int nxc,
                                                    int nyc, const T *__restrict__ dinvc, T *__restrict__ bc,
                                                    const int *done) {
    if (*done) return;
    __shared__ T sd[LdsTile<TY>::Ht][MW], sb[LdsTile<TY>::Ht][MW], se[LdsTile<TY>::Ht][MW], sn[LdsTile<TY>::Ht][MW];
    __shared__ T s1[LdsTile<TY>::Ht][MW];            // first sweep; then the residual on the tile
    __shared__ T s2[TY + 2][TX + 2];    // second sweep on the 1-ring region
    const MgTile t = mg_tile(g, gx, TY);
    if (t.r0 > ny || t.c0 > nx) return;
    {
        T dv[LdsTile<TY>::I1], bv[LdsTile<TY>::I1];
        mg_stage_ops<T, TY>(sd, sb, se, sn, c, b, nx, ny, P, t, dv, bv);
#pragma unroll
        for (int q = 0; q < LdsTile<TY>::I1; ++q) {
            const int e = threadIdx.x + q * NT;
            if (e < LdsTile<TY>::S1) {
                const int ly = e / MW, lx = e - ly * MW;
                const int j = t.r0 - MH + ly, i = t.c0 - MH + lx;
                const bool in = (j >= 0) && (j <= ny + 1) && (i >= 0) && (i <= nx + 1);
                s1[ly][lx] = (in && dv[q] > (T)0) ? (T)MG_W1 * dv[q] * bv[q] : (T)0;
            }
        }
    }
    // one coarse cell per thread for the restriction: 32 x 8 coarse cells per tile
    const int cxl = threadIdx.x & 31, cyl = threadIdx.x >> 5;
    const int I = (t.c0 + 1) / 2 + cxl, J = (t.r0 + 1) / 2 + cyl;
    const bool cin = (cyl < TY / 2) && (I <= nxc) && (J <= nyc);
    const size_t kc = cin ? (size_t)J * Pc + I : 0;
    const T dcv = dinvc[kc];
    __syncthreads();
    mg_ring_sweep_lds<T, TY>(sd, sb, se, sn, s1, s2, nx, ny, t, (T)MG_W2);
    __syncthreads();
    T (*sr)[TX] = reinterpret_cast<T (*)[TX]>(&s1[0][0]);
    {
        const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
#pragma unroll
        for (int m = 0; m < TY / 4; ++m) {
            const int ly = ty + 4 * m;
            const int j = t.r0 + ly, i = t.c0 + tx;
            const bool in = (j <= ny) && (i <= nx);
            const int y = ly + 1, x = tx + 1;          // in s2
            const int Y = ly + MH, X = tx + MH;        // in the two-ring arrays
            const T e = se[Y][X], w = se[Y][X - 1], n = sn[Y][X], so = sn[Y - 1][X];
            const T xv = s2[y][x];
            const T Ax = (e + w + n + so) * xv - e * s2[y][x + 1] - w * s2[y][x - 1] - n * s2[y + 1][x] -
                         so * s2[y - 1][x];
            sr[ly][tx] = (in && sd[Y][X] > (T)0) ? sb[Y][X] - Ax : (T)0;
            if (in) x2out[(size_t)j * P + i] = xv;
        }
    }
    __syncthreads();
    if (cin) {
        const T sum = (sr[2 * cyl][2 * cxl] + sr[2 * cyl][2 * cxl + 1]) +
                      (sr[2 * cyl + 1][2 * cxl] + sr[2 * cyl + 1][2 * cxl + 1]);
        bc[kc] = dcv > (T)0 ? sum : (T)0;
    }
}
template <class T, int TY>
__global__ __launch_bounds__(NT) void k_mg_down_lds(int nx, int ny, int P, int gx, PoisCoefT<T> c,
                                                    const T *__restrict__ b, T *__restrict__ x2out, int Pc, int nxc,
                                                    int nyc, const T *__restrict__ dinvc, T *__restrict__ bc,
                                                    const int *done) {
    mg_down_lds_body<T, TY>(SoloGrid{}, nx, ny, P, gx, c, b, x2out, Pc, nxc, nyc, dinvc, bc, done);
}

template <class T, bool STATS, int TY, class G>
__device__ __forceinline__ void mg_up_lds_body(const G &g, int nx, int ny, int P, int gx, PoisCoefT<T> c, const T *__restrict__ b,
                                                  const T *__restrict__ x2, const T *__restrict__ xc, int Pc,
                                                  T *__restrict__ z, double *pout, int nblk, const int *done) {
    if (*done) return;
    __shared__ T sd[LdsTile<TY>::Ht][MW], sb[LdsTile<TY>::Ht][MW], se[LdsTile<TY>::Ht][MW], sn[LdsTile<TY>::Ht][MW];
    __shared__ T s1[LdsTile<TY>::Ht][MW];
    __shared__ T s2[TY + 2][TX + 2];
    const MgTile t = mg_tile(g, gx, TY);
    double v[4] = {0, 0, 0, 0};
    const bool live = !(t.r0 > ny || t.c0 > nx);
    if (live) {
        T xv[LdsTile<TY>::I1], ec[LdsTile<TY>::I1];
#pragma unroll
        for (int q = 0; q < LdsTile<TY>::I1; ++q) {
            const int e = threadIdx.x + q * NT;
            const int ly = e / MW, lx = e - ly * MW;
            const int j = t.r0 - MH + ly, i = t.c0 - MH + lx;
            const bool in = (e < LdsTile<TY>::S1) && (j >= 1) && (j <= ny) && (i >= 1) && (i <= nx);
            const size_t k = in ? (size_t)j * P + i : 0;
            const size_t kc = in ? (size_t)((j + 1) >> 1) * Pc + ((i + 1) >> 1) : 0;
            xv[q] = x2[k];
            ec[q] = xc[kc];
        }
        T dv[LdsTile<TY>::I1], bv[LdsTile<TY>::I1];
        mg_stage_ops<T, TY>(sd, sb, se, sn, c, b, nx, ny, P, t, dv, bv);
#pragma unroll
        for (int q = 0; q < LdsTile<TY>::I1; ++q) {
            const int e = threadIdx.x + q * NT;
            if (e < LdsTile<TY>::S1) {
                const int ly = e / MW, lx = e - ly * MW;
                const int j = t.r0 - MH + ly, i = t.c0 - MH + lx;
                const bool in = (j >= 1) && (j <= ny) && (i >= 1) && (i <= nx);
                s1[ly][lx] = (in && dv[q] > (T)0) ? xv[q] + (T)MG_CGC * ec[q] : (T)0;
            }
        }
        __syncthreads();
        mg_ring_sweep_lds<T, TY>(sd, sb, se, sn, s1, s2, nx, ny, t, (T)MG_W1);
    } else {
        __syncthreads();
    }
    __syncthreads();
    if (live) {
        const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
#pragma unroll
        for (int m = 0; m < TY / 4; ++m) {
            const int ly = ty + 4 * m;
            const int j = t.r0 + ly, i = t.c0 + tx;
            const bool in = (j <= ny) && (i <= nx);
            const int y = ly + 1, x = tx + 1;
            const int Y = ly + MH, X = tx + MH;
            const T e = se[Y][X], w = se[Y][X - 1], n = sn[Y][X], so = sn[Y - 1][X], dd = sd[Y][X], bb = sb[Y][X];
            const T xv = s2[y][x];
            const T Ax = (e + w + n + so) * xv - e * s2[y][x + 1] - w * s2[y][x - 1] - n * s2[y + 1][x] -
                         so * s2[y - 1][x];
            const T zv = (in && dd > (T)0) ? xv + (T)MG_W2 * dd * (bb - Ax) : (T)0;
            if (in) z[(size_t)j * P + i] = zv;
            if (STATS && in) {
                const double bd = bb, zd = zv;
                v[0] += bd * zd;
                v[1] += zd;
                v[2] += bd;
                v[3] += bd * bd;
            }
        }
    }
    if (STATS) put_partials<4>(g, v, pout, nblk);
}
template <class T, bool STATS, int TY>
__global__ __launch_bounds__(NT) void k_mg_up_lds(int nx, int ny, int P, int gx, PoisCoefT<T> c, const T *__restrict__ b,
                                                  const T *__restrict__ x2, const T *__restrict__ xc, int Pc,
                                                  T *__restrict__ z, double *pout, int nblk, const int *done) {
    mg_up_lds_body<T, STATS, TY>(SoloGrid{}, nx, ny, P, gx, c, b, x2, xc, Pc, z, pout, nblk, done);
}

// Two weighted-Jacobi sweeps from a zero guess, the residual, and its
// restriction: x2 (written to x2out) and b_coarse.  The first sweep from
// zero is pointwise (x1 = omega D^-1 b), so it is formed at the five points
// of the second sweep's stencil instead of being staged: two phases with one
// barrier between the sweeps and the residual.  Tiles of TX x TY cells: TY =
// MTY, or MTY_SMALL on levels too small to give every compute unit a tile
// (there each work-group's serial chain of loads is what the launch waits
// for, and shorter tiles shorten it).
template <class T, int TY, class G>
__device__ __forceinline__ void mg_down_body(const G &g, int nx, int ny, int P, int gx, PoisCoefT<T> c,
                                                const T *__restrict__ b, T *__restrict__ x2out,
                                                int Pc, int nxc, int nyc, const T *__restrict__ dinvc,
                                                T *__restrict__ bc, const int *done) {
    if (*done) return;
    static_assert(TY % 4 == 0 && TY <= MTY, "tile rows: a multiple of the 4 row groups, at most MTY");
    __shared__ T s2[TY + 2][TX + 2];    // x after two sweeps, on the tile and a one-cell ring
    __shared__ T sr[TY][TX];            // residual on the tile
    const MgTile t = mg_tile(g, gx, TY);
    if (t.r0 > ny || t.c0 > nx) return;
    MgCellOps<T, TY / 4> o;
    mg_load_tile_ops<T, TY / 4>(o, c, b, nx, ny, P, t);
    // one coarse cell per thread for the restriction: 32 x (TY / 2) coarse
    // cells per tile
    const int cxl = threadIdx.x & 31, cyl = threadIdx.x >> 5;
    const int I = (t.c0 + 1) / 2 + cxl, J = (t.r0 + 1) / 2 + cyl;
    const bool cin = (cyl < TY / 2) && (I <= nxc) && (J <= nyc);
    const size_t kc = cin ? (size_t)J * Pc + I : 0;
    const T dcv = dinvc[kc];
    for (int e = threadIdx.x; e < (TY + 2) * (TX + 2); e += NT) {
        const int ly = e / (TX + 2), lx = e - ly * (TX + 2);
        const int j = t.r0 - 1 + ly, i = t.c0 - 1 + lx;
        const bool in = (j >= 1) && (j <= ny) && (i >= 1) && (i <= nx);
        // outside the real cells a stand-in cell whose neighbours exist
        const size_t k = in ? (size_t)j * P + i : (size_t)P + 1;
        const T dv = c.dinv[k], bv = b[k];
        const T de = c.dinv[k + 1], dw = c.dinv[k - 1], dn = c.dinv[k + P], ds = c.dinv[k - P];
        const T be = b[k + 1], bw = b[k - 1], bn = b[k + P], bs = b[k - P];
        const T ce = c.cx[k], cw = c.cx[k - 1], cn = c.cy[k], cs = c.cy[k - P];
        const T w1 = (T)MG_W1;
        const T xv = dv > (T)0 ? w1 * dv * bv : (T)0;
        const T xe = de > (T)0 ? w1 * de * be : (T)0, xw = dw > (T)0 ? w1 * dw * bw : (T)0;
        const T xn = dn > (T)0 ? w1 * dn * bn : (T)0, xs = ds > (T)0 ? w1 * ds * bs : (T)0;
        const T Ax = (ce + cw + cn + cs) * xv - ce * xe - cw * xw - cn * xn - cs * xs;
        s2[ly][lx] = (in && dv > (T)0) ? xv + (T)MG_W2 * dv * (bv - Ax) : (T)0;
    }
    __syncthreads();
    {
        const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
#pragma unroll
        for (int m = 0; m < TY / 4; ++m) {
            const int ly = ty + 4 * m;
            const int j = t.r0 + ly, i = t.c0 + tx;
            const bool in = (j <= ny) && (i <= nx);
            const int y = ly + 1, x = tx + 1;
            const T xv = s2[y][x];
            const T Ax = (o.e[m] + o.w[m] + o.n[m] + o.s[m]) * xv - o.e[m] * s2[y][x + 1] -
                         o.w[m] * s2[y][x - 1] - o.n[m] * s2[y + 1][x] - o.s[m] * s2[y - 1][x];
            sr[ly][tx] = (in && o.d[m] > (T)0) ? o.b[m] - Ax : (T)0;
            if (in) x2out[(size_t)j * P + i] = xv;
        }
    }
    __syncthreads();
    if (cin) {
        const T sum = (sr[2 * cyl][2 * cxl] + sr[2 * cyl][2 * cxl + 1]) +
                      (sr[2 * cyl + 1][2 * cxl] + sr[2 * cyl + 1][2 * cxl + 1]);
        bc[kc] = dcv > (T)0 ? sum : (T)0;
    }
}
template <class T, int TY = MTY>
__global__ __launch_bounds__(NT) void k_mg_down(int nx, int ny, int P, int gx, PoisCoefT<T> c,
                                                const T *__restrict__ b, T *__restrict__ x2out,
                                                int Pc, int nxc, int nyc, const T *__restrict__ dinvc,
                                                T *__restrict__ bc, const int *done) {
    mg_down_body<T, TY>(SoloGrid{}, nx, ny, P, gx, c, b, x2out, Pc, nxc, nyc, dinvc, bc, done);
}

// The coarse correction interpolated onto x2, then two weighted-Jacobi
// sweeps: z.  With STATS, partials of (b.z, z, b, b.b).  The interpolated
// start value is pointwise, so it is formed at the five points of the first
// sweep's stencil instead of being staged: one barrier, between the sweeps.
// Tiles of TX x TY cells, as in k_mg_down.
template <class T, bool STATS, int TY, class G>
__device__ __forceinline__ void mg_up_body(const G &g, int nx, int ny, int P, int gx, PoisCoefT<T> c, const T *__restrict__ b,
                                              const T *__restrict__ x2, const T *__restrict__ xc, int Pc,
                                              T *__restrict__ z, double *pout, int nblk, const int *done) {
    if (*done) return;
    static_assert(TY % 4 == 0 && TY <= MTY, "tile rows: a multiple of the 4 row groups, at most MTY");
    __shared__ T s2[TY + 2][TX + 2];    // x after the first sweep, on the tile and a one-cell ring
    const MgTile t = mg_tile(g, gx, TY);
    double v[4] = {0, 0, 0, 0};
    const bool live = !(t.r0 > ny || t.c0 > nx);
    MgCellOps<T, TY / 4> o;
    if (live) {
        mg_load_tile_ops<T, TY / 4>(o, c, b, nx, ny, P, t);
        // start value x2 + interpolated correction at cell (j, i): 0 outside
        // the real cells and at inactive ones
        auto start = [&](int j, int i, size_t k) -> T {
            const bool in = (j >= 1) && (j <= ny) && (i >= 1) && (i <= nx);
            const size_t kk = in ? k : 0;
            const size_t kc = in ? (size_t)((j + 1) >> 1) * Pc + ((i + 1) >> 1) : 0;
            const T dv = c.dinv[kk], xv = x2[kk], ec = xc[kc];
            return (in && dv > (T)0) ? xv + (T)MG_CGC * ec : (T)0;
        };
        for (int e = threadIdx.x; e < (TY + 2) * (TX + 2); e += NT) {
            const int ly = e / (TX + 2), lx = e - ly * (TX + 2);
            const int j = t.r0 - 1 + ly, i = t.c0 - 1 + lx;
            const bool in = (j >= 1) && (j <= ny) && (i >= 1) && (i <= nx);
            const size_t k = in ? (size_t)j * P + i : (size_t)P + 1;
            const int jj = in ? j : 1, ii = in ? i : 1;
            const T dv = c.dinv[k], bv = b[k];
            const T ce = c.cx[k], cw = c.cx[k - 1], cn = c.cy[k], cs = c.cy[k - P];
            const T xv = start(jj, ii, k);
            const T xe = start(jj, ii + 1, k + 1), xw = start(jj, ii - 1, k - 1);
            const T xn = start(jj + 1, ii, k + P), xs = start(jj - 1, ii, k - P);
            const T Ax = (ce + cw + cn + cs) * xv - ce * xe - cw * xw - cn * xn - cs * xs;
            s2[ly][lx] = (in && dv > (T)0) ? xv + (T)MG_W1 * dv * (bv - Ax) : (T)0;
        }
    }
    __syncthreads();
    if (live) {
        const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
#pragma unroll
        for (int m = 0; m < TY / 4; ++m) {
            const int ly = ty + 4 * m;
            const int j = t.r0 + ly, i = t.c0 + tx;
            const bool in = (j <= ny) && (i <= nx);
            const int y = ly + 1, x = tx + 1;
            const T xv = s2[y][x];
            const T Ax = (o.e[m] + o.w[m] + o.n[m] + o.s[m]) * xv - o.e[m] * s2[y][x + 1] -
                         o.w[m] * s2[y][x - 1] - o.n[m] * s2[y + 1][x] - o.s[m] * s2[y - 1][x];
            const T zv = (in && o.d[m] > (T)0) ? xv + (T)MG_W2 * o.d[m] * (o.b[m] - Ax) : (T)0;
            if (in) z[(size_t)j * P + i] = zv;
            if (STATS && in) {
                const double bd = o.b[m], zd = zv;
                v[0] += bd * zd;
                v[1] += zd;
                v[2] += bd;
                v[3] += bd * bd;
            }
        }
    }
    if (STATS) put_partials<4>(g, v, pout, nblk);
}
template <class T, bool STATS, int TY = MTY>
__global__ __launch_bounds__(NT) void k_mg_up(int nx, int ny, int P, int gx, PoisCoefT<T> c, const T *__restrict__ b,
                                              const T *__restrict__ x2, const T *__restrict__ xc, int Pc,
                                              T *__restrict__ z, double *pout, int nblk, const int *done) {
    mg_up_body<T, STATS, TY>(SoloGrid{}, nx, ny, P, gx, c, b, x2, xc, Pc, z, pout, nblk, done);
}

// The coarse end of the cycle in one work-group of TT threads: every level
// from the tail's first down to the coarsest and back, one phase after the
// other with work-group barriers between them (the levels are a few thousand
// cells: one launch instead of two per level, each of which would be a
// latency-bound launch of a few work-groups).  The arithmetic and its order
// per cell are those of k_mg_down, k_mg_coarsest and k_mg_up.  The level
// arrays stay in global memory (L2); within one work-group a barrier makes
// the global writes of one phase visible to the next.
constexpr int TT = 1024;
constexpr int MAX_TAIL = 10;
template <class T>
struct TailLevel {
    const T *cx, *cy, *dinv;
    T *b, *x, *xt;
    int nx, ny, P;
};
template <class T>
struct TailDesc {
    TailLevel<T> lv[MAX_TAIL];
    int nlev;            // levels of the tail, the last one the coarsest
    int ncoarse;         // unknowns of the coarsest grid
    const int *idx;
    const double *pinv;
    const int *done;     // the solve's done flag: nothing to do once set
    int lofs[MAX_TAIL];  // k_mg_tail_lds: offset of each level's arrays in LDS (elements)
    T *out;              // k_mg_tail_lds: where the tail's first level's result goes
};

template <class T>
__device__ inline T tail_Ax(const TailLevel<T> &L, const T *v, size_t k) {
    const T ce = L.cx[k], cw = L.cx[k - 1], cn = L.cy[k], cs = L.cy[k - L.P];
    return (ce + cw + cn + cs) * v[k] - ce * v[k + 1] - cw * v[k - 1] - cn * v[k + L.P] - cs * v[k - L.P];
}

template <class T>
__device__ __forceinline__ void mg_tail_body(const TailDesc<T> &d) {
    if (*d.done) return;
    const T w1 = (T)MG_W1, w2 = (T)MG_W2;
    // down: two sweeps from zero, the residual restricted to the next level
    for (int l = 0; l + 1 < d.nlev; ++l) {
        const TailLevel<T> &L = d.lv[l];
        const TailLevel<T> &C = d.lv[l + 1];
        const int ncell = L.nx * L.ny;
        for (int e = threadIdx.x; e < ncell; e += TT) {
            const size_t k = (size_t)(e / L.nx + 1) * L.P + (e % L.nx + 1);
            const T dv = L.dinv[k], bv = L.b[k];
            L.xt[k] = dv > (T)0 ? w1 * dv * bv : (T)0;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < ncell; e += TT) {
            const size_t k = (size_t)(e / L.nx + 1) * L.P + (e % L.nx + 1);
            const T dv = L.dinv[k], bv = L.b[k];
            const T xv = L.xt[k];
            L.x[k] = dv > (T)0 ? xv + w2 * dv * (bv - tail_Ax(L, L.xt, k)) : (T)0;
        }
        __syncthreads();
        const int nc = C.nx * C.ny;
        for (int e = threadIdx.x; e < nc; e += TT) {
            const int I = e % C.nx + 1, J = e / C.nx + 1;
            T r[2][2];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int bb = 0; bb < 2; ++bb) {
                    const int j = 2 * J - 1 + a, i = 2 * I - 1 + bb;
                    T rv = (T)0;
                    if (j <= L.ny && i <= L.nx) {
                        const size_t k = (size_t)j * L.P + i;
                        const T dv = L.dinv[k];
                        if (dv > (T)0) rv = L.b[k] - tail_Ax(L, L.x, k);
                    }
                    r[a][bb] = rv;
                }
            const size_t kc = (size_t)J * C.P + I;
            const T sum = (r[0][0] + r[0][1]) + (r[1][0] + r[1][1]);
            C.b[kc] = C.dinv[kc] > (T)0 ? sum : (T)0;
        }
        __syncthreads();
    }
    // coarsest: x = A^+ b with the dense pseudo-inverse
    {
        const TailLevel<T> &L = d.lv[d.nlev - 1];
        __shared__ double sb[1024];
        for (int i = threadIdx.x; i < d.ncoarse; i += TT) sb[i] = L.b[d.idx[i]];
        __syncthreads();
        for (int i = threadIdx.x; i < d.ncoarse; i += TT) {
            double acc = 0.0;
            for (int j2 = 0; j2 < d.ncoarse; ++j2) acc += d.pinv[(size_t)i * d.ncoarse + j2] * sb[j2];
            L.x[d.idx[i]] = (T)acc;
        }
        __syncthreads();
    }
    // up: the coarse correction interpolated onto x2, then two sweeps
    for (int l = d.nlev - 2; l >= 0; --l) {
        const TailLevel<T> &L = d.lv[l];
        const TailLevel<T> &C = d.lv[l + 1];
        const T *xc = (l + 2 == d.nlev) ? C.x : C.xt;
        const int ncell = L.nx * L.ny;
        for (int e = threadIdx.x; e < ncell; e += TT) {
            const int i = e % L.nx + 1, j = e / L.nx + 1;
            const size_t k = (size_t)j * L.P + i;
            const size_t kc = (size_t)((j + 1) >> 1) * C.P + ((i + 1) >> 1);
            const T dv = L.dinv[k], xv = L.x[k], ec = xc[kc];
            L.xt[k] = dv > (T)0 ? xv + (T)MG_CGC * ec : (T)0;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < ncell; e += TT) {
            const size_t k = (size_t)(e / L.nx + 1) * L.P + (e % L.nx + 1);
            const T dv = L.dinv[k], bv = L.b[k];
            const T xv = L.xt[k];
            L.x[k] = dv > (T)0 ? xv + w1 * dv * (bv - tail_Ax(L, L.xt, k)) : (T)0;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < ncell; e += TT) {
            const size_t k = (size_t)(e / L.nx + 1) * L.P + (e % L.nx + 1);
            const T dv = L.dinv[k], bv = L.b[k];
            const T xv = L.x[k];
            L.xt[k] = dv > (T)0 ? xv + w2 * dv * (bv - tail_Ax(L, L.x, k)) : (T)0;
        }
        __syncthreads();
    }
}
template <class T>
__global__ __launch_bounds__(TT) void k_mg_tail(TailDesc<T> d) {
    mg_tail_body<T>(d);
}

// The coarse end of the cycle as k_mg_tail, with every level's arrays (the
// coefficients, b, x and xt, in compact (nx+2) x (ny+2) rows) held in LDS:
// each phase then waits for LDS instead of L2.  The levels are loaded once;
// the result of the tail's first level is written to d.out.  Same arithmetic
// per cell as k_mg_tail; the interpolated start value and the first sweep on
// the way up, and the two sweeps from zero on the way down, are formed in one
// phase each (the start values at the five points of the stencil).
template <class T>
__device__ inline T lds_Ax(const T *cx, const T *cy, const T *v, int k, int W) {
    const T ce = cx[k], cw = cx[k - 1], cn = cy[k], cs = cy[k - W];
    return (ce + cw + cn + cs) * v[k] - ce * v[k + 1] - cw * v[k - 1] - cn * v[k + W] - cs * v[k - W];
}

template <class T>
__device__ __forceinline__ void mg_tail_lds_body(const TailDesc<T> &d) {
    if (*d.done) return;
    extern __shared__ double tail_lds[];
    T *const sm = reinterpret_cast<T *>(tail_lds);
    const T w1 = (T)MG_W1, w2 = (T)MG_W2;
    // level l's six arrays start at sm + d.lofs[l], each (nx+2)(ny+2) long
    auto arr = [&](int l, int a) { return sm + d.lofs[l] + a * (d.lv[l].nx + 2) * (d.lv[l].ny + 2); };
    for (int l = 0; l < d.nlev; ++l) {
        const TailLevel<T> &L = d.lv[l];
        const int W = L.nx + 2, n = W * (L.ny + 2);
        T *cx = arr(l, 0), *cy = arr(l, 1), *dv = arr(l, 2), *b = arr(l, 3), *x = arr(l, 4), *xt = arr(l, 5);
        // TL entries per thread at a time, every load issued before the
        // first store
        constexpr int TL = 4;
        for (int e0 = 0; e0 < n; e0 += TL * TT) {
            T vcx[TL], vcy[TL], vdv[TL], vb[TL];
#pragma unroll
            for (int u = 0; u < TL; ++u) {
                const int e = e0 + u * TT + threadIdx.x;
                const int ee = e < n ? e : 0;
                const int j = ee / W, i = ee - j * W;
                const size_t k = (size_t)j * L.P + i;
                vcx[u] = L.cx[k];
                vcy[u] = L.cy[k];
                vdv[u] = L.dinv[k];
                vb[u] = l == 0 ? L.b[k] : (T)0;
            }
#pragma unroll
            for (int u = 0; u < TL; ++u) {
                const int e = e0 + u * TT + threadIdx.x;
                if (e < n) {
                    cx[e] = vcx[u];
                    cy[e] = vcy[u];
                    dv[e] = vdv[u];
                    b[e] = vb[u];
                    x[e] = (T)0;
                    xt[e] = (T)0;
                }
            }
        }
    }
    __syncthreads();
    // down: two sweeps from zero (the first formed at the stencil's points),
    // then the residual restricted to the next level
    for (int l = 0; l + 1 < d.nlev; ++l) {
        const TailLevel<T> &L = d.lv[l];
        const int W = L.nx + 2;
        const T *cx = arr(l, 0), *cy = arr(l, 1), *dv = arr(l, 2), *b = arr(l, 3);
        T *x = arr(l, 4);
        const int ncell = L.nx * L.ny;
        auto x1 = [&](int k) { return dv[k] > (T)0 ? w1 * dv[k] * b[k] : (T)0; };
        for (int e = threadIdx.x; e < ncell; e += TT) {
            const int k = (e / L.nx + 1) * W + (e % L.nx + 1);
            const T ce = cx[k], cw = cx[k - 1], cn = cy[k], cs = cy[k - W];
            const T xv = x1(k);
            const T Ax = (ce + cw + cn + cs) * xv - ce * x1(k + 1) - cw * x1(k - 1) - cn * x1(k + W) - cs * x1(k - W);
            x[k] = dv[k] > (T)0 ? xv + w2 * dv[k] * (b[k] - Ax) : (T)0;
        }
        __syncthreads();
        const TailLevel<T> &C = d.lv[l + 1];
        const int Wc = C.nx + 2;
        const T *dvc = arr(l + 1, 2);
        T *bc = arr(l + 1, 3);
        const int nc = C.nx * C.ny;
        for (int e = threadIdx.x; e < nc; e += TT) {
            const int I = e % C.nx + 1, J = e / C.nx + 1;
            T r[2][2];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int bb = 0; bb < 2; ++bb) {
                    const int j = 2 * J - 1 + a, i = 2 * I - 1 + bb;
                    T rv = (T)0;
                    if (j <= L.ny && i <= L.nx) {
                        const int k = j * W + i;
                        if (dv[k] > (T)0) rv = b[k] - lds_Ax(cx, cy, x, k, W);
                    }
                    r[a][bb] = rv;
                }
            const int kc = J * Wc + I;
            const T sum = (r[0][0] + r[0][1]) + (r[1][0] + r[1][1]);
            bc[kc] = dvc[kc] > (T)0 ? sum : (T)0;
        }
        __syncthreads();
    }
    // coarsest: x = A^+ b with the dense pseudo-inverse (global, L2).  Eight
    // threads per row: thread s of a row sums the columns s, s+8, s+16, ...
    // in order, with CL loads in flight at a time; the row's eight partial
    // sums are then combined by lane exchanges (a fixed order).
    {
        const int l = d.nlev - 1;
        const TailLevel<T> &L = d.lv[l];
        const int W = L.nx + 2;
        const T *b = arr(l, 3);
        T *x = arr(l, 4);
        __shared__ double sb[1024];
        const int n = d.ncoarse;
        for (int i = threadIdx.x; i < n; i += TT) {
            const int k = d.idx[i];
            sb[i] = b[(k / L.P) * W + k % L.P];
        }
        __syncthreads();
        constexpr int CL = 16;
        const int sl = threadIdx.x & 7;
        for (int i0 = 0; i0 < n; i0 += TT / 8) {
            const int i = i0 + (threadIdx.x >> 3);
            const bool row = i < n;
            const double *prow = d.pinv + (size_t)(row ? i : 0) * n;
            double acc = 0.0;
            for (int c0 = sl; c0 < n; c0 += 8 * CL) {
                double a[CL];
#pragma unroll
                for (int u = 0; u < CL; ++u) {
                    const int c = c0 + 8 * u;
                    a[u] = prow[c < n ? c : 0];
                }
#pragma unroll
                for (int u = 0; u < CL; ++u) {
                    const int c = c0 + 8 * u;
                    if (c < n) acc += a[u] * sb[c];
                }
            }
            acc += __shfl_xor(acc, 1);
            acc += __shfl_xor(acc, 2);
            acc += __shfl_xor(acc, 4);
            if (row && sl == 0) {
                const int k = d.idx[i];
                x[(k / L.P) * W + k % L.P] = (T)acc;
            }
        }
        __syncthreads();
    }
    // up: the interpolated start value and the first sweep (into xt), then
    // the second sweep (into x)
    for (int l = d.nlev - 2; l >= 0; --l) {
        const TailLevel<T> &L = d.lv[l];
        const TailLevel<T> &C = d.lv[l + 1];
        const int W = L.nx + 2, Wc = C.nx + 2;
        const T *cx = arr(l, 0), *cy = arr(l, 1), *dv = arr(l, 2), *b = arr(l, 3), *xcs = arr(l + 1, 4);
        T *x = arr(l, 4), *xt = arr(l, 5);
        const int ncell = L.nx * L.ny;
        auto start = [&](int j, int i) {
            const bool in = (j >= 1) && (j <= L.ny) && (i >= 1) && (i <= L.nx);
            const int k = in ? j * W + i : 0;
            const int kc = in ? ((j + 1) >> 1) * Wc + ((i + 1) >> 1) : 0;
            return (in && dv[k] > (T)0) ? x[k] + (T)MG_CGC * xcs[kc] : (T)0;
        };
        for (int e = threadIdx.x; e < ncell; e += TT) {
            const int j = e / L.nx + 1, i = e % L.nx + 1;
            const int k = j * W + i;
            const T ce = cx[k], cw = cx[k - 1], cn = cy[k], cs = cy[k - W];
            const T xv = start(j, i);
            const T Ax = (ce + cw + cn + cs) * xv - ce * start(j, i + 1) - cw * start(j, i - 1) -
                         cn * start(j + 1, i) - cs * start(j - 1, i);
            xt[k] = dv[k] > (T)0 ? xv + w1 * dv[k] * (b[k] - Ax) : (T)0;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < ncell; e += TT) {
            const int k = (e / L.nx + 1) * W + (e % L.nx + 1);
            x[k] = dv[k] > (T)0 ? xt[k] + w2 * dv[k] * (b[k] - lds_Ax(cx, cy, xt, k, W)) : (T)0;
        }
        __syncthreads();
    }
    // the tail's first level's result to global memory (interior cells)
    {
        const TailLevel<T> &L = d.lv[0];
        const int W = L.nx + 2;
        const T *x = arr(0, 4);
        for (int e = threadIdx.x; e < L.nx * L.ny; e += TT) {
            const int j = e / L.nx + 1, i = e % L.nx + 1;
            d.out[(size_t)j * L.P + i] = x[j * W + i];
        }
    }
}
template <class T>
__global__ __launch_bounds__(TT) void k_mg_tail_lds(TailDesc<T> d) {
    mg_tail_lds_body<T>(d);
}

// One work-group sums the partials of a producer into a single group's worth
// (so that consumers read N values instead of N per producer group).
template <int NS, int NM, int BT>
__device__ __forceinline__ void reduce_partials_body(const double *pin, int nin, double *pout) {
    double t[NS + NM];
    get_totals<NS, NM, BT>(pin, nin, t);
    if (threadIdx.x < NS + NM) pout[threadIdx.x] = t[threadIdx.x];
}
template <int NS, int NM = 0, int BT = NT>
__global__ __launch_bounds__(BT) void k_reduce_partials(const double *pin, int nin, double *pout) {
    reduce_partials_body<NS, NM, BT>(pin, nin, pout);
}

// G work-groups sum the partials of a producer into G sets (group g takes
// the producers' groups [g nin / G, (g+1) nin / G)), stored slot-major for a
// consumer that sums G values per slot.  Spreads a large reduction over
// several compute units instead of one.
template <int NS, class G>
__device__ __forceinline__ void reduce_partials_split_body(const G &g, const double *pin, int nin, double *pout) {
    const int ng = g.n(), ig = g.b();
    const int lo = (int)((long)ig * nin / ng), hi = (int)((long)(ig + 1) * nin / ng);
    double a[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) a[k] = 0.0;
    for (int b = lo + threadIdx.x; b < hi; b += NT) {
#pragma unroll
        for (int k = 0; k < NS; ++k) a[k] += pin[(size_t)k * nin + b];
    }
    double t[NS];
    block_reduce<NS, 0>(a, t);
    if (threadIdx.x < NS) pout[(size_t)threadIdx.x * ng + ig] = t[threadIdx.x];
}
template <int NS>
__global__ __launch_bounds__(NT) void k_reduce_partials_split(const double *pin, int nin, double *pout) {
    reduce_partials_split_body<NS>(SoloGrid{}, pin, nin, pout);
}
constexpr int PRED_RED = 16;  // groups of the predictor CG's partial reduction

// Coarsest grid: x = A^+ b with the dense pseudo-inverse on the n unknowns.
template <class T>
__device__ __forceinline__ void mg_coarsest_body(int n, const int *__restrict__ idx,
                                                    const double *__restrict__ pinv, const T *__restrict__ b,
                                                    T *__restrict__ x, const int *done) {
    if (*done) return;
    __shared__ double sb[1024];
    for (int i = threadIdx.x; i < n; i += NT) sb[i] = b[idx[i]];
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += NT) {
        double acc = 0.0;
        for (int j2 = 0; j2 < n; ++j2) acc += pinv[(size_t)i * n + j2] * sb[j2];
        x[idx[i]] = (T)acc;
    }
}
template <class T>
__global__ __launch_bounds__(NT) void k_mg_coarsest(int n, const int *__restrict__ idx,
                                                    const double *__restrict__ pinv, const T *__restrict__ b,
                                                    T *__restrict__ x, const int *done) {
    mg_coarsest_body<T>(n, idx, pinv, b, x, done);
}

// Direction and operator for the multigrid-preconditioned solve:
// p = (z - mean z) + beta p_old; q = A p.  Consumes the statistics written by
// the last smoothing sweep (b.z, z, b, b.b) and, on the first iteration, |f|^2
// from init (pinit; without it, the norm of the cycle's input b is taken).
template <class T, class G>
__device__ __forceinline__ void pois_dir_z_body(const G &g, Dims d, PoisCoefT<T> pc, const T *__restrict__ z,
                                                   const T *__restrict__ pold, T *__restrict__ pnew,
                                                   T *__restrict__ q, CgState *st, int first, int par,
                                                   const double *pin, int nin, const double *pinit, int ninit,
                                                   double *pout) {
    if (st->done) return;
    double t[4];
    get_totals<4>(pin, nin, t);
    double fn2;
    if (first) {
        if (pinit) {
            double f[1];
            get_totals<1>(pinit, ninit, f);
            fn2 = f[0];
        } else {
            fn2 = t[3];
        }
    } else {
        fn2 = st->fnorm2;
    }
    const DirStep ds = cg_decide(g, st, first, par, fn2, t[0], t[1], t[2], t[3]);
    if (ds.stop) return;
    const T beta = (T)ds.beta, m = (T)ds.mean;
    __shared__ T sp[PTY + 2][TX + 2];
    const int P = d.pitch;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    double v[1] = {0.0};
    // every load of a phase is issued before its first use, and the tile
    // phase's operands before the barrier (as in the staged cycle kernels)
    constexpr int NS = (PTY + 2) * (TX + 2), IS = (NS + NT - 1) / NT, R = PTY / 4;
    for_tiles(g, d, [&](int, int c0, int r0) {
        {
            T di[IS], zv[IS], po[IS];
#pragma unroll
            for (int u = 0; u < IS; ++u) {
                const int e = threadIdx.x + u * NT;
                const int ly = e / (TX + 2), lx = e - ly * (TX + 2);
                const int j = r0 - 1 + ly, i = c0 - 1 + lx;
                const bool in = (e < NS) && (j >= 0) && (j < d.rows) && (i >= 0) && (i < P);
                const size_t k = in ? (size_t)j * P + i : 0;
                di[u] = pc.dinv[k];
                zv[u] = z[k];
                po[u] = first ? (T)0 : pold[k];
            }
#pragma unroll
            for (int u = 0; u < IS; ++u) {
                const int e = threadIdx.x + u * NT;
                if (e < NS) {
                    const int ly = e / (TX + 2), lx = e - ly * (TX + 2);
                    const int j = r0 - 1 + ly, i = c0 - 1 + lx;
                    const bool in = (j >= 0) && (j < d.rows) && (i >= 0) && (i < P);
                    sp[ly][lx] = (in && di[u] > (T)0) ? (zv[u] - m) + beta * po[u] : (T)0;
                }
            }
        }
        const int i = c0 + tx;
        T dv[R], ce[R], cw[R], cn[R], cs[R];
#pragma unroll
        for (int u = 0; u < R; ++u) {
            const int j = r0 + ty + 4 * u;
            const bool in = j < d.rows;
            const size_t k = in ? (size_t)j * P + i : 0;
            const size_t kw = in && i > 0 ? k - 1 : k, ks = in && j > 0 ? k - P : k;
            dv[u] = pc.dinv[k], ce[u] = pc.cx[k], cw[u] = pc.cx[kw], cn[u] = pc.cy[k], cs[u] = pc.cy[ks];
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < R; ++u) {
            const int lj = ty + 4 * u;
            const int j = r0 + lj;
            if (j < d.rows) {
                const size_t k = (size_t)j * P + i;
                const T pcv = sp[lj + 1][tx + 1];
                T qv = (ce[u] + cw[u] + cn[u] + cs[u]) * pcv - ce[u] * sp[lj + 1][tx + 2] - cw[u] * sp[lj + 1][tx] -
                       cn[u] * sp[lj + 2][tx + 1] - cs[u] * sp[lj][tx + 1];
                qv = dv[u] > (T)0 ? qv : (T)0;
                pnew[k] = pcv;
                q[k] = qv;
                v[0] += (double)pcv * (double)qv;
            }
        }
        __syncthreads();
    });
    put_partials<1>(g, v, pout, d.nblk);
}
template <class T>
__global__ __launch_bounds__(NT) void k_pois_dir_z(Dims d, PoisCoefT<T> pc, const T *__restrict__ z,
                                                   const T *__restrict__ pold, T *__restrict__ pnew,
                                                   T *__restrict__ q, CgState *st, int first, int par,
                                                   const double *pin, int nin, const double *pinit, int ninit,
                                                   double *pout) {
    pois_dir_z_body<T>(SoloGrid{}, d, pc, z, pold, pnew, q, st, first, par, pin, nin, pinit, ninit, pout);
}

// ---------------------------------------------------------------------------
// predictor (eq:pm_prediction): H = (rho/tau) V - mu visc(strain(., 0))
// ---------------------------------------------------------------------------

// Predictor kernels work on tiles of 64 x 8 faces of both velocity
// components per work-group, staged in LDS with a one-face halo.  The float
// CG of the inner solves of precision 1 takes tiles of 64 x 16 faces: its
// launch waits on the same chain of dependent loads per tile as the FP64
// one for half the bytes per face, so taller tiles put more of them in
// flight per chain.
constexpr int HTY = 8;
constexpr int HTY_F32 = 16;
template <class T>
__device__ __host__ constexpr int pred_rows() {
    return std::is_same<T, double>::value ? HTY : HTY_F32;
}

// LDS of a predictor tile of TH rows: the staged face field on the tile and
// a one-face halo, and its node strains (eq:offdiag).  The cell strains
// (eq:diag) are formed where a face needs them, which keeps the tile at
// 20 KB in FP64.
template <class T, int TH = HTY>
struct PredTileNx {
    T spx[TH + 2][TX + 2], spy[TH + 2][TX + 2];
    T snx[TH + 1][TX + 1], sny[TH + 1][TX + 1];
};

// The strains of the staged field (rows r0-1 .. r0+HTY, cols c0-1 .. c0+TX
// staged in spx, spy).  GEO: the node weights are the symmetric geometric form
// (cross weight = sqrt of the product of the two diagonal ones), so the cross
// weights are formed instead of read.
//
// The strain arithmetic of the predictor tiles, shared by the kernels that
// read the coefficient arrays and those that read the class table.  Every
// product that meets a sum is written as an explicit fused multiply-add, so
// the compiler has no contraction left to choose and both paths round alike.
//   cell strain   w (e v_e - b v_w)                       (eq:diag)
//   node strains  gx = bn v_n - bs v_s, gy = be u_e - bw u_w,
//                 S = (a gx + b gy) / 2, (c gx + d gy) / 2  (eq:offdiag)
//   face term     B^aa (S_+ - S_-) + B^ab (N_+ - N_-)      (eq:divD)
template <class T>
__device__ inline T strain_cell(T w, T e, T b, T ve, T vw) {
    return w * fma(e, ve, -(b * vw));
}
template <class T>
__device__ inline void strain_node(T bxn, T bxs, T bye, T byw, T a, T b, T cc, T dd, T pn, T ps, T qe, T qw, T &snx,
                                   T &sny) {
    const T gxv = fma(bxn, pn, -(bxs * ps));
    const T gyv = fma(bye, qe, -(byw * qw));
    snx = (T)0.5 * fma(a, gxv, b * gyv);
    sny = (T)0.5 * fma(cc, gxv, dd * gyv);
}
template <class T>
__device__ inline T strain_face(T baa, T sp, T sm, T bab, T np, T nm) {
    return fma(baa, sp - sm, bab * (np - nm));
}

// Node strains of the tile (eq:offdiag) from the coefficient arrays: nodes
// (r0 - 1 .. r0 + TH - 1) x (c0 - 1 .. c0 + TX - 1).
template <class T, bool GEO, int TH>
__device__ inline void pred_tile_strains(PredTileNx<T, TH> &s, const ViscCoefT<T> &c, int P, int rows, int c0,
                                         int r0) {
    for (int e = threadIdx.x; e < (TH + 1) * (TX + 1); e += NT) {
        const int ly = e / (TX + 1), lx = e - ly * (TX + 1);
        const int j = r0 - 1 + ly, i = c0 - 1 + lx;
        const bool in = (j >= 0) && (j + 1 < rows) && (i >= 0) && (i + 1 < P);
        const size_t k = in ? (size_t)j * P + i : 0;
        const T bxn = c.bxy[k + P], bxs = c.bxy[k], bye = c.byx[k + 1], byw = c.byx[k];
        const T a = c.nxx[k], dd = c.nyy[k];
        T b, cc;
        if (GEO) {
            b = cc = sqrt(a * dd);
        } else {
            b = c.nxy[k];
            cc = c.nyx[k];
        }
        T sx, sy;
        strain_node(bxn, bxs, bye, byw, a, b, cc, dd, s.spx[ly + 1][lx], s.spx[ly][lx], s.spy[ly][lx + 1],
                    s.spy[ly][lx], sx, sy);
        s.snx[ly][lx] = in ? sx : (T)0;
        s.sny[ly][lx] = in ? sy : (T)0;
    }
}

// K v = visc(strain(v, 0)) (Sec. 4.3) at tile entry (ly, tx), index k: the two
// cell strains S_xx of the x-face and S_yy of the y-face are formed here
// (eq:diag), the node strains come from the tile.
template <class T, int TH = HTY>
__device__ inline void pred_tile_K(const PredTileNx<T, TH> &s, const ViscCoefT<T> &c, size_t k, int ly, int tx, int i,
                                   int P, int rows, T &kx, T &ky) {
    const T bxx = c.bxx[k], bxy = c.bxy[k], byy = c.byy[k], byx = c.byx[k];
    const bool in0 = i >= 1, in1 = i + 1 < P;
    const size_t k0 = in0 ? k : 1, k1 = in1 ? k + 1 : 1;
    const T w0 = c.wxx[k0], e0 = c.bxx[k0], b0 = c.bxx[k0 - 1];
    const T w1 = c.wxx[k1], e1 = c.bxx[k1], b1 = c.bxx[k1 - 1];
    const T s0 = in0 ? strain_cell(w0, e0, b0, s.spx[ly + 1][tx + 1], s.spx[ly + 1][tx]) : (T)0;
    const T s1 = in1 ? strain_cell(w1, e1, b1, s.spx[ly + 1][tx + 2], s.spx[ly + 1][tx + 1]) : (T)0;
    kx = strain_face(bxx, s1, s0, bxy, s.snx[ly + 1][tx + 1], s.snx[ly][tx + 1]);
    // the y-face's two cell strains S_yy (cells j and j + 1 of column i)
    const int j = (int)(k / (size_t)P);
    const bool iny0 = j >= 1, iny1 = j + 1 < rows;
    const size_t q0 = iny0 ? k : (size_t)P, q1 = iny1 ? k + P : (size_t)P;
    const T wy0 = c.wyy[q0], n0 = c.byy[q0], m0 = c.byy[q0 - P];
    const T wy1 = c.wyy[q1], n1 = c.byy[q1], m1 = c.byy[q1 - P];
    const T t0 = iny0 ? strain_cell(wy0, n0, m0, s.spy[ly + 1][tx + 1], s.spy[ly][tx + 1]) : (T)0;
    const T t1 = iny1 ? strain_cell(wy1, n1, m1, s.spy[ly + 2][tx + 1], s.spy[ly + 1][tx + 1]) : (T)0;
    ky = strain_face(byy, t1, t0, byx, s.sny[ly + 1][tx + 1], s.sny[ly + 1][tx]);
}

// Node strain at tile node (ly, lx) (node (r0 - 1 + ly, c0 - 1 + lx)) from the
// node's row of the class table: the operations of pred_tile_strains.
template <class T, bool GEO, int TH = HTY>
__device__ inline void pred_node_strain_row(PredTileNx<T, TH> &s, const T *row, int ly, int lx, bool in) {
    const T bxn = row[PR_BXY_N], bxs = row[PR_BXY], bye = row[PR_BYX_E], byw = row[PR_BYX];
    const T a = row[PR_NXX], dd = row[PR_NYY];
    T b, cc;
    if (GEO) {
        b = cc = sqrt(a * dd);
    } else {
        b = row[PR_NXY];
        cc = row[PR_NYX];
    }
    T sx, sy;
    strain_node(bxn, bxs, bye, byw, a, b, cc, dd, s.spx[ly + 1][lx], s.spx[ly][lx], s.spy[ly][lx + 1],
                s.spy[ly][lx], sx, sy);
    s.snx[ly][lx] = in ? sx : (T)0;
    s.sny[ly][lx] = in ? sy : (T)0;
}

// The same with the values from the entry's row of the class table (where a
// neighbour is outside the grid the strain is 0, as above).
template <class T, int TH = HTY>
__device__ inline void pred_tile_K_row(const PredTileNx<T, TH> &s, const T *row, size_t k, int ly, int tx, int i, int P,
                                       int rows, T &kx, T &ky) {
    const T bxx = row[PR_BXX], bxy = row[PR_BXY], byy = row[PR_BYY], byx = row[PR_BYX];
    const bool in0 = i >= 1, in1 = i + 1 < P;
    const T w0 = row[PR_WXX], b0 = row[PR_BXX_W];
    const T w1 = row[PR_WXX_E], e1 = row[PR_BXX_E];
    const T s0 = in0 ? strain_cell(w0, bxx, b0, s.spx[ly + 1][tx + 1], s.spx[ly + 1][tx]) : (T)0;
    const T s1 = in1 ? strain_cell(w1, e1, bxx, s.spx[ly + 1][tx + 2], s.spx[ly + 1][tx + 1]) : (T)0;
    kx = strain_face(bxx, s1, s0, bxy, s.snx[ly + 1][tx + 1], s.snx[ly][tx + 1]);
    const int j = (int)(k / (size_t)P);
    const bool iny0 = j >= 1, iny1 = j + 1 < rows;
    const T wy0 = row[PR_WYY], m0 = row[PR_BYY_S];
    const T wy1 = row[PR_WYY_N], n1 = row[PR_BYY_N];
    const T t0 = iny0 ? strain_cell(wy0, byy, m0, s.spy[ly + 1][tx + 1], s.spy[ly][tx + 1]) : (T)0;
    const T t1 = iny1 ? strain_cell(wy1, n1, byy, s.spy[ly + 2][tx + 1], s.spy[ly + 1][tx + 1]) : (T)0;
    ky = strain_face(byy, t1, t0, byx, s.sny[ly + 1][tx + 1], s.sny[ly + 1][tx]);
}

// Predictor CG with one launch per iteration (Jacobi-preconditioned CG on
// H x = f, Sec. 4.3; M = inverse of H's diagonal).  Launch `it` receives the
// partial sums of launch it-1, reduced to a few sets: p.q, q.Mr, q.Mq, q.r,
// q.q, r.Mr and r.r of iteration it-1.  From them, identically in every
// group:
//   alpha = r.Mr / p.q,
//   r'.Mr' = r.Mr - 2 alpha q.Mr + alpha^2 q.Mq   (r' = r - alpha q),
//   r'.r'  = r.r  - 2 alpha q.r  + alpha^2 q.q,
//   beta = r'.Mr' / r.Mr, and the stopping test on r'.r'.
// Every product is summed afresh from the current vectors, so the expansion
// carries no error from one iteration to the next.  On its tile the launch
// then applies the update of iteration it-1 (x += alpha p_old, r' = r -
// alpha q), stages p = M r' + beta p_old on the tile and a one-face halo,
// forms the strains and H p, and writes r', p, H p with the seven partial
// products of the next launch.  Launch 0 starts from the residual kernel's
// statistics (f.f, r.Mr, -, -, r.r) with beta = 0 and no update.  r, p and
// H p alternate between two buffers (the halo of the old value is read while
// the new one is written); x is updated in place (tile only).  Launches
// after the one that stopped return at once (stop_it).  The tile keeps no
// cell strains (20 KB of LDS in FP64) and the register budget is set for
// seven waves per SIMD (70 VGPRs, no spills): the launch is bound by HBM
// latency, and more resident waves hide more of it.  Tiles are 64 x 8 faces
// in FP64 and 64 x 16 in float (pred_rows).  With CLS the coefficients come
// from the class table (pc.cls, pc.tab).
template <class T, bool GEO, bool CLS, class G>
__device__ __forceinline__ void pred_cg_body(const G &g, 
    int P, int rows, int gx, int gy, size_t n, PredCoefT<T> pc, CgState *st, int it, T *__restrict__ x,
    const T *__restrict__ rin, T *__restrict__ rout, const T *__restrict__ pold, T *__restrict__ pnew,
    const T *__restrict__ qin, T *__restrict__ qout, const double *tin, int nin, double *part) {
    constexpr int TH = pred_rows<T>();  // tile rows
    if (st->stop_it < it) return;
    double fn2, rr, alpha = 0.0, beta = 0.0;
    bool breakdown = false;
    if (it == 0) {
        double t[5];
        get_totals<5>(tin, nin, t);
        fn2 = t[0];
        rr = t[4];
    } else {
        double t[7];
        get_totals<7>(tin, nin, t);
        fn2 = st->fnorm2;
        breakdown = !(t[0] > 0.0 && t[0] < INFINITY && t[5] > 0.0 && t[5] < INFINITY);
        alpha = breakdown ? 0.0 : t[5] / t[0];
        const double rz = t[5] - 2.0 * alpha * t[1] + alpha * alpha * t[2];
        rr = t[6] - 2.0 * alpha * t[3] + alpha * alpha * t[4];
        beta = breakdown ? 0.0 : rz / t[5];
    }
    // an unconverged residual or a beta that is not finite (or a negative
    // beta) ends the solve as a breakdown; a NaN never counts as converged
    const bool conv = !breakdown && rr <= st->tol2 * fn2;
    if (!conv && !(rr < INFINITY && beta >= 0.0 && beta < INFINITY)) breakdown = true;
    const bool stop = breakdown || conv || it >= st->maxit;
    if (g.b() == 0 && threadIdx.x == 0) {
        if (it == 0) st->fnorm2 = fn2;
        if (stop) {
            st->done = 1;
            st->status = conv ? 0 : (breakdown ? CCNS_EBREAKDOWN : CCNS_ENOTCONV);
            st->it_final = breakdown ? max(it - 1, 0) : it;
            st->rnorm2_final = rr;
            st->stop_it = it;
        }
    }
    const int L = logical_group(g, ((g.n() + 7) / 8) * 8);
    const bool live = L < gx * gy;
    const int c0 = (L % gx) * TX, r0 = (L / gx) * TH;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const T a = (T)alpha, b = (T)beta;
    if (stop) {
        // the last update, x += alpha p_old, on the tile
        if (live && it >= 1 && !breakdown) {
            for (int ly = ty; ly < TH; ly += 4) {
                const int j = r0 + ly, i = c0 + tx;
                if (j >= rows) break;
                const size_t k = (size_t)j * P + i;
                const T ox = pold[k], oy = pold[n + k];
                x[k] = x[k] + a * ox;
                x[n + k] = x[n + k] + a * oy;
            }
        }
        return;
    }
    __shared__ PredTileNx<T, TH> s;
    double v[7] = {0, 0, 0, 0, 0, 0, 0};
    // r' and M^-1 of this thread's tile faces stay in registers for the
    // products of the last phase (rows ty, ty + 4, ... of the tile)
    constexpr int RW = TH / 4;
    T rxs[RW], rys[RW], hxs[RW], hys[RW];
    int cl[RW];
    // the Jacobi diagonal at entry k
    auto jacobi = [&](size_t k, T &hx, T &hy, int &ck) {
        if constexpr (CLS) {
            ck = pc.cls[k];
            const T *row = pc.tab + (size_t)ck * PCW;
            hx = row[PR_HDX];
            hy = row[PR_HDY];
        } else {
            hx = pc.hdx[k];
            hy = pc.hdy[k];
        }
    };
    if (live) {
        // the tile: r', x += alpha p_old, p = M r' + beta p_old
#pragma unroll
        for (int m = 0; m < RW; ++m) {
            const int ly = ty + 4 * m;
            const int j = r0 + ly, i = c0 + tx;
            const bool in = j < rows;
            const size_t k = in ? (size_t)j * P + i : 0;
            T hx, hy;
            jacobi(k, hx, hy, cl[m]);
            T rx = rin[k], ry = rin[n + k];
            T px = hx * rx, py = hy * ry;
            if (it >= 1) {
                const T qx = qin[k], qy = qin[n + k], ox = pold[k], oy = pold[n + k];
                rx = rx - a * qx;
                ry = ry - a * qy;
                px = hx * rx + b * ox;
                py = hy * ry + b * oy;
                if (in) {
                    x[k] = x[k] + a * ox;
                    x[n + k] = x[n + k] + a * oy;
                }
            }
            rxs[m] = rx;
            rys[m] = ry;
            hxs[m] = hx;
            hys[m] = hy;
            s.spx[ly + 1][tx + 1] = in ? px : (T)0;
            s.spy[ly + 1][tx + 1] = in ? py : (T)0;
        }
        // the one-face halo: rows r0-1 and r0+TH (TX+2 faces each), columns
        // c0-1 and c0+TX (TH faces each)
        for (int e = threadIdx.x; e < 2 * (TX + 2) + 2 * TH; e += NT) {
            int ly, lx;
            if (e < 2 * (TX + 2)) {
                ly = e < TX + 2 ? 0 : TH + 1;
                lx = e < TX + 2 ? e : e - (TX + 2);
            } else {
                const int f = e - 2 * (TX + 2);
                ly = 1 + (f >> 1);
                lx = (f & 1) ? TX + 1 : 0;
            }
            const int j = r0 - 1 + ly, i = c0 - 1 + lx;
            const bool in = (j >= 0) && (j < rows) && (i >= 0) && (i < P);
            const size_t k = in ? (size_t)j * P + i : 0;
            T hx, hy;
            int ck;
            jacobi(k, hx, hy, ck);
            T rx = rin[k], ry = rin[n + k];
            T px = hx * rx, py = hy * ry;
            if (it >= 1) {
                const T qx = qin[k], qy = qin[n + k], ox = pold[k], oy = pold[n + k];
                rx = rx - a * qx;
                ry = ry - a * qy;
                px = hx * rx + b * ox;
                py = hy * ry + b * oy;
            }
            s.spx[ly][lx] = in ? px : (T)0;
            s.spy[ly][lx] = in ? py : (T)0;
        }
    }
    __syncthreads();
    if (live) {
        if constexpr (CLS) {
            // node strains: the nodes at this thread's own entries, whose class
            // rows it already indexes, then the tile's first row and column of
            // nodes
#pragma unroll
            for (int m = 0; m < RW; ++m) {
                const int ly = ty + 4 * m;
                const int j = r0 + ly, i = c0 + tx;
                pred_node_strain_row<T, GEO>(s, pc.tab + (size_t)cl[m] * PCW, ly + 1, tx + 1,
                                             (j + 1 < rows) && (i + 1 < P));
            }
            for (int e = threadIdx.x; e < TX + 1 + TH; e += NT) {
                const int ly = e <= TX ? 0 : e - TX, lx = e <= TX ? e : 0;
                const int j = r0 - 1 + ly, i = c0 - 1 + lx;
                const bool in = (j >= 0) && (j + 1 < rows) && (i >= 0) && (i + 1 < P);
                const size_t k = in ? (size_t)j * P + i : 0;
                pred_node_strain_row<T, GEO>(s, pc.tab + (size_t)pc.cls[k] * PCW, ly, lx, in);
            }
        } else {
            pred_tile_strains<T, GEO>(s, pc.vc, P, rows, c0, r0);
        }
    }
    __syncthreads();
    if (live) {
        const T rt = (T)pc.rt, mu = (T)pc.mu;
#pragma unroll
        for (int m = 0; m < RW; ++m) {
            const int ly = ty + 4 * m;
            const int j = r0 + ly, i = c0 + tx;
            if (j >= rows) break;
            const size_t k = (size_t)j * P + i;
            T vu, vv, kx, ky;
            if constexpr (CLS) {
                const T *row = pc.tab + (size_t)cl[m] * PCW;
                vu = row[PR_VU];
                vv = row[PR_VV];
                pred_tile_K_row<T>(s, row, k, ly, tx, i, P, rows, kx, ky);
            } else {
                vu = pc.vu[k];
                vv = pc.vv[k];
                pred_tile_K<T>(s, pc.vc, k, ly, tx, i, P, rows, kx, ky);
            }
            const T rx = rxs[m], ry = rys[m], hx = hxs[m], hy = hys[m];
            const T px = s.spx[ly + 1][tx + 1], py = s.spy[ly + 1][tx + 1];
            const T qx = vu > (T)0 ? rt * vu * px - mu * kx : (T)0;
            const T qy = vv > (T)0 ? rt * vv * py - mu * ky : (T)0;
            const T pxo = vu > (T)0 ? px : (T)0, pyo = vv > (T)0 ? py : (T)0;
            if (it >= 1) {
                rout[k] = rx;
                rout[n + k] = ry;
            }
            pnew[k] = pxo;
            pnew[n + k] = pyo;
            qout[k] = qx;
            qout[n + k] = qy;
            const T zrx = hx * rx, zry = hy * ry, zqx = hx * qx, zqy = hy * qy;
            const double dqx = qx, dqy = qy, drx = rx, dry = ry;
            v[0] += (double)pxo * dqx + (double)pyo * dqy;
            v[1] += dqx * (double)zrx + dqy * (double)zry;
            v[2] += dqx * (double)zqx + dqy * (double)zqy;
            v[3] += dqx * drx + dqy * dry;
            v[4] += dqx * dqx + dqy * dqy;
            v[5] += drx * (double)zrx + dry * (double)zry;
            v[6] += drx * drx + dry * dry;
        }
    }
    put_partials<7>(g, v, part, g.n());
}
template <class T, bool GEO, bool CLS = false>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(7))) void k_pred_cg(
    int P, int rows, int gx, int gy, size_t n, PredCoefT<T> pc, CgState *st, int it, T *__restrict__ x,
    const T *__restrict__ rin, T *__restrict__ rout, const T *__restrict__ pold, T *__restrict__ pnew,
    const T *__restrict__ qin, T *__restrict__ qout, const double *tin, int nin, double *part) {
    pred_cg_body<T, GEO, CLS>(SoloGrid{}, P, rows, gx, gy, n, pc, st, it, x, rin, rout, pold, pnew, qin, qout, tin, nin, part);
}

// Predictor residual r = rhs - H x in FP64 on the tiles of k_pred_cg
// (x staged in LDS, masked to the unknowns), with the statistics of r.
//  MIX = false: r is stored; partials (f.f, r.z, z, r, r.r), z = M^-1 r.
//  MIX = true (precision 1): r is rounded to float into r32 (right-hand side
//  of the inner solve, whose start value x32 is cleared); partials
//  (r32.r32, r32.z, z, r32, r32.r32, f.f, r.r) with z = M32^-1 r32.
// With CLS the coefficients come from the class table, as in k_pred_cg.
template <bool MIX, bool GEO, bool CLS, class G>
__device__ __forceinline__ void pred_resid_body(const G &g, int P, int rows, int gx, int gy, size_t n, PredCoefT<double> pc,
                                                   const double *__restrict__ rhs, const double *__restrict__ xs,
                                                   double *__restrict__ r, CgState *st, double *pout,
                                                   float *__restrict__ r32, float *__restrict__ x32,
                                                   const float *__restrict__ hd32) {
    __shared__ PredTileNx<double> s;
    const int L = logical_group(g, ((g.n() + 7) / 8) * 8);
    const bool live = L < gx * gy;
    const int c0 = (L % gx) * TX, r0 = (L / gx) * HTY;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    double v[7] = {0, 0, 0, 0, 0, 0, 0};
    constexpr int RW = HTY / 4;
    int cl[RW];
    // face volumes at entry k (they mark the unknowns)
    auto volumes = [&](size_t k, double &mx, double &my, int &ck) {
        if constexpr (CLS) {
            ck = pc.cls[k];
            const double *row = pc.tab + (size_t)ck * PCW;
            mx = row[PR_VU];
            my = row[PR_VV];
        } else {
            mx = pc.vu[k];
            my = pc.vv[k];
        }
    };
    if (live) {
#pragma unroll
        for (int m = 0; m < RW; ++m) {
            const int ly = ty + 4 * m;
            const int j = r0 + ly, i = c0 + tx;
            const bool in = j < rows;
            const size_t k = in ? (size_t)j * P + i : 0;
            double mx, my;
            volumes(k, mx, my, cl[m]);
            const double ux = xs[k], uy = xs[n + k];
            s.spx[ly + 1][tx + 1] = (in && mx > 0.0) ? ux : 0.0;
            s.spy[ly + 1][tx + 1] = (in && my > 0.0) ? uy : 0.0;
        }
        // the one-face halo, as in k_pred_cg
        for (int e = threadIdx.x; e < 2 * (TX + 2) + 2 * HTY; e += NT) {
            int ly, lx;
            if (e < 2 * (TX + 2)) {
                ly = e < TX + 2 ? 0 : HTY + 1;
                lx = e < TX + 2 ? e : e - (TX + 2);
            } else {
                const int f = e - 2 * (TX + 2);
                ly = 1 + (f >> 1);
                lx = (f & 1) ? TX + 1 : 0;
            }
            const int j = r0 - 1 + ly, i = c0 - 1 + lx;
            const bool in = (j >= 0) && (j < rows) && (i >= 0) && (i < P);
            const size_t k = in ? (size_t)j * P + i : 0;
            double mx, my;
            int ck;
            volumes(k, mx, my, ck);
            const double ux = xs[k], uy = xs[n + k];
            s.spx[ly][lx] = (in && mx > 0.0) ? ux : 0.0;
            s.spy[ly][lx] = (in && my > 0.0) ? uy : 0.0;
        }
    }
    __syncthreads();
    if (live) {
        if constexpr (CLS) {
#pragma unroll
            for (int m = 0; m < RW; ++m) {
                const int ly = ty + 4 * m;
                const int j = r0 + ly, i = c0 + tx;
                pred_node_strain_row<double, GEO>(s, pc.tab + (size_t)cl[m] * PCW, ly + 1, tx + 1,
                                                  (j + 1 < rows) && (i + 1 < P));
            }
            for (int e = threadIdx.x; e < TX + 1 + HTY; e += NT) {
                const int ly = e <= TX ? 0 : e - TX, lx = e <= TX ? e : 0;
                const int j = r0 - 1 + ly, i = c0 - 1 + lx;
                const bool in = (j >= 0) && (j + 1 < rows) && (i >= 0) && (i + 1 < P);
                const size_t k = in ? (size_t)j * P + i : 0;
                pred_node_strain_row<double, GEO>(s, pc.tab + (size_t)pc.cls[k] * PCW, ly, lx, in);
            }
        } else {
            pred_tile_strains<double, GEO>(s, pc.vc, P, rows, c0, r0);
        }
    }
    __syncthreads();
    if (live) {
#pragma unroll
        for (int m = 0; m < RW; ++m) {
            const int ly = ty + 4 * m;
            const int j = r0 + ly, i = c0 + tx;
            if (j >= rows) break;
            const size_t k = (size_t)j * P + i;
            double kv[2], mv[2], hd[2];
            if constexpr (CLS) {
                const double *row = pc.tab + (size_t)cl[m] * PCW;
                pred_tile_K_row<double>(s, row, k, ly, tx, i, P, rows, kv[0], kv[1]);
                mv[0] = row[PR_VU], mv[1] = row[PR_VV], hd[0] = row[PR_HDX], hd[1] = row[PR_HDY];
            } else {
                pred_tile_K<double>(s, pc.vc, k, ly, tx, i, P, rows, kv[0], kv[1]);
                mv[0] = pc.vu[k], mv[1] = pc.vv[k], hd[0] = pc.hdx[k], hd[1] = pc.hdy[k];
            }
            const double xv[2] = {s.spx[ly + 1][tx + 1], s.spy[ly + 1][tx + 1]};
#pragma unroll
            for (int comp = 0; comp < 2; ++comp) {
                const size_t o = comp == 0 ? k : n + k;
                if (MIX) {
                    x32[o] = 0.0f;
                    r32[o] = 0.0f;
                }
                if (!(mv[comp] > 0.0)) continue;
                const double f = rhs[o];
                const double rv = f - (pc.rt * mv[comp] * xv[comp] - pc.mu * kv[comp]);
                if (MIX) {
                    const float rf = (float)rv;
                    r32[o] = rf;
                    const float sf = hd32[o] * rf;
                    const double rd = rf, sd = sf;
                    v[0] += rd * rd;
                    v[1] += rd * sd;
                    v[2] += sd;
                    v[3] += rd;
                    v[4] += rd * rd;
                    v[5] += f * f;
                    v[6] += rv * rv;
                } else {
                    r[o] = rv;
                    const double sv = hd[comp] * rv;
                    v[0] += f * f;
                    v[1] += rv * sv;
                    v[2] += sv;
                    v[3] += rv;
                    v[4] += rv * rv;
                }
            }
        }
    }
    if (g.b() == 0 && threadIdx.x == 0) {
        st->done = 0;
        st->status = 0;
        st->it_final = 0;
        st->stop_it = 0x7fffffff;
    }
    if (MIX) {
        put_partials<7>(g, v, pout, g.n());
    } else {
        double w[5] = {v[0], v[1], v[2], v[3], v[4]};
        put_partials<5>(g, w, pout, g.n());
    }
}
template <bool MIX, bool GEO, bool CLS = false>
__global__ __launch_bounds__(NT) void k_pred_resid(int P, int rows, int gx, int gy, size_t n, PredCoefT<double> pc,
                                                   const double *__restrict__ rhs, const double *__restrict__ xs,
                                                   double *__restrict__ r, CgState *st, double *pout,
                                                   float *__restrict__ r32, float *__restrict__ x32,
                                                   const float *__restrict__ hd32) {
    pred_resid_body<MIX, GEO, CLS>(SoloGrid{}, P, rows, gx, gy, n, pc, rhs, xs, r, st, pout, r32, x32, hd32);
}

// conv^n (eq:convective), the predictor right-hand side (eq:pm_prediction):
// (rho/tau) M U^n - (3/2) rho conv^n + (1/2) rho conv^{n-1} - pres(P) +
// mu (K U^n + 2 visc(strain(0, D))) + rho M g, and U* := U^n as the start
// value, on the tiles of k_pred_cg: K U^n from the masked U^n staged in LDS
// with its node strains formed once per node (cell strains where a face
// needs them); convection and the pressure gradient in index form.  With CLS
// the viscous coefficients come from the class table, as in k_pred_cg.
//
// Outflow walls (wall bits `ofl`, faces with a corrector factor gf != 0 but
// no mass): U* on such a face is U^n of the interior face next to it (zero
// normal gradient), as is U* of the tangential velocity beyond the wall.
// Both halves of the viscous term see the face's own velocity (U^n in the
// explicit half, U* in the implicit one), so K is applied to U^n + U* there;
// the constant Dirichlet part vd leaves those faces out.
struct OutflowDesc {
    int nx, ny, ofl;
    const double *gfx, *gfy;  // corrector factors: nonzero on the outflow faces the projection corrects
};
__device__ inline bool outflow_xface(const OutflowDesc &o, int j, int i) {
    return j >= 1 && j <= o.ny && (((o.ofl & CCNS_WALL_W) && i == 0) || ((o.ofl & CCNS_WALL_E) && i == o.nx));
}
__device__ inline bool outflow_yface(const OutflowDesc &o, int j, int i) {
    return i >= 1 && i <= o.nx && (((o.ofl & CCNS_WALL_S) && j == 0) || ((o.ofl & CCNS_WALL_N) && j == o.ny));
}

template <bool GEO, bool CLS, class G>
__device__ __forceinline__ void pred_rhs_body(const G &g, int P, int rows, int gx, int gy, size_t n, PredCoefT<double> pc,
                                                 const double *__restrict__ ax, const double *__restrict__ ay,
                                                 const double *__restrict__ hbx, const double *__restrict__ hby,
                                                 const double *__restrict__ dx, const double *__restrict__ dy,
                                                 const double *__restrict__ ux, const double *__restrict__ uy,
                                                 const double *__restrict__ pr, const double *__restrict__ vdx,
                                                 const double *__restrict__ vdy, double *__restrict__ convx,
                                                 double *__restrict__ convy, double *__restrict__ rhs,
                                                 double *__restrict__ xs, double rho, double gxv, double gyv,
                                                 int conv_valid, OutflowDesc of) {
    __shared__ PredTileNx<double> s;
    const int L = logical_group(g, ((g.n() + 7) / 8) * 8);
    if (L >= gx * gy) return;
    const int c0 = (L % gx) * TX, r0 = (L / gx) * HTY;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    constexpr int RW = HTY / 4;
    int cl[RW];
    // face volumes at entry k (they mark the unknowns)
    auto volumes = [&](size_t k, double &mx, double &my, int &ck) {
        if constexpr (CLS) {
            ck = pc.cls[k];
            const double *row = pc.tab + (size_t)ck * PCW;
            mx = row[PR_VU];
            my = row[PR_VV];
        } else {
            mx = pc.vu[k];
            my = pc.vv[k];
        }
    };
    // the value K sees at entry k: U^n on unknowns, U^n + U* on outflow faces
    auto stage_x = [&](bool in, size_t k, int j, int i, double mx, double u) -> double {
        if (!in) return 0.0;
        if (mx > 0.0) return u;
        if (of.ofl && outflow_xface(of, j, i) && of.gfx[k] != 0.0) return u + ux[i == 0 ? k + 1 : k - 1];
        return 0.0;
    };
    auto stage_y = [&](bool in, size_t k, int j, int i, double my, double v) -> double {
        if (!in) return 0.0;
        if (my > 0.0) return v;
        if (of.ofl && outflow_yface(of, j, i) && of.gfy[k] != 0.0) return v + uy[j == 0 ? k + P : k - P];
        return 0.0;
    };
#pragma unroll
    for (int m = 0; m < RW; ++m) {
        const int ly = ty + 4 * m;
        const int j = r0 + ly, i = c0 + tx;
        const bool in = j < rows;
        const size_t k = in ? (size_t)j * P + i : 0;
        double mx, my;
        volumes(k, mx, my, cl[m]);
        const double u = ux[k], v = uy[k];
        s.spx[ly + 1][tx + 1] = stage_x(in, k, j, i, mx, u);
        s.spy[ly + 1][tx + 1] = stage_y(in, k, j, i, my, v);
    }
    // the one-face halo, as in k_pred_cg
    for (int e = threadIdx.x; e < 2 * (TX + 2) + 2 * HTY; e += NT) {
        int ly, lx;
        if (e < 2 * (TX + 2)) {
            ly = e < TX + 2 ? 0 : HTY + 1;
            lx = e < TX + 2 ? e : e - (TX + 2);
        } else {
            const int f = e - 2 * (TX + 2);
            ly = 1 + (f >> 1);
            lx = (f & 1) ? TX + 1 : 0;
        }
        const int j = r0 - 1 + ly, i = c0 - 1 + lx;
        const bool in = (j >= 0) && (j < rows) && (i >= 0) && (i < P);
        const size_t k = in ? (size_t)j * P + i : 0;
        double mx, my;
        int ck;
        volumes(k, mx, my, ck);
        const double u = ux[k], v = uy[k];
        s.spx[ly][lx] = stage_x(in, k, j, i, mx, u);
        s.spy[ly][lx] = stage_y(in, k, j, i, my, v);
    }
    __syncthreads();
    if constexpr (CLS) {
#pragma unroll
        for (int m = 0; m < RW; ++m) {
            const int ly = ty + 4 * m;
            const int j = r0 + ly, i = c0 + tx;
            pred_node_strain_row<double, GEO>(s, pc.tab + (size_t)cl[m] * PCW, ly + 1, tx + 1,
                                              (j + 1 < rows) && (i + 1 < P));
        }
        for (int e = threadIdx.x; e < TX + 1 + HTY; e += NT) {
            const int ly = e <= TX ? 0 : e - TX, lx = e <= TX ? e : 0;
            const int j = r0 - 1 + ly, i = c0 - 1 + lx;
            const bool in = (j >= 0) && (j + 1 < rows) && (i >= 0) && (i + 1 < P);
            const size_t k = in ? (size_t)j * P + i : 0;
            pred_node_strain_row<double, GEO>(s, pc.tab + (size_t)pc.cls[k] * PCW, ly, lx, in);
        }
    } else {
        pred_tile_strains<double, GEO>(s, pc.vc, P, rows, c0, r0);
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < RW; ++m) {
        const int ly = ty + 4 * m;
        const int j = r0 + ly, i = c0 + tx;
        if (j >= rows) break;
        const size_t k = (size_t)j * P + i;
        double kx, ky, mx, my;
        if constexpr (CLS) {
            const double *row = pc.tab + (size_t)cl[m] * PCW;
            pred_tile_K_row<double>(s, row, k, ly, tx, i, P, rows, kx, ky);
            mx = row[PR_VU], my = row[PR_VV];
        } else {
            pred_tile_K<double>(s, pc.vc, k, ly, tx, i, P, rows, kx, ky);
            mx = pc.vu[k], my = pc.vv[k];
        }
        const double u = ux[k], v = uy[k];
        double us = u, vs = v;
        if (of.ofl) {
            // U* on outflow faces, and beyond the outflow walls, from the
            // interior neighbour (zero normal gradient)
            if (mx == 0.0 && outflow_xface(of, j, i) && of.gfx[k] != 0.0) us = ux[i == 0 ? k + 1 : k - 1];
            if (my == 0.0 && outflow_yface(of, j, i) && of.gfy[k] != 0.0) vs = uy[j == 0 ? k + P : k - P];
            if (i >= 1 && i <= of.nx - 1) {
                if ((of.ofl & CCNS_WALL_S) && j == 0) us = ux[k + P];
                if ((of.ofl & CCNS_WALL_N) && j == of.ny + 1) us = ux[k - P];
            }
            if (j >= 1 && j <= of.ny - 1) {
                if ((of.ofl & CCNS_WALL_W) && i == 0) vs = uy[k + 1];
                if ((of.ofl & CCNS_WALL_E) && i == of.nx + 1) vs = uy[k - 1];
            }
        }
        xs[k] = us;
        xs[n + k] = vs;
        if (mx > 0.0) {
            const double cv = conv_x(ax, ay, ux, uy, hbx, dx, k, P);
            const double cold = conv_valid ? convx[k] : cv;
            convx[k] = cv;
            const double presv = ax[k] * (pr[k + 1] - pr[k]);
            rhs[k] = pc.rt * mx * u - 1.5 * rho * cv + 0.5 * rho * cold - presv + pc.mu * (kx + 2.0 * vdx[k]) +
                     rho * mx * gxv;
        } else {
            rhs[k] = 0.0;
        }
        if (my > 0.0) {
            const double cv = conv_y(ax, ay, ux, uy, hby, dy, k, P);
            const double cold = conv_valid ? convy[k] : cv;
            convy[k] = cv;
            const double presv = ay[k] * (pr[k + P] - pr[k]);
            rhs[n + k] = pc.rt * my * v - 1.5 * rho * cv + 0.5 * rho * cold - presv + pc.mu * (ky + 2.0 * vdy[k]) +
                         rho * my * gyv;
        } else {
            rhs[n + k] = 0.0;
        }
    }
}
template <bool GEO, bool CLS = false>
__global__ __launch_bounds__(NT) void k_pred_rhs(int P, int rows, int gx, int gy, size_t n, PredCoefT<double> pc,
                                                 const double *__restrict__ ax, const double *__restrict__ ay,
                                                 const double *__restrict__ hbx, const double *__restrict__ hby,
                                                 const double *__restrict__ dx, const double *__restrict__ dy,
                                                 const double *__restrict__ ux, const double *__restrict__ uy,
                                                 const double *__restrict__ pr, const double *__restrict__ vdx,
                                                 const double *__restrict__ vdy, double *__restrict__ convx,
                                                 double *__restrict__ convy, double *__restrict__ rhs,
                                                 double *__restrict__ xs, double rho, double gxv, double gyv,
                                                 int conv_valid, OutflowDesc of) {
    pred_rhs_body<GEO, CLS>(SoloGrid{}, P, rows, gx, gy, n, pc, ax, ay, hbx, hby, dx, dy, ux, uy, pr, vdx, vdy, convx, convy, rhs, xs, rho, gxv, gyv, conv_valid, of);
}

// ---------------------------------------------------------------------------
// corrector, pressure update and diagnostics
// ---------------------------------------------------------------------------

// U^{n+1} = U* - (tau/rho) (A/V_f) dPhi on pressure-coupled faces (eq:pm_projection).
template <class G>
__device__ __forceinline__ void correct_body(const G &g, Dims d, const double *__restrict__ gx, const double *__restrict__ gy,
                                                const double *__restrict__ usx, const double *__restrict__ usy,
                                                const double *__restrict__ phi, double *__restrict__ ux,
                                                double *__restrict__ uy, double s) {
    const size_t P = d.pitch;
    struct In {
        double g1, g2, us, vs, p0, pe, pn;
    };
    auto load = [&](size_t k) {
        // the east and north neighbours exist wherever g1, g2 are nonzero
        const size_t ke = k + 1 < d.n ? k + 1 : k, kn = k + P < d.n ? k + P : k;
        return In{gx[k], gy[k], usx[k], usy[k], phi[k], phi[ke], phi[kn]};
    };
    for_cells_batched<TY / 4>(g, d, load, [&](int, int, int, size_t k, const In &v) {
        ux[k] = (v.g1 != 0.0) ? v.us - s * v.g1 * (v.pe - v.p0) : v.us;
        uy[k] = (v.g2 != 0.0) ? v.vs - s * v.g2 * (v.pn - v.p0) : v.vs;
    });
}
__global__ __launch_bounds__(NT) void k_correct(Dims d, const double *__restrict__ gx, const double *__restrict__ gy,
                                                const double *__restrict__ usx, const double *__restrict__ usy,
                                                const double *__restrict__ phi, double *__restrict__ ux,
                                                double *__restrict__ uy, double s) {
    correct_body(SoloGrid{}, d, gx, gy, usx, usy, phi, ux, uy, s);
}

// Force of the fluid on the bodies: the momentum it exchanges with them
// through the capacities (pressure on the cut cells' projected surface,
// strain on the second-kind capacities), from the table of cut cells and
// nodes.  One work-group; each thread sums a strided share of the rows and
// the shares are added in a fixed order.
constexpr int FT = 1024;
__global__ __launch_bounds__(FT) void k_forces(const double *__restrict__ tab, int nfc, int nfn, int cap, int P,
                                               const double *__restrict__ dinv, const double *__restrict__ pr,
                                               const double *__restrict__ ux, const double *__restrict__ uy,
                                               const double *__restrict__ dx, const double *__restrict__ dy,
                                               double two_mu, double *__restrict__ out) {
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int e = threadIdx.x; e < nfc; e += FT) {
        const double *r = tab + (size_t)e * FORCE_W;
        const size_t k = (size_t)r[FC_J] * P + (size_t)r[FC_I];
        const double p = dinv[k] > 0.0 ? pr[k] : 0.0;
        v[0] += p * r[FC_WPX];
        v[1] += p * r[FC_WPY];
        const double sxx = r[FC_WXX] * (r[FC_BXX_E] * (ux[k] - dx[k]) - r[FC_BXX_W] * (ux[k - 1] - dx[k - 1]) +
                                        r[FC_AXX] * (dx[k] - dx[k - 1]));
        const double syy = r[FC_WYY] * (r[FC_BYY_N] * (uy[k] - dy[k]) - r[FC_BYY_S] * (uy[k - P] - dy[k - P]) +
                                        r[FC_AYY] * (dy[k] - dy[k - P]));
        v[2] += sxx * r[FC_WVX];
        v[3] += syy * r[FC_WVY];
    }
    const double *tn = tab + (size_t)cap * FORCE_W;
    for (int e = threadIdx.x; e < nfn; e += FT) {
        const double *r = tn + (size_t)e * FORCE_W;
        const size_t k = (size_t)r[FN_J] * P + (size_t)r[FN_I];
        const double gx = r[FN_BXY_A] * (ux[k + P] - dx[k + P]) - r[FN_BXY_B] * (ux[k] - dx[k]) +
                          r[FN_AXY] * (dx[k + P] - dx[k]);
        const double gy = r[FN_BYX_R] * (uy[k + 1] - dy[k + 1]) - r[FN_BYX_L] * (uy[k] - dy[k]) +
                          r[FN_AYX] * (dy[k + 1] - dy[k]);
        v[2] += 0.5 * (r[FN_NXX] * gx + r[FN_NXY] * gy) * r[FN_WNX];
        v[3] += 0.5 * (r[FN_NYX] * gx + r[FN_NYY] * gy) * r[FN_WNY];
    }
    __shared__ double red[4][FT];
    for (int q = 0; q < 4; ++q) red[q][threadIdx.x] = v[q];
    __syncthreads();
    for (int w = FT / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int q = 0; q < 4; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = red[0][0];
        out[1] = red[1][0];
        out[2] = two_mu * red[2][0];
        out[3] = two_mu * red[3][0];
    }
}

struct DiagCoef {
    const double *ax, *ay, *het, *dinv, *vur, *vvr, *vu, *vv, *cx, *cy, *vinv;
};

// Divergence max / net flux, kinetic energy and momentum of U; optionally
// P += Phi - (tau mu / 2 rho) V^-1 L Phi (eq:pm_update).
template <class G>
__device__ __forceinline__ void diag_body(const G &g, Dims d, DiagCoef c, const double *__restrict__ ux,
                                             const double *__restrict__ uy, const double *__restrict__ phi,
                                             double *__restrict__ pr, double pcoef, int update_p, double rho,
                                             double *pout) {
    const size_t P = d.pitch;
    double v[5] = {0, 0, 0, 0, 0};
    for_cells(g, d, [&](int, int j, int i, size_t k) {
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
    put_partials<4, 1>(g, v, pout, d.nblk);
}
__global__ __launch_bounds__(NT) void k_diag(Dims d, DiagCoef c, const double *__restrict__ ux,
                                             const double *__restrict__ uy, const double *__restrict__ phi,
                                             double *__restrict__ pr, double pcoef, int update_p, double rho,
                                             double *pout) {
    diag_body(SoloGrid{}, d, c, ux, uy, phi, pr, pcoef, update_p, rho, pout);
}

__device__ __forceinline__ void diag_final_body(const double *pin, int nin, DiagState *ds) {
    double t[5];
    get_totals<4, 1>(pin, nin, t);
    if (threadIdx.x == 0) {
        ds->mass = t[0];
        ds->ke = t[1];
        ds->momx = t[2];
        ds->momy = t[3];
        ds->divmax = t[4];
    }
}
__global__ __launch_bounds__(NT) void k_diag_final(const double *pin, int nin, DiagState *ds) {
    diag_final_body(pin, nin, ds);
}

// U = D on every face that is not a velocity unknown (vm = 0 there).
// A set velocity field keeps the Dirichlet data on the faces that are no
// unknowns, except where the step carries the velocity as state: outflow
// faces (corrector factor gf != 0) and, beyond an outflow wall, the
// tangential velocity (component 0: x, 1: y).
__global__ __launch_bounds__(NT) void k_keep_dirichlet(Dims d, double *__restrict__ u,
                                                       const double *__restrict__ dd,
                                                       const double *__restrict__ vm,
                                                       const double *__restrict__ gf, OutflowDesc of, int comp) {
    for_cells(d, [&](int, int j, int i, size_t k) {
        if (vm[k] > 0.0) return;
        if (of.ofl) {
            if (gf[k] != 0.0) return;
            if (comp == 0 && i >= 1 && i <= of.nx - 1 &&
                (((of.ofl & CCNS_WALL_S) && j == 0) || ((of.ofl & CCNS_WALL_N) && j == of.ny + 1)))
                return;
            if (comp == 1 && j >= 1 && j <= of.ny - 1 &&
                (((of.ofl & CCNS_WALL_W) && i == 0) || ((of.ofl & CCNS_WALL_E) && i == of.nx + 1)))
                return;
        }
        u[k] = dd[k];
    });
}

// ---------------------------------------------------------------------------
// operator applies (parity entry points)
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(NT) void k_op_cont(Dims d, const double *ax, const double *ay, const double *het,
                                                const double *ux, const double *uy, double *out) {
    const size_t P = d.pitch;
    for_cells(d, [&](int, int j, int i, size_t k) {
        if (i < 1 || i > d.nx || j < 1 || j > d.ny) { out[k] = 0.0; return; }
        out[k] = ax[k] * ux[k] - ax[k - 1] * ux[k - 1] + ay[k] * uy[k] - ay[k - P] * uy[k - P] + het[k];
    });
}

__global__ __launch_bounds__(NT) void k_op_pres(Dims d, const double *ax, const double *ay, const double *p,
                                                double *gx, double *gy) {
    const size_t P = d.pitch;
    for_cells(d, [&](int, int j, int i, size_t k) {
        auto pv = [&](int jj, int ii) {
            return (ii >= 1 && ii <= d.nx && jj >= 1 && jj <= d.ny) ? p[(size_t)jj * P + ii] : 0.0;
        };
        gx[k] = (i >= 0 && i <= d.nx && j >= 1 && j <= d.ny) ? ax[k] * (pv(j, i + 1) - pv(j, i)) : 0.0;
        gy[k] = (i >= 1 && i <= d.nx && j >= 0 && j <= d.ny) ? ay[k] * (pv(j + 1, i) - pv(j, i)) : 0.0;
    });
}

// mode 0: visc(strain(U, D)) = K U_unknowns + vD; mode 1: H p (p masked).
// mode 0: visc(strain(U, D)) with U given on the unknowns and on the outflow
// faces (the faces without mass whose corrector factor gfx, gfy is nonzero;
// the constant part vd leaves them out), D elsewhere; mode 1: H U.
__global__ __launch_bounds__(NT) void k_op_visc(Dims d, PredCoef pc, const double *vdx, const double *vdy,
                                                const double *gfx, const double *gfy, const double *ux,
                                                const double *uy, double *ox, double *oy, int mode) {
    const size_t P = d.pitch;
    auto pxm = [&](size_t kk) { return (pc.vu[kk] > 0.0 || (mode == 0 && gfx[kk] != 0.0)) ? ux[kk] : 0.0; };
    auto pym = [&](size_t kk) { return (pc.vv[kk] > 0.0 || (mode == 0 && gfy[kk] != 0.0)) ? uy[kk] : 0.0; };
    for_cells(d, [&](int, int j, int i, size_t k) {
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
    for_cells(d, [&](int, int j, int i, size_t k) {
        ox[k] = (i >= 1 && i <= d.nx - 1 && j >= 1 && j <= d.ny) ? conv_x(ax, ay, ux, uy, hbx, dx, k, P) : 0.0;
        oy[k] = (i >= 1 && i <= d.nx && j >= 1 && j <= d.ny - 1) ? conv_y(ax, ay, ux, uy, hby, dy, k, P) : 0.0;
    });
}

__global__ __launch_bounds__(NT) void k_op_lap(Dims d, PoisCoef pc, const double *phi, double *out) {
    const size_t P = d.pitch;
    for_cells(d, [&](int, int j, int i, size_t k) {
        if (!(pc.dinv[k] > 0.0)) { out[k] = 0.0; return; }
        const double ph = phi[k];
        out[k] = pc.cx[k] * (phi[k + 1] - ph) - pc.cx[k - 1] * (ph - phi[k - 1]) + pc.cy[k] * (phi[k + P] - ph) -
                 pc.cy[k - P] * (ph - phi[k - P]);
    });
}

__global__ __launch_bounds__(NT) void k_op_kin(Dims d, const double *vur, const double *vvr, const double *ux,
                                               const double *uy, double *out) {
    const size_t P = d.pitch;
    for_cells(d, [&](int, int j, int i, size_t k) {
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
    A_PR1X, A_PR1Y,  // predictor r (pong)
    A_PQ1X, A_PQ1Y,  // predictor q (pong)
    A_RHSX, A_RHSY,  // predictor right-hand side
    A_B, A_R, A_P0, A_P1, A_Q,  // Poisson
    A_Z, A_ZT,                  // multigrid output and its ping-pong partner
    A_T0, A_T1, A_T2, A_T3,     // scratch for operator applies
    A_COUNT
};

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Partial-sum buffers: each holds up to 8 slots of NBMAX groups.
enum Part { PB_RHS, PB_INIT, PB_DIR, PB_UPD, PB_DIAG, PB_MG, PB_COUNT };

// Multigrid levels: grid sizes from the fine one by halving (rounding up)
// until both sides are at most 16 cells, and at least one coarse level (the
// finest level's up-sweep writes the statistics the CG reads, so even a grid
// of at most 16 x 16 cells gets a cycle level above its coarsest grid).
std::vector<std::pair<int, int>> mg_sizes(int nx, int ny) {
    std::vector<std::pair<int, int>> v{{nx, ny}};
    while (v.size() < 2 || v.back().first > 16 || v.back().second > 16)
        v.push_back({(v.back().first + 1) / 2, (v.back().second + 1) / 2});
    return v;
}
constexpr int MG_ARRS = 6;  // cx, cy, dinv, b, x, xt per coarse level

// Float arrays of precision 1 (FP32 inner solves), in allocation order.
// Pairs of face components are adjacent (the y array starts n floats after
// the x array), as the face kernels index them.
enum Arr32 {
    G_CX, G_CY, G_DINV,                 // Poisson coefficients
    G_R, G_X, G_P0, G_P1, G_Q, G_Z, G_ZT,  // Poisson inner vectors
    G_VU, G_VV, G_BXX, G_BXY, G_BYY, G_BYX, G_WXX, G_WYY, G_NXX, G_NXY, G_NYX, G_NYY,
    G_HDX, G_HDY,    // predictor Jacobi diagonal (pair)
    G_PRX, G_PRY,    // predictor inner r (pair)
    G_PXX, G_PXY,    // predictor inner x = correction (pair)
    G_PP0X, G_PP0Y, G_PP1X, G_PP1Y, G_PQX, G_PQY,
    G_PR1X, G_PR1Y, G_PQ1X, G_PQ1Y,  // pong partners of r and q
    G_COUNT
};

struct WsPlan {
    Layout L;
    size_t arr_bytes;   // bytes per array
    size_t part_off, part_bytes, state_off;
    std::vector<Layout> mgL;       // coarse levels (index 1..)
    std::vector<size_t> mg_off;    // byte offset of each coarse level's arrays
    size_t pinv_off, idx_off;      // coarsest-grid pseudo-inverse and unknown list
    int ncoarse;                   // cells of the coarsest grid
    // precision 1 only (else 0): float arrays and float coarse levels
    size_t arr32_bytes, f32_off;
    std::vector<size_t> mg32_off;
    // predictor coefficient classes: one int per entry, up to max_cls rows of
    // PCW values (FP64)
    size_t cls_off, tab_off, tab32_off;
    int max_cls;
    // force tables (cells, nodes: up to force_cap rows of FORCE_W each) and
    // the four sums
    size_t force_off;
    int force_cap;
    size_t total;
};

WsPlan plan(int nx, int ny, int precision) {
    WsPlan w;
    w.L = make_layout(nx, ny);
    w.arr_bytes = align_up(w.L.n * sizeof(double), 256);
    w.part_off = w.arr_bytes * A_COUNT;
    // partial sums: up to 8 slots for the largest number of work-groups any
    // kernel launches (one 64 x 8 tile per group)
    const size_t groups = ((size_t)(w.L.pitch / TX) * ((w.L.rows + 7) / 8) + 7) / 8 * 8;
    w.part_bytes = align_up(std::max<size_t>(NBMAX, groups) * 8 * sizeof(double), 256);
    w.state_off = w.part_off + w.part_bytes * PB_COUNT;
    size_t off = w.state_off + 4096;
    auto sizes = mg_sizes(nx, ny);
    w.mgL.push_back(w.L);
    w.mg_off.push_back(0);
    for (size_t l = 1; l < sizes.size(); ++l) {
        Layout Lc = make_layout(sizes[l].first, sizes[l].second);
        w.mgL.push_back(Lc);
        w.mg_off.push_back(off);
        off += MG_ARRS * align_up(Lc.n * sizeof(double), 256);
    }
    w.ncoarse = sizes.back().first * sizes.back().second;
    w.pinv_off = off;
    off += align_up((size_t)w.ncoarse * w.ncoarse * sizeof(double), 256);
    w.idx_off = off;
    off += align_up((size_t)w.ncoarse * sizeof(int), 256);
    w.arr32_bytes = 0;
    w.f32_off = 0;
    w.mg32_off.assign(w.mgL.size(), 0);
    if (precision == 1) {
        // n * 4 bytes is a multiple of 256 (the pitch is a multiple of 64)
        w.arr32_bytes = w.L.n * sizeof(float);
        w.f32_off = off;
        off += w.arr32_bytes * G_COUNT;
        for (size_t l = 1; l < w.mgL.size(); ++l) {
            w.mg32_off[l] = off;
            off += MG_ARRS * align_up(w.mgL[l].n * sizeof(float), 256);
        }
    }
    w.cls_off = off;
    off += align_up(w.L.n * sizeof(int), 256);
    w.max_cls = (int)std::max<size_t>(1024, w.L.n / 16);
    w.tab_off = off;
    off += align_up((size_t)w.max_cls * PCW * sizeof(double), 256);
    w.tab32_off = off;  // the same rows in float (precision 1)
    if (precision == 1) off += align_up((size_t)w.max_cls * PCW * sizeof(float), 256);
    // the cut cells and nodes of the bodies: a few per cell of their outline,
    // well within eight box perimeters
    w.force_cap = 8 * (nx + ny) + 1024;
    w.force_off = off;
    off += align_up(((size_t)2 * w.force_cap * FORCE_W + 8) * sizeof(double), 256);
    w.total = off;
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
    double *part[PB_COUNT];
    CgState *st_pred, *st_pois;
    CgState *st_pred_in, *st_pois_in;  // inner solves of precision 1
    DiagState *diag;
    double *outer;      // totals of the FP64 residual statistics (precision 1)
    CgState *h_st;      // pinned host copies (for a context without allocations: the members below)
    DiagState *h_diag;
    double *h_outer;
    int static_dev;     // device whose static workspace the context uses, or -1
    CgState st_host;
    DiagState diag_host;
    double outer_host[8];
    float *f[G_COUNT];  // precision 1 arrays
    int last_pois_in, last_pred_in;
    Dims dc, df;        // cell tiles (1 component) and face tiles (2 components)
    Dims dp;            // tiles of the Poisson stencil kernels (PTY rows)
    int conv_valid;
    int n_active;
    int last_pois_it, last_pred_it;
    int pbuf_pois;
    int init_nblk;      // groups of the last init kernel (its partials feed the first direction)
    // multigrid hierarchy (level 0 shares the Poisson arrays)
    template <class T>
    struct LevelT {
        Layout L;
        Dims d;      // PTY-row tiles
        T *cx, *cy, *dinv, *b, *x, *xt;
    };
    using Level = LevelT<double>;
    std::vector<Level> mg;
    std::vector<LevelT<float>> mg32;   // the same hierarchy in float (precision 1)
    double *pinv;
    int *pidx;
    int ncoarse_act;
    int tail_lds;       // bytes of dynamic LDS the LDS-resident coarse end may use (0: not used)
    // predictor coefficient classes (ncls = 0: the predictor CG reads the
    // coefficient arrays)
    int ncls;
    int *cls;
    double *tab;
    float *tab32;      // the table in float (precision 1), or null
    // force on the bodies: table rows (nfc cells, then nfn nodes; nfc < 0:
    // more cut cells than the workspace holds) and the four sums
    int nfc, nfn;
    double *ftab, *fsum;
    // kernel form of each cycle level: [FP64][down, up][level]
    unsigned char mgf[2][2][16];
    // optional kernel timing: start/stop events attached to sampled launches
    int timing;
    std::vector<hipEvent_t> evpool;
    size_t evused;
    struct TimedLaunch {
        size_t ev;  // first event of the pair
        int kid;    // timing slot
        int it;     // CG iteration of the launch
    };
    std::vector<TimedLaunch> evlog;
    double t_ms[4];    // Poisson direction, Poisson update, predictor CG iteration, its reduction
    long t_count[4];
    std::string err;
};

namespace {

ccns_status fail(ccns_ctx *c, ccns_status s, const std::string &msg) {
    if (c) c->err = msg;
    return s;
}

void release_static(int dev);

// Frees a context (after its stream's work); release: the context was
// handed out, so its static workspace, if any, becomes free for the next one.
void destroy_ctx(ccns_ctx *ctx, bool release) {
    if (!ctx) return;
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->static_dev < 0) {
        if (ctx->h_st) (void)hipHostFree(ctx->h_st);
        if (ctx->h_diag) (void)hipHostFree(ctx->h_diag);
        if (ctx->h_outer) (void)hipHostFree(ctx->h_outer);
    }
    for (hipEvent_t e : ctx->evpool) (void)hipEventDestroy(e);
    if (release && ctx->static_dev >= 0) release_static(ctx->static_dev);
    delete ctx;
}

#define HIPCHK(ctx, call)                                                                   \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(ctx, CCNS_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// One tile per work-group (the stencil kernels of the CG iterations: enough
// wavefronts in flight to cover the memory latency).
Dims make_dims_1(const Layout &L, int ncomp, int ty) {
    Dims d;
    d.nx = L.nx;
    d.ny = L.ny;
    d.rows = L.rows;
    d.pitch = L.pitch;
    d.gx = L.pitch / TX;
    d.ty = ty;
    d.gy = (L.rows + ty - 1) / ty;
    d.ntile = d.gx * d.gy;
    d.ncomp = ncomp;
    d.tpb = 1;
    d.nblk = ((d.ntile * ncomp + 7) / 8) * 8;
    d.n = L.n;
    return d;
}

Dims make_dims(const Layout &L, int ncomp, int ty) {
    Dims d;
    d.nx = L.nx;
    d.ny = L.ny;
    d.rows = L.rows;
    d.pitch = L.pitch;
    d.gx = L.pitch / TX;
    d.ty = ty;
    d.gy = (L.rows + ty - 1) / ty;
    d.ntile = d.gx * d.gy;
    d.ncomp = ncomp;
    const int total = d.ntile * ncomp;
    d.tpb = (total + NBMAX - 1) / NBMAX;
    const int groups = (total + d.tpb - 1) / d.tpb;
    d.nblk = ((groups + 7) / 8) * 8;
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

PredCoefT<double> pred_coef_t(ccns_ctx *c) {
    PredCoef pc = pred_coef(c);
    return PredCoefT<double>{ViscCoefT<double>{pc.vc.bxx, pc.vc.bxy, pc.vc.byy, pc.vc.byx, pc.vc.wxx, pc.vc.wyy,
                                               pc.vc.nxx, pc.vc.nxy, pc.vc.nyx, pc.vc.nyy},
                             pc.vu, pc.vv, pc.hdx, pc.hdy, pc.rt, pc.mu, nullptr, nullptr};
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

// Groups of an element-wise kernel over ntot entries.
int flat_blocks(size_t ntot) {
    size_t b = (ntot + (size_t)NT * UPT - 1) / ((size_t)NT * UPT);
    b = std::min<size_t>(std::max<size_t>(b, 8), NBMAX);
    return (int)((b + 7) / 8 * 8);
}
// Groups of the CG update kernel (UT threads, UPT entries per thread and pass).
int update_blocks(size_t ntot) {
    size_t b = (ntot + (size_t)UT * UPT - 1) / ((size_t)UT * UPT);
    b = std::min<size_t>(std::max<size_t>(b, 8), NBMAX);
    return (int)((b + 7) / 8 * 8);
}

hipEvent_t next_event(ccns_ctx *c) {
    if (c->evused == c->evpool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        c->evpool.push_back(e);
    }
    return c->evpool[c->evused++];
}

// Launches a kernel on the context's stream.  When tm, HIP start and stop
// events are attached to the dispatch itself (hipExtLaunchKernelGGL), so the
// sampled time is the kernel's own duration without the gap of a separate
// event packet, and the pair is logged for timing slot kid with the CG
// iteration it of the launch.
template <typename... KArgs, typename... Args>
void launch(ccns_ctx *c, bool tm, int kid, int it, void (*kernel)(KArgs...), dim3 grid, dim3 block,
            Args... args) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const size_t i0 = c->evused;
    if (tm) {
        e0 = next_event(c);
        e1 = e0 ? next_event(c) : nullptr;
    }
    if (e0 && e1) {
        c->evlog.push_back({i0, kid, it});
        hipExtLaunchKernelGGL(kernel, grid, block, 0, c->stream, e0, e1, 0, args...);
    } else {
        kernel<<<grid, block, 0, c->stream>>>(args...);
    }
}

// Adds the durations of the sampled launches of a finished solve whose
// iteration came before it_stop (the launch that stopped the solve, and any
// after it, return early and are not the kernel's cost).
void harvest_events(ccns_ctx *c, int it_stop) {
    for (const auto &e : c->evlog) {
        float ms = 0.f;
        if (e.it < it_stop && hipEventElapsedTime(&ms, c->evpool[e.ev], c->evpool[e.ev + 1]) == hipSuccess) {
            c->t_ms[e.kid] += ms;
            c->t_count[e.kid] += 1;
        }
    }
    c->evlog.clear();
    c->evused = 0;
}

// Runs CG iterations (after the caller launched the init kernel, whose
// partials are in PB_INIT) until the device flags the end of the solve.
// dir(first, par, pold, pnew, pin, nin, pout, tm, it) launches the
// direction+operator kernel of iteration it (timed when tm) and returns the
// number of partials it leaves in PB_DIR; finish() runs after it.  T is the storage type of the vectors.
template <class T, class Dir, class Finish>
ccns_status cg_loop(ccns_ctx *c, CgState *st, T *x, T *r, T *const pbuf[2], int &par_buf, T *q, const T *dinv,
                    size_t ntot, int &last_it, Dir dir, Finish finish, ccns_solve_info *info, int kid) {
    const int nl = update_blocks(ntot);
    int chunk = std::max(4, last_it + 1);
    int it = 0;
    bool first = true;
    for (;;) {
        for (int u = 0; u < chunk; ++u, ++it) {
            const int par = it & 1;
            const bool tm = c->timing && (it % 8 == 4) && it < last_it;
            const int nd = dir(first ? 1 : 0, par, pbuf[par_buf], pbuf[par_buf ^ 1],
                               first ? c->part[PB_INIT] : c->part[PB_UPD], first ? c->init_nblk : nl,
                               c->part[PB_DIR], tm, it);
            finish();
            launch(c, tm, kid + 1, it, k_cg_update<T>, dim3(nl), dim3(UT), ntot, nl, dinv, x, r,
                   (const T *)pbuf[par_buf ^ 1], (const T *)q, st, par, (const double *)c->part[PB_DIR], nd,
                   c->part[PB_UPD]);
            par_buf ^= 1;
            first = false;
        }
        HIPCHK(c, hipGetLastError());
        HIPCHK(c, hipMemcpyAsync(c->h_st, st, sizeof(CgState), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        if (c->h_st->done) break;
        chunk = 8;
    }
    last_it = c->h_st->it_final;
    if (c->timing) harvest_events(c, c->h_st->it_final);
    if (info) {
        info->iterations = c->h_st->it_final;
        info->outer = 1;
        info->rel_residual =
            c->h_st->fnorm2 > 0 ? std::sqrt(c->h_st->rnorm2_final / c->h_st->fnorm2) : 0.0;
        info->status = c->h_st->status;
        info->inner_status = CCNS_OK;
        info->inner_fail_sweep = -1;
    }
    return (ccns_status)c->h_st->status;
}

OutflowDesc outflow_desc(const ccns_ctx *c) {
    return OutflowDesc{c->g.nx, c->g.ny, c->prm.outflow, c->a[A_GX], c->a[A_GY]};
}

void set_cg(ccns_ctx *c, CgState *st, double tol, int maxit, int zero_mean, int n_active) {
    CgState h{};
    h.tol2 = tol * tol;
    h.maxit = maxit;
    h.zero_mean = zero_mean;
    h.n_active = std::max(n_active, 1);
    h.done = 1;
    (void)hipMemcpyAsync(st, &h, sizeof(CgState), hipMemcpyHostToDevice, c->stream);
    (void)hipStreamSynchronize(c->stream);
}

// Relative tolerance of the next inner solve (precision 1).
__global__ void k_set_tol(CgState *st, double tol2) {
    if (threadIdx.x == 0) st->tol2 = tol2;
}

// Jacobi-preconditioned CG for the pressure; the init kernel's partials are
// in PB_INIT (init_nblk groups).
template <class T>
ccns_status jacobi_cg(ccns_ctx *c, PoisCoefT<T> pc, CgState *st, T *x, T *r, T *p0, T *p1, T *q, int &last_it,
                      ccns_solve_info *info) {
    T *pb[2] = {p0, p1};
    auto dir = [&](int first, int par, T *pold, T *pnew, const double *pin, int nin2, double *pout, bool tm,
                   int it) {
        launch(c, tm, 0, it, k_pois_dir<T>, dim3(c->dp.nblk), dim3(NT), c->dp, pc, (const T *)r, (const T *)pold, pnew, q,
               st, first, par, pin, nin2, pout);
        return c->dp.nblk;
    };
    return cg_loop<T>(c, st, x, r, pb, c->pbuf_pois, q, pc.dinv, c->w.L.n, last_it, dir, [] {}, info, 0);
}

// Pressure solve (precision 0, Jacobi); b is in A_B with its sum's partials
// in PB_RHS (nin groups).
ccns_status pressure_solve_dev(ccns_ctx *c, int nin, ccns_solve_info *info) {
    PoisCoef pc = pois_coef(c);
    k_pois_init<false><<<c->dc.nblk, NT, 0, c->stream>>>(c->dc, pc, c->a[A_B], c->a[A_PHI], c->a[A_R], c->st_pois,
                                                         c->part[PB_RHS], nin, c->part[PB_INIT], nullptr, nullptr,
                                                         nullptr);
    c->init_nblk = c->dc.nblk;
    return jacobi_cg<double>(c, pc, c->st_pois, c->a[A_PHI], c->a[A_R], c->a[A_P0], c->a[A_P1], c->a[A_Q],
                             c->last_pois_it, info);
}

constexpr int MG_NU = 2;          // pre- and post-smoothing sweeps

// Builds the coarse levels on the host from the fine Poisson weights and
// uploads them (and their float copies in precision 1); the coarsest grid
// gets a dense pseudo-inverse.
// Coefficient classes of the predictor CG (PredRow): the row of every entry
// of the face layout, with equal rows (bit for bit) sharing one class.  A
// neighbour outside the grid contributes 0 (the kernel never uses such a
// value).  Leaves ncls = 0 (the CG then reads the coefficient arrays) when
// there are more classes than the workspace's table holds.
ccns_status pred_classes(ccns_ctx *c, const HostCoef &hc) {
    c->ncls = 0;
    c->cls = (int *)(c->base + c->w.cls_off);
    c->tab = (double *)(c->base + c->w.tab_off);
    c->tab32 = c->prm.precision == 1 ? (float *)(c->base + c->w.tab32_off) : nullptr;
    if (c->prm.coef_tables == 1) return CCNS_OK;
    const Layout &L = c->w.L;
    const long P = L.pitch, rows = L.rows, W = c->g.nx + 2;
    auto at = [&](const std::vector<double> &v, long j, long i) -> double {
        return (j >= 0 && j < rows && i >= 0 && i < W) ? v[(size_t)(j * W + i)] : 0.0;
    };
    std::vector<int> cls(L.n);
    std::vector<double> tab;
    std::unordered_map<std::string, int> index;
    double row[PCW], last[PCW];
    int lastc = -1;
    for (long j = 0; j < rows; ++j)
        for (long i = 0; i < P; ++i) {
            row[PR_HDX] = at(hc.hdx, j, i);
            row[PR_HDY] = at(hc.hdy, j, i);
            row[PR_VU] = at(hc.vu, j, i);
            row[PR_VV] = at(hc.vv, j, i);
            row[PR_BXX_W] = at(hc.bxx, j, i - 1);
            row[PR_BXX] = at(hc.bxx, j, i);
            row[PR_BXX_E] = at(hc.bxx, j, i + 1);
            row[PR_WXX] = at(hc.wxx, j, i);
            row[PR_WXX_E] = at(hc.wxx, j, i + 1);
            row[PR_BYY_S] = at(hc.byy, j - 1, i);
            row[PR_BYY] = at(hc.byy, j, i);
            row[PR_BYY_N] = at(hc.byy, j + 1, i);
            row[PR_WYY] = at(hc.wyy, j, i);
            row[PR_WYY_N] = at(hc.wyy, j + 1, i);
            row[PR_BXY] = at(hc.bxy, j, i);
            row[PR_BYX] = at(hc.byx, j, i);
            row[PR_BXY_N] = at(hc.bxy, j + 1, i);
            row[PR_BYX_E] = at(hc.byx, j, i + 1);
            row[PR_NXX] = at(hc.nxx, j, i);
            row[PR_NYY] = at(hc.nyy, j, i);
            row[PR_NXY] = at(hc.nxy, j, i);
            row[PR_NYX] = at(hc.nyx, j, i);
            for (int u = PR_COUNT; u < PCW; ++u) row[u] = 0.0;
            int id = lastc;
            if (lastc < 0 || std::memcmp(row, last, sizeof row) != 0) {
                std::string key((const char *)row, sizeof row);
                auto f = index.find(key);
                if (f == index.end()) {
                    id = (int)(tab.size() / PCW);
                    if (id >= c->w.max_cls) return CCNS_OK;
                    index.emplace(std::move(key), id);
                    tab.insert(tab.end(), row, row + PCW);
                } else {
                    id = f->second;
                }
                std::memcpy(last, row, sizeof row);
                lastc = id;
            }
            cls[(size_t)(j * P + i)] = id;
        }
    HIPCHK(c, hipMemcpyAsync(c->cls, cls.data(), cls.size() * sizeof(int), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->tab, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
    // the float rows are the float arrays' values (each converted once)
    std::vector<float> tab32;
    if (c->tab32) {
        tab32.assign(tab.begin(), tab.end());
        HIPCHK(c, hipMemcpyAsync(c->tab32, tab32.data(), tab32.size() * sizeof(float), hipMemcpyHostToDevice,
                                 c->stream));
    }
    // the host vectors are released when this returns: wait for the copies
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->ncls = (int)(tab.size() / PCW);
    return CCNS_OK;
}

ccns_status mg_setup(ccns_ctx *c, const HostCoef &hc) {
    const WsPlan &w = c->w;
    const bool mix = c->prm.precision == 1;
    c->mg.clear();
    c->mg32.clear();
    ccns_ctx::Level l0;
    l0.L = w.L;
    l0.d = make_dims(w.L, 1, PTY);
    l0.cx = c->a[A_CX];
    l0.cy = c->a[A_CY];
    l0.dinv = c->a[A_DINV];
    l0.b = c->a[A_R];
    l0.x = c->a[A_Z];
    l0.xt = c->a[A_ZT];
    c->mg.push_back(l0);
    if (mix) {
        ccns_ctx::LevelT<float> f0;
        f0.L = w.L;
        f0.d = l0.d;
        f0.cx = c->f[G_CX];
        f0.cy = c->f[G_CY];
        f0.dinv = c->f[G_DINV];
        f0.b = c->f[G_R];
        f0.x = c->f[G_Z];
        f0.xt = c->f[G_ZT];
        c->mg32.push_back(f0);
    }
    std::vector<double> cx = hc.cx, cy = hc.cy, dinv = hc.dinv;
    std::vector<std::vector<float>> keep;  // float copies in flight
    int nx = c->g.nx, ny = c->g.ny;
    for (size_t l = 1; l < w.mgL.size(); ++l) {
        const Layout &Lc = w.mgL[l];
        std::vector<double> cxc, cyc, dic;
        coarsen_poisson(nx, ny, cx, cy, dinv, Lc.nx, Lc.ny, cxc, cyc, dic);
        ccns_ctx::Level lv;
        lv.L = Lc;
        lv.d = make_dims(Lc, 1, PTY);
        const size_t ab = align_up(Lc.n * sizeof(double), 256);
        char *base = c->base + w.mg_off[l];
        double **dst[MG_ARRS] = {&lv.cx, &lv.cy, &lv.dinv, &lv.b, &lv.x, &lv.xt};
        for (int k = 0; k < MG_ARRS; ++k) *dst[k] = (double *)(base + k * ab);
        const size_t Wc = Lc.nx + 2;
        const std::vector<double> *src[3] = {&cxc, &cyc, &dic};
        double *dd[3] = {lv.cx, lv.cy, lv.dinv};
        for (int k = 0; k < 3; ++k)
            HIPCHK(c, hipMemcpy2DAsync(dd[k], Lc.pitch * sizeof(double), src[k]->data(), Wc * sizeof(double),
                                       Wc * sizeof(double), Lc.ny + 2, hipMemcpyHostToDevice, c->stream));
        c->mg.push_back(lv);
        if (mix) {
            ccns_ctx::LevelT<float> fv;
            fv.L = Lc;
            fv.d = lv.d;
            const size_t ab32 = align_up(Lc.n * sizeof(float), 256);
            char *b32 = c->base + w.mg32_off[l];
            float **d32[MG_ARRS] = {&fv.cx, &fv.cy, &fv.dinv, &fv.b, &fv.x, &fv.xt};
            for (int k = 0; k < MG_ARRS; ++k) *d32[k] = (float *)(b32 + k * ab32);
            float *df[3] = {fv.cx, fv.cy, fv.dinv};
            for (int k = 0; k < 3; ++k) {
                keep.emplace_back(src[k]->begin(), src[k]->end());
                HIPCHK(c, hipMemcpy2DAsync(df[k], Lc.pitch * sizeof(float), keep.back().data(), Wc * sizeof(float),
                                           Wc * sizeof(float), Lc.ny + 2, hipMemcpyHostToDevice, c->stream));
            }
            c->mg32.push_back(fv);
        }
        cx.swap(cxc);
        cy.swap(cyc);
        dinv.swap(dic);
        nx = Lc.nx;
        ny = Lc.ny;
    }
    // coarsest grid: dense operator on its unknowns and its pseudo-inverse
    const Layout &Lc = c->mg.back().L;
    const size_t Wc = nx + 2;
    std::vector<int> idx, pos((size_t)(ny + 2) * Wc, -1);
    for (int j = 1; j <= ny; ++j)
        for (int i = 1; i <= nx; ++i)
            if (dinv[(size_t)j * Wc + i] > 0.0) {
                pos[(size_t)j * Wc + i] = (int)idx.size();
                idx.push_back(j * Lc.pitch + i);
            }
    const int n = (int)idx.size();
    if (n > 1024) return fail(c, CCNS_EINVAL, "coarsest multigrid grid too large");
    std::vector<double> A((size_t)n * n, 0.0);
    for (int j = 1; j <= ny; ++j)
        for (int i = 1; i <= nx; ++i) {
            const size_t k = (size_t)j * Wc + i;
            const int r = pos[k];
            if (r < 0) continue;
            const double ce = cx[k], cw = cx[k - 1], cn = cy[k], cs = cy[k - Wc];
            A[(size_t)r * n + r] = ce + cw + cn + cs;
            if (ce > 0 && pos[k + 1] >= 0) A[(size_t)r * n + pos[k + 1]] = -ce;
            if (cw > 0 && pos[k - 1] >= 0) A[(size_t)r * n + pos[k - 1]] = -cw;
            if (cn > 0 && pos[k + Wc] >= 0) A[(size_t)r * n + pos[k + Wc]] = -cn;
            if (cs > 0 && pos[k - Wc] >= 0) A[(size_t)r * n + pos[k - Wc]] = -cs;
        }
    std::vector<double> Pinv = pseudo_inverse_spsd(A, n);
    c->pinv = (double *)(c->base + w.pinv_off);
    c->pidx = (int *)(c->base + w.idx_off);
    c->ncoarse_act = n;
    if (n > 0) {
        HIPCHK(c, hipMemcpyAsync(c->pinv, Pinv.data(), Pinv.size() * sizeof(double), hipMemcpyHostToDevice,
                                 c->stream));
        HIPCHK(c, hipMemcpyAsync(c->pidx, idx.data(), idx.size() * sizeof(int), hipMemcpyHostToDevice, c->stream));
    }
    // the host vectors above are released when this returns: wait for the copies
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return CCNS_OK;
}

// First level of the fused coarse end of the cycle: the first level (after
// the finest) of at most TAIL_CELLS cells.
constexpr long TAIL_CELLS = 64 * 32;
template <class T>
size_t tail_start(const std::vector<ccns_ctx::LevelT<T>> &mg) {
    for (size_t l = 1; l < mg.size(); ++l)
        if ((long)mg[l].L.nx * mg[l].L.ny <= TAIL_CELLS && mg.size() - l <= (size_t)MAX_TAIL) return l;
    return mg.size() - 1;
}

// The cycle levels (those with down- and up-sweep kernels, above the
// LDS-resident coarse end) of a hierarchy.
template <class T>
size_t cycle_levels(const std::vector<ccns_ctx::LevelT<T>> &mg) {
    return mg.size() > 1 ? tail_start(mg) : 0;
}

// The finest level's up-sweep writes the statistics of z per work-group, so
// its tiles fix the order of those sums: it keeps 64 x MTY tiles (forms 1-3),
// and every form then gives the same bits.
bool mg_forms_valid(unsigned long long forms) {
    for (int l = 0; l < MG_FORM_LEVELS; ++l)
        for (int h = 0; h < 2; ++h)
            if (((forms >> (2 * MG_FORM_BITS * l + MG_FORM_BITS * h)) & 7u) > MGF_STAGED_LDS_HALF) return false;
    const unsigned up0 = (forms >> MG_FORM_BITS) & 7u;
    if (up0 == MGF_PLAIN_SHORT || up0 == MGF_STAGED_LDS_HALF) return false;
    return forms >> (2 * MG_FORM_BITS * MG_FORM_LEVELS) == 0;
}

// Each level's forms: the requested ones, and where none is given (0) the
// default: below the finest level, 64 x MTY_SMALL tiles where 64 x MTY ones
// would give fewer than MG_SMALL_GROUPS work-groups; otherwise the staged
// forms, except the FP32 way down, which is faster pointwise at every level.
template <class T>
void resolve_mg_forms(ccns_ctx *c, const std::vector<ccns_ctx::LevelT<T>> &mg, unsigned long long forms) {
    const int dbl = sizeof(T) == 8;
    for (size_t l = 0; l < 16; ++l) {
        int fd = MGF_AUTO, fu = MGF_AUTO;
        if (l < (size_t)MG_FORM_LEVELS) {
            fd = (int)((forms >> (2 * MG_FORM_BITS * l)) & 7u);
            fu = (int)((forms >> (2 * MG_FORM_BITS * l + MG_FORM_BITS)) & 7u);
        }
        if (l < mg.size()) {
            const int gx = (mg[l].L.nx + TX - 1) / TX;
            const bool small = l >= 1 && gx * ((mg[l].L.ny + MTY - 1) / MTY) < MG_SMALL_GROUPS;
            if (fd == MGF_AUTO) fd = small ? MGF_PLAIN_SHORT : (dbl ? MGF_STAGED : MGF_PLAIN);
            if (fu == MGF_AUTO) fu = small ? MGF_PLAIN_SHORT : MGF_STAGED;
        }
        c->mgf[dbl][0][l] = (unsigned char)fd;
        c->mgf[dbl][1][l] = (unsigned char)fu;
    }
}

// Work-groups of a cycle kernel of the given form on a level of nx x ny
// cells (one tile of 64 x the form's rows each, a multiple of 8 groups).
int mg_form_groups(int nx, int ny, int form) {
    const int ty = form == MGF_PLAIN_SHORT ? MTY_SMALL : form == MGF_STAGED_LDS_HALF ? MTY / 2 : MTY;
    const int gx = (nx + TX - 1) / TX;
    return ((gx * ((ny + ty - 1) / ty) + 7) / 8) * 8;
}

// z = V(b) on level l of a hierarchy; returns the array holding the result.
// On level 0 the last kernel also writes the residual statistics, reduced to
// one group in PB_MG.  Every kernel returns at once when *done is set (a
// cycle launched after the solve stopped).
template <class T>
T *vcycle(ccns_ctx *c, std::vector<ccns_ctx::LevelT<T>> &mg, size_t l, const T *b, const int *done) {
    ccns_ctx::LevelT<T> &L = mg[l];
    hipStream_t s = c->stream;
    if (l + 1 == mg.size()) {
        k_mg_coarsest<T><<<1, NT, 0, s>>>(c->ncoarse_act, c->pidx, c->pinv, b, L.x, done);
        return L.x;
    }
    if (l >= 1 && l == tail_start(mg)) {
        // b is this level's b array (written by the restriction above)
        TailDesc<T> d{};
        d.nlev = (int)(mg.size() - l);
        for (int t = 0; t < d.nlev; ++t) {
            ccns_ctx::LevelT<T> &M = mg[l + t];
            d.lv[t] = TailLevel<T>{M.cx, M.cy, M.dinv, M.b, M.x, M.xt, M.L.nx, M.L.ny, M.L.pitch};
        }
        d.ncoarse = c->ncoarse_act;
        d.idx = c->pidx;
        d.pinv = c->pinv;
        d.done = done;
        d.out = d.nlev >= 2 ? L.xt : L.x;
        size_t elems = 0;
        for (int t = 0; t < d.nlev; ++t) {
            d.lofs[t] = (int)elems;
            elems += 6 * (size_t)(d.lv[t].nx + 2) * (d.lv[t].ny + 2);
        }
        if (elems * sizeof(T) <= (size_t)c->tail_lds)
            k_mg_tail_lds<T><<<1, TT, elems * sizeof(T), s>>>(d);
        else
            k_mg_tail<T><<<1, TT, 0, s>>>(d);
        return d.out;
    }
    PoisCoefT<T> pc{L.cx, L.cy, L.dinv};
    const int gx = (L.L.nx + TX - 1) / TX;
    ccns_ctx::LevelT<T> &C = mg[l + 1];
    const int fd = c->mgf[sizeof(T) == 8][0][l], fu = c->mgf[sizeof(T) == 8][1][l];
    const int nbd = mg_form_groups(L.L.nx, L.L.ny, fd), nbu = mg_form_groups(L.L.nx, L.L.ny, fu);
    switch (fd) {
    case MGF_STAGED:
        k_mg_down_staged<T><<<nbd, NT, 0, s>>>(L.L.nx, L.L.ny, L.L.pitch, gx, pc, b, L.x, C.L.pitch, C.L.nx,
                                               C.L.ny, C.dinv, C.b, done);
        break;
    case MGF_STAGED_LDS:
        k_mg_down_lds<T, MTY><<<nbd, NT, 0, s>>>(L.L.nx, L.L.ny, L.L.pitch, gx, pc, b, L.x, C.L.pitch, C.L.nx,
                                                 C.L.ny, C.dinv, C.b, done);
        break;
    case MGF_STAGED_LDS_HALF:
        k_mg_down_lds<T, MTY / 2><<<nbd, NT, 0, s>>>(L.L.nx, L.L.ny, L.L.pitch, gx, pc, b, L.x, C.L.pitch, C.L.nx,
                                                     C.L.ny, C.dinv, C.b, done);
        break;
    case MGF_PLAIN:
        k_mg_down<T><<<nbd, NT, 0, s>>>(L.L.nx, L.L.ny, L.L.pitch, gx, pc, b, L.x, C.L.pitch, C.L.nx, C.L.ny,
                                        C.dinv, C.b, done);
        break;
    default:
        k_mg_down<T, MTY_SMALL><<<nbd, NT, 0, s>>>(L.L.nx, L.L.ny, L.L.pitch, gx, pc, b, L.x, C.L.pitch, C.L.nx,
                                                   C.L.ny, C.dinv, C.b, done);
    }
    const T *xc = vcycle<T>(c, mg, l + 1, C.b, done);
    // on level 0 the up-sweep also writes the statistics of z, reduced to PB_MG
    auto up = [&](auto stats) {
        constexpr bool S = decltype(stats)::value;
        double *po = S ? c->part[PB_UPD] : nullptr;
        switch (fu) {
        case MGF_STAGED:
            k_mg_up_staged<T, S><<<nbu, NT, 0, s>>>(L.L.nx, L.L.ny, L.L.pitch, gx, pc, b, L.x, xc, C.L.pitch, L.xt,
                                                    po, nbu, done);
            break;
        case MGF_STAGED_LDS:
            k_mg_up_lds<T, S, MTY><<<nbu, NT, 0, s>>>(L.L.nx, L.L.ny, L.L.pitch, gx, pc, b, L.x, xc, C.L.pitch, L.xt,
                                                      po, nbu, done);
            break;
        case MGF_STAGED_LDS_HALF:
            k_mg_up_lds<T, S, MTY / 2><<<nbu, NT, 0, s>>>(L.L.nx, L.L.ny, L.L.pitch, gx, pc, b, L.x, xc, C.L.pitch,
                                                          L.xt, po, nbu, done);
            break;
        case MGF_PLAIN:
            k_mg_up<T, S><<<nbu, NT, 0, s>>>(L.L.nx, L.L.ny, L.L.pitch, gx, pc, b, L.x, xc, C.L.pitch, L.xt, po,
                                             nbu, done);
            break;
        default:
            k_mg_up<T, S, MTY_SMALL><<<nbu, NT, 0, s>>>(L.L.nx, L.L.ny, L.L.pitch, gx, pc, b, L.x, xc, C.L.pitch,
                                                        L.xt, po, nbu, done);
        }
    };
    if (l == 0) {
        up(std::true_type{});
        k_reduce_partials<4><<<1, NT, 0, s>>>(c->part[PB_UPD], nbu, c->part[PB_MG]);
    } else {
        up(std::false_type{});
    }
    return L.xt;
}

// Multigrid-preconditioned CG on A x = f, the residual r of the start value
// x being given.  pinit: partials whose slot 0 is |f|^2 (ninit groups), or
// NULL when r is f itself (zero start value).
template <class T>
ccns_status mg_cg(ccns_ctx *c, std::vector<ccns_ctx::LevelT<T>> &mg, PoisCoefT<T> pc, CgState *st, T *x, T *r,
                  T *p0, T *p1, T *q, const double *pinit, int ninit, int &last_it, ccns_solve_info *info) {
    const Dims &dp = c->dp;
    const size_t ntot = c->w.L.n;
    const int nl = update_blocks(ntot);
    T *pb[2] = {p0, p1};
    int &pbuf = c->pbuf_pois;
    T *z = vcycle<T>(c, mg, 0, r, &st->done);
    int chunk = std::max(2, last_it + 1);
    int it = 0;
    for (;;) {
        for (int u = 0; u < chunk; ++u, ++it) {
            const int par = it & 1;
            const bool tm = c->timing && (it % 8 == 4) && it < last_it;
            launch(c, tm, 0, it, k_pois_dir_z<T>, dim3(dp.nblk), dim3(NT), dp, pc, (const T *)z, (const T *)pb[pbuf],
                   pb[pbuf ^ 1], q, st, it == 0 ? 1 : 0, par, (const double *)c->part[PB_MG], 1, pinit, ninit,
                   c->part[PB_DIR]);
            launch(c, tm, 1, it, k_cg_update<T, false>, dim3(nl), dim3(UT), ntot, nl, pc.dinv, x, r,
                   (const T *)pb[pbuf ^ 1], (const T *)q, st, par, (const double *)c->part[PB_DIR], dp.nblk,
                   c->part[PB_UPD]);
            pbuf ^= 1;
            z = vcycle<T>(c, mg, 0, r, &st->done);
        }
        HIPCHK(c, hipGetLastError());
        HIPCHK(c, hipMemcpyAsync(c->h_st, st, sizeof(CgState), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        if (c->h_st->done) break;
        chunk = 2;
    }
    last_it = c->h_st->it_final;
    if (c->timing) harvest_events(c, c->h_st->it_final);
    if (info) {
        info->iterations = c->h_st->it_final;
        info->outer = 1;
        info->rel_residual = c->h_st->fnorm2 > 0 ? std::sqrt(c->h_st->rnorm2_final / c->h_st->fnorm2) : 0.0;
        info->status = c->h_st->status;
        info->inner_status = CCNS_OK;
        info->inner_fail_sweep = -1;
    }
    return (ccns_status)c->h_st->status;
}

// Pressure solve (precision 0, multigrid); b is in A_B with its sum's
// partials in PB_RHS (nin groups); the start value is A_PHI.
ccns_status pressure_solve_mg(ccns_ctx *c, int nin, ccns_solve_info *info) {
    PoisCoef pc = pois_coef(c);
    k_pois_init<false><<<c->dc.nblk, NT, 0, c->stream>>>(c->dc, pc, c->a[A_B], c->a[A_PHI], c->a[A_R], c->st_pois,
                                                         c->part[PB_RHS], nin, c->part[PB_INIT], nullptr, nullptr,
                                                         nullptr);
    return mg_cg<double>(c, c->mg, pc, c->st_pois, c->a[A_PHI], c->a[A_R], c->a[A_P0], c->a[A_P1], c->a[A_Q],
                         c->part[PB_INIT], c->dc.nblk, c->last_pois_it, info);
}

// Limits of the refinement loops of precision 1.
constexpr int MAX_OUTER = 20;
constexpr double INNER_TOL_MIN = 1e-5, INNER_TOL_MAX = 0.1;

double inner_tol(double reduction) {
    if (!(reduction > 0.0)) return INNER_TOL_MAX;  // also a NaN
    return std::min(INNER_TOL_MAX, std::max(INNER_TOL_MIN, 0.5 * reduction));
}

ccns_status read_outer(ccns_ctx *c, const double *src, int n) {
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipMemcpyAsync(c->h_outer, src, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return CCNS_OK;
}

// Statuses of the inner solves of a refinement loop: the worst one (a
// breakdown before a solve that hit its iteration limit) and the first sweep
// whose inner solve did not converge (-1: every one converged).
struct InnerRecord {
    ccns_status status = CCNS_OK;
    int sweep = -1;
};
void note_inner(InnerRecord &r, int status, int sweep) {
    if (status == CCNS_OK) return;
    if (r.sweep < 0) r.sweep = sweep;
    if (r.status == CCNS_OK || status == CCNS_EBREAKDOWN) r.status = (ccns_status)status;
}

// Pressure solve in precision 1: iterative refinement.  Each sweep forms the
// residual r = f - A phi in FP64 (FP64 coefficients), solves A d = r in float
// (float coefficients and vectors, FP64 dot products) to a relative
// tolerance, and adds d to phi in FP64.  Stops when max |cont(U^{n+1}, D)|
// / (u_ref h) = (tau/rho) max |r| / (u_ref h) is at most div_tol / 2 (div_tol
// > 0), else when |r|_2 <= pcg_tol |f|_2.
ccns_status pressure_solve_mixed(ccns_ctx *c, int nin, ccns_solve_info *info) {
    PoisCoef pc = pois_coef(c);
    PoisCoefT<float> pf{c->f[G_CX], c->f[G_CY], c->f[G_DINV]};
    const ccns_params &p = c->prm;
    const double sdiv = (p.tau / p.rho) / (p.u_ref * std::min(c->g.hx, c->g.hy));
    double bn2 = 0.0, rn2 = 0.0;
    int inner_its = 0, sweeps = 0;
    InnerRecord inner;
    ccns_status st = CCNS_ENOTCONV;
    for (int o = 0;; ++o) {
        k_pois_init<true><<<c->dc.nblk, NT, 0, c->stream>>>(c->dc, pc, c->a[A_B], c->a[A_PHI], nullptr,
                                                            c->st_pois_in, o == 0 ? c->part[PB_RHS] : nullptr, nin,
                                                            c->part[PB_INIT], c->f[G_R], c->f[G_X], c->f[G_DINV]);
        c->init_nblk = c->dc.nblk;
        k_reduce_partials<7, 1><<<1, NT, 0, c->stream>>>(c->part[PB_INIT], c->dc.nblk, c->outer);
        ccns_status s = read_outer(c, c->outer, 8);
        if (s != CCNS_OK) return s;
        if (o == 0) bn2 = c->h_outer[5];
        rn2 = c->h_outer[6];
        const double rmax = c->h_outer[7];
        double need;  // reduction of the residual still needed
        bool conv;
        if (p.div_tol > 0.0) {
            conv = sdiv * rmax <= 0.5 * p.div_tol;
            need = rmax > 0.0 ? 0.5 * p.div_tol / (sdiv * rmax) : 1.0;
        } else {
            conv = rn2 <= p.pcg_tol * p.pcg_tol * bn2;
            need = rn2 > 0.0 ? p.pcg_tol * std::sqrt(bn2 / rn2) : 1.0;
        }
        if (!(bn2 > 0.0) || c->n_active == 0) conv = true;
        if (conv) {
            st = CCNS_OK;
            break;
        }
        if (o >= MAX_OUTER) break;
        const double it = inner_tol(need);
        k_set_tol<<<1, 1, 0, c->stream>>>(c->st_pois_in, it * it);
        ccns_solve_info si{};
        if (p.precond == 1)
            mg_cg<float>(c, c->mg32, pf, c->st_pois_in, c->f[G_X], c->f[G_R], c->f[G_P0], c->f[G_P1], c->f[G_Q],
                         nullptr, 0, c->last_pois_in, &si);
        else
            jacobi_cg<float>(c, pf, c->st_pois_in, c->f[G_X], c->f[G_R], c->f[G_P0], c->f[G_P1], c->f[G_Q],
                             c->last_pois_in, &si);
        if (si.status == CCNS_EDEVICE) return CCNS_EDEVICE;
        inner_its += si.iterations;
        ++sweeps;
        note_inner(inner, si.status, o);
        // an inner solve that broke down before its first update leaves the
        // correction at zero: the next sweep would start from the same state
        if (si.status == CCNS_EBREAKDOWN && si.iterations == 0) {
            st = CCNS_EBREAKDOWN;
            break;
        }
        k_add_correction<<<flat_blocks(c->w.L.n), NT, 0, c->stream>>>(c->w.L.n, c->a[A_PHI], c->f[G_X]);
    }
    c->last_pois_it = inner_its;
    if (info) {
        info->iterations = inner_its;
        info->outer = sweeps;
        info->rel_residual = bn2 > 0.0 ? std::sqrt(rn2 / bn2) : 0.0;
        info->status = st;
        info->inner_status = inner.status;
        info->inner_fail_sweep = inner.sweep;
    }
    return st;
}

// Pressure solve on b in A_B (partials of its sum in PB_RHS), by precision
// and preconditioner.
ccns_status pressure_solve_any(ccns_ctx *c, int nin, ccns_solve_info *info) {
    if (c->prm.precision == 1) return pressure_solve_mixed(c, nin, info);
    return c->prm.precond == 1 ? pressure_solve_mg(c, nin, info) : pressure_solve_dev(c, nin, info);
}

// conv^n and the predictor right-hand side; U* := U^n.
void predictor_rhs(ccns_ctx *c) {
    PredCoefT<double> pc = pred_coef_t(c);
    const Layout &L = c->w.L;
    const int gx = L.pitch / TX, gy = (L.rows + HTY - 1) / HTY;
    const int nb = ((gx * gy + 7) / 8) * 8;
    if (c->ncls) {
        pc.cls = c->cls;
        pc.tab = c->tab;
    }
    const bool geo = c->prm.visc_form == 0;
    auto k = c->ncls ? (geo ? k_pred_rhs<true, true> : k_pred_rhs<false, true>)
                     : (geo ? k_pred_rhs<true, false> : k_pred_rhs<false, false>);
    k<<<nb, NT, 0, c->stream>>>(L.pitch, L.rows, gx, gy, L.n, pc, c->a[A_AX], c->a[A_AY], c->a[A_HBX], c->a[A_HBY],
                                c->a[A_DX], c->a[A_DY], c->a[A_UX], c->a[A_UY], c->a[A_P], c->a[A_VDX], c->a[A_VDY],
                                c->a[A_CONVX], c->a[A_CONVY], c->a[A_RHSX], c->a[A_USX], c->prm.rho, c->prm.gx,
                                c->prm.gy, c->conv_valid, outflow_desc(c));
    c->conv_valid = 1;
}

// Jacobi-PCG on H x = f with storage type T, one k_pred_cg launch and one
// reduction of its partials (to PRED_RED sets) per iteration; the residual
// kernel's statistics are in PB_INIT (one group), its residual in r[0].
// Launches are issued in chunks between looks at the device's stopping flag.
template <class T>
ccns_status pred_cg(ccns_ctx *c, PredCoefT<T> pc, CgState *st, T *x, T *const r[2], T *const p[2],
                    T *const q[2], int &last_it, ccns_solve_info *info) {
    c->init_nblk = 1;
    const Layout &L = c->w.L;
    const int gx = L.pitch / TX, gy = (L.rows + pred_rows<T>() - 1) / pred_rows<T>();
    const int nb = ((gx * gy + 7) / 8) * 8;
    const bool geo = c->prm.visc_form == 0;
    auto kern = pc.cls ? (geo ? k_pred_cg<T, true, true> : k_pred_cg<T, false, true>)
                       : (geo ? k_pred_cg<T, true, false> : k_pred_cg<T, false, false>);
    int chunk = std::max(4, last_it + 1);
    int it = 0;
    for (;;) {
        for (int u = 0; u < chunk; ++u, ++it) {
            const int b = it & 1, a = b ^ 1;
            const T *rin = it == 0 ? r[0] : r[a];
            const double *tin = it == 0 ? c->part[PB_INIT] : c->part[PB_UPD];
            const int nin = it == 0 ? c->init_nblk : PRED_RED;
            const bool tm = c->timing && (it % 8 == 4) && it < last_it;
            launch(c, tm, 2, it, kern, dim3(nb), dim3(NT), L.pitch, L.rows, gx,
                   gy, L.n, pc, st, it, x, rin, r[b], (const T *)p[a], p[b], (const T *)q[a], q[b], tin, nin,
                   c->part[PB_DIR]);
            launch(c, tm, 3, it, k_reduce_partials_split<7>, dim3(PRED_RED), dim3(NT), (const double *)c->part[PB_DIR],
                   nb, c->part[PB_UPD]);
        }
        HIPCHK(c, hipGetLastError());
        HIPCHK(c, hipMemcpyAsync(c->h_st, st, sizeof(CgState), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        if (c->h_st->done) break;
        chunk = 8;
    }
    last_it = c->h_st->it_final;
    if (c->timing) harvest_events(c, c->h_st->it_final);
    if (info) {
        info->iterations = c->h_st->it_final;
        info->outer = 1;
        info->rel_residual = c->h_st->fnorm2 > 0 ? std::sqrt(std::max(c->h_st->rnorm2_final, 0.0) / c->h_st->fnorm2)
                                                 : 0.0;
        info->status = c->h_st->status;
        info->inner_status = CCNS_OK;
        info->inner_fail_sweep = -1;
    }
    return (ccns_status)c->h_st->status;
}

// r = rhs - H x in FP64 (tiled residual kernel), its statistics reduced to
// one group in PB_INIT (NS = 5, or 7 with MIX).
template <bool MIX>
void pred_residual(ccns_ctx *c, CgState *st) {
    PredCoefT<double> pd = pred_coef_t(c);
    const Layout &L = c->w.L;
    const int gx = L.pitch / TX, gy = (L.rows + HTY - 1) / HTY;
    const int nb = ((gx * gy + 7) / 8) * 8;
    float *r32 = MIX ? c->f[G_PRX] : nullptr, *x32 = MIX ? c->f[G_PXX] : nullptr;
    const float *hd32 = MIX ? c->f[G_HDX] : nullptr;
    if (c->ncls) {
        pd.cls = c->cls;
        pd.tab = c->tab;
    }
    const bool geo = c->prm.visc_form == 0;
    auto kern = c->ncls ? (geo ? k_pred_resid<MIX, true, true> : k_pred_resid<MIX, false, true>)
                        : (geo ? k_pred_resid<MIX, true, false> : k_pred_resid<MIX, false, false>);
    kern<<<nb, NT, 0, c->stream>>>(L.pitch, L.rows, gx, gy, L.n, pd, c->a[A_RHSX], c->a[A_USX], c->a[A_PRX], st,
                                   c->part[PB_RHS], r32, x32, hd32);
    if (MIX)
        k_reduce_partials<7><<<1, NT, 0, c->stream>>>(c->part[PB_RHS], nb, c->part[PB_INIT]);
    else
        k_reduce_partials<5><<<1, NT, 0, c->stream>>>(c->part[PB_RHS], nb, c->part[PB_INIT]);
}

ccns_status predict_dev(ccns_ctx *c, ccns_solve_info *info) {
    predictor_rhs(c);
    pred_residual<false>(c, c->st_pred);
    PredCoefT<double> pd = pred_coef_t(c);
    if (c->ncls) {
        pd.cls = c->cls;
        pd.tab = c->tab;
    }
    double *r[2] = {c->a[A_PRX], c->a[A_PR1X]}, *p[2] = {c->a[A_PP0X], c->a[A_PP1X]},
           *q[2] = {c->a[A_PQX], c->a[A_PQ1X]};
    return pred_cg<double>(c, pd, c->st_pred, c->a[A_USX], r, p, q, c->last_pred_it, info);
}

// Predictor in precision 1: iterative refinement as for the pressure, with
// the FP64 residual rhs - H U* and float inner Jacobi-PCG; stops when
// |r|_2 <= pred_tol |rhs|_2.
ccns_status predict_mixed(ccns_ctx *c, ccns_solve_info *info) {
    PredCoef pc = pred_coef(c);
    PredCoefT<float> pf{ViscCoefT<float>{c->f[G_BXX], c->f[G_BXY], c->f[G_BYY], c->f[G_BYX], c->f[G_WXX],
                                         c->f[G_WYY], c->f[G_NXX], c->f[G_NXY], c->f[G_NYX], c->f[G_NYY]},
                        c->f[G_VU], c->f[G_VV], c->f[G_HDX], c->f[G_HDY], pc.rt, pc.mu, nullptr, nullptr};
    if (c->ncls) {
        pf.cls = c->cls;
        pf.tab = c->tab32;
    }
    const double tol = c->prm.pred_tol;
    predictor_rhs(c);
    double fn2 = 0.0, rn2 = 0.0;
    int inner_its = 0, sweeps = 0;
    InnerRecord inner;
    ccns_status st = CCNS_ENOTCONV;
    for (int o = 0;; ++o) {
        pred_residual<true>(c, c->st_pred_in);
        ccns_status s = read_outer(c, c->part[PB_INIT], 7);
        if (s != CCNS_OK) return s;
        fn2 = c->h_outer[5];
        rn2 = c->h_outer[6];
        if (!(fn2 > 0.0) || rn2 <= tol * tol * fn2) {
            st = CCNS_OK;
            break;
        }
        if (o >= MAX_OUTER) break;
        const double it = inner_tol(tol * std::sqrt(fn2 / rn2));
        k_set_tol<<<1, 1, 0, c->stream>>>(c->st_pred_in, it * it);
        ccns_solve_info si{};
        float *r[2] = {c->f[G_PRX], c->f[G_PR1X]}, *p[2] = {c->f[G_PP0X], c->f[G_PP1X]},
              *q[2] = {c->f[G_PQX], c->f[G_PQ1X]};
        pred_cg<float>(c, pf, c->st_pred_in, c->f[G_PXX], r, p, q, c->last_pred_in, &si);
        if (si.status == CCNS_EDEVICE) return CCNS_EDEVICE;
        inner_its += si.iterations;
        ++sweeps;
        note_inner(inner, si.status, o);
        if (si.status == CCNS_EBREAKDOWN && si.iterations == 0) {
            st = CCNS_EBREAKDOWN;
            break;
        }
        k_add_correction<<<flat_blocks(2 * c->w.L.n), NT, 0, c->stream>>>(2 * c->w.L.n, c->a[A_USX], c->f[G_PXX]);
    }
    c->last_pred_it = inner_its;
    if (info) {
        info->iterations = inner_its;
        info->outer = sweeps;
        info->rel_residual = fn2 > 0.0 ? std::sqrt(rn2 / fn2) : 0.0;
        info->status = st;
        info->inner_status = inner.status;
        info->inner_fail_sweep = inner.sweep;
    }
    return st;
}

ccns_status predict_any(ccns_ctx *c, ccns_solve_info *info) {
    return c->prm.precision == 1 ? predict_mixed(c, info) : predict_dev(c, info);
}

ccns_status diag_dev(ccns_ctx *c, int update_p, ccns_step_info *info) {
    DiagCoef dc{c->a[A_AX], c->a[A_AY], c->a[A_HET], c->a[A_DINV], c->a[A_VUR], c->a[A_VVR],
                c->a[A_VU], c->a[A_VV], c->a[A_CX], c->a[A_CY], c->a[A_VINV]};
    const double pcoef = c->prm.tau * c->prm.mu / (2.0 * c->prm.rho);
    k_diag<<<c->dc.nblk, NT, 0, c->stream>>>(c->dc, dc, c->a[A_UX], c->a[A_UY], c->a[A_PHI], c->a[A_P], pcoef,
                                             update_p, c->prm.rho, c->part[PB_DIAG]);
    k_diag_final<<<1, NT, 0, c->stream>>>(c->part[PB_DIAG], c->dc.nblk, c->diag);
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
    k_pois_rhs<<<c->dc.nblk, NT, 0, c->stream>>>(c->dc, pc, c->a[A_AX], c->a[A_AY], c->a[A_HET], c->a[A_USX],
                                                 c->a[A_USY], c->a[A_B], c->prm.rho / c->prm.tau,
                                                 c->part[PB_RHS]);
    ccns_solve_info si{};
    ccns_status s = pressure_solve_any(c, c->dc.nblk, &si);
    if (info) info->poisson = si;
    k_correct<<<c->dc.nblk, NT, 0, c->stream>>>(c->dc, c->a[A_GX], c->a[A_GY], c->a[A_USX], c->a[A_USY],
                                                c->a[A_PHI], c->a[A_UX], c->a[A_UY], c->prm.tau / c->prm.rho);
    ccns_status s2 = diag_dev(c, update_p, info);
    if (s2 != CCNS_OK) return s2;
    return s;
}

// Clears n 8-byte words (the workspace at context creation: a kernel rather
// than a memset node, so that the clear orders like every other launch).
__global__ __launch_bounds__(NT) void k_zero(size_t n, unsigned long long *__restrict__ p) {
    for (size_t k = (size_t)blockIdx.x * NT + threadIdx.x; k < n; k += (size_t)gridDim.x * NT) p[k] = 0ull;
}

}  // namespace

// Workspace of the contexts that allocate nothing (ccns_ctx_create_static):
// one array per device, which the device holds until the process ends.  In
// host code `scratch` only names the symbol; its device address comes from
// hipGetSymbolAddress, once per device (static_workspace below).
constexpr size_t STATIC_WS_BYTES = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[STATIC_WS_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
struct StaticSlot {
    std::once_flag once;
    void *ptr = nullptr;           // device address of `scratch` on this device
    hipError_t err = hipSuccess;
    std::atomic<int> used{0};      // 1 while a context uses it
};
StaticSlot g_static[MAX_DEVICES];

void release_static(int dev) { g_static[dev].used.store(0); }

// Device address of the static workspace on the current device (taken once
// per device, with that device current), or null.
void *static_workspace(int dev) {
    StaticSlot &s = g_static[dev];
    std::call_once(s.once, [&] { s.err = hipGetSymbolAddress(&s.ptr, HIP_SYMBOL(scratch)); });
    return s.err == hipSuccess ? s.ptr : nullptr;
}

ccns_status create_ctx(const ccns_grid *grid, const ccns_params *params, const double *caps_host,
                       const double *dirichlet_host, void *dev_workspace, size_t ws_bytes, void *hip_stream,
                       int static_dev, ccns_ctx **out);

}  // namespace

extern "C" {

size_t ccns_workspace_bytes(const ccns_grid *grid, const ccns_params *params) {
    if (!grid || grid->nx < 2 || grid->ny < 2) return 0;
    return plan(grid->nx, grid->ny, params ? params->precision : 0).total;
}

const char *ccns_last_error(const ccns_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int ccns_coef_classes(const ccns_ctx *ctx) { return ctx ? ctx->ncls : -1; }

ccns_status ccns_ctx_create(const ccns_grid *grid, const ccns_params *params, const double *caps_host,
                            const double *dirichlet_host, void *dev_workspace, size_t ws_bytes, void *hip_stream,
                            ccns_ctx **out) {
    return create_ctx(grid, params, caps_host, dirichlet_host, dev_workspace, ws_bytes, hip_stream, -1, out);
}

ccns_status ccns_ctx_create_static(const ccns_grid *grid, const ccns_params *params, const double *caps_host,
                                   const double *dirichlet_host, void *hip_stream, ccns_ctx **out) {
    if (!out) return CCNS_EINVAL;
    *out = nullptr;
    if (!grid || !params || !caps_host || !dirichlet_host) return CCNS_EINVAL;
    const size_t need = ccns_workspace_bytes(grid, params);
    if (need == 0) return CCNS_EINVAL;
    if (need > STATIC_WS_BYTES) return CCNS_ENOMEM;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return CCNS_EDEVICE;
    void *ws = static_workspace(dev);
    if (!ws) return CCNS_EDEVICE;
    int expect = 0;
    if (!g_static[dev].used.compare_exchange_strong(expect, 1)) return CCNS_ESTATE;
    const ccns_status st = create_ctx(grid, params, caps_host, dirichlet_host, ws, STATIC_WS_BYTES, hip_stream,
                                      dev, out);
    if (st != CCNS_OK) g_static[dev].used.store(0);
    return st;
}

}  // extern "C"

namespace {

ccns_status create_ctx(const ccns_grid *grid, const ccns_params *params, const double *caps_host,
                       const double *dirichlet_host, void *dev_workspace, size_t ws_bytes, void *hip_stream,
                       int static_dev, ccns_ctx **out) {
    if (!out) return CCNS_EINVAL;
    *out = nullptr;
    if (!grid || !params || !caps_host || !dirichlet_host || !dev_workspace) return CCNS_EINVAL;
    if (params->precision < 0 || params->precision > 1 || params->precond < 0 || params->precond > 1 ||
        params->coef_tables < 0 || params->coef_tables > 1 || params->outflow < 0 || params->outflow > 15 ||
        !mg_forms_valid(params->mg_forms))
        return CCNS_EINVAL;
    ccns_ctx *c = new (std::nothrow) ccns_ctx();
    if (!c) return CCNS_ENOMEM;
    c->g = *grid;
    c->g.xf = c->g.yf = nullptr;   // the geometry is in the capacities; the abscissas are the caller's
    c->prm = *params;
    c->static_dev = static_dev;
    c->w = plan(grid->nx, grid->ny, params->precision);
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
    for (int k = 0; k < PB_COUNT; ++k) c->part[k] = (double *)(c->base + c->w.part_off + (size_t)k * c->w.part_bytes);
    c->st_pred = (CgState *)(c->base + c->w.state_off);
    c->st_pois = c->st_pred + 1;
    c->st_pred_in = c->st_pred + 2;
    c->st_pois_in = c->st_pred + 3;
    c->diag = (DiagState *)(c->st_pred + 4);
    c->outer = (double *)(c->base + c->w.state_off + 2048);
    for (int k = 0; k < G_COUNT; ++k)
        c->f[k] = params->precision == 1 ? (float *)(c->base + c->w.f32_off + (size_t)k * c->w.arr32_bytes) : nullptr;
    c->dc = make_dims(c->w.L, 1, TY);
    c->df = make_dims(c->w.L, 2, TY);
    c->dp = make_dims_1(c->w.L, 1, PTY);
    c->init_nblk = c->dc.nblk;
    c->conv_valid = 0;
    c->last_pois_it = c->last_pred_it = 16;
    c->last_pois_in = c->last_pred_in = 8;
    c->pbuf_pois = 0;
    c->timing = 0;
    {
        // LDS for the coarse end of the cycle: what one work-group may hold,
        // less the kernel's static arrays
        int dev = 0, lmax = 0;
        c->tail_lds = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&lmax, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
            lmax > 16384) {
            const int dyn = lmax - 16384;
            if (hipFuncSetAttribute((const void *)k_mg_tail_lds<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    dyn) == hipSuccess &&
                hipFuncSetAttribute((const void *)k_mg_tail_lds<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    dyn) == hipSuccess)
                c->tail_lds = dyn;
        }
        (void)hipGetLastError();
    }
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
    if (static_dev >= 0) {
        // no allocation: the host copies of the solver state live in the
        // context record (the device-to-host copies then go through pageable
        // memory, and the calls wait for them as they do for pinned memory)
        c->h_st = &c->st_host;
        c->h_diag = &c->diag_host;
        c->h_outer = c->outer_host;
    } else if (hipHostMalloc((void **)&c->h_st, sizeof(CgState)) != hipSuccess ||
               hipHostMalloc((void **)&c->h_diag, sizeof(DiagState)) != hipSuccess ||
               hipHostMalloc((void **)&c->h_outer, 8 * sizeof(double)) != hipSuccess) {
        destroy_ctx(c, false);
        return CCNS_EDEVICE;
    }
    // zero the whole workspace (it is a multiple of 256 bytes), then upload
    // the coefficient fields
    k_zero<<<flat_blocks(c->w.total / 8), NT, 0, c->stream>>>(c->w.total / 8, (unsigned long long *)c->base);
    if (hipGetLastError() != hipSuccess) {
        destroy_ctx(c, false);
        return CCNS_EDEVICE;
    }
    const std::vector<double> *src[] = {&hc.cx, &hc.cy, &hc.dinv, &hc.gx, &hc.gy, &hc.ax, &hc.ay, &hc.het,
                                        &hc.hbx, &hc.hby, &hc.dx, &hc.dy, &hc.vu, &hc.vv, &hc.bxx, &hc.bxy,
                                        &hc.byy, &hc.byx, &hc.wxx, &hc.wyy, &hc.nxx, &hc.nxy, &hc.nyx, &hc.nyy,
                                        &hc.hdx, &hc.hdy, &hc.vinv, &hc.vur, &hc.vvr, &hc.vdx, &hc.vdy};
    for (int k = 0; k <= A_VDY; ++k) {
        if ((s = to_dev(c, c->a[k], src[k]->data(), hipMemcpyHostToDevice)) != CCNS_OK) {
            destroy_ctx(c, false);
            return s;
        }
    }
    if (params->precision == 1) {
        // float copies of the coefficients of the inner solves
        const std::vector<double> *s32[] = {&hc.cx, &hc.cy, &hc.dinv};
        const int d32[] = {G_CX, G_CY, G_DINV};
        const std::vector<double> *p32[] = {&hc.vu, &hc.vv, &hc.bxx, &hc.bxy, &hc.byy, &hc.byx, &hc.wxx, &hc.wyy,
                                            &hc.nxx, &hc.nxy, &hc.nyx, &hc.nyy, &hc.hdx, &hc.hdy};
        const int q32[] = {G_VU, G_VV, G_BXX, G_BXY, G_BYY, G_BYX, G_WXX, G_WYY, G_NXX, G_NXY, G_NYX, G_NYY,
                           G_HDX, G_HDY};
        std::vector<float> tmp;
        const size_t W = grid->nx + 2;
        auto up32 = [&](float *dst, const std::vector<double> &v) {
            tmp.assign(v.begin(), v.end());
            return hipMemcpy2DAsync(dst, c->w.L.pitch * sizeof(float), tmp.data(), W * sizeof(float),
                                    W * sizeof(float), grid->ny + 2, hipMemcpyHostToDevice, c->stream) == hipSuccess &&
                   hipStreamSynchronize(c->stream) == hipSuccess;
        };
        bool ok = true;
        for (int k = 0; k < 3 && ok; ++k) ok = up32(c->f[d32[k]], *s32[k]);
        for (int k = 0; k < 14 && ok; ++k) ok = up32(c->f[q32[k]], *p32[k]);
        if (!ok) {
            destroy_ctx(c, false);
            return CCNS_EDEVICE;
        }
    }
    // state: U = D everywhere (the caller sets the initial field), P = Phi = 0
    to_dev(c, c->a[A_UX], hc.dx.data(), hipMemcpyHostToDevice);
    to_dev(c, c->a[A_UY], hc.dy.data(), hipMemcpyHostToDevice);
    if (params->precond == 1 && (s = mg_setup(c, hc)) != CCNS_OK) {
        destroy_ctx(c, false);
        return s;
    }
    resolve_mg_forms<double>(c, c->mg, params->mg_forms);
    resolve_mg_forms<float>(c, c->mg32, params->mg_forms);
    if ((s = pred_classes(c, hc)) != CCNS_OK) {
        destroy_ctx(c, false);
        return s;
    }
    // force tables: kept only when they fit the workspace's share
    c->ftab = (double *)(c->base + c->w.force_off);
    c->fsum = c->ftab + (size_t)2 * c->w.force_cap * FORCE_W;
    c->nfc = (int)(hc.fcell.size() / FORCE_W);
    c->nfn = (int)(hc.fnode.size() / FORCE_W);
    if (c->nfc > c->w.force_cap || c->nfn > c->w.force_cap) {
        c->nfc = c->nfn = -1;
    } else {
        // (the host rows live until the synchronisation below)
        hipError_t e1 = hipSuccess, e2 = hipSuccess;
        if (c->nfc)
            e1 = hipMemcpyAsync(c->ftab, hc.fcell.data(), hc.fcell.size() * sizeof(double), hipMemcpyHostToDevice,
                                c->stream);
        if (c->nfn)
            e2 = hipMemcpyAsync(c->ftab + (size_t)c->w.force_cap * FORCE_W, hc.fnode.data(),
                                hc.fnode.size() * sizeof(double), hipMemcpyHostToDevice, c->stream);
        if (e1 != hipSuccess || e2 != hipSuccess) {
            (void)hipStreamSynchronize(c->stream);
            destroy_ctx(c, false);
            return CCNS_EDEVICE;
        }
    }
    set_cg(c, c->st_pred, params->pred_tol, params->pred_maxit, 0, hc.n_uact + hc.n_vact);
    // with outflow faces the pressure beyond them is held: not singular
    const int singular = hc.n_out == 0;
    set_cg(c, c->st_pois, params->pcg_tol, params->pcg_maxit, singular, hc.n_active);
    set_cg(c, c->st_pred_in, INNER_TOL_MIN, params->pred_maxit, 0, hc.n_uact + hc.n_vact);
    set_cg(c, c->st_pois_in, INNER_TOL_MIN, params->pcg_maxit, singular, hc.n_active);
    if (hipStreamSynchronize(c->stream) != hipSuccess) {
        destroy_ctx(c, false);
        return CCNS_EDEVICE;
    }
    *out = c;
    return CCNS_OK;
}

}  // namespace

extern "C" {

void ccns_ctx_destroy(ccns_ctx *ctx) { destroy_ctx(ctx, true); }

static const int kFieldArr[CCNS_NFIELDS] = {A_UX, A_UY, A_P, A_PHI, A_CONVX, A_CONVY, A_USX, A_USY, A_B};

ccns_status ccns_field_set(ccns_ctx *c, int field, const double *src, int is_device) {
    if (!c || !src || field < 0 || field >= CCNS_NFIELDS) return fail(c, CCNS_EINVAL, "bad field");
    ccns_status s = to_dev(c, c->a[kFieldArr[field]], src, is_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice);
    if (s != CCNS_OK) return s;
    if (field == CCNS_F_CONVX || field == CCNS_F_CONVY) c->conv_valid = 1;
    if (field == CCNS_F_UX)
        k_keep_dirichlet<<<c->dc.nblk, NT, 0, c->stream>>>(c->dc, c->a[A_UX], c->a[A_DX], c->a[A_VU], c->a[A_GX],
                                                            outflow_desc(c), 0);
    if (field == CCNS_F_UY)
        k_keep_dirichlet<<<c->dc.nblk, NT, 0, c->stream>>>(c->dc, c->a[A_UY], c->a[A_DY], c->a[A_VV], c->a[A_GY],
                                                            outflow_desc(c), 1);
    HIPCHK(c, hipGetLastError());
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
        k_op_cont<<<c->dc.nblk, NT, 0, c->stream>>>(c->dc, c->a[A_AX], c->a[A_AY], c->a[A_HET], t0, t1, t2);
        if ((s = from_dev(c, out[0], t2, D2D))) return s;
        break;
    case CCNS_OP_PRES:
        if ((s = to_dev(c, t0, in[0], D2D))) return s;
        k_op_pres<<<c->dc.nblk, NT, 0, c->stream>>>(c->dc, c->a[A_AX], c->a[A_AY], t0, t1, t2);
        if ((s = from_dev(c, out[0], t1, D2D)) || (s = from_dev(c, out[1], t2, D2D))) return s;
        break;
    case CCNS_OP_VISC:
    case CCNS_OP_H:
        if ((s = to_dev(c, t0, in[0], D2D)) || (s = to_dev(c, t1, in[1], D2D))) return s;
        k_op_visc<<<c->dc.nblk, NT, 0, c->stream>>>(c->dc, pred_coef(c), c->a[A_VDX], c->a[A_VDY], c->a[A_GX],
                                                    c->a[A_GY], t0, t1, t2, t3,
                                                       op == CCNS_OP_VISC ? 0 : 1);
        if ((s = from_dev(c, out[0], t2, D2D)) || (s = from_dev(c, out[1], t3, D2D))) return s;
        break;
    case CCNS_OP_CONV:
        if ((s = to_dev(c, t0, in[0], D2D)) || (s = to_dev(c, t1, in[1], D2D))) return s;
        k_op_conv<<<c->dc.nblk, NT, 0, c->stream>>>(c->dc, c->a[A_AX], c->a[A_AY], c->a[A_HBX], c->a[A_HBY],
                                                       c->a[A_DX], c->a[A_DY], t0, t1, t2, t3);
        if ((s = from_dev(c, out[0], t2, D2D)) || (s = from_dev(c, out[1], t3, D2D))) return s;
        break;
    case CCNS_OP_LAP:
        if ((s = to_dev(c, t0, in[0], D2D))) return s;
        k_op_lap<<<c->dc.nblk, NT, 0, c->stream>>>(c->dc, pois_coef(c), t0, t1);
        if ((s = from_dev(c, out[0], t1, D2D))) return s;
        break;
    case CCNS_OP_KINETIC:
        if ((s = to_dev(c, t0, in[0], D2D)) || (s = to_dev(c, t1, in[1], D2D))) return s;
        k_op_kin<<<c->dc.nblk, NT, 0, c->stream>>>(c->dc, c->a[A_VUR], c->a[A_VVR], t0, t1, t2);
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
    k_pois_sum<<<c->dc.nblk, NT, 0, c->stream>>>(c->dc, pois_coef(c), c->a[A_B], c->part[PB_RHS]);
    s = pressure_solve_any(c, c->dc.nblk, info);
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
    return predict_any(c, info);
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
        ccns_status s1 = predict_any(c, &si.pred);
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
    // timing creates HIP events: not for a context that allocates nothing
    if (enable == 1 && c->static_dev >= 0) return fail(c, CCNS_ESTATE, "timing needs events: not available on a static context");
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

ccns_status ccns_forces(ccns_ctx *c, double *forces_host) {
    if (!c || !forces_host) return fail(c, CCNS_EINVAL, "null argument");
    if (c->nfc < 0) return fail(c, CCNS_ENOMEM, "more cut cells than the workspace's force table holds");
    k_forces<<<1, FT, 0, c->stream>>>(c->ftab, c->nfc, c->nfn, c->w.force_cap, c->w.L.pitch, c->a[A_DINV], c->a[A_P],
                                      c->a[A_UX], c->a[A_UY], c->a[A_DX], c->a[A_DY], 2.0 * c->prm.mu, c->fsum);
    HIPCHK(c, hipGetLastError());
    // through the context's own (pinned) read-back buffer, as every other read-back
    HIPCHK(c, hipMemcpyAsync(c->h_outer, c->fsum, 4 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    std::memcpy(forces_host, c->h_outer, 4 * sizeof(double));
    return CCNS_OK;
}

ccns_status ccns_set_mg_forms(ccns_ctx *c, unsigned long long forms) {
    if (!c || !mg_forms_valid(forms)) return fail(c, CCNS_EINVAL, "bad multigrid forms");
    c->prm.mg_forms = forms;
    resolve_mg_forms<double>(c, c->mg, forms);
    resolve_mg_forms<float>(c, c->mg32, forms);
    return CCNS_OK;
}

int ccns_mg_levels(const ccns_ctx *c, int *nx, int *ny, int *forms, int cap) {
    if (!c || c->prm.precond != 1) return 0;
    const int dbl = c->prm.precision == 1 ? 0 : 1;
    const int n = (int)std::min<size_t>(dbl ? cycle_levels(c->mg) : cycle_levels(c->mg32), MG_FORM_LEVELS);
    for (int l = 0; l < n && l < cap; ++l) {
        if (nx) nx[l] = c->mg[l].L.nx;
        if (ny) ny[l] = c->mg[l].L.ny;
        if (forms) forms[l] = c->mgf[dbl][0][l] | (c->mgf[dbl][1][l] << MG_FORM_BITS);
    }
    return n;
}

}  // extern "C"

// ===========================================================================
// fused batches: one launch per phase over the tiles of every simulation
// ===========================================================================

namespace {

// A simulation of a fused batch as the batched kernels see it: the
// arguments its solo launches take, gathered once.  The cycle levels and
// the coarse end are those of the context's multigrid hierarchy (FP64, and
// in precision 1 the float one of the inner solves).
constexpr int BATCH_LEVELS = 16;
template <class T>
struct BatchLevelT {
    int nx, ny, P, gx;         // the level
    PoisCoefT<T> pc;
    const T *b;
    T *x, *xt;
    int Pc, nxc, nyc;          // the next coarser level
    const T *dinvc;
    T *bc;
    const T *xc;               // the coarser level's result (its up-sweep, or the coarse end)
    int fd, fu, nbd, nbu;      // kernel forms and work-groups of the down- and up-sweep
};
enum BatchBottom { BOT_COARSEST = 0, BOT_TAIL_LDS = 1, BOT_TAIL = 2 };
template <class T>
struct BatchCycle {
    int ncyc;                  // cycle levels
    BatchLevelT<T> lv[BATCH_LEVELS];
    int bottom;                // BatchBottom
    TailDesc<T> tail;
    int tail_bytes;            // LDS the tail's levels take (BOT_TAIL_LDS)
    const T *cb;               // the coarsest grid's b and x (BOT_COARSEST)
    T *cxo;
    const T *z;                // the cycle's result on the finest level
};
struct BatchSim {
    const int *active;           // precision 1: 1 while the simulation takes part in the sweep
    int P, rows, pgx, pgy, pnb;  // layout; predictor tiles and work-groups
    int pgy32, pnb32;            // the same for the float predictor CG's taller tiles
    size_t n;
    PredCoefT<double> pd;
    PredCoefT<float> pf;         // precision 1: the inner predictor solve's coefficients
    double rho, grav_x, grav_y, rho_tau, tau_rho, pcoef;
    int conv_valid;
    OutflowDesc of;
    double *a[A_COUNT];
    float *f[G_COUNT];
    double *part[PB_COUNT];
    double *outer;
    CgState *st_pred, *st_pois, *st_pred_in, *st_pois_in;
    DiagState *diag;
    DiagCoef dgc;
    Dims dc, dp;
    int nl;                      // work-groups of the CG update
    int fb1, fb2;                // work-groups of the correction over n and 2n entries
    int ncoarse;
    const int *pidx;
    const double *pinv;
    BatchCycle<double> mg;
    BatchCycle<float> mg32;
};
template <class T>
__host__ __device__ __forceinline__ const BatchCycle<T> &cycle_of(const BatchSim &s) {
    if constexpr (std::is_same<T, double>::value)
        return s.mg;
    else
        return s.mg32;
}
// The pressure CG's state: the FP64 solve, or the inner float solve.
template <class T>
__device__ __forceinline__ CgState *pois_state(const BatchSim &s) {
    return std::is_same<T, double>::value ? s.st_pois : s.st_pois_in;
}

// Work-group table entries: simulation index (high bits) and the group's
// index within that simulation's grid.
constexpr int BATCH_SIM_SHIFT = 22;
constexpr unsigned BATCH_LOCAL_MASK = (1u << BATCH_SIM_SHIFT) - 1;
constexpr int BATCH_MAX_SIMS = 1 << (32 - BATCH_SIM_SHIFT);

// The batched kernel of an operation: work-group blockIdx.x runs group
// (map & mask) of simulation (map >> shift), with u the launch's uniform
// argument (the CG iteration, the cycle level or the sweep).  A simulation
// outside the current refinement sweep (precision 1) does nothing.  Every
// operation's run is forced inline: an operation instantiated in two kernels
// is otherwise compiled as a called function, with a stack frame and the
// register budget of a call (measured: the predictor CG at 2.2 times its
// time).
template <class Op>
__global__ __launch_bounds__(Op::BT) void k_batch(const BatchSim *__restrict__ sims, const unsigned *__restrict__ map,
                                                  int u) {
    const unsigned e = map[blockIdx.x];
    const BatchSim &s = sims[e >> BATCH_SIM_SHIFT];
    if (s.active && !*s.active) return;
    Op::run(SubGrid{(int)(e & BATCH_LOCAL_MASK), Op::groups(s, u)}, s, u);
}
// The same with the register budget of k_pred_cg (seven waves per SIMD).
template <class Op>
__global__ __launch_bounds__(Op::BT) __attribute__((amdgpu_waves_per_eu(7))) void k_batch_w7(
    const BatchSim *__restrict__ sims, const unsigned *__restrict__ map, int u) {
    const unsigned e = map[blockIdx.x];
    const BatchSim &s = sims[e >> BATCH_SIM_SHIFT];
    if (s.active && !*s.active) return;
    Op::run(SubGrid{(int)(e & BATCH_LOCAL_MASK), Op::groups(s, u)}, s, u);
}
// The same two with the CG iteration read from device memory (*itp): the
// launches of one iteration are then the same for every iteration, and a
// HIP graph captured once replays them; k_batch_count moves the counter.
template <class Op>
__global__ __launch_bounds__(Op::BT) void k_batch_it(const BatchSim *__restrict__ sims,
                                                     const unsigned *__restrict__ map, const int *itp) {
    const int u = *itp;
    const unsigned e = map[blockIdx.x];
    const BatchSim &s = sims[e >> BATCH_SIM_SHIFT];
    if (s.active && !*s.active) return;
    Op::run(SubGrid{(int)(e & BATCH_LOCAL_MASK), Op::groups(s, u)}, s, u);
}
template <class Op>
__global__ __launch_bounds__(Op::BT) __attribute__((amdgpu_waves_per_eu(7))) void k_batch_it_w7(
    const BatchSim *__restrict__ sims, const unsigned *__restrict__ map, const int *itp) {
    const int u = *itp;
    const unsigned e = map[blockIdx.x];
    const BatchSim &s = sims[e >> BATCH_SIM_SHIFT];
    if (s.active && !*s.active) return;
    Op::run(SubGrid{(int)(e & BATCH_LOCAL_MASK), Op::groups(s, u)}, s, u);
}
// *itp = v (v >= 0), or *itp + 1 (v < 0).
__global__ void k_batch_count(int *itp, int v) {
    if (threadIdx.x == 0) *itp = v >= 0 ? v : *itp + 1;
}

template <bool GEO, bool CLS>
struct OpPredRhs {
    static constexpr int BT = NT;
    __device__ __forceinline__ static int groups(const BatchSim &s, int) { return s.pnb; }
    __device__ __forceinline__ static void run(const SubGrid &g, const BatchSim &s, int) {
        pred_rhs_body<GEO, CLS>(g, s.P, s.rows, s.pgx, s.pgy, s.n, s.pd, s.a[A_AX], s.a[A_AY], s.a[A_HBX],
                                s.a[A_HBY], s.a[A_DX], s.a[A_DY], s.a[A_UX], s.a[A_UY], s.a[A_P], s.a[A_VDX],
                                s.a[A_VDY], s.a[A_CONVX], s.a[A_CONVY], s.a[A_RHSX], s.a[A_USX], s.rho, s.grav_x,
                                s.grav_y, s.conv_valid, s.of);
    }
};
// The predictor residual rhs - H U*: FP64 (MIX = false), or rounded to the
// float right-hand side of the inner solve (MIX).
template <bool MIX, bool GEO, bool CLS>
struct OpPredResid {
    static constexpr int BT = NT;
    __device__ __forceinline__ static int groups(const BatchSim &s, int) { return s.pnb; }
    __device__ __forceinline__ static void run(const SubGrid &g, const BatchSim &s, int) {
        if constexpr (MIX)
            pred_resid_body<true, GEO, CLS>(g, s.P, s.rows, s.pgx, s.pgy, s.n, s.pd, s.a[A_RHSX], s.a[A_USX],
                                            s.a[A_PRX], s.st_pred_in, s.part[PB_RHS], s.f[G_PRX], s.f[G_PXX],
                                            s.f[G_HDX]);
        else
            pred_resid_body<false, GEO, CLS>(g, s.P, s.rows, s.pgx, s.pgy, s.n, s.pd, s.a[A_RHSX], s.a[A_USX],
                                             s.a[A_PRX], s.st_pred, s.part[PB_RHS], nullptr, nullptr, nullptr);
    }
};
// Launch u = it of the predictor CG in storage type T (r, p and H p
// alternate between two buffers by the parity of it, as in the solo solve).
template <class T, bool GEO, bool CLS>
struct OpPredCg {
    static constexpr int BT = NT;
    __device__ __forceinline__ static int groups(const BatchSim &s, int) {
        return std::is_same<T, double>::value ? s.pnb : s.pnb32;
    }
    __device__ __forceinline__ static void run(const SubGrid &g, const BatchSim &s, int it) {
        const int b = it & 1;
        const double *tin = it == 0 ? s.part[PB_INIT] : s.part[PB_UPD];
        const int nin = it == 0 ? 1 : PRED_RED;
        if constexpr (std::is_same<T, double>::value) {
            double *r[2] = {s.a[A_PRX], s.a[A_PR1X]}, *p[2] = {s.a[A_PP0X], s.a[A_PP1X]},
                   *q[2] = {s.a[A_PQX], s.a[A_PQ1X]};
            pred_cg_body<double, GEO, CLS>(g, s.P, s.rows, s.pgx, s.pgy, s.n, s.pd, s.st_pred, it, s.a[A_USX],
                                           it == 0 ? r[0] : r[b ^ 1], r[b], p[b ^ 1], p[b], q[b ^ 1], q[b], tin,
                                           nin, s.part[PB_DIR]);
        } else {
            float *r[2] = {s.f[G_PRX], s.f[G_PR1X]}, *p[2] = {s.f[G_PP0X], s.f[G_PP1X]},
                  *q[2] = {s.f[G_PQX], s.f[G_PQ1X]};
            pred_cg_body<float, GEO, CLS>(g, s.P, s.rows, s.pgx, s.pgy32, s.n, s.pf, s.st_pred_in, it, s.f[G_PXX],
                                          it == 0 ? r[0] : r[b ^ 1], r[b], p[b ^ 1], p[b], q[b ^ 1], q[b], tin,
                                          nin, s.part[PB_DIR]);
        }
    }
};
template <class T>
struct OpPredSplit {
    static constexpr int BT = NT;
    __device__ __forceinline__ static int groups(const BatchSim &, int) { return PRED_RED; }
    __device__ __forceinline__ static void run(const SubGrid &g, const BatchSim &s, int) {
        reduce_partials_split_body<7>(g, s.part[PB_DIR], std::is_same<T, double>::value ? s.pnb : s.pnb32,
                                      s.part[PB_UPD]);
    }
};
// One-group reductions.
enum BatchReduce {
    RED_PRED = 0,      // the FP64 predictor residual's statistics
    RED_CYCLE = 1,     // the FP64 cycle's statistics of z
    RED_DIAG = 2,      // the diagnostics
    RED_PRED_MIX = 3,  // the precision-1 predictor residual's statistics
    RED_POIS_MIX = 4,  // the precision-1 pressure residual's statistics (to `outer`)
    RED_CYCLE32 = 5    // the float cycle's statistics of z
};
struct OpReduce {
    static constexpr int BT = NT;
    __device__ __forceinline__ static int groups(const BatchSim &, int) { return 1; }
    __device__ __forceinline__ static void run(const SubGrid &, const BatchSim &s, int u) {
        switch (u) {
        case RED_PRED: reduce_partials_body<5, 0, NT>(s.part[PB_RHS], s.pnb, s.part[PB_INIT]); break;
        case RED_CYCLE: reduce_partials_body<4, 0, NT>(s.part[PB_UPD], s.mg.lv[0].nbu, s.part[PB_MG]); break;
        case RED_DIAG: diag_final_body(s.part[PB_DIAG], s.dc.nblk, s.diag); break;
        case RED_PRED_MIX: reduce_partials_body<7, 0, NT>(s.part[PB_RHS], s.pnb, s.part[PB_INIT]); break;
        case RED_POIS_MIX: reduce_partials_body<7, 1, NT>(s.part[PB_INIT], s.dc.nblk, s.outer); break;
        default: reduce_partials_body<4, 0, NT>(s.part[PB_UPD], s.mg32.lv[0].nbu, s.part[PB_MG]);
        }
    }
};
struct OpPoisRhs {
    static constexpr int BT = NT;
    __device__ __forceinline__ static int groups(const BatchSim &s, int) { return s.dc.nblk; }
    __device__ __forceinline__ static void run(const SubGrid &g, const BatchSim &s, int) {
        pois_rhs_body(g, s.dc, PoisCoef{s.a[A_CX], s.a[A_CY], s.a[A_DINV]}, s.a[A_AX], s.a[A_AY], s.a[A_HET],
                      s.a[A_USX], s.a[A_USY], s.a[A_B], s.rho_tau, s.part[PB_RHS]);
    }
};
// The pressure solve's first residual (FP64), or the residual of sweep u of
// the refinement (MIX; sweep 0 also removes the mean of b where needed).
template <bool MIX>
struct OpPoisInit {
    static constexpr int BT = NT;
    __device__ __forceinline__ static int groups(const BatchSim &s, int) { return s.dc.nblk; }
    __device__ __forceinline__ static void run(const SubGrid &g, const BatchSim &s, int u) {
        const PoisCoef pc{s.a[A_CX], s.a[A_CY], s.a[A_DINV]};
        if constexpr (MIX)
            pois_init_body<true>(g, s.dc, pc, s.a[A_B], s.a[A_PHI], nullptr, s.st_pois_in,
                                 u == 0 ? s.part[PB_RHS] : nullptr, s.dc.nblk, s.part[PB_INIT], s.f[G_R], s.f[G_X],
                                 s.f[G_DINV]);
        else
            pois_init_body<false>(g, s.dc, pc, s.a[A_B], s.a[A_PHI], s.a[A_R], s.st_pois, s.part[PB_RHS], s.dc.nblk,
                                  s.part[PB_INIT], nullptr, nullptr, nullptr);
    }
};
// The multigrid CG's direction and update of iteration u = it, in storage
// type T; the search directions alternate between the two p buffers from
// the first (the first direction reads no old one).
template <class T>
struct OpDirZ {
    static constexpr int BT = NT;
    __device__ __forceinline__ static int groups(const BatchSim &s, int) { return s.dp.nblk; }
    __device__ __forceinline__ static void run(const SubGrid &g, const BatchSim &s, int it) {
        if constexpr (std::is_same<T, double>::value) {
            double *pold = (it & 1) ? s.a[A_P1] : s.a[A_P0], *pnew = (it & 1) ? s.a[A_P0] : s.a[A_P1];
            pois_dir_z_body<double>(g, s.dp, PoisCoef{s.a[A_CX], s.a[A_CY], s.a[A_DINV]}, s.mg.z, pold, pnew,
                                    s.a[A_Q], s.st_pois, it == 0 ? 1 : 0, it & 1, s.part[PB_MG], 1, s.part[PB_INIT],
                                    s.dc.nblk, s.part[PB_DIR]);
        } else {
            float *pold = (it & 1) ? s.f[G_P1] : s.f[G_P0], *pnew = (it & 1) ? s.f[G_P0] : s.f[G_P1];
            pois_dir_z_body<float>(g, s.dp, PoisCoefT<float>{s.f[G_CX], s.f[G_CY], s.f[G_DINV]}, s.mg32.z, pold,
                                   pnew, s.f[G_Q], s.st_pois_in, it == 0 ? 1 : 0, it & 1, s.part[PB_MG], 1, nullptr,
                                   0, s.part[PB_DIR]);
        }
    }
};
template <class T>
struct OpUpdate {
    static constexpr int BT = UT;
    __device__ __forceinline__ static int groups(const BatchSim &s, int) { return s.nl; }
    __device__ __forceinline__ static void run(const SubGrid &g, const BatchSim &s, int it) {
        if constexpr (std::is_same<T, double>::value)
            cg_update_body<double, false>(g, s.n, s.nl, s.a[A_DINV], s.a[A_PHI], s.a[A_R],
                                          (it & 1) ? s.a[A_P0] : s.a[A_P1], s.a[A_Q], s.st_pois, it & 1,
                                          s.part[PB_DIR], s.dp.nblk, s.part[PB_UPD]);
        else
            cg_update_body<float, false>(g, s.n, s.nl, s.f[G_DINV], s.f[G_X], s.f[G_R],
                                         (it & 1) ? s.f[G_P0] : s.f[G_P1], s.f[G_Q], s.st_pois_in, it & 1,
                                         s.part[PB_DIR], s.dp.nblk, s.part[PB_UPD]);
    }
};
// Down- and up-sweep of cycle level u in form F (MgForm), storage type T.
template <class T, int F>
struct OpMgDown {
    static constexpr int BT = NT;
    __device__ __forceinline__ static int groups(const BatchSim &s, int l) { return cycle_of<T>(s).lv[l].nbd; }
    __device__ __forceinline__ static void run(const SubGrid &g, const BatchSim &s, int l) {
        const BatchLevelT<T> &L = cycle_of<T>(s).lv[l];
        const int *done = &pois_state<T>(s)->done;
        if constexpr (F == MGF_STAGED)
            mg_down_staged_body<T>(g, L.nx, L.ny, L.P, L.gx, L.pc, L.b, L.x, L.Pc, L.nxc, L.nyc, L.dinvc, L.bc,
                                   done);
        else if constexpr (F == MGF_STAGED_LDS)
            mg_down_lds_body<T, MTY>(g, L.nx, L.ny, L.P, L.gx, L.pc, L.b, L.x, L.Pc, L.nxc, L.nyc, L.dinvc, L.bc,
                                     done);
        else if constexpr (F == MGF_STAGED_LDS_HALF)
            mg_down_lds_body<T, MTY / 2>(g, L.nx, L.ny, L.P, L.gx, L.pc, L.b, L.x, L.Pc, L.nxc, L.nyc, L.dinvc,
                                         L.bc, done);
        else if constexpr (F == MGF_PLAIN)
            mg_down_body<T, MTY>(g, L.nx, L.ny, L.P, L.gx, L.pc, L.b, L.x, L.Pc, L.nxc, L.nyc, L.dinvc, L.bc, done);
        else
            mg_down_body<T, MTY_SMALL>(g, L.nx, L.ny, L.P, L.gx, L.pc, L.b, L.x, L.Pc, L.nxc, L.nyc, L.dinvc, L.bc,
                                       done);
    }
};
// The finest level's up-sweep (STATS) writes the statistics of z.
template <class T, int F, bool STATS>
struct OpMgUp {
    static constexpr int BT = NT;
    __device__ __forceinline__ static int groups(const BatchSim &s, int l) { return cycle_of<T>(s).lv[l].nbu; }
    __device__ __forceinline__ static void run(const SubGrid &g, const BatchSim &s, int l) {
        const BatchLevelT<T> &L = cycle_of<T>(s).lv[l];
        const int *done = &pois_state<T>(s)->done;
        double *po = STATS ? s.part[PB_UPD] : nullptr;
        if constexpr (F == MGF_STAGED)
            mg_up_staged_body<T, STATS>(g, L.nx, L.ny, L.P, L.gx, L.pc, L.b, L.x, L.xc, L.Pc, L.xt, po, L.nbu, done);
        else if constexpr (F == MGF_STAGED_LDS)
            mg_up_lds_body<T, STATS, MTY>(g, L.nx, L.ny, L.P, L.gx, L.pc, L.b, L.x, L.xc, L.Pc, L.xt, po, L.nbu,
                                          done);
        else if constexpr (F == MGF_STAGED_LDS_HALF)
            mg_up_lds_body<T, STATS, MTY / 2>(g, L.nx, L.ny, L.P, L.gx, L.pc, L.b, L.x, L.xc, L.Pc, L.xt, po, L.nbu,
                                              done);
        else if constexpr (F == MGF_PLAIN)
            mg_up_body<T, STATS, MTY>(g, L.nx, L.ny, L.P, L.gx, L.pc, L.b, L.x, L.xc, L.Pc, L.xt, po, L.nbu, done);
        else
            mg_up_body<T, STATS, MTY_SMALL>(g, L.nx, L.ny, L.P, L.gx, L.pc, L.b, L.x, L.xc, L.Pc, L.xt, po, L.nbu,
                                            done);
    }
};
template <class T>
struct OpCoarsest {
    static constexpr int BT = NT;
    __device__ __forceinline__ static int groups(const BatchSim &, int) { return 1; }
    __device__ __forceinline__ static void run(const SubGrid &, const BatchSim &s, int) {
        const BatchCycle<T> &y = cycle_of<T>(s);
        mg_coarsest_body<T>(s.ncoarse, s.pidx, s.pinv, y.cb, y.cxo, &pois_state<T>(s)->done);
    }
};
template <class T, bool LDS>
struct OpTail {
    static constexpr int BT = TT;
    __device__ __forceinline__ static int groups(const BatchSim &, int) { return 1; }
    __device__ __forceinline__ static void run(const SubGrid &, const BatchSim &s, int) {
        if constexpr (LDS)
            mg_tail_lds_body<T>(cycle_of<T>(s).tail);
        else
            mg_tail_body<T>(cycle_of<T>(s).tail);
    }
};
// x += dx after an inner solve of precision 1: the predictor's U* (u = 0)
// or the pressure's Phi (u = 1).
struct OpAddCorr {
    static constexpr int BT = NT;
    __device__ __forceinline__ static int groups(const BatchSim &s, int u) { return u == 0 ? s.fb2 : s.fb1; }
    __device__ __forceinline__ static void run(const SubGrid &g, const BatchSim &s, int u) {
        if (u == 0)
            add_correction_body(g, 2 * s.n, s.a[A_USX], s.f[G_PXX]);
        else
            add_correction_body(g, s.n, s.a[A_PHI], s.f[G_X]);
    }
};
struct OpCorrect {
    static constexpr int BT = NT;
    __device__ __forceinline__ static int groups(const BatchSim &s, int) { return s.dc.nblk; }
    __device__ __forceinline__ static void run(const SubGrid &g, const BatchSim &s, int) {
        correct_body(g, s.dc, s.a[A_GX], s.a[A_GY], s.a[A_USX], s.a[A_USY], s.a[A_PHI], s.a[A_UX], s.a[A_UY],
                     s.tau_rho);
    }
};
struct OpDiag {
    static constexpr int BT = NT;
    __device__ __forceinline__ static int groups(const BatchSim &s, int) { return s.dc.nblk; }
    __device__ __forceinline__ static void run(const SubGrid &g, const BatchSim &s, int) {
        diag_body(g, s.dc, s.dgc, s.a[A_UX], s.a[A_UY], s.a[A_PHI], s.a[A_P], s.pcoef, 1, s.rho, s.part[PB_DIAG]);
    }
};

// What a gather reads from each simulation.
enum BatchGather {
    GAT_PRED = 0,      // the FP64 predictor CG's state
    GAT_POIS = 1,      // the FP64 pressure CG's state
    GAT_DIAG = 2,      // the diagnostics
    GAT_PRED_IN = 3,   // the inner predictor CG's state (precision 1)
    GAT_POIS_IN = 4,   // the inner pressure CG's state (precision 1)
    GAT_PRED_RES = 5,  // the predictor residual's statistics (precision 1; 7 values)
    GAT_POIS_RES = 6   // the pressure residual's statistics (precision 1; 8 values)
};
// Copies every simulation's solver state, diagnostics or residual
// statistics into one array for a single read-back.
__global__ __launch_bounds__(NT) void k_batch_gather(const BatchSim *__restrict__ sims, int n, int which,
                                                     CgState *__restrict__ cg, DiagState *__restrict__ dg,
                                                     double *__restrict__ st8) {
    const int k = blockIdx.x * NT + threadIdx.x;
    if (k >= n) return;
    const BatchSim &s = sims[k];
    switch (which) {
    case GAT_PRED: cg[k] = *s.st_pred; break;
    case GAT_POIS: cg[k] = *s.st_pois; break;
    case GAT_DIAG: dg[k] = *s.diag; break;
    case GAT_PRED_IN: cg[k] = *s.st_pred_in; break;
    case GAT_POIS_IN: cg[k] = *s.st_pois_in; break;
    default: {
        const double *src = which == GAT_PRED_RES ? s.part[PB_INIT] : s.outer;
        const int m = which == GAT_PRED_RES ? 7 : 8;
        for (int q = 0; q < 8; ++q) st8[(size_t)k * 8 + q] = q < m ? src[q] : 0.0;
    }
    }
}
// The relative tolerance of the next inner solve of every simulation in
// the sweep (which = 0: predictor, 1: pressure), from tol2[k].
__global__ __launch_bounds__(NT) void k_batch_set_tol(const BatchSim *__restrict__ sims, int n, int which,
                                                      const double *__restrict__ tol2) {
    const int k = blockIdx.x * NT + threadIdx.x;
    if (k >= n) return;
    const BatchSim &s = sims[k];
    if (s.active && !*s.active) return;
    (which == 0 ? s.st_pred_in : s.st_pois_in)->tol2 = tol2[k];
}

// A launch of the fused batch: its slice of the work-group table.
struct BatchTable {
    size_t off = 0;
    int nblk = 0;
};

}  // namespace

struct ccns_batch {
    std::vector<ccns_ctx *> sims;
    std::vector<int> order;  // simulation indices, largest grid first
    int nthreads = 0;
    // fused batches only
    bool fused = false;
    int prec = 0;                   // the precision of every simulation
    hipStream_t stream = nullptr;
    BatchSim *dsims = nullptr;      // device copies of the descriptors
    unsigned *dmap = nullptr;       // work-group tables
    CgState *dcg = nullptr, *hcg = nullptr;       // gathered solver states (device, pinned host)
    DiagState *ddg = nullptr, *hdg = nullptr;     // gathered diagnostics
    double *dst8 = nullptr, *hst8 = nullptr;      // gathered residual statistics (8 per simulation)
    // precision 1: the sweep's active flags and inner tolerances, uploaded
    // from a ring of pinned slots (a slot is reused only after a read-back
    // has waited for the stream, so no upload still reads it)
    int *dact = nullptr;
    double *dtol = nullptr;
    char *hring = nullptr;
    int ring_used = 0;
    std::vector<int> act;
    std::vector<double> tol2;
    std::vector<BatchSim> hsims;
    std::vector<unsigned char> forms;  // the cycle forms the tables were built for
    size_t map_cap = 0;
    int maxcyc = 0, tail_lds = 0;
    // CG iterations as HIP graphs (one iteration of the predictor CG and one
    // of the pressure CG, with the iteration number in *dit), rebuilt with
    // the tables; off: every launch is queued one by one
    bool graphs = true;
    int *dit = nullptr;
    hipGraphExec_t gpred = nullptr, gpois = nullptr;
    BatchTable pred[4], pred32[4], one, split, dc, dp, upd, fb1, fb2;
    BatchTable down[BATCH_LEVELS][6], up[BATCH_LEVELS][6], bot[3];
};

namespace {

constexpr int BATCH_RING = 8;

size_t ring_slot_bytes(int n) { return align_up((size_t)n * (sizeof(int) + sizeof(double)), 256); }

// The descriptor of cycle hierarchy mg (FP64 or float) of context c, whose
// solve's done flag is *done.
template <class T>
void batch_cycle(BatchCycle<T> &y, ccns_ctx *c, std::vector<ccns_ctx::LevelT<T>> &mg, const int *done) {
    const int dbl = std::is_same<T, double>::value ? 1 : 0;
    const int ncyc = (int)cycle_levels(mg);
    y.ncyc = ncyc;
    // the coarse end below the cycle levels: the coarsest grid's
    // pseudo-inverse, or the one-group tail of the small levels
    const size_t ts = (size_t)ncyc;
    const T *bottom_out;
    if (ts + 1 == mg.size()) {
        y.bottom = BOT_COARSEST;
        y.cb = mg[ts].b;
        y.cxo = mg[ts].x;
        bottom_out = mg[ts].x;
    } else {
        TailDesc<T> &d = y.tail;
        d.nlev = (int)(mg.size() - ts);
        for (int t = 0; t < d.nlev; ++t) {
            auto &M = mg[ts + t];
            d.lv[t] = TailLevel<T>{M.cx, M.cy, M.dinv, M.b, M.x, M.xt, M.L.nx, M.L.ny, (int)M.L.pitch};
        }
        d.ncoarse = c->ncoarse_act;
        d.idx = c->pidx;
        d.pinv = c->pinv;
        d.done = done;
        d.out = d.nlev >= 2 ? mg[ts].xt : mg[ts].x;
        size_t elems = 0;
        for (int t = 0; t < d.nlev; ++t) {
            d.lofs[t] = (int)elems;
            elems += 6 * (size_t)(d.lv[t].nx + 2) * (d.lv[t].ny + 2);
        }
        y.bottom = elems * sizeof(T) <= (size_t)c->tail_lds ? BOT_TAIL_LDS : BOT_TAIL;
        y.tail_bytes = (int)(elems * sizeof(T));
        bottom_out = d.out;
    }
    for (int l = 0; l < ncyc; ++l) {
        auto &F = mg[l];
        auto &C = mg[l + 1];
        BatchLevelT<T> &v = y.lv[l];
        v.nx = F.L.nx;
        v.ny = F.L.ny;
        v.P = (int)F.L.pitch;
        v.gx = (F.L.nx + TX - 1) / TX;
        v.pc = PoisCoefT<T>{F.cx, F.cy, F.dinv};
        v.b = F.b;
        v.x = F.x;
        v.xt = F.xt;
        v.Pc = (int)C.L.pitch;
        v.nxc = C.L.nx;
        v.nyc = C.L.ny;
        v.dinvc = C.dinv;
        v.bc = C.b;
        v.xc = l + 1 < ncyc ? mg[l + 1].xt : bottom_out;
        v.fd = c->mgf[dbl][0][l];
        v.fu = c->mgf[dbl][1][l];
        v.nbd = mg_form_groups(v.nx, v.ny, v.fd);
        v.nbu = mg_form_groups(v.nx, v.ny, v.fu);
    }
    y.z = ncyc >= 1 ? mg[0].xt : bottom_out;
}

// The descriptor of context c (multigrid preconditioner; precision 0 or 1).
BatchSim batch_sim(ccns_batch *b, int k) {
    ccns_ctx *c = b->sims[k];
    BatchSim s{};
    s.active = b->prec == 1 ? b->dact + k : nullptr;
    const Layout &L = c->w.L;
    s.P = (int)L.pitch;
    s.rows = (int)L.rows;
    s.pgx = (int)(L.pitch / TX);
    s.pgy = (int)((L.rows + HTY - 1) / HTY);
    s.pnb = ((s.pgx * s.pgy + 7) / 8) * 8;
    s.pgy32 = (int)((L.rows + HTY_F32 - 1) / HTY_F32);
    s.pnb32 = ((s.pgx * s.pgy32 + 7) / 8) * 8;
    s.n = L.n;
    s.pd = pred_coef_t(c);
    if (c->ncls) {
        s.pd.cls = c->cls;
        s.pd.tab = c->tab;
    }
    const ccns_params &p = c->prm;
    if (p.precision == 1) {
        s.pf = PredCoefT<float>{ViscCoefT<float>{c->f[G_BXX], c->f[G_BXY], c->f[G_BYY], c->f[G_BYX], c->f[G_WXX],
                                                 c->f[G_WYY], c->f[G_NXX], c->f[G_NXY], c->f[G_NYX], c->f[G_NYY]},
                                c->f[G_VU], c->f[G_VV], c->f[G_HDX], c->f[G_HDY], p.rho / p.tau, p.mu, nullptr,
                                nullptr};
        if (c->ncls) {
            s.pf.cls = c->cls;
            s.pf.tab = c->tab32;
        }
        for (int q = 0; q < G_COUNT; ++q) s.f[q] = c->f[q];
    }
    s.rho = p.rho;
    s.grav_x = p.gx;
    s.grav_y = p.gy;
    s.rho_tau = p.rho / p.tau;
    s.tau_rho = p.tau / p.rho;
    s.pcoef = p.tau * p.mu / (2.0 * p.rho);
    s.conv_valid = c->conv_valid;
    s.of = outflow_desc(c);
    for (int q = 0; q < A_COUNT; ++q) s.a[q] = c->a[q];
    for (int q = 0; q < PB_COUNT; ++q) s.part[q] = c->part[q];
    s.outer = c->outer;
    s.st_pred = c->st_pred;
    s.st_pois = c->st_pois;
    s.st_pred_in = c->st_pred_in;
    s.st_pois_in = c->st_pois_in;
    s.diag = c->diag;
    s.dgc = DiagCoef{c->a[A_AX], c->a[A_AY], c->a[A_HET], c->a[A_DINV], c->a[A_VUR], c->a[A_VVR],
                     c->a[A_VU], c->a[A_VV], c->a[A_CX], c->a[A_CY], c->a[A_VINV]};
    s.dc = c->dc;
    s.dp = c->dp;
    s.nl = update_blocks(L.n);
    s.fb1 = flat_blocks(L.n);
    s.fb2 = flat_blocks(2 * L.n);
    s.ncoarse = c->ncoarse_act;
    s.pidx = c->pidx;
    s.pinv = c->pinv;
    batch_cycle<double>(s.mg, c, c->mg, &c->st_pois->done);
    if (p.precision == 1) batch_cycle<float>(s.mg32, c, c->mg32, &c->st_pois_in->done);
    return s;
}

int pred_variant(const ccns_ctx *c) { return (c->prm.visc_form == 0 ? 1 : 0) | (c->ncls ? 2 : 0); }

// The cycle levels' forms of context c in the batch's precision: every one
// resolved, the finest level's up-sweep in a form that writes the
// statistics (1-3), between 1 and BATCH_LEVELS cycle levels.
template <class T>
bool batch_forms_ok(const ccns_ctx *c, const std::vector<ccns_ctx::LevelT<T>> &mg) {
    const int dbl = std::is_same<T, double>::value ? 1 : 0;
    const int ncyc = (int)cycle_levels(mg);
    if (ncyc < 1 || ncyc > BATCH_LEVELS) return false;
    for (int l = 0; l < ncyc; ++l) {
        const int fd = c->mgf[dbl][0][l], fu = c->mgf[dbl][1][l];
        if (fd < MGF_STAGED || fd > MGF_STAGED_LDS_HALF || fu < MGF_STAGED || fu > MGF_STAGED_LDS_HALF ||
            (l == 0 && fu > MGF_PLAIN))
            return false;
    }
    return true;
}

void batch_drop_graphs(ccns_batch *b);

// Builds the descriptors and the work-group tables of every launch (the
// simulations in the batch's order, largest first, so that the big grids'
// groups are dispatched first), and uploads them.
ccns_status batch_build(ccns_batch *b) {
    const int n = (int)b->sims.size();
    const int dbl = b->prec == 1 ? 0 : 1;  // the forms of the cycle the batch runs
    batch_drop_graphs(b);
    b->hsims.resize(n);
    b->forms.clear();
    b->maxcyc = 0;
    b->tail_lds = 0;
    for (int k = 0; k < n; ++k) {
        ccns_ctx *c = b->sims[k];
        if (!(b->prec == 1 ? batch_forms_ok<float>(c, c->mg32) : batch_forms_ok<double>(c, c->mg)))
            return CCNS_EINVAL;
        b->hsims[k] = batch_sim(b, k);
        b->forms.insert(b->forms.end(), &c->mgf[dbl][0][0], &c->mgf[dbl][0][0] + 2 * 16);
        const int ncyc = b->prec == 1 ? b->hsims[k].mg32.ncyc : b->hsims[k].mg.ncyc;
        const int bottom = b->prec == 1 ? b->hsims[k].mg32.bottom : b->hsims[k].mg.bottom;
        const int tb = b->prec == 1 ? b->hsims[k].mg32.tail_bytes : b->hsims[k].mg.tail_bytes;
        b->maxcyc = std::max(b->maxcyc, ncyc);
        if (bottom == BOT_TAIL_LDS) b->tail_lds = std::max(b->tail_lds, tb);
    }
    // the LDS-resident coarse ends take up to the context's budget of dynamic LDS
    if (b->tail_lds > 0) {
        const void *kt = b->prec == 1 ? (const void *)k_batch<OpTail<float, true>>
                                      : (const void *)k_batch<OpTail<double, true>>;
        if (hipFuncSetAttribute(kt, hipFuncAttributeMaxDynamicSharedMemorySize, b->tail_lds) != hipSuccess)
            return CCNS_EDEVICE;
    }
    std::vector<unsigned> map;
    bool ok = true;
    auto table = [&](auto pick, auto groups) {
        BatchTable t;
        t.off = map.size();
        for (int k : b->order) {
            if (!pick(k)) continue;
            const long gcount = groups(k);
            if (gcount > (long)BATCH_LOCAL_MASK + 1) ok = false;
            for (long g = 0; g < gcount && ok; ++g) map.push_back(((unsigned)k << BATCH_SIM_SHIFT) | (unsigned)g);
        }
        t.nblk = (int)(map.size() - t.off);
        return t;
    };
    const auto &S = b->hsims;
    auto all = [](int) { return true; };
    for (int v = 0; v < 4; ++v) {
        b->pred[v] = table([&](int k) { return pred_variant(b->sims[k]) == v; }, [&](int k) { return S[k].pnb; });
        b->pred32[v] = table([&](int k) { return b->prec == 1 && pred_variant(b->sims[k]) == v; },
                             [&](int k) { return S[k].pnb32; });
    }
    b->one = table(all, [](int) { return 1; });
    b->split = table(all, [](int) { return PRED_RED; });
    b->dc = table(all, [&](int k) { return S[k].dc.nblk; });
    b->dp = table(all, [&](int k) { return S[k].dp.nblk; });
    b->upd = table(all, [&](int k) { return S[k].nl; });
    b->fb1 = table(all, [&](int k) { return b->prec == 1 ? S[k].fb1 : 0; });
    b->fb2 = table(all, [&](int k) { return b->prec == 1 ? S[k].fb2 : 0; });
    auto lvl = [&](int k, int l) -> const auto & { return S[k].mg.lv[l]; };
    auto lvl32 = [&](int k, int l) -> const auto & { return S[k].mg32.lv[l]; };
    auto ncyc = [&](int k) { return b->prec == 1 ? S[k].mg32.ncyc : S[k].mg.ncyc; };
    auto fd = [&](int k, int l) { return b->prec == 1 ? lvl32(k, l).fd : lvl(k, l).fd; };
    auto fu = [&](int k, int l) { return b->prec == 1 ? lvl32(k, l).fu : lvl(k, l).fu; };
    auto nbd = [&](int k, int l) { return b->prec == 1 ? lvl32(k, l).nbd : lvl(k, l).nbd; };
    auto nbu = [&](int k, int l) { return b->prec == 1 ? lvl32(k, l).nbu : lvl(k, l).nbu; };
    for (int l = 0; l < BATCH_LEVELS; ++l)
        for (int f = 0; f < 6; ++f) {
            b->down[l][f] = table([&](int k) { return l < ncyc(k) && fd(k, l) == f; }, [&](int k) { return nbd(k, l); });
            b->up[l][f] = table([&](int k) { return l < ncyc(k) && fu(k, l) == f; }, [&](int k) { return nbu(k, l); });
        }
    for (int t = 0; t < 3; ++t)
        b->bot[t] = table([&](int k) { return (b->prec == 1 ? S[k].mg32.bottom : S[k].mg.bottom) == t; },
                          [](int) { return 1; });
    if (!ok) return CCNS_EINVAL;
    if (map.size() > b->map_cap) {
        if (b->dmap) (void)hipFree(b->dmap);
        b->dmap = nullptr;
        if (hipMalloc(&b->dmap, map.size() * sizeof(unsigned)) != hipSuccess) return CCNS_ENOMEM;
        b->map_cap = map.size();
    }
    if (hipMemcpyAsync(b->dmap, map.data(), map.size() * sizeof(unsigned), hipMemcpyHostToDevice, b->stream) !=
            hipSuccess ||
        hipMemcpyAsync(b->dsims, S.data(), S.size() * sizeof(BatchSim), hipMemcpyHostToDevice, b->stream) !=
            hipSuccess ||
        hipStreamSynchronize(b->stream) != hipSuccess)
        return CCNS_EDEVICE;
    b->ring_used = 0;
    return CCNS_OK;
}

template <class Op>
void blaunch(ccns_batch *b, const BatchTable &t, int u, size_t lds = 0) {
    if (t.nblk > 0)
        hipLaunchKernelGGL(k_batch<Op>, dim3(t.nblk), dim3(Op::BT), lds, b->stream, b->dsims, b->dmap + t.off, u);
}
template <class Op>
void blaunch_w7(ccns_batch *b, const BatchTable &t, int u) {
    if (t.nblk > 0)
        hipLaunchKernelGGL(k_batch_w7<Op>, dim3(t.nblk), dim3(Op::BT), 0, b->stream, b->dsims, b->dmap + t.off, u);
}
// Launches of a CG iteration: with it >= 0 the iteration is an argument;
// with it < 0 (while a graph is captured) the kernels read it from *dit.
template <class Op>
void blaunch_iter(ccns_batch *b, const BatchTable &t, int it) {
    if (t.nblk <= 0) return;
    if (it >= 0)
        hipLaunchKernelGGL(k_batch<Op>, dim3(t.nblk), dim3(Op::BT), 0, b->stream, b->dsims, b->dmap + t.off, it);
    else
        hipLaunchKernelGGL(k_batch_it<Op>, dim3(t.nblk), dim3(Op::BT), 0, b->stream, b->dsims, b->dmap + t.off,
                           (const int *)b->dit);
}
template <class Op>
void blaunch_iter_w7(ccns_batch *b, const BatchTable &t, int it) {
    if (t.nblk <= 0) return;
    if (it >= 0)
        hipLaunchKernelGGL(k_batch_w7<Op>, dim3(t.nblk), dim3(Op::BT), 0, b->stream, b->dsims, b->dmap + t.off, it);
    else
        hipLaunchKernelGGL(k_batch_it_w7<Op>, dim3(t.nblk), dim3(Op::BT), 0, b->stream, b->dsims, b->dmap + t.off,
                           (const int *)b->dit);
}

// One V-cycle of every simulation on its finest level's residual, in
// storage type T: the down-sweeps level by level, the coarse ends, the
// up-sweeps back up, and the reduction of the statistics of z.
template <class T>
void batch_vcycle(ccns_batch *b) {
    for (int l = 0; l < b->maxcyc; ++l) {
        blaunch<OpMgDown<T, MGF_STAGED>>(b, b->down[l][MGF_STAGED], l);
        blaunch<OpMgDown<T, MGF_STAGED_LDS>>(b, b->down[l][MGF_STAGED_LDS], l);
        blaunch<OpMgDown<T, MGF_PLAIN>>(b, b->down[l][MGF_PLAIN], l);
        blaunch<OpMgDown<T, MGF_PLAIN_SHORT>>(b, b->down[l][MGF_PLAIN_SHORT], l);
        blaunch<OpMgDown<T, MGF_STAGED_LDS_HALF>>(b, b->down[l][MGF_STAGED_LDS_HALF], l);
    }
    blaunch<OpCoarsest<T>>(b, b->bot[BOT_COARSEST], 0);
    blaunch<OpTail<T, true>>(b, b->bot[BOT_TAIL_LDS], 0, (size_t)b->tail_lds);
    blaunch<OpTail<T, false>>(b, b->bot[BOT_TAIL], 0);
    for (int l = b->maxcyc - 1; l >= 1; --l) {
        blaunch<OpMgUp<T, MGF_STAGED, false>>(b, b->up[l][MGF_STAGED], l);
        blaunch<OpMgUp<T, MGF_STAGED_LDS, false>>(b, b->up[l][MGF_STAGED_LDS], l);
        blaunch<OpMgUp<T, MGF_PLAIN, false>>(b, b->up[l][MGF_PLAIN], l);
        blaunch<OpMgUp<T, MGF_PLAIN_SHORT, false>>(b, b->up[l][MGF_PLAIN_SHORT], l);
        blaunch<OpMgUp<T, MGF_STAGED_LDS_HALF, false>>(b, b->up[l][MGF_STAGED_LDS_HALF], l);
    }
    blaunch<OpMgUp<T, MGF_STAGED, true>>(b, b->up[0][MGF_STAGED], 0);
    blaunch<OpMgUp<T, MGF_STAGED_LDS, true>>(b, b->up[0][MGF_STAGED_LDS], 0);
    blaunch<OpMgUp<T, MGF_PLAIN, true>>(b, b->up[0][MGF_PLAIN], 0);
    blaunch<OpReduce>(b, b->one, std::is_same<T, double>::value ? RED_CYCLE : RED_CYCLE32);
}

// One iteration of every simulation's predictor CG in storage type T
// (it < 0: the iteration number from *dit, which the last launch moves on).
template <class T>
void batch_pred_iter(ccns_batch *b, int it) {
    const BatchTable *t = std::is_same<T, double>::value ? b->pred : b->pred32;
    blaunch_iter_w7<OpPredCg<T, false, false>>(b, t[0], it);
    blaunch_iter_w7<OpPredCg<T, true, false>>(b, t[1], it);
    blaunch_iter_w7<OpPredCg<T, false, true>>(b, t[2], it);
    blaunch_iter_w7<OpPredCg<T, true, true>>(b, t[3], it);
    blaunch_iter<OpPredSplit<T>>(b, b->split, it);
    if (it < 0) hipLaunchKernelGGL(k_batch_count, dim3(1), dim3(64), 0, b->stream, b->dit, -1);
}
// One iteration of every simulation's multigrid-preconditioned pressure CG.
template <class T>
void batch_pois_iter(ccns_batch *b, int it) {
    blaunch_iter<OpDirZ<T>>(b, b->dp, it);
    blaunch_iter<OpUpdate<T>>(b, b->upd, it);
    batch_vcycle<T>(b);
    if (it < 0) hipLaunchKernelGGL(k_batch_count, dim3(1), dim3(64), 0, b->stream, b->dit, -1);
}

void batch_drop_graphs(ccns_batch *b) {
    if (b->gpred) (void)hipGraphExecDestroy(b->gpred);
    if (b->gpois) (void)hipGraphExecDestroy(b->gpois);
    b->gpred = b->gpois = nullptr;
}

// Captures the launches fill() queues as a graph.  A capture the runtime
// refuses leaves the batch queueing its launches one by one.
template <class F>
void batch_capture(ccns_batch *b, hipGraphExec_t &exec, F fill) {
    if (exec || !b->graphs) return;
    hipGraph_t g = nullptr;
    bool ok = hipStreamBeginCapture(b->stream, hipStreamCaptureModeRelaxed) == hipSuccess;
    if (ok) {
        fill();
        ok = hipStreamEndCapture(b->stream, &g) == hipSuccess && g;
    }
    if (ok) ok = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0) == hipSuccess;
    if (g) (void)hipGraphDestroy(g);
    if (!ok) {
        exec = nullptr;
        (void)hipGetLastError();
        batch_drop_graphs(b);
        b->graphs = false;
    }
}

// Queues one CG iteration it: by replaying the captured graph (the
// iteration number then lives in *dit, set to 0 before the first), or
// launch by launch.
template <class T>
ccns_status batch_iterate(ccns_batch *b, bool pred, int it) {
    if (b->graphs) {
        hipGraphExec_t &exec = pred ? b->gpred : b->gpois;
        batch_capture(b, exec, [&] { pred ? batch_pred_iter<T>(b, -1) : batch_pois_iter<T>(b, -1); });
    }
    if (b->graphs) {
        if (it == 0) hipLaunchKernelGGL(k_batch_count, dim3(1), dim3(64), 0, b->stream, b->dit, 0);
        if (hipGraphLaunch(pred ? b->gpred : b->gpois, b->stream) != hipSuccess) return CCNS_EDEVICE;
    } else if (pred) {
        batch_pred_iter<T>(b, it);
    } else {
        batch_pois_iter<T>(b, it);
    }
    return CCNS_OK;
}

// Reads every simulation's solver state, diagnostics or residual
// statistics (BatchGather) after the work queued so far.
ccns_status batch_read(ccns_batch *b, int which) {
    const int n = (int)b->sims.size();
    hipLaunchKernelGGL(k_batch_gather, dim3((n + NT - 1) / NT), dim3(NT), 0, b->stream, b->dsims, n, which, b->dcg,
                       b->ddg, b->dst8);
    if (hipGetLastError() != hipSuccess) return CCNS_EDEVICE;
    hipError_t e;
    if (which == GAT_DIAG)
        e = hipMemcpyAsync(b->hdg, b->ddg, n * sizeof(DiagState), hipMemcpyDeviceToHost, b->stream);
    else if (which == GAT_PRED_RES || which == GAT_POIS_RES)
        e = hipMemcpyAsync(b->hst8, b->dst8, (size_t)n * 8 * sizeof(double), hipMemcpyDeviceToHost, b->stream);
    else
        e = hipMemcpyAsync(b->hcg, b->dcg, n * sizeof(CgState), hipMemcpyDeviceToHost, b->stream);
    if (e != hipSuccess || hipStreamSynchronize(b->stream) != hipSuccess) return CCNS_EDEVICE;
    b->ring_used = 0;  // every upload queued so far has been read
    return CCNS_OK;
}

// Uploads the active flags and inner tolerances (precision 1) for the
// launches queued after this.
ccns_status batch_upload(ccns_batch *b) {
    const int n = (int)b->sims.size();
    if (b->ring_used == BATCH_RING) {
        if (hipStreamSynchronize(b->stream) != hipSuccess) return CCNS_EDEVICE;
        b->ring_used = 0;
    }
    char *slot = b->hring + (size_t)b->ring_used++ * ring_slot_bytes(n);
    std::memcpy(slot, b->act.data(), n * sizeof(int));
    std::memcpy(slot + (size_t)n * sizeof(int), b->tol2.data(), n * sizeof(double));
    if (hipMemcpyAsync(b->dact, slot, n * sizeof(int), hipMemcpyHostToDevice, b->stream) != hipSuccess ||
        hipMemcpyAsync(b->dtol, slot + (size_t)n * sizeof(int), n * sizeof(double), hipMemcpyHostToDevice,
                       b->stream) != hipSuccess)
        return CCNS_EDEVICE;
    return CCNS_OK;
}

ccns_solve_info solve_info(const CgState &h, bool clamp) {
    ccns_solve_info i{};
    i.iterations = h.it_final;
    i.outer = 1;
    const double r2 = clamp ? std::max(h.rnorm2_final, 0.0) : h.rnorm2_final;
    i.rel_residual = h.fnorm2 > 0 ? std::sqrt(r2 / h.fnorm2) : 0.0;
    i.status = h.status;
    i.inner_status = CCNS_OK;
    i.inner_fail_sweep = -1;
    return i;
}

// The contexts' own work first (their set-up and any solo calls), and the
// descriptors again where a context changed (its first convection, its
// cycle forms).
ccns_status batch_begin(ccns_batch *b) {
    const int n = (int)b->sims.size();
    const int dbl = b->prec == 1 ? 0 : 1;
    for (ccns_ctx *c : b->sims)
        if (hipStreamSynchronize(c->stream) != hipSuccess) return CCNS_EDEVICE;
    bool rebuild = false;
    for (int k = 0; k < n && !rebuild; ++k) {
        const ccns_ctx *c = b->sims[k];
        rebuild = b->hsims[k].conv_valid != c->conv_valid ||
                  std::memcmp(&b->forms[(size_t)k * 32], &c->mgf[dbl][0][0], 32) != 0;
    }
    return rebuild ? batch_build(b) : CCNS_OK;
}

// The predictor's right-hand side of every simulation (conv^n; U* := U^n).
void batch_pred_rhs(ccns_batch *b) {
    blaunch<OpPredRhs<false, false>>(b, b->pred[0], 0);
    blaunch<OpPredRhs<true, false>>(b, b->pred[1], 0);
    blaunch<OpPredRhs<false, true>>(b, b->pred[2], 0);
    blaunch<OpPredRhs<true, true>>(b, b->pred[3], 0);
    for (ccns_ctx *c : b->sims) c->conv_valid = 1;
}

// The correction's end: U^{n+1}, the pressure update and the diagnostics.
ccns_status batch_finish(ccns_batch *b, std::vector<ccns_step_info> &info, std::vector<ccns_status> &st) {
    const int n = (int)b->sims.size();
    blaunch<OpCorrect>(b, b->dc, 0);
    blaunch<OpDiag>(b, b->dc, 0);
    blaunch<OpReduce>(b, b->one, RED_DIAG);
    ccns_status s = batch_read(b, GAT_DIAG);
    if (s != CCNS_OK) return s;
    for (int k = 0; k < n; ++k) {
        const ccns_ctx *c = b->sims[k];
        const DiagState &d = b->hdg[k];
        info[k].div_max = d.divmax > 0 ? d.divmax : 0.0;
        info[k].div_rel = info[k].div_max / (c->prm.u_ref * std::min(c->g.hx, c->g.hy));
        info[k].ke = d.ke;
        info[k].mass = d.mass;
        info[k].mom_x = d.momx;
        info[k].mom_y = d.momy;
        ccns_status w = CCNS_OK;
        if (info[k].pred.status != CCNS_OK) w = (ccns_status)info[k].pred.status;
        if (info[k].poisson.status != CCNS_OK) w = (ccns_status)info[k].poisson.status;
        if (w != CCNS_OK) st[k] = w;
    }
    return CCNS_OK;
}

// Runs CG iterations of every simulation in lockstep until all of their
// solves have stopped: iter(it) queues iteration it; the done flags come
// back in one read-back (gather `which`) per chunk.  Returns the number of
// iterations queued.
template <class Iter>
ccns_status batch_cg(ccns_batch *b, int first_chunk, int next_chunk, int which, Iter iter, int &its) {
    const int n = (int)b->sims.size();
    int chunk = first_chunk;
    its = 0;
    for (;;) {
        for (int u = 0; u < chunk; ++u, ++its) {
            ccns_status s = iter(its);
            if (s != CCNS_OK) return s;
        }
        ccns_status s = batch_read(b, which);
        if (s != CCNS_OK) return s;
        bool all = true;
        for (int k = 0; k < n; ++k) all = all && (b->hcg[k].done || (b->prec == 1 && !b->act[k]));
        if (all) return CCNS_OK;
        chunk = next_chunk;
    }
}

// One projection step of every simulation in precision 0.  Each phase is
// one launch (per kernel variant) over all of their work-groups; each CG
// runs in lockstep, a simulation whose solve has stopped returning at once
// from its groups.
ccns_status batch_fused_step(ccns_batch *b, std::vector<ccns_step_info> &info, std::vector<ccns_status> &st) {
    const int n = (int)b->sims.size();
    ccns_status s = batch_begin(b);
    if (s != CCNS_OK) return s;
    // predictor
    batch_pred_rhs(b);
    blaunch<OpPredResid<false, false, false>>(b, b->pred[0], 0);
    blaunch<OpPredResid<false, true, false>>(b, b->pred[1], 0);
    blaunch<OpPredResid<false, false, true>>(b, b->pred[2], 0);
    blaunch<OpPredResid<false, true, true>>(b, b->pred[3], 0);
    blaunch<OpReduce>(b, b->one, RED_PRED);
    int last = 0, its = 0;
    for (ccns_ctx *c : b->sims) last = std::max(last, c->last_pred_it);
    s = batch_cg(b, std::max(4, last + 1), 8, GAT_PRED, [&](int it) { return batch_iterate<double>(b, true, it); },
                 its);
    if (s != CCNS_OK) return s;
    for (int k = 0; k < n; ++k) {
        info[k].pred = solve_info(b->hcg[k], true);
        b->sims[k]->last_pred_it = b->hcg[k].it_final;
    }
    // corrector: the pressure solve, then the correction, the pressure
    // update and the diagnostics
    blaunch<OpPoisRhs>(b, b->dc, 0);
    blaunch<OpPoisInit<false>>(b, b->dc, 0);
    batch_vcycle<double>(b);
    last = 0;
    for (ccns_ctx *c : b->sims) last = std::max(last, c->last_pois_it);
    s = batch_cg(b, std::max(2, last + 1), 2, GAT_POIS, [&](int it) { return batch_iterate<double>(b, false, it); },
                 its);
    if (s != CCNS_OK) return s;
    for (int k = 0; k < n; ++k) {
        info[k].poisson = solve_info(b->hcg[k], false);
        b->sims[k]->last_pois_it = b->hcg[k].it_final;
        b->sims[k]->pbuf_pois = its & 1;
    }
    return batch_finish(b, info, st);
}

// Per-simulation record of a refinement loop (precision 1), as the solo
// solves keep it.
struct Refine {
    double f2 = 0.0, r2 = 0.0;  // |f|^2 and |r|^2 of the FP64 residual
    int inner_its = 0, sweeps = 0;
    InnerRecord inner;
    ccns_status status = CCNS_ENOTCONV;
};

// The inner solves of one sweep have ended: each active simulation's record
// takes its inner solve's iterations and status; one that broke down before
// its first update leaves the loop (its correction is zero), as in the solo
// loop.  Returns whether any left, so that the flags go up again before the
// correction.
bool batch_note_inner(ccns_batch *b, std::vector<Refine> &rec, int o, bool pred) {
    bool changed = false;
    for (size_t k = 0; k < b->sims.size(); ++k) {
        if (!b->act[k]) continue;
        const CgState &h = b->hcg[k];
        rec[k].inner_its += h.it_final;
        ++rec[k].sweeps;
        note_inner(rec[k].inner, h.status, o);
        (pred ? b->sims[k]->last_pred_in : b->sims[k]->last_pois_in) = h.it_final;
        if (h.status == CCNS_EBREAKDOWN && h.it_final == 0) {
            rec[k].status = CCNS_EBREAKDOWN;
            b->act[k] = 0;
            changed = true;
        }
    }
    return changed;
}

ccns_solve_info refine_info(const Refine &r) {
    ccns_solve_info i{};
    i.iterations = r.inner_its;
    i.outer = r.sweeps;
    i.rel_residual = r.f2 > 0.0 ? std::sqrt(r.r2 / r.f2) : 0.0;
    i.status = r.status;
    i.inner_status = r.inner.status;
    i.inner_fail_sweep = r.inner.sweep;
    return i;
}

// One projection step of every simulation in precision 1: the predictor and
// the pressure solves are iterative refinements whose sweeps run in
// lockstep.  Each sweep forms every active simulation's FP64 residual, reads
// all of their statistics in one read-back, decides for each, as its solo
// solve does, whether it has converged and to which tolerance its inner
// float solve runs, then runs the inner solves in lockstep and adds the
// corrections.  A simulation out of the sweep does nothing in its launches.
ccns_status batch_fused_step_mixed(ccns_batch *b, std::vector<ccns_step_info> &info, std::vector<ccns_status> &st) {
    const int n = (int)b->sims.size();
    ccns_status s = batch_begin(b);
    if (s != CCNS_OK) return s;
    std::fill(b->act.begin(), b->act.end(), 1);
    if ((s = batch_upload(b)) != CCNS_OK) return s;
    batch_pred_rhs(b);
    // predictor
    std::vector<Refine> rec(n);
    for (int o = 0;; ++o) {
        blaunch<OpPredResid<true, false, false>>(b, b->pred[0], 0);
        blaunch<OpPredResid<true, true, false>>(b, b->pred[1], 0);
        blaunch<OpPredResid<true, false, true>>(b, b->pred[2], 0);
        blaunch<OpPredResid<true, true, true>>(b, b->pred[3], 0);
        blaunch<OpReduce>(b, b->one, RED_PRED_MIX);
        if ((s = batch_read(b, GAT_PRED_RES)) != CCNS_OK) return s;
        bool any = false;
        int last = 0;
        for (int k = 0; k < n; ++k) {
            if (!b->act[k]) continue;
            const double tol = b->sims[k]->prm.pred_tol;
            rec[k].f2 = b->hst8[(size_t)k * 8 + 5];
            rec[k].r2 = b->hst8[(size_t)k * 8 + 6];
            const double f2 = rec[k].f2, r2 = rec[k].r2;
            if (!(f2 > 0.0) || r2 <= tol * tol * f2) {
                rec[k].status = CCNS_OK;
                b->act[k] = 0;
            } else if (o >= MAX_OUTER) {
                b->act[k] = 0;
            } else {
                const double t = inner_tol(tol * std::sqrt(f2 / r2));
                b->tol2[k] = t * t;
                any = true;
                last = std::max(last, b->sims[k]->last_pred_in);
            }
        }
        if (!any) break;
        if ((s = batch_upload(b)) != CCNS_OK) return s;
        hipLaunchKernelGGL(k_batch_set_tol, dim3((n + NT - 1) / NT), dim3(NT), 0, b->stream, b->dsims, n, 0, b->dtol);
        int its = 0;
        s = batch_cg(b, std::max(4, last + 1), 8, GAT_PRED_IN,
                     [&](int it) { return batch_iterate<float>(b, true, it); }, its);
        if (s != CCNS_OK) return s;
        if (batch_note_inner(b, rec, o, true) && (s = batch_upload(b)) != CCNS_OK) return s;
        blaunch<OpAddCorr>(b, b->fb2, 0);
    }
    for (int k = 0; k < n; ++k) {
        info[k].pred = refine_info(rec[k]);
        b->sims[k]->last_pred_it = rec[k].inner_its;
    }
    // corrector
    std::fill(b->act.begin(), b->act.end(), 1);
    if ((s = batch_upload(b)) != CCNS_OK) return s;
    blaunch<OpPoisRhs>(b, b->dc, 0);
    rec.assign(n, Refine{});
    for (int o = 0;; ++o) {
        blaunch<OpPoisInit<true>>(b, b->dc, o);
        blaunch<OpReduce>(b, b->one, RED_POIS_MIX);
        if ((s = batch_read(b, GAT_POIS_RES)) != CCNS_OK) return s;
        bool any = false;
        int last = 0;
        for (int k = 0; k < n; ++k) {
            if (!b->act[k]) continue;
            const ccns_ctx *c = b->sims[k];
            const ccns_params &p = c->prm;
            const double sdiv = (p.tau / p.rho) / (p.u_ref * std::min(c->g.hx, c->g.hy));
            const double *h = b->hst8 + (size_t)k * 8;
            if (o == 0) rec[k].f2 = h[5];
            rec[k].r2 = h[6];
            const double bn2 = rec[k].f2, rn2 = rec[k].r2, rmax = h[7];
            double need;
            bool conv;
            if (p.div_tol > 0.0) {
                conv = sdiv * rmax <= 0.5 * p.div_tol;
                need = rmax > 0.0 ? 0.5 * p.div_tol / (sdiv * rmax) : 1.0;
            } else {
                conv = rn2 <= p.pcg_tol * p.pcg_tol * bn2;
                need = rn2 > 0.0 ? p.pcg_tol * std::sqrt(bn2 / rn2) : 1.0;
            }
            if (!(bn2 > 0.0) || c->n_active == 0) conv = true;
            if (conv) {
                rec[k].status = CCNS_OK;
                b->act[k] = 0;
            } else if (o >= MAX_OUTER) {
                b->act[k] = 0;
            } else {
                const double t = inner_tol(need);
                b->tol2[k] = t * t;
                any = true;
                last = std::max(last, c->last_pois_in);
            }
        }
        if (!any) break;
        if ((s = batch_upload(b)) != CCNS_OK) return s;
        hipLaunchKernelGGL(k_batch_set_tol, dim3((n + NT - 1) / NT), dim3(NT), 0, b->stream, b->dsims, n, 1, b->dtol);
        batch_vcycle<float>(b);
        int its = 0;
        s = batch_cg(b, std::max(2, last + 1), 2, GAT_POIS_IN,
                     [&](int it) { return batch_iterate<float>(b, false, it); }, its);
        if (s != CCNS_OK) return s;
        if (batch_note_inner(b, rec, o, false) && (s = batch_upload(b)) != CCNS_OK) return s;
        blaunch<OpAddCorr>(b, b->fb1, 1);
    }
    for (int k = 0; k < n; ++k) {
        info[k].poisson = refine_info(rec[k]);
        b->sims[k]->last_pois_it = rec[k].inner_its;
    }
    std::fill(b->act.begin(), b->act.end(), 1);
    if ((s = batch_upload(b)) != CCNS_OK) return s;
    return batch_finish(b, info, st);
}

void batch_free(ccns_batch *b) {
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    if (b->dsims) (void)hipFree(b->dsims);
    if (b->dmap) (void)hipFree(b->dmap);
    if (b->dcg) (void)hipFree(b->dcg);
    if (b->ddg) (void)hipFree(b->ddg);
    if (b->dst8) (void)hipFree(b->dst8);
    batch_drop_graphs(b);
    if (b->dit) (void)hipFree(b->dit);
    if (b->dact) (void)hipFree(b->dact);
    if (b->dtol) (void)hipFree(b->dtol);
    if (b->hcg) (void)hipHostFree(b->hcg);
    if (b->hdg) (void)hipHostFree(b->hdg);
    if (b->hst8) (void)hipHostFree(b->hst8);
    if (b->hring) (void)hipHostFree(b->hring);
    if (b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

}  // namespace

namespace {
// Severity order of statuses for the batch result.
int severity(ccns_status s) {
    switch (s) {
    case CCNS_OK: return 0;
    case CCNS_ENOTCONV: return 1;
    case CCNS_EBREAKDOWN: return 2;
    case CCNS_ESTATE: return 3;
    case CCNS_EINVAL: return 4;
    case CCNS_ENOMEM: return 5;
    default: return 6;  // CCNS_EDEVICE
    }
}
}  // namespace

extern "C" {

ccns_status ccns_batch_create(int n, ccns_ctx *const *ctxs, int nthreads, ccns_batch **out) {
    if (!out) return CCNS_EINVAL;
    *out = nullptr;
    if (n < 1 || !ctxs || nthreads < 0) return CCNS_EINVAL;
    std::vector<ccns_ctx *> v, sorted;
    try {
        v.assign(ctxs, ctxs + n);
        sorted = v;
    } catch (...) {
        return CCNS_ENOMEM;
    }
    for (ccns_ctx *c : v)
        if (!c) return CCNS_EINVAL;
    std::sort(sorted.begin(), sorted.end());
    if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end()) return CCNS_EINVAL;
    ccns_batch *b = new (std::nothrow) ccns_batch();
    if (!b) return CCNS_ENOMEM;
    try {
        b->sims = v;
        b->order.resize(n);
    } catch (...) {
        delete b;
        return CCNS_ENOMEM;
    }
    for (int k = 0; k < n; ++k) b->order[k] = k;
    std::stable_sort(b->order.begin(), b->order.end(), [&](int x, int y) {
        return (long)v[x]->g.nx * v[x]->g.ny > (long)v[y]->g.nx * v[y]->g.ny;
    });
    b->nthreads = nthreads > 0 ? nthreads : std::min(n, 16);
    *out = b;
    return CCNS_OK;
}

ccns_status ccns_batch_create_fused(int n, ccns_ctx *const *ctxs, ccns_batch **out) {
    if (!out) return CCNS_EINVAL;
    *out = nullptr;
    if (n < 1 || n > BATCH_MAX_SIMS || !ctxs || !ctxs[0]) return CCNS_EINVAL;
    const int prec = ctxs[0]->prm.precision;
    for (int k = 0; k < n; ++k)
        if (!ctxs[k] || ctxs[k]->prm.precision != prec || ctxs[k]->prm.precond != 1) return CCNS_EINVAL;
    ccns_batch *b = nullptr;
    ccns_status s = ccns_batch_create(n, ctxs, 1, &b);
    if (s != CCNS_OK) return s;
    b->fused = true;
    b->prec = prec;
    s = CCNS_ENOMEM;
    if (hipStreamCreate(&b->stream) == hipSuccess && hipMalloc(&b->dsims, n * sizeof(BatchSim)) == hipSuccess &&
        hipMalloc(&b->dcg, n * sizeof(CgState)) == hipSuccess &&
        hipMalloc(&b->ddg, n * sizeof(DiagState)) == hipSuccess &&
        hipMalloc(&b->dst8, (size_t)n * 8 * sizeof(double)) == hipSuccess &&
        hipMalloc(&b->dact, n * sizeof(int)) == hipSuccess && hipMalloc(&b->dtol, n * sizeof(double)) == hipSuccess &&
        hipMalloc(&b->dit, sizeof(int)) == hipSuccess &&
        hipHostMalloc(&b->hcg, n * sizeof(CgState)) == hipSuccess &&
        hipHostMalloc(&b->hdg, n * sizeof(DiagState)) == hipSuccess &&
        hipHostMalloc(&b->hst8, (size_t)n * 8 * sizeof(double)) == hipSuccess &&
        hipHostMalloc(&b->hring, BATCH_RING * ring_slot_bytes(n)) == hipSuccess) {
        try {
            b->act.assign(n, 1);
            b->tol2.assign(n, 0.0);
            s = batch_build(b);
        } catch (...) {
            s = CCNS_ENOMEM;
        }
    }
    if (s != CCNS_OK) {
        batch_free(b);
        return s;
    }
    *out = b;
    return CCNS_OK;
}

ccns_status ccns_batch_step(ccns_batch *b, int nsteps, ccns_step_info *per_sim, int *per_status) {
    if (!b || nsteps < 0) return CCNS_EINVAL;
    const int n = (int)b->sims.size();
    std::vector<ccns_status> st;
    std::vector<ccns_step_info> info;
    try {
        st.assign(n, CCNS_OK);
        info.resize(n);
    } catch (...) {
        return CCNS_ENOMEM;
    }
    if (b->fused) {
        ccns_status e = CCNS_OK;
        try {
            for (int k = 0; k < nsteps && e == CCNS_OK; ++k)
                e = b->prec == 1 ? batch_fused_step_mixed(b, info, st) : batch_fused_step(b, info, st);
        } catch (...) {
            e = CCNS_ENOMEM;
        }
        if (e != CCNS_OK) {
            for (int k = 0; k < n; ++k) {
                if (per_sim) per_sim[k] = info[k];
                if (per_status) per_status[k] = e;
            }
            return e;
        }
        ccns_status worst = CCNS_OK;
        for (int k = 0; k < n; ++k) {
            if (severity(st[k]) > severity(worst)) worst = st[k];
            if (per_sim) per_sim[k] = info[k];
            if (per_status) per_status[k] = st[k];
        }
        return worst;
    }
    std::atomic<int> next{0};
    auto worker = [&]() {
        for (;;) {
            const int k = next.fetch_add(1);
            if (k >= n) return;
            const int s = b->order[k];
            st[s] = ccns_step(b->sims[s], nsteps, &info[s]);
        }
    };
    const int nt = std::min(b->nthreads, n);
    std::vector<std::thread> pool;
    try {
        pool.reserve(nt > 1 ? nt - 1 : 0);
        for (int t = 1; t < nt; ++t) pool.emplace_back(worker);
    } catch (...) {
        // fewer threads than asked for: the ones started and this one share the work
    }
    worker();
    for (std::thread &t : pool) t.join();
    ccns_status worst = CCNS_OK;
    for (int s = 0; s < n; ++s) {
        if (severity(st[s]) > severity(worst)) worst = st[s];
        if (per_sim) per_sim[s] = info[s];
        if (per_status) per_status[s] = st[s];
    }
    return worst;
}

ccns_status ccns_batch_graphs(ccns_batch *b, int enable) {
    if (!b || !b->fused || (enable != 0 && enable != 1)) return CCNS_EINVAL;
    if (hipStreamSynchronize(b->stream) != hipSuccess) return CCNS_EDEVICE;
    batch_drop_graphs(b);
    b->graphs = enable == 1;
    return CCNS_OK;
}

void ccns_batch_destroy(ccns_batch *b) { batch_free(b); }

}  // extern "C"
