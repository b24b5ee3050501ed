// Device-side building blocks shared by the kernels of libccns: work
// distribution over tiles, deterministic reductions without atomics, and the
// index form of the staggered operators (Sec. 4).
#ifndef CCNS_KERN_H
#define CCNS_KERN_H

#include <hip/hip_runtime.h>

#include <cstddef>

namespace ccns {

constexpr int NT = 256;     // threads per work-group (4 wavefronts)
constexpr int TX = 64;      // tile width: one wavefront per tile row
constexpr int TY = 8;       // tile rows of the face kernels and simple cell kernels
constexpr int NBMAX = 512;  // at most this many work-groups per kernel

// A field grid split in tiles of TX x ty entries.  Work-group b works on a
// contiguous range of tpb tiles; groups are numbered so that each of the 8
// XCDs (which receive groups round-robin) owns a contiguous band of rows, so
// the halo rows of a tile are in the L2 of the XCD that needs them.
struct Dims {
    int nx, ny, rows, pitch;
    int gx, gy, ntile, ncomp;  // tiles per component, components (1 cells, 2 faces)
    int ty;                    // tile rows (multiple of 4)
    int tpb;                   // tiles per work-group
    int nblk;                  // work-groups launched (multiple of 8)
    size_t n;                  // entries per component array (rows * pitch)
};

// The work-group's place in the grid of one simulation.  A kernel launched
// for one simulation is that grid (SoloGrid: blockIdx.x of gridDim.x); a
// batched launch runs the work-groups of many simulations' grids side by
// side, and each group gets its index and count within its own simulation's
// share (SubGrid).  The kernels' arithmetic sees only these two numbers, so a
// simulation computes the same values in either kind of launch.
struct SoloGrid {
    __device__ int b() const { return (int)blockIdx.x; }
    __device__ int n() const { return (int)gridDim.x; }
};
struct SubGrid {
    int bb, nn;
    __device__ int b() const { return bb; }
    __device__ int n() const { return nn; }
};

template <class G>
__device__ inline int logical_group(const G &g, int nblk) {
    const int b = g.b();
    return (b & 7) * (nblk >> 3) + (b >> 3);
}
__device__ inline int logical_group(int nblk) { return logical_group(SoloGrid{}, nblk); }

// Calls f(comp, c0, r0) for every tile of this work-group.
template <class G, class F>
__device__ inline void for_tiles(const G &g, const Dims &d, F f) {
    const int L = logical_group(g, d.nblk);
    const int total = d.ntile * d.ncomp;
    const int t0 = L * d.tpb, t1 = min(t0 + d.tpb, total);
    for (int t = t0; t < t1; ++t) {
        const int comp = t / d.ntile, tt = t - comp * d.ntile;
        f(comp, (tt % d.gx) * TX, (tt / d.gx) * d.ty);
    }
}
template <class F>
__device__ inline void for_tiles(const Dims &d, F f) {
    for_tiles(SoloGrid{}, d, f);
}

// Calls f(comp, j, i, k) for every entry of this work-group's tiles.
template <class G, class F>
__device__ inline void for_cells(const G &g, const Dims &d, F f) {
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for_tiles(g, d, [&](int comp, int c0, int r0) {
        const int i = c0 + tx;
        for (int rr = ty; rr < d.ty; rr += 4) {
            const int j = r0 + rr;
            if (j < d.rows) f(comp, j, i, (size_t)j * d.pitch + i);
        }
    });
}
template <class F>
__device__ inline void for_cells(const Dims &d, F f) {
    for_cells(SoloGrid{}, d, f);
}

// The same for tiles of exactly 4 R rows, in two passes per tile: load(k)
// for each of the thread's R entries (k = 0 stands in for entries past the
// last row), then f(comp, j, i, k, loaded value) for the real ones.  All of
// a thread's loads are then in flight together instead of one entry's loads
// waiting for the previous entry's.
template <int R, class G, class LD, class F>
__device__ inline void for_cells_batched(const G &g, const Dims &d, LD load, F f) {
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for_tiles(g, d, [&](int comp, int c0, int r0) {
        const int i = c0 + tx;
        decltype(load((size_t)0)) vals[R];
#pragma unroll
        for (int m = 0; m < R; ++m) {
            const int j = r0 + ty + 4 * m;
            vals[m] = load(j < d.rows ? (size_t)j * d.pitch + i : (size_t)0);
        }
#pragma unroll
        for (int m = 0; m < R; ++m) {
            const int j = r0 + ty + 4 * m;
            if (j < d.rows) f(comp, j, i, (size_t)j * d.pitch + i, vals[m]);
        }
    });
}
template <int R, class LD, class F>
__device__ inline void for_cells_batched(const Dims &d, LD load, F f) {
    for_cells_batched<R>(SoloGrid{}, d, load, f);
}

// ---------------------------------------------------------------------------
// reductions: wavefront shuffles, one block pass, per-group partials stored
// slot-major (part[slot * nblk + group]); the consumer (the next kernel, or a
// one-group kernel) sums them in a fixed order.  No atomics, no fences: the
// kernel boundary makes the partials visible, and every result is
// reproducible bit for bit.
// ---------------------------------------------------------------------------

__device__ inline double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}
__device__ inline double wave_max(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
    return v;
}

// Block-level reduction of NS sums followed by NM maxima over a work-group
// of BT threads; the result is in out[] for every thread.  The wavefront
// results are combined in a fixed order (adjacent pairs, level by level).
template <int NS, int NM, int BT = NT>
__device__ inline void block_reduce(const double (&v)[NS + NM], double (&out)[NS + NM]) {
    constexpr int NW = BT / 64;
    __shared__ double part[NS + NM][NW];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NS + NM; ++k) {
        const double s = (k < NS) ? wave_sum(v[k]) : wave_max(v[k]);
        if (lane == 0) part[k][w] = s;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NS + NM; ++k) {
        double q[NW];
#pragma unroll
        for (int i = 0; i < NW; ++i) q[i] = part[k][i];
#pragma unroll
        for (int m = NW; m > 1; m /= 2)
#pragma unroll
            for (int i = 0; i < m / 2; ++i)
                q[i] = (k < NS) ? q[2 * i] + q[2 * i + 1] : fmax(q[2 * i], q[2 * i + 1]);
        out[k] = q[0];
    }
    __syncthreads();
}

template <int NS, int NM = 0, int BT = NT, class G>
__device__ inline void put_partials(const G &g, const double (&v)[NS + NM], double *part, int nblk) {
    double t[NS + NM];
    block_reduce<NS, NM, BT>(v, t);
    if (threadIdx.x == 0) {
        const int b = g.b();
#pragma unroll
        for (int k = 0; k < NS + NM; ++k) part[(size_t)k * nblk + b] = t[k];
    }
}
template <int NS, int NM = 0, int BT = NT>
__device__ inline void put_partials(const double (&v)[NS + NM], double *part, int nblk) {
    put_partials<NS, NM, BT>(SoloGrid{}, v, part, nblk);
}

template <int NS, int NM = 0, int BT = NT>
__device__ inline void get_totals(const double *part, int nblk, double (&tot)[NS + NM]) {
    double a[NS + NM];
#pragma unroll
    for (int k = 0; k < NS + NM; ++k) a[k] = (k < NS) ? 0.0 : -INFINITY;
    // U groups' values in flight per thread (groups of 1024 threads have no
    // registers to spare), then a remainder; the order of the sums is fixed
    // by (nblk, BT)
    constexpr int U = BT >= 1024 ? 1 : 4;
    int b = threadIdx.x;
    for (; b + (U - 1) * BT < nblk; b += U * BT) {
        double x[U][NS + NM];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int k = 0; k < NS + NM; ++k) x[u][k] = part[(size_t)k * nblk + b + u * BT];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int k = 0; k < NS + NM; ++k) a[k] = (k < NS) ? a[k] + x[u][k] : fmax(a[k], x[u][k]);
    }
    for (; b < nblk; b += BT) {
#pragma unroll
        for (int k = 0; k < NS + NM; ++k) {
            const double x = part[(size_t)k * nblk + b];
            a[k] = (k < NS) ? a[k] + x : fmax(a[k], x);
        }
    }
    block_reduce<NS, NM, BT>(a, tot);
}

// ---------------------------------------------------------------------------
// operators in index form (k = j*pitch + i)
// ---------------------------------------------------------------------------

struct ViscCoef {
    const double *bxx, *bxy, *byy, *byx, *wxx, *wyy, *nxx, *nxy, *nyx, *nyy;
};

// visc(strain(p, 0)) at x-face k (eq:diag, eq:offdiag, Sec. 4.3) for a face
// vector given by loaders px(k), py(k).
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

}  // namespace ccns

#endif
