/*
 * ccns3d -- the projection step of the conservative cut-cell method in three
 * dimensions, on MI355X (gfx950).  Part of libccns.so.
 *
 * The paper states its operators in two dimensions and extends them to
 * three by adding an index (Sec. 2.1, after eq:differentiation); its
 * capacities come from a level set through Marching Cubes or Vofi in 3-D
 * (Sec. 3.1).  These calls carry the first-kind capacities (Sec. 3.2, 3.4)
 * and the projection of Sec. 4.6 to three dimensions for bodies at rest
 * inside a closed box (boundary data D = 0, so the boundary terms of
 * eq:divergence vanish and no second-kind capacity is needed):
 *   (tau / rho) cont(M^-1 pres(Phi), 0) = cont(U*, 0)     (eq:pm_poisson)
 *   U = U* - (tau / rho) M^-1 pres(Phi)                    (eq:pm_projection)
 * with cont and pres of eq:divergence and eq:compatibility on 7-point
 * stencils, M = diag(V_alpha) of the shifted control volumes (Sec. 4.5), and
 * Phi the zero-mean solution (the problem is singular; Sec. 4.6).
 *
 * Conventions (as in ccns.h):
 *  - Host field arrays ("dense layout") are row-major (nz+2) x (ny+2) x
 *    (nx+2) doubles with one ghost layer: cell (i,j,k) at [k][j][i] for i in
 *    1..nx (likewise j, k); x-face (i+1/2, j, k) at [k][j][i] for i in
 *    0..nx (0 and nx on the walls); y- and z-faces likewise.
 *  - Device memory is owned by the caller: one workspace of
 *    ccns3_workspace_bytes() bytes, kept alive until ccns3_ctx_destroy.
 *    All device work is enqueued on the caller's HIP stream, and a call that
 *    reads or writes caller arrays synchronizes that stream before it
 *    returns.
 *  - Functions return a ccns_status, declared in ccns.h; ccns3_last_error()
 *    describes the last failure of a context.
 */
#ifndef CCNS3D_H
#define CCNS3D_H

#include <stddef.h>

#include "ccns.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Uniform grid of nx*ny*nz cells of hx*hy*hz, lower corner (x0, y0, z0). */
typedef struct {
    int nx, ny, nz;
    double x0, y0, z0;
    double hx, hy, hz;
} ccns3_grid;

enum { CCNS3_SPHERE = 0, CCNS3_ZCYLINDER = 1 };

/* A solid body (fluid lies outside it).  Sphere: centre (cx, cy, cz),
 * radius r.  Z-cylinder: the infinite cylinder of radius r about the line
 * through (cx, cy) parallel to z (cz unused).  The bodies of one call are
 * disjoint. */
typedef struct {
    int kind;
    double cx, cy, cz, r;
} ccns3_body;

/* rho: density (> 0); tau: time step (> 0); tol: relative residual of the
 * Poisson solve, ||r||_2 <= tol ||b||_2; maxit: iteration limit of the
 * solve; mass_floor: theta, the smallest shifted volume the projection
 * divides by is theta hx hy hz (M_f = max(V_f, theta hx hy hz); 0 gives
 * M = diag(V) exactly); precond: the CG's preconditioner, 0 Jacobi
 * (1 / diag), 1 a geometric multigrid V-cycle (2x2x2 agglomeration, half
 * the sum of the covered fine face weights on each coarse face, weighted
 * Jacobi two sweeps down and two up, the dense pseudo-inverse on a coarsest
 * grid of at most 256 cells), 2 the same cycle with its fields stored in
 * FP32 (FP64 arithmetic; the CG itself stays FP64).  The projection method
 * leaves the solver open (Sec. 4.6); all three reach the same FP64
 * tolerance test. */
typedef struct {
    double rho, tau, tol, mass_floor;
    int maxit;
    int precond;
} ccns3_params;

/* Figures of one projection.  div_rel: max over the pressure unknowns of
 * |cont(U, 0)| after the correction, over the largest face flux |A U|. */
typedef struct {
    int iterations;
    int status;          /* ccns_status of the Poisson solve */
    double rel_residual; /* ||r||_2 / ||b||_2 of the recursively updated residual */
    double div_rel;
    int n_active;        /* pressure unknowns */
} ccns3_info;

/* Number of doubles ccns3_capacities writes: 7 arrays of
 * (nx+2)(ny+2)(nz+2) in the dense layout, in the order V (cells), A^x, A^y,
 * A^z (faces), V^x, V^y, V^z (the control volumes of the x-, y- and z-face
 * unknowns).  0 for an invalid grid. */
size_t ccns3_caps_count(const ccns3_grid *grid);

/* First-kind capacities of the fluid outside the bodies (Sec. 3.2:
 * eq:volumefirstkind, eq:surfacefirstkindx/y with a third index; Sec. 3.4
 * for the half-cell shifted volumes), on the host.  Face areas are plane
 * sections in closed form; volumes are integrals along x of the section
 * areas (adaptive Gauss-Kronrod split where the section circle meets the
 * rectangle's lines and corners).  Values below 1e-12 of the full face or
 * cell are set to 0.  V^alpha is written on the interior faces only (0 on
 * the walls, which carry no unknown).  out: ccns3_caps_count() doubles,
 * caller-owned.  Returns CCNS_EINVAL for a bad grid or body (r <= 0 or not
 * finite, unknown kind). */
ccns_status ccns3_capacities(const ccns3_grid *grid, const ccns3_body *bodies, int nbodies, double *out);

/* Bytes of device workspace a context needs: the solver's fields and, for
 * the multigrid preconditioner, its coarse levels (about one field more) and
 * the coarsest grid's dense pseudo-inverse.  0 for an invalid grid, or for
 * one whose padded fields exceed 2^31 - 1 elements (the kernels index them
 * in 32 bits; about 1,290^3 cells). */
size_t ccns3_workspace_bytes(const ccns3_grid *grid);

typedef struct ccns3_ctx ccns3_ctx;

/* Creates a context from the capacities (host, ccns3_caps_count() doubles
 * in the order of ccns3_capacities) and derives on the host the velocity and
 * pressure unknowns and the Poisson face weights:
 *  - a face is a velocity unknown when it is interior, A > 0 and V^alpha > 0;
 *  - c_f = A_f^2 / max(V_f, theta hx hy hz) on the unknowns;
 *  - the pressure unknowns are the largest set of fluid cells connected
 *    through faces with c_f > 0, and c_f is kept only between two of them.
 * workspace: device memory of at least ccns3_workspace_bytes(), 256-byte
 * aligned, caller-owned.  stream: a hipStream_t (NULL: the null stream).
 * The velocity and Phi start at zero.  Errors: CCNS_EINVAL (bad grid,
 * params, NaN or negative capacity), CCNS_ENOMEM (workspace too small),
 * CCNS_EDEVICE. */
ccns_status ccns3_ctx_create(const ccns3_grid *grid, const ccns3_params *params, const double *caps_host,
                             void *workspace, size_t workspace_bytes, void *stream, ccns3_ctx **out);
void ccns3_ctx_destroy(ccns3_ctx *ctx);

enum { CCNS3_F_UX = 0, CCNS3_F_UY = 1, CCNS3_F_UZ = 2, CCNS3_F_PHI = 3, CCNS3_NFIELDS = 4 };

/* Copies a field from (is_device = 0: host, else device) memory in the dense
 * layout into the context; the ghost layer is read as given.  Before
 * ccns3_project the velocity fields hold U*, and PHI the initial guess of
 * the Poisson solve. */
ccns_status ccns3_field_set(ccns3_ctx *ctx, int field, const double *src, int is_device);
/* Copies a field out of the context into dense-layout memory. */
ccns_status ccns3_field_get(ccns3_ctx *ctx, int field, double *dst, int is_device);

/* The projection step (Sec. 4.6 in three dimensions): b = -(rho/tau)
 * cont(U*, 0) on the pressure unknowns minus its mean; preconditioned CG
 * (params.precond) on (-L) Phi = b from the current PHI, L = cont(M^-1 pres(.), 0); PHI
 * minus its mean over the unknowns; then U = U* - (tau/rho) M^-1 pres(PHI)
 * on the faces with c_f > 0, U* on the other unknowns and 0 on every other
 * face.  info (may be NULL) receives the solve's figures.  Returns the
 * solve's status (CCNS_ENOTCONV or CCNS_EBREAKDOWN leave the last iterate in
 * PHI and its projection in U).  The tolerance is relative to ||b||: a field
 * that is already divergence-free has b at rounding level, which a solve
 * started from a nonzero PHI cannot reach relative to itself, so such a
 * projection starts from PHI = 0. */
ccns_status ccns3_project(ccns3_ctx *ctx, ccns3_info *info);

/* out = -L in on the cells (device arrays, dense layout): sum over the six
 * faces of c_f (in_c - in_nb) on the pressure unknowns, 0 elsewhere.  For
 * checking the operator the solve uses. */
ccns_status ccns3_apply_poisson(ccns3_ctx *ctx, const double *in_dev, double *out_dev);

/* Live timing of the Poisson CG's kernels with HIP events around each
 * launch on the context's stream: ms[0], count[0] the direction-and-operator
 * kernel, ms[1], count[1] the update kernel, ms[2], count[2] (multigrid
 * only) the finest level's first up-sweep of the cycle, accumulated over the
 * launches that did an iteration's work since the last reset; ms and count
 * point to 3 elements each.  enable: 1 on, 0 off,
 * -1 leave unchanged; 0 and 1 also reset the accumulators (after they are
 * returned).  ms and count may be NULL. */
ccns_status ccns3_timing(ccns3_ctx *ctx, int enable, double *ms, long *count);

const char *ccns3_last_error(const ccns3_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif
