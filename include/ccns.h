/*
 * ccns -- conservative cut-cell Navier-Stokes hot path on MI355X (gfx950).
 *
 * C interface of the device library libccns.so.  The calls follow the
 * statement of the discrete problem in Quiros Rodriguez, Fullana,
 * Le Chenadec, Sayadi, "A Conservative Cartesian Cut Cell Method for the
 * Solution of the Incompressible Navier-Stokes Equations on Staggered
 * Meshes": geometry in (Sec. 3.1), capacities (Sec. 3.2-3.4), the staggered
 * operators (Sec. 4.1-4.4), and the projection method II time step
 * (Sec. 4.6).
 *
 * Conventions shared by every call
 *  - Host field arrays ("dense layout") are row-major (ny+2) x (nx+2) doubles
 *    with one ghost ring: cell (i,j) at [j][i]; x-face (i+1/2, j) at [j][i];
 *    y-face (i, j+1/2) at [j][i]; node (i+1/2, j+1/2) at [j][i].  Real cells
 *    are 1..nx x 1..ny; real x-faces i = 0..nx (0 and nx on the walls).
 *  - Device memory is owned by the caller: one workspace buffer of
 *    ccns_workspace_bytes() bytes, passed to ccns_ctx_create and kept alive
 *    until ccns_ctx_destroy.  The library never allocates device memory
 *    itself.  All device work is enqueued on the caller's HIP stream.
 *  - Functions return a ccns_status.  No C++ exception crosses the
 *    interface.  On error, ccns_last_error() describes the failure.
 *  - A context is not thread-safe; use one context per host thread.
 *  - Device arrays passed to a call must be ready when it is made: the
 *    library orders its own work on the context's stream only, and
 *    synchronizes that stream before any call that reads or writes caller
 *    arrays returns.
 */
#ifndef CCNS_H
#define CCNS_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CCNS_OK = 0,
    CCNS_EINVAL = -1,      /* bad argument (sizes, NaN/negative capacity, rho<=0 ...) */
    CCNS_ENOMEM = -2,      /* workspace smaller than ccns_workspace_bytes() */
    CCNS_ENOTCONV = -3,    /* an iterative solve hit its iteration limit; outputs hold the last iterate */
    CCNS_EBREAKDOWN = -4,  /* CG breakdown (p^T A p <= 0); outputs hold the last iterate */
    CCNS_EDEVICE = -5,     /* a HIP runtime call failed */
    CCNS_ESTATE = -6       /* call not valid in the context's current state */
} ccns_status;

/* Cartesian grid of nx*ny cells, lower-left corner (x0, y0).  The cell
 * edges are the abscissas of Sec. 3.1.
 *
 * xf = yf = NULL: a uniform grid of cells hx*hy.
 * xf != NULL: the nx+1 cell-edge abscissas x_{1/2} .. x_{nx+1/2}, finite and
 *   strictly increasing, with xf[0] = x0 (likewise yf, ny+1 ordinates): a
 *   stretched rectilinear mesh.  The ghost cells beyond the walls repeat the
 *   width of their neighbours.  The metric enters the method through the
 *   capacities alone, so hx and hy are then reference spacings (the smallest
 *   ones, say): they scale the small-capacity thresholds, the mass floor
 *   theta hx hy and the divergence diagnostic.
 * Only ccns_capacities reads xf and yf, during the call (the caller keeps
 * ownership); the other entry points take the grid for its sizes and
 * reference spacings and the capacities for its geometry. */
typedef struct {
    int nx, ny;
    double x0, y0, hx, hy;
    const double *xf, *yf;
} ccns_grid;

/* Synthetic bodies.  Fluid is where the body's level set is positive.
 *  CCNS_CIRCLE : centre (cx, cy), radius a
 *  CCNS_ELLIPSE: centre (cx, cy), semi-axes a, b, rotation `angle` (rad)
 *  CCNS_NACA4  : symmetric NACA 4-digit section, leading edge (cx, cy),
 *                chord `chord`, thickness ratio t, angle of attack `angle`
 *                (nose up: trailing edge below the leading edge). */
enum { CCNS_CIRCLE = 0, CCNS_ELLIPSE = 1, CCNS_NACA4 = 2 };
typedef struct {
    int kind;
    double cx, cy, a, b, angle, chord, t;
} ccns_body;

/* A user level set: returns > 0 in the fluid. */
typedef double (*ccns_levelset_fn)(double x, double y, void *user);

/* Capacity arrays, each in the dense host layout, stored one after the other
 * in this order (the symbols of Sec. 3.2-3.4; staggered-grid names
 * A^{xx} etc. as in Sec. 3.4):
 *   V Ax Ay Bx By Wx Wy | Vu Axx Axy Bxx Bxy Wxx Wxy | Vv Ayy Ayx Byy Byx Wyy Wyx */
enum {
    CCNS_CAP_V = 0, CCNS_CAP_AX, CCNS_CAP_AY, CCNS_CAP_BX, CCNS_CAP_BY, CCNS_CAP_WX, CCNS_CAP_WY,
    CCNS_CAP_VU, CCNS_CAP_AXX, CCNS_CAP_AXY, CCNS_CAP_BXX, CCNS_CAP_BXY, CCNS_CAP_WXX, CCNS_CAP_WXY,
    CCNS_CAP_VV, CCNS_CAP_AYY, CCNS_CAP_AYX, CCNS_CAP_BYY, CCNS_CAP_BYX, CCNS_CAP_WYY, CCNS_CAP_WYX,
    CCNS_NCAPS
};

/* Number of doubles ccns_capacities writes: CCNS_NCAPS*(ny+2)*(nx+2). */
size_t ccns_caps_count(const ccns_grid *grid);

/* Capacities of the first and second kind (eq:volumefirstkind, eq:centroid,
 * eq:surfacefirstkindx/y, eq:volumesecondkindx/y, eq:surfacesecondkindx/y)
 * on the pressure grid and the two half-cell shifted velocity grids
 * (Sec. 3.4), computed on the host from the fluid level set.
 * The fluid is outside every body in `bodies` (nbody >= 0) and, if `fn` is
 * not NULL, also where fn(x, y, user) > 0.  Box reading: each grid's fluid
 * lies inside its own box (the pressure box; the velocity grids' boxes
 * extend half a cell across their own normal walls); node lines on the
 * tangential walls are dry; pressure-grid wall faces are wetted.
 * caps_host: caller-owned host buffer of ccns_caps_count() doubles.
 * Capacities below 1e-12 h (lengths) or 1e-12 hx hy (volumes) are 0.
 * On a stretched grid (xf or yf set) every control volume, face and strip
 * takes the extents of its own edges and centroids.
 * Errors: CCNS_EINVAL for a bad grid (abscissas not finite and strictly
 * increasing, xf[0] != x0, yf[0] != y0) or body. */
ccns_status ccns_capacities(const ccns_grid *grid, const ccns_body *bodies, int nbody,
                            ccns_levelset_fn fn, void *user, double *caps_host);

/* The capacities of ccns_capacities computed on the device, for bodies bounded
 * by conics (circles and ellipses, at most 16, whose circumscribed discs do
 * not overlap; no user level set): the same arrays, layout and readings (each
 * grid's box, wet pressure-grid wall faces, centroid of an empty control
 * volume at its centre, exact measures of full control volumes, faces and
 * strips, capacities below 1e-12 h or 1e-12 hx hy set to 0).  The measure of
 * the fluid in a rectangle or on a segment is in closed form: the chords of a
 * conic along vertical and horizontal lines, integrated piecewise between the
 * points where they cross the rectangle's rows (Sec. 3.2-3.4).
 *  caps_dev     device buffer of ccns_caps_count() doubles (caller-owned)
 *  dev_scratch  device buffer of ccns_capacities_scratch_bytes() bytes for
 *               the control volumes' centroids (caller-owned)
 *  hip_stream   the work is enqueued on it; the call does not wait
 * Errors: CCNS_EINVAL (bad grid, a stretched grid, a body that is not a
 * circle or an ellipse, overlapping bodies, more than 16 bodies),
 * CCNS_ENOMEM (scratch too small),
 * CCNS_EDEVICE. */
size_t ccns_capacities_scratch_bytes(const ccns_grid *grid);
ccns_status ccns_capacities_device(const ccns_grid *grid, const ccns_body *bodies, int nbody,
                                   double *caps_dev, void *dev_scratch, size_t scratch_bytes,
                                   void *hip_stream);

/* Solver parameters.
 *  rho, mu, tau   density, dynamic viscosity, time step (> 0)
 *  u_ref          reference velocity of the divergence diagnostic
 *  gx, gy         gravity (body force rho*M*g of eq:semidiscrete)
 *  pcg_tol        Poisson: stop when ||r||_2 <= pcg_tol ||b||_2
 *  pred_tol       predictor: same criterion
 *  div_tol        precision 1: the pressure refinement stops once
 *                 (tau/rho) max|r| / (u_ref min(hx,hy)) <= div_tol / 2, which
 *                 bounds the step's div_rel by div_tol; 0 selects the 2-norm
 *                 test with pcg_tol instead
 *  pcg_maxit, pred_maxit   iteration limits
 *  precision      0 = FP64 throughout; 1 = iterative refinement: each sweep
 *                 forms the residual in FP64 with FP64 coefficients, solves
 *                 for the correction with float vectors, float coefficients
 *                 and float stencils (dot products summed in FP64), and adds
 *                 it in FP64.  Both solves; the predictor stops at the same
 *                 2-norm test as in precision 0 (pred_tol).  The state and
 *                 every explicit phase stay FP64.
 *  visc_form      node strain weights: 0 symmetric (geometric mean of the two
 *                 node volumes for the cross coupling), 1 as printed in
 *                 eq:offdiag (not symmetric; apply only), 2 arithmetic mean
 *  poisson_weight 0: Poisson face weight A^2/V_f (mass matrix explicit);
 *                 1: A^2 (the printed equations with unit mass matrix)
 *  mass_floor     theta in [0, 1]: every volume the step divides by is at
 *                 least theta hx hy: the mass matrix of the time derivative
 *                 and of the projection, M_f = max(V_f, theta hx hy) on
 *                 velocity unknowns, and the cell volume of the pressure
 *                 update, V^-1 -> 1/max(V, theta hx hy).  theta = 0 gives
 *                 M = V exactly.  A sliver cell with open faces otherwise
 *                 turns the pressure update's volume average into a spike
 *                 that the next predictor feeds back (an instability that
 *                 grows by orders of magnitude per step).
 *  precond        Poisson preconditioner: 0 Jacobi (diagonal); 1 geometric
 *                 multigrid V-cycle (2x2 cell agglomeration, weighted-Jacobi
 *                 smoothing, pseudo-inverse on the coarsest grid).  The
 *                 paper does not fix the solver; both converge to the same
 *                 solution of eq:pm_poisson.
 *  coef_tables    0: the predictor's kernels (right-hand side, residual and
 *                 CG, FP64 and the float inner CG of precision 1) read their
 *                 coefficients through a table of the distinct coefficient
 *                 neighbourhoods (one index per entry) when there are at
 *                 most max(1024, n/16) of them (n: entries of the padded
 *                 layout), else from the coefficient arrays; 1: always from
 *                 the arrays.  Both read the same values: the results are
 *                 identical bit for bit.
 *  outflow        walls with a homogeneous Neumann velocity and a zero
 *                 pressure beyond them (end of Sec. 4.6), a sum of
 *                 CCNS_WALL_W/E/S/N (0: Dirichlet data on every wall).  Each
 *                 step takes the velocity of the faces normal to such a wall
 *                 from the interior face next to them (zero normal gradient,
 *                 from U^n), likewise the tangential velocity beyond the wall
 *                 that the convective flux through it reads; the projection
 *                 corrects the outflow faces with the pressure beyond the
 *                 wall held at zero, so the Poisson problem is not singular
 *                 and no mean is removed.  The Dirichlet data of those faces
 *                 are then unused: the cells next to an outflow wall must be
 *                 uncut (CCNS_EINVAL otherwise), where the data cancel out of
 *                 every operator.
 *  mg_forms       kernel forms of the multigrid cycle's down- and up-sweep
 *                 kernels, per cycle level (level 0 the finest): level l in
 *                 bits 6l..6l+2 (down) and 6l+3..6l+5 (up), for l < 10:
 *                 0 the default, 1 staged first sweep with the tile ring's
 *                 operands in registers, 2 the same with them in LDS, 3 first
 *                 sweep pointwise on 64 x 16 tiles, 4 the same on 64 x 4
 *                 tiles, 5 form 2 on 64 x 8 tiles (4 and 5 not for level
 *                 0's up-sweep, whose tiles fix the order of the
 *                 preconditioner's statistics).  Every form
 *                 computes the same values bit for bit; they differ in speed
 *                 by level size (see ccns_mg_levels).
 */
#define CCNS_WALL_W 1
#define CCNS_WALL_E 2
#define CCNS_WALL_S 4
#define CCNS_WALL_N 8
#define CCNS_MG_FORM_STAGED 1
#define CCNS_MG_FORM_STAGED_LDS 2
#define CCNS_MG_FORM_PLAIN 3
#define CCNS_MG_FORM_PLAIN_SHORT 4
#define CCNS_MG_FORM_STAGED_LDS_HALF 5
typedef struct {
    double rho, mu, tau, u_ref, gx, gy;
    double pcg_tol, pred_tol, div_tol;
    int pcg_maxit, pred_maxit;
    int precision;
    int visc_form;
    int poisson_weight;
    int precond;
    double mass_floor;
    int coef_tables;
    int outflow;
    unsigned long long mg_forms;
} ccns_params;

typedef struct ccns_ctx ccns_ctx;

/* Device workspace needed for a context on this grid (bytes). */
size_t ccns_workspace_bytes(const ccns_grid *grid, const ccns_params *params);

/* Create a context: validates the capacities (no NaN, no negative value),
 * derives the activity masks and coefficient fields (Poisson face weights,
 * corrector factors, viscous node/cell weights, Jacobi diagonals, the
 * Dirichlet contributions cont(0,D) and visc(strain(U~,D))), and uploads
 * everything into the workspace on `hip_stream`.
 *  caps_host   ccns_caps_count() doubles (ccns_capacities layout)
 *  dirichlet_host  2*(ny+2)*(nx+2) doubles: D^x then D^y (dense layout);
 *              the staggered Dirichlet data of Sec. 4, constant in time.
 *  dev_workspace   device buffer of ws_bytes >= ccns_workspace_bytes()
 *  hip_stream  hipStream_t (NULL = default stream)
 * With coef_tables = 0 it also builds the predictor's coefficient classes
 * (host work of one pass over the layout) and uploads their table.
 * Errors: CCNS_EINVAL (also for precision, precond or coef_tables out of
 * range), CCNS_ENOMEM, CCNS_EDEVICE. */
ccns_status ccns_ctx_create(const ccns_grid *grid, const ccns_params *params,
                            const double *caps_host, const double *dirichlet_host,
                            void *dev_workspace, size_t ws_bytes, void *hip_stream,
                            ccns_ctx **out);
void ccns_ctx_destroy(ccns_ctx *ctx);
const char *ccns_last_error(const ccns_ctx *ctx);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): ccns_ctx_create without a
 * workspace argument.  The context uses the library's static workspace of
 * the current device, an array of CCNS_STATIC_WORKSPACE_BYTES (64 MiB) that
 * each device the library runs on holds until the process ends, and calls no
 * hipMalloc, hipHostMalloc, hipFree or other allocating routine (its host
 * copies of the solver state live in the context record, which is on the host
 * heap as every context is).  Everything else is as ccns_ctx_create: the same
 * kernels, the same results bit for bit.
 *  - Size limit: ccns_workspace_bytes(grid, params) <= 64 MiB, e.g. grids up to
 *    256 x 256 cells in either precision; larger ones fail with CCNS_ENOMEM.
 *  - One such context per device at a time: the workspace is shared, so a
 *    second call while one lives on the current device fails with
 *    CCNS_ESTATE; ccns_ctx_destroy releases it.  The workspace keeps the last
 *    context's contents; creation clears all of it.
 *  - ccns_timing cannot be enabled on it (HIP events are allocated).
 * Errors: as ccns_ctx_create, plus CCNS_ENOMEM (too large) and CCNS_ESTATE. */
#define CCNS_STATIC_WORKSPACE_BYTES ((size_t)64 << 20)
ccns_status ccns_ctx_create_static(const ccns_grid *grid, const ccns_params *params,
                                   const double *caps_host, const double *dirichlet_host,
                                   void *hip_stream, ccns_ctx **out);

/* Number of coefficient classes the predictor's kernels of this context
 * read (see coef_tables in ccns_params); 0 when they read the coefficient
 * arrays, -1 for a null context. */
int ccns_coef_classes(const ccns_ctx *ctx);

/* Fields held in the workspace (FP64). */
enum {
    CCNS_F_UX = 0,   /* U^x, x-faces */
    CCNS_F_UY,       /* U^y, y-faces */
    CCNS_F_P,        /* pressure P^{n-1/2}, cells */
    CCNS_F_PHI,      /* last Poisson solution Phi^n (warm start), cells */
    CCNS_F_CONVX,    /* conv^{n-1}, x-faces */
    CCNS_F_CONVY,
    CCNS_F_USX,      /* predicted U* of the last step, x-faces */
    CCNS_F_USY,
    CCNS_F_B,        /* Poisson right-hand side of the last solve, cells */
    CCNS_NFIELDS
};

/* Copy a field between the workspace and a dense (ny+2)x(nx+2) array.
 * `is_device` != 0: the array is device memory, else host memory.
 * Setting CCNS_F_UX/UY: faces that are not velocity unknowns (on a wall
 * normal to them, without fluid in their control volume, or closed, A = 0)
 * take the Dirichlet value whatever the array holds there, except the
 * outflow faces and the tangential velocity beyond an outflow wall, which
 * the step carries as state.
 * Setting CCNS_F_CONVX/Y marks conv^{n-1} as valid (otherwise the first
 * step takes conv^{-1} := conv^0).  Errors: CCNS_EINVAL (bad field). */
ccns_status ccns_field_set(ccns_ctx *ctx, int field, const double *src, int is_device);
ccns_status ccns_field_get(ccns_ctx *ctx, int field, double *dst, int is_device);

/* Operator applies on dense device arrays (FP64), for parity checks.
 *  CCNS_OP_CONT : in = {Ux, Uy}  out = {c}     c = cont(U, D) (eq:divergence), cells
 *  CCNS_OP_PRES : in = {P}       out = {gx, gy} pres(P) = A dP/dxi (eq:compatibility), real faces
 *  CCNS_OP_VISC : in = {Ux, Uy}  out = {vx, vy} visc(strain(U, D)) (eq:diag, eq:offdiag, Sec. 4.3), interior faces
 *  CCNS_OP_CONV : in = {Ux, Uy}  out = {cx, cy} conv(U, U, D, D) (eq:convective), interior faces
 *  CCNS_OP_LAP  : in = {phi}     out = {q}     q = L phi = cont(M^-1 pres(phi), 0), active cells
 *  CCNS_OP_H    : in = {px, py}  out = {hx, hy} H p = (rho/tau) V p - mu visc(strain(p, 0)), unknown faces
 *  CCNS_OP_KINETIC: in = {Ux, Uy} out = {k}    kinetic(U) (Sec. 4.5), cells
 * D is the context's Dirichlet data.  U is read on the unknowns and, for
 * CCNS_OP_CONT, CCNS_OP_VISC and CCNS_OP_CONV, on every face (outflow faces
 * included; elsewhere the caller passes D there).  Outputs are written on
 * the index range stated and set to 0 elsewhere.  in/out: arrays of device pointers to dense
 * (ny+2)x(nx+2) doubles.  Errors: CCNS_EINVAL (unknown op). */
enum { CCNS_OP_CONT = 0, CCNS_OP_PRES, CCNS_OP_VISC, CCNS_OP_CONV, CCNS_OP_LAP, CCNS_OP_H, CCNS_OP_KINETIC };
ccns_status ccns_apply(ccns_ctx *ctx, int op, const double *const *in, double *const *out);

typedef struct {
    int iterations;        /* CG iterations (precision 1: inner iterations of all sweeps) */
    int outer;             /* refinement sweeps (precision 1), else 1 */
    double rel_residual;   /* final ||r||_2 / ||b||_2 (FP64) */
    int status;            /* ccns_status of this solve */
    int inner_status;      /* precision 1: CCNS_EBREAKDOWN if an inner solve broke down, else
                              CCNS_ENOTCONV if one hit its iteration limit, else CCNS_OK;
                              precision 0: CCNS_OK */
    int inner_fail_sweep;  /* precision 1: first sweep whose inner solve did not converge, -1 if
                              none.  An inner breakdown before its first update ends the solve
                              with status CCNS_EBREAKDOWN (the next sweep would repeat it). */
} ccns_solve_info;

typedef struct {
    ccns_solve_info pred;  /* predictor solve (eq:pm_prediction) */
    ccns_solve_info poisson; /* pressure solve (eq:pm_poisson) */
    double div_max;        /* max |cont(U^{n+1}, D)| over pressure unknowns */
    double div_rel;        /* div_max / (u_ref * min(hx, hy)) */
    double ke;             /* sum of kinetic(U^{n+1}) over cells (Sec. 4.5) */
    double mass;           /* sum of cont(U^{n+1}, D) over cells (net boundary flux) */
    double mom_x, mom_y;   /* sum of rho V_alpha U_alpha over unknown faces */
} ccns_step_info;

/* Pressure solve (eq:pm_poisson, Sec. 4.6 with the zero-mean projection):
 * solves L phi = b on the pressure unknowns by CG with the context's
 * preconditioner (params.precond: Jacobi or the multigrid V-cycle; in
 * precision 1 inside the FP64 refinement loop), starting from the current
 * CCNS_F_PHI, after removing the mean of b where the problem is singular
 * (no outflow wall).
 * b, phi: dense device arrays (phi may be NULL: the result stays in
 * CCNS_F_PHI).  Errors: CCNS_ENOTCONV, CCNS_EBREAKDOWN (outputs written). */
ccns_status ccns_pressure_solve(ccns_ctx *ctx, const double *b, double *phi, ccns_solve_info *info);

/* Make the current velocity discretely divergence-free (the initial
 * projection): Poisson from cont(U, D), then the corrector.  P is unchanged. */
ccns_status ccns_project(ccns_ctx *ctx, ccns_step_info *info);

/* Advance nsteps projection-method-II time steps (eq:pm_prediction,
 * eq:pm_poisson, eq:pm_projection, eq:pm_update).  info (may be NULL)
 * receives the last step's figures.  The state stays on the device; the host
 * reads a few scalars per step.  Errors: CCNS_ENOTCONV, CCNS_EBREAKDOWN. */
ccns_status ccns_step(ccns_ctx *ctx, int nsteps, ccns_step_info *info);

/* The phases of one step, for inspection:
 *  ccns_predict  conv^n and the predictor solve (writes CCNS_F_USX/USY)
 *  ccns_correct  Poisson right-hand side from U*, pressure solve, corrector
 *                and pressure update (writes U, P, PHI, B) */
ccns_status ccns_predict(ccns_ctx *ctx, ccns_solve_info *info);
ccns_status ccns_correct(ccns_ctx *ctx, ccns_step_info *info);

/* Kernel timing for measurement.  While enabled, iterations 4, 12, 20, ...
 * of each CG solve (never the first, whose kernels do less) are bracketed
 * with HIP events on the context's stream.
 * ms[4] and count[4] (may be NULL) receive the accumulated milliseconds and
 * launch counts since the last reset, in the order: Poisson
 * direction+operator kernel, Poisson update with the preconditioner that
 * follows it, predictor CG iteration kernel, reduction of its partial
 * products.  enable: 1 on, 0 off, -1 leave unchanged; 0 and 1 also reset
 * the accumulators (after they are returned). */
ccns_status ccns_timing(ccns_ctx *ctx, int enable, double *ms, long *count);

/* Diagnostics of the current state (FP64 reductions on the device). */
ccns_status ccns_diagnostics(ccns_ctx *ctx, ccns_step_info *info);

/* Force of the fluid on the bodies for the current state (P of the last
 * step, U), a reading of the drag and lift that Sec. 5 reports without a
 * discrete formula: the momentum the fluid exchanges with the bodies through
 * the capacities in eq:semidiscrete.  With S the strain of eq:diag and
 * eq:offdiag on (U, D) (node strains S_x, S_y of the x and y rows):
 *   F^p_x = sum_cells P (A^x_{i-1/2} - A^x_{i+1/2}),  F^p_y likewise in y
 *   F^v_x = 2 mu [sum_cells S_xx (B^xx_{i+1/2} - B^xx_{i-1/2})
 *                 + sum_nodes S_x (B^xy above - B^xy below)],  F^v_y likewise
 * over the cells and the nodes off the box's walls; only cut cells and nodes
 * contribute (bodies clear of the walls).  Summed by one work-group in a
 * fixed order.  Drag and lift coefficients: (F^p + F^v) / (rho U^2 L / 2).
 *  forces_host  caller-owned host array of 4 doubles:
 *               {F^p_x, F^p_y, F^v_x, F^v_y}; the call waits for them
 * Errors: CCNS_EINVAL (null argument), CCNS_ENOMEM (more cut cells or nodes
 * than the context's table holds: 8 (nx + ny) + 1024 each), CCNS_EDEVICE. */
ccns_status ccns_forces(ccns_ctx *ctx, double *forces_host);

/* Multigrid cycle kernel forms (see ccns_params.mg_forms), for tuning.
 * ccns_set_mg_forms: the forms of the context's next cycles (0 restores the
 * defaults); the results do not change.  Errors: CCNS_EINVAL (a field above
 * 5, level 0's up-sweep in form 4 or 5, or bits above level 9).
 * ccns_mg_levels: the number of cycle levels (levels with down- and
 * up-sweep kernels, at most 10; 0 without the multigrid preconditioner); for
 * the first `cap` of them writes the cells nx[l] x ny[l] and the forms in
 * use, forms[l] = down | up << 3 (host arrays, caller-owned, may be NULL). */
ccns_status ccns_set_mg_forms(ccns_ctx *ctx, unsigned long long forms);
int ccns_mg_levels(const ccns_ctx *ctx, int *nx, int *ny, int *forms, int cap);

/* Batches of independent simulations of any sizes (the ragged batches of
 * many uneven simulations that share one GPU).  A batch borrows contexts
 * the caller created and still owns; each should have its own HIP stream,
 * so that the kernels of different simulations run concurrently.
 *
 * ccns_batch_create: n >= 1 distinct contexts; nthreads host threads drive
 *   them (each runs whole projection steps of one simulation at a time, the
 *   largest simulations first; 0 = one per simulation up to 16).  Errors:
 *   CCNS_EINVAL (n < 1, NULL or repeated context, nthreads < 0).
 * ccns_batch_step: advances every simulation by nsteps projection steps,
 *   exactly as ccns_step on each context alone would (the kernels' fixed
 *   reduction order makes each result bit-identical to a solo run).
 *   per_sim (may be NULL): n ccns_step_info, the last step of each;
 *   per_status (may be NULL): n statuses.  Returns the worst status:
 *   CCNS_EDEVICE if any simulation hit a device error, else a solver status
 *   (CCNS_ENOTCONV, CCNS_EBREAKDOWN) if any, else CCNS_OK.
 * ccns_batch_destroy: frees the batch (not the contexts).
 *
 * ccns_batch_create_fused: a batch whose steps run each phase of every
 *   simulation in one launch (one per kernel variant): the work-groups of
 *   all simulations' grids side by side, each group on its own
 *   simulation's arrays through a table of (simulation, group) entries, on
 *   the batch's own HIP stream.  The conjugate-gradient solves run in
 *   lockstep: each simulation keeps its own solver state, a simulation
 *   whose solve has stopped does nothing in the later launches, and the
 *   host reads all stopping flags in one read-back per chunk of iterations.
 *   In precision 1 the refinement sweeps run in lockstep too: each sweep
 *   forms every simulation's FP64 residual, reads all of their statistics
 *   in one read-back, takes each simulation's decisions (converged, or the
 *   tolerance of its inner float solve) as its solo solve does, and runs
 *   the inner solves of the simulations still refining together.  Each
 *   simulation's kernels, and so its results, are those of its solo steps
 *   bit for bit.  1 <= n <= 1024 distinct contexts on the current device,
 *   all of one precision, each with the multigrid preconditioner (precond
 *   1); ccns_batch_step and ccns_batch_destroy as above.  A step waits for
 *   each context's stream before it starts and returns after its own work
 *   ends; the contexts must not be used elsewhere meanwhile.  Errors:
 *   CCNS_EINVAL (n out of range, a NULL or repeated context, precisions
 *   that differ, the Jacobi preconditioner), CCNS_ENOMEM (device or host
 *   memory for the batch's tables), CCNS_EDEVICE. */
typedef struct ccns_batch ccns_batch;
ccns_status ccns_batch_create(int n, ccns_ctx *const *ctxs, int nthreads, ccns_batch **out);
ccns_status ccns_batch_create_fused(int n, ccns_ctx *const *ctxs, ccns_batch **out);

/* Fused batches: each conjugate-gradient iteration of all simulations (its
 * launches of every kernel variant, the multigrid cycle included) is
 * captured once as a HIP graph and replayed per iteration, the iteration
 * number kept in device memory (enable = 1, the default); with enable = 0
 * every launch is queued one by one.  The results are the same bit for bit.
 * A capture the runtime refuses turns the graphs off.  Errors: CCNS_EINVAL
 * (NULL, not a fused batch, enable not 0 or 1), CCNS_EDEVICE. */
ccns_status ccns_batch_graphs(ccns_batch *batch, int enable);
ccns_status ccns_batch_step(ccns_batch *batch, int nsteps, ccns_step_info *per_sim, int *per_status);
void ccns_batch_destroy(ccns_batch *batch);

#ifdef __cplusplus
}
#endif
#endif /* CCNS_H */
