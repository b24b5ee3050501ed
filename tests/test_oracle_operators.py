"""Pins of the oracle's operators (Sec. 2.3, Sec. 4) against what the paper
and the mathematics fix: the printed worked examples, the literal Morinishi
compositions versus the expanded index forms, constant-state preservation,
summation by parts, the kinetic-energy identity of the convective term
(eq:kinetic), skew-symmetry for divergence-free fluxes, symmetry and
definiteness of the viscous operator, exactness for linear shear between
mesh-aligned cut walls, and the classical MAC formulas away from bodies."""

import json
import os

import numpy as np
import pytest

import workloads as W
from oracle import calculus as C
from oracle import geometry
from oracle import operators as ops
from oracle.solvers import assemble

GOLD = os.path.join(os.path.dirname(__file__), "golden", "worked_examples_1d.json")


def _ev(expr, env):
    return float(eval(expr, {"__builtins__": {}}, env))


# ---------------------------------------------------------------------------
# worked examples (Sec. 2.2, Sec. 2.3)
# ---------------------------------------------------------------------------

def _row_arrays(ex, env, key_cells, faces_key):
    """1-D layout along x (one row, padded): cell k at column k+2, face
    (k+1/2) at column k+2."""
    ncol = 8
    cells = np.zeros((3, ncol))
    faces = np.zeros((3, ncol))
    for k, e in enumerate(ex[key_cells]):
        cells[1, k + 2] = _ev(e, env)
    for name, e in ex[faces_key].items():
        num = int(name.split("/")[0])      # "-1/2" -> -1, "3/2" -> 3
        k = (num - 1) // 2                 # face between cells k and k+1
        faces[1, k + 2] = _ev(e, env)
    return cells, faces


def test_worked_example_gradD_and_poisson_rows():
    gold = json.load(open(GOLD))["gradD"]
    env = dict(f=0.23, g=0.71, hx=1.0, hy=0.6, T1=1.3, T2=-0.4, T3=2.2, D1=0.9)
    _, A = _row_arrays(gold, env, "V", "A_faces")
    B, Wf = _row_arrays(gold, env, "B", "W_faces")
    T = np.zeros_like(B)
    D = np.zeros_like(B)
    T[1, 3:6] = [env["T1"], env["T2"], env["T3"]]
    D[1, 3] = env["D1"]
    Q = ops.gradD_lit(A, B, Wf, T, D, "x")
    for name, e in gold["Q"].items():
        k = (int(name.split("/")[0]) - 1) // 2
        assert abs(Q[1, k + 2] - _ev(e, env)) < 1e-14, name
    # Poisson rows: divergence with the boundary closure N = Q
    rows = ops.divN_lit(A, B, Q, Q, "x")
    pr = gold["poisson_rows"]
    for cell in (0, 1, 2):
        assert abs(rows[1, cell + 2] - _ev(pr[f"cell{cell}"], env)) < 1e-13
    # divergence rows with an independent boundary value N at the dry face
    N = Q.copy()
    N[1, 2] = 0.37
    rows = ops.divN_lit(A, B, Q, N, "x")
    dr = gold["divergence_rows"]
    env2 = dict(env, Q3h=Q[1, 3], Q5h=Q[1, 4], N1h=0.37)
    assert abs(rows[1, 3] - _ev(dr["cell1"], env2)) < 1e-13
    assert abs(rows[1, 4] - _ev(dr["cell2"], env2)) < 1e-13


def test_worked_example_tentative_gradient_fails_by_factor_two():
    gold = json.load(open(GOLD))["v2"]
    env = dict(g=0.4, hx=1.0, hy=0.7, T1=1.1, T2=2.9, D1=0.3)
    V, A = _row_arrays(gold, env, "V", "A_faces")
    T = np.zeros_like(V)
    D = np.zeros_like(V)
    T[1, 3:5] = [env["T1"], env["T2"]]
    D[1, 3] = env["D1"]
    Q = ops.grad_v2_lit(A, V, T, D, "x")
    for name, e in gold["Q"].items():
        k = (int(name.split("/")[0]) - 1) // 2
        assert abs(Q[1, k + 2] - _ev(e, env)) < 1e-14, name
    # the boundary value is half of the exact one-sided derivative over g/2
    exact = (env["T1"] - env["D1"]) / (env["g"] / 2)
    assert abs(Q[1, 2] / exact - 0.5) < 1e-14


# ---------------------------------------------------------------------------
# literal compositions == expanded forms
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def rcaps():
    return W.random_capacities(9, 7, seed=11, hx=0.3, hy=0.2, zero_frac=0.1)


def _rand(shape, seed):
    return W.random_field(shape, seed)


def test_literal_equals_expanded(rcaps):
    c = rcaps
    sh = c["V"].shape
    Ux, Uy, Dx, Dy, P, Utx, Uty, Dtx, Dty = [_rand(sh, 100 + k) for k in range(9)]
    s = np.s_[1:-1, 1:-1]
    a, b = ops.cont(c, Ux, Uy, Dx, Dy), ops.cont_lit(c, Ux, Uy, Dx, Dy)
    assert np.allclose(a[s], b[s], rtol=1e-14, atol=1e-15)
    (px, py), (lx, ly) = ops.pres(c, P), ops.pres_lit(c, P)
    assert np.allclose(px[1:-1, 1:-2], lx[1:-1, 1:-2], atol=1e-15)
    assert np.allclose(py[1:-2, 1:-1], ly[1:-2, 1:-1], atol=1e-15)
    Sxx, Syy, Sx, Sy = ops.strain(c, Ux, Uy, Dx, Dy, "literal")
    L = ops.strain_lit(c, Ux, Uy, Dx, Dy)
    sc = np.max(np.abs(L[0][s]))
    assert np.allclose(Sxx[s], L[0][s], atol=1e-14 * sc)
    assert np.allclose(Syy[s], L[1][s], atol=1e-14 * np.max(np.abs(L[1][s])))
    # the printed form reads the node capacities of the neighbouring nodes
    # (they cancel), so it is defined one node in from the array edge
    n = np.s_[1:-2, 1:-2]
    assert np.allclose(Sx[n], L[2][n], atol=1e-14 * np.max(np.abs(L[2][n])))
    assert np.allclose(Sy[n], L[2][n], atol=1e-14 * np.max(np.abs(L[2][n])))
    vx, vy = ops.visc(c, Sxx, Syy, Sx, Sy)
    wx, wy = ops.visc_lit(c, L[0], L[1], L[2])
    sx, sy = np.s_[2:-2, 1:-2], np.s_[1:-2, 2:-2]
    assert np.allclose(vx[sx], wx[sx], atol=1e-13 * np.max(np.abs(wx[sx])))
    assert np.allclose(vy[sy], wy[sy], atol=1e-13 * np.max(np.abs(wy[sy])))
    cx, cy = ops.conv(c, Ux, Uy, Utx, Uty, Dx, Dy, Dtx, Dty)
    kx, ky = ops.conv_lit(c, Ux, Uy, Utx, Uty, Dx, Dy, Dtx, Dty)
    assert np.allclose(cx[1:-1, 1:-2], kx[1:-1, 1:-2], atol=1e-15)
    assert np.allclose(cy[1:-2, 1:-1], ky[1:-2, 1:-1], atol=1e-15)
    assert np.allclose(ops.kinetic(c, Ux, Uy)[s], ops.kinetic_lit(c, Ux, Uy)[s], atol=1e-15)


def test_divergence_of_boundary_closure(rcaps):
    """eq:divD: div(Q, Q) summed over alpha equals sum_beta B_beta dQ_beta/dxi_beta."""
    c = rcaps
    sh = c["V"].shape
    Qx, Qy = _rand(sh, 7), _rand(sh, 8)
    lhs = ops.divN_lit(c["Ax"], c["Bx"], Qx, Qx, "x") + ops.divN_lit(c["Ay"], c["By"], Qy, Qy, "y")
    rhs = (C.F(c["Bx"], "c") * C.d_x(C.F(Qx, "u"))).a + (C.F(c["By"], "c") * C.d_y(C.F(Qy, "v"))).a
    s = np.s_[1:-1, 1:-1]
    assert np.allclose(lhs[s], rhs[s], atol=1e-14)


# ---------------------------------------------------------------------------
# structure
# ---------------------------------------------------------------------------

def test_summation_by_parts(rcaps):
    """eq:compatibility: <P, cont(U, 0)> = -<pres(P), U> over all real faces,
    and the assembled matrices satisfy G = -D^T entry by entry."""
    c = rcaps
    ny, nx = c["V"].shape[0] - 2, c["V"].shape[1] - 2
    sh = c["V"].shape
    P = np.zeros(sh)
    P[1:-1, 1:-1] = _rand((ny, nx), 3)
    Ux, Uy = np.zeros(sh), np.zeros(sh)
    Ux[1:-1, 0:nx + 1] = _rand((ny, nx + 1), 4)
    Uy[0:ny + 1, 1:-1] = _rand((ny + 1, nx), 5)
    z = np.zeros(sh)
    lhs = np.sum(P * ops.cont(c, Ux, Uy, z, z))
    px, py = ops.pres(c, P)
    rhs = -(np.sum(px * Ux) + np.sum(py * Uy))
    assert abs(lhs - rhs) < 1e-13 * (abs(lhs) + 1)
    # entry-wise on assembled matrices
    mask_p = np.zeros(sh, bool)
    mask_p[1:-1, 1:-1] = True
    mu = np.zeros(sh, bool)
    mu[1:-1, 0:nx + 1] = True
    idx_p = np.flatnonzero(mask_p.ravel())
    idx_u = np.flatnonzero(mu.ravel())
    Dm = np.zeros((len(idx_p), len(idx_u)))
    for k, g in enumerate(idx_u):
        e = np.zeros(sh).ravel()
        e[g] = 1.0
        Dm[:, k] = ops.cont(c, e.reshape(sh), z, z, z).ravel()[idx_p]
    Gm = np.zeros((len(idx_u), len(idx_p)))
    for k, g in enumerate(idx_p):
        e = np.zeros(sh).ravel()
        e[g] = 1.0
        Gm[:, k] = ops.pres(c, e.reshape(sh))[0].ravel()[idx_u]
    assert np.array_equal(Gm, -Dm.T)


@pytest.fixture(scope="module")
def c1caps():
    case = W.cylinder_64()
    return geometry.capacities(case.grid, case.bodies), case


def test_constant_states_are_preserved(c1caps):
    c, case = c1caps
    sh = c["V"].shape
    k = 1.7
    U = np.full(sh, k)
    V = np.full(sh, -0.6)
    s = np.s_[1:-1, 1:-1]
    assert np.max(np.abs(ops.cont(c, U, V, U, V)[s])) < 1e-15
    px, py = ops.pres(c, np.full(sh, 3.0))
    assert np.max(np.abs(px[1:-1, 1:-2])) == 0.0 and np.max(np.abs(py[1:-2, 1:-1])) == 0.0
    cx, cy = ops.conv(c, U, V, U, V, U, V, U, V)
    assert np.max(np.abs(cx)) < 1e-16 and np.max(np.abs(cy)) < 1e-16
    for form in ("literal", "geometric", "mean"):
        vx, vy = ops.viscous(c, U, V, U, V, form)
        assert np.max(np.abs(vx)) < 1e-12 and np.max(np.abs(vy)) < 1e-12


def _stream_velocity(c, psi):
    """Velocity whose mass fluxes are a discrete curl: A^x U^x = psi_{j+1/2} - psi_{j-1/2},
    A^y U^y = -(psi_{i+1/2} - psi_{i-1/2}), so cont(U, 0) = 0 in every cell."""
    Ux = np.zeros_like(psi)
    Uy = np.zeros_like(psi)
    Ux[1:, :] = (psi[1:, :] - psi[:-1, :]) * C.safe_inv(c["Ax"][1:, :])
    Uy[:, 1:] = -(psi[:, 1:] - psi[:, :-1]) * C.safe_inv(c["Ay"][:, 1:])
    return Ux, Uy


def test_kinetic_energy_identity_of_convection(rcaps):
    """eq:kinetic, face by face, with D != 0 and U+ != U (eq:u-dot-qdm with the
    permanent product eq:permanent)."""
    c = rcaps
    sh = c["V"].shape
    Ux, Uy, Utx, Uty, Dx, Dy, Dtx, Dty = [_rand(sh, 40 + k) for k in range(8)]
    cx, cy = ops.conv(c, Ux, Uy, Utx, Uty, Dx, Dy, Dtx, Dty)
    F = C.F
    fx, fy = F(c["Ax"] * Ux, "u"), F(c["Ay"] * Uy, "v")
    utx, uty = F(Utx, "u"), F(Uty, "v")
    Bx, By, Ax, Ay = F(c["Bx"], "c"), F(c["By"], "c"), F(c["Ax"], "u"), F(c["Ay"], "v")
    dx, dy = F(Dx, "u"), F(Dy, "v")
    cnt = F(ops.cont(c, Ux, Uy, Dx, Dy), "c")
    brx = (C.d_x(C.i_x((C.i_x(Bx) - Ax) * dx)) - C.i_x(C.i_x(C.d_x(Bx) * dx))
           + C.d_y(C.i_x((C.i_y(By) - Ay) * dy)) - C.i_x(C.i_y(C.d_y(By) * dy)))
    rhs_x = (C.d_x(C.i_x(fx) * C.p_x(utx, utx) * 0.5) + C.d_y(C.i_x(fy) * C.p_y(utx, utx) * 0.5)
             + brx * (utx * F(Dtx, "u") * 0.5) + utx * utx * 0.5 * C.i_x(cnt))
    bry = (C.d_x(C.i_y((C.i_x(Bx) - Ax) * dx)) - C.i_y(C.i_x(C.d_x(Bx) * dx))
           + C.d_y(C.i_y((C.i_y(By) - Ay) * dy)) - C.i_y(C.i_y(C.d_y(By) * dy)))
    rhs_y = (C.d_x(C.i_y(fx) * C.p_x(uty, uty) * 0.5) + C.d_y(C.i_y(fy) * C.p_y(uty, uty) * 0.5)
             + bry * (uty * F(Dty, "v") * 0.5) + uty * uty * 0.5 * C.i_y(cnt))
    sx, sy = np.s_[2:-2, 2:-3], np.s_[2:-3, 2:-2]
    assert np.allclose((Utx * cx)[sx], rhs_x.a[sx], atol=1e-14)
    assert np.allclose((Uty * cy)[sy], rhs_y.a[sy], atol=1e-14)


def test_convection_skew_symmetric_for_divergence_free_flux(rcaps):
    """With cont(U, 0) = 0 and D = 0, V -> conv(U, V, 0, 0) is skew-symmetric on
    fields vanishing on the walls, so U^T conv(U, U) = 0."""
    c = dict(rcaps)
    for k in ("Ax", "Ay"):   # all faces wetted so the curl construction is defined
        c[k] = np.where(c[k] > 0, c[k], 0.5 * np.max(c[k]))
    sh = c["V"].shape
    psi = np.zeros(sh)
    psi[1:-2, 1:-2] = _rand((sh[0] - 3, sh[1] - 3), 9)
    Ux, Uy = _stream_velocity(c, psi)
    z = np.zeros(sh)
    assert np.max(np.abs(ops.cont(c, Ux, Uy, z, z)[1:-1, 1:-1])) < 1e-14
    ny, nx = sh[0] - 2, sh[1] - 2
    mu = np.zeros(sh, bool)
    mu[1:-1, 1:nx] = True
    mv = np.zeros(sh, bool)
    mv[1:ny, 1:-1] = True
    Wx = np.where(mu, _rand(sh, 10), 0.0)
    Wy = np.where(mv, _rand(sh, 11), 0.0)
    Vx = np.where(mu, _rand(sh, 12), 0.0)
    Vy = np.where(mv, _rand(sh, 13), 0.0)
    a = ops.conv(c, Ux, Uy, Wx, Wy, z, z, z, z)
    b = ops.conv(c, Ux, Uy, Vx, Vy, z, z, z, z)
    lhs = np.sum(Vx * a[0] * mu) + np.sum(Vy * a[1] * mv)
    rhs = -(np.sum(Wx * b[0] * mu) + np.sum(Wy * b[1] * mv))
    assert abs(lhs - rhs) < 1e-13 * (abs(lhs) + 1.0)
    Um = (np.where(mu, Ux, 0.0), np.where(mv, Uy, 0.0))
    cu = ops.conv(c, Ux, Uy, Um[0], Um[1], z, z, z, z)
    e = np.sum(Um[0] * cu[0] * mu) + np.sum(Um[1] * cu[1] * mv)
    assert abs(e) < 1e-13 * np.sqrt(np.sum(Um[0] ** 2) + np.sum(Um[1] ** 2)) * np.max(np.abs(cu[0]))


def _visc_matrix(c, mu_mask, mv_mask, form):
    sh = c["V"].shape
    m2 = np.stack([mu_mask, mv_mask])
    z = np.zeros(sh)

    def K(U2):
        vx, vy = ops.viscous(c, np.where(mu_mask, U2[0], 0), np.where(mv_mask, U2[1], 0), z, z, form)
        return np.stack([np.where(mu_mask, vx, 0.0), np.where(mv_mask, vy, 0.0)])

    A, _ = assemble(K, m2)
    return A.toarray()


def _body_box_masks():
    g = W.GridSpec(8, 8, 0.0, 0.0, 1.0, 1.0)
    body = W.Body(W.CIRCLE, 0.47, 0.52, a=0.21)
    c = geometry.capacities(g, [body])
    sh = c["V"].shape
    J, I = np.indices(sh)
    mu = (I >= 1) & (I <= 7) & (J >= 1) & (J <= 8) & (c["Vu"] > 0)
    mv = (I >= 1) & (I <= 8) & (J >= 1) & (J <= 7) & (c["Vv"] > 0)
    return c, mu, mv


def test_viscous_operator_symmetric_negative_definite():
    c, mu, mv = _body_box_masks()
    K = _visc_matrix(c, mu, mv, "geometric")
    assert np.max(np.abs(K - K.T)) < 1e-13 * np.max(np.abs(K))
    ev = np.linalg.eigvalsh(0.5 * (K + K.T))
    assert ev.max() < 0.0
    Km = _visc_matrix(c, mu, mv, "mean")
    assert np.max(np.abs(Km - Km.T)) < 1e-13 * np.max(np.abs(Km))
    # the printed node strain is not symmetric where W^xy != W^yx
    Kl = _visc_matrix(c, mu, mv, "literal")
    asym = np.max(np.abs(Kl - Kl.T)) / np.max(np.abs(Kl))
    assert asym > 1e-3


def test_linear_shear_between_mesh_aligned_walls_is_exact():
    """Couette flow U = a (y - y0), V = 0 between horizontal walls cutting
    through cells: the viscous term vanishes on every unknown (first-order
    exactness of the strain at mesh-aligned boundaries, Sec. 2.3)."""
    g = W.GridSpec(6, 8, 0.0, 0.0, 0.6, 0.8)
    y0, y1 = 0.137, 0.618
    geo = geometry.LevelSetGeometry(phi=lambda x, y: np.minimum(np.asarray(y, float) - y0, y1 - np.asarray(y, float)) + 0 * np.asarray(x, float))
    c = geometry.capacities(g, [], geo=geo)
    a = 2.3
    sh = c["V"].shape
    Ux = np.where(c["Vu"] > 0, a * (c["Yu"] - y0), 0.0)
    Uy = np.zeros(sh)
    # wall velocities: 0 on the lower wall, a (y1 - y0) on the upper one
    Dx = np.where(c["Yu"] > 0.5 * (y0 + y1), a * (y1 - y0), 0.0)
    # the wall-normal faces of the box carry the profile itself (U = D there)
    Dx[:, 0] = Ux[:, 0]
    Dx[:, g.nx] = Ux[:, g.nx]
    Dy = np.zeros(sh)
    for form in ("literal", "geometric"):
        vx, vy = ops.viscous(c, Ux, Uy, Dx, Dy, form)
        J, I = np.indices(sh)
        act = (I >= 1) & (I <= g.nx - 1) & (J >= 1) & (J <= g.ny) & (c["Vu"] > 0)
        # y-faces beside the box's side walls are left out: there the cut
        # x-volumes of the wall faces would need two Dirichlet values at once
        actv = (I >= 2) & (I <= g.nx - 1) & (J >= 1) & (J <= g.ny - 1) & (c["Vv"] > 0)
        assert np.max(np.abs(vx[act])) < 1e-13, form
        assert np.max(np.abs(vy[actv])) < 1e-13, form


def test_classical_mac_away_from_bodies():
    """No body, uniform grid: the operators reduce to the textbook MAC formulas
    (the full-cell reductions of the 1-D example of Sec. 2.3, written here
    directly in h)."""
    g = W.GridSpec(7, 6, 0.0, 0.0, 0.7, 0.9)
    hx, hy = g.hx, g.hy
    c = geometry.capacities(g, [])
    sh = c["V"].shape
    u, v, Pm = _rand(sh, 1), _rand(sh, 2), _rand(sh, 3)
    z = np.zeros(sh)
    cont = ops.cont(c, u, v, u, v)
    for j in range(1, g.ny + 1):
        for i in range(1, g.nx + 1):
            ref = hy * (u[j, i] - u[j, i - 1]) + hx * (v[j, i] - v[j - 1, i])
            assert abs(cont[j, i] - ref) < 1e-14
    vx, vy = ops.viscous(c, u, v, z, z, "geometric")
    cx, cy = ops.conv(c, u, v, u, v, z, z, z, z)
    for j in range(2, g.ny):
        for i in range(2, g.nx - 1):
            lap = (hy / hx) * (u[j, i + 1] - 2 * u[j, i] + u[j, i - 1]) \
                + 0.5 * (hx / hy) * (u[j + 1, i] - 2 * u[j, i] + u[j - 1, i]) \
                + 0.5 * ((v[j, i + 1] - v[j, i]) - (v[j - 1, i + 1] - v[j - 1, i]))
            assert abs(vx[j, i] - lap) < 1e-13
            ue = 0.5 * (u[j, i] + u[j, i + 1])
            uw = 0.5 * (u[j, i - 1] + u[j, i])
            vn = 0.5 * (v[j, i] + v[j, i + 1])
            vs = 0.5 * (v[j - 1, i] + v[j - 1, i + 1])
            un = 0.5 * (u[j, i] + u[j + 1, i])
            us = 0.5 * (u[j - 1, i] + u[j, i])
            ref = hy * (ue * ue - uw * uw) + hx * (vn * un - vs * us)
            assert abs(cx[j, i] - ref) < 1e-14
    px, py = ops.pres(c, Pm)
    for j in range(1, g.ny + 1):
        for i in range(1, g.nx):
            assert abs(px[j, i] - hy * (Pm[j, i + 1] - Pm[j, i])) < 1e-15
