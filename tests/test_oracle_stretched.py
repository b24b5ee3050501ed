"""Pins of the oracle on stretched rectilinear meshes (user-defined abscissas,
Sec. 3.1): the capacities carry the metric, so the operators of Sec. 4 need
no change.  Checked against what the mathematics fixes:

  * the fluid area is the box minus the body, exactly;
  * without a body the operators are the textbook finite-volume forms on a
    non-uniform mesh: cont = dy (u_e - u_w) + dx (v_n - v_s), the Poisson
    operator's face weight dy / (x_{i+1} - x_i) (centre to centre), pres the
    face length times the pressure difference;
  * linear fields are differentiated exactly: the strains of a linear
    velocity sampled at the staggered centroids are its constant gradients,
    so visc vanishes on interior faces, and L of a linear pressure sampled
    at the cell centroids vanishes on interior cells;
  * with a body, the divergence identity of the step and the symmetry and
    positive definiteness of H hold;
  * the projection step stays second order in space and time on a smoothly
    stretched mesh (Taylor-Green vortex with exact time-dependent Dirichlet
    data): the error falls by about 4 per halving."""

import math

import numpy as np

import workloads as W
from oracle import derived, geometry, operators as ops, pmii
from oracle.solvers import assemble


def _grid(nx=12, ny=10, ax=0.5, ay=0.4, lx=1.2, ly=1.0):
    return W.GridSpec(nx, ny, 0.0, 0.0, lx, ly, xf=W.stretched_edges(nx, 0.0, lx, ax),
                      yf=W.stretched_edges(ny, 0.0, ly, ay))


def test_spacing_varies():
    g = _grid()
    dx = np.diff(g.xf)
    assert dx.max() / dx.min() > 2.5
    assert abs(g.edges(0)[1] - 0.0) == 0.0 and abs(g.edges(0)[g.nx + 1] - 1.2) < 1e-15


def test_area_of_a_circle_on_a_stretched_mesh():
    g = _grid(40, 32)
    c = geometry.capacities(g, [W.Body(W.CIRCLE, 0.53, 0.47, a=0.21)])
    area = g.lx * g.ly - math.pi * 0.21 ** 2
    assert abs(c["V"][1:-1, 1:-1].sum() - area) < 1e-13 * area
    # first moment of the fluid: the box's minus the disc's
    J, I = np.indices(c["V"].shape)
    mx = (c["V"] * c["X"])[1:-1, 1:-1].sum()
    ref = 0.5 * g.lx ** 2 * g.ly - math.pi * 0.21 ** 2 * 0.53
    assert abs(mx - ref) < 1e-13 * abs(ref)


def test_textbook_finite_volume_forms_without_body():
    g = _grid()
    c = geometry.capacities(g, [])
    xe, ye, xc, yc = g.edges(0), g.edges(1), g.centres(0), g.centres(1)
    dx, dy = np.diff(xe), np.diff(ye)          # cell widths, cells 0 .. n+1
    rng = np.random.default_rng(4)
    sh = c["V"].shape
    u, v, P = rng.uniform(-1, 1, sh), rng.uniform(-1, 1, sh), rng.uniform(-1, 1, sh)
    cont = ops.cont(c, u, v, u, v)
    for j in range(1, g.ny + 1):
        for i in range(1, g.nx + 1):
            ref = dy[j] * (u[j, i] - u[j, i - 1]) + dx[i] * (v[j, i] - v[j - 1, i])
            assert abs(cont[j, i] - ref) < 1e-14
            assert abs(c["V"][j, i] - dx[i] * dy[j]) < 1e-15
    px, py = ops.pres(c, P)
    for j in range(1, g.ny + 1):
        for i in range(1, g.nx):
            assert abs(px[j, i] - dy[j] * (P[j, i + 1] - P[j, i])) < 1e-14
    pr = derived.prepare(c, g.nx, g.ny)
    L = derived.laplacian(pr, np.where(pr.act_p, P, 0.0))
    Pm = np.where(pr.act_p, P, 0.0)
    for j in range(2, g.ny):
        for i in range(2, g.nx):
            w = lambda a, b: dy[j] / (xc[b] - xc[a])       # noqa: E731
            s = lambda a, b: dx[i] / (yc[b] - yc[a])       # noqa: E731
            ref = (w(i, i + 1) * (Pm[j, i + 1] - Pm[j, i]) - w(i - 1, i) * (Pm[j, i] - Pm[j, i - 1])
                   + s(j, j + 1) * (Pm[j + 1, i] - Pm[j, i]) - s(j - 1, j) * (Pm[j, i] - Pm[j - 1, i]))
            assert abs(L[j, i] - ref) < 1e-13 * (1 + abs(ref))


def test_linear_fields_are_differentiated_exactly():
    g = _grid()
    c = geometry.capacities(g, [])
    xe, ye, xc, yc = g.edges(0), g.edges(1), g.centres(0), g.centres(1)
    # the second-kind capacities span the distances between centroids
    # (Sec. 3.3), so a linear velocity is sampled at the centroids of the
    # staggered control volumes; on a stretched mesh these lie between two
    # cell centres, not on the face
    XU, YU, XV, YV = c["Xu"], c["Yu"], c["Xv"], c["Yv"]
    a, b, cc, d = 0.7, -0.3, 0.4, 0.9
    u, v = a * XU + b * YU, cc * XV + d * YV
    # strains (Sec. 4.3) of a linear field are its constant gradients
    z = np.zeros_like(u)
    sxx, syy, sx, sy = ops.strain(c, u, v, z, z, "geometric")
    for j in range(2, g.ny):
        for i in range(2, g.nx):
            assert abs(sxx[j, i] - a) < 1e-12 and abs(syy[j, i] - d) < 1e-12
            assert abs(sx[j, i] - 0.5 * (b + cc)) < 1e-12 and abs(sy[j, i] - 0.5 * (b + cc)) < 1e-12
    vx, vy = ops.viscous(c, u, v, z, z, "geometric")
    for j in range(3, g.ny - 1):
        for i in range(3, g.nx - 2):
            assert abs(vx[j, i]) < 1e-12 and abs(vy[j, i]) < 1e-12
    XP, YP = np.meshgrid(xc[:-1], yc[:-1])
    pr = derived.prepare(c, g.nx, g.ny)
    L = derived.laplacian(pr, np.where(pr.act_p, 0.3 * XP - 0.8 * YP, 0.0))
    assert np.max(np.abs(L[2:-2, 2:-2])) < 1e-13


def test_step_identities_with_a_body_on_a_stretched_mesh():
    g = _grid(24, 20)
    case = W.Case("stretched", g, [W.Body(W.CIRCLE, 0.6, 0.48, a=0.2)], re=100.0, noise=1e-2, seed=3, cfl=0.25)
    c = geometry.capacities(g, case.bodies)
    pr = derived.prepare(c, g.nx, g.ny)
    Dx, Dy = W.dirichlet(case)
    st = pmii.Stepper(pr, pmii.Params(rho=1.0, mu=case.mu, tau=case.tau, pcg_tol=1e-12, pred_tol=1e-13),
                      Dx, Dy, min(g.hx, g.hy))
    H, _ = assemble(st.apply_H, st.mask2)
    Hd = H.toarray()
    assert np.max(np.abs(Hd - Hd.T)) < 1e-12 * np.max(np.abs(Hd))
    assert np.linalg.eigvalsh(0.5 * (Hd + Hd.T)).min() > 0.0
    s = pmii.initial_state(pr, Dx, Dy, case.u_inf, W.perturbation(case))
    assert st.project(s).div_rel < 1e-9
    for _ in range(3):
        (usx, usy), _c = st.predict(s, pmii.StepInfo())
        b = st.poisson_rhs(usx, usy)
        phi = st.solve_poisson(b, s.Phi, pmii.StepInfo())
        ux, uy = st.correct(usx, usy, phi)
        d = ops.cont(c, ux, uy, Dx, Dy)
        resid = b - derived.laplacian(pr, phi)
        assert np.max(np.abs(d - (st.prm.tau / st.prm.rho) * resid)[pr.act_p]) < 1e-14
        info = st.step(s)
        assert info.div_rel < 1e-8 and info.pred_status == 0 and info.cg_status == 0


def _taylor_green_error_stretched(n, nu=0.05, T=0.5, cfl=0.25, amp=0.3):
    L = np.pi
    g = W.GridSpec(n, n, 0.0, 0.0, L, L, xf=W.stretched_edges(n, 0.0, L, amp),
                   yf=W.stretched_edges(n, 0.0, L, amp))
    caps = geometry.capacities(g, [])
    pr = derived.prepare(caps, n, n)
    xe, ye, xc, yc = g.edges(0), g.edges(1), g.centres(0), g.centres(1)
    XU, YU = np.meshgrid(xe[1:], yc[:-1])
    XV, YV = np.meshgrid(xc[:-1], ye[1:])
    XP, YP = np.meshgrid(xc[:-1], yc[:-1])

    def vel(t):
        F = np.exp(-2.0 * nu * t)
        return np.sin(XU) * np.cos(YU) * F, -np.cos(XV) * np.sin(YV) * F

    def pres(t):
        return 0.25 * (np.cos(2 * XP) + np.cos(2 * YP)) * np.exp(-4.0 * nu * t)

    h = min(g.hx, g.hy)
    tau = cfl * h
    steps = int(round(T / tau))
    tau = T / steps
    prm = pmii.Params(rho=1.0, mu=nu, tau=tau, pcg_tol=1e-12, pred_tol=1e-13)
    D0 = vel(0.0)
    st = pmii.Stepper(pr, prm, D0[0], D0[1], h)
    s = pmii.State(D0[0].copy(), D0[1].copy(), np.where(pr.act_p, pres(-0.5 * tau), 0.0), np.zeros_like(XP))
    st.project(s)
    for k in range(steps):
        st.step(s, D_next=vel((k + 1) * tau))
    ue, ve = vel(T)
    return max(np.max(np.abs(s.Ux - ue)[pr.act_u]), np.max(np.abs(s.Uy - ve)[pr.act_v]))


def test_taylor_green_second_order_on_a_stretched_mesh():
    e = [_taylor_green_error_stretched(n) for n in (16, 32, 64)]
    r1, r2 = e[0] / e[1], e[1] / e[2]
    assert e[2] < 3e-3, e
    assert r1 > 3.0 and r2 > 3.0, (e, r1, r2)
