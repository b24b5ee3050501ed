"""Pins of the oracle's outflow walls (homogeneous Neumann velocity, zero
pressure beyond the wall; end of Sec. 4.6), checked against what the
mathematics fixes:

  * the Poisson operator with an outflow face is the composition
    cont(M^-1 pres(Phi), 0) of eq:pm_poisson with the pressure beyond the
    wall at zero, and it is negative definite (no constant null space),
    while without outflow faces the constants are its null space;
  * a uniform stream through an empty channel is an exact steady solution
    (inflow on the west, outflow on the other walls);
  * with a body: every step is divergence-free, the net volume flux through
    the walls vanishes (what enters on the west leaves through the outflow
    walls), the outflow data of the next step are the zero-gradient
    extrapolation of the current velocity, and the non-singular pressure
    solve agrees with a direct sparse solve;
  * mirror symmetry: the same flow entering from the east (outflow on the
    west) or with the outflow on the south instead of the north, on the
    mirrored geometry and the mirrored initial state, is the mirror image of
    the original to rounding, which pins the index and sign of every wall's
    branch against the others."""

import numpy as np
import pytest

import workloads as W
from oracle import derived, geometry, operators as ops, pmii
from oracle.solvers import assemble


def _setup(case, theta=0.05, pcg_tol=1e-12, D=None):
    g = case.grid
    caps = geometry.capacities(g, case.bodies)
    pr = derived.prepare(caps, g.nx, g.ny, vol_floor=theta * g.hx * g.hy, outflow=case.outflow)
    Dx, Dy = W.dirichlet(case) if D is None else D
    prm = pmii.Params(rho=case.rho, mu=case.mu, tau=case.tau, u_inf=case.u_inf, pcg_tol=pcg_tol, pred_tol=1e-13)
    st = pmii.Stepper(pr, prm, Dx, Dy, min(g.hx, g.hy))
    return caps, pr, st, Dx, Dy


def _wall_flux(caps, g, Ux, Uy):
    """Net volume flux out of the box through its four walls."""
    nx, ny = g.nx, g.ny
    Ax, Ay = caps["Ax"], caps["Ay"]
    return ((Ax[1:-1, nx] * Ux[1:-1, nx]).sum() - (Ax[1:-1, 0] * Ux[1:-1, 0]).sum()
            + (Ay[ny, 1:-1] * Uy[ny, 1:-1]).sum() - (Ay[0, 1:-1] * Uy[0, 1:-1]).sum())


def test_poisson_operator_is_the_composition_and_definite():
    case = W.outflow_cylinder(12)
    caps, pr, st, Dx, Dy = _setup(case)
    assert not pr.singular and pr.out_u.sum() == case.grid.ny and pr.out_v.sum() == 2 * case.grid.nx
    rng = np.random.default_rng(21)
    phi = np.where(pr.act_p, rng.uniform(-1, 1, pr.act_p.shape), 0.0)
    # cont(M^-1 pres(Phi), 0) on the faces the projection corrects, with the
    # pressure beyond every wall at zero
    px, py = ops.pres(caps, phi)
    Mu, Mv = pr.Mu, pr.Mv
    qx = np.where(pr.proj_u & (Mu > 0), px / np.where(Mu > 0, Mu, 1.0), 0.0)
    qy = np.where(pr.proj_v & (Mv > 0), py / np.where(Mv > 0, Mv, 1.0), 0.0)
    z = np.zeros_like(phi)
    ref = np.where(pr.act_p, ops.cont(caps, qx, qy, z, z), 0.0)
    L = derived.laplacian(pr, phi)
    assert np.max(np.abs(L - ref)) < 1e-13 * np.max(np.abs(ref))
    A, idx = assemble(st.apply_A, pr.act_p)
    ev = np.linalg.eigvalsh(A.toarray())
    assert ev.min() > 1e-6 * ev.max()
    # the same geometry without outflow walls: the constants span the null space
    pr0 = derived.prepare(caps, case.grid.nx, case.grid.ny, vol_floor=0.05 * case.grid.hx * case.grid.hy)
    assert pr0.singular
    one = np.where(pr0.act_p, 1.0, 0.0)
    assert np.max(np.abs(derived.laplacian(pr0, one))) < 1e-14 * np.max(pr0.diag)
    assert np.max(np.abs(derived.laplacian(pr, one))) > 0.1 * np.min(pr.diag[pr.act_p])


@pytest.mark.parametrize("outflow", ["E", "ESN"])
def test_uniform_stream_is_steady(outflow):
    g = W.GridSpec(24, 12, 0.0, 0.0, 2.0, 1.0)
    case = W.Case("empty_channel", g, [], re=100.0, cfl=0.25, noise=0.0, outflow=outflow)
    caps, pr, st, Dx, Dy = _setup(case)
    s = pmii.initial_state(pr, Dx, Dy, case.u_inf)
    assert st.project(s).div_rel < 1e-13
    for _ in range(4):
        st.step(s)
    ux = np.where(pr.proj_u, s.Ux - case.u_inf, 0.0)
    uy = np.where(pr.proj_v, s.Uy, 0.0)
    assert np.max(np.abs(ux)) < 1e-13 and np.max(np.abs(uy)) < 1e-13
    assert np.max(np.abs(s.P)) < 1e-10 and np.max(np.abs(s.Phi)) < 1e-10


def test_step_with_a_body_conserves_volume():
    case = W.outflow_cylinder(24)
    g = case.grid
    caps, pr, st, Dx, Dy = _setup(case)
    s = pmii.initial_state(pr, Dx, Dy, case.u_inf, W.perturbation(case))
    st.project(s)
    inflow = (caps["Ax"][1:-1, 0] * Dx[1:-1, 0]).sum()
    for n in range(4):
        Dn = st.outflow_data(s.Ux, s.Uy)
        # zero normal gradient on the outflow faces, tangential ghosts likewise
        assert np.array_equal(Dn[0][1:-1, g.nx][pr.out_u[1:-1, g.nx]], s.Ux[1:-1, g.nx - 1][pr.out_u[1:-1, g.nx]])
        assert np.array_equal(Dn[1][g.ny, 1:-1][pr.out_v[g.ny, 1:-1]], s.Uy[g.ny - 1, 1:-1][pr.out_v[g.ny, 1:-1]])
        assert np.array_equal(Dn[1][0, 1:-1][pr.out_v[0, 1:-1]], s.Uy[1, 1:-1][pr.out_v[0, 1:-1]])
        assert np.array_equal(Dn[1][1:g.ny, g.nx + 1], s.Uy[1:g.ny, g.nx])
        assert np.array_equal(Dn[0][g.ny + 1, 1:g.nx], s.Ux[g.ny, 1:g.nx])
        # the west wall keeps its Dirichlet data
        assert np.array_equal(Dn[0][:, 0], Dx[:, 0])
        (usx, usy), _c = st.predict(s, pmii.StepInfo(), D_next=Dn)
        b = st.poisson_rhs(usx, usy)
        assert abs(b[pr.act_p].sum()) > 1e-8 * np.abs(b).max()    # no mean removed: not needed
        phi = st.solve_poisson(b, s.Phi, pmii.StepInfo())
        ux, uy = st.correct(usx, usy, phi)
        d = ops.cont(caps, ux, uy, st.Dx, st.Dy)
        resid = b - derived.laplacian(pr, phi)
        assert np.max(np.abs(d - (st.prm.tau / st.prm.rho) * resid)[pr.act_p]) < 1e-13
        if n == 0:
            phx = st.solve_poisson(b, s.Phi, pmii.StepInfo(), solver="direct")
            assert np.max(np.abs(phi - phx)) < 1e-9 * np.max(np.abs(phx))
        st.Dx, st.Dy = Dx, Dy       # back to D^n: the step below redoes this one
        st.vD = st.dirichlet_viscous(Dx, Dy)
        info = st.step(s)
        assert info.div_rel < 1e-10 and info.cg_status == 0 and info.pred_status == 0
        assert abs(_wall_flux(caps, g, s.Ux, s.Uy)) < 1e-11 * inflow
        assert np.array_equal(st.Dx, Dn[0]) and np.array_equal(st.Dy, Dn[1])
        Dx, Dy = st.Dx, st.Dy
    # the outflow faces carry the projected flux, not their Dirichlet data
    assert np.max(np.abs(s.Ux[1:-1, g.nx] - st.Dx[1:-1, g.nx])) > 1e-8


def _mirror_x(a, nx, face):
    """Mirror image in x: x-faces i -> nx - i (0..nx), cells i -> nx + 1 - i."""
    b = np.zeros_like(a)
    if face:
        b[:, 0:nx + 1] = a[:, nx::-1]
    else:
        b[:, :] = a[:, ::-1]
    return b


def _mirror_y(a, ny, face):
    b = np.zeros_like(a)
    if face:
        b[0:ny + 1, :] = a[ny::-1, :]
    else:
        b[:, :] = a[::-1, :]
    return b


@pytest.mark.parametrize("axis", ["x", "y"])
def test_mirror_images(axis):
    g = W.GridSpec(32, 16, 0.0, 0.0, 4.0, 2.0)
    if axis == "x":
        a = W.Case("a", g, [W.Body(W.CIRCLE, 1.2, 1.1, a=0.25)], re=100.0, cfl=0.25, noise=1e-2, seed=3,
                   outflow="ESN")
        b = W.Case("b", g, [W.Body(W.CIRCLE, 4.0 - 1.2, 1.1, a=0.25)], re=100.0, cfl=0.25, outflow="WSN")
        mu_, mv_ = (lambda f: -_mirror_x(f, g.nx, True)), (lambda f: _mirror_x(f, g.nx, False))
        mp = lambda f: _mirror_x(f, g.nx, False)       # noqa: E731
    else:
        a = W.Case("a", g, [W.Body(W.CIRCLE, 1.2, 1.2, a=0.25)], re=100.0, cfl=0.25, noise=1e-2, seed=3,
                   outflow="EN")
        b = W.Case("b", g, [W.Body(W.CIRCLE, 1.2, 2.0 - 1.2, a=0.25)], re=100.0, cfl=0.25, outflow="ES")
        mu_, mv_ = (lambda f: _mirror_y(f, g.ny, False)), (lambda f: -_mirror_y(f, g.ny, True))
        mp = lambda f: _mirror_y(f, g.ny, False)       # noqa: E731
    capsA, prA, stA, DxA, DyA = _setup(a)
    DxB, DyB = mu_(DxA), mv_(DyA)
    capsB, prB, stB, _, _ = _setup(b, D=(DxB, DyB))
    assert np.array_equal(mp(prA.act_p), prB.act_p)
    sA = pmii.initial_state(prA, DxA, DyA, a.u_inf, W.perturbation(a))
    sB = pmii.State(mu_(sA.Ux), mv_(sA.Uy), np.zeros_like(sA.P), np.zeros_like(sA.P))
    stA.project(sA)
    stB.project(sB)
    for _ in range(3):
        stA.step(sA)
        stB.step(sB)
    sc = np.max(np.abs(sA.Ux))
    if axis == "x":
        cmp_u = (mu_(sA.Ux) - sB.Ux)[:, 0:g.nx + 1]
        cmp_v = (mv_(sA.Uy) - sB.Uy)[:, 1:g.nx + 1]
    else:
        cmp_u = (mu_(sA.Ux) - sB.Ux)[1:g.ny + 1, :]
        cmp_v = (mv_(sA.Uy) - sB.Uy)[0:g.ny + 1, :]
    assert np.max(np.abs(cmp_u)) < 1e-9 * sc and np.max(np.abs(cmp_v)) < 1e-9 * sc
    pa, pb = np.where(prB.act_p, mp(sA.P), 0.0), np.where(prB.act_p, sB.P, 0.0)
    assert np.max(np.abs(pa - pb)) < 1e-8 * np.max(np.abs(pa))
