"""Pins of the oracle's small-volume floor.

The paper's mass matrix is M = diag(V) (eq:semidiscrete, Sec. 4.5).  With
theta > 0 every volume the step divides by is at least theta hx hy: the mass
matrix of the velocity unknowns, M_f = max(V_f, theta hx hy), in the
predictor and in the projection's M^-1, and the cell volume of the pressure
update.  That is a departure from M = diag(V) wherever a cut volume is below
theta hx hy, so the floored branch is pinned here by properties that a floor
applied in the wrong place, or in a different way in two places, breaks:

  * above the floor nothing changes: with every volume the step divides by
    above theta hx hy, the prepared arrays and three steps are identical bit
    for bit to theta = 0 (a floor added instead of taken as a maximum, or
    applied to every face, fails this);
  * the Poisson operator stays symmetric with the constants as its null space
    (a floor applied to one side of a face only breaks the symmetry);
  * the divergence identity cont(U^{n+1}, D) = (tau/rho)(b - L Phi) holds to
    round-off (the Poisson weights and the corrector must use the same M);
  * the projection is orthogonal in the mass matrix the predictor uses:
    M (U^{n+1} - U*) is a discrete gradient, -(tau/rho) A dPhi (a corrector
    that divides by V while the predictor uses M fails it);
  * the predictor matrix H = (rho/tau) M - mu K is symmetric positive definite
    and its Jacobi diagonal is its assembled diagonal;
  * the pressure update leaves the volume-weighted mean alone:
    sum V_p (P^+ - P - Phi) = 0, V_p the update's (floored) cell volume;
  * in a closed no-slip box the kinetic energy of the mass matrix the step
    uses, U^T M U / 2, decreases every step.

Each test first asserts that the geometry has velocity unknowns (and cells)
whose volume is below the floor, so the floored branch is exercised."""

import numpy as np
import pytest

import workloads as W
from oracle import derived, geometry, operators as ops, pmii
from oracle.solvers import assemble

THETA = 0.05


def _stepper(case, theta, pcg_tol=1e-12, D=None):
    g = case.grid
    caps = geometry.capacities(g, case.bodies)
    pr = derived.prepare(caps, g.nx, g.ny, vol_floor=theta * g.hx * g.hy)
    Dx, Dy = W.dirichlet(case) if D is None else D
    prm = pmii.Params(rho=case.rho, mu=case.mu, tau=case.tau, pcg_tol=pcg_tol, pred_tol=1e-13)
    return caps, pr, pmii.Stepper(pr, prm, Dx, Dy, min(g.hx, g.hy)), Dx, Dy


def _below(caps, pr, g, theta):
    f = theta * g.hx * g.hy
    nu = int(np.sum(pr.act_u & (caps["Vu"] < f)))
    nv = int(np.sum(pr.act_v & (caps["Vv"] < f)))
    ncell = int(np.sum(pr.act_p & (caps["V"] < f)))
    return nu + nv, ncell


def test_floor_changes_nothing_above_it():
    """cylinder_64: every velocity volume and every cell volume is above
    0.05 hx hy, so theta = 0.05 and theta = 0 give the same arrays and the
    same three steps, bit for bit."""
    case = W.cylinder_64()
    g = case.grid
    caps, pr0, st0, Dx, Dy = _stepper(case, 0.0)
    _, pr1, st1, _, _ = _stepper(case, THETA)
    f = THETA * g.hx * g.hy
    assert caps["Vu"][pr0.act_u].min() > f and caps["Vv"][pr0.act_v].min() > f
    assert caps["V"][caps["V"] > 0].min() > f
    for name in ("cx", "cy", "gx", "gy", "diag", "Mu", "Mv", "Vp"):
        assert np.array_equal(getattr(pr0, name), getattr(pr1, name)), name
    s0 = pmii.initial_state(pr0, Dx, Dy, case.u_inf, W.perturbation(case))
    s1 = pmii.initial_state(pr1, Dx, Dy, case.u_inf, W.perturbation(case))
    st0.project(s0)
    st1.project(s1)
    for _ in range(3):
        st0.step(s0)
        st1.step(s1)
    for a, b in ((s0.Ux, s1.Ux), (s0.Uy, s1.Uy), (s0.P, s1.P), (s0.Phi, s1.Phi)):
        assert np.array_equal(a, b)


@pytest.fixture(scope="module")
def flat():
    case = W.flat_top_cylinder(24)
    caps, pr, st, Dx, Dy = _stepper(case, THETA)
    nfaces, ncells = _below(caps, pr, case.grid, THETA)
    assert nfaces >= 1 and ncells >= 1, (nfaces, ncells)
    return case, caps, pr, st, Dx, Dy


def test_floored_poisson_operator_symmetric_with_constant_null_space(flat):
    case, caps, pr, st, Dx, Dy = flat
    ones = np.where(pr.act_p, 1.0, 0.0)
    assert np.max(np.abs(derived.laplacian(pr, ones))) < 1e-13
    A, _ = assemble(st.apply_A, pr.act_p)
    assert np.max(np.abs((A - A.T).toarray())) == 0.0


def test_floored_step_divergence_identity_projection_and_pressure_mean(flat):
    case, caps, pr, st, Dx, Dy = flat
    s = pmii.initial_state(pr, Dx, Dy, case.u_inf, W.perturbation(case))
    assert st.project(s).div_rel < 1e-8
    sc = st.prm.tau / st.prm.rho
    f = THETA * case.grid.hx * case.grid.hy
    for _ in range(3):
        (usx, usy), _c = st.predict(s, pmii.StepInfo())
        b = st.poisson_rhs(usx, usy)
        phi = st.solve_poisson(b, s.Phi, pmii.StepInfo())
        ux, uy = st.correct(usx, usy, phi)
        # divergence identity (the Poisson weights and the corrector agree)
        d = ops.cont(caps, ux, uy, Dx, Dy)
        resid = b - derived.laplacian(pr, phi)
        assert np.max(np.abs(d - sc * resid)[pr.act_p]) < 1e-14 * max(1.0, np.max(np.abs(b)))
        # the correction is a gradient in the predictor's mass matrix, also on
        # the faces whose volume is floored
        gxp, gyp = ops.pres(caps, phi)
        ex = np.where(pr.act_u, st.Vu * (ux - usx) + sc * gxp, 0.0)
        ey = np.where(pr.act_v, st.Vv * (uy - usy) + sc * gyp, 0.0)
        scale = sc * max(np.max(np.abs(gxp)), np.max(np.abs(gyp)))
        assert max(np.max(np.abs(ex)), np.max(np.abs(ey))) < 1e-13 * scale
        floored = pr.act_u & (caps["Vu"] < f)
        assert np.any(floored & (np.abs(ux - usx) > 0.0))
        # the pressure update keeps the mean weighted by its own volumes
        P1 = st.pressure_update(s.P, phi)
        m = np.sum((pr.Vp * (P1 - s.P - phi))[pr.act_p])
        assert abs(m) < 1e-12 * np.sum(np.abs(pr.Vp * phi)[pr.act_p])
        info = st.step(s)
        assert info.div_rel < 1e-8 and info.cg_status == 0 and info.pred_status == 0


def test_floored_predictor_matrix_spd(flat):
    case, caps, pr, st, Dx, Dy = flat
    H, _ = assemble(st.apply_H, st.mask2)
    Hd = H.toarray()
    assert np.max(np.abs(Hd - Hd.T)) < 1e-12 * np.max(np.abs(Hd))
    assert np.linalg.eigvalsh(0.5 * (Hd + Hd.T)).min() > 0.0
    assert np.allclose(np.diag(Hd), st.Hdiag[st.mask2], rtol=1e-14)


def test_floored_energy_decays_in_closed_box():
    """No-slip box (D = 0) around the flat-topped circle, divergence-free
    start: U^T M U / 2 in the step's own (floored) mass matrix decreases."""
    case = W.flat_top_cylinder(24)
    g = case.grid
    z = np.zeros((g.ny + 2, g.nx + 2))
    caps, pr, st, _, _ = _stepper(case, THETA, D=(z, z))
    assert _below(caps, pr, g, THETA)[0] >= 1
    noisy = W.Case("box", g, case.bodies, re=case.re, noise=1.0, seed=7, cfl=case.cfl)
    px, py = W.perturbation(noisy)
    s = pmii.State(np.where(pr.act_u, px, 0.0), np.where(pr.act_v, py, 0.0), z.copy(), z.copy())
    st.project(s)

    def energy():
        return 0.5 * float(np.sum(st.Vu * s.Ux ** 2) + np.sum(st.Vv * s.Uy ** 2))

    e = [energy()]
    for _ in range(5):
        st.step(s)
        e.append(energy())
    assert all(b < a for a, b in zip(e[:-1], e[1:])), e
