"""Pins of the oracle's force on the bodies (oracle.forces, a reading for the
drag and lift coefficients of Sec. 5), against what the mathematics fixes:

  * a uniform pressure and a fluid at rest exert no force (the projections
    of a closed surface cancel);
  * summation by parts: for fields whose pressure and strain vanish near the
    box's walls, the force is exactly minus the momentum that the discrete
    pres and visc operators put into the fluid, summed over the faces (the
    reading is the discrete momentum exchange of eq:semidiscrete);
  * Archimedes: a pressure rising linearly with height pushes a disc up by
    the gradient times its area, to first order in h (the cell pressure
    stands for the pressure on the cell's piece of the surface);
  * mirror symmetry: the mirrored flow has the same drag and the opposite
    lift, to rounding;
  * the flow past the paper's cylinder set-up drags the body downstream."""

import math

import numpy as np
import pytest

import workloads as W
from oracle import derived, forces, geometry, operators as ops, pmii


def _disc_case(n, cy=0.487):
    g = W.GridSpec(n, n, 0.0, 0.0, 1.0, 1.0)
    return g, geometry.capacities(g, [W.Body(W.CIRCLE, 0.503, cy, a=0.2)])


def test_uniform_pressure_and_rest():
    g, c = _disc_case(48)
    pr = derived.prepare(c, g.nx, g.ny)
    z = np.zeros_like(c["V"])
    F = forces.forces(c, np.where(pr.act_p, 3.7, 0.0), z, z, z, z, mu=0.1)
    assert max(abs(f) for f in F) < 1e-14
    # a flow that differs from the data only next to the walls (where the
    # walls' shear acts) exerts no force on the body
    case = W.Case("disc", g, [W.Body(W.CIRCLE, 0.503, 0.487, a=0.2)], re=100.0)
    Dx, Dy = W.dirichlet(case)
    J, I = np.indices(z.shape)
    edge = (I <= 2) | (I >= g.nx - 1) | (J <= 2) | (J >= g.ny - 1)
    rng = np.random.default_rng(40)
    Ux = np.where(pr.act_u & edge, Dx + rng.uniform(-1, 1, z.shape), Dx)
    Uy = np.where(pr.act_v & edge, Dy + rng.uniform(-1, 1, z.shape), Dy)
    assert np.abs(ops.strain(c, Ux, Uy, Dx, Dy)[2]).max() > 0.1
    F = forces.forces(c, z, Ux, Uy, Dx, Dy, mu=0.1)
    assert max(abs(f) for f in F) == 0.0


def test_summation_by_parts():
    g, c = _disc_case(48)
    case = W.Case("disc", g, [W.Body(W.CIRCLE, 0.503, 0.487, a=0.2)], re=100.0)
    pr = derived.prepare(c, g.nx, g.ny)
    Dx, Dy = W.dirichlet(case)
    rng = np.random.default_rng(41)
    sh = c["V"].shape
    J, I = np.indices(sh)
    inner = (I >= 4) & (I <= g.nx - 3) & (J >= 4) & (J <= g.ny - 3)
    P = np.where(pr.act_p & inner, rng.uniform(-1, 1, sh), 0.0)
    px, py = ops.pres(c, P)
    F = forces.forces(c, P, Dx, Dy, Dx, Dy, mu=0.0)
    # the fluid receives -pres(P): the bodies +pres(P)
    assert abs(F[0] - px.sum()) < 1e-13 and abs(F[1] - py.sum()) < 1e-13
    assert abs(F[0]) > 1e-3 and abs(F[1]) > 1e-3
    # velocity: the Dirichlet data plus a perturbation of the unknowns away
    # from the walls (the strain vanishes where U = D is uniform)
    Ux = np.where(pr.act_u & inner, Dx + rng.uniform(-1, 1, sh), Dx)
    Uy = np.where(pr.act_v & inner, Dy + rng.uniform(-1, 1, sh), Dy)
    mu = 0.3
    vx, vy = ops.viscous(c, Ux, Uy, Dx, Dy, "geometric")
    F = forces.forces(c, np.zeros(sh), Ux, Uy, Dx, Dy, mu=mu)
    # the fluid receives +2 mu visc(S): the bodies -2 mu visc(S)
    assert abs(F[2] + 2 * mu * vx.sum()) < 1e-12 * (1 + abs(F[2]))
    assert abs(F[3] + 2 * mu * vy.sum()) < 1e-12 * (1 + abs(F[3]))
    assert abs(F[2]) > 1e-2 and abs(F[3]) > 1e-2


def test_archimedes_first_order():
    errs = []
    for n in (32, 64, 128):
        g, c = _disc_case(n)
        P = np.where(c["V"] > 0, 2.0 * c["Y"], 0.0)
        z = np.zeros_like(P)
        F = forces.forces(c, P, z, z, z, z, mu=0.0)
        errs.append(F[1] + 2.0 * math.pi * 0.2 ** 2)
        assert abs(F[0]) < 5e-3 / n
    for n, e in zip((32, 64, 128), errs):
        assert abs(e) < 0.4 / n, errs
    assert abs(errs[2]) < 0.7 * abs(errs[0]) and abs(errs[1]) < 0.7 * abs(errs[0]), errs


def _flow(case, steps=3):
    g = case.grid
    c = geometry.capacities(g, case.bodies)
    pr = derived.prepare(c, g.nx, g.ny, vol_floor=0.05 * g.hx * g.hy, outflow=case.outflow)
    Dx, Dy = W.dirichlet(case)
    prm = pmii.Params(rho=case.rho, mu=case.mu, tau=case.tau, u_inf=case.u_inf, pcg_tol=1e-12, pred_tol=1e-13)
    st = pmii.Stepper(pr, prm, Dx, Dy, min(g.hx, g.hy))
    return c, pr, st, Dx, Dy


def test_mirror_symmetry():
    g = W.GridSpec(48, 24, 0.0, 0.0, 4.0, 2.0)
    a = W.Case("a", g, [W.Body(W.CIRCLE, 1.2, 1.13, a=0.25)], re=100.0, cfl=0.25, noise=1e-2, seed=5)
    b = W.Case("b", g, [W.Body(W.CIRCLE, 1.2, 2.0 - 1.13, a=0.25)], re=100.0, cfl=0.25)
    cA, prA, stA, DxA, DyA = _flow(a)
    my = lambda f, face: (np.concatenate([f[g.ny::-1], f[g.ny + 1:]]) if face else f[::-1])  # noqa: E731
    cB = geometry.capacities(g, b.bodies)
    DxB, DyB = my(DxA, False), -my(DyA, True)
    prB = derived.prepare(cB, g.nx, g.ny, vol_floor=0.05 * g.hx * g.hy)
    stB = pmii.Stepper(prB, stA.prm, DxB, DyB, stA.h)
    sA = pmii.initial_state(prA, DxA, DyA, a.u_inf, W.perturbation(a))
    sB = pmii.State(my(sA.Ux, False), -my(sA.Uy, True), np.zeros_like(sA.P), np.zeros_like(sA.P))
    stA.project(sA)
    stB.project(sB)
    for _ in range(3):
        stA.step(sA)
        stB.step(sB)
    FA = forces.forces(cA, sA.P, sA.Ux, sA.Uy, stA.Dx, stA.Dy, a.mu, pmask=prA.act_p)
    FB = forces.forces(cB, sB.P, sB.Ux, sB.Uy, stB.Dx, stB.Dy, b.mu, pmask=prB.act_p)
    sc = max(abs(f) for f in FA)
    assert abs(FA[0] - FB[0]) < 1e-9 * sc and abs(FA[2] - FB[2]) < 1e-9 * sc
    assert abs(FA[1] + FB[1]) < 1e-9 * sc and abs(FA[3] + FB[3]) < 1e-9 * sc


@pytest.mark.parametrize("outflow", ["", "ESN"])
def test_drag_points_downstream(outflow):
    case = W.outflow_cylinder(24, outflow=outflow)
    c, pr, st, Dx, Dy = _flow(case)
    s = pmii.initial_state(pr, Dx, Dy, case.u_inf, W.perturbation(case))
    st.project(s)
    for _ in range(5):
        st.step(s)
    F = forces.forces(c, s.P, s.Ux, s.Uy, st.Dx, st.Dy, case.mu, pmask=pr.act_p)
    cd, cl = forces.coefficients(F, case.rho, case.u_inf, case.ref_length)
    assert F[0] > 0 and F[2] > 0 and 0.5 < cd < 50.0, (F, cd)
    assert abs(cl) < 0.5 * cd
