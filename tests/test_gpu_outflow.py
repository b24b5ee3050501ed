"""Outflow walls on the device (homogeneous Neumann velocity, zero pressure
beyond the wall; end of Sec. 4.6) against the oracle, on the paper's cylinder
set-up (inflow on the west, outflow on the other three walls):

  * precision 1: ten steps within 1e-6 of the oracle's FP64 trajectory, each
    step's divergence (measured by the oracle on the device's state) below
    1e-8;
  * the predicted velocity of every outflow face, and beyond the outflow
    walls, is the interior neighbour's (zero normal gradient), and the net
    volume flux through the walls of the device's state vanishes;
  * a body that cuts the cells next to an outflow wall is refused (the
    wall's data would no longer cancel out of the operators).
The phase-by-phase and FP64 trajectory parity of the same case (both
preconditioners, both mass floors) is in the parity tests."""

import numpy as np
import pytest

import workloads as W
from oracle import pmii
from tests.gpu_common import case_setup, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _host(t):
    return t.cpu().numpy()


def _wall_flux(caps, g, Ux, Uy):
    nx, ny = g.nx, g.ny
    Ax, Ay = caps["Ax"], caps["Ay"]
    return ((Ax[1:-1, nx] * Ux[1:-1, nx]).sum() - (Ax[1:-1, 0] * Ux[1:-1, 0]).sum()
            + (Ay[ny, 1:-1] * Uy[ny, 1:-1]).sum() - (Ay[0, 1:-1] * Uy[0, 1:-1]).sum())


@pytest.mark.parametrize("theta", [0.0, 0.05])
def test_mixed_trajectory(theta):
    from paper_2211_10698_amd import ccns
    case = W.outflow_cylinder(48)
    caps, pr, st, ctx, Dx, Dy = case_setup(case, pcg_tol=1e-13, pred_tol=1e-14, precision=1, mass_floor=theta)
    ctx.close()
    # the device's tolerances of precision 1 (the oracle stays at 1e-13)
    caps, _, _, ctx, _, _ = case_setup(case, pcg_tol=1e-10, pred_tol=1e-10, precision=1, mass_floor=theta)
    s0 = pmii.initial_state(pr, Dx, Dy, case.u_inf, W.perturbation(case))
    ctx.set_field(ccns.F_UX, s0.Ux)
    ctx.set_field(ccns.F_UY, s0.Uy)
    st.project(s0)
    assert ctx.project().div_rel <= 1e-8
    for n in range(case.steps):
        st.step(s0)
        di = ctx.step(1, check=False)
        assert di.pred.status == 0 and di.poisson.status == 0, (n, di.as_dict())
        assert di.div_rel <= 1e-8, n
        ux, uy = _host(ctx.get_field(ccns.F_UX)), _host(ctx.get_field(ccns.F_UY))
        st_check = pmii.Stepper(pr, st.prm, st.Dx, st.Dy, st.h, jacobi=False)
        assert st_check.diagnostics(ux, uy, pmii.StepInfo()).div_rel <= 1e-8, n
    assert rel(ux, s0.Ux) < 1e-6 and rel(uy, s0.Uy) < 1e-6
    ctx.close()


def test_outflow_values_and_volume_budget():
    from paper_2211_10698_amd import ccns
    case = W.outflow_cylinder(48)
    g = case.grid
    caps, pr, st, ctx, Dx, Dy = case_setup(case, pcg_tol=1e-12, pred_tol=1e-13)
    s0 = pmii.initial_state(pr, Dx, Dy, case.u_inf, W.perturbation(case))
    ctx.set_field(ccns.F_UX, s0.Ux)
    ctx.set_field(ccns.F_UY, s0.Uy)
    ctx.project()
    inflow = (caps["Ax"][1:-1, 0] * Dx[1:-1, 0]).sum()
    for n in range(3):
        ux, uy = _host(ctx.get_field(ccns.F_UX)), _host(ctx.get_field(ccns.F_UY))
        assert abs(_wall_flux(caps, g, ux, uy)) < 1e-11 * inflow, n
        ctx.predict()
        usx, usy = _host(ctx.get_field(ccns.F_USX)), _host(ctx.get_field(ccns.F_USY))
        ou, ov = pr.out_u, pr.out_v
        assert np.array_equal(usx[:, g.nx][ou[:, g.nx]], ux[:, g.nx - 1][ou[:, g.nx]])
        assert np.array_equal(usy[g.ny, :][ov[g.ny, :]], uy[g.ny - 1, :][ov[g.ny, :]])
        assert np.array_equal(usy[0, :][ov[0, :]], uy[1, :][ov[0, :]])
        assert np.array_equal(usy[1:g.ny, g.nx + 1], uy[1:g.ny, g.nx])
        assert np.array_equal(usx[g.ny + 1, 1:g.nx], ux[g.ny, 1:g.nx])
        assert np.array_equal(usx[0, 1:g.nx], ux[1, 1:g.nx])
        info = ctx.correct()
        assert info.div_rel < 1e-9 and info.poisson.status == 0
    ux = _host(ctx.get_field(ccns.F_UX))
    # the outflow faces carry the projected flux
    assert np.max(np.abs(ux[1:-1, g.nx] - Dx[1:-1, g.nx])) > 1e-6
    ctx.close()


def test_rejects_a_body_at_an_outflow_wall():
    from paper_2211_10698_amd import ccns
    g = W.GridSpec(48, 24, 0.0, 0.0, 4.0, 2.0)
    case = W.Case("touching", g, [W.Body(W.CIRCLE, 3.9, 1.0, a=0.25)], re=100.0, cfl=0.25, outflow="E")
    with pytest.raises(ccns.CcnsError):
        case_setup(case, pcg_tol=1e-10)
    # the same body is accepted when that wall holds Dirichlet data
    case = W.Case("touching", g, [W.Body(W.CIRCLE, 3.9, 1.0, a=0.25)], re=100.0, cfl=0.25, outflow="N")
    case_setup(case, pcg_tol=1e-10)[3].close()
