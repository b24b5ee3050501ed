"""Precision 1: FP32 inner solves with FP64 residuals and FP64 refinement.

The bar (the FP64 oracle is the reference): velocities within 1e-6 relative
of the oracle's FP64 trajectory, and every step's max |cont(U, D)| / (U h)
at most 1e-8, as checked by the oracle's own diagnostics on the device's
state.  The pressure solve alone, run to a 2-norm tolerance, must satisfy the
oracle's residual test exactly as the FP64 solve does."""

import numpy as np
import pytest

import workloads as W
from oracle import derived, pmii
from tests.gpu_common import case_setup, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CASES = {
    "cylinder_64": lambda: W.cylinder_64(),
    "channel_130x73": lambda: W.scaled_cylinder(130, 73, 2.6, 1.46, seed=5),
    "flat_top_64": lambda: W.flat_top_cylinder(64),
}
# small-volume floor: 0 is the paper's mass matrix, 0.05 the floored reading
THETAS = (0.0, 0.05)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _host(t):
    return t.cpu().numpy()


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("precond", ["jacobi", "mg"])
def test_mixed_pressure_solve_meets_fp64_residual(name, precond):
    case = CASES[name]()
    # 2-norm criterion (div_tol 0): |b - L phi| <= tol |b| in FP64
    caps, pr, st, ctx, Dx, Dy = case_setup(case, pcg_tol=1e-10, precond=precond, precision=1, div_tol=0.0)
    rng = np.random.default_rng(3)
    b = np.where(pr.act_p, rng.uniform(-1, 1, pr.act_p.shape), 0.0)
    phi_d, info, status = ctx.pressure_solve(_dev(b))
    assert status == 0 and info.outer >= 2
    bm = b - np.where(pr.act_p, b[pr.act_p].mean(), 0.0)
    pd = _host(phi_d)
    res = bm - derived.laplacian(pr, pd)
    assert np.linalg.norm(res[pr.act_p]) <= 1.01 * 1e-10 * np.linalg.norm(bm[pr.act_p])
    assert info.rel_residual <= 1e-10
    phi_o = st.solve_poisson(bm, np.zeros_like(b), pmii.StepInfo(), solver="direct") if pr.n_active < 6000 else None
    if phi_o is not None:
        pz = np.where(pr.act_p, pd - pd[pr.act_p].mean(), 0.0)
        assert rel(pz, phi_o, pr.act_p) < 1e-6


@pytest.mark.parametrize("theta", THETAS)
@pytest.mark.parametrize("name", sorted(CASES))
def test_mixed_trajectory_against_fp64_oracle(name, theta):
    from paper_2211_10698_amd import ccns
    case = CASES[name]()
    # oracle: FP64 with tight tolerances; device: precision 1 at its defaults
    caps, pr, st, ctx, Dx, Dy = case_setup(case, pcg_tol=1e-13, pred_tol=1e-14, precision=1, div_tol=1e-8,
                                           mass_floor=theta)
    ctx.close()
    cp = ccns.make_params(case.rho, case.mu, case.tau, u_ref=case.u_inf, pcg_tol=1e-10, pred_tol=1e-10,
                          div_tol=1e-8, precision=1, mass_floor=theta)
    ctx = ccns.Context(case.grid, cp, np.stack([caps[k] for k in ccns.CAP_NAMES]), Dx, Dy)
    s0 = pmii.initial_state(pr, Dx, Dy, case.u_inf, W.perturbation(case))
    ctx.set_field(ccns.F_UX, s0.Ux)
    ctx.set_field(ccns.F_UY, s0.Uy)
    st.project(s0)
    info = ctx.project()
    assert info.div_rel <= 1e-8
    for n in range(case.steps):
        st.step(s0)
        di = ctx.step(1)
        assert di.div_rel <= 1e-8, n
        assert di.poisson.outer >= 1 and di.pred.outer >= 1
        ux, uy = _host(ctx.get_field(ccns.F_UX)), _host(ctx.get_field(ccns.F_UY))
        od = st.diagnostics(ux, uy, pmii.StepInfo())
        assert od.div_rel <= 1e-8, n
    assert rel(ux, s0.Ux) < 1e-6
    assert rel(uy, s0.Uy) < 1e-6


def test_mixed_step_full_size_properties():
    """One precision-1 step at the full 2048x1024 size: the FP64 predictor
    residual and the divergence, measured by the oracle on the device's
    state."""
    from paper_2211_10698_amd import ccns
    case = W.channel_cylinder_2048()
    print(f"[mixed] set-up {case.name}", flush=True)
    caps, pr, st, ctx, Dx, Dy = case_setup(case, pred_tol=1e-12, precision=1, div_tol=1e-8)
    s0 = pmii.initial_state(pr, Dx, Dy, case.u_inf, W.perturbation(case))
    ctx.set_field(ccns.F_UX, s0.Ux)
    ctx.set_field(ccns.F_UY, s0.Uy)
    assert ctx.project().div_rel <= 1e-8
    Un = (_host(ctx.get_field(ccns.F_UX)), _host(ctx.get_field(ccns.F_UY)))
    Pn = _host(ctx.get_field(ccns.F_P))
    sn = pmii.State(Un[0].copy(), Un[1].copy(), Pn.copy(), np.zeros_like(Pn))
    pinfo = ctx.predict()
    assert pinfo.status == 0
    conv_n = st.convection(*Un)
    rhs = st.predictor_rhs(sn, conv_n, conv_n)
    Us = (_host(ctx.get_field(ccns.F_USX)), _host(ctx.get_field(ccns.F_USY)))
    U2 = np.stack([np.where(pr.act_u, Us[0], 0.0), np.where(pr.act_v, Us[1], 0.0)])
    res = np.where(st.mask2, rhs - st.apply_H(U2), 0.0)
    assert np.linalg.norm(res) <= 2 * 1e-12 * np.linalg.norm(rhs)
    info = ctx.correct()
    assert info.poisson.status == 0 and info.div_rel <= 1e-8
    ux, uy = _host(ctx.get_field(ccns.F_UX)), _host(ctx.get_field(ccns.F_UY))
    od = st.diagnostics(ux, uy, pmii.StepInfo())
    assert od.div_rel <= 1e-8
