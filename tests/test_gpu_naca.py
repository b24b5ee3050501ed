"""The 4096x2048 NACA0012 workload (chord 1 at 5 degrees, Re 1000).

The oracle's generic-level-set quadrature is pure Python and would take
hours at this size, so both sides use the library's capacities here (the
two capacity back-ends are compared against each other at small sizes in
the CPU tests).  Checked at full size:
  * every operator apply, element by element against the oracle;
  * FP64 and precision-1 runs side by side for 100 steps: every step below
    1e-8 divergence, and the precision-1 velocity within 1e-6 (relative to
    the largest velocity) of the FP64 run at steps 1, 10 and 100 (the FP64
    device run stands in for the FP64 oracle, which it matches on the
    smaller cases)."""

import numpy as np
import pytest

import workloads as W
from oracle import derived, operators as ops
from tests.gpu_common import rel, step_against_oracle_systems

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def naca():
    from paper_2211_10698_amd import ccns
    case = W.naca_4096()
    print(f"[naca] capacities {case.grid.nx}x{case.grid.ny}", flush=True)
    capsarr = ccns.ccns_capacities(case.grid, case.bodies)
    return case, capsarr


def _masks(caps, g):
    J, I = np.indices((g.ny + 2, g.nx + 2))
    au = (I >= 1) & (I <= g.nx - 1) & (J >= 1) & (J <= g.ny) & (caps[7] > 0) & (caps[1] > 0)
    av = (I >= 1) & (I <= g.nx) & (J >= 1) & (J <= g.ny - 1) & (caps[14] > 0) & (caps[2] > 0)
    return au, av


def test_naca_operator_applies_full_size(naca):
    from paper_2211_10698_amd import ccns
    case, capsarr = naca
    g = case.grid
    caps = {k: capsarr[i] for i, k in enumerate(ccns.CAP_NAMES)}
    pr = derived.prepare(caps, g.nx, g.ny, vol_floor=case.mass_floor * g.hx * g.hy)
    Dx, Dy = W.dirichlet(case)
    ctx = ccns.Context(g, ccns.make_params(case.rho, case.mu, case.tau, mass_floor=case.mass_floor), capsarr, Dx, Dy)
    rng = np.random.default_rng(21)
    sh = pr.act_p.shape
    Ux = np.where(pr.act_u, rng.uniform(-1, 1, sh), Dx)
    Uy = np.where(pr.act_v, rng.uniform(-1, 1, sh), Dy)
    P = np.where(pr.act_p, rng.uniform(-1, 1, sh), 0.0)
    dev = lambda a: torch.from_numpy(a).to("cuda")  # noqa: E731
    (c,) = ctx.apply(ccns.OP_CONT, [dev(Ux), dev(Uy)])
    assert rel(c.cpu().numpy(), ops.cont(caps, Ux, Uy, Dx, Dy)) < 1e-13
    gx, gy = ctx.apply(ccns.OP_PRES, [dev(P)])
    rx, ry = ops.pres(caps, P)
    assert rel(gx.cpu().numpy(), rx) < 1e-14 and rel(gy.cpu().numpy(), ry) < 1e-14
    vx, vy = ctx.apply(ccns.OP_VISC, [dev(Ux), dev(Uy)])
    wx, wy = ops.viscous(caps, Ux, Uy, Dx, Dy, "geometric")
    assert rel(vx.cpu().numpy(), wx, pr.act_u) < 1e-12 and rel(vy.cpu().numpy(), wy, pr.act_v) < 1e-12
    cx, cy = ctx.apply(ccns.OP_CONV, [dev(Ux), dev(Uy)])
    kx, ky = ops.conv(caps, Ux, Uy, Ux, Uy, Dx, Dy, Dx, Dy)
    assert rel(cx.cpu().numpy(), kx) < 1e-13 and rel(cy.cpu().numpy(), ky) < 1e-13
    (q,) = ctx.apply(ccns.OP_LAP, [dev(P)])
    assert rel(q.cpu().numpy(), derived.laplacian(pr, P)) < 1e-13
    ctx.close()


def test_naca_step_against_oracle_systems(naca):
    from oracle import pmii
    from paper_2211_10698_amd import ccns
    case, capsarr = naca
    g = case.grid
    caps = {k: capsarr[i] for i, k in enumerate(ccns.CAP_NAMES)}
    pr = derived.prepare(caps, g.nx, g.ny, vol_floor=case.mass_floor * g.hx * g.hy)
    Dx, Dy = W.dirichlet(case)
    prm = pmii.Params(rho=case.rho, mu=case.mu, tau=case.tau, u_inf=case.u_inf, pcg_tol=case.pcg_tol,
                      pred_tol=1e-12)
    # the oracle stepper only applies operators here (no solve)
    st = pmii.Stepper(pr, prm, Dx, Dy, min(g.hx, g.hy), jacobi=False)
    ctx = ccns.Context(g, ccns.make_params(case.rho, case.mu, case.tau, u_ref=case.u_inf, pcg_tol=case.pcg_tol,
                                           pred_tol=1e-12, mass_floor=case.mass_floor), capsarr, Dx, Dy)
    assert ctx.coef_classes() > 0
    step_against_oracle_systems(case, pr, st, ctx, Dx, Dy, "-naca")
    ctx.close()


def test_naca_mixed_against_fp64_100_steps(naca):
    from paper_2211_10698_amd import ccns
    case, capsarr = naca
    g = case.grid
    Dx, Dy = W.dirichlet(case)
    au, av = _masks(capsarr, g)
    px, py = W.perturbation(case)
    ctxs = []
    for prec in (0, 1):
        prm = ccns.make_params(case.rho, case.mu, case.tau, u_ref=case.u_inf, pcg_tol=case.pcg_tol,
                               pred_tol=1e-12, precision=prec, div_tol=1e-8, mass_floor=case.mass_floor)
        ctx = ccns.Context(g, prm, capsarr, Dx, Dy)
        ctx.set_field(ccns.F_UX, np.where(au, case.u_inf + px, Dx))
        ctx.set_field(ccns.F_UY, np.where(av, py, Dy))
        assert ctx.project().div_rel <= 1e-8
        ctxs.append(ctx)
    errs = {}
    for n in range(1, case.steps + 1):
        infos = [c.step(1) for c in ctxs]
        assert all(i.div_rel <= 1e-8 for i in infos), n
        if n in (1, 10, 100):
            u64 = [ctxs[0].get_field(f).cpu().numpy() for f in (ccns.F_UX, ccns.F_UY)]
            u32 = [ctxs[1].get_field(f).cpu().numpy() for f in (ccns.F_UX, ccns.F_UY)]
            umax = max(np.abs(u64[0]).max(), np.abs(u64[1]).max())
            errs[n] = max(np.abs(a - b).max() for a, b in zip(u32, u64)) / umax
            print(f"[naca] step {n}: mixed vs fp64 max velocity error {errs[n]:.2e} "
                  f"(iterations fp64 {infos[0].poisson.iterations}/{infos[0].pred.iterations}, "
                  f"mixed {infos[1].poisson.iterations}/{infos[1].pred.iterations})", flush=True)
    assert all(e <= 1e-6 for e in errs.values()), errs
    for c in ctxs:
        c.close()
