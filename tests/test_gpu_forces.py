"""The device's force on the bodies (ccns_forces) against the oracle's
(oracle.forces, the same reading of the drag and lift of Sec. 5) on the same
state: after steps of the paper's cylinder set-up and of the three-ellipse
case, and on random fields set on the isolated-pocket case (whose pocket
cells carry no pressure).  The sums differ only in their order: 1e-12 of the
largest component."""

import numpy as np
import pytest

import workloads as W
from oracle import forces, pmii
from tests.gpu_common import case_setup

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _host(t):
    return t.cpu().numpy()


def _check(ctx, caps, pr, Dx, Dy, mu):
    from paper_2211_10698_amd import ccns
    fd = np.array(ctx.forces())
    P = _host(ctx.get_field(ccns.F_P))
    ux, uy = _host(ctx.get_field(ccns.F_UX)), _host(ctx.get_field(ccns.F_UY))
    fo = np.array(forces.forces(caps, P, ux, uy, Dx, Dy, mu, pmask=pr.act_p))
    scale = np.max(np.abs(fo))
    assert scale > 0
    assert np.max(np.abs(fd - fo)) <= 1e-12 * scale, (fd, fo)
    return fd


@pytest.mark.parametrize("name", ["outflow", "ellipses"])
def test_forces_after_steps(name):
    from paper_2211_10698_amd import ccns
    case = W.outflow_cylinder(48) if name == "outflow" else W.ellipses(96)
    caps = None
    if name == "ellipses":
        arr = ccns.ccns_capacities(case.grid, case.bodies)
        caps = {k: arr[i] for i, k in enumerate(ccns.CAP_NAMES)}
    caps, pr, st, ctx, Dx, Dy = case_setup(case, pcg_tol=1e-10, caps=caps)
    s0 = pmii.initial_state(pr, Dx, Dy, case.u_inf, W.perturbation(case))
    ctx.set_field(ccns.F_UX, s0.Ux)
    ctx.set_field(ccns.F_UY, s0.Uy)
    ctx.project()
    for n in range(5):
        ctx.step(1)
        fd = _check(ctx, caps, pr, Dx, Dy, case.mu)
    cd, cl = forces.coefficients(fd, case.rho, case.u_inf, case.ref_length)
    print(f"[forces] {case.name}: Cd {cd:.4f} Cl {cl:.4f}", flush=True)
    assert fd[0] + fd[2] > 0     # the flow drags the bodies downstream
    ctx.close()


def test_forces_of_set_fields_with_a_pocket():
    from paper_2211_10698_amd import ccns
    case = W.pocket(64)
    arr = ccns.ccns_capacities(case.grid, case.bodies)
    caps = {k: arr[i] for i, k in enumerate(ccns.CAP_NAMES)}
    caps, pr, st, ctx, Dx, Dy = case_setup(case, pcg_tol=1e-10, caps=caps)
    rng = np.random.default_rng(17)
    sh = pr.act_p.shape
    # pressure everywhere (the pocket cells' values must not count)
    ctx.set_field(ccns.F_P, rng.uniform(-1, 1, sh))
    ctx.set_field(ccns.F_UX, np.where(pr.act_u, rng.uniform(-1, 1, sh), Dx))
    ctx.set_field(ccns.F_UY, np.where(pr.act_v, rng.uniform(-1, 1, sh), Dy))
    _check(ctx, caps, pr, Dx, Dy, case.mu)
    ctx.close()
