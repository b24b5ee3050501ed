"""The predictor CG's coefficient classes: a context that reads the
coefficients through the class table (one index per entry) and one that
reads the coefficient arrays give the same fields, bit for bit, step after
step, in both precisions and both symmetric node-weight forms; a field of
all-distinct coefficients falls back to the arrays."""

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _masks(caps, g):
    J, I = np.indices((g.ny + 2, g.nx + 2))
    au = (I >= 1) & (I <= g.nx - 1) & (J >= 1) & (J <= g.ny) & (caps[7] > 0) & (caps[1] > 0)
    av = (I >= 1) & (I <= g.nx) & (J >= 1) & (J <= g.ny - 1) & (caps[14] > 0) & (caps[2] > 0)
    return au, av


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("visc_form", [0, 2])
def test_classes_equal_arrays_bit_for_bit(precision, visc_form):
    from paper_2211_10698_amd import ccns
    # several tiles in both directions and a ragged tail (pitch 320, rows 139)
    case = W.scaled_cylinder(258, 137, 5.16, 2.74, seed=7)
    g = case.grid
    print(f"[classes] {g.nx}x{g.ny} precision {precision} visc_form {visc_form}", flush=True)
    caps = ccns.ccns_capacities(g, case.bodies)
    Dx, Dy = W.dirichlet(case)
    au, av = _masks(caps, g)
    px, py = W.perturbation(case)
    ctxs = []
    for tables in (0, 1):
        prm = ccns.make_params(case.rho, case.mu, case.tau, u_ref=case.u_inf, pcg_tol=case.pcg_tol,
                               pred_tol=1e-12, precision=precision, div_tol=1e-8, visc_form=visc_form,
                               mass_floor=case.mass_floor, coef_tables=tables)
        ctx = ccns.Context(g, prm, caps, Dx, Dy)
        ctx.set_field(ccns.F_UX, np.where(au, case.u_inf + px, Dx))
        ctx.set_field(ccns.F_UY, np.where(av, py, Dy))
        ctx.project()
        ctxs.append(ctx)
    n = (g.ny + 2) * ((g.nx + 2 + 63) // 64 * 64)
    assert 0 < ctxs[0].coef_classes() <= max(1024, n // 16)
    assert ctxs[1].coef_classes() == 0
    for step in range(5):
        infos = [c.step(1) for c in ctxs]
        assert infos[0].pred.iterations == infos[1].pred.iterations > 0
        for f in (ccns.F_UX, ccns.F_UY, ccns.F_P, ccns.F_USX, ccns.F_USY):
            a = ctxs[0].get_field(f).cpu().numpy()
            b = ctxs[1].get_field(f).cpu().numpy()
            assert np.array_equal(a, b), (step, f)
    for c in ctxs:
        c.close()


def test_distinct_coefficients_fall_back_to_arrays():
    from paper_2211_10698_amd import ccns
    nx, ny = 200, 120
    g = W.GridSpec(nx, ny, 0.0, 0.0, 2.0, 1.2)
    rc = W.random_capacities(nx, ny, seed=3, hx=g.hx, hy=g.hy)
    caps = np.stack([rc[k] for k in ccns.CAP_NAMES])
    z = np.zeros((ny + 2, nx + 2))
    ctx = ccns.Context(g, ccns.make_params(1.0, 0.01, 0.005), caps, z, z)
    assert ctx.coef_classes() == 0
    ctx.close()
