"""Shared set-up of the GPU parity tests: builds an oracle stepper and a
device context on the same capacities (computed by the oracle) and the same
seeded inputs."""

import numpy as np

import workloads as W
from oracle import derived, geometry, pmii


def case_setup(case, pcg_tol=None, pred_tol=1e-12, visc_form="geometric", caps=None, precond="mg",
               precision=0, div_tol=1e-8, mass_floor=None):
    from paper_2211_10698_amd import ccns

    g = case.grid
    if caps is None:
        caps = geometry.capacities(g, case.bodies)
    theta = case.mass_floor if mass_floor is None else mass_floor
    pr = derived.prepare(caps, g.nx, g.ny, vol_floor=theta * g.hx * g.hy)
    Dx, Dy = W.dirichlet(case)
    tol = case.pcg_tol if pcg_tol is None else pcg_tol
    prm = pmii.Params(rho=case.rho, mu=case.mu, tau=case.tau, u_inf=case.u_inf, pcg_tol=tol,
                      pred_tol=pred_tol, visc_form=visc_form)
    st = pmii.Stepper(pr, prm, Dx, Dy, min(g.hx, g.hy))
    form = {"geometric": 0, "literal": 1, "mean": 2}[visc_form]
    cp = ccns.make_params(case.rho, case.mu, case.tau, u_ref=case.u_inf, pcg_tol=tol, pred_tol=pred_tol,
                          visc_form=form, precision=precision, div_tol=div_tol, mass_floor=theta,
                          precond={"jacobi": ccns.PRECOND_JACOBI, "mg": ccns.PRECOND_MG}[precond])
    capsarr = np.stack([caps[k] for k in ccns.CAP_NAMES])
    ctx = ccns.Context(g, cp, capsarr, Dx, Dy)
    return caps, pr, st, ctx, Dx, Dy


def rel(a, b, mask=None):
    a = np.asarray(a)
    b = np.asarray(b)
    if mask is not None:
        a, b = a[mask], b[mask]
    den = max(np.max(np.abs(b)), 1e-300)
    return float(np.max(np.abs(a - b)) / den)
