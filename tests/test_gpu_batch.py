"""Ragged batches: several uneven simulations stepped together through
ccns_batch_step give bit for bit the fields and solver figures of each
simulation stepped alone, and each member matches the oracle as a solo run
does; both with one host thread and one HIP stream per simulation and with
the fused batch (one launch per phase over every simulation's
work-groups)."""

import numpy as np
import pytest

import workloads as W
from oracle import geometry, pmii
from tests.gpu_common import rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _cases():
    return [
        ("cyl64", W.cylinder_64(), 0),
        ("chan130", W.scaled_cylinder(130, 73, 2.6, 1.46, seed=5), 0),
        ("cyl96_mixed", W.scaled_cylinder(96, 96, 1.0, 1.0, seed=7), 1),
        ("ell200", W.Case("ell200", W.GridSpec(200, 120, 0.0, 0.0, 1.0, 0.6),
                          [W.Body(W.ELLIPSE, 0.41, 0.3, a=0.12, b=0.06, angle=0.4)], re=200.0, steps=3,
                          noise=1e-2, seed=8), 0),
        ("cyl40", W.scaled_cylinder(40, 40, 1.0, 1.0, seed=9), 1),
        ("cyl260", W.scaled_cylinder(260, 132, 2.0, 1.015, seed=10), 0),
    ]


_CAPS = {}


def _context(case, precision, stream):
    from paper_2211_10698_amd import ccns
    g = case.grid
    if case.name not in _CAPS:
        _CAPS[case.name] = ccns.ccns_capacities(g, case.bodies)
    caps = _CAPS[case.name]
    Dx, Dy = W.dirichlet(case)
    prm = ccns.make_params(case.rho, case.mu, case.tau, u_ref=case.u_inf, pcg_tol=1e-10, pred_tol=1e-12,
                           mass_floor=case.mass_floor,
                           precision=precision, div_tol=1e-8)
    ctx = ccns.Context(g, prm, caps, Dx, Dy, stream=stream)
    px, py = W.perturbation(case)
    sh = (g.ny + 2, g.nx + 2)
    J, I = np.indices(sh)
    au = (I >= 1) & (I <= g.nx - 1) & (J >= 1) & (J <= g.ny) & (caps[7] > 0) & (caps[1] > 0)
    av = (I >= 1) & (I <= g.nx) & (J >= 1) & (J <= g.ny - 1) & (caps[14] > 0) & (caps[2] > 0)
    ctx.set_field(ccns.F_UX, np.where(au, case.u_inf + px, Dx))
    ctx.set_field(ccns.F_UY, np.where(av, py, Dy))
    ctx.project()
    return ctx


def _state(ctx):
    from paper_2211_10698_amd import ccns
    return [ctx.get_field(f).cpu().numpy() for f in (ccns.F_UX, ccns.F_UY, ccns.F_P, ccns.F_PHI)]


def test_batch_matches_solo_runs_bit_for_bit():
    from paper_2211_10698_amd import ccns
    cases = _cases()
    nsteps = 3
    solo = []
    for name, case, prec in cases:
        print(f"[batch] solo {name}", flush=True)
        ctx = _context(case, prec, torch.cuda.current_stream())
        infos = [ctx.step(1) for _ in range(nsteps)]
        solo.append((_state(ctx), infos[-1].as_dict()))
        ctx.close()
    streams = [torch.cuda.Stream() for _ in cases]
    ctxs = [_context(case, prec, s) for (name, case, prec), s in zip(cases, streams)]
    torch.cuda.synchronize()
    batch = ccns.Batch(ctxs, nthreads=4)
    print("[batch] batch step", flush=True)
    st, infos, sts = batch.step(nsteps)
    assert st == ccns.OK and all(s == ccns.OK for s in sts)
    for (name, _, _), ctx, info, (ref, rinfo) in zip(cases, ctxs, infos, solo):
        got = _state(ctx)
        for a, b in zip(got, ref):
            assert np.array_equal(a, b), name
        assert info.as_dict() == rinfo, name
    batch.close()
    for c in ctxs:
        c.close()


@pytest.mark.parametrize("fused", [False, True])
@pytest.mark.parametrize("theta", [0.0, 0.05])
@pytest.mark.parametrize("name", ["cylinder_64", "flat_top_64"])
def test_batch_member_matches_oracle(name, theta, fused):
    """A 64x64 case inside a batch against the oracle (10 steps at tight
    tolerances, as the solo trajectory test), at the paper's mass matrix
    (theta = 0) and with the small-volume floor; in a batch of streams and
    in a fused batch."""
    from paper_2211_10698_amd import ccns
    from oracle import derived
    case = W.cylinder_64() if name == "cylinder_64" else W.flat_top_cylinder(64)
    g = case.grid
    caps = geometry.capacities(g, case.bodies)
    pr = derived.prepare(caps, g.nx, g.ny, vol_floor=theta * g.hx * g.hy)
    Dx, Dy = W.dirichlet(case)
    st = pmii.Stepper(pr, pmii.Params(rho=case.rho, mu=case.mu, tau=case.tau, pcg_tol=1e-13, pred_tol=1e-14),
                      Dx, Dy, g.hx)
    s0 = pmii.initial_state(pr, Dx, Dy, case.u_inf, W.perturbation(case))
    capsarr = np.stack([caps[k] for k in ccns.CAP_NAMES])
    prm = ccns.make_params(case.rho, case.mu, case.tau, pcg_tol=1e-13, pred_tol=1e-14, mass_floor=theta)
    streams = [torch.cuda.Stream() for _ in range(3)]
    ctxs = [ccns.Context(g, prm, capsarr, Dx, Dy, stream=s) for s in streams]
    for c in ctxs:
        c.set_field(ccns.F_UX, s0.Ux)
        c.set_field(ccns.F_UY, s0.Uy)
        c.project()
    st.project(s0)
    batch = ccns.Batch(ctxs, nthreads=3, fused=fused)
    for _ in range(case.steps):
        st.step(s0)
    status, infos, _ = batch.step(case.steps)
    assert status == ccns.OK
    for c in ctxs:
        assert rel(c.get_field(ccns.F_UX).cpu().numpy(), s0.Ux) < 1e-11
        assert rel(c.get_field(ccns.F_UY).cpu().numpy(), s0.Uy) < 1e-11
    batch.close()
    for c in ctxs:
        c.close()


def _fused_cases():
    """FP64 multigrid cases of every kernel variant the fused launches group:
    the coefficient class table and the arrays, the two viscous forms,
    several cycle depths and kernel forms, the coarsest-grid and LDS-tail
    ends, outflow walls and a stretched mesh."""
    from paper_2211_10698_amd import tune
    return [
        ("cyl64", W.cylinder_64(), {}),
        ("chan130", W.scaled_cylinder(130, 73, 2.6, 1.46, seed=5), {}),
        ("ell200_arrays", W.Case("ell200", W.GridSpec(200, 120, 0.0, 0.0, 1.0, 0.6),
                                 [W.Body(W.ELLIPSE, 0.41, 0.3, a=0.12, b=0.06, angle=0.4)], re=200.0, steps=3,
                                 noise=1e-2, seed=8), {"coef_tables": 1}),
        ("cyl260_literal", W.scaled_cylinder(260, 132, 2.0, 1.015, seed=10), {"visc_form": 1}),
        ("tiny12", W.Case("tiny12", W.GridSpec(12, 12, 0.0, 0.0, 1.0, 1.0), [W.Body(W.CIRCLE, 0.47, 0.52, a=0.2)],
                          re=100.0, steps=3, noise=1e-2, seed=11), {}),
        ("outflow48", W.outflow_cylinder(48), {}),
        ("stretched48", W.stretched_cylinder(48), {}),
        ("cyl300_forms", W.scaled_cylinder(300, 300, 1.0, 1.0, seed=12),
         {"mg_forms": tune.pack([(5, 2), (2, 5), (4, 1), (3, 4)])}),
    ]


def _context_mg(case, stream, extra):
    from paper_2211_10698_amd import ccns
    g = case.grid
    key = (case.name, g.nx, g.ny)
    if key not in _CAPS:
        _CAPS[key] = ccns.ccns_capacities(g, case.bodies)
    caps = _CAPS[key]
    Dx, Dy = W.dirichlet(case)
    prm = ccns.make_params(case.rho, case.mu, case.tau, u_ref=case.u_inf, pcg_tol=1e-10, pred_tol=1e-12,
                           mass_floor=case.mass_floor, outflow=case.outflow, **extra)
    ctx = ccns.Context(g, prm, caps, Dx, Dy, stream=stream)
    px, py = W.perturbation(case)
    sh = (g.ny + 2, g.nx + 2)
    J, I = np.indices(sh)
    au = (I >= 1) & (I <= g.nx - 1) & (J >= 1) & (J <= g.ny) & (caps[7] > 0) & (caps[1] > 0)
    av = (I >= 1) & (I <= g.nx) & (J >= 1) & (J <= g.ny - 1) & (caps[14] > 0) & (caps[2] > 0)
    ctx.set_field(ccns.F_UX, np.where(au, case.u_inf + px, Dx))
    ctx.set_field(ccns.F_UY, np.where(av, py, Dy))
    ctx.project()
    return ctx


@pytest.mark.parametrize("graphs", [True, False])
@pytest.mark.parametrize("precision", [0, 1])
def test_fused_batch_matches_solo_runs_bit_for_bit(precision, graphs):
    """Three steps of the fused batch give each simulation's solo fields and
    step figures bit for bit, in FP64 and in precision 1 (FP32 inner solves
    with FP64 refinement, whose sweeps run in lockstep), with each CG
    iteration replayed from a captured graph (every replay, with the
    batch's read-backs between chunks of them, enters the compared fields)
    and launched one by one; so do two fused steps followed by a solo step
    on each context (the contexts carry on from a fused step as from their
    own)."""
    from paper_2211_10698_amd import ccns
    cases = [(name, case, dict(extra, precision=precision, div_tol=1e-8)) for name, case, extra in _fused_cases()]
    nsteps = 3
    solo = []
    for name, case, extra in cases:
        print(f"[fused] solo {name} precision {precision}", flush=True)
        ctx = _context_mg(case, torch.cuda.current_stream(), extra)
        infos = [ctx.step(1) for _ in range(nsteps)]
        solo.append((_state(ctx), infos[-1].as_dict()))
        ctx.close()
    for split in (False, True):
        ctxs = [_context_mg(case, torch.cuda.Stream(), extra) for _, case, extra in cases]
        torch.cuda.synchronize()
        batch = ccns.Batch(ctxs, fused=True, graphs=graphs)
        print(f"[fused] batch steps, graphs {graphs} (then a solo step: {split})", flush=True)
        if split:
            st, _, _ = batch.step(nsteps - 1)
            assert st == ccns.OK
            infos = [c.step(1) for c in ctxs]
        else:
            st, infos, sts = batch.step(nsteps)
            assert st == ccns.OK and all(s == ccns.OK for s in sts)
        for (name, _, _), ctx, info, (ref, rinfo) in zip(cases, ctxs, infos, solo):
            got = _state(ctx)
            for a, b in zip(got, ref):
                assert np.array_equal(a, b), name
            assert info.as_dict() == rinfo, name
        batch.close()
        for c in ctxs:
            c.close()


def test_fused_batch_refuses_other_solvers():
    """The fused batch runs the multigrid preconditioner with one precision
    for all of its simulations: a context with the Jacobi preconditioner, or
    of another precision than the others, is refused."""
    from paper_2211_10698_amd import ccns
    case = W.cylinder_64()
    good = _context_mg(case, torch.cuda.current_stream(), {})
    for extra in ({"precision": 1}, {"precond": ccns.PRECOND_JACOBI}):
        other = _context_mg(case, torch.cuda.current_stream(), extra)
        with pytest.raises(ccns.CcnsError):
            ccns.Batch([good, other], fused=True)
        other.close()
    with pytest.raises(ccns.CcnsError):
        ccns.Batch([good, good], fused=True)
    b = ccns.Batch([good], fused=True)
    st, infos, _ = b.step(0)
    assert st == ccns.OK
    b.close()
    good.close()
