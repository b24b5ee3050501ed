"""Throughput of the cut-cell projection step on one MI355X.

Workload (default): the 2048x1024 channel [0,20]x[0,10] with a cylinder of
diameter 1 at (5,5), free stream 1 plus seeded 1e-3 divergence-free noise,
Re = 100, CFL 0.5, FP64, pressure solve to a relative residual of 1e-10
(which keeps max|cont(U, D)| / (U h) below 1e-8 every step).  A step is one
full projection-method-II step: convection and predictor right-hand side,
the viscous predictor solve, the Poisson right-hand side, the pressure
solve, the corrector and the pressure update, with the diagnostics.

Prints one JSON line.  `value` is whole-job cell-steps per second (in
millions) with the state resident in HBM.  `roofline` reports the Poisson
operator kernel (the dominant kernel): algorithmic bytes per launch over its
mean duration, timed with HIP events on the library's stream inside the
timed region.  `cpu_baseline` times the FP64 CPU oracle on a bounded sample
of the same workload (see its `sample` field).
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

HBM_PEAK_GBS = 8000.0
# Poisson operator kernel, FP64: reads r, dinv, p_old, c^x, c^y and writes
# p, q -- 7 arrays of 8 bytes per cell
POIS_APPLY_BYTES_PER_CELL = 56.0
POIS_UPDATE_BYTES_PER_CELL = 56.0   # reads x, p, r, q, dinv; writes x, r

WORKLOADS = {
    "channel_cylinder_2048x1024": W.channel_cylinder_2048,
    "cylinder_64": W.cylinder_64,
    "naca0012_4096x2048": W.naca_4096,
}


def unknown_masks(caps, nx, ny):
    """Velocity unknowns: faces interior to the box with fluid in their
    staggered control volume (the same rule the library applies)."""
    sh = (ny + 2, nx + 2)
    J, I = np.indices(sh)
    au = (I >= 1) & (I <= nx - 1) & (J >= 1) & (J <= ny) & (caps[7] > 0)
    av = (I >= 1) & (I <= nx) & (J >= 1) & (J <= ny - 1) & (caps[14] > 0)
    return au, av


def cpu_baseline(case, n_cg_per_step, iters_sample=20):
    """Times the oracle on the host: one full predictor phase plus a fixed
    number of Poisson PCG iterations, plus the corrector/pressure update of
    the same workload, then scales to one step with the Poisson iteration
    count the device needed per step."""
    from oracle import derived, geometry, pmii, solvers

    g = case.grid
    caps = geometry.capacities(g, case.bodies)
    pr = derived.prepare(caps, g.nx, g.ny)
    Dx, Dy = W.dirichlet(case)
    prm = pmii.Params(rho=case.rho, mu=case.mu, tau=case.tau, pcg_tol=case.pcg_tol)
    st = pmii.Stepper(pr, prm, Dx, Dy, min(g.hx, g.hy))
    s0 = pmii.initial_state(pr, Dx, Dy, case.u_inf, W.perturbation(case))
    t0 = time.perf_counter()
    (usx, usy), _ = st.predict(s0, pmii.StepInfo())
    b = st.poisson_rhs(usx, usy)
    t1 = time.perf_counter()
    phi, it, _, _ = solvers.pcg(st.apply_A, -b, s0.Phi, st.Pdinv, pr.act_p, 0.0, iters_sample, zero_mean=True)
    t2 = time.perf_counter()
    ux, uy = st.correct(usx, usy, phi)
    st.pressure_update(s0.P, phi)
    st.diagnostics(ux, uy, pmii.StepInfo())
    t3 = time.perf_counter()
    per_it = (t2 - t1) / max(it, 1)
    step_s = (t1 - t0) + (t3 - t2) + per_it * n_cg_per_step
    return {
        "value": g.nx * g.ny / step_s / 1e6,
        "unit": "Mcell-steps/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"one step of the {case.name} workload on the full grid: predictor phase "
                   f"({t1 - t0:.2f} s) and corrector/pressure update ({t3 - t2:.2f} s) timed whole; "
                   f"{it} Poisson PCG iterations timed ({per_it * 1e3:.1f} ms each) and scaled to the "
                   f"{n_cg_per_step:.0f} iterations per step the device needed; numpy runs single-threaded"),
        "seconds_per_step": step_s,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="channel_cylinder_2048x1024", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(independent simulations shard across GPUs without communication).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2211_10698_amd import ccns

    case = WORKLOADS[args.workload]()
    g = case.grid
    t_setup = time.perf_counter()
    caps = ccns.ccns_capacities(g, case.bodies)
    Dx, Dy = W.dirichlet(case)
    params = ccns.make_params(case.rho, case.mu, case.tau, u_ref=case.u_inf, pcg_tol=case.pcg_tol,
                              pred_tol=1e-12)
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    ctx = ccns.Context(g, params, caps, Dx, Dy, stream=stream)
    au, av = unknown_masks(caps, g.nx, g.ny)
    px, py = W.perturbation(case)
    ctx.set_field(ccns.F_UX, np.where(au, case.u_inf + px, Dx))
    ctx.set_field(ccns.F_UY, np.where(av, py, Dy))
    ctx.project()
    setup_s = time.perf_counter() - t_setup
    print(f"[bench] setup {setup_s:.1f}s: {case.name} {g.nx}x{g.ny}", file=sys.stderr, flush=True)

    for k in range(args.warmup):
        info = ctx.step(1)
        print(f"[bench] warmup {k}: cg {info.poisson.iterations} pred {info.pred.iterations} "
              f"div_rel {info.div_rel:.2e}", file=sys.stderr, flush=True)

    ctx.timing(1)
    infos = []
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    t0 = time.perf_counter()
    for k in range(args.steps):
        info = ctx.step(1)
        infos.append(info.as_dict())
        print(f"[bench] step {k}: cg {info.poisson.iterations} pred {info.pred.iterations} "
              f"div_rel {info.div_rel:.2e}", file=sys.stderr, flush=True)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    ms, cnt = ctx.timing(0)
    elapsed = max(wall, gpu_ms * 1e-3)
    cells = g.nx * g.ny
    value = cells * args.steps / elapsed / 1e6
    div_max = max(i["div_rel"] for i in infos)
    n_cg = float(np.mean([i["cg_iters"] for i in infos]))
    apply_ms = ms[0] / max(cnt[0], 1)
    upd_ms = ms[1] / max(cnt[1], 1)
    achieved = POIS_APPLY_BYTES_PER_CELL * cells / (apply_ms * 1e-3) / 1e9
    out = {
        "metric": "Mcell-steps/s at 1e-8 divergence",
        "value": value,
        "unit": "Mcell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": case.name, "nx": g.nx, "ny": g.ny, "re": case.re, "cfl": case.cfl,
                   "pcg_tol": case.pcg_tol, "precond": "multigrid", "precision": "fp64"},
        "div_rel_max": div_max,
        "cg_iters_per_step": n_cg,
        "pred_iters_per_step": float(np.mean([i["pred_iters"] for i in infos])),
        "roofline": {
            "kernel": "k_pois_dir_apply",
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
            "bytes_per_launch": POIS_APPLY_BYTES_PER_CELL * cells,
            "mean_launch_us": apply_ms * 1e3,
            "timed_launches": cnt[0],
            "update_kernel_GBs": POIS_UPDATE_BYTES_PER_CELL * cells / (upd_ms * 1e-3) / 1e9,
            "update_mean_launch_us": upd_ms * 1e3,
        },
        "cpu_baseline": None,
    }
    if div_max > 1e-8:
        out["warning"] = "divergence above 1e-8 in a timed step"
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        cb = cpu_baseline(case, n_cg)
        out["cpu_baseline"] = {k: cb[k] for k in ("value", "unit", "cores", "kind", "sample")}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
