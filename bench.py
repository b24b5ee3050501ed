"""Throughput of the cut-cell projection step on one MI355X.

Workload (default): the 4096x2048 box [0,8]x[0,4] around a NACA0012 section
(chord 1 at 5 degrees, leading edge at (2,2)), free stream 1 plus seeded
1e-3 divergence-free noise, Re = 1000, CFL 0.5, FP64, pressure solve to a
relative residual of 1e-10 (which keeps max|cont(U, D)| / (U h) below 1e-8
every step).  `--workload channel_cylinder_2048x1024` runs the 2048x1024
channel cylinder instead, `--precision mixed` the FP32 inner solves with FP64
refinement.  A step is one full projection-method-II step: convection and
predictor right-hand side, the viscous predictor solve, the Poisson
right-hand side, the pressure solve, the corrector and the pressure update,
with the diagnostics.

Prints one JSON line.  `value` is whole-job cell-steps per second (in
millions) with the state resident in HBM.  `roofline` reports the dominant
kernel, the predictor's CG iteration kernel (k_pred_cg): algorithmic bytes
per launch over its mean duration, timed with HIP events on the library's
stream inside the timed region (iterations 4, 12, 20, ... of each solve).
`cpu_baseline` times the FP64 CPU oracle on a bounded sample of the same
workload (see its `sample` field).
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
from paper_2211_10698_amd import tune  # noqa: E402

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
DEVICE_SRC = os.path.join(ROOT, "paper_2211_10698_amd", "csrc", "ccns_device.hip")
KERNEL_HDR = os.path.join(ROOT, "paper_2211_10698_amd", "csrc", "ccns_kern.h")
# Algorithmic bytes per cell of one predictor CG iteration: the scope's figure
# for the method (27 values of 8 bytes per cell: the CG vectors and the
# viscous and mass coefficients of both face components), the roofline's
# `achieved`.  Half of it for the float vectors of the mixed mode.
PRED_CG_SCOPE_BYTES_PER_CELL = 216.0
# What the kernel itself has to move.
# Predictor CG iteration (k_pred_cg), per cell = one x-face and one y-face:
# reads r, H p and p of the previous iteration, x and M^-1 (2 components
# each), M^x, M^y, B^xx, B^xy, B^yy, B^yx, 1/W^xx, 1/W^yy and the two diagonal
# node weights (the cross weight of the symmetric form is their geometric
# mean, formed in the kernel); writes r, x, p and H p (2 each).
PRED_CG_VALUES_PER_CELL = 28
# The same kernel reading its coefficients through the class table: the 12
# coefficient values become one 4-byte class index per entry (the table rows
# are shared by every entry of a class and stay in cache).
PRED_CG_VALUES_PER_CELL_CLS = 16
PRED_CG_INDEX_BYTES = 4.0
# Poisson direction+operator (multigrid path): reads z, p_old, 1/diag, c^x,
# c^y; writes p, A p.
POIS_DIR_BYTES_PER_CELL = 7 * 8.0
# Poisson CG update (multigrid path): reads x, p, r, A p; writes x, r.
POIS_UPDATE_BYTES_PER_CELL = 6 * 8.0

WORKLOADS = {
    "naca0012_4096x2048": W.naca_4096,
    "channel_cylinder_2048x1024": W.channel_cylinder_2048,
    "cylinder_64": W.cylinder_64,
    "paper_cylinder_2048x1024": W.paper_cylinder,
    "batched_cylinders_256": None,   # ragged batch, see run_batched
    "serving_trace": None,           # served requests, see run_serving
    "sphere_projection_256": None,   # the 3-D projection step, see run_projection3d
}

# The 3-D Poisson CG's direction-and-operator kernel: reads z, p_old and the
# three face weights c^x, c^y, c^z of its cell; writes p and (-L) p.  The
# update kernel reads 1/diag, p, (-L) p, x, r and writes x, r, z.
DIR3_BYTES_PER_CELL = 7 * 8.0
UPDATE3_BYTES_PER_ELEMENT = 8 * 8.0
# With the multigrid preconditioner the update forms no z: p, q, x, r read,
# x and r written.
UPDATE3_MG_BYTES_PER_ELEMENT = 6 * 8.0
# The finest level's up-sweep of the 3-D multigrid cycle: reads the iterate,
# the right-hand side, 1/diag and c^x, c^y, c^z of its cell and the coarse
# correction (one value per eight cells); writes the new iterate.
SWEEP3_BYTES_PER_CELL = 7 * 8.0 + 1.0
# The same with the cycle's fields in FP32: the iterate, 1/diag and the three
# weights in FP32, the residual r in FP64, the coarse correction in FP32.
SWEEP3_F32_BYTES_PER_CELL = 6 * 4.0 + 8.0 + 0.5


# Device helpers whose text a kernel's counter readings also depend on.
KERNEL_DEPS = {
    "k_pred_cg": ["pred_cg_body", "pred_rows", "ViscCoefT", "PredCoefT", "PredTileNx", "pred_tile_strains", "pred_tile_K",
                  "pred_tile_K_row", "pred_node_strain_row", "strain_cell", "strain_node", "strain_face"],
}


def kernel_digest(name):
    """SHA-1 of a kernel's source text (its definition in the device source,
    the device helpers it calls, and the shared device header), so that
    stored counter readings are used only while the kernel they were taken
    on is unchanged."""
    import hashlib
    import re

    src = open(DEVICE_SRC).read()
    m = re.search(r"__global__[^\n]*\b" + re.escape(name) + r"\(.*?\n}\n", src, re.S)
    if m is None:
        return None
    h = hashlib.sha1(m.group(0).encode())
    for dep in KERNEL_DEPS.get(name, []):
        # every definition of the name (overloads included)
        ds = list(re.finditer(r"^(?:template <[^\n]*>\n)?(?:struct " + re.escape(dep) + r"\b|__device__[^\n]*\b"
                              + re.escape(dep) + r"\().*?^};?$", src, re.S | re.M))
        if not ds:
            return None
        for d in ds:
            h.update(d.group(0).encode())
    h.update(open(KERNEL_HDR, "rb").read())
    return h.hexdigest()


def stored_traffic(name, workload, classes):
    """HBM bytes per launch of `name` from the committed counter summary, or
    None when there is none for this workload and coefficient path, or the
    kernel has changed."""
    try:
        t = json.load(open(TRAFFIC_FILE)).get(f"{name}@{workload}")
    except (OSError, ValueError):
        return None
    if (not t or t.get("workload") != workload or t.get("kernel_sha1") != kernel_digest(name)
            or t.get("coef_classes", False) != classes):
        return None
    return t["bytes_per_launch"]


def file_digest(*paths):
    """SHA-1 of whole source files: the 3-D kernels' counter readings are
    used only while their source and the shared device header are
    unchanged."""
    import hashlib

    h = hashlib.sha1()
    for p in paths:
        h.update(open(p, "rb").read())
    return h.hexdigest()


SRC3 = os.path.join(ROOT, "paper_2211_10698_amd", "csrc", "ccns3d.hip")
SWEEP3_KERNEL = {1: "k3_mg_tile<2, 0, double", 2: "k3_mg_tile<2, 0, float"}


def traffic3_key(precond):
    return f"k3_mg_tile<T_POST1>@sphere_projection_256/{'fp32' if precond == 2 else 'fp64'}"


def stored_traffic3(precond):
    """HBM bytes per launch of the 3-D cycle's finest up-sweep from the
    committed counter summary, or None when there is none or the 3-D source
    has changed."""
    try:
        t = json.load(open(TRAFFIC_FILE)).get(traffic3_key(precond))
    except (OSError, ValueError):
        return None
    if not t or t.get("source_sha1") != file_digest(SRC3, KERNEL_HDR):
        return None
    return t["bytes_per_launch"]


def summarize_counters(root, kernel, workload, classes, key=None, digest=None):
    """Turns four rocprofv3 --pmc runs into the stored traffic figure:
    root/fetch and root/write hold FETCH_SIZE and WRITE_SIZE of the bench
    run, root/cfetch and root/cwrite the same counters over the plain copies
    of --calibrate-copy.  Each counter is scaled by (bytes the copy moved) /
    (what the counter read for it); the result is the median over the
    kernel's full launches."""
    import csv
    import glob
    import statistics

    def med(sub, pat, counter):
        vals = []
        for f in glob.glob(os.path.join(root, sub, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(f)):
                if pat in r["Kernel_Name"] and r["Counter_Name"] == counter:
                    vals.append(float(r["Counter_Value"]))
        big = max(vals)
        vals = [v for v in vals if v > 0.5 * big]   # full launches, not early exits
        return statistics.median(vals), len(vals)

    copy_kib = CALIB_BYTES / 1024.0
    cf, _ = med("cfetch", "copyBuffer", "FETCH_SIZE")
    cw, _ = med("cwrite", "copyBuffer", "WRITE_SIZE")
    fk, nf = med("fetch", kernel, "FETCH_SIZE")
    wk, nw = med("write", kernel, "WRITE_SIZE")
    sf, sw = copy_kib / cf, copy_kib / cw
    rec = {"workload": workload, "coef_classes": classes,
           **({"source_sha1": digest} if digest else {"kernel_sha1": kernel_digest(kernel)}),
           "fetch_kib": fk, "write_kib": wk,
           "launches": [nf, nw], "copy_fetch_kib": cf, "copy_write_kib": cw, "fetch_scale": sf,
           "write_scale": sw, "bytes_per_launch": (fk * sf + wk * sw) * 1024.0}
    try:
        data = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        data = {}
    data[key or f"{kernel}@{workload}"] = rec
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(data, f, indent=1)
        f.write("\n")
    print(json.dumps({kernel: rec}))


CALIB_BYTES = 1 << 30


def calibrate_copy(reps=3):
    """Three device-to-device copies of 1 GiB: the reference reading for the
    FETCH_SIZE / WRITE_SIZE counters (each copy reads and writes 1 GiB)."""
    import torch

    a = torch.empty(CALIB_BYTES // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(f"[bench] copied {reps} x {CALIB_BYTES} bytes", flush=True)


def unknown_masks(caps, nx, ny):
    """Velocity unknowns: open faces (A > 0) interior to the box with fluid
    in their staggered control volume (the rule the library applies)."""
    sh = (ny + 2, nx + 2)
    J, I = np.indices(sh)
    au = (I >= 1) & (I <= nx - 1) & (J >= 1) & (J <= ny) & (caps[7] > 0) & (caps[1] > 0)
    av = (I >= 1) & (I <= nx) & (J >= 1) & (J <= ny - 1) & (caps[14] > 0) & (caps[2] > 0)
    return au, av


def host_cpu():
    """Model name and logical core count of the host."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, os.cpu_count()


def cpu_baseline(case, caps_arr, n_pred, n_cg, iters_sample=5):
    """Times the FP64 oracle on the host on the full grid of the workload:
    the explicit phases of one step whole (convection and the predictor
    right-hand side; the Poisson right-hand side; the corrector and the
    pressure update with the diagnostics), and `iters_sample` iterations of
    each of its two Jacobi-PCG solves.  A whole step is then the explicit
    phases plus the per-iteration times scaled to the iteration counts one
    step needs with that algorithm (n_pred predictor and n_cg Poisson
    iterations, see the caller): an extrapolation, labelled as such.  The
    oracle's operators are vectorised numpy on one thread."""
    from oracle import derived, pmii, solvers

    g = case.grid
    names = ("V", "Ax", "Ay", "Bx", "By", "Wx", "Wy", "Vu", "Axx", "Axy", "Bxx", "Bxy", "Wxx", "Wxy",
             "Vv", "Ayy", "Ayx", "Byy", "Byx", "Wyy", "Wyx")
    caps = {k: caps_arr[i] for i, k in enumerate(names)}
    pr = derived.prepare(caps, g.nx, g.ny, vol_floor=case.mass_floor * g.hx * g.hy, outflow=case.outflow)
    Dx, Dy = W.dirichlet(case)
    prm = pmii.Params(rho=case.rho, mu=case.mu, tau=case.tau, pcg_tol=case.pcg_tol)
    st = pmii.Stepper(pr, prm, Dx, Dy, min(g.hx, g.hy), jacobi=False)
    s0 = pmii.initial_state(pr, Dx, Dy, case.u_inf, W.perturbation(case))
    t0 = time.perf_counter()
    conv_n = st.convection(s0.Ux, s0.Uy)
    rhs = st.predictor_rhs(s0, conv_n, conv_n)
    t1 = time.perf_counter()
    # the cost of an iteration does not depend on the preconditioner's values:
    # the mass part of H's diagonal stands in for the probed diagonal
    dmass = np.where(st.mask2, 1.0 / np.maximum((prm.rho / prm.tau) * np.stack([st.Vu, st.Vv]), 1e-300), 0.0)
    U0 = np.stack([s0.Ux, s0.Uy])
    _, itp, _, _ = solvers.pcg(st.apply_H, rhs, U0, dmass, st.mask2, 0.0, iters_sample)
    t2 = time.perf_counter()
    b = st.poisson_rhs(s0.Ux, s0.Uy)
    t3 = time.perf_counter()
    phi, itc, _, _ = solvers.pcg(st.apply_A, -b, s0.Phi, st.Pdinv, pr.act_p, 0.0, iters_sample,
                                 zero_mean=pr.singular)
    t4 = time.perf_counter()
    ux, uy = st.correct(s0.Ux, s0.Uy, phi)
    st.pressure_update(s0.P, phi)
    st.diagnostics(ux, uy, pmii.StepInfo())
    t5 = time.perf_counter()
    per_pred = (t2 - t1) / max(itp, 1)
    per_cg = (t4 - t3) / max(itc, 1)
    explicit = (t1 - t0) + (t3 - t2) + (t5 - t4)
    step_s = explicit + per_pred * n_pred + per_cg * n_cg
    model, ncpu = host_cpu()
    return {
        "value": g.nx * g.ny / step_s / 1e6,
        "unit": "Mcell-steps/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"the FP64 oracle (numpy, one thread) on the full {g.nx}x{g.ny} grid of {case.name}: the "
                   f"explicit phases of one step timed whole ({explicit:.2f} s: convection and predictor "
                   f"right-hand side {t1 - t0:.2f} s, Poisson right-hand side {t3 - t2:.2f} s, corrector, "
                   f"pressure update and diagnostics {t5 - t4:.2f} s), {itp} predictor Jacobi-PCG iterations "
                   f"({per_pred:.2f} s each) and {itc} Poisson Jacobi-PCG iterations ({per_cg:.2f} s each) timed; "
                   f"a step is EXTRAPOLATED to {n_pred} predictor and {n_cg} Poisson iterations, the counts of "
                   f"one step of this workload with the oracle's algorithm (Jacobi-PCG for both solves; the "
                   f"counts were taken by the library's Jacobi-PCG on the same step, which matches the "
                   f"oracle's count within 2 in the parity tests); host {model}, {ncpu} logical cores"),
        "seconds_per_step": step_s,
        "extrapolated": True,
        "host_cpu": model,
        "host_logical_cores": ncpu,
        "threads": 1,
    }


def host_inputs(ccns, case):
    """Host part of a simulation's set-up (no GPU calls): capacities from the
    library and the seeded inputs."""
    g = case.grid
    caps = ccns.ccns_capacities(g, case.bodies)
    Dx, Dy = W.dirichlet(case)
    au, av = unknown_masks(caps, g.nx, g.ny)
    px, py = W.perturbation(case)
    return caps, Dx, Dy, np.where(au, case.u_inf + px, Dx), np.where(av, py, Dy)


def setup_context(ccns, case, precision, stream, host, coef_tables=0, mg_forms=True):
    """Context, initial field and initial projection of one simulation (set-up,
    outside any timed region)."""
    caps, Dx, Dy, ux0, uy0 = host
    params = ccns.make_params(case.rho, case.mu, case.tau, u_ref=case.u_inf, pcg_tol=case.pcg_tol,
                              pred_tol=1e-12, precision=precision, div_tol=1e-8, mass_floor=case.mass_floor,
                              coef_tables=coef_tables)
    ctx = ccns.Context(case.grid, params, caps, Dx, Dy, stream=stream)
    ctx.set_field(ccns.F_UX, ux0)
    ctx.set_field(ccns.F_UY, uy0)
    ctx.project()
    if mg_forms:
        tune.apply_cached(ctx, precision)
    return ctx


def run_batched(args):
    """The ragged batch: 256 cylinder simulations of 128^2 .. 1024^2 cells
    (seeded sizes, radii, centres and Reynolds numbers), advanced together
    by ccns_batch_step: by default as a fused batch (one launch per phase
    over every simulation's work-groups), else (--batch-mode streams) with
    16 host threads and one stream per simulation.  A step advances every
    simulation by one projection step; value = total cell-steps / time."""
    import concurrent.futures as cf

    import torch
    from paper_2211_10698_amd import ccns

    cases = W.batched_cylinders(256)
    prec = 1 if args.precision == "mixed" else 0
    mode = "streams" if args.batch_mode == "streams" else "fused"
    torch.cuda.set_device(0)
    t_setup = time.perf_counter()
    # a fused batch runs on its own stream: the contexts can share one
    shared = torch.cuda.Stream()
    streams = [shared if mode == "fused" else torch.cuda.Stream() for _ in cases]
    ctxs = []
    with cf.ThreadPoolExecutor(max_workers=8) as ex:
        for case, stream, host in zip(cases, streams, ex.map(lambda c: host_inputs(ccns, c), cases)):
            ctxs.append(setup_context(ccns, case, prec, stream, host, 0 if args.coef_tables == "auto" else 1,
                                      args.mg_forms == "tuned"))
    torch.cuda.synchronize()
    cells = sum(c.grid.nx * c.grid.ny for c in cases)
    print(f"[bench] setup {time.perf_counter() - t_setup:.1f}s: {len(cases)} simulations, {cells} cells",
          file=sys.stderr, flush=True)
    batch = ccns.Batch(ctxs, nthreads=16, fused=mode == "fused", graphs=args.batch_graphs == "on")
    failures = []

    def record(tag, st, infos, sts):
        # a simulation whose solve did not converge: its figures and the
        # statuses of its inner solves (precision 1)
        for k, (i, s) in enumerate(zip(infos, sts)):
            if s != ccns.OK:
                failures.append({"step": tag, "simulation": cases[k].name, "status": int(s), **i.as_dict()})
                print(f"[bench] {tag}: {cases[k].name} status {s}: {i.as_dict()}", file=sys.stderr, flush=True)

    for k in range(args.warmup):
        st, infos, sts = batch.step(1, check=False)
        record(f"warmup {k}", st, infos, sts)
        print(f"[bench] warmup {k}: worst div_rel {max(i.div_rel for i in infos):.2e}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    divs, cg, pred = [], [], []
    for k in range(args.steps):
        st, infos, sts = batch.step(1, check=False)
        record(f"step {k}", st, infos, sts)
        divs.append(max(i.div_rel for i in infos))
        cg.append(float(np.mean([i.poisson.iterations for i in infos])))
        pred.append(float(np.mean([i.pred.iterations for i in infos])))
        print(f"[bench] step {k}: worst div_rel {divs[-1]:.2e}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sizes = {}
    for c in cases:
        sizes[c.grid.nx] = sizes.get(c.grid.nx, 0) + 1
    out = {
        "metric": "Mcell-steps/s at 1e-8 divergence",
        "value": cells * args.steps / wall / 1e6,
        "unit": "Mcell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if prec else "f64",
        "data": "synthetic",
        "config": {"workload": "batched_cylinders_256", "simulations": len(cases), "cells": cells,
                   "coef_classes_used": sum(1 for c in ctxs if c.coef_classes() > 0),
                   "sizes": {str(k): v for k, v in sorted(sizes.items())}, "precond": "multigrid",
                   "precision": "fp32 inner + fp64 refinement, div_rel <= 1e-8" if prec else "fp64",
                   "batch_mode": ("fused: one launch per phase over all simulations' work-groups" if mode == "fused"
                                  else "streams: 16 host threads, one stream per simulation"),
                   "cg_iterations_as_graphs": mode == "fused" and args.batch_graphs == "on"},
        "div_rel_max": max(divs),
        "cg_iters_per_step_mean": float(np.mean(cg)),
        "pred_iters_per_step_mean": float(np.mean(pred)),
        "roofline": None,
        "cpu_baseline": None,
        "failures": failures,
    }
    if max(divs) > 1e-8:
        out["warning"] = "divergence above 1e-8 in a timed step"
    if failures:
        out["warning"] = f"{len(failures)} simulation steps ended with a solver status other than OK"
    print(json.dumps(out), flush=True)
    batch.close()
    for c in ctxs:
        c.close()


def run_serving(args):
    """The serving trace: Poisson arrivals (20 per second) of simulations of
    256^2 .. 2048^2 cells with 1-3 ellipses, 100 steps each, served by the
    continuous-batching server under an HBM budget of 85% of free device
    memory.  The first --requests requests of the seeded trace are served in
    real time; the line reports latency percentiles (queue and service
    separately) and the served throughput."""
    import torch
    from paper_2211_10698_amd import serve

    if not args.serving_unresolved:
        raise SystemExit("serving_trace: two runs of this line since the force tables wrote nothing for 180 s and "
                         "were stopped, with no cause found; it runs only with --serving-unresolved")
    torch.cuda.set_device(0)
    reqs = W.serving_trace()[: args.requests]
    prec = 1 if args.precision == "mixed" else 0
    srv = serve.Server(precision=prec, threads=16, prep_workers=8, rounds=args.serve_mode == "rounds")
    t0 = time.perf_counter()
    recs = srv.run(reqs, log=lambda m: print(m, file=sys.stderr, flush=True))
    wall = time.perf_counter() - t0
    summ = serve.summarize(recs, wall)
    busy = sum(r.completion - r.start for r in recs)
    out = {
        "metric": "served latency p50 (s)",
        "value": summ["latency_p50_s"],
        "unit": "s",
        "n_gpus": 1,
        "steps": int(sum(r.steps for r in recs)),
        "warmup": 0,
        "ms_per_step": None,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if prec else "f64",
        "data": "synthetic",
        "config": {"workload": "serving_trace", "requests": len(reqs), "arrival_rate_per_s": 20.0,
                   "steps_per_request": 100, "hbm_budget_bytes": srv.budget,
                   "precision": "fp32 inner + fp64 refinement, div_rel <= 1e-8" if prec else "fp64",
                   "serve_mode": ("rounds: all running simulations step together in a fused batch"
                                  if args.serve_mode == "rounds" else "workers: a step worker and stream per simulation")},
        "serving": summ,
        "max_admitted_bytes": srv.max_used,
        "mean_concurrency": busy / wall,
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def run_projection3d(args):
    """The projection step in three dimensions: 256^3 cells around a sphere
    in a closed box, U* seeded on every interior face.  A step resets U* (a
    device-to-device copy) and Phi = 0, then runs one projection (b, the
    Jacobi-PCG to 1e-12, the correction); value = cells projected per
    second.  The roofline entry is the multigrid cycle's finest-level up-sweep
    (the cycle's sweeps are the largest share of the step), timed live with
    HIP events around each of its launches."""
    import torch
    from oracle import geometry3d as G3, pmii3d as P3
    from paper_2211_10698_amd import ccns3d
    import workloads.three_d as T

    torch.cuda.set_device(0)
    case = T.sphere_box_256()
    g = case.grid
    t_setup = time.perf_counter()
    caps = ccns3d.capacities(g, case.bodies)
    precond = {"jacobi": 0, "multigrid": 1, "multigrid-fp32": 2}[args.precond3d]
    ctx = ccns3d.Context3(g, ccns3d.make_params(case.rho, case.tau, tol=case.tol, mass_floor=case.mass_floor,
                                                precond=precond), caps)
    U = [torch.from_numpy(u).cuda() for u in T.face_velocity(case)]
    zero = torch.zeros(g.shape, dtype=torch.float64, device="cuda")
    fields = (ccns3d.F_UX, ccns3d.F_UY, ccns3d.F_UZ)

    def step():
        for f, u in zip(fields, U):
            ctx.set_field(f, u)
        ctx.set_field(ccns3d.F_PHI, zero)
        return ctx.project()

    print(f"[bench] setup {time.perf_counter() - t_setup:.1f}s: {case.name} {g.nx}x{g.ny}x{g.nz}",
          file=sys.stderr, flush=True)
    for k in range(args.warmup):
        info = step()
        print(f"[bench] warmup {k}: cg {info.iterations} div_rel {info.div_rel:.2e}", file=sys.stderr, flush=True)
    ctx.timing(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for k in range(args.steps):
        infos.append(step())
        print(f"[bench] step {k}: cg {infos[-1].iterations} div_rel {infos[-1].div_rel:.2e}", file=sys.stderr,
              flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    (dms, dn), (ums, un), (sms, sn) = ctx.timing(0)
    cells = g.cells
    dir_us = dms * 1e3 / max(dn, 1)
    upd_us = ums * 1e3 / max(un, 1)
    sw_us = sms * 1e3 / max(sn, 1)
    sweep_bytes = SWEEP3_F32_BYTES_PER_CELL if precond == 2 else SWEEP3_BYTES_PER_CELL
    achieved = sweep_bytes * cells / (sw_us * 1e-6) / 1e9
    n_elem = (g.nx + 2 + 15) // 16 * 16 * (g.ny + 2) * (g.nz + 2)
    cpu = None
    if not args.no_cpu_baseline:
        # the oracle's projection (Jacobi-PCG to the same tolerance) on a 40^3
        # sphere box, scaled to cells per second
        sc = T.sphere_box(40)
        t1 = time.perf_counter()
        pr = P3.prepare(G3.capacities(sc.grid, sc.bodies), sc.grid, sc.mass_floor)
        t2 = time.perf_counter()
        _, _, oinfo = P3.project(pr, T.face_velocity(sc), sc.rho, sc.tau, solver="pcg", tol=sc.tol)
        t3 = time.perf_counter()
        cpu = {"value": sc.grid.cells / (t3 - t2) / 1e6, "unit": "Mcell-projections/s", "cores": 1,
               "kind": "oracle",
               "sample": f"one oracle projection of sphere_box(40) (64,000 cells; the oracle's Jacobi-PCG, "
                         f"{oinfo['iterations']} iterations to {sc.tol:g}) in {t3 - t2:.1f} s after {t2 - t1:.1f} s "
                         f"of capacities; the device runs the multigrid-PCG ({infos[-1].iterations} iterations at "
                         f"256^3), so the ratio mixes the two solvers' iteration counts with the hardware"}
    out = {
        "metric": "Mcell-projections/s (3-D projection step, div_rel <= 1e-10)",
        "value": cells * args.steps / wall / 1e6,
        "unit": "Mcell-projections/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32" if precond == 2 else "f64",
        "data": "synthetic",
        "config": {"workload": "sphere_projection_256", "cells": cells, "grid": [g.nx, g.ny, g.nz],
                   "bodies": "sphere r=0.3 in the unit box",
                   "solver": ("Jacobi-PCG", "multigrid-PCG (V-cycle, 2x2x2 agglomeration)",
                              "multigrid-PCG, the cycle's fields in FP32 (FP64 CG)")[precond] + ", tol 1e-12",
                   "mass_floor": case.mass_floor},
        "cg_iterations": [i.iterations for i in infos],
        "div_rel_max": max(i.div_rel for i in infos),
        "kernels_us": {"k3_stencil<DIR>": dir_us, "k3_update": upd_us, "k3_mg_tile<T_POST1> (finest up-sweep)": sw_us,
                       "dir_GBps": DIR3_BYTES_PER_CELL * cells / (dir_us * 1e-6) / 1e9,
                       "update_GBps": (UPDATE3_MG_BYTES_PER_ELEMENT if precond else UPDATE3_BYTES_PER_ELEMENT) *
                       n_elem / (upd_us * 1e-6) / 1e9},
        "roofline": ({"bound": "hbm", "achieved": achieved, "peak": 8000.0, "unit": "GB/s",
                      "frac": achieved / 8000.0, "traffic": stored_traffic3(precond),
                      "kernel": "k3_mg_tile<T_POST1> (the cycle's finest-level up-sweep)",
                      "bytes_per_cell": sweep_bytes, "mean_launch_us": sw_us, "timed_launches": sn}
                     if precond else
                     {"bound": "hbm", "achieved": DIR3_BYTES_PER_CELL * cells / (dir_us * 1e-6) / 1e9,
                      "peak": 8000.0, "unit": "GB/s",
                      "frac": DIR3_BYTES_PER_CELL * cells / (dir_us * 1e-6) / 1e9 / 8000.0, "traffic": None,
                      "kernel": "k3_stencil<DIR>", "bytes_per_cell": DIR3_BYTES_PER_CELL, "mean_launch_us": dir_us,
                      "timed_launches": dn}),
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="naca0012_4096x2048", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"],
                    help="fp64, or mixed: FP32 inner solves with FP64 residuals and refinement to "
                         "div_rel <= 1e-8")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--requests", type=int, default=40, help="serving_trace: requests served")
    ap.add_argument("--serving-unresolved", action="store_true",
                    help="serving_trace: run the line although its last two runs went silent (see the design notes)")
    ap.add_argument("--serve-mode", default="workers", choices=["workers", "rounds"],
                    help="serving_trace: a step worker per simulation, or fused rounds of all running ones")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run the plain copies that calibrate the HBM byte counters")
    ap.add_argument("--summarize-counters", metavar="DIR",
                    help="store the HBM traffic of the predictor kernel from rocprofv3 counter runs under DIR")
    ap.add_argument("--mass-floor", type=float, default=None,
                    help="small-volume floor theta (default: the workload's, 0.05); 0 is the paper's mass "
                         "matrix M = diag(V)")
    ap.add_argument("--mg-forms", default="tuned", choices=["tuned", "default"],
                    help="multigrid cycle kernel forms: the tuned ones cached for this GPU's level sizes "
                         "(paper_2211_10698_amd/mg_forms.json), or the library's defaults")
    ap.add_argument("--batch-mode", default="fused", choices=["fused", "streams"],
                    help="batched_cylinders_256: one launch per phase over all simulations (fused) "
                         "or 16 host threads with a stream per simulation")
    ap.add_argument("--batch-graphs", default="on", choices=["on", "off"],
                    help="batched_cylinders_256, fused: replay each CG iteration from a captured HIP graph")
    ap.add_argument("--coef-tables", default="auto", choices=["auto", "off"],
                    help="auto: the predictor CG reads its coefficients through the class table when it "
                         "fits (the library's default); off: from the coefficient arrays")
    ap.add_argument("--precond3d", default="multigrid", choices=["multigrid", "multigrid-fp32", "jacobi"],
                    help="sphere_projection_256: the Poisson CG's preconditioner (multigrid-fp32: the cycle's "
                         "fields in FP32, the CG in FP64)")
    args = ap.parse_args()
    if args.summarize_counters and args.workload == "sphere_projection_256":
        pc = {"jacobi": 0, "multigrid": 1, "multigrid-fp32": 2}[args.precond3d]
        if not pc:
            raise SystemExit("the 3-D counter summary covers the multigrid cycle's up-sweep")
        summarize_counters(args.summarize_counters, SWEEP3_KERNEL[pc], args.workload, False, key=traffic3_key(pc),
                           digest=file_digest(SRC3, KERNEL_HDR))
        return
    if args.summarize_counters:
        summarize_counters(args.summarize_counters, "k_pred_cg", args.workload, args.coef_tables == "auto")
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(independent simulations shard across GPUs without communication).", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.workload == "batched_cylinders_256":
        run_batched(args)
        return
    if args.workload == "serving_trace":
        run_serving(args)
        return
    if args.workload == "sphere_projection_256":
        run_projection3d(args)
        return
    from paper_2211_10698_amd import ccns

    case = WORKLOADS[args.workload]()
    if args.mass_floor is not None:
        case.mass_floor = args.mass_floor
    g = case.grid
    t_setup = time.perf_counter()
    caps = ccns.ccns_capacities(g, case.bodies)
    Dx, Dy = W.dirichlet(case)
    mixed = args.precision == "mixed"
    params = ccns.make_params(case.rho, case.mu, case.tau, u_ref=case.u_inf, pcg_tol=case.pcg_tol,
                              pred_tol=1e-12, precision=1 if mixed else 0, div_tol=1e-8,
                              mass_floor=case.mass_floor, coef_tables=0 if args.coef_tables == "auto" else 1,
                              outflow=case.outflow)
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    ctx = ccns.Context(g, params, caps, Dx, Dy, stream=stream)
    au, av = unknown_masks(caps, g.nx, g.ny)
    px, py = W.perturbation(case)
    ctx.set_field(ccns.F_UX, np.where(au, case.u_inf + px, Dx))
    ctx.set_field(ccns.F_UY, np.where(av, py, Dy))
    ctx.project()
    ncls = ctx.coef_classes()
    forms = tune.apply_cached(ctx, 1 if mixed else 0) if args.mg_forms == "tuned" else 0
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
    # mean duration per timed kernel (None: no launch of it was sampled, e.g. the
    # short inner pressure solves of the mixed mode stop before iteration 4)
    mean_us = [ms[k] / cnt[k] * 1e3 if cnt[k] > 0 else None for k in range(4)]

    def rate(bytes_per_cell, us):
        return esz * bytes_per_cell * cells / (us * 1e-6) / 1e9 if us else None

    # the timed kernels run in float in the inner solves of the mixed mode
    esz = 0.5 if mixed else 1.0
    kname = "k_pred_cg<float>" if mixed else "k_pred_cg"
    # algorithmic bytes of a predictor CG iteration: the scope's figure for
    # the method (the roofline's `achieved`), and what this kernel moves (the
    # coefficient class table replaces twelve coefficient values per cell by
    # one 4-byte index)
    scope_bytes = esz * PRED_CG_SCOPE_BYTES_PER_CELL
    if ncls:
        pred_bytes = esz * 8.0 * PRED_CG_VALUES_PER_CELL_CLS + PRED_CG_INDEX_BYTES
    else:
        pred_bytes = esz * 8.0 * PRED_CG_VALUES_PER_CELL
    us = mean_us[2]
    achieved = scope_bytes * cells / (us * 1e-6) / 1e9 if us else None
    moved = pred_bytes * cells / (us * 1e-6) / 1e9 if us else None
    traffic = None if mixed else stored_traffic("k_pred_cg", case.name, ncls > 0)
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
        "dtype": "f32+f64" if mixed else "f64",
        "data": "synthetic",
        "config": {"workload": case.name, "nx": g.nx, "ny": g.ny, "re": case.re, "cfl": case.cfl,
                   "pcg_tol": case.pcg_tol, "pred_tol": 1e-12, "precond": "multigrid",
                   "precision": "fp32 inner + fp64 refinement, div_rel <= 1e-8" if mixed else "fp64",
                   "coef_classes": ncls, "mass_floor": case.mass_floor,
                   "mg_forms": {"word": forms, "levels": ctx.mg_levels()}},
        "div_rel_max": div_max,
        "cg_iters_per_step": n_cg,
        "pred_iters_per_step": float(np.mean([i["pred_iters"] for i in infos])),
        "roofline": {
            "kernel": kname,
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS if achieved else None,
            "traffic": traffic,
            "bytes_per_cell": scope_bytes,
            "bytes_per_launch": scope_bytes * cells,
            "kernel_bytes_per_cell": pred_bytes,
            "kernel_bytes_per_launch": pred_bytes * cells,
            "achieved_kernel_bytes": moved,
            "frac_kernel_bytes": moved / HBM_PEAK_GBS if moved else None,
            "traffic_rate": traffic / (us * 1e-6) / 1e9 if (traffic and us) else None,
            "coef_classes": bool(ncls),
            "mean_launch_us": us,
            "timed_launches": cnt[2],
        },
        "kernels": {
            kname: {"us": mean_us[2], "GBs": moved},
            "k_reduce_partials<7>": {"us": mean_us[3]},
            "k_pois_dir_z": {"us": mean_us[0], "GBs": rate(POIS_DIR_BYTES_PER_CELL, mean_us[0])},
            "k_cg_update (Poisson)": {"us": mean_us[1], "GBs": rate(POIS_UPDATE_BYTES_PER_CELL, mean_us[1])},
        },
        "cpu_baseline": None,
    }
    if div_max > 1e-8:
        out["warning"] = "divergence above 1e-8 in a timed step"
    if case.bodies:
        # drag and lift of the final state (after the timed region)
        F = ctx.forces()
        q = 0.5 * case.rho * case.u_inf ** 2 * case.ref_length
        out["forces"] = {"cd": (F[0] + F[2]) / q, "cl": (F[1] + F[3]) / q, "pressure_x": F[0], "pressure_y": F[1],
                         "viscous_x": F[2], "viscous_y": F[3], "time": case.tau * (args.warmup + args.steps)}
    if not args.no_cpu_baseline:
        # the oracle solves both systems with Jacobi-PCG: count the iterations
        # that algorithm needs in one step of this workload (an FP64 Jacobi
        # context of the library stepped once from the current state: same
        # algorithm as the oracle), to scale the oracle's timed sample
        pj = ccns.make_params(case.rho, case.mu, case.tau, u_ref=case.u_inf, pcg_tol=case.pcg_tol,
                              pred_tol=1e-12, precond=ccns.PRECOND_JACOBI, mass_floor=case.mass_floor,
                              outflow=case.outflow)
        cj = ccns.Context(g, pj, caps, Dx, Dy, stream=stream)
        for f in (ccns.F_UX, ccns.F_UY, ccns.F_P, ccns.F_PHI, ccns.F_CONVX, ccns.F_CONVY):
            cj.set_field(f, ctx.get_field(f))
        jinfo = cj.step(1, check=False)
        n_pred, n_jac = jinfo.pred.iterations, jinfo.poisson.iterations
        cj.close()
        print(f"[bench] cpu baseline (oracle): Jacobi-PCG iterations per step {n_pred} predictor, {n_jac} "
              f"pressure ...", file=sys.stderr, flush=True)
        cb = cpu_baseline(case, caps, n_pred, n_jac)
        out["cpu_baseline"] = {k: cb[k] for k in ("value", "unit", "cores", "kind", "sample", "extrapolated",
                                                  "host_cpu", "host_logical_cores", "threads")}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
