"""Serving loop: many independent simulation requests on one GPU.

A request is a simulation case (grid, bodies, Reynolds number, step count)
with an arrival time.  The server

  * admits requests in arrival order (first come, first served) while their
    device footprint (ccns_workspace_bytes plus field buffers) fits in an HBM
    budget; a request that does not fit waits at the head of the queue;
  * prepares each admitted request on a preparation worker, overlapping the
    GPU work of the running batch: the capacities (on the device, in closed
    form, when every body is a circle or an ellipse; else from the level set
    on the host), the seeded inputs, a context on a stream of its own and the
    initial projection;
  * runs every prepared simulation on a step worker of its own (continuous
    batching without rounds: a simulation joins the GPU as soon as it is
    prepared, shares it with the others, each on its own stream, and leaves
    as soon as its last step is done, releasing its budget); or, with
    rounds=True, batches the time steps of every prepared simulation: each
    round advances all of them by one step in a fused batch (one launch per
    phase over all of their work-groups), a simulation prepared during a
    round joins at the next one, and one whose last step is done leaves,
    releasing its budget.

Latency = completion - arrival, split into queue time (arrival to admission)
and service time (admission to completion, which includes preparation).
Every simulation's result is independent of the others that share the
batch: the kernels reduce in a fixed order, so a request served in a mix
returns the same fields, bit for bit, as served alone.

This module is orchestration only; all numerical work runs in libccns.
"""

from __future__ import annotations

import collections
import concurrent.futures as cf
import dataclasses
import time
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import ccns


@dataclasses.dataclass
class Record:
    """Timeline and figures of one served request (times in seconds from the
    start of the run)."""

    index: int
    name: str
    cells: int
    steps: int
    bytes: int
    arrival: float
    admit: float = float("nan")
    prepared: float = float("nan")
    caps_s: float = float("nan")
    start: float = float("nan")
    completion: float = float("nan")
    div_rel_max: float = 0.0
    # drag and lift coefficients of the final state (ccns_forces)
    cd: float = float("nan")
    cl: float = float("nan")
    status: int = ccns.OK
    note: str = ""
    fields: Optional[Dict[str, np.ndarray]] = None

    @property
    def latency(self):
        return self.completion - self.arrival

    @property
    def queue(self):
        return self.admit - self.arrival

    @property
    def service(self):
        return self.completion - self.admit

    @property
    def preparation(self):
        return self.prepared - self.admit


def _seeded_inputs(case):
    """The synthetic requests' inputs: free-stream Dirichlet data with
    no-slip near the bodies, and the seeded divergence-free perturbation."""
    import workloads as W

    Dx, Dy = W.dirichlet(case)
    px, py = W.perturbation(case)
    return Dx, Dy, px, py


def footprint(case, params) -> int:
    """Device bytes one simulation holds while it is served: the workspace
    plus the dense field buffers used while its inputs are uploaded, or the
    capacity arrays and their scratch while the capacities are computed on
    the device (21 + 6 arrays), whichever is more."""
    import ctypes as C

    L = ccns.lib()
    g = ccns.make_grid(case.grid)
    ws = L.ccns_workspace_bytes(C.byref(g), C.byref(params))
    n = (case.grid.nx + 2) * (case.grid.ny + 2)
    return int(ws + 256 + max(8, ccns.NCAPS + 6) * n * 8)


def default_budget(fraction=0.85) -> int:
    """A fraction of the device memory that is free now."""
    import torch

    free, total = torch.cuda.mem_get_info()
    return int(fraction * free)


class Server:
    """Continuous-batching server for simulation requests on one GPU."""

    def __init__(self, hbm_budget: Optional[int] = None, precision: int = 1, threads: int = 16,
                 prep_workers: int = 4, keep_fields: bool = False, inputs=None, device_caps: bool = True,
                 forces: bool = False, rounds: bool = False):
        self.budget = hbm_budget if hbm_budget is not None else default_budget()
        # rounds: every running simulation steps in one fused batch per round
        self.rounds = rounds
        self.precision = precision
        self.threads = threads
        self.prep_workers = prep_workers
        self.keep_fields = keep_fields
        self.device_caps = device_caps
        # drag and lift of each request's final state (off by default: the
        # served trace has not been run with it)
        self.forces = forces
        # inputs(case) -> (Dx, Dy, ux_perturbation, uy_perturbation)
        self.inputs = inputs if inputs is not None else _seeded_inputs
        self.max_used = 0      # largest admitted footprint total seen by the last run
        # a multigrid-preconditioned pressure solve needs tens of iterations;
        # a request whose solve fails is stopped (status and note recorded)
        self.pcg_maxit = 2000

    def _params(self, case):
        return ccns.make_params(case.rho, case.mu, case.tau, u_ref=case.u_inf, pcg_tol=case.pcg_tol,
                                pred_tol=1e-12, precision=self.precision, div_tol=1e-8,
                                mass_floor=case.mass_floor, pcg_maxit=self.pcg_maxit, pred_maxit=500)

    def _prepare(self, case):
        """Preparation worker: capacities (closed form on the device for
        circles and ellipses, else the host quadrature), the request's seeded
        inputs, a context on a fresh stream, the initial field and the initial
        projection.  Returns (context, stream, projection info, seconds spent
        on the capacities)."""
        import torch

        g = case.grid
        stream = torch.cuda.Stream()
        t0 = time.perf_counter()
        if self.device_caps and case.bodies and all(b.kind in (ccns.CIRCLE, ccns.ELLIPSE) for b in case.bodies):
            with torch.cuda.stream(stream):
                caps = ccns.ccns_capacities_device(g, case.bodies, stream).cpu().numpy()
        else:
            caps = ccns.ccns_capacities(g, case.bodies)
        t_caps = time.perf_counter() - t0
        Dx, Dy, px, py = self.inputs(case)
        sh = (g.ny + 2, g.nx + 2)
        J, I = np.indices(sh)
        au = (I >= 1) & (I <= g.nx - 1) & (J >= 1) & (J <= g.ny) & (caps[7] > 0) & (caps[1] > 0)
        av = (I >= 1) & (I <= g.nx) & (J >= 1) & (J <= g.ny - 1) & (caps[14] > 0) & (caps[2] > 0)
        ctx = ccns.Context(g, self._params(case), caps, Dx, Dy, stream=stream)
        ctx.set_field(ccns.F_UX, np.where(au, case.u_inf + px, Dx))
        ctx.set_field(ccns.F_UY, np.where(av, py, Dy))
        info = ctx.project()
        return ctx, stream, info, t_caps

    @staticmethod
    def _run_steps(ctx, case, clock, forces=False):
        """Step worker: advances one simulation through all its steps (the GPU
        is shared with the other running simulations, each on its own
        stream), stopping at the first failed solve, then takes the drag and
        lift coefficients of the final state.  Returns (start, completion,
        div_rel_max, status, note, (cd, cl))."""
        steps = case.steps
        start = clock()
        div, status, note = 0.0, ccns.OK, ""
        for n in range(steps):
            info = ctx.step(1, check=False)
            div = max(div, info.div_rel)
            status, note = Server._check(info, n, status, note)
            if status != ccns.OK:
                break
        end = clock()
        return start, end, div, status, note, Server._coefficients(ctx, case, forces)

    @staticmethod
    def _check(info, n, status, note):
        """The first failed solve of step n (status and note), if any."""
        for name, si in (("predictor", info.pred), ("pressure", info.poisson)):
            if si.status != ccns.OK and status == ccns.OK:
                status = si.status
                note = (f"step {n}: {name} solve status {si.status} after {si.iterations} iterations, "
                        f"{si.outer} sweeps, relative residual {si.rel_residual:.2e}, inner status "
                        f"{si.inner_status} (first at sweep {si.inner_fail_sweep})")
        return status, note

    @staticmethod
    def _coefficients(ctx, case, forces):
        """(C_d, C_l) of the final state when asked for, else NaNs."""
        coef = (float("nan"), float("nan"))
        if forces and case.bodies:
            try:
                F = ctx.forces()
                q = 0.5 * case.rho * case.u_inf ** 2 * case.ref_length
                coef = ((F[0] + F[2]) / q, (F[1] + F[3]) / q)
            except ccns.CcnsError:
                pass
        return coef

    def run(self, requests: Sequence, log=None) -> List[Record]:
        """Serves the requests (objects with .case and .arrival, arrival in
        seconds from the start) in real time; returns one Record each.

        Every running simulation is driven by a step worker of its own (at
        most `threads` at a time), so a simulation joins the GPU as soon as it
        is prepared and leaves as soon as its last step is done: no
        simulation waits for another's step.  With rounds=True this thread
        steps all running simulations together, one fused batch step per
        round, while the preparation workers keep preparing."""
        order = sorted(range(len(requests)), key=lambda k: requests[k].arrival)
        recs = []
        for k in order:
            c = requests[k].case
            recs.append(Record(k, c.name, c.grid.nx * c.grid.ny, c.steps, footprint(c, self._params(c)),
                               requests[k].arrival))
        for r in recs:
            if r.bytes > self.budget:
                raise ValueError(f"request {r.name} needs {r.bytes} bytes, more than the budget {self.budget}")
        cases = {r.index: requests[r.index].case for r in recs}
        self.max_used = 0
        queue = collections.deque()
        free = self.budget
        nxt = 0
        preparing = {}       # host-preparation future -> record
        running = {}         # step future -> (record, context)
        members = []         # rounds: [record, context, steps done] of every running simulation
        batch, batch_key = None, None
        done = 0
        t0 = time.perf_counter()
        clock = lambda: time.perf_counter() - t0  # noqa: E731
        prep_pool = cf.ThreadPoolExecutor(max_workers=self.prep_workers)
        step_pool = cf.ThreadPoolExecutor(max_workers=self.threads)
        try:
            while done < len(recs):
                now = clock()
                while nxt < len(recs) and recs[nxt].arrival <= now:
                    queue.append(recs[nxt])
                    nxt += 1
                while queue and queue[0].bytes <= free:
                    r = queue.popleft()
                    free -= r.bytes
                    self.max_used = max(self.max_used, self.budget - free)
                    r.admit = clock()
                    preparing[prep_pool.submit(self._prepare, cases[r.index])] = r
                finished = []
                for fut in [f for f in preparing if f.done()]:
                    r = preparing.pop(fut)
                    ctx, stream, info, r.caps_s = fut.result()
                    r.prepared = clock()
                    r.div_rel_max = info.div_rel
                    if self.rounds:
                        r.start = r.prepared
                        members.append([r, ctx, 0])
                    else:
                        running[step_pool.submit(self._run_steps, ctx, cases[r.index], clock, self.forces)] = (r, ctx)
                for fut in [f for f in running if f.done()]:
                    r, ctx = running.pop(fut)
                    r.start, r.completion, div, r.status, r.note, (r.cd, r.cl) = fut.result()
                    r.div_rel_max = max(r.div_rel_max, div)
                    finished.append((r, ctx))
                if self.rounds and members:
                    # one round: every running simulation advances one step
                    key = tuple(id(m[1]) for m in members)
                    if batch is None or key != batch_key:
                        if batch is not None:
                            batch.close()
                        batch, batch_key = ccns.Batch([m[1] for m in members], fused=True), key
                    _, infos, _ = batch.step(1, check=False)
                    stay = []
                    for m, info in zip(members, infos):
                        r, ctx, n = m
                        r.div_rel_max = max(r.div_rel_max, info.div_rel)
                        r.status, r.note = self._check(info, n, r.status, r.note)
                        m[2] = n + 1
                        if m[2] >= cases[r.index].steps or r.status != ccns.OK:
                            r.completion = clock()
                            r.cd, r.cl = self._coefficients(ctx, cases[r.index], self.forces)
                            finished.append((r, ctx))
                        else:
                            stay.append(m)
                    if len(stay) != len(members):
                        batch.close()
                        batch, batch_key = None, None
                    members = stay
                for r, ctx in finished:
                    if self.keep_fields:
                        r.fields = {n: ctx.get_field(f).cpu().numpy()
                                    for n, f in (("ux", ccns.F_UX), ("uy", ccns.F_UY), ("p", ccns.F_P))}
                    ctx.close()
                    free += r.bytes
                    done += 1
                    if log:
                        log(f"[serve] {r.name} done: latency {r.latency:.2f}s "
                            f"(queue {r.queue:.2f}s, service {r.service:.2f}s){' ' + r.note if r.note else ''}")
                if self.rounds and members:
                    continue
                waits = list(preparing) + list(running)
                timeout = 0.005
                if nxt < len(recs):
                    timeout = max(0.0, min(timeout, recs[nxt].arrival - clock()))
                if waits:
                    cf.wait(waits, timeout=timeout, return_when=cf.FIRST_COMPLETED)
                else:
                    time.sleep(timeout)
        finally:
            if batch is not None:
                batch.close()
            step_pool.shutdown(wait=True)
            prep_pool.shutdown(wait=True)
        return sorted(recs, key=lambda r: r.index)


def summarize(recs: Sequence[Record], wall: float) -> dict:
    """p50/p99 latency, queue and service times, and throughput."""
    lat = np.array([r.latency for r in recs])
    que = np.array([r.queue for r in recs])
    svc = np.array([r.service for r in recs])
    cell_steps = sum(r.cells * r.steps for r in recs)
    return {
        "requests": len(recs),
        "latency_p50_s": float(np.percentile(lat, 50)),
        "latency_p99_s": float(np.percentile(lat, 99)),
        "queue_p50_s": float(np.percentile(que, 50)),
        "queue_p99_s": float(np.percentile(que, 99)),
        "service_p50_s": float(np.percentile(svc, 50)),
        "service_p99_s": float(np.percentile(svc, 99)),
        "preparation_p50_s": float(np.percentile([r.preparation for r in recs], 50)),
        "preparation_p99_s": float(np.percentile([r.preparation for r in recs], 99)),
        "capacities_p50_s": float(np.percentile([r.caps_s for r in recs], 50)),
        "throughput_mcell_steps_s": cell_steps / wall / 1e6,
        "wall_s": wall,
        "div_rel_max": float(max(r.div_rel_max for r in recs)),
        "statuses": sorted({int(r.status) for r in recs}),
        "drag_coefficient_range": [float(np.nanmin([r.cd for r in recs])), float(np.nanmax([r.cd for r in recs]))]
        if any(np.isfinite(r.cd) for r in recs) else None,
    }
