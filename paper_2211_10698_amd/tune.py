"""Tuning of the multigrid cycle's kernel forms, per level and precision.

Each cycle level runs a down-sweep kernel (two smoothing sweeps, the
residual and its restriction) and an up-sweep kernel (the interpolated
correction and two sweeps) in one of five forms (ccns_params.mg_forms):

  1  staged first sweep, the tile ring's operands in registers, 64 x 16 tiles
  2  the same with every operand of the ring in LDS (64 KB per work-group in
     FP64: fewer loads, two work-groups per compute unit)
  3  first sweep formed pointwise at the second sweep's stencil, 64 x 16 tiles
  4  the same on 64 x 4 tiles (more work-groups on small levels)
  5  form 2 on 64 x 8 tiles (about 38 KB of LDS: four work-groups per unit)

Forms 4 and 5 are not used for the finest level's up-sweep, whose tiles fix
the order of the preconditioner's statistics.

All of them compute the same values bit for bit; which is fastest depends on
the level's size and the precision.  `tune` times pressure solves on a
context with each form in turn, level by level, and keeps the fastest;
`mg_forms.json` beside this module caches the choices per device, precision
and level size, and `apply_cached` gives a new context the cached forms of
its levels (the library's defaults elsewhere).

    python -m paper_2211_10698_amd.tune --grids 4096x2048,2048x1024 --out FILE
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time
from typing import Dict, List, Optional, Sequence, Tuple

from . import ccns

FORMS = {
    1: "staged, ring operands in registers, 64x16 tiles",
    2: "staged, ring operands in LDS, 64x16 tiles",
    3: "pointwise first sweep, 64x16 tiles",
    4: "pointwise first sweep, 64x4 tiles",
    5: "staged, ring operands in LDS, 64x8 tiles",
}
CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "mg_forms.json")


def pack(pairs: Sequence[Tuple[int, int]]) -> int:
    """The mg_forms word of per-level (down, up) forms (0: the default)."""
    v = 0
    for level, (down, up) in enumerate(pairs):
        if not (0 <= down <= 5 and 0 <= up <= 5) or level >= 10 or (level == 0 and up in (4, 5)):
            raise ValueError(f"level {level}: forms ({down}, {up})")
        v |= (down << (6 * level)) | (up << (6 * level + 3))
    return v


def unpack(word: int, levels: int) -> List[Tuple[int, int]]:
    return [((word >> (6 * k)) & 7, (word >> (6 * k + 3)) & 7) for k in range(levels)]


def precision_key(precision: int) -> str:
    # the cycle runs in FP64 in precision 0 and in float inside the
    # refinement of precision 1
    return "f32" if precision == 1 else "f64"


def device_key() -> str:
    """The device's architecture (its gfx name): marketing names depend on
    how the runtime finds them (a profiler can change them)."""
    import torch

    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    arch = getattr(p, "gcnArchName", "") or torch.cuda.get_device_name(torch.cuda.current_device())
    return arch.split(":")[0]


def load_cache(path: str = CACHE) -> Dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def lookup(levels: Sequence[Tuple[int, int]], precision: int, device: str, cache: Optional[Dict] = None) -> int:
    """The cached forms of these level sizes ((nx, ny) per level), 0 where
    none is cached.  A size tuned as a coarse level may be a grid's finest
    one, whose up-sweep cannot take forms 4 and 5: it keeps the default."""
    cache = load_cache() if cache is None else cache
    table = cache.get(device, {}).get(precision_key(precision), {})
    pairs = []
    for level, (nx, ny) in enumerate(levels):
        down, up = table.get(f"{nx}x{ny}", (0, 0))
        if level == 0 and up in (4, 5):
            up = 0
        pairs.append((down, up))
    return pack(pairs)


def apply_cached(ctx, precision: int, cache: Optional[Dict] = None) -> int:
    """Gives `ctx` the cached forms of its cycle levels; returns the word."""
    levels = [(nx, ny) for nx, ny, _, _ in ctx.mg_levels()]
    if not levels:
        return 0
    word = lookup(levels, precision, device_key(), cache)
    if word:
        ctx.set_mg_forms(word)
    return word


def tune(ctx, b, reps: int = 3, log=None) -> Dict:
    """Times pressure solves of b from Phi = 0 on `ctx` (every form gives the
    same iterates, so only the kernels' speed differs) and picks, level by
    level and for the down- and up-sweep in turn, the fastest form with the
    others at their best so far.  Returns the levels, the chosen forms and
    the solve times."""
    import torch

    levels = [(nx, ny) for nx, ny, _, _ in ctx.mg_levels()]
    best = [(0, 0)] * len(levels)
    zero = torch.zeros_like(b)

    def timed(pairs):
        ctx.set_mg_forms(pack(pairs))
        ts = []
        for r in range(reps + 1):
            ctx.set_field(ccns.F_PHI, zero)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.pressure_solve(b)
            ts.append(time.perf_counter() - t0)
        return min(ts[1:])

    t_default = timed(best)
    trials = []
    for lv in range(len(levels)):
        for half in (0, 1):
            res = {}
            for f in FORMS:
                if lv == 0 and half == 1 and f in (4, 5):
                    continue
                pairs = list(best)
                pair = list(pairs[lv])
                pair[half] = f
                pairs[lv] = tuple(pair)
                res[f] = timed(pairs)
            f_best = min(res, key=res.get)
            pair = list(best[lv])
            pair[half] = f_best
            best[lv] = tuple(pair)
            trials.append({"level": lv, "size": levels[lv], "sweep": "down" if half == 0 else "up",
                           "ms": {FORMS[f]: res[f] * 1e3 for f in res}})
            if log:
                log(f"[tune] level {lv} {levels[lv][0]}x{levels[lv][1]} {'down' if half == 0 else 'up'}: "
                    + ", ".join(f"{f}: {res[f] * 1e3:.3f} ms" for f in res))
    t_best = timed(best)
    ctx.set_mg_forms(pack(best))
    return {"levels": levels, "forms": best, "solve_ms_default": t_default * 1e3, "solve_ms_tuned": t_best * 1e3,
            "trials": trials}


def merge(cache: Dict, device: str, precision: int, result: Dict) -> Dict:
    table = cache.setdefault(device, {}).setdefault(precision_key(precision), {})
    for (nx, ny), (d, u) in zip(result["levels"], result["forms"]):
        table[f"{nx}x{ny}"] = [int(d), int(u)]
    return cache


def _context_for(nx: int, ny: int, precision: int):
    """A channel of nx x ny cells around a circle (the benchmarks' body
    family), stepped once: its last pressure right-hand side is the system
    the tuner solves."""
    import numpy as np
    import torch

    import workloads as W

    h = 1.0 / 256
    g = W.GridSpec(nx, ny, 0.0, 0.0, nx * h, ny * h)
    r = 0.1 * min(nx, ny) * h
    case = W.Case(f"tune_{nx}x{ny}", g, [W.Body(W.CIRCLE, 0.3 * nx * h, 0.5 * ny * h, a=r)], re=100.0,
                  noise=1e-3, seed=9)
    caps = ccns.ccns_capacities_device(g, case.bodies).cpu().numpy()
    Dx, Dy = W.dirichlet(case)
    px, py = W.perturbation(case)
    prm = ccns.make_params(case.rho, case.mu, case.tau, u_ref=case.u_inf, pcg_tol=1e-10, precision=precision,
                           mass_floor=case.mass_floor)
    ctx = ccns.Context(g, prm, caps, Dx, Dy)
    sh = (ny + 2, nx + 2)
    J, I = np.indices(sh)
    au = (I >= 1) & (I <= nx - 1) & (J >= 1) & (J <= ny) & (caps[7] > 0) & (caps[1] > 0)
    av = (I >= 1) & (I <= nx) & (J >= 1) & (J <= ny - 1) & (caps[14] > 0) & (caps[2] > 0)
    ctx.set_field(ccns.F_UX, np.where(au, case.u_inf + px, Dx))
    ctx.set_field(ccns.F_UY, np.where(av, py, Dy))
    ctx.project()
    ctx.step(1)
    b = ctx.get_field(ccns.F_B).clone()
    torch.cuda.synchronize()
    return ctx, b


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--grids", default="4096x2048,2048x1024,2048x2048,1024x1024,512x512")
    ap.add_argument("--precision", default="both", choices=["fp64", "mixed", "both"])
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--out", default=None, help="cache file to merge into (default: print only)")
    args = ap.parse_args(argv)
    import torch

    torch.cuda.set_device(0)
    dev = device_key()
    cache = load_cache(args.out) if args.out else {}
    precs = {"fp64": [0], "mixed": [1], "both": [0, 1]}[args.precision]
    for spec in args.grids.split(","):
        nx, ny = (int(v) for v in spec.split("x"))
        for p in precs:
            print(f"[tune] {nx}x{ny} {precision_key(p)}: set-up", file=sys.stderr, flush=True)
            ctx, b = _context_for(nx, ny, p)
            res = tune(ctx, b, args.reps, log=lambda m: print(m, file=sys.stderr, flush=True))
            print(json.dumps({"grid": spec, "precision": precision_key(p), "forms": res["forms"],
                              "levels": res["levels"], "solve_ms_default": res["solve_ms_default"],
                              "solve_ms_tuned": res["solve_ms_tuned"]}), flush=True)
            merge(cache, dev, p, res)
            ctx.close()
            if args.out:
                with open(args.out, "w") as f:
                    json.dump(cache, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
