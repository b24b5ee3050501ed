"""CPU-side checks of the device library: it loads, exports every function
declared in include/ccns.h, validates arguments, and its host capacity code
agrees with the oracle's independent integration."""

import os
import re

import numpy as np
import pytest

import workloads as W
from oracle import geometry

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            names |= set(re.findall(r"\b(ccns3?_[a-z_]+)\s*\(", txt))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    from paper_2211_10698_amd import ccns
    L = ccns.lib()
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n
    assert set(ccns.EXPORTED) <= set(names)
    from paper_2211_10698_amd import ccns3d
    assert set(ccns3d.EXPORTED) <= set(names) and all(hasattr(ccns3d.lib(), n) for n in ccns3d.EXPORTED)


def test_argument_validation_without_gpu():
    import ctypes as C
    from paper_2211_10698_amd import ccns
    L = ccns.lib()
    bad = ccns.Grid(1, 1, 0.0, 0.0, 1.0, 1.0)
    assert L.ccns_workspace_bytes(C.byref(bad), None) == 0
    g = ccns.Grid(8, 8, 0.0, 0.0, 0.125, 0.125)
    out = np.zeros(L.ccns_caps_count(C.byref(g)))
    b = ccns.make_bodies([W.Body(W.CIRCLE, 0.5, 0.5, a=-1.0)])
    st = L.ccns_capacities(C.byref(g), b, 1, ccns.LEVELSET_FN(), None, out.ctypes.data)
    assert st == ccns.EINVAL
    h = C.c_void_p()
    p = ccns.make_params(1.0, 0.01, 0.01)
    assert L.ccns_ctx_create(C.byref(g), C.byref(p), None, None, None, 0, None, C.byref(h)) == ccns.EINVAL
    # precision 1 needs the float arrays on top of the FP64 workspace
    p1 = ccns.make_params(1.0, 0.01, 0.01, precision=1)
    assert L.ccns_workspace_bytes(C.byref(g), C.byref(p1)) > L.ccns_workspace_bytes(C.byref(g), C.byref(p))
    # unknown precision, preconditioner or coefficient path: rejected before any device work
    caps = np.zeros(L.ccns_caps_count(C.byref(g)))
    dir2 = np.zeros(2 * 10 * 10)
    for bad_p in (ccns.make_params(1.0, 0.01, 0.01, precision=2), ccns.make_params(1.0, 0.01, 0.01, precond=5),
                  ccns.make_params(1.0, 0.01, 0.01, coef_tables=2), ccns.make_params(1.0, 0.01, 0.01, outflow=16),
                  ccns.make_params(1.0, 0.01, 0.01, mg_forms=6), ccns.make_params(1.0, 0.01, 0.01, mg_forms=1 << 60),
                  ccns.make_params(1.0, 0.01, 0.01, mg_forms=4 << 3)):
        assert L.ccns_ctx_create(C.byref(g), C.byref(bad_p), caps.ctypes.data, dir2.ctypes.data,
                                 C.c_void_p(256), 1 << 30, None, C.byref(h)) == ccns.EINVAL
    # batches: empty, NULL member, repeated member (checked before any member is read)
    bh = C.c_void_p()
    fake = (C.c_void_p * 2)(4096, 4096)
    assert L.ccns_batch_create(0, fake, 0, C.byref(bh)) == ccns.EINVAL
    assert L.ccns_batch_create(2, (C.c_void_p * 2)(4096, None), 0, C.byref(bh)) == ccns.EINVAL
    assert L.ccns_batch_create(2, fake, 0, C.byref(bh)) == ccns.EINVAL
    assert L.ccns_batch_create(1, fake, -1, C.byref(bh)) == ccns.EINVAL
    assert L.ccns_batch_step(None, 1, None, None) == ccns.EINVAL


@pytest.mark.parametrize("name", ["cylinder_64", "offcentre_40", "channel_cylinder_2048x1024"])
def test_library_capacities_match_oracle(name):
    from paper_2211_10698_amd import ccns
    if name == "cylinder_64":
        case = W.cylinder_64()
        g, bodies = case.grid, case.bodies
    elif name == "channel_cylinder_2048x1024":
        case = W.channel_cylinder_2048()     # the benchmark's full size
        g, bodies = case.grid, case.bodies
    else:
        g = W.GridSpec(40, 36, -0.1, 0.05, 1.2, 1.08)
        bodies = [W.Body(W.CIRCLE, 0.4711, 0.5302, a=0.2113)]
    a = ccns.ccns_capacities(g, bodies)
    b = geometry.capacities(g, bodies)
    h = max(g.hx, g.hy)
    for k, n in enumerate(ccns.CAP_NAMES):
        # first-kind capacities agree to rounding; second-kind ones are
        # measured on lines/strips placed at centroids, whose rounding they
        # amplify near tangencies and in slivers
        scale = h * h if n[0] in "VW" else h
        tol = 1e-11 if n[0] in "VA" else (1e-8 if n[0] == "W" else 1e-6)
        assert np.max(np.abs(a[k] - b[n])) <= tol * scale, n


@pytest.mark.slow
def test_library_capacities_match_oracle_ellipse_and_naca():
    """Generic level sets (no closed form on either side)."""
    from paper_2211_10698_amd import ccns
    # coarse grids: the oracle's generic quadrature is pure Python (about a
    # minute for both); every cell of the body's outline is still cut
    for g, body in ((W.GridSpec(7, 6, 0.0, 0.0, 1.0, 0.857), W.Body(W.ELLIPSE, 0.52, 0.41, a=0.27, b=0.13, angle=0.6)),
                    (W.GridSpec(12, 4, 1.8, 1.8, 1.5, 0.5), W.Body(W.NACA4, 2.0, 2.0, angle=0.087, chord=1.0, t=0.12))):
        a = ccns.ccns_capacities(g, [body])
        b = geometry.capacities(g, [body])
        h = max(g.hx, g.hy)
        for k, n in enumerate(ccns.CAP_NAMES):
            scale = h * h if n[0] in "VW" else h
            tol = 1e-10 if n[0] in "VA" else (1e-8 if n[0] == "W" else 1e-6)
            assert np.max(np.abs(a[k] - b[n])) <= tol * scale, n


def test_library_capacities_on_a_stretched_mesh():
    """User abscissas (Sec. 3.1): the library's capacities against the
    oracle's closed-form circle path on the same stretched mesh, and the
    abscissas are validated."""
    import ctypes as C
    from paper_2211_10698_amd import ccns
    case = W.stretched_cylinder(24)
    g = case.grid
    a = ccns.ccns_capacities(g, case.bodies)
    b = geometry.capacities(g, case.bodies)
    h = max(np.diff(g.xf).max(), np.diff(g.yf).max())
    for k, n in enumerate(ccns.CAP_NAMES):
        scale = h * h if n[0] == "V" or n[0] == "W" else h
        tol = 1e-11 if n[0] in "VA" else (1e-8 if n[0] == "W" else 1e-6)
        assert np.max(np.abs(a[k] - b[n])) <= tol * scale, n
    # the full cells carry their own widths and heights
    dx, dy = np.diff(g.xf), np.diff(g.yf)
    V = a[ccns.CAP_NAMES.index("V")]
    assert abs(V[1, 1] - dx[0] * dy[0]) < 1e-15 and abs(V[1, 5] - dx[4] * dy[0]) < 1e-15
    assert abs(V[1:-1, 1:-1].sum() - (g.lx * g.ly - np.pi * 0.25 ** 2)) < 1e-12
    L = ccns.lib()
    bad = list(g.xf)
    bad[3], bad[4] = bad[4], bad[3]
    for xf in (bad, [g.x0 + 1e-3] + list(g.xf[1:]), list(g.xf[:-1]) + [float("nan")]):
        gc = ccns.make_grid(g)
        gc.xf = (C.c_double * len(xf))(*xf)
        out = np.zeros(L.ccns_caps_count(C.byref(gc)))
        assert L.ccns_capacities(C.byref(gc), None, 0, ccns.LEVELSET_FN(), None, out.ctypes.data) == ccns.EINVAL


def test_multigrid_form_words_and_cache():
    """The tuner's form words pack and unpack (3 bits per sweep and level),
    and the committed cache holds forms 1-4 per device, precision and level
    size."""
    import json
    from paper_2211_10698_amd import tune
    pairs = [(2, 2), (1, 1), (3, 1), (4, 4)]
    w = tune.pack(pairs)
    assert tune.unpack(w, 4) == pairs and w < 1 << 24
    with pytest.raises(ValueError):
        tune.pack([(6, 1)])
    with pytest.raises(ValueError):
        tune.pack([(1, 4)])
    cache = json.load(open(tune.CACHE))
    assert cache
    for dev, per in cache.items():
        assert set(per) <= {"f64", "f32"}
        for prec, table in per.items():
            for size, forms in table.items():
                nx, ny = (int(v) for v in size.split("x"))
                assert nx > 0 and ny > 0 and len(forms) == 2 and all(1 <= f <= 5 for f in forms)
    # lookups by level size; missing levels keep the defaults (0)
    dev = next(iter(cache))
    prec = next(iter(cache[dev]))
    size = next(iter(cache[dev][prec]))
    nx, ny = (int(v) for v in size.split("x"))
    p = 1 if prec == "f32" else 0
    w = tune.lookup([(nx, ny), (3, 3)], p, dev, cache)
    assert tune.unpack(w, 2) == [tuple(cache[dev][prec][size]), (0, 0)]
    # a size cached with a short-tile up-sweep (tuned as a coarse level) as a
    # grid's finest level keeps the default up-sweep there
    small = {dev: {prec: {"128x128": [4, 5], "64x64": [5, 4]}}}
    w = tune.lookup([(128, 128), (64, 64)], p, dev, small)
    assert tune.unpack(w, 2) == [(4, 0), (5, 4)]
