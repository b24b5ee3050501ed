"""Capacities computed on the device (ccns_capacities_device: closed-form
conic integrals) against the oracle and the host computation.

  * Circles: against the oracle's closed-form circle path (oracle.geometry
    CircleGeometry, an independent derivation): V and A (all three grids) to
    1e-12 of their scale (hx hy for volumes, h for lengths), on a grid with
    ragged sizes and two circles, one of them flat against a grid line.
  * Ellipses: against the oracle's generic level-set quadrature on a small
    grid (V and A to 1e-11, that quadrature's accuracy), and against the host
    library's quadrature on the serving trace's three-ellipse case at 96 x 96
    (V and A to 1e-12).
  * B and W depend on the centroids, which in a sliver control volume (a few
    1e-12 of a cell) are fixed by first moments that cancel to 1e-10 of
    their size: there no two back-ends agree beyond 1e-5 h (B) and 1e-9
    hx hy (W), and that is the bound used (parity unpinned at slivers, as for
    the host computation).
  * Identities that hold for any geometry: the full-cell values are the
    host's bit for bit (so the predictor's coefficient classes form), the
    total fluid volume is the box area minus the bodies' areas."""

import math

import numpy as np
import pytest

import workloads as W
from oracle import geometry

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

VOL = ("V", "Wx", "Wy", "Vu", "Wxx", "Wxy", "Vv", "Wyy", "Wyx")


def _scale(name, g):
    return g.hx * g.hy if name in VOL else max(g.hx, g.hy)


def _device(case):
    from paper_2211_10698_amd import ccns
    print(f"[caps-device] {case.name} {case.grid.nx}x{case.grid.ny}", flush=True)
    d = ccns.ccns_capacities_device(case.grid, case.bodies)
    torch.cuda.synchronize()
    return {k: d[i].cpu().numpy() for i, k in enumerate(ccns.CAP_NAMES)}


VA = ("V", "Ax", "Ay", "Vu", "Axx", "Axy", "Vv", "Ayy", "Ayx")
B_TOL, W_TOL = 1e-5, 1e-9


def _compare(dev, ref, g, tol_vol, tol_len, names=None):
    from paper_2211_10698_amd import ccns
    worst = {}
    for k in names or ccns.CAP_NAMES:
        e = float(np.max(np.abs(dev[k] - ref[k]))) / _scale(k, g)
        worst[k] = e
        assert e <= (tol_vol if k in VOL else tol_len), (k, e)
    return worst


def test_circles_against_oracle_closed_form():
    h = 1.0 / 96
    top = math.floor((0.3 + 0.12) / h) * h - 0.02 * h
    g = W.GridSpec(131, 77, 0.0, 0.0, 131 * h, 77 * h)
    case = W.Case("two_circles", g, [W.Body(W.CIRCLE, 0.41, top - 0.12, a=0.12),
                                     W.Body(W.CIRCLE, 0.98, 0.37, a=0.17)], re=100.0)
    dev = _device(case)
    ref = geometry.capacities(g, case.bodies)
    worst = _compare(dev, ref, g, 1e-12, 1e-12, names=VA)
    _compare(dev, ref, g, W_TOL, B_TOL)
    print(f"[caps-device] circles: worst V/A {max(worst.values()):.2e}", flush=True)
    # the fluid volume: the box minus the two discs
    area = g.lx * g.ly - math.pi * (0.12 ** 2 + 0.17 ** 2)
    assert abs(dev["V"][1:-1, 1:-1].sum() - area) < 1e-12 * area


def test_ellipse_against_oracle_quadrature():
    g = W.GridSpec(20, 18, 0.0, 0.0, 1.0, 0.9)
    case = W.Case("ellipse", g, [W.Body(W.ELLIPSE, 0.48, 0.44, a=0.27, b=0.13, angle=0.61)], re=100.0)
    dev = _device(case)
    ref = geometry.capacities(g, case.bodies)
    worst = _compare(dev, ref, g, 1e-11, 1e-11, names=VA)
    _compare(dev, ref, g, W_TOL, B_TOL)
    print(f"[caps-device] ellipse vs oracle: worst V/A {max(worst.values()):.2e}", flush=True)
    area = g.lx * g.ly - math.pi * 0.27 * 0.13
    assert abs(dev["V"][1:-1, 1:-1].sum() - area) < 1e-12 * area


def test_ellipses_against_host_library():
    from paper_2211_10698_amd import ccns
    case = W.ellipses(96)
    g = case.grid
    dev = _device(case)
    host = ccns.ccns_capacities(g, case.bodies)
    ref = {k: host[i] for i, k in enumerate(ccns.CAP_NAMES)}
    worst = _compare(dev, ref, g, 1e-12, 1e-12, names=VA)
    _compare(dev, ref, g, W_TOL, B_TOL)
    print(f"[caps-device] ellipses vs host: worst V/A {max(worst.values()):.2e}", flush=True)
    # full control volumes, faces and strips carry the same values bit for bit
    for k in ccns.CAP_NAMES:
        full = ref[k] == (g.hx * g.hy if k in VOL else (g.hy if k in ("Ax", "Bx", "Axx", "Bxx", "Ayx", "Byx")
                                                        else g.hx))
        assert np.array_equal(dev[k][full], ref[k][full]), k


def test_rejects_what_it_cannot_integrate():
    from paper_2211_10698_amd import ccns
    g = W.GridSpec(32, 32, 0.0, 0.0, 1.0, 1.0)
    with pytest.raises(ccns.CcnsError):
        ccns.ccns_capacities_device(g, [W.Body(W.NACA4, 0.2, 0.5, chord=0.5, t=0.12)])
    with pytest.raises(ccns.CcnsError):
        ccns.ccns_capacities_device(g, [W.Body(W.CIRCLE, 0.5, 0.5, a=0.2), W.Body(W.CIRCLE, 0.7, 0.5, a=0.2)])
