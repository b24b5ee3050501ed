"""CPU checks of the library's three-dimensional capacities: they agree with
the oracle's independent integration (sections by planes x = const and a
chord integral in the library; by planes z = const and disc quadrants in
the oracle), and the calls validate their arguments without a GPU."""

import ctypes as C

import numpy as np
import pytest

import workloads.three_d as T
from oracle import geometry3d as G3

_ORACLE = {}


def _oracle(case):
    if case.name not in _ORACLE:
        _ORACLE[case.name] = G3.capacities(case.grid, case.bodies)
    return _ORACLE[case.name]


@pytest.mark.parametrize("make", [T.tiny_box, lambda: T.sphere_box(16), lambda: T.two_spheres(20, 18, 14),
                                  lambda: T.zcylinder_box(12, 10, 3)])
def test_library_capacities_match_the_oracle(make):
    from paper_2211_10698_amd import ccns3d
    case = make()
    g = case.grid
    a = ccns3d.capacities(g, case.bodies)
    b = _oracle(case)
    full = {"V": g.hx * g.hy * g.hz, "Vx": g.hx * g.hy * g.hz, "Vy": g.hx * g.hy * g.hz, "Vz": g.hx * g.hy * g.hz,
            "Ax": g.hy * g.hz, "Ay": g.hx * g.hz, "Az": g.hx * g.hy}
    for k, n in enumerate(ccns3d.CAP_NAMES):
        assert np.abs(a[k] - b[n]).max() <= 1e-13 * full[n], n
        # the same cut cells and faces are zero on both sides
        assert np.array_equal(a[k] > 0, b[n] > 0), n


def test_argument_validation():
    from paper_2211_10698_amd import ccns3d
    L = ccns3d.lib()
    bad = ccns3d.Grid3C(0, 4, 4, 0, 0, 0, 1, 1, 1)
    assert L.ccns3_caps_count(C.byref(bad)) == 0
    assert L.ccns3_workspace_bytes(C.byref(bad)) == 0
    # fields beyond 32-bit element indices are refused (1,400^3 cells)
    huge = ccns3d.Grid3C(1400, 1400, 1400, 0, 0, 0, 1.0 / 1400, 1.0 / 1400, 1.0 / 1400)
    assert L.ccns3_workspace_bytes(C.byref(huge)) == 0
    fits = ccns3d.Grid3C(1024, 1024, 1024, 0, 0, 0, 1.0 / 1024, 1.0 / 1024, 1.0 / 1024)
    assert L.ccns3_workspace_bytes(C.byref(fits)) > 0
    g = ccns3d.Grid3C(4, 4, 4, 0, 0, 0, 0.25, 0.25, 0.25)
    out = np.zeros(L.ccns3_caps_count(C.byref(g)))
    for body in (ccns3d.Body3C(0, 0.5, 0.5, 0.5, -0.1), ccns3d.Body3C(7, 0.5, 0.5, 0.5, 0.1),
                 ccns3d.Body3C(0, float("nan"), 0.5, 0.5, 0.1)):
        arr = (ccns3d.Body3C * 1)(body)
        assert L.ccns3_capacities(C.byref(g), arr, 1, out.ctypes.data) == -1
    h = C.c_void_p()
    p = ccns3d.make_params(1.0, 0.01)
    caps = np.zeros(L.ccns3_caps_count(C.byref(g)))
    # NULL workspace, a misaligned one, a bad time step, a negative capacity:
    # refused before any device work
    assert L.ccns3_ctx_create(C.byref(g), C.byref(p), caps.ctypes.data, None, 1 << 30, None, C.byref(h)) == -1
    assert L.ccns3_ctx_create(C.byref(g), C.byref(p), caps.ctypes.data, C.c_void_p(4096 + 8), 1 << 30, None,
                              C.byref(h)) == -1
    bad_p = ccns3d.make_params(1.0, -0.01)
    assert L.ccns3_ctx_create(C.byref(g), C.byref(bad_p), caps.ctypes.data, C.c_void_p(4096), 1 << 30, None,
                              C.byref(h)) == -1
    bad_pc = ccns3d.make_params(1.0, 0.01, precond=3)
    assert L.ccns3_ctx_create(C.byref(g), C.byref(bad_pc), caps.ctypes.data, C.c_void_p(4096), 1 << 30, None,
                              C.byref(h)) == -1
    assert L.ccns3_ctx_create(C.byref(g), C.byref(p), caps.ctypes.data, C.c_void_p(4096), 16, None,
                              C.byref(h)) == -2
    neg = caps.copy()
    neg[5] = -1.0
    assert L.ccns3_ctx_create(C.byref(g), C.byref(p), neg.ctypes.data, C.c_void_p(4096), 1 << 30, None,
                              C.byref(h)) == -1
    assert L.ccns3_project(None, None) == -1
