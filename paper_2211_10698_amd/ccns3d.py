"""ctypes binding of the three-dimensional projection calls of libccns
(include/ccns3d.h).  Argument marshalling only: the capacities run in the
library's host code, every step of the projection in its HIP kernels.
PyTorch supplies device memory (the workspace and dense field tensors) and
the stream."""

from __future__ import annotations

import ctypes as C
from typing import Sequence

import numpy as np

from . import ccns
from .ccns import CcnsError, OK

SPHERE, ZCYLINDER = 0, 1
CAP_NAMES = ("V", "Ax", "Ay", "Az", "Vx", "Vy", "Vz")
F_UX, F_UY, F_UZ, F_PHI = range(4)
EXPORTED = ("ccns3_caps_count", "ccns3_capacities", "ccns3_workspace_bytes", "ccns3_ctx_create",
            "ccns3_ctx_destroy", "ccns3_field_set", "ccns3_field_get", "ccns3_project", "ccns3_apply_poisson",
            "ccns3_timing", "ccns3_last_error")


class Grid3C(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("x0", C.c_double), ("y0", C.c_double),
                ("z0", C.c_double), ("hx", C.c_double), ("hy", C.c_double), ("hz", C.c_double)]


class Body3C(C.Structure):
    _fields_ = [("kind", C.c_int), ("cx", C.c_double), ("cy", C.c_double), ("cz", C.c_double), ("r", C.c_double)]


class Params3(C.Structure):
    _fields_ = [("rho", C.c_double), ("tau", C.c_double), ("tol", C.c_double), ("mass_floor", C.c_double),
                ("maxit", C.c_int), ("precond", C.c_int)]


class Info3(C.Structure):
    _fields_ = [("iterations", C.c_int), ("status", C.c_int), ("rel_residual", C.c_double), ("div_rel", C.c_double),
                ("n_active", C.c_int)]

    def as_dict(self):
        return {"iterations": self.iterations, "status": self.status, "rel_residual": self.rel_residual,
                "div_rel": self.div_rel, "n_active": self.n_active}


_bound = False


def lib():
    """libccns with the 3-D signatures declared (no fallback path)."""
    global _bound
    L = ccns.lib()
    if not _bound:
        P = C.POINTER
        L.ccns3_caps_count.restype = C.c_size_t
        L.ccns3_caps_count.argtypes = [P(Grid3C)]
        L.ccns3_capacities.restype = C.c_int
        L.ccns3_capacities.argtypes = [P(Grid3C), P(Body3C), C.c_int, C.c_void_p]
        L.ccns3_workspace_bytes.restype = C.c_size_t
        L.ccns3_workspace_bytes.argtypes = [P(Grid3C)]
        L.ccns3_ctx_create.restype = C.c_int
        L.ccns3_ctx_create.argtypes = [P(Grid3C), P(Params3), C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p,
                                       P(C.c_void_p)]
        L.ccns3_ctx_destroy.restype = None
        L.ccns3_ctx_destroy.argtypes = [C.c_void_p]
        L.ccns3_field_set.restype = C.c_int
        L.ccns3_field_set.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_int]
        L.ccns3_field_get.restype = C.c_int
        L.ccns3_field_get.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_int]
        L.ccns3_project.restype = C.c_int
        L.ccns3_project.argtypes = [C.c_void_p, P(Info3)]
        L.ccns3_apply_poisson.restype = C.c_int
        L.ccns3_apply_poisson.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.ccns3_timing.restype = C.c_int
        L.ccns3_timing.argtypes = [C.c_void_p, C.c_int, P(C.c_double), P(C.c_long)]
        L.ccns3_last_error.restype = C.c_char_p
        L.ccns3_last_error.argtypes = [C.c_void_p]
        _bound = True
    return L


def make_grid(g) -> Grid3C:
    return Grid3C(g.nx, g.ny, g.nz, g.x0, g.y0, g.z0, g.hx, g.hy, g.hz)


def make_bodies(bodies: Sequence):
    arr = (Body3C * max(1, len(bodies)))()
    for k, b in enumerate(bodies):
        arr[k] = Body3C(int(b.kind), b.cx, b.cy, b.cz, b.r)
    return arr


def capacities(g, bodies) -> np.ndarray:
    """The library's host capacities: (7, nz+2, ny+2, nx+2) in the order of
    CAP_NAMES."""
    L = lib()
    gc = make_grid(g)
    n = L.ccns3_caps_count(C.byref(gc))
    if n == 0:
        raise CcnsError(ccns.EINVAL, "bad grid")
    out = np.zeros(n)
    st = L.ccns3_capacities(C.byref(gc), make_bodies(bodies), len(bodies), out.ctypes.data)
    if st != OK:
        raise CcnsError(st, "ccns3_capacities")
    return out.reshape(7, g.nz + 2, g.ny + 2, g.nx + 2)


def make_params(rho, tau, tol=1e-12, mass_floor=0.05, maxit=100000, precond=1) -> Params3:
    """precond: 0 Jacobi, 1 the multigrid V-cycle, 2 the cycle stored in
    FP32 (ccns3_params)."""
    return Params3(rho, tau, tol, mass_floor, maxit, precond)


class Context3:
    """One 3-D projection problem on the device: owns a torch workspace
    tensor; runs on `stream` (default: torch's current stream)."""

    def __init__(self, g, params: Params3, caps: np.ndarray, stream=None, device="cuda"):
        import torch

        self.torch = torch
        self.g = g
        self.shape = g.shape
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device(self.device.type, torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        L = lib()
        self.gc = make_grid(g)
        nbytes = L.ccns3_workspace_bytes(C.byref(self.gc))
        if nbytes == 0:
            raise CcnsError(ccns.EINVAL, "bad grid")
        caps = np.ascontiguousarray(caps, dtype=np.float64)
        if caps.size != L.ccns3_caps_count(C.byref(self.gc)):
            raise CcnsError(ccns.EINVAL, "capacity array of the wrong size")
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        ptr = (self.ws.data_ptr() + 255) // 256 * 256
        self._ready()
        if self.stream.cuda_stream != torch.cuda.current_stream(self.device).cuda_stream:
            self.ws.record_stream(self.stream)
        h = C.c_void_p()
        st = L.ccns3_ctx_create(C.byref(self.gc), C.byref(params), caps.ctypes.data, C.c_void_p(ptr), nbytes,
                                C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if st != OK:
            raise CcnsError(st, "ccns3_ctx_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().ccns3_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _ready(self):
        cur = self.torch.cuda.current_stream(self.device)
        if cur.cuda_stream != self.stream.cuda_stream:
            cur.synchronize()

    def _chk(self, st, what):
        if st != OK:
            msg = lib().ccns3_last_error(self.h)
            raise CcnsError(st, f"{what}: {msg.decode() if msg else ''}")

    def set_field(self, field: int, arr):
        t = self.torch
        if isinstance(arr, np.ndarray):
            a = np.ascontiguousarray(arr, dtype=np.float64)
            if a.shape != self.shape:
                raise ValueError(f"field shape {a.shape}, expected {self.shape}")
            return self._chk(lib().ccns3_field_set(self.h, field, a.ctypes.data, 0), "field_set")
        a = arr.to(device=self.device, dtype=t.float64).contiguous()
        if tuple(a.shape) != self.shape:
            raise ValueError(f"field shape {tuple(a.shape)}, expected {self.shape}")
        self._ready()
        return self._chk(lib().ccns3_field_set(self.h, field, a.data_ptr(), 1), "field_set")

    def get_field(self, field: int):
        out = self.torch.zeros(self.shape, dtype=self.torch.float64, device=self.device)
        self._ready()
        self._chk(lib().ccns3_field_get(self.h, field, out.data_ptr(), 1), "field_get")
        return out

    def project(self, check=True) -> Info3:
        info = Info3()
        st = lib().ccns3_project(self.h, C.byref(info))
        if check:
            self._chk(st, "project")
        return info

    def timing(self, enable=-1):
        """((ms, count) of the direction kernel, of the update kernel, of the
        finest level's first up-sweep of the multigrid cycle); see
        ccns3_timing."""
        ms = (C.c_double * 3)()
        cnt = (C.c_long * 3)()
        self._chk(lib().ccns3_timing(self.h, enable, ms, cnt), "timing")
        return (ms[0], cnt[0]), (ms[1], cnt[1]), (ms[2], cnt[2])

    def apply_poisson(self, x):
        """(-L) x on the cells (dense layout), a device tensor."""
        t = self.torch
        a = (x if isinstance(x, t.Tensor) else t.from_numpy(np.ascontiguousarray(x, dtype=np.float64)))
        a = a.to(device=self.device, dtype=t.float64).contiguous()
        out = t.zeros(self.shape, dtype=t.float64, device=self.device)
        self._ready()
        self._chk(lib().ccns3_apply_poisson(self.h, a.data_ptr(), out.data_ptr()), "apply_poisson")
        return out
