"""ctypes binding of libccns (include/ccns.h).  Argument marshalling only:
every step of the method runs in the library's HIP kernels.  PyTorch
supplies device memory (the workspace and dense field tensors) and the
stream."""

from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libccns.so")

OK, EINVAL, ENOMEM, ENOTCONV, EBREAKDOWN, EDEVICE, ESTATE = 0, -1, -2, -3, -4, -5, -6
STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "ENOTCONV", -4: "EBREAKDOWN", -5: "EDEVICE", -6: "ESTATE"}
CIRCLE, ELLIPSE, NACA4 = 0, 1, 2
NCAPS = 21
CAP_NAMES = ("V", "Ax", "Ay", "Bx", "By", "Wx", "Wy",
             "Vu", "Axx", "Axy", "Bxx", "Bxy", "Wxx", "Wxy",
             "Vv", "Ayy", "Ayx", "Byy", "Byx", "Wyy", "Wyx")
F_UX, F_UY, F_P, F_PHI, F_CONVX, F_CONVY, F_USX, F_USY, F_B = range(9)
OP_CONT, OP_PRES, OP_VISC, OP_CONV, OP_LAP, OP_H, OP_KINETIC = range(7)
_OP_ARITY = {OP_CONT: (2, 1), OP_PRES: (1, 2), OP_VISC: (2, 2), OP_CONV: (2, 2), OP_LAP: (1, 1),
             OP_H: (2, 2), OP_KINETIC: (2, 1)}


class Grid(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("x0", C.c_double), ("y0", C.c_double),
                ("hx", C.c_double), ("hy", C.c_double),
                ("xf", C.POINTER(C.c_double)), ("yf", C.POINTER(C.c_double))]


class BodyC(C.Structure):
    _fields_ = [("kind", C.c_int), ("cx", C.c_double), ("cy", C.c_double), ("a", C.c_double),
                ("b", C.c_double), ("angle", C.c_double), ("chord", C.c_double), ("t", C.c_double)]


class Params(C.Structure):
    _fields_ = [("rho", C.c_double), ("mu", C.c_double), ("tau", C.c_double), ("u_ref", C.c_double),
                ("gx", C.c_double), ("gy", C.c_double), ("pcg_tol", C.c_double), ("pred_tol", C.c_double),
                ("div_tol", C.c_double), ("pcg_maxit", C.c_int), ("pred_maxit", C.c_int),
                ("precision", C.c_int), ("visc_form", C.c_int), ("poisson_weight", C.c_int),
                ("precond", C.c_int), ("mass_floor", C.c_double), ("coef_tables", C.c_int),
                ("outflow", C.c_int), ("mg_forms", C.c_ulonglong)]


class SolveInfo(C.Structure):
    _fields_ = [("iterations", C.c_int), ("outer", C.c_int), ("rel_residual", C.c_double), ("status", C.c_int),
                ("inner_status", C.c_int), ("inner_fail_sweep", C.c_int)]


class StepInfo(C.Structure):
    _fields_ = [("pred", SolveInfo), ("poisson", SolveInfo), ("div_max", C.c_double), ("div_rel", C.c_double),
                ("ke", C.c_double), ("mass", C.c_double), ("mom_x", C.c_double), ("mom_y", C.c_double)]

    def as_dict(self):
        return {"pred_iters": self.pred.iterations, "pred_status": self.pred.status,
                "pred_outer": self.pred.outer, "pred_inner_status": self.pred.inner_status,
                "cg_iters": self.poisson.iterations, "cg_outer": self.poisson.outer,
                "cg_relres": self.poisson.rel_residual, "cg_status": self.poisson.status,
                "cg_inner_status": self.poisson.inner_status, "cg_inner_fail_sweep": self.poisson.inner_fail_sweep,
                "div_max": self.div_max, "div_rel": self.div_rel, "ke": self.ke, "mass": self.mass,
                "mom_x": self.mom_x, "mom_y": self.mom_y}


LEVELSET_FN = C.CFUNCTYPE(C.c_double, C.c_double, C.c_double, C.c_void_p)

_lib = None


def lib():
    """The loaded library.  Raises if it has not been built: there is no
    fallback path."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libccns.so is not built ({LIB_PATH}); run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        P = C.POINTER
        L.ccns_caps_count.restype = C.c_size_t
        L.ccns_caps_count.argtypes = [P(Grid)]
        L.ccns_capacities.restype = C.c_int
        L.ccns_capacities.argtypes = [P(Grid), P(BodyC), C.c_int, LEVELSET_FN, C.c_void_p, C.c_void_p]
        L.ccns_capacities_scratch_bytes.restype = C.c_size_t
        L.ccns_capacities_scratch_bytes.argtypes = [P(Grid)]
        L.ccns_capacities_device.restype = C.c_int
        L.ccns_capacities_device.argtypes = [P(Grid), P(BodyC), C.c_int, C.c_void_p, C.c_void_p, C.c_size_t,
                                             C.c_void_p]
        L.ccns_workspace_bytes.restype = C.c_size_t
        L.ccns_workspace_bytes.argtypes = [P(Grid), P(Params)]
        L.ccns_ctx_create.restype = C.c_int
        L.ccns_ctx_create.argtypes = [P(Grid), P(Params), C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t,
                                      C.c_void_p, P(C.c_void_p)]
        L.ccns_ctx_create_static.restype = C.c_int
        L.ccns_ctx_create_static.argtypes = [P(Grid), P(Params), C.c_void_p, C.c_void_p, C.c_void_p,
                                             P(C.c_void_p)]
        L.ccns_ctx_destroy.restype = None
        L.ccns_ctx_destroy.argtypes = [C.c_void_p]
        L.ccns_last_error.restype = C.c_char_p
        L.ccns_last_error.argtypes = [C.c_void_p]
        L.ccns_coef_classes.restype = C.c_int
        L.ccns_coef_classes.argtypes = [C.c_void_p]
        for name in ("ccns_field_set", "ccns_field_get"):
            f = getattr(L, name)
            f.restype = C.c_int
            f.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_int]
        L.ccns_apply.restype = C.c_int
        L.ccns_apply.argtypes = [C.c_void_p, C.c_int, P(C.c_void_p), P(C.c_void_p)]
        L.ccns_pressure_solve.restype = C.c_int
        L.ccns_pressure_solve.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, P(SolveInfo)]
        for name in ("ccns_project", "ccns_correct", "ccns_diagnostics"):
            f = getattr(L, name)
            f.restype = C.c_int
            f.argtypes = [C.c_void_p, P(StepInfo)]
        L.ccns_predict.restype = C.c_int
        L.ccns_predict.argtypes = [C.c_void_p, P(SolveInfo)]
        L.ccns_forces.restype = C.c_int
        L.ccns_forces.argtypes = [C.c_void_p, P(C.c_double)]
        L.ccns_set_mg_forms.restype = C.c_int
        L.ccns_set_mg_forms.argtypes = [C.c_void_p, C.c_ulonglong]
        L.ccns_mg_levels.restype = C.c_int
        L.ccns_mg_levels.argtypes = [C.c_void_p, P(C.c_int), P(C.c_int), P(C.c_int), C.c_int]
        L.ccns_timing.restype = C.c_int
        L.ccns_timing.argtypes = [C.c_void_p, C.c_int, P(C.c_double), P(C.c_long)]
        L.ccns_step.restype = C.c_int
        L.ccns_step.argtypes = [C.c_void_p, C.c_int, P(StepInfo)]
        L.ccns_batch_create.restype = C.c_int
        L.ccns_batch_create.argtypes = [C.c_int, P(C.c_void_p), C.c_int, P(C.c_void_p)]
        L.ccns_batch_create_fused.restype = C.c_int
        L.ccns_batch_create_fused.argtypes = [C.c_int, P(C.c_void_p), P(C.c_void_p)]
        L.ccns_batch_graphs.restype = C.c_int
        L.ccns_batch_graphs.argtypes = [C.c_void_p, C.c_int]
        L.ccns_batch_step.restype = C.c_int
        L.ccns_batch_step.argtypes = [C.c_void_p, C.c_int, P(StepInfo), P(C.c_int)]
        L.ccns_batch_destroy.restype = None
        L.ccns_batch_destroy.argtypes = [C.c_void_p]
        _lib = L
    return _lib


EXPORTED = ("ccns_caps_count", "ccns_capacities", "ccns_capacities_scratch_bytes", "ccns_capacities_device",
            "ccns_workspace_bytes", "ccns_ctx_create", "ccns_ctx_create_static",
            "ccns_ctx_destroy", "ccns_last_error", "ccns_coef_classes", "ccns_field_set", "ccns_field_get", "ccns_apply",
            "ccns_pressure_solve", "ccns_project", "ccns_step", "ccns_predict", "ccns_correct",
            "ccns_diagnostics", "ccns_forces", "ccns_set_mg_forms", "ccns_mg_levels", "ccns_timing",
            "ccns_batch_create", "ccns_batch_create_fused", "ccns_batch_graphs", "ccns_batch_step",
            "ccns_batch_destroy")


class CcnsError(RuntimeError):
    def __init__(self, status, msg=""):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def make_grid(spec) -> Grid:
    """The C grid of a GridSpec; a stretched spec's abscissas are copied into
    ctypes arrays that the structure keeps alive."""
    g = Grid(spec.nx, spec.ny, spec.x0, spec.y0, spec.hx, spec.hy)
    xf, yf = getattr(spec, "xf", None), getattr(spec, "yf", None)
    if xf is not None:
        g.xf = (C.c_double * len(xf))(*xf)
    if yf is not None:
        g.yf = (C.c_double * len(yf))(*yf)
    return g


def make_bodies(bodies):
    arr = (BodyC * max(len(bodies), 1))()
    for k, b in enumerate(bodies):
        arr[k] = BodyC(b.kind, b.cx, b.cy, b.a, b.b, b.angle, b.chord, b.t)
    return arr


def ccns_capacities(spec, bodies, fn=None) -> np.ndarray:
    """Capacities (21, ny+2, nx+2) computed by the library on the host."""
    L = lib()
    g = make_grid(spec)
    n = L.ccns_caps_count(C.byref(g))
    out = np.zeros(n, dtype=np.float64)
    cb = LEVELSET_FN(fn) if fn is not None else LEVELSET_FN()
    st = L.ccns_capacities(C.byref(g), make_bodies(bodies), len(bodies), cb, None, out.ctypes.data)
    if st != OK:
        raise CcnsError(st, "ccns_capacities")
    return out.reshape(NCAPS, spec.ny + 2, spec.nx + 2)


def ccns_capacities_device(spec, bodies, stream=None):
    """Capacities (21, ny+2, nx+2) computed on the device (circles and
    ellipses): a float64 tensor on the current device, ready when the
    stream's queued work is."""
    import torch

    L = lib()
    g = make_grid(spec)
    n = L.ccns_caps_count(C.byref(g))
    nscr = L.ccns_capacities_scratch_bytes(C.byref(g))
    caps = torch.empty(n, dtype=torch.float64, device="cuda")
    scratch = torch.empty(nscr, dtype=torch.uint8, device="cuda")
    s = stream if stream is not None else torch.cuda.current_stream()
    cur = torch.cuda.current_stream()
    if cur.cuda_stream != s.cuda_stream:
        cur.synchronize()
    st = L.ccns_capacities_device(C.byref(g), make_bodies(bodies), len(bodies), C.c_void_p(caps.data_ptr()),
                                  C.c_void_p(scratch.data_ptr()), nscr, C.c_void_p(s.cuda_stream))
    if st != OK:
        raise CcnsError(st, "ccns_capacities_device")
    if cur.cuda_stream != s.cuda_stream:
        s.synchronize()   # the scratch tensor is freed on return
    return caps.view(NCAPS, spec.ny + 2, spec.nx + 2)


PRECOND_JACOBI, PRECOND_MG = 0, 1
WALL_BITS = {"W": 1, "E": 2, "S": 4, "N": 8}


def make_params(rho, mu, tau, u_ref=1.0, pcg_tol=1e-10, pred_tol=1e-12, div_tol=1e-8, pcg_maxit=200000,
                pred_maxit=500, precision=0, visc_form=0, poisson_weight=0, gx=0.0, gy=0.0,
                precond=PRECOND_MG, mass_floor=0.05, coef_tables=0, outflow="", mg_forms=0) -> Params:
    """outflow: the outflow walls as letters of "WESN" (or the C bitmask);
    mg_forms: the multigrid cycle's kernel forms (paper_2211_10698_amd.tune)."""
    if isinstance(outflow, str):
        if any(w not in "WESN" for w in outflow):
            raise ValueError(f"outflow walls {outflow!r}: letters of 'WESN'")
        outflow = sum(WALL_BITS[w] for w in set(outflow))
    return Params(rho, mu, tau, u_ref, gx, gy, pcg_tol, pred_tol, div_tol, pcg_maxit, pred_maxit, precision,
                  visc_form, poisson_weight, precond, mass_floor, coef_tables, outflow, mg_forms)


STATIC_WORKSPACE_BYTES = 64 << 20


class Context:
    """One simulation on the device.  Owns a torch workspace tensor, or with
    static=True uses the library's static workspace (ccns_ctx_create_static:
    no allocation; one such context per device at a time)."""

    def __init__(self, spec, params: Params, caps: np.ndarray, dx: np.ndarray, dy: np.ndarray,
                 device="cuda", stream=None, static=False):
        import torch

        self.torch = torch
        self.spec = spec
        self.shape = (spec.ny + 2, spec.nx + 2)
        L = lib()
        self.g = make_grid(spec)
        self.params = params
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device(self.device.type, torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        caps = np.ascontiguousarray(caps, dtype=np.float64)
        dirichlet = np.ascontiguousarray(np.stack([dx, dy]), dtype=np.float64)
        h = C.c_void_p()
        if static:
            self.ws = None
            st = L.ccns_ctx_create_static(C.byref(self.g), C.byref(params), caps.ctypes.data, dirichlet.ctypes.data,
                                          C.c_void_p(self.stream.cuda_stream), C.byref(h))
            if st != OK:
                raise CcnsError(st, "ccns_ctx_create_static")
            self.h = h
            return
        nbytes = L.ccns_workspace_bytes(C.byref(self.g), C.byref(params))
        if nbytes == 0:
            raise CcnsError(EINVAL, "bad grid")
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        self.ws_ptr = (base + 255) // 256 * 256
        self.ws_bytes = nbytes
        # The workspace was allocated on torch's current stream, whose caching
        # allocator may hand out a block that work still queued on that stream
        # uses; the library clears and fills it on the context's own stream.
        # Wait for the current stream first, and tell the allocator that the
        # block is in use on the context's stream (so that it is not handed
        # out again while work queued there may still touch it).
        self._ready()
        if self.stream.cuda_stream != torch.cuda.current_stream(self.device).cuda_stream:
            self.ws.record_stream(self.stream)
        st = L.ccns_ctx_create(C.byref(self.g), C.byref(params), caps.ctypes.data, dirichlet.ctypes.data,
                               C.c_void_p(self.ws_ptr), nbytes, C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if st != OK:
            raise CcnsError(st, "ccns_ctx_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().ccns_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, st, what):
        if st not in (OK,):
            msg = lib().ccns_last_error(self.h)
            raise CcnsError(st, f"{what}: {msg.decode() if msg else ''}")
        return st

    def _dense(self):
        return self.torch.zeros(self.shape, dtype=self.torch.float64, device=self.device)

    def _ready(self):
        """Tensors handed to the library were made (allocated, filled,
        converted) on torch's current stream; the library works on the
        context's stream.  Wait for the former before a call: the library
        synchronizes its own stream before it returns."""
        cur = self.torch.cuda.current_stream(self.device)
        if cur.cuda_stream != self.stream.cuda_stream:
            cur.synchronize()

    def set_field(self, field: int, arr):
        t = self.torch
        if isinstance(arr, np.ndarray):
            a = np.ascontiguousarray(arr, dtype=np.float64)
            return self._chk(lib().ccns_field_set(self.h, field, a.ctypes.data, 0), "field_set")
        a = arr.to(dtype=t.float64).contiguous()
        self._ready()
        return self._chk(lib().ccns_field_set(self.h, field, a.data_ptr(), 1), "field_set")

    def get_field(self, field: int):
        out = self._dense()
        self._ready()
        self._chk(lib().ccns_field_get(self.h, field, out.data_ptr(), 1), "field_get")
        return out

    def apply(self, op: int, inputs: Sequence):
        t = self.torch
        nin, nout = _OP_ARITY[op]
        ins = [x if not isinstance(x, np.ndarray) else t.from_numpy(np.ascontiguousarray(x)).to(self.device)
               for x in inputs]
        ins = [x.to(dtype=t.float64).contiguous() for x in ins]
        outs = [self._dense() for _ in range(nout)]
        self._ready()
        pin = (C.c_void_p * nin)(*[x.data_ptr() for x in ins])
        pout = (C.c_void_p * nout)(*[x.data_ptr() for x in outs])
        self._chk(lib().ccns_apply(self.h, op, pin, pout), "apply")
        return outs

    def pressure_solve(self, b, check=True):
        t = self.torch
        b = b.to(dtype=t.float64).contiguous()
        phi = self._dense()
        self._ready()
        info = SolveInfo()
        st = lib().ccns_pressure_solve(self.h, b.data_ptr(), phi.data_ptr(), C.byref(info))
        if check:
            self._chk(st, "pressure_solve")
        return phi, info, st

    def project(self):
        info = StepInfo()
        self._chk(lib().ccns_project(self.h, C.byref(info)), "project")
        return info

    def predict(self, check=True):
        info = SolveInfo()
        st = lib().ccns_predict(self.h, C.byref(info))
        if check:
            self._chk(st, "predict")
        return info

    def correct(self, check=True):
        info = StepInfo()
        st = lib().ccns_correct(self.h, C.byref(info))
        if check:
            self._chk(st, "correct")
        return info

    def step(self, n=1, check=True):
        info = StepInfo()
        st = lib().ccns_step(self.h, n, C.byref(info))
        if check:
            self._chk(st, "step")
        return info

    def coef_classes(self) -> int:
        """Coefficient classes the predictor's CG reads (0: the arrays)."""
        return int(lib().ccns_coef_classes(self.h))

    def timing(self, enable=-1):
        """Accumulated (ms, count) per timed kernel; see ccns_timing."""
        ms = (C.c_double * 4)()
        cnt = (C.c_long * 4)()
        self._chk(lib().ccns_timing(self.h, enable, ms, cnt), "timing")
        return list(ms), list(cnt)

    def diagnostics(self):
        info = StepInfo()
        self._chk(lib().ccns_diagnostics(self.h, C.byref(info)), "diagnostics")
        return info

    def forces(self):
        """(F^p_x, F^p_y, F^v_x, F^v_y) on the bodies; see ccns_forces."""
        out = (C.c_double * 4)()
        self._chk(lib().ccns_forces(self.h, out), "forces")
        return tuple(out)

    def set_mg_forms(self, forms):
        self._chk(lib().ccns_set_mg_forms(self.h, int(forms)), "set_mg_forms")

    def mg_levels(self):
        """[(nx, ny, down form, up form)] of the multigrid cycle levels."""
        nx, ny, fm = (C.c_int * 10)(), (C.c_int * 10)(), (C.c_int * 10)()
        n = lib().ccns_mg_levels(self.h, nx, ny, fm, 10)
        return [(nx[k], ny[k], fm[k] & 7, fm[k] >> 3) for k in range(n)]


class Batch:
    """A ragged batch of contexts stepped together (ccns_batch_*).  The
    contexts stay owned by the caller and must outlive the batch.  fused:
    one launch per phase over every simulation's work-groups
    (ccns_batch_create_fused; one precision for all, the multigrid
    preconditioner), else one host thread and stream per simulation."""

    def __init__(self, contexts: Sequence["Context"], nthreads: int = 0, fused: bool = False, graphs: bool = True):
        self.contexts = list(contexts)
        self.fused = fused
        arr = (C.c_void_p * len(self.contexts))(*[c.h.value for c in self.contexts])
        h = C.c_void_p()
        if fused:
            st = lib().ccns_batch_create_fused(len(self.contexts), arr, C.byref(h))
            if st != OK:
                raise CcnsError(st, "ccns_batch_create_fused")
            if not graphs:
                st = lib().ccns_batch_graphs(h, 0)
                if st != OK:
                    lib().ccns_batch_destroy(h)
                    raise CcnsError(st, "ccns_batch_graphs")
        else:
            st = lib().ccns_batch_create(len(self.contexts), arr, nthreads, C.byref(h))
            if st != OK:
                raise CcnsError(st, "ccns_batch_create")
        self.h = h

    def step(self, n=1, check=True):
        """Advances every simulation by n steps; returns (worst status,
        per-simulation StepInfo list, per-simulation statuses)."""
        m = len(self.contexts)
        infos = (StepInfo * m)()
        sts = (C.c_int * m)()
        st = lib().ccns_batch_step(self.h, n, infos, sts)
        if check and st not in (OK,):
            raise CcnsError(st, "ccns_batch_step")
        return st, list(infos), list(sts)

    def close(self):
        if getattr(self, "h", None):
            lib().ccns_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

