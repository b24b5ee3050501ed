"""Projection method II time step (Sec. 4.6: eq:pm_prediction, eq:pm_poisson,
eq:pm_projection, eq:pm_update) on the operators of oracle.operators.

Readings (the paper states the scheme with unit mass matrices and density):
  * Poisson:   (tau/rho) cont(M^-1 pres(Phi), 0) = cont(U*, D^{n+1})
  * corrector: U^{n+1} = U* - (tau/rho) M^-1 pres(Phi)
  * pressure:  P^{n+1/2} = P^{n-1/2} + Phi - (tau mu / 2 rho) V^-1 cont(M^-1 pres(Phi), 0)
    With M = V = 1 and rho = 1 these are the printed equations.
  * AB2 start: conv^{-1} := conv^0; P^{-1/2} = 0; Phi^0 = 0.
  * Without outflow walls the Poisson right-hand side has its mean over the
    pressure unknowns removed (the problem is singular: pure Neumann in Phi).
  * Predictor: Jacobi-PCG on H = (rho/tau) M - mu K, K U = visc(strain(U, 0)),
    started from U^n, relative tolerance 1e-12; Poisson: Jacobi-PCG with the
    zero-mean projection, started from Phi^n.
  * Dirichlet data: eq:pm_prediction carries D at both time levels; with data
    that change in time (Stepper.step(..., D_next)), convection and the
    explicit viscous half use D^n, the implicit half, U* on the non-unknown
    faces and the rest of the step D^{n+1}.
  * Outflow walls (homogeneous Neumann velocity, zero pressure beyond the
    wall; end of Sec. 4.6): each step takes D^{n+1} on such a wall from U^n
    by a zero normal gradient (explicitly): a face normal to the wall gets
    the velocity of the interior face next to it, and the tangential
    velocity beyond the wall (the ghost row or column, which the convective
    flux through the wall reads) that of the first row or column inside.
    U* on the outflow faces is that D^{n+1}; the projection then corrects
    them with the zero pressure beyond the wall, which makes the Poisson
    problem non-singular: no mean is removed from its right-hand side or
    solution.  The tangential stress on every wall is zero already: the node
    lines on the walls are dry, so the strain there carries no flux.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import operators as ops
from .derived import Prepared, inactive_dirichlet, laplacian
from .solvers import OK, coloured_diagonal, pcg


@dataclass
class Params:
    rho: float
    mu: float
    tau: float
    u_inf: float = 1.0
    gx: float = 0.0
    gy: float = 0.0
    pcg_tol: float = 1e-10
    pcg_maxit: int = 100000
    pred_tol: float = 1e-12
    pred_maxit: int = 500
    visc_form: str = "geometric"


@dataclass
class State:
    Ux: np.ndarray
    Uy: np.ndarray
    P: np.ndarray
    Phi: np.ndarray
    conv_prev: tuple = None
    n: int = 0


@dataclass
class StepInfo:
    pred_iters: int = 0
    pred_status: int = OK
    cg_iters: int = 0
    cg_relres: float = 0.0
    cg_status: int = OK
    div_max: float = 0.0
    div_rel: float = 0.0
    ke: float = 0.0
    extra: dict = field(default_factory=dict)


class Stepper:
    def __init__(self, pr: Prepared, prm: Params, Dx, Dy, h, jacobi=True):
        """jacobi=False skips probing the predictor's Jacobi diagonal (a
        stepper used only to apply the operators and to check residuals,
        not to solve)."""
        self.pr = pr
        self.prm = prm
        self.Dx = Dx
        self.Dy = Dy
        self.h = h
        c = pr.caps
        # mass matrix of the unknowns (the cut-cell volumes, floored)
        self.Vu = np.where(pr.act_u, pr.Mu if pr.Mu is not None else c["Vu"], 0.0)
        self.Vv = np.where(pr.act_v, pr.Mv if pr.Mv is not None else c["Vv"], 0.0)
        self.mask2 = np.stack([pr.act_u, pr.act_v])
        self.vD = self.dirichlet_viscous(Dx, Dy)
        # Jacobi diagonal of H, probed on unit combs
        self.Hdiag = self.Hdinv = None
        if jacobi:
            self.Hdiag = coloured_diagonal(self.apply_H, self.mask2.shape, self.mask2)
            self.Hdinv = np.where(self.mask2 & (self.Hdiag > 0), 1.0 / np.where(self.Hdiag > 0, self.Hdiag, 1.0),
                                  0.0)
        self.Pdinv = np.where(pr.act_p & (pr.diag > 0), 1.0 / np.where(pr.diag > 0, pr.diag, 1.0), 0.0)

    def dirichlet_viscous(self, Dx, Dy):
        """Dirichlet contribution of the viscous term, visc(strain(U~, D)) with
        U~ = D on the non-unknown faces and 0 on unknowns."""
        pr = self.pr
        ix, iy = inactive_dirichlet(pr, Dx, Dy)
        vdx, vdy = ops.viscous(pr.caps, ix, iy, Dx, Dy, self.prm.visc_form)
        return np.stack([np.where(pr.act_u, vdx, 0.0), np.where(pr.act_v, vdy, 0.0)])

    def set_dirichlet(self, Dx, Dy):
        """Make (Dx, Dy) the current Dirichlet data (time-dependent data: the
        next time level's, set inside the step)."""
        self.Dx, self.Dy = Dx, Dy
        self.vD = self.dirichlet_viscous(Dx, Dy)

    # --- linear operators -------------------------------------------------
    def apply_K(self, U2):
        z = np.zeros_like(U2[0])
        vx, vy = ops.viscous(self.pr.caps, np.where(self.pr.act_u, U2[0], 0.0),
                             np.where(self.pr.act_v, U2[1], 0.0), z, z, self.prm.visc_form)
        return np.stack([np.where(self.pr.act_u, vx, 0.0), np.where(self.pr.act_v, vy, 0.0)])

    def apply_H(self, U2):
        prm = self.prm
        V2 = np.stack([self.Vu, self.Vv])
        return (prm.rho / prm.tau) * V2 * U2 - prm.mu * self.apply_K(U2)

    def apply_A(self, phi):
        """A = -L (symmetric positive semi-definite)."""
        return -laplacian(self.pr, phi)

    # --- phases -------------------------------------------------------------
    def full_velocity(self, U2):
        return (np.where(self.pr.act_u, U2[0], self.Dx), np.where(self.pr.act_v, U2[1], self.Dy))

    def convection(self, Ux, Uy):
        cx, cy = ops.conv(self.pr.caps, Ux, Uy, Ux, Uy, self.Dx, self.Dy, self.Dx, self.Dy)
        return np.stack([np.where(self.pr.act_u, cx, 0.0), np.where(self.pr.act_v, cy, 0.0)])

    def predictor_rhs(self, st: State, conv_n, conv_prev, vD_next=None):
        """Right-hand side of eq:pm_prediction.  The explicit half of the
        viscous term is visc(strain(U^n, D^n)); the implicit half contributes
        the Dirichlet part of D^{n+1} (vD_next; the current data when D is
        constant in time)."""
        prm, pr = self.prm, self.pr
        vD_next = self.vD if vD_next is None else vD_next
        px, py = ops.pres(pr.caps, np.where(pr.act_p, st.P, 0.0))
        vx, vy = ops.viscous(pr.caps, st.Ux, st.Uy, self.Dx, self.Dy, prm.visc_form)
        V2 = np.stack([self.Vu, self.Vv])
        U2 = np.stack([st.Ux, st.Uy])
        g2 = np.stack([np.full_like(self.Vu, prm.gx), np.full_like(self.Vv, prm.gy)])
        rhs = ((prm.rho / prm.tau) * V2 * U2 - 1.5 * prm.rho * conv_n + 0.5 * prm.rho * conv_prev
               - np.stack([px, py]) + prm.mu * np.stack([vx, vy]) + prm.mu * vD_next
               + prm.rho * V2 * g2)
        return np.where(self.mask2, rhs, 0.0)

    def predict(self, st: State, info: StepInfo, D_next=None):
        """U* of eq:pm_prediction.  With D_next (time-dependent Dirichlet
        data), convection and the explicit viscous half use the current data
        D^n, the implicit half and U* on the non-unknown faces D^{n+1}, which
        becomes the current data for the rest of the step.  With outflow
        walls and no D_next, D^{n+1} is the outflow data of U^n."""
        if D_next is None and not self.pr.singular:
            D_next = self.outflow_data(st.Ux, st.Uy)
        conv_n = self.convection(st.Ux, st.Uy)
        conv_prev = conv_n if st.conv_prev is None else st.conv_prev
        vD_next = None if D_next is None else self.dirichlet_viscous(*D_next)
        rhs = self.predictor_rhs(st, conv_n, conv_prev, vD_next)
        if D_next is not None:
            self.Dx, self.Dy = D_next
            self.vD = vD_next
        U0 = np.stack([st.Ux, st.Uy])
        Us, it, rr, status = pcg(self.apply_H, rhs, U0, self.Hdinv, self.mask2,
                                 self.prm.pred_tol, self.prm.pred_maxit)
        info.pred_iters, info.pred_status = it, status
        return self.full_velocity(Us), conv_n

    def outflow_data(self, Ux, Uy):
        """D^{n+1} on the outflow walls from U^n (zero normal gradient); the
        current data everywhere else."""
        pr = self.pr
        Dx, Dy = self.Dx.copy(), self.Dy.copy()
        nx, ny = pr.nx, pr.ny
        if "W" in pr.outflow:
            Dx[:, 0] = np.where(pr.out_u[:, 0], Ux[:, 1], Dx[:, 0])
            Dy[1:ny, 0] = Uy[1:ny, 1]
        if "E" in pr.outflow:
            Dx[:, nx] = np.where(pr.out_u[:, nx], Ux[:, nx - 1], Dx[:, nx])
            Dy[1:ny, nx + 1] = Uy[1:ny, nx]
        if "S" in pr.outflow:
            Dy[0, :] = np.where(pr.out_v[0, :], Uy[1, :], Dy[0, :])
            Dx[0, 1:nx] = Ux[1, 1:nx]
        if "N" in pr.outflow:
            Dy[ny, :] = np.where(pr.out_v[ny, :], Uy[ny - 1, :], Dy[ny, :])
            Dx[ny + 1, 1:nx] = Ux[ny, 1:nx]
        return Dx, Dy

    def poisson_rhs(self, Ux, Uy):
        prm, pr = self.prm, self.pr
        b = (prm.rho / prm.tau) * ops.cont(pr.caps, Ux, Uy, self.Dx, self.Dy)
        b = np.where(pr.act_p, b, 0.0)
        if pr.n_active and pr.singular:
            b = np.where(pr.act_p, b - b[pr.act_p].sum() / pr.n_active, 0.0)
        return b

    def solve_poisson(self, b, phi0, info: StepInfo, tol=None, solver="pcg"):
        pr = self.pr
        tol = self.prm.pcg_tol if tol is None else tol
        if solver == "direct":
            from scipy.sparse.linalg import spsolve
            from .solvers import assemble, direct_zero_mean
            A, idx = assemble(self.apply_A, pr.act_p)
            x = np.zeros(pr.act_p.size)
            rhs = -b.ravel()[idx]
            x[idx] = direct_zero_mean(A, rhs) if pr.singular else spsolve(A.tocsc(), rhs)
            phi = x.reshape(b.shape)
            info.cg_iters, info.cg_status = 0, OK
        else:
            phi, it, rr, status = pcg(self.apply_A, -b, phi0, self.Pdinv, pr.act_p, tol,
                                      self.prm.pcg_maxit, zero_mean=pr.singular)
            info.cg_iters, info.cg_relres, info.cg_status = it, rr, status
        if pr.n_active and pr.singular:
            phi = np.where(pr.act_p, phi - phi[pr.act_p].sum() / pr.n_active, 0.0)
        return phi

    def correct(self, Ux, Uy, phi):
        prm, pr = self.prm, self.pr
        s = prm.tau / prm.rho
        Ux = Ux.copy()
        Uy = Uy.copy()
        dpx = np.zeros_like(phi)
        dpy = np.zeros_like(phi)
        dpx[:, :-1] = phi[:, 1:] - phi[:, :-1]
        dpy[:-1, :] = phi[1:, :] - phi[:-1, :]
        Ux = np.where(pr.proj_u, Ux - s * pr.gx * dpx, Ux)
        Uy = np.where(pr.proj_v, Uy - s * pr.gy * dpy, Uy)
        return Ux, Uy

    def pressure_update(self, P, phi):
        prm, pr = self.prm, self.pr
        Lphi = laplacian(pr, phi)
        V = pr.Vp if pr.Vp is not None else pr.caps["V"]
        Vinv = np.where(pr.act_p & (V > 0), 1.0 / np.where(V > 0, V, 1.0), 0.0)
        return np.where(pr.act_p, P + phi - (prm.tau * prm.mu / (2.0 * prm.rho)) * Vinv * Lphi, 0.0)

    def diagnostics(self, Ux, Uy, info: StepInfo):
        pr = self.pr
        d = ops.cont(pr.caps, Ux, Uy, self.Dx, self.Dy)
        dm = float(np.max(np.abs(d[pr.act_p]))) if pr.n_active else 0.0
        info.div_max = dm
        info.div_rel = dm / (self.prm.u_inf * self.h)
        info.ke = float(ops.kinetic(pr.caps, Ux, Uy)[1:-1, 1:-1].sum())
        return info

    def project(self, st: State, solver="pcg"):
        """Make st.U discretely divergence-free (initial condition)."""
        info = StepInfo()
        b = self.poisson_rhs(st.Ux, st.Uy)
        phi = self.solve_poisson(b, np.zeros_like(b), info, solver=solver)
        st.Ux, st.Uy = self.correct(st.Ux, st.Uy, phi)
        return self.diagnostics(st.Ux, st.Uy, info)

    def step(self, st: State, solver="pcg", D_next=None) -> StepInfo:
        """One PmII step; D_next: Dirichlet data of the next time level when
        it changes in time (else the current data holds at both levels)."""
        info = StepInfo()
        (Usx, Usy), conv_n = self.predict(st, info, D_next)
        b = self.poisson_rhs(Usx, Usy)
        phi = self.solve_poisson(b, st.Phi, info, solver=solver)
        Ux, Uy = self.correct(Usx, Usy, phi)
        st.P = self.pressure_update(st.P, phi)
        st.Ux, st.Uy, st.Phi = Ux, Uy, phi
        st.conv_prev = conv_n
        st.n += 1
        info.extra["b_norm"] = float(np.sqrt(np.sum(b ** 2)))
        return self.diagnostics(Ux, Uy, info)


def initial_state(pr: Prepared, Dx, Dy, u_inf, pert=None):
    """Free stream (u_inf, 0) on velocity unknowns plus an optional
    perturbation, D elsewhere; P = Phi = 0."""
    Ux = np.where(pr.act_u, u_inf, Dx)
    Uy = np.where(pr.act_v, 0.0, Dy)
    if pert is not None:
        Ux = np.where(pr.act_u, Ux + pert[0], Ux)
        Uy = np.where(pr.act_v, Uy + pert[1], Uy)
    z = np.zeros_like(Ux)
    return State(Ux, Uy, z.copy(), z.copy())
