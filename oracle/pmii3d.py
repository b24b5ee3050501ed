"""The projection step of projection method II in three dimensions, with
the velocity at rest on the walls and on the bodies (D = 0).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The operators of Sec. 4.1 carry over to three dimensions by adding an index
(Sec. 2.1, after eq:differentiation); with D = 0 the boundary terms of
eq:divergence vanish:
  cont(U, 0)_c  = sum over alpha of the difference, across cell c, of
                  A_alpha U_alpha                            (eq:divergence)
  pres_alpha(P) = A_alpha (difference of P across the face)  (eq:compatibility)
  M_alpha       = diag(V_alpha), the shifted control volumes (Sec. 4.5)
and the projection (Sec. 4.6) solves
  (tau / rho) cont(M^-1 pres(Phi), 0) = cont(U*, 0)           (eq:pm_poisson)
  U = U* - (tau / rho) M^-1 pres(Phi)                         (eq:pm_projection)
with Phi known up to a constant (every wall is closed): the solution with
zero mean over the pressure unknowns.  The density stands where the
two-dimensional step of this package puts it (the time step of eq:pm_poisson
over rho, as the pressure gradient is divided by rho in the momentum
equation).

Readings, the same as in two dimensions (derived.py):
  * a face is a velocity unknown when it is interior to the box, its
    control volume has fluid (V_alpha > 0) and it is open (A_alpha > 0); every
    other face holds D = 0;
  * M_f = max(V_f, theta hx hy hz) on the unknowns (theta = 0: M = diag(V));
  * the Poisson face weight is c_f = A_f^2 / M_f; a cell is a pressure
    unknown when it has fluid and lies in the largest set of cells connected
    through faces with c_f > 0, and c_f is kept only between two such cells;
  * the projection corrects the faces with c_f > 0; the other unknowns keep
    U*.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components

from workloads.three_d import Grid3

from . import solvers


@dataclass
class Prep3:
    grid: Grid3
    A: tuple          # (Ax, Ay, Az) face areas
    act: tuple        # bool velocity unknowns per face grid
    M: tuple          # mass of the unknowns (0 elsewhere)
    c: tuple          # Poisson face weights A^2 / M between pressure unknowns
    gfac: tuple       # corrector factors A / M where c > 0
    act_p: np.ndarray  # bool pressure unknowns
    diag: np.ndarray   # diagonal of -L on the pressure unknowns

    @property
    def n_active(self):
        return int(self.act_p.sum())


def _shift(a, axis, d):
    """b[..., i, ...] = a[..., i + d, ...] along a field axis (0 x, 1 y, 2 z),
    zero where i + d falls off the array."""
    ax = 2 - axis
    out = np.zeros_like(a)
    src = [slice(None)] * 3
    dst = [slice(None)] * 3
    if d > 0:
        src[ax], dst[ax] = slice(d, None), slice(None, -d)
    else:
        src[ax], dst[ax] = slice(None, d), slice(-d, None)
    out[tuple(dst)] = a[tuple(src)]
    return out


def prepare(caps: dict, g: Grid3, mass_floor: float = 0.0) -> Prep3:
    sh = g.shape
    k, j, i = np.indices(sh)
    ci, cj, ck = (i >= 1) & (i <= g.nx), (j >= 1) & (j <= g.ny), (k >= 1) & (k <= g.nz)
    fi, fj, fk = (i >= 1) & (i <= g.nx - 1), (j >= 1) & (j <= g.ny - 1), (k >= 1) & (k <= g.nz - 1)
    interior = (fi & cj & ck, ci & fj & ck, ci & cj & fk)
    A = (caps["Ax"], caps["Ay"], caps["Az"])
    Vf = (caps["Vx"], caps["Vy"], caps["Vz"])
    floor = mass_floor * g.hx * g.hy * g.hz
    act = tuple(interior[a] & (Vf[a] > 0.0) & (A[a] > 0.0) for a in range(3))
    M = tuple(np.where(act[a], np.maximum(Vf[a], floor), 0.0) for a in range(3))
    c = [np.where(act[a], A[a] ** 2 / np.where(act[a], M[a], 1.0), 0.0) for a in range(3)]
    fluid = ci & cj & ck & (caps["V"] > 0.0)
    idx = -np.ones(sh, dtype=np.int64)
    nf = int(fluid.sum())
    idx[fluid] = np.arange(nf)
    rows, cols = [], []
    for a in range(3):
        e = (c[a] > 0.0) & fluid & _shift(fluid, a, 1)
        kk, jj, ii = np.nonzero(e)
        nb = (kk + (a == 2), jj + (a == 1), ii + (a == 0))
        rows.append(idx[kk, jj, ii])
        cols.append(idx[nb])
    r, cc = np.concatenate(rows), np.concatenate(cols)
    act_p = np.zeros(sh, dtype=bool)
    if nf:
        ncomp, lab = connected_components(coo_matrix((np.ones(len(r)), (r, cc)), shape=(nf, nf)), directed=False)
        act_p[fluid] = lab == int(np.argmax(np.bincount(lab, minlength=ncomp)))
    c = tuple(np.where(act_p & _shift(act_p, a, 1), c[a], 0.0) for a in range(3))
    gfac = tuple(np.where(c[a] > 0.0, A[a] / np.where(c[a] > 0.0, M[a], 1.0), 0.0) for a in range(3))
    diag = sum(c[a] + _shift(c[a], a, -1) for a in range(3))
    return Prep3(g, A, act, M, c, gfac, act_p, np.where(act_p, diag, 0.0))


def cont(A: tuple, U: tuple) -> np.ndarray:
    """eq:divergence with D = 0 on the real cells: for each direction, the
    flux A U through the cell's high face minus that through its low face."""
    out = np.zeros_like(U[0])
    for a in range(3):
        F = A[a] * U[a]
        out += F - _shift(F, a, -1)
    out[0, :, :] = out[-1, :, :] = 0.0
    out[:, 0, :] = out[:, -1, :] = 0.0
    out[:, :, 0] = out[:, :, -1] = 0.0
    return out


def pres(A: tuple, P: np.ndarray) -> tuple:
    """eq:compatibility: on each face, A times the difference of P across it
    (the cell above minus the cell below)."""
    return tuple(A[a] * (_shift(P, a, 1) - P) for a in range(3))


def laplacian(pr: Prep3, phi: np.ndarray) -> np.ndarray:
    """L phi = cont(M^-1 pres(phi), 0) on the pressure unknowns:
    sum over the six faces of c_f (phi_nb - phi_c)."""
    flux = tuple(pr.c[a] * (_shift(phi, a, 1) - phi) for a in range(3))
    out = sum(flux[a] - _shift(flux[a], a, -1) for a in range(3))
    return np.where(pr.act_p, out, 0.0)


def matrix(pr: Prep3):
    """-L restricted to the pressure unknowns (sparse) and their flat
    indices."""
    return solvers.assemble(lambda x: -laplacian(pr, x), pr.act_p)


def rhs(pr: Prep3, U: tuple, rho: float, tau: float) -> np.ndarray:
    """b = -(rho / tau) cont(U*, 0) on the pressure unknowns, minus its mean
    over them (the problem is singular; Sec. 4.6)."""
    Um = tuple(np.where(pr.act[a], U[a], 0.0) for a in range(3))
    b = np.where(pr.act_p, -(rho / tau) * cont(pr.A, Um), 0.0)
    if pr.n_active:
        b = np.where(pr.act_p, b - b[pr.act_p].sum() / pr.n_active, 0.0)
    return b


def correct(pr: Prep3, U: tuple, phi: np.ndarray, rho: float, tau: float) -> tuple:
    """eq:pm_projection on the faces with c > 0; the other unknowns keep U*,
    every other face holds D = 0."""
    G = pres(pr.A, phi)
    return tuple(np.where(pr.c[a] > 0.0, U[a] - (tau / rho) * np.where(pr.c[a] > 0.0, G[a] / np.where(
        pr.c[a] > 0.0, pr.M[a], 1.0), 0.0), np.where(pr.act[a], U[a], 0.0)) for a in range(3))


def project(pr: Prep3, U: tuple, rho: float, tau: float, solver: str = "direct", tol: float = 1e-13,
            maxit: int = 100000):
    """The projection step: returns (Phi, U, info).  solver 'direct' is the
    zero-mean sparse solve; 'pcg' the Jacobi-PCG of solvers.pcg."""
    b = rhs(pr, U, rho, tau)
    info = {"iterations": 0, "status": solvers.OK}
    if solver == "direct":
        K, idx = matrix(pr)
        x = solvers.direct_zero_mean(K, b.ravel()[idx])
        phi = np.zeros(pr.grid.shape)
        phi.ravel()[idx] = x
    else:
        dinv = np.where(pr.act_p, 1.0 / np.where(pr.act_p, pr.diag, 1.0), 0.0)
        phi, it, rel, st = solvers.pcg(lambda x: -laplacian(pr, x), b, np.zeros(pr.grid.shape), dinv, pr.act_p,
                                       tol, maxit, zero_mean=True)
        phi = np.where(pr.act_p, phi - phi[pr.act_p].mean(), 0.0)
        info = {"iterations": it, "status": st, "rel_residual": rel}
    Un = correct(pr, U, phi, rho, tau)
    div = cont(pr.A, Un)
    flux = max(float(np.max(np.abs(pr.A[a] * Un[a]))) for a in range(3))
    info["div_rel"] = float(np.max(np.abs(np.where(pr.act_p, div, 0.0)))) / flux if flux > 0 else 0.0
    return phi, Un, info
