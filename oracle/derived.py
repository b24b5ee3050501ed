"""Activity masks and coefficient fields for the projection step (Sec. 4.6).

Readings taken where the paper is silent:
  * A velocity face is an unknown when it is interior to the box (not on a
    wall that is normal to it) and its staggered control volume has fluid.
    Every other face holds its Dirichlet value, U = D.
  * The Poisson operator is cont(M^-1 pres(Phi), 0): face coefficient
    c_f = A_f^2 / V_f (weight 'volume'), which is the paper's statement with
    the mass matrix of Sec. 4.5 made explicit; weight 'literal' drops the
    mass matrix (c_f = A_f^2).
  * A cell is a pressure unknown when it has fluid and belongs to the largest
    set of cells connected through faces with c_f > 0; cells outside it (fluid
    pockets cut off by the body) hold Phi = P = 0.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components

from .calculus import safe_inv


@dataclass
class Prepared:
    caps: dict
    nx: int
    ny: int
    act_u: np.ndarray   # bool, x-face unknowns
    act_v: np.ndarray   # bool, y-face unknowns
    act_p: np.ndarray   # bool, pressure unknowns
    cx: np.ndarray      # Poisson face coefficients (x-faces)
    cy: np.ndarray
    gx: np.ndarray      # corrector factors A_f / V_f (x-faces)
    gy: np.ndarray
    diag: np.ndarray    # diagonal of -L (cells)
    n_active: int


def prepare(caps: dict, nx: int, ny: int, weight: str = "volume") -> Prepared:
    shape = (ny + 2, nx + 2)
    J, I = np.indices(shape)
    act_u = (I >= 1) & (I <= nx - 1) & (J >= 1) & (J <= ny) & (caps["Vu"] > 0.0)
    act_v = (I >= 1) & (I <= nx) & (J >= 1) & (J <= ny - 1) & (caps["Vv"] > 0.0)
    if weight == "volume":
        wu, wv = safe_inv(caps["Vu"]), safe_inv(caps["Vv"])
    elif weight == "literal":
        wu, wv = np.ones(shape), np.ones(shape)
    else:
        raise ValueError(weight)
    cx = np.where(act_u, caps["Ax"] ** 2 * wu, 0.0)
    cy = np.where(act_v, caps["Ay"] ** 2 * wv, 0.0)

    fluid = (I >= 1) & (I <= nx) & (J >= 1) & (J <= ny) & (caps["V"] > 0.0)
    idx = -np.ones(shape, dtype=np.int64)
    idx[fluid] = np.arange(int(fluid.sum()))
    rows, cols = [], []
    ex = (cx > 0.0) & fluid & np.roll(fluid, -1, axis=1)
    jj, ii = np.nonzero(ex)
    rows.append(idx[jj, ii])
    cols.append(idx[jj, ii + 1])
    ey = (cy > 0.0) & fluid & np.roll(fluid, -1, axis=0)
    jj, ii = np.nonzero(ey)
    rows.append(idx[jj, ii])
    cols.append(idx[jj + 1, ii])
    nf = int(fluid.sum())
    r = np.concatenate(rows) if rows else np.zeros(0, np.int64)
    cc = np.concatenate(cols) if cols else np.zeros(0, np.int64)
    G = coo_matrix((np.ones(len(r)), (r, cc)), shape=(nf, nf))
    ncomp, lab = connected_components(G, directed=False)
    act_p = np.zeros(shape, dtype=bool)
    if nf:
        sizes = np.bincount(lab, minlength=ncomp)
        big = int(np.argmax(sizes))
        act_p[fluid] = lab == big
    # a face couples pressures only between two active cells
    cx = np.where(act_p & np.roll(act_p, -1, axis=1), cx, 0.0)
    cy = np.where(act_p & np.roll(act_p, -1, axis=0), cy, 0.0)
    gx = np.where(cx > 0.0, caps["Ax"] * wu, 0.0)
    gy = np.where(cy > 0.0, caps["Ay"] * wv, 0.0)
    diag = np.zeros(shape)
    diag[1:-1, 1:-1] = cx[1:-1, 1:-1] + cx[1:-1, :-2] + cy[1:-1, 1:-1] + cy[:-2, 1:-1]
    diag = np.where(act_p, diag, 0.0)
    return Prepared(caps, nx, ny, act_u, act_v, act_p, cx, cy, gx, gy, diag, int(act_p.sum()))


def laplacian(pr: Prepared, phi):
    """(L phi)_ij = sum over the four faces of c_f (phi_nb - phi_ij), active cells."""
    out = np.zeros_like(phi)
    s = np.s_[1:-1, 1:-1]
    out[s] = (pr.cx[1:-1, 1:-1] * (phi[1:-1, 2:] - phi[s])
              - pr.cx[1:-1, :-2] * (phi[s] - phi[1:-1, :-2])
              + pr.cy[1:-1, 1:-1] * (phi[2:, 1:-1] - phi[s])
              - pr.cy[:-2, 1:-1] * (phi[s] - phi[:-2, 1:-1]))
    return np.where(pr.act_p, out, 0.0)


def inactive_dirichlet(pr: Prepared, Dx, Dy):
    """Velocity field equal to D on the non-unknown faces and 0 on unknowns."""
    return np.where(pr.act_u, 0.0, Dx), np.where(pr.act_v, 0.0, Dy)
