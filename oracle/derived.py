"""Activity masks and coefficient fields for the projection step (Sec. 4.6).

Readings taken where the paper is silent:
  * A velocity face is an unknown when it is interior to the box (not on a
    wall that is normal to it), its staggered control volume has fluid and
    the face itself is open (A > 0).  Every other face holds its Dirichlet
    value, U = D.  A closed face carries no flux and takes no part in the
    projection; left free, the velocity of such a face (the sliver between
    the two sides of a thin trailing edge, say) is driven by the explicit
    convective term divided by a tiny mass and grows without bound.
  * Small control volumes: the paper does not treat them.  Every volume the
    step divides by is at least vol_floor = theta hx hy (the mass matrix M
    of the velocity unknowns, M_f = max(V_f, vol_floor), and the cell volume
    of the pressure update).  Without it, a sliver cell with open faces
    turns the pressure update's volume average V^-1 L Phi into a spike that
    the next predictor feeds back; the NACA section's trailing edge at 4096
    x 2048 then grows by orders of magnitude per step.  theta = 0.05 removes
    that growth; theta = 0 is M = V exactly.
  * The Poisson operator is cont(M^-1 pres(Phi), 0): face coefficient
    c_f = A_f^2 / V_f (weight 'volume'), which is the paper's statement with
    the mass matrix of Sec. 4.5 made explicit; weight 'literal' drops the
    mass matrix (c_f = A_f^2).
  * A cell is a pressure unknown when it has fluid and belongs to the largest
    set of cells connected through faces with c_f > 0; cells outside it (fluid
    pockets cut off by the body) hold Phi = P = 0.
  * Outflow walls (end of Sec. 4.6): the faces on such a wall, normal to it,
    are corrected by the projection like interior unknowns, and the pressure
    beyond the wall (the ghost cell) is held at zero, so pres on those faces
    is still the negative transpose of cont (eq:compatibility).  Their
    control volume is the staggered one that straddles the wall, mass
    M_f = max(V_f, vol_floor), and the Poisson operator gains their weight
    c_f on the diagonal of the cell inside: with one such face it is no
    longer singular.
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
    Mu: np.ndarray = None    # mass matrix of the x-face unknowns (0 elsewhere)
    Mv: np.ndarray = None
    Vp: np.ndarray = None    # cell volumes of the pressure update (floored)
    out_u: np.ndarray = None  # bool, x-faces on outflow walls that the projection corrects
    out_v: np.ndarray = None
    outflow: str = ""        # the outflow walls, letters of "WESN"
    singular: bool = True    # no outflow face: Phi is known up to a constant

    @property
    def proj_u(self):
        """x-faces the projection corrects: unknowns and outflow faces."""
        return self.act_u if self.out_u is None else self.act_u | self.out_u

    @property
    def proj_v(self):
        return self.act_v if self.out_v is None else self.act_v | self.out_v


def outflow_faces(caps: dict, nx: int, ny: int, outflow: str):
    """Faces normal to an outflow wall (W: i = 0, E: i = nx in the x-face
    layout; S: j = 0, N: j = ny in the y-face layout) whose staggered control
    volume has fluid and whose aperture is open."""
    shape = (ny + 2, nx + 2)
    J, I = np.indices(shape)
    wall_u = np.zeros(shape, bool)
    wall_v = np.zeros(shape, bool)
    rows, cols = (J >= 1) & (J <= ny), (I >= 1) & (I <= nx)
    if "W" in outflow:
        wall_u |= rows & (I == 0)
    if "E" in outflow:
        wall_u |= rows & (I == nx)
    if "S" in outflow:
        wall_v |= cols & (J == 0)
    if "N" in outflow:
        wall_v |= cols & (J == ny)
    out_u = wall_u & (caps["Vu"] > 0.0) & (caps["Ax"] > 0.0)
    out_v = wall_v & (caps["Vv"] > 0.0) & (caps["Ay"] > 0.0)
    return out_u, out_v


def prepare(caps: dict, nx: int, ny: int, weight: str = "volume", vol_floor: float = 0.0,
            outflow: str = "") -> Prepared:
    """vol_floor: the smallest volume the step divides by (theta hx hy): the
    mass matrix of the velocity unknowns is max(V_f, vol_floor) and the
    pressure update divides by max(V, vol_floor).  outflow: the walls (any of
    "WESN") with a homogeneous Neumann velocity and a zero pressure beyond."""
    if any(w not in "WESN" for w in outflow):
        raise ValueError(outflow)
    shape = (ny + 2, nx + 2)
    J, I = np.indices(shape)
    act_u = (I >= 1) & (I <= nx - 1) & (J >= 1) & (J <= ny) & (caps["Vu"] > 0.0) & (caps["Ax"] > 0.0)
    act_v = (I >= 1) & (I <= nx) & (J >= 1) & (J <= ny - 1) & (caps["Vv"] > 0.0) & (caps["Ay"] > 0.0)
    out_u, out_v = outflow_faces(caps, nx, ny, outflow)
    Mu = np.where(act_u | out_u, np.maximum(caps["Vu"], vol_floor), 0.0)
    Mv = np.where(act_v | out_v, np.maximum(caps["Vv"], vol_floor), 0.0)
    if weight == "volume":
        wu, wv = safe_inv(Mu), safe_inv(Mv)
    elif weight == "literal":
        wu, wv = np.ones(shape), np.ones(shape)
    else:
        raise ValueError(weight)
    cx = np.where(act_u | out_u, caps["Ax"] ** 2 * wu, 0.0)
    cy = np.where(act_v | out_v, caps["Ay"] ** 2 * wv, 0.0)

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
    # a face couples pressures only between two active cells; an outflow face
    # needs an active cell inside the wall (beyond it the pressure is zero)
    cx = np.where((act_p & np.roll(act_p, -1, axis=1)) | (out_u & (act_p | np.roll(act_p, -1, axis=1))), cx, 0.0)
    cy = np.where((act_p & np.roll(act_p, -1, axis=0)) | (out_v & (act_p | np.roll(act_p, -1, axis=0))), cy, 0.0)
    out_u = out_u & (cx > 0.0)
    out_v = out_v & (cy > 0.0)
    gx = np.where(cx > 0.0, caps["Ax"] * wu, 0.0)
    gy = np.where(cy > 0.0, caps["Ay"] * wv, 0.0)
    diag = np.zeros(shape)
    diag[1:-1, 1:-1] = cx[1:-1, 1:-1] + cx[1:-1, :-2] + cy[1:-1, 1:-1] + cy[:-2, 1:-1]
    diag = np.where(act_p, diag, 0.0)
    Vp = np.where(caps["V"] > 0.0, np.maximum(caps["V"], vol_floor), 0.0)
    singular = not (out_u.any() or out_v.any())
    return Prepared(caps, nx, ny, act_u, act_v, act_p, cx, cy, gx, gy, diag, int(act_p.sum()), Mu, Mv, Vp,
                    out_u, out_v, "".join(w for w in "WESN" if w in outflow), singular)


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
