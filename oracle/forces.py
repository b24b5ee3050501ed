"""Force of the fluid on the bodies: a reading for the drag and lift
coefficients that the paper reports for its cylinder and airfoil cases
(Sec. 5) without stating a discrete formula.

Test infrastructure: only the tests, the smoke check and the benchmark's
CPU baseline use this package.

Reading.  The discrete momentum equation (eq:semidiscrete) exchanges
momentum with the bodies through the capacities: summed over the faces, the
pressure gradient pres (eq:compatibility) and the viscous term visc (Sec.
4.3) telescope, and what remains of a field that vanishes near the box's
walls is a sum over the cut cells and nodes.  The force on the bodies is
minus what the fluid receives there:

  pressure   F^p_x = sum_cells P_ij (A^x_{i-1/2,j} - A^x_{i+1/2,j})
             F^p_y = sum_cells P_ij (A^y_{i,j-1/2} - A^y_{i,j+1/2})
  viscous    F^v_x = 2 mu [ sum_cells S_xx,ij (B^xx_{i+1/2,j} - B^xx_{i-1/2,j})
                          + sum_nodes S_x,n (B^xy above n - B^xy below n) ]
             F^v_y = 2 mu [ sum_cells S_yy,ij (B^yy_{i,j+1/2} - B^yy_{i,j-1/2})
                          + sum_nodes S_y,n (B^yx right of n - B^yx left of n) ]

with S the strain of eq:diag and eq:offdiag on (U, D) (S_x, S_y: the node
strain seen by the x and y rows) and 2 mu the stress of the two viscous
halves of eq:pm_prediction.  The node sums leave out the nodes on the box's
walls (whose terms are the walls' shear, not the bodies'); every uncut cell
and node contributes zero, so only the cells and nodes cut by a body count
(bodies must stay clear of the walls).  A^x_w - A^x_e is the x-projection of
the body's surface in the cell, so F^p is the integral of the cell pressure
over it; the error is first order in h.  Coefficients: C = F / (rho U^2 L / 2)
with the body's reference length L (diameter or chord)."""

from __future__ import annotations

import numpy as np

from . import operators as ops


def forces(c, P, Ux, Uy, Dx, Dy, mu, visc_form="geometric", pmask=None):
    """(F^p_x, F^p_y, F^v_x, F^v_y) on all bodies.  P: cell pressures (zero
    off the pressure unknowns, or pass pmask); U, D as for ops.strain."""
    P = np.asarray(P, dtype=np.float64)
    if pmask is not None:
        P = np.where(pmask, P, 0.0)
    ny, nx = P.shape[0] - 2, P.shape[1] - 2
    s = np.s_[1:-1, 1:-1]
    Ax, Ay = c["Ax"], c["Ay"]
    fpx = float(np.sum(P[s] * (Ax[1:-1, :-2] - Ax[1:-1, 1:-1])))
    fpy = float(np.sum(P[s] * (Ay[:-2, 1:-1] - Ay[1:-1, 1:-1])))
    Sxx, Syy, Sx, Sy = ops.strain(c, Ux, Uy, Dx, Dy, visc_form)
    Bxx, Byy, Bxy, Byx = c["Bxx"], c["Byy"], c["Bxy"], c["Byx"]
    vx = np.sum(Sxx[s] * (Bxx[1:-1, 1:-1] - Bxx[1:-1, :-2]))
    vy = np.sum(Syy[s] * (Byy[1:-1, 1:-1] - Byy[:-2, 1:-1]))
    # node (j, i) is (x_{i+1/2}, y_{j+1/2}); the x-faces below and above it
    # are (j, i) and (j+1, i), the y-faces left and right (j, i) and (j, i+1)
    vx += np.sum(Sx[1:ny, 0:nx + 1] * (Bxy[2:ny + 1, 0:nx + 1] - Bxy[1:ny, 0:nx + 1]))
    vy += np.sum(Sy[0:ny + 1, 1:nx] * (Byx[0:ny + 1, 2:nx + 1] - Byx[0:ny + 1, 1:nx]))
    return fpx, fpy, float(2.0 * mu * vx), float(2.0 * mu * vy)


def coefficients(F, rho, u_ref, length):
    """(C_d, C_l) from the total force (F^p + F^v)."""
    q = 0.5 * rho * u_ref * u_ref * length
    return (F[0] + F[2]) / q, (F[1] + F[3]) / q
