"""Discrete operators of the method (Sec. 2.3 and Sec. 4), in two forms.

  *_lit  the operators exactly as the paper writes them, composed from the
         difference / interpolation primitives of oracle.calculus
         (eq:gradD, eq:divN, eq:divergence, eq:compatibility, eq:diag,
         eq:offdiag, eq:divD, eq:convective, kinetic of Sec. 4.5);
  plain  the same operators expanded by hand into index form (the algebra is
         stated in each docstring).  The tests check that both forms agree.

All arrays use the (ny+2, nx+2) layout of oracle.geometry.  `c` is the dict of
capacities returned by oracle.geometry.capacities (or any dict with the same
keys).  Outputs are zero outside the index range stated for each operator.
"""

from __future__ import annotations

import numpy as np

from .calculus import F, d_x, d_y, i_x, i_y, safe_inv

# ---------------------------------------------------------------------------
# literal compositions
# ---------------------------------------------------------------------------


def gradD_lit(A, B, W, T, D, axis):
    """Scalar cut-cell gradient (eq:gradD) along `axis` ('x' or 'y').
    T, D, B at cells; A, W at faces of that axis.  Result at those faces."""
    d, m = (d_x, i_x) if axis == "x" else (d_y, i_y)
    fpos = "u" if axis == "x" else "v"
    T, D, B = F(T, "c"), F(D, "c"), F(B, "c")
    A, W = F(A, fpos), F(W, fpos)
    core = d(B * T) + d((m(A) - B) * D) - m(d(A) * D)
    return (core * safe_inv(W.a)).a


def grad_v2_lit(A, V, T, D, axis):
    """The superseded tentative C-grid gradient of Sec. 2.1 (eq:grad-v2), with
    capacities interpolated to the staggered location.  Kept only for the
    negative test of Sec. 2.2."""
    d, m = (d_x, i_x) if axis == "x" else (d_y, i_y)
    fpos = "u" if axis == "x" else "v"
    A = F(A, fpos)
    T, D, V = F(T, "c"), F(D, "c"), F(V, "c")
    core = d(m(A) * T) - m(d(A) * D)
    return (core * safe_inv(m(V).a)).a


def divN_lit(A, B, Q, N, axis):
    """One axis of the cut-cell divergence (eq:divN): Q, N, A at faces of
    `axis`, B at cells.  Result at cells."""
    d, m = (d_x, i_x) if axis == "x" else (d_y, i_y)
    fpos = "u" if axis == "x" else "v"
    A, Q, N = F(A, fpos), F(Q, fpos), F(N, fpos)
    B = F(B, "c")
    return (d(A * Q) + d((m(B) - A) * N) - m(d(B) * N)).a


def cont_lit(c, Ux, Uy, Dx, Dy):
    """Volume-integrated divergence cont(U, D) (eq:divergence), at cells."""
    return divN_lit(c["Ax"], c["Bx"], Ux, Dx, "x") + divN_lit(c["Ay"], c["By"], Uy, Dy, "y")


def pres_lit(c, P):
    """pres_alpha(P) = A_alpha dP/dxi_alpha (eq:compatibility), at faces."""
    Pf = F(P, "c")
    return (F(c["Ax"], "u") * d_x(Pf)).a, (F(c["Ay"], "v") * d_y(Pf)).a


def strain_lit(c, Ux, Uy, Dx, Dy):
    """Strain rate as printed: S_xx, S_yy (eq:diag) at cells and S_xy
    (eq:offdiag) at nodes, with its two separate node volumes W^xy, W^yx."""
    ux, uy, dx, dy = F(Ux, "u"), F(Uy, "v"), F(Dx, "u"), F(Dy, "v")
    Bxx, Axx, Wxx = F(c["Bxx"], "u"), F(c["Axx"], "c"), c["Wxx"]
    Byy, Ayy, Wyy = F(c["Byy"], "v"), F(c["Ayy"], "c"), c["Wyy"]
    Sxx = (d_x(Bxx * ux) + d_x((i_x(Axx) - Bxx) * dx) - i_x(d_x(Axx) * dx)) * safe_inv(Wxx)
    Syy = (d_y(Byy * uy) + d_y((i_y(Ayy) - Byy) * dy) - i_y(d_y(Ayy) * dy)) * safe_inv(Wyy)
    Bxy, Axy = F(c["Bxy"], "u"), F(c["Axy"], "n")
    Byx, Ayx = F(c["Byx"], "v"), F(c["Ayx"], "n")
    gx = d_y(Bxy * ux) + d_y((i_y(Axy) - Bxy) * dx) - i_y(d_y(Axy) * dx)
    gy = d_x(Byx * uy) + d_x((i_x(Ayx) - Byx) * dy) - i_x(d_x(Ayx) * dy)
    Sxy = gx * (0.5 * safe_inv(c["Wxy"])) + gy * (0.5 * safe_inv(c["Wyx"]))
    return Sxx.a, Syy.a, Sxy.a


def visc_lit(c, Sxx, Syy, Sxy_x, Sxy_y=None):
    """visc_alpha(S) = sum_beta B_alpha beta dS_alpha beta/dxi_beta (Sec. 4.3).
    Sxy_x is the node strain seen by the x-momentum rows and Sxy_y the one
    seen by the y rows (identical for the paper's single S_xy)."""
    if Sxy_y is None:
        Sxy_y = Sxy_x
    vx = F(c["Bxx"], "u") * d_x(F(Sxx, "c")) + F(c["Bxy"], "u") * d_y(F(Sxy_x, "n"))
    vy = F(c["Byx"], "v") * d_x(F(Sxy_y, "n")) + F(c["Byy"], "v") * d_y(F(Syy, "c"))
    return vx.a, vy.a


def conv_lit(c, Ux, Uy, Utx, Uty, Dx, Dy, Dtx, Dty):
    """Convective transport conv_alpha(U, U+, D, D+) (eq:convective)."""
    ux, uy = F(Ux, "u"), F(Uy, "v")
    utx, uty = F(Utx, "u"), F(Uty, "v")
    dx, dy, dtx, dty = F(Dx, "u"), F(Dy, "v"), F(Dtx, "u"), F(Dty, "v")
    Ax, Ay, Bx, By = F(c["Ax"], "u"), F(c["Ay"], "v"), F(c["Bx"], "c"), F(c["By"], "c")
    fx = Ax * ux
    fy = Ay * uy
    # alpha = x
    cx = d_x(i_x(fx) * i_x(utx)) + d_y(i_x(fy) * i_y(utx))
    brx = (d_x(i_x((i_x(Bx) - Ax) * dx)) - i_x(i_x(d_x(Bx) * dx))
           + d_y(i_x((i_y(By) - Ay) * dy)) - i_x(i_y(d_y(By) * dy)))
    cx = cx + brx * (0.5 * (utx + dtx))
    # alpha = y
    cy = d_x(i_y(fx) * i_x(uty)) + d_y(i_y(fy) * i_y(uty))
    bry = (d_x(i_y((i_x(Bx) - Ax) * dx)) - i_y(i_x(d_x(Bx) * dx))
           + d_y(i_y((i_y(By) - Ay) * dy)) - i_y(i_y(d_y(By) * dy)))
    cy = cy + bry * (0.5 * (uty + dty))
    return cx.a, cy.a


def kinetic_lit(c, Ux, Uy):
    """kinetic(U) = sum_alpha 1/2 overbar^alpha(V_alpha U_alpha U_alpha), at cells."""
    ux, uy = F(Ux, "u"), F(Uy, "v")
    return (i_x(F(c["Vu"], "u") * ux * ux) * 0.5 + i_y(F(c["Vv"], "v") * uy * uy) * 0.5).a


# ---------------------------------------------------------------------------
# expanded index forms
# ---------------------------------------------------------------------------


def _z(a):
    return np.zeros_like(np.asarray(a, dtype=np.float64))


def cont(c, Ux, Uy, Dx, Dy):
    """cont at cells i=1..nx, j=1..ny.  Expanding eq:divergence, the B of the
    neighbouring cells cancels and what remains is
      A^x_{i+1/2}(U-D)_{i+1/2} - A^x_{i-1/2}(U-D)_{i-1/2} + B^x_ij (D_{i+1/2}-D_{i-1/2})
    plus the same along y."""
    Ax, Ay, Bx, By = c["Ax"], c["Ay"], c["Bx"], c["By"]
    ex = Ux - Dx
    ey = Uy - Dy
    out = _z(Ux)
    s = np.s_[1:-1, 1:-1]
    out[s] = (Ax[1:-1, 1:-1] * ex[1:-1, 1:-1] - Ax[1:-1, :-2] * ex[1:-1, :-2]
              + Bx[s] * (Dx[1:-1, 1:-1] - Dx[1:-1, :-2])
              + Ay[1:-1, 1:-1] * ey[1:-1, 1:-1] - Ay[:-2, 1:-1] * ey[:-2, 1:-1]
              + By[s] * (Dy[1:-1, 1:-1] - Dy[:-2, 1:-1]))
    return out


def pres(c, P):
    """pres at every real face: A^x_{i+1/2}(P_{i+1}-P_i) for i = 0..nx, rows
    1..ny (pressure outside the box taken as 0, which makes pres the exact
    negative transpose of U -> cont(U, 0) over all real faces)."""
    Pz = np.array(P, dtype=np.float64)
    Pz[0, :] = 0.0
    Pz[-1, :] = 0.0
    Pz[:, 0] = 0.0
    Pz[:, -1] = 0.0
    px = _z(P)
    py = _z(P)
    px[1:-1, 0:-1] = c["Ax"][1:-1, 0:-1] * (Pz[1:-1, 1:] - Pz[1:-1, :-1])
    py[0:-1, 1:-1] = c["Ay"][0:-1, 1:-1] * (Pz[1:, 1:-1] - Pz[:-1, 1:-1])
    return px, py


def node_coefficients(c, form="geometric"):
    """Weights of the node strain.  S seen by the x rows is
    (nxx*gx + nxy*gy)/2 and by the y rows (nyx*gx + nyy*gy)/2, where gx and
    gy are the bracketed differences of eq:offdiag.
      'literal'   : nxx = nyx = 1/W^xy, nxy = nyy = 1/W^yx (the printed form,
                    not symmetric where W^xy != W^yx)
      'geometric' : nxx = 1/W^xy, nyy = 1/W^yx, nxy = nyx = 1/sqrt(W^xy W^yx)
                    (symmetric, equal to the printed form wherever the two
                    node volumes agree)
      'mean'      : all four = 1/Wbar, Wbar = (W^xy + W^yx)/2."""
    wxy, wyx = c["Wxy"], c["Wyx"]
    ixy, iyx = safe_inv(wxy), safe_inv(wyx)
    if form == "literal":
        return ixy, iyx, ixy, iyx
    if form == "geometric":
        g = safe_inv(np.sqrt(wxy * wyx))
        return ixy, g, g, iyx
    if form == "mean":
        m = safe_inv(0.5 * (wxy + wyx))
        return m, m, m, m
    raise ValueError(form)


def strain(c, Ux, Uy, Dx, Dy, form="geometric"):
    """Strain rate in index form (eq:diag, eq:offdiag expanded):
      W^xx_ij S_xx = B^xx_{i+1/2}(U-D)_{i+1/2} - B^xx_{i-1/2}(U-D)_{i-1/2}
                     + A^xx_ij (D_{i+1/2} - D_{i-1/2})         cells 1..nx x 1..ny
      gx = B^xy_{j+1}(U-D)_{j+1} - B^xy_j (U-D)_j + A^xy (D_{j+1} - D_j)  at node
      gy = B^yx_{i+1}(V-D)_{i+1} - B^yx_i (V-D)_i + A^yx (D_{i+1} - D_i)   at node
    nodes i = 0..nx, j = 0..ny.  Returns Sxx, Syy, Sx (node strain for the x
    rows), Sy (for the y rows)."""
    ex, ey = Ux - Dx, Uy - Dy
    Sxx, Syy = _z(Ux), _z(Ux)
    s = np.s_[1:-1, 1:-1]
    Sxx[s] = (c["Bxx"][1:-1, 1:-1] * ex[1:-1, 1:-1] - c["Bxx"][1:-1, :-2] * ex[1:-1, :-2]
              + c["Axx"][s] * (Dx[1:-1, 1:-1] - Dx[1:-1, :-2])) * safe_inv(c["Wxx"][s])
    Syy[s] = (c["Byy"][1:-1, 1:-1] * ey[1:-1, 1:-1] - c["Byy"][:-2, 1:-1] * ey[:-2, 1:-1]
              + c["Ayy"][s] * (Dy[1:-1, 1:-1] - Dy[:-2, 1:-1])) * safe_inv(c["Wyy"][s])
    gx, gy = _z(Ux), _z(Ux)
    n = np.s_[0:-1, 0:-1]
    gx[n] = (c["Bxy"][1:, :-1] * ex[1:, :-1] - c["Bxy"][:-1, :-1] * ex[:-1, :-1]
             + c["Axy"][n] * (Dx[1:, :-1] - Dx[:-1, :-1]))
    gy[n] = (c["Byx"][:-1, 1:] * ey[:-1, 1:] - c["Byx"][:-1, :-1] * ey[:-1, :-1]
             + c["Ayx"][n] * (Dy[:-1, 1:] - Dy[:-1, :-1]))
    nxx, nxy, nyx, nyy = node_coefficients(c, form)
    Sx = 0.5 * (nxx * gx + nxy * gy)
    Sy = 0.5 * (nyx * gx + nyy * gy)
    Sx[-1, :] = 0.0
    Sx[:, -1] = 0.0
    Sy[-1, :] = 0.0
    Sy[:, -1] = 0.0
    return Sxx, Syy, Sx, Sy


def visc(c, Sxx, Syy, Sx, Sy):
    """visc in index form at interior faces:
      x-face (i+1/2, j), i=1..nx-1: B^xx (Sxx_{i+1} - Sxx_i) + B^xy (Sx_{j+1/2} - Sx_{j-1/2})
      y-face (i, j+1/2), j=1..ny-1: B^yy (Syy_{j+1} - Syy_j) + B^yx (Sy_{i+1/2} - Sy_{i-1/2})"""
    vx, vy = _z(Sxx), _z(Sxx)
    vx[1:-1, 1:-2] = (c["Bxx"][1:-1, 1:-2] * (Sxx[1:-1, 2:-1] - Sxx[1:-1, 1:-2])
                      + c["Bxy"][1:-1, 1:-2] * (Sx[1:-1, 1:-2] - Sx[:-2, 1:-2]))
    vy[1:-2, 1:-1] = (c["Byy"][1:-2, 1:-1] * (Syy[2:-1, 1:-1] - Syy[1:-2, 1:-1])
                      + c["Byx"][1:-2, 1:-1] * (Sy[1:-2, 1:-1] - Sy[1:-2, :-2]))
    return vx, vy


def viscous(c, Ux, Uy, Dx, Dy, form="geometric"):
    """visc(strain(U, D)) at interior faces."""
    return visc(c, *strain(c, Ux, Uy, Dx, Dy, form))


def het(c, Dx, Dy):
    """cont(0, D): the boundary (heterogeneous) part of the divergence."""
    z = np.zeros_like(Dx)
    return cont(c, z, z, Dx, Dy)


def conv(c, Ux, Uy, Utx, Uty, Dx, Dy, Dtx, Dty):
    """conv in index form at interior faces.  The boundary bracket of
    eq:convective equals the interpolation of het = cont(0, D) onto the
    staggered control volume (differences and interpolations along different
    axes commute), so
      conv_x(i+1/2,j) = Fxx_{i+1} - Fxx_i + Fxy_{j+1/2} - Fxy_{j-1/2}
                        + (het_i + het_{i+1})/2 * (U+ + D+)_{i+1/2}/2
      Fxx_i   = (A^x U^x_{i-1/2} + A^x U^x_{i+1/2})/2 * (U+_{i-1/2} + U+_{i+1/2})/2
      Fxy_n   = (A^y U^y_{i,j+1/2} + A^y U^y_{i+1,j+1/2})/2 * (U+_{j} + U+_{j+1})/2
    and symmetrically for y."""
    fx = c["Ax"] * Ux
    fy = c["Ay"] * Uy
    h = het(c, Dx, Dy)
    Fxx, Fyy, Fxy, Fyx = _z(Ux), _z(Ux), _z(Ux), _z(Ux)
    Fxx[:, 1:] = 0.25 * (fx[:, :-1] + fx[:, 1:]) * (Utx[:, :-1] + Utx[:, 1:])
    Fyy[1:, :] = 0.25 * (fy[:-1, :] + fy[1:, :]) * (Uty[:-1, :] + Uty[1:, :])
    Fxy[:-1, :-1] = 0.25 * (fy[:-1, :-1] + fy[:-1, 1:]) * (Utx[:-1, :-1] + Utx[1:, :-1])
    Fyx[:-1, :-1] = 0.25 * (fx[:-1, :-1] + fx[1:, :-1]) * (Uty[:-1, :-1] + Uty[:-1, 1:])
    cx, cy = _z(Ux), _z(Ux)
    cx[1:-1, 1:-2] = (Fxx[1:-1, 2:-1] - Fxx[1:-1, 1:-2] + Fxy[1:-1, 1:-2] - Fxy[:-2, 1:-2]
                      + 0.25 * (h[1:-1, 1:-2] + h[1:-1, 2:-1]) * (Utx[1:-1, 1:-2] + Dtx[1:-1, 1:-2]))
    cy[1:-2, 1:-1] = (Fyy[2:-1, 1:-1] - Fyy[1:-2, 1:-1] + Fyx[1:-2, 1:-1] - Fyx[1:-2, :-2]
                      + 0.25 * (h[1:-2, 1:-1] + h[2:-1, 1:-1]) * (Uty[1:-2, 1:-1] + Dty[1:-2, 1:-1]))
    return cx, cy


def kinetic(c, Ux, Uy):
    """kinetic at cells 1..nx x 1..ny: (V^x U^x^2 at the two x-faces)/4 + (y)/4."""
    ex = c["Vu"] * Ux * Ux
    ey = c["Vv"] * Uy * Uy
    out = _z(Ux)
    out[1:-1, 1:-1] = 0.25 * (ex[1:-1, :-2] + ex[1:-1, 1:-1] + ey[:-2, 1:-1] + ey[1:-1, 1:-1])
    return out
