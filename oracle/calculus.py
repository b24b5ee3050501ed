"""Morinishi's discrete calculus on the staggered layout.

Positions: 'c' cell (i, j), 'u' x-face (i+1/2, j), 'v' y-face (i, j+1/2),
'n' node (i+1/2, j+1/2); all stored at [j, i] of a (ny+2, nx+2) array.

  d_x   unit-spacing difference along x (eq:differentiation)
  i_x   midpoint interpolation along x (eq:interpolation)
  p_x   permanent product along x (eq:permanent)
and the same along y.  Moving along x maps c<->u and v<->n; along y maps
c<->v and u<->n.  Entries whose stencil leaves the array are NaN, so a result
that depends on them is visibly invalid.
"""

from __future__ import annotations

import numpy as np

_XMAP = {"c": "u", "u": "c", "v": "n", "n": "v"}
_YMAP = {"c": "v", "v": "c", "u": "n", "n": "u"}
# a move is "forward" (result at +1/2) when the source is at an integer
# position along that axis
_XFWD = {"c": True, "v": True, "u": False, "n": False}
_YFWD = {"c": True, "u": True, "v": False, "n": False}


class F:
    """A field tagged with its position."""

    __slots__ = ("a", "pos")

    def __init__(self, a, pos):
        self.a = np.asarray(a, dtype=np.float64)
        self.pos = pos

    def _chk(self, o):
        if isinstance(o, F):
            if o.pos != self.pos:
                raise ValueError(f"position mismatch {self.pos} vs {o.pos}")
            return o.a
        return o

    def __add__(self, o):
        return F(self.a + self._chk(o), self.pos)

    __radd__ = __add__

    def __sub__(self, o):
        return F(self.a - self._chk(o), self.pos)

    def __rsub__(self, o):
        return F(self._chk(o) - self.a, self.pos)

    def __mul__(self, o):
        return F(self.a * self._chk(o), self.pos)

    __rmul__ = __mul__

    def __truediv__(self, o):
        return F(self.a / self._chk(o), self.pos)

    def __neg__(self):
        return F(-self.a, self.pos)


def _shift_pair(a, axis, forward):
    """(a_lo, a_hi) such that the result at index k combines a[k] and a[k+1]
    (forward) or a[k-1] and a[k] (backward)."""
    lo = np.full_like(a, np.nan)
    hi = np.full_like(a, np.nan)
    if axis == 1:
        if forward:
            lo[:, :-1], hi[:, :-1] = a[:, :-1], a[:, 1:]
        else:
            lo[:, 1:], hi[:, 1:] = a[:, :-1], a[:, 1:]
    else:
        if forward:
            lo[:-1, :], hi[:-1, :] = a[:-1, :], a[1:, :]
        else:
            lo[1:, :], hi[1:, :] = a[:-1, :], a[1:, :]
    return lo, hi


def d_x(f: F) -> F:
    lo, hi = _shift_pair(f.a, 1, _XFWD[f.pos])
    return F(hi - lo, _XMAP[f.pos])


def d_y(f: F) -> F:
    lo, hi = _shift_pair(f.a, 0, _YFWD[f.pos])
    return F(hi - lo, _YMAP[f.pos])


def i_x(f: F) -> F:
    lo, hi = _shift_pair(f.a, 1, _XFWD[f.pos])
    return F(0.5 * (hi + lo), _XMAP[f.pos])


def i_y(f: F) -> F:
    lo, hi = _shift_pair(f.a, 0, _YFWD[f.pos])
    return F(0.5 * (hi + lo), _YMAP[f.pos])


def p_x(f: F, g: F) -> F:
    """Permanent product (f_{k+1} g_k + g_{k+1} f_k)/2 along x."""
    if f.pos != g.pos:
        raise ValueError("position mismatch")
    flo, fhi = _shift_pair(f.a, 1, _XFWD[f.pos])
    glo, ghi = _shift_pair(g.a, 1, _XFWD[g.pos])
    return F(0.5 * (fhi * glo + ghi * flo), _XMAP[f.pos])


def p_y(f: F, g: F) -> F:
    if f.pos != g.pos:
        raise ValueError("position mismatch")
    flo, fhi = _shift_pair(f.a, 0, _YFWD[f.pos])
    glo, ghi = _shift_pair(g.a, 0, _YFWD[g.pos])
    return F(0.5 * (fhi * glo + ghi * flo), _YMAP[f.pos])


def safe_inv(a):
    """Reciprocal with 1/0 := 0 (empty faces and cells)."""
    a = np.asarray(a, dtype=np.float64)
    out = np.zeros_like(a)
    nz = a != 0.0
    out[nz] = 1.0 / a[nz]
    return out
