"""Level sets of the synthetic bodies (geometry input, Sec. 3.1).

A body is given by a function phi(x, y) that is positive in the fluid.  The
paper only requires a signed function whose zero set is the boundary; the
capacities are integrals of the fluid characteristic function (eq:characteristic).
"""

from __future__ import annotations

import math

import numpy as np

from workloads import CIRCLE, ELLIPSE, NACA4, Body


def naca_half_thickness(xi, t):
    """Half-thickness of a symmetric NACA 4-digit section (chord units),
    open trailing edge, from the published thickness polynomial."""
    xi = np.clip(xi, 0.0, 1.0)
    return 5.0 * t * (0.2969 * np.sqrt(xi) - 0.1260 * xi - 0.3516 * xi ** 2
                      + 0.2843 * xi ** 3 - 0.1015 * xi ** 4)


def body_phi(body: Body, x, y):
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    if body.kind == CIRCLE:
        return np.hypot(x - body.cx, y - body.cy) - body.a
    if body.kind == ELLIPSE:
        c, s = math.cos(body.angle), math.sin(body.angle)
        xr = c * (x - body.cx) + s * (y - body.cy)
        yr = -s * (x - body.cx) + c * (y - body.cy)
        return np.sqrt((xr / body.a) ** 2 + (yr / body.b) ** 2) - 1.0
    if body.kind == NACA4:
        c, s = math.cos(body.angle), math.sin(body.angle)
        # chord direction (c, -s): nose-up for a positive angle
        dx, dy = x - body.cx, y - body.cy
        xi = (dx * c - dy * s) / body.chord
        eta = (dx * s + dy * c) / body.chord
        inside_span = (xi >= 0.0) & (xi <= 1.0)
        f_span = np.abs(eta) - naca_half_thickness(xi, body.t)
        f_front = np.hypot(xi, eta)
        f_back = np.hypot(xi - 1.0, np.maximum(np.abs(eta) - naca_half_thickness(1.0, body.t), 0.0)) + 1e-300
        f = np.where(inside_span, f_span, np.where(xi < 0.0, f_front, f_back))
        return f * body.chord
    raise ValueError(f"unknown body kind {body.kind}")


def make_phi(bodies):
    """Level set of the fluid outside all bodies: the minimum over bodies."""
    bodies = list(bodies)

    def phi(x, y):
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        if not bodies:
            return np.ones(np.broadcast(x, y).shape)
        out = body_phi(bodies[0], x, y)
        for b in bodies[1:]:
            out = np.minimum(out, body_phi(b, x, y))
        return out

    return phi
