"""Pins of the three-dimensional oracle (oracle.geometry3d, oracle.pmii3d)
against what the mathematics fixes independently of it: the two-dimensional
oracle's closed-form disc integrals and capacities, exact volumes and plane
sections of spheres, a volume integral taken along another axis, the
transpose relation of eq:compatibility, the textbook 7-point Laplacian
without bodies, and the two-dimensional projection for a z-invariant case."""

import math

import numpy as np
import pytest
from scipy import integrate

import workloads as W
import workloads.three_d as T
from oracle import derived, geometry, geometry3d as G3, operators, pmii3d as P3, solvers

_CAPS = {}


def _caps(case):
    if case.name not in _CAPS:
        _CAPS[case.name] = G3.capacities(case.grid, case.bodies)
    return _CAPS[case.name]


def test_disc_rectangle_area_matches_the_two_dimensional_oracle():
    """The section areas (inclusion-exclusion of disc quadrants) against the
    2-D oracle's disc moments (integrals of the upper and lower arcs)."""
    rng = np.random.default_rng(3)
    for _ in range(3000):
        cx, cy = rng.uniform(-1, 1, 2)
        r = rng.uniform(0.01, 1.0)
        xa, ya = rng.uniform(-1.5, 1.5, 2)
        xb, yb = xa + rng.uniform(0, 1.2), ya + rng.uniform(0, 1.2)
        a = G3.disc_rect_area(cx, cy, r, xa, xb, ya, yb)
        b = geometry.disc_rect_moments(cx, cy, r, xa, xb, ya, yb)[0]
        assert abs(a - b) <= 1e-14 * max(r * r, 1e-3)


@pytest.mark.parametrize("make", [lambda: T.sphere_box(16), lambda: T.two_spheres(20, 18, 14)])
def test_sphere_volumes_and_plane_sections(make):
    """Sum of V = box - 4/3 pi r^3 per sphere; the wet areas of a whole grid
    plane of faces = plane area - pi rho^2 for each sphere it cuts."""
    case = make()
    g = case.grid
    c = _caps(case)
    exact = g.lx * g.ly * g.lz - sum(4.0 / 3.0 * math.pi * b.r ** 3 for b in case.bodies)
    assert abs(c["V"][1:-1, 1:-1, 1:-1].sum() - exact) <= 1e-13 * exact
    for axis, name, n, (la, lb), h, o in ((0, "Ax", g.nx, (g.ly, g.lz), g.hx, g.x0),
                                          (1, "Ay", g.ny, (g.lx, g.lz), g.hy, g.y0),
                                          (2, "Az", g.nz, (g.lx, g.ly), g.hz, g.z0)):
        for f in range(0, n + 1):
            pos = o + f * h
            cut = sum(math.pi * (b.r ** 2 - (pos - (b.cx, b.cy, b.cz)[axis]) ** 2) for b in case.bodies
                      if abs(pos - (b.cx, b.cy, b.cz)[axis]) < b.r)
            a = c[name]
            plane = a[1:-1, 1:-1, f] if axis == 0 else (a[1:-1, f, 1:-1] if axis == 1 else a[f, 1:-1, 1:-1])
            assert abs(plane.sum() - (la * lb - cut)) <= 1e-13 * la * lb, (name, f)


def test_small_sphere_on_a_node():
    """A sphere of radius 0.45 centred on a grid node of unit cells: each of
    the eight cells around the node loses an eighth of it, each of the
    twelve faces through the node a quarter disc, and the shifted control
    volume that straddles the node's plane a quarter of the sphere."""
    g = T.Grid3(4, 4, 4, 0.0, 0.0, 0.0, 4.0, 4.0, 4.0)
    r = 0.45
    c = G3.capacities(g, [T.Body3(T.SPHERE, 2.0, 2.0, 2.0, r)])
    vs = 4.0 / 3.0 * math.pi * r ** 3
    for k in (2, 3):
        for j in (2, 3):
            for i in (2, 3):
                assert abs(c["V"][k, j, i] - (1.0 - vs / 8.0)) < 1e-14
    for k in (2, 3):
        for j in (2, 3):
            assert abs(c["Ax"][k, j, 2] - (1.0 - math.pi * r * r / 4.0)) < 1e-14
            assert abs(c["Ay"][k, 2, j] - (1.0 - math.pi * r * r / 4.0)) < 1e-14
            assert abs(c["Az"][2, k, j] - (1.0 - math.pi * r * r / 4.0)) < 1e-14
            assert abs(c["Vx"][k, j, 2] - (1.0 - vs / 4.0)) < 1e-14
            assert abs(c["Vz"][2, k, j] - (1.0 - vs / 4.0)) < 1e-14
    # untouched cells and faces are full
    assert c["V"][1, 1, 1] == 1.0 and c["Ax"][1, 1, 1] == 1.0 and c["Vy"][1, 1, 1] == 1.0


def test_volume_integral_along_another_axis():
    """The oracle integrates section areas along z; the same fluid volumes
    integrated along x (sections by planes x = const, a disc in (y, z)) on
    cut boxes next to the sphere."""
    case = T.sphere_box(10)
    b = case.bodies[0]
    rng = np.random.default_rng(5)
    done = 0
    while done < 40:
        xa, ya, za = rng.uniform(0.1, 0.8, 3)
        h = rng.uniform(0.05, 0.15)
        xb, yb, zb = xa + h, ya + h, za + h

        def solid_x(x):
            d = x - b.cx
            if abs(d) >= b.r:
                return 0.0
            return G3.disc_rect_area(b.cy, b.cz, math.sqrt(b.r * b.r - d * d), ya, yb, za, zb)

        v = G3.box_fluid_volume([b], xa, xb, ya, yb, za, zb)
        if not 0.0 < v < h ** 3:
            continue
        pts = sorted({x for x in (b.cx - b.r, b.cx + b.r) if xa < x < xb}
                     | {b.cx + s * math.sqrt(b.r ** 2 - d * d) for s in (-1, 1)
                        for d in [abs(ya - b.cy), abs(yb - b.cy), abs(za - b.cz), abs(zb - b.cz)]
                        + [math.hypot(y - b.cy, z - b.cz) for y in (ya, yb) for z in (za, zb)]
                        if d < b.r and xa < b.cx + s * math.sqrt(b.r ** 2 - d * d) < xb})
        edges = [xa] + pts + [xb]
        solid = sum(integrate.quad(solid_x, p, q, epsabs=1e-16, epsrel=1e-12, limit=200)[0]
                    for p, q in zip(edges[:-1], edges[1:]) if q - p > 1e-12)
        assert abs((h ** 3 - solid) - v) <= 1e-12 * h ** 3
        done += 1


def test_z_cylinder_is_the_two_dimensional_circle_times_the_depth():
    """A cylinder along z: every capacity is the 2-D oracle's (independent
    closed-form arcs) times hz, and A^z is the 2-D cell volume."""
    case = T.zcylinder_box(12, 10, 3)
    g = case.grid
    c = _caps(case)
    b = case.bodies[0]
    g2 = W.GridSpec(g.nx, g.ny, g.x0, g.y0, g.lx, g.ly)
    c2 = geometry.capacities(g2, [W.Body(W.CIRCLE, b.cx, b.cy, a=b.r)])
    s = np.s_[1:-1, 1:-1]
    for k in range(1, g.nz + 1):
        assert np.allclose(c["V"][k][s], g.hz * c2["V"][s], rtol=0, atol=1e-15)
        assert np.allclose(c["Az"][k][s], c2["V"][s], rtol=0, atol=1e-15)
        # interior faces (the 2-D oracle reads the wall faces as wetted from
        # inside; the walls carry no unknown here)
        assert np.allclose(c["Ax"][k][1:-1, 1:-2], g.hz * c2["Ax"][1:-1, 1:-2], rtol=0, atol=1e-15)
        assert np.allclose(c["Ay"][k][1:-2, 1:-1], g.hz * c2["Ay"][1:-2, 1:-1], rtol=0, atol=1e-15)
        assert np.allclose(c["Vx"][k][1:-1, 1:-2], g.hz * c2["Vu"][1:-1, 1:-2], rtol=0, atol=1e-15)
        assert np.allclose(c["Vy"][k][1:-2, 1:-1], g.hz * c2["Vv"][1:-2, 1:-1], rtol=0, atol=1e-15)


def test_pres_is_minus_the_transpose_of_cont():
    """eq:compatibility, by brute force on unit vectors (tiny box), and the
    Poisson operator is symmetric, annihilates constants and -L is positive
    semi-definite."""
    case = T.tiny_box()
    g = case.grid
    c = _caps(case)
    A = (c["Ax"], c["Ay"], c["Az"])
    sh = g.shape
    ncell = int(np.prod(sh))
    C = []  # rows: cells, columns: faces of the three grids
    for a in range(3):
        cols = []
        for f in range(ncell):
            U = [np.zeros(sh) for _ in range(3)]
            U[a].ravel()[f] = 1.0
            cols.append(P3.cont(A, tuple(U)).ravel())
        C.append(np.array(cols).T)
    C = np.hstack(C)
    Pm = []
    for cidx in range(ncell):
        P = np.zeros(sh)
        P.ravel()[cidx] = 1.0
        G = P3.pres(A, P)
        Pm.append(np.concatenate([x.ravel() for x in G]))
    Pm = np.array(Pm).T  # faces x cells
    # on the real cells and the faces between real cells (the ghost layer
    # carries no unknown)
    k, j, i = np.indices(sh)
    real = ((i >= 1) & (i <= g.nx) & (j >= 1) & (j <= g.ny) & (k >= 1) & (k <= g.nz)).ravel()
    faces = np.concatenate([((i >= 1) & (i <= g.nx - 1) & (j >= 1) & (j <= g.ny) & (k >= 1) & (k <= g.nz)).ravel(),
                            ((i >= 1) & (i <= g.nx) & (j >= 1) & (j <= g.ny - 1) & (k >= 1) & (k <= g.nz)).ravel(),
                            ((i >= 1) & (i <= g.nx) & (j >= 1) & (j <= g.ny) & (k >= 1) & (k <= g.nz - 1)).ravel()])
    assert np.array_equal(Pm[np.ix_(faces, real)], -C[np.ix_(real, faces)].T)
    pr = P3.prepare(c, g, 0.05)
    K, idx = P3.matrix(pr)
    Kd = K.toarray()
    assert np.abs(Kd - Kd.T).max() <= 1e-15 * np.abs(Kd).max()
    assert np.abs(Kd @ np.ones(len(idx))).max() <= 1e-14 * np.abs(Kd).max()
    ev = np.linalg.eigvalsh(Kd)
    assert ev.min() >= -1e-13 * ev.max() and ev[1] > 1e-8 * ev.max()


def test_without_bodies_the_operator_is_the_seven_point_laplacian():
    g = T.Grid3(6, 5, 4, 0.0, 0.0, 0.0, 1.2, 0.8, 0.6)
    c = G3.capacities(g, [])
    pr = P3.prepare(c, g, 0.05)
    phi = T.random_cells(T.Case3("box", g, []), 7)
    Lphi = P3.laplacian(pr, phi)
    hx, hy, hz = g.hx, g.hy, g.hz
    ref = np.zeros(g.shape)
    for k in range(1, g.nz + 1):
        for j in range(1, g.ny + 1):
            for i in range(1, g.nx + 1):
                s = 0.0
                for (di, dj, dk), w in (((1, 0, 0), hy * hz / hx), ((0, 1, 0), hx * hz / hy), ((0, 0, 1), hx * hy / hz)):
                    for sg in (1, -1):
                        ii, jj, kk = i + sg * di, j + sg * dj, k + sg * dk
                        if 1 <= ii <= g.nx and 1 <= jj <= g.ny and 1 <= kk <= g.nz:
                            s += w * (phi[kk, jj, ii] - phi[k, j, i])
                ref[k, j, i] = s
    assert np.abs(Lphi - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("theta", [0.0, 0.05])
def test_projection_is_divergence_free_and_idempotent(theta):
    case = T.two_spheres(20, 18, 14, mass_floor=theta)
    c = _caps(case)
    pr = P3.prepare(c, case.grid, theta)
    U = T.face_velocity(case)
    phi, Un, info = P3.project(pr, U, case.rho, case.tau)
    assert info["div_rel"] < 1e-11
    assert abs(phi[pr.act_p].sum()) <= 1e-12 * np.abs(phi).max() * pr.n_active
    phi2, Un2, _ = P3.project(pr, Un, case.rho, case.tau)
    assert np.abs(phi2).max() <= 1e-9 * np.abs(phi).max()
    assert max(np.abs(a - b).max() for a, b in zip(Un2, Un)) <= 1e-9
    # the Jacobi-PCG reaches the direct solution
    phi3, _, info3 = P3.project(pr, U, case.rho, case.tau, solver="pcg", tol=1e-12)
    assert info3["status"] == solvers.OK
    assert np.abs(phi3 - phi).max() <= 1e-9 * np.abs(phi).max()
    if theta == 0.0:
        # the paper's mass matrix: some unknowns have control volumes below
        # the 0.05 floor, so the two readings differ here
        g = case.grid
        assert any((pr.act[a] & (pr.M[a] < 0.05 * g.hx * g.hy * g.hz)).any() for a in range(3))


def test_z_invariant_projection_is_the_two_dimensional_one():
    """A z-cylinder with a z-invariant U* (U*_z = 0): Phi is the 2-D oracle's
    zero-mean Poisson solution on every layer and U_x, U_y its projected
    velocity."""
    case = T.zcylinder_box(24, 20, 4)
    g = case.grid
    c = _caps(case)
    pr = P3.prepare(c, g, case.mass_floor)
    rng = np.random.default_rng(11)
    ux2 = rng.uniform(-1, 1, (g.ny + 2, g.nx + 2))
    uy2 = rng.uniform(-1, 1, (g.ny + 2, g.nx + 2))
    U = (np.zeros(g.shape), np.zeros(g.shape), np.zeros(g.shape))
    for k in range(1, g.nz + 1):
        U[0][k] = ux2
        U[1][k] = uy2
    phi, Un, info = P3.project(pr, U, case.rho, case.tau)
    b = case.bodies[0]
    g2 = W.GridSpec(g.nx, g.ny, g.x0, g.y0, g.lx, g.ly)
    c2 = geometry.capacities(g2, [W.Body(W.CIRCLE, b.cx, b.cy, a=b.r)])
    pr2 = derived.prepare(c2, g.nx, g.ny, vol_floor=case.mass_floor * g.hx * g.hy)
    um, vm = np.where(pr2.act_u, ux2, 0.0), np.where(pr2.act_v, uy2, 0.0)
    z2 = np.zeros_like(ux2)
    b2 = np.where(pr2.act_p, -(case.rho / case.tau) * operators.cont(c2, um, vm, z2, z2), 0.0)
    b2 = np.where(pr2.act_p, b2 - b2[pr2.act_p].mean(), 0.0)
    K2, idx2 = solvers.assemble(lambda x: -derived.laplacian(pr2, x), pr2.act_p)
    phi2 = np.zeros_like(ux2)
    phi2.ravel()[idx2] = solvers.direct_zero_mean(K2, b2.ravel()[idx2])
    for k in range(1, g.nz + 1):
        assert np.abs(phi[k] - phi2).max() <= 1e-9 * np.abs(phi2).max(), k
        ux = np.where(pr2.cx > 0, um - (case.tau / case.rho) * pr2.gx * (np.roll(phi2, -1, 1) - phi2), um)
        assert np.abs(Un[0][k] - ux).max() <= 1e-9
    assert np.abs(Un[2]).max() <= 1e-9
