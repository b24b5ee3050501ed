"""Linear solves of the projection step.

The paper only says the Poisson equation is solved iteratively, with the
updates kept in the space of zero-mean solutions (end of Sec. 4.6).  Two
solvers are provided:
  pcg     textbook Jacobi-preconditioned conjugate gradients; for the singular
          Poisson problem the preconditioned residual is projected to zero
          mean over the unknowns, which keeps every update zero-mean.
  direct  sparse LU of the same matrix, bordered with the zero-mean
          constraint: the plain definition of the solution the iteration
          approximates.
"""

from __future__ import annotations

import numpy as np
from scipy.sparse import coo_matrix, bmat, csr_matrix
from scipy.sparse.linalg import spsolve

OK = 0
ENOTCONV = -3
EBREAKDOWN = -4


def pcg(apply_A, f, x0, dinv, mask, tol, maxit, zero_mean=False):
    """Solve A x = f on the entries where `mask` is True.

    apply_A(x) must return A x (zero off the mask).  dinv is the inverse of
    A's diagonal (Jacobi preconditioner).  Stops when ||r||_2 <= tol ||f||_2.
    Returns (x, iterations, relative residual, status)."""
    m = mask
    n = int(m.sum())
    x = np.where(m, x0, 0.0)
    fn = float(np.sqrt(np.sum(f[m] ** 2)))
    if fn == 0.0:
        return np.zeros_like(x), 0, 0.0, OK

    def precond(r):
        z = np.where(m, dinv * r, 0.0)
        if zero_mean:
            z = np.where(m, z - z[m].sum() / n, 0.0)
        return z

    r = np.where(m, f - apply_A(x), 0.0)
    rn = float(np.sqrt(np.sum(r[m] ** 2)))
    if rn <= tol * fn:
        return x, 0, rn / fn, OK
    z = precond(r)
    p = z.copy()
    rz = float(np.sum(r[m] * z[m]))
    status = ENOTCONV
    k = 0
    for k in range(1, maxit + 1):
        q = np.where(m, apply_A(p), 0.0)
        pq = float(np.sum(p[m] * q[m]))
        if not pq > 0.0:
            status = EBREAKDOWN
            break
        alpha = rz / pq
        x = x + alpha * p
        r = r - alpha * q
        rn = float(np.sqrt(np.sum(r[m] ** 2)))
        if rn <= tol * fn:
            status = OK
            break
        z = precond(r)
        rz_new = float(np.sum(r[m] * z[m]))
        beta = rz_new / rz
        rz = rz_new
        p = z + beta * p
    return x, k, rn / fn, status


def assemble(apply_A, mask):
    """Sparse matrix of a linear map restricted to the masked entries, built by
    applying it to unit vectors (column by column).  For small grids."""
    idx = np.flatnonzero(mask.ravel())
    n = len(idx)
    rows, cols, vals = [], [], []
    e = np.zeros(mask.size)
    for k, g in enumerate(idx):
        e[g] = 1.0
        col = apply_A(e.reshape(mask.shape)).ravel()[idx]
        e[g] = 0.0
        nz = np.flatnonzero(col)
        rows.append(nz)
        cols.append(np.full(len(nz), k))
        vals.append(col[nz])
    return coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n)).tocsr(), idx


def direct_zero_mean(A: csr_matrix, f):
    """Solve A x = f with sum(x) = 0 for a symmetric A whose null space is the
    constants: bordered system [[A, 1], [1^T, 0]]."""
    n = A.shape[0]
    one = csr_matrix(np.ones((n, 1)))
    K = bmat([[A, one], [one.T, None]], format="csc")
    sol = spsolve(K, np.concatenate([f, [0.0]]))
    return sol[:n]


def coloured_diagonal(apply_A, shape, mask, stride=3):
    """Diagonal of a nearest-neighbour linear map by probing with combs of
    unit entries spaced `stride` apart along the last two axes, one leading
    component at a time (for stacked fields such as (U^x, U^y))."""
    d = np.zeros(shape)
    lead = shape[:-2]
    for comp in np.ndindex(*lead) if lead else [()]:
        for a in range(stride):
            for b in range(stride):
                e = np.zeros(shape)
                e[comp + (slice(a, None, stride), slice(b, None, stride))] = 1.0
                e = np.where(mask, e, 0.0)
                y = apply_A(e)
                d += np.where(e > 0.0, y, 0.0)
    return d
