"""Factored implicit viscous solve (oracle side).  TEST INFRASTRUCTURE ONLY.

Paper, "Fluid Mechanics" subsection, eq. ``nstime_discr``: with Crank-Nicolson
viscous terms the provisional velocity satisfies
    (1 - beta lap) (u_hat - u_n) = explicit terms,  beta = alpha dt / (2 Re);
"Fluid domain" parallelisation subsection: the implicit operator is split
into one tridiagonal solve per grid line and direction (Thomas' algorithm,
with a Sherman-Morrison correction along the two periodic directions), so no
global sparse matrix is formed.  The split (approximate factorisation) solves
    (1 - beta L_x) (1 - beta L_z) (1 - beta L_y) du = r.
The three one-dimensional operators act on different indices and their
coefficients depend only on their own index, so they commute and the order
of the three solves does not change du (up to rounding).

Readings (the paper gives no formulas for this step):
* L_x, L_z: the periodic uniform second differences (u is on x faces, w on
  z faces, but the face spacing is the same uniform dx, dz);
* L_y at cell centres (u, w and any cell-centred scalar): the wall-normal
  part of L_h with the velocity wall condition, which is the complement of
  the pressure-correction one (paper's boundary-condition paragraph after
  eq. ``pressure``): velocity prescribed (homogeneous for the increment,
  a Dirichlet face half a cell from the first centre) where the pressure
  correction is Neumann, zero normal gradient where it is Dirichlet (the
  ``neumann_velocity`` outlet);
* L_y on the y faces (the wall-normal component v, rows 0..ny of an
  (ny+1, nz, nx) array): the second difference across interior faces,
  ((v[j+1]-v[j])/dyf[j] - (v[j]-v[j-1])/dyf[j-1]) / dyc[j], with the wall
  rows held (the increment is zero there); only prescribed-velocity walls
  are defined for this component here.

This module builds each one-dimensional matrix densely and solves all the
lines of a direction with ``numpy.linalg.solve``: the plain definition, with
no Thomas or Sherman-Morrison steps of its own.
"""

import numpy as np

from .grid import geometry


def velocity_bc(g):
    """Wall conditions of the velocity increment: the complement of g.bc."""
    flip = {"neumann": "dirichlet", "dirichlet": "neumann"}
    return (flip[g.bc[0]], flip[g.bc[1]])


def periodic_matrix(n, h, beta):
    """Dense n x n matrix of (1 - beta D2) for the periodic second difference
    (x[i+1] - 2 x[i] + x[i-1]) / h^2; neighbours wrap, and for n = 1 or 2
    both neighbours fold onto the same entries."""
    r = beta / (h * h)
    A = np.zeros((n, n))
    for i in range(n):
        A[i, i] += 1.0 + 2.0 * r
        A[i, (i + 1) % n] -= r
        A[i, (i - 1) % n] -= r
    return A


def cell_y_matrix(g, beta):
    """Dense ny x ny matrix of (1 - beta L_y) at cell centres, velocity walls."""
    gv = geometry(g.nx, g.ny, g.nz, g.Lx, g.Lz, g.yf, bc=velocity_bc(g))
    A = np.eye(g.ny)
    for j in range(g.ny):
        A[j, j] += beta * (gv.a[j] + gv.c[j])
        if j > 0:
            A[j, j - 1] -= beta * gv.a[j]
        if j < g.ny - 1:
            A[j, j + 1] -= beta * gv.c[j]
    return A


def face_y_matrix(g, beta):
    """Dense (ny-1) x (ny-1) matrix of (1 - beta L_y) over the interior faces
    j = 1..ny-1 (row r is face r + 1); the wall faces are held at zero."""
    if velocity_bc(g) != ("dirichlet", "dirichlet"):
        raise ValueError("the y-face component is defined here for prescribed-velocity walls only")
    n = g.ny - 1
    A = np.eye(n)
    for r in range(n):
        j = r + 1
        lo = 1.0 / (g.dyc[j] * g.dyf[j - 1])
        up = 1.0 / (g.dyc[j] * g.dyf[j])
        A[r, r] += beta * (lo + up)
        if r > 0:
            A[r, r - 1] -= beta * lo
        if r < n - 1:
            A[r, r + 1] -= beta * up
    return A


def solve_lines(A, f, axis):
    """Solve A x = f along `axis` for every line of f."""
    moved = np.moveaxis(np.asarray(f, dtype=np.float64), axis, 0)
    shp = moved.shape
    out = np.linalg.solve(A, moved.reshape(shp[0], -1)).reshape(shp)
    return np.moveaxis(out, 0, axis)


def factored_solve(f, g, beta, where="cells", order="xzy"):
    """du = (1 - beta L_y)^-1 (1 - beta L_z)^-1 (1 - beta L_x)^-1 f.

    `where` = "cells": f has shape (ny, nz, nx).
    `where` = "yfaces": f has shape (ny+1, nz, nx); rows 0 and ny of the
    result are zero (the increment vanishes on prescribed-velocity walls)
    and f's wall rows are ignored.
    `order` permutes the three solves (they commute; used as a check)."""
    if beta < 0 or not np.isfinite(beta):
        raise ValueError("beta must be finite and >= 0")
    f = np.asarray(f, dtype=np.float64)
    if where == "cells":
        if f.shape != (g.ny, g.nz, g.nx):
            raise ValueError("cell field must have shape (ny, nz, nx)")
        Ay = cell_y_matrix(g, beta)
        work = f.copy()
    elif where == "yfaces":
        if f.shape != (g.ny + 1, g.nz, g.nx):
            raise ValueError("y-face field must have shape (ny+1, nz, nx)")
        Ay = face_y_matrix(g, beta)
        work = f[1:g.ny].copy()
    else:
        raise ValueError("where must be 'cells' or 'yfaces'")
    mats = {"x": (periodic_matrix(g.nx, g.dx, beta), 2), "z": (periodic_matrix(g.nz, g.dz, beta), 1),
            "y": (Ay, 0)}
    for d in order:
        A, ax = mats[d]
        work = solve_lines(A, work, ax)
    if where == "cells":
        return work
    out = np.zeros_like(f)
    out[1:g.ny] = work
    return out
