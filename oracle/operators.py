"""Discrete staggered operators D, G and L_h (oracle side).

Paper, "Fluid Mechanics" subsection: centred second-order finite differences
on a staggered grid; the projection u_{n+1} = u* - alpha dt grad(phi)
(eq. ``velsolen``) and the elliptic problem lap(phi) = (div u* - q)/(alpha dt)
(eq. ``elliptic``).  With the pressure correction at cell centres and the
velocity components on the cell faces, L_h = D G.

Staggered layout used here (a reading; the paper gives no array layout):
* ``u[j, k, i]`` lives on the x face at x = i dx (west face of cell i),
  periodic, shape ``(ny, nz, nx)``;
* ``w[j, k, i]`` lives on the z face at z = k dz (south face of cell k),
  periodic, shape ``(ny, nz, nx)``;
* ``v[j, k, i]`` lives on the y face ``yf[j]``, shape ``(ny + 1, nz, nx)``;
  ``v[0]`` and ``v[ny]`` are the wall values.
"""

import numpy as np


def divergence(u, v, w, g):
    """(D u)[j,k,i]: net outflow of cell (j,k,i) divided by its volume."""
    dyf = g.dyf.reshape(-1, 1, 1)
    return ((np.roll(u, -1, axis=2) - u) / g.dx
            + (v[1:] - v[:-1]) / dyf
            + (np.roll(w, -1, axis=1) - w) / g.dz)


def gradient(phi, g):
    """(G phi) on the faces: returns (gx, gy, gz) laid out like (u, v, w).

    On a Neumann wall face the wall-normal component is zero, so that the
    projection leaves the wall-normal velocity unchanged (paper's
    boundary-condition paragraph after eq. ``pressure``).  On a Dirichlet
    wall face (phi = 0 there) it is the one-sided difference over the half
    cell between the wall and the nearest centre.
    """
    gx = (phi - np.roll(phi, 1, axis=2)) / g.dx
    gz = (phi - np.roll(phi, 1, axis=1)) / g.dz
    gy = np.zeros((g.ny + 1,) + phi.shape[1:], dtype=phi.dtype)
    dyc = g.dyc[1:g.ny].reshape(-1, 1, 1)
    gy[1:g.ny] = (phi[1:] - phi[:-1]) / dyc
    if g.bc[0] == "dirichlet":
        gy[0] = (phi[0] - 0) / (g.yc[0] - g.yf[0])
    if g.bc[1] == "dirichlet":
        gy[g.ny] = (0 - phi[g.ny - 1]) / (g.yf[g.ny] - g.yc[g.ny - 1])
    return gx, gy, gz


def rhs_from_velocity(u, v, w, q, g, alpha_dt):
    """Right-hand side of the elliptic equation (eq. ``elliptic``):
    (D u* - q) / (alpha dt); q (mass sources, cell centred) may be None."""
    d = divergence(u, v, w, g)
    if q is not None:
        d = d - q
    return d / alpha_dt


def projection_step(u, v, w, p, phi, g, alpha_dt, visc):
    """Projection (eq. ``velsolen``) and pressure update (eq. ``pressure``):
    u_{n+1} = u* - alpha dt G phi, and p_{n+1} = p_n + phi - visc L_h phi with
    visc = alpha dt / (2 Re) for implicit viscous terms, 0 for explicit ones.
    Returns new arrays (u, v, w, p); p may be None."""
    gx, gy, gz = gradient(phi, g)
    un = u - alpha_dt * gx
    vn = v - alpha_dt * gy
    wn = w - alpha_dt * gz
    pn = None
    if p is not None:
        pn = p + phi - visc * laplacian(phi, g)
    return un, vn, wn, pn


def laplacian(phi, g):
    """7-point staggered Laplacian L_h phi, written out stencil by stencil.

    x and z: periodic second differences; y: the difference of the two face
    fluxes, a[j] (phi[j-1] - phi[j]) + c[j] (phi[j+1] - phi[j]), where the
    value beyond a wall is the wall value 0 (Dirichlet wall; a Neumann wall
    has a[0] = 0 or c[ny-1] = 0, so it carries no flux).  The diagonal
    b = -(a + c) is not formed, so no rounding of it enters the operator.  Works in any float dtype
    (``numpy.longdouble`` for manufactured right-hand sides) provided the
    geometry was built in that dtype.
    """
    out = (np.roll(phi, -1, axis=2) - 2 * phi + np.roll(phi, 1, axis=2)) / (g.dx * g.dx)
    out = out + (np.roll(phi, -1, axis=1) - 2 * phi + np.roll(phi, 1, axis=1)) / (g.dz * g.dz)
    a = g.a.reshape(-1, 1, 1)
    c = g.c.reshape(-1, 1, 1)
    ylap = np.zeros_like(phi)
    ylap[1:] += a[1:] * (phi[:-1] - phi[1:])
    ylap[:-1] += c[:-1] * (phi[1:] - phi[:-1])
    if g.bc[0] == "dirichlet":
        ylap[0] += a[0] * (0 - phi[0])
    if g.bc[1] == "dirichlet":
        ylap[-1] += c[-1] * (0 - phi[-1])
    return out + ylap


def weighted_mean(f, g):
    """Volume-weighted mean sum(V f) / sum(V), V = dx dz dyf[j]."""
    w = g.dyf.reshape(-1, 1, 1)
    return float((w * f).sum() / (g.dyf.sum() * g.nx * g.nz))
