"""Dense bordered solve of the discrete Neumann problem (oracle pin).

Independent of the FFT route: the full N x N matrix of L_h is assembled cell
by cell from the stencil (paper, "Fluid Mechanics" subsection: staggered
centred second-order differences, periodic x and z, Neumann y walls) and the
constant null space is removed with a border:

    [ L_h  1 ] [phi]   [f]
    [ V^T  0 ] [ mu] = [0]

V^T L_h = 0 (the sum over cells of volume times L_h phi telescopes to the
zero wall fluxes), so mu is the volume-weighted mean of f and phi is the
zero-weighted-mean solution of L_h phi = f - mu.  Intended for N <= ~4000.
"""

import numpy as np

from .grid import geometry


def _index(j, k, i, nz, nx):
    return (j * nz + k) * nx + i


def laplacian_matrix(g):
    """Dense L_h, rows and columns in C order of ``[ny][nz][nx]``."""
    nx, ny, nz = g.nx, g.ny, g.nz
    N = nx * ny * nz
    A = np.zeros((N, N), dtype=np.float64)
    for j in range(ny):
        for k in range(nz):
            for i in range(nx):
                r = _index(j, k, i, nz, nx)
                # x: periodic second difference (entries add, so nx = 1 or 2 work)
                A[r, _index(j, k, (i + 1) % nx, nz, nx)] += 1 / g.dx ** 2
                A[r, _index(j, k, (i - 1) % nx, nz, nx)] += 1 / g.dx ** 2
                A[r, r] -= 2 / g.dx ** 2
                A[r, _index(j, (k + 1) % nz, i, nz, nx)] += 1 / g.dz ** 2
                A[r, _index(j, (k - 1) % nz, i, nz, nx)] += 1 / g.dz ** 2
                A[r, r] -= 2 / g.dz ** 2
                # y: flux differences; no flux through the walls
                if j + 1 < ny:
                    t = 1 / (g.dyf[j] * (g.yc[j + 1] - g.yc[j]))
                    A[r, _index(j + 1, k, i, nz, nx)] += t
                    A[r, r] -= t
                if j > 0:
                    t = 1 / (g.dyf[j] * (g.yc[j] - g.yc[j - 1]))
                    A[r, _index(j - 1, k, i, nz, nx)] += t
                    A[r, r] -= t
                # Dirichlet wall: phi = 0 on the wall face, half a cell away
                if j == 0 and g.bc[0] == "dirichlet":
                    A[r, r] -= 1 / (g.dyf[0] * (g.yc[0] - g.yf[0]))
                if j == ny - 1 and g.bc[1] == "dirichlet":
                    A[r, r] -= 1 / (g.dyf[ny - 1] * (g.yf[ny] - g.yc[ny - 1]))
    return A


def bordered_matrix(g):
    A = laplacian_matrix(g)
    N = A.shape[0]
    vol = np.repeat(g.dyf * g.dx * g.dz, g.nz * g.nx)
    B = np.zeros((N + 1, N + 1), dtype=np.float64)
    B[:N, :N] = A
    B[:N, N] = 1.0
    B[N, :N] = vol
    return B


def dense_solve(f, Lx, Lz, yf, bc=("neumann", "neumann")):
    """Returns (phi, mu) from the bordered dense system (LAPACK gesv); with a
    Dirichlet wall L_h is non-singular and is solved directly (mu = 0)."""
    f = np.asarray(f, dtype=np.float64)
    ny, nz, nx = f.shape
    g = geometry(nx, ny, nz, Lx, Lz, yf, bc=bc)
    if not g.singular:
        return np.linalg.solve(laplacian_matrix(g), f.ravel()).reshape(ny, nz, nx), 0.0
    B = bordered_matrix(g)
    rhs = np.concatenate([f.ravel(), [0.0]])
    sol = np.linalg.solve(B, rhs)
    return sol[:-1].reshape(ny, nz, nx), float(sol[-1])
