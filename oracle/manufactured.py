"""Manufactured solutions from the discrete eigenfunctions (oracle pin).

In x and z the discrete periodic Laplacian has the textbook eigenvectors
cos(kx x + kz z + theta) sampled at the cell centres.  In y the operator
A_y = diag(dyf)^-1 K (K symmetric tridiagonal, Neumann walls) is similar to
the symmetric matrix diag(dyf)^-1/2 K diag(dyf)^-1/2, whose eigenpairs LAPACK
computes (``scipy.linalg.eigh_tridiagonal``); v = diag(dyf)^-1/2 u are then
eigenvectors of A_y.  A field phi* = sum_m A_m cos(...) v_p(y) is therefore a
sum of discrete eigenfunctions of L_h (paper, "Fluid Mechanics" subsection:
the staggered operator; the FFT solver's diagonalisation of the periodic
directions in the "Fluid domain" subsection).

The right-hand side f = L_h phi* is formed by applying the 7-point operator in
``numpy.longdouble`` to the FP64 values of phi*, so phi* is the exact discrete
solution of the rounded f up to one rounding of f; every p >= 1 or
(kx, kz) != 0 term has zero weighted mean, so phi* also satisfies the pin.
"""

import numpy as np
from scipy.linalg import eigh_tridiagonal

from .grid import geometry
from .operators import laplacian


def y_eigenpairs(g):
    """Eigenpairs (mu_p, v_p) of the y operator, p = 0..ny-1, mu decreasing
    (mu_0 = 0, the constant mode, with Neumann walls); v_p scaled to max-norm
    1 with v_p[0] > 0 (v_p[argmax] > 0 when a Dirichlet lower wall makes
    v_p[0] small)."""
    ny = g.ny
    s = np.sqrt(g.dyf)
    # K[j, j+1] = 1 / dyc[j+1]; diagonal of K = -(sum of the two face terms)
    off = 1.0 / g.dyc[1:ny]
    kdiag = np.zeros(ny)
    kdiag[:-1] -= off
    kdiag[1:] -= off
    # a Dirichlet wall adds the wall-face term 1 / (half cell) to its row
    if g.bc[0] == "dirichlet":
        kdiag[0] -= 1.0 / (g.yc[0] - g.yf[0])
    if g.bc[1] == "dirichlet":
        kdiag[-1] -= 1.0 / (g.yf[ny] - g.yc[ny - 1])
    d = kdiag / g.dyf
    e = off / (s[:-1] * s[1:])
    mu, U = eigh_tridiagonal(d, e)
    order = np.argsort(-mu)
    mu = mu[order]
    V = U[:, order] / s.reshape(-1, 1)
    V = V / np.abs(V).max(axis=0, keepdims=True)
    if g.singular:
        V = V * np.where(V[0] < 0, -1.0, 1.0)
        mu[0] = 0.0
    else:
        pick = V[np.argmax(np.abs(V), axis=0), np.arange(ny)]
        V = V * np.where(pick < 0, -1.0, 1.0)
    return mu, V


def manufactured_field(nx, ny, nz, Lx, Lz, yf, modes, bc=("neumann", "neumann")):
    """phi*[ny,nz,nx] and f = L_h phi* (longdouble, rounded to FP64).

    ``modes`` is an iterable of (kx, kz, p, amplitude, phase) with integer
    index wavenumbers kx, kz and y-mode index p."""
    g = geometry(nx, ny, nz, Lx, Lz, yf, bc=bc)
    _, V = y_eigenpairs(g)
    x = (np.arange(nx) + 0.5) * g.dx
    z = (np.arange(nz) + 0.5) * g.dz
    phi = np.zeros((ny, nz, nx))
    for kx, kz, p, amp, th in modes:
        arg = (2 * np.pi * kx / Lx) * x.reshape(1, -1) + (2 * np.pi * kz / Lz) * z.reshape(-1, 1) + th
        phi += amp * np.cos(arg)[None, :, :] * V[:, int(p)].reshape(-1, 1, 1)
    gl = geometry(nx, ny, nz, np.longdouble(Lx), np.longdouble(Lz),
                  np.asarray(yf, dtype=np.longdouble), dtype=np.longdouble, bc=bc)
    f = laplacian(phi.astype(np.longdouble), gl).astype(np.float64)
    return phi, f
