"""Staggered-grid geometry and y-operator coefficients (oracle side).

Paper, "Fluid Mechanics" subsection: second-order centred finite differences
on a Cartesian staggered grid, uniform spacing in the two periodic directions
(required by the FFT solver, stated where the elliptic equation's solution
method is given) and arbitrary spacing in the wall-normal direction.

Conventions (readings of the paper, listed in the design doc):
* arrays are C-ordered ``[ny][nz][nx]``: x fastest, the wall-normal y slowest;
* ``nx, ny, nz`` count pressure cells; ``yf`` holds the ``ny + 1`` y faces;
* pressure points sit at cell centres: x_i = (i + 1/2) dx, z_k = (k + 1/2) dz,
  y_j = (yf[j] + yf[j+1]) / 2.
"""

from dataclasses import dataclass

import numpy as np


@dataclass
class Geometry:
    nx: int
    ny: int
    nz: int
    Lx: float
    Lz: float
    dx: float
    dz: float
    yf: np.ndarray    # (ny+1,) face coordinates
    dyf: np.ndarray   # (ny,)   cell widths yf[j+1] - yf[j]
    yc: np.ndarray    # (ny,)   cell centres
    dyc: np.ndarray   # (ny+1,) centre distances; dyc[j] = yc[j] - yc[j-1] for 1 <= j <= ny-1, walls unused (nan)
    a: np.ndarray     # (ny,) wall-side face coefficient of row j (a[0]: lower wall, 0 if Neumann)
    b: np.ndarray     # (ny,) diagonal, -(a + c)
    c: np.ndarray     # (ny,) upper face coefficient (c[ny-1]: upper wall, 0 if Neumann)
    bc: tuple = ("neumann", "neumann")   # (lower wall, upper wall) condition on phi

    @property
    def singular(self):
        """Neumann at both walls: L_h has the constants as null space."""
        return self.bc == ("neumann", "neumann")


BCS = ("neumann", "dirichlet")


def geometry(nx, ny, nz, Lx, Lz, yf, dtype=np.float64, bc=("neumann", "neumann")):
    """Grid spacings and the coefficients of the 1-D y operator.

    The y part of L_h at cell j is the difference of the two face fluxes
    (phi[j+1]-phi[j])/dyc[j+1] and (phi[j]-phi[j-1])/dyc[j], divided by the
    cell width dyf[j].  Wall faces (paper's boundary-condition paragraph after
    eq. ``pressure``):
    * "neumann" (the default configuration): zero flux, so a[0] = 0 or
      c[ny-1] = 0;
    * "dirichlet" (the ``neumann_velocity`` outlet option, applied to the
      upper wall there): phi = 0 on the wall face, half a cell from the
      centre, so the wall flux is (0 - phi[0]) / (dyf[0] / 2) and
      a[0] = 2 / dyf[0]^2 (likewise c[ny-1] = 2 / dyf[ny-1]^2).
    """
    nx, ny, nz = int(nx), int(ny), int(nz)
    if nx < 1 or nz < 1 or ny < 2:
        raise ValueError("need nx >= 1, nz >= 1, ny >= 2")
    yf = np.asarray(yf, dtype=dtype)
    if yf.shape != (ny + 1,):
        raise ValueError(f"yf must have ny+1 = {ny + 1} entries, got {yf.shape}")
    if not np.all(np.isfinite(yf)) or not np.all(np.diff(yf) > 0):
        raise ValueError("yf must be finite and strictly increasing")
    Lx = dtype(Lx)
    Lz = dtype(Lz)
    if not (np.isfinite(Lx) and np.isfinite(Lz) and Lx > 0 and Lz > 0):
        raise ValueError("Lx and Lz must be finite and positive")
    bc = tuple(bc)
    if len(bc) != 2 or any(w not in BCS for w in bc):
        raise ValueError(f"bc must be two of {BCS}")
    dx = Lx / nx
    dz = Lz / nz
    dyf = yf[1:] - yf[:-1]
    yc = (yf[1:] + yf[:-1]) / 2
    dyc = np.full(ny + 1, np.nan, dtype=dtype)
    dyc[1:ny] = yc[1:] - yc[:-1]
    a = np.zeros(ny, dtype=dtype)
    c = np.zeros(ny, dtype=dtype)
    for j in range(ny):
        if j > 0:
            a[j] = 1 / (dyf[j] * dyc[j])
        if j < ny - 1:
            c[j] = 1 / (dyf[j] * dyc[j + 1])
    if bc[0] == "dirichlet":
        a[0] = 1 / (dyf[0] * (dyf[0] / 2))
    if bc[1] == "dirichlet":
        c[ny - 1] = 1 / (dyf[ny - 1] * (dyf[ny - 1] / 2))
    b = -(a + c)
    return Geometry(nx, ny, nz, Lx, Lz, dx, dz, yf, dyf, yc, dyc, a, b, c, bc)


def lambda_x(g, dtype=np.float64):
    """Eigenvalues of the periodic second difference in x, for kx = 0..nx//2.

    Textbook closed form: exp(i 2 pi kx i / nx) is an eigenvector of
    (phi[i+1] - 2 phi[i] + phi[i-1]) / dx^2 with eigenvalue
    -(4 / dx^2) sin^2(pi kx / nx).
    """
    k = np.arange(g.nx // 2 + 1, dtype=dtype)
    return -(4 / g.dx ** 2) * np.sin(np.pi * k / g.nx) ** 2


def lambda_z(g, dtype=np.float64):
    """Same closed form along z, for kz = 0..nz-1 (FFT ordering)."""
    k = np.arange(g.nz, dtype=dtype)
    return -(4 / g.dz ** 2) * np.sin(np.pi * k / g.nz) ** 2
