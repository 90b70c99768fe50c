"""FFT + tridiagonal direct solve of L_h phi = f (oracle side).

Paper: the elliptic equation (eq. ``elliptic``) is solved with FFTs in the
two uniform periodic directions, which leave one independent tridiagonal
system along the wall-normal direction for each horizontal Fourier mode; the
inverse FFTs then return the correction to physical space ("Fluid domain"
parallelisation subsection, and the remark on the FFT solver's need for
uniform x1, x2 spacing that closes the "Fluid Mechanics" subsection).  The
pressure correction has homogeneous Neumann conditions at the walls and its
arbitrary constant is fixed by a reference value (boundary-condition
paragraph after eq. ``pressure``).

The solver reaches the exact discrete solution (up to rounding), so this is
the plain definition written out:
    L_h phi = f - m,   sum_cells V phi = 0,   m = sum V f / sum V,
with V = dx dz dyf[j] the cell volume.  Steps, in order:
  1. remove the volume-weighted mean m of f (makes the singular Neumann
     problem compatible; the paper is silent on incompatible data);
  2. F = FFT_z(RFFT_x(f)), unnormalised;
  3. for every (kx, kz) != (0, 0): Thomas elimination of
     a_j X_{j-1} + (b_j + lx(kx) + lz(kz)) X_j + c_j X_{j+1} = F_j;
  4. for (0, 0): integrate the face flux from the lower wall, then the
     potential, then remove its weighted mean;
  5. phi = IRFFT_x(IFFT_z(X)).
"""

import numpy as np

from .grid import geometry, lambda_x, lambda_z


def thomas_modes(a, b, c, lam, F):
    """Thomas elimination for many systems sharing a, b, c but with diagonal
    shifts ``lam`` (broadcast against F[0]).  F has shape (ny, ...)."""
    ny = F.shape[0]
    cp = np.empty((ny,) + np.shape(lam), dtype=np.float64)
    dp = np.empty(F.shape, dtype=F.dtype)
    den = b[0] + lam
    cp[0] = c[0] / den
    dp[0] = F[0] / den
    for j in range(1, ny):
        den = b[j] + lam - a[j] * cp[j - 1]
        cp[j] = c[j] / den
        dp[j] = (F[j] - a[j] * dp[j - 1]) / den
    X = np.empty_like(dp)
    X[ny - 1] = dp[ny - 1]
    for j in range(ny - 2, -1, -1):
        X[j] = dp[j] - cp[j] * X[j + 1]
    return X


def zero_mode_flux_integration(g, ghat):
    """(0,0)-mode y problem: (flux[j+1] - flux[j]) / dyf[j] = ghat[j] with
    zero flux at both walls, flux[j] = (X[j] - X[j-1]) / dyc[j]; the
    solution is pinned to zero weighted mean.  ``ghat`` must be compatible
    (sum dyf ghat = 0); the returned residual flux at the upper wall shows how
    far it is from that.  Textbook double integration of the 1-D Neumann
    problem."""
    ny = g.ny
    flux = np.zeros(ny + 1, dtype=np.float64)
    for j in range(ny):
        flux[j + 1] = flux[j] + g.dyf[j] * ghat[j]
    X = np.zeros(ny, dtype=np.float64)
    for j in range(1, ny):
        X[j] = X[j - 1] + g.dyc[j] * flux[j]
    X = X - (g.dyf * X).sum() / g.dyf.sum()
    return X, flux[ny]


def solve_modes(g, F):
    """Step 3 and 4 on the spectral array F[ny, nz, nx//2+1] (unnormalised
    DFT coefficients of a compatible right-hand side)."""
    lam = lambda_z(g).reshape(-1, 1) + lambda_x(g).reshape(1, -1)
    lam_safe = lam.copy()
    lam_safe[0, 0] = -1.0          # placeholder; the (0,0) column is replaced below
    X = thomas_modes(g.a, g.b, g.c, lam_safe, F)
    X00, _ = zero_mode_flux_integration(g, F[:, 0, 0].real)
    X[:, 0, 0] = X00
    return X


def solve(f, Lx, Lz, yf):
    """Solve L_h phi = f - m with zero volume-weighted mean.

    ``f`` is C-ordered ``[ny][nz][nx]``; ``yf`` are the ny+1 wall-normal face
    coordinates; x and z are periodic with lengths Lx and Lz.  Returns
    ``(phi, m)`` where m is the removed volume-weighted mean of f.
    Any nx >= 1, nz >= 1, ny >= 2 is accepted (odd sizes included).
    """
    f = np.asarray(f, dtype=np.float64)
    if f.ndim != 3:
        raise ValueError("f must be 3-D [ny][nz][nx]")
    ny, nz, nx = f.shape
    if not np.all(np.isfinite(f)):
        raise ValueError("f must be finite")
    g = geometry(nx, ny, nz, Lx, Lz, yf)
    w = g.dyf.reshape(-1, 1, 1)
    m = float((w * f).sum() / (g.dyf.sum() * nx * nz))
    F = np.fft.fft(np.fft.rfft(f - m, axis=2), axis=1)
    X = solve_modes(g, F)
    phi = np.fft.irfft(np.fft.ifft(X, axis=1), n=nx, axis=2)
    return phi, m
