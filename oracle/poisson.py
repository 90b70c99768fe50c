"""FFT + tridiagonal direct solve of L_h phi = f (oracle side).

Paper: the elliptic equation (eq. ``elliptic``) is solved with FFTs in the
two uniform periodic directions, which leave one independent tridiagonal
system along the wall-normal direction for each horizontal Fourier mode; the
inverse FFTs then return the correction to physical space ("Fluid domain"
parallelisation subsection, and the remark on the FFT solver's need for
uniform x1, x2 spacing that closes the "Fluid Mechanics" subsection).  The
pressure correction has homogeneous Neumann conditions at the walls and its
arbitrary constant is fixed by a reference value (boundary-condition
paragraph after eq. ``pressure``); with the ``neumann_velocity`` outlet
option the upper wall takes a homogeneous Dirichlet condition instead, and
the problem is no longer singular.

The solver reaches the exact discrete solution (up to rounding), so this is
the plain definition written out.  Neumann at both walls:
    L_h phi = f - m,   sum_cells V phi = 0,   m = sum V f / sum V,
with V = dx dz dyf[j] the cell volume; with a Dirichlet wall, L_h phi = f
(m = 0, no constant to fix).  Steps, in order:
  1. remove the volume-weighted mean m of f (makes the singular Neumann
     problem compatible; the paper is silent on incompatible data);
  2. F = FFT_z(RFFT_x(f)), unnormalised;
  3. for every (kx, kz) != (0, 0): Thomas elimination of
     a_j X_{j-1} + (b_j + lx(kx) + lz(kz)) X_j + c_j X_{j+1} = F_j,
     b_j = -(a_j + c_j) (see ``thomas_modes`` for the pivot form);
  4. for (0, 0), Neumann at both walls: integrate the face flux from the
     lower wall, then the potential, then remove its weighted mean (with a
     Dirichlet wall (0, 0) is an ordinary system of step 3, shift 0);
  5. phi = IRFFT_x(IFFT_z(X)).
"""

import numpy as np

from .grid import geometry, lambda_x, lambda_z


def thomas_modes(a, c, L, F):
    """Thomas elimination for many systems sharing the face coefficients a, c,
    each with its own shift L = -lambda >= 0 (broadcast against F[0]):

        a_j X_{j-1} - (a_j + c_j + L) X_j + c_j X_{j+1} = F_j,   X_{-1} = X_{ny} = 0

    (a_0 = 0 or c_{ny-1} = 0 at a Neumann wall; at a Dirichlet wall the
    outside value is the wall value 0).  The diagonal of the y operator is
    minus the sum of the two face coefficients (the operator is a difference
    of face fluxes), so the elimination is written with eps_j = 1 - g_j,
    where X_j = g_j X_{j+1} + d'_j is the back-substitution form: the pivot
    is -(c_j + L + a_j eps_{j-1}), a sum of non-negative terms, and the
    diagonal is never formed or rounded.  eps_{-1} = 1 because the value
    beyond the lower wall does not depend on X_0 (g_{-1} = 0).  In exact
    arithmetic this is the textbook Thomas algorithm; in floating point it
    avoids the cancellation that costs plain Thomas up to ~1e-11 relative
    accuracy on the near-singular low modes of stretched grids.
    """
    ny = F.shape[0]
    L = np.asarray(L, dtype=np.float64)
    D = np.empty((ny,) + L.shape, dtype=np.float64)     # minus the pivots
    dp = np.empty(F.shape, dtype=F.dtype)
    eps = np.ones(L.shape, dtype=np.float64)
    prev = np.zeros(F.shape[1:], dtype=F.dtype)
    for j in range(ny):
        n = L + a[j] * eps
        D[j] = c[j] + n
        eps = n / D[j]
        dp[j] = (a[j] * prev - F[j]) / D[j]
        prev = dp[j]
    X = np.empty_like(dp)
    X[ny - 1] = dp[ny - 1]
    for j in range(ny - 2, -1, -1):
        X[j] = dp[j] + (c[j] / D[j]) * X[j + 1]
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
    L = -(lambda_z(g).reshape(-1, 1) + lambda_x(g).reshape(1, -1))
    if g.singular:
        L[0, 0] = 1.0              # placeholder; the singular (0,0) column is replaced below
    X = thomas_modes(g.a, g.c, L, F)
    if g.singular:
        X00, _ = zero_mode_flux_integration(g, F[:, 0, 0].real)
        X[:, 0, 0] = X00
    return X


def solve(f, Lx, Lz, yf, bc=("neumann", "neumann"), workers=None):
    """Solve L_h phi = f - m with zero volume-weighted mean (Neumann walls),
    or L_h phi = f when a wall is Dirichlet (``bc`` = (lower, upper), each
    "neumann" or "dirichlet"; m = 0 then).

    ``f`` is C-ordered ``[ny][nz][nx]``; ``yf`` are the ny+1 wall-normal face
    coordinates; x and z are periodic with lengths Lx and Lz.  Returns
    ``(phi, m)`` where m is the removed volume-weighted mean of f.
    Any nx >= 1, nz >= 1, ny >= 2 is accepted (odd sizes included).
    ``workers``: None takes numpy's FFTs (one thread); an integer takes
    scipy.fft's with that many threads (the same transforms; timing only).
    """
    f = np.asarray(f, dtype=np.float64)
    if f.ndim != 3:
        raise ValueError("f must be 3-D [ny][nz][nx]")
    ny, nz, nx = f.shape
    if not np.all(np.isfinite(f)):
        raise ValueError("f must be finite")
    g = geometry(nx, ny, nz, Lx, Lz, yf, bc=bc)
    w = g.dyf.reshape(-1, 1, 1)
    m = float((w * f).sum() / (g.dyf.sum() * nx * nz)) if g.singular else 0.0
    if workers is None:
        F = np.fft.fft(np.fft.rfft(f - m, axis=2), axis=1)
    else:
        import scipy.fft as sfft
        F = sfft.fft(sfft.rfft(f - m, axis=2, workers=workers), axis=1, workers=workers)
    X = solve_modes(g, F)
    if workers is None:
        phi = np.fft.irfft(np.fft.ifft(X, axis=1), n=nx, axis=2)
    else:
        phi = sfft.irfft(sfft.ifft(X, axis=1, workers=workers), n=nx, axis=2, workers=workers)
    return phi, m
