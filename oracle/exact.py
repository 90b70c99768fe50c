"""Exact rational solve of the bordered Neumann problem (oracle pin).

Brute force on tiny grids in ``fractions.Fraction`` arithmetic: the matrix of
L_h (staggered centred differences, periodic x and z, Neumann y walls; paper,
"Fluid Mechanics" subsection) is assembled here with its own loops, bordered
by the constant null vector and the cell volumes, and solved by Gauss-Jordan
elimination without rounding.  Used only to write ``tests/golden`` fixtures
and to pin the floating-point oracle.
"""

from fractions import Fraction


def exact_bordered_solve(f, Lx, Lz, yf):
    """f: nested lists [ny][nz][nx] of Fractions/ints; Lx, Lz, yf rational.

    Returns (phi nested lists of Fractions, mu Fraction)."""
    ny = len(f)
    nz = len(f[0])
    nx = len(f[0][0])
    Lx = Fraction(Lx)
    Lz = Fraction(Lz)
    yf = [Fraction(y) for y in yf]
    dx = Lx / nx
    dz = Lz / nz
    h = [yf[j + 1] - yf[j] for j in range(ny)]
    mid = [(yf[j + 1] + yf[j]) / 2 for j in range(ny)]
    N = nx * ny * nz

    def idx(j, k, i):
        return (j * nz + k) * nx + i

    M = [[Fraction(0)] * (N + 2) for _ in range(N + 1)]   # last column: rhs
    for j in range(ny):
        for k in range(nz):
            for i in range(nx):
                r = idx(j, k, i)
                for di in (-1, 1):
                    M[r][idx(j, k, (i + di) % nx)] += 1 / (dx * dx)
                    M[r][r] -= 1 / (dx * dx)
                for dk in (-1, 1):
                    M[r][idx(j, (k + dk) % nz, i)] += 1 / (dz * dz)
                    M[r][r] -= 1 / (dz * dz)
                for dj in (-1, 1):
                    jj = j + dj
                    if 0 <= jj < ny:
                        t = 1 / (h[j] * abs(mid[jj] - mid[j]))
                        M[r][idx(jj, k, i)] += t
                        M[r][r] -= t
                M[r][N] = Fraction(1)
                M[r][N + 1] = Fraction(f[j][k][i])
                M[N][r] = h[j] * dx * dz
    # Gauss-Jordan with exact pivot search for a nonzero entry
    n = N + 1
    for col in range(n):
        piv = next(r for r in range(col, n) if M[r][col] != 0)
        M[col], M[piv] = M[piv], M[col]
        p = M[col][col]
        M[col] = [x / p for x in M[col]]
        for r in range(n):
            if r != col and M[r][col] != 0:
                fac = M[r][col]
                M[r] = [x - fac * y for x, y in zip(M[r], M[col])]
    sol = [M[r][n] for r in range(n)]
    phi = [[[sol[idx(j, k, i)] for i in range(nx)] for k in range(nz)] for j in range(ny)]
    return phi, sol[N]
