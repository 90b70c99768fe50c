"""Pins of the oracle's Dirichlet-wall variant (paper: the ``neumann_velocity``
option gives the pressure correction a homogeneous Dirichlet condition at
the upper wall; boundary-condition paragraph and input-variable table).

Each wall is "neumann" or "dirichlet"; a Dirichlet wall holds phi = 0 on the
wall face, half a cell from the nearest centre.  With a Dirichlet wall the
discrete problem is non-singular: no mean is removed and no constant fixed.
Pinned against (1) a dense direct solve of the assembled stencil, (2)
closed-form eigenvectors of the uniform-grid y operator, (3) manufactured
solutions on stretched grids, and (4) planted mistakes that the pins must
catch."""

import numpy as np
import pytest

import oracle
import oracle.poisson as op
from oracle.grid import geometry, lambda_x, lambda_z
from oracle.operators import laplacian
from paper_2609_19130_amd import synth

BCS = [("neumann", "dirichlet"), ("dirichlet", "neumann"), ("dirichlet", "dirichlet")]


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("nx,ny,nz", [(4, 5, 3), (3, 6, 2), (5, 4, 1), (2, 7, 4)])
def test_dirichlet_matches_dense_solve(bc, nx, ny, nz):
    yf = synth.tanh_faces(ny, 2.0)
    f = np.random.default_rng(nx * 100 + ny * 10 + nz).standard_normal((ny, nz, nx)) + 0.3
    phi, m = oracle.solve(f, 1.7, 0.9, yf, bc=bc)
    ref, mu = oracle.dense_solve(f, 1.7, 0.9, yf, bc=bc)
    assert m == 0.0 and mu == 0.0
    assert rel(phi, ref) <= 1e-12


def closed_form_y(bc, ny, dy):
    """Eigenpairs of the uniform cell-centred y operator (textbook):
    Neumann-Dirichlet cos((p+1/2) pi (j+1/2)/ny), Dirichlet-Neumann
    sin((p+1/2) pi (j+1/2)/ny), both with mu = -(4/dy^2) sin^2((2p+1) pi/(4 ny));
    Dirichlet-Dirichlet sin((p+1) pi (j+1/2)/ny) with
    mu = -(4/dy^2) sin^2((p+1) pi/(2 ny))."""
    j = np.arange(ny) + 0.5
    out = []
    for p in range(ny):
        if bc == ("neumann", "dirichlet"):
            v, t = np.cos((p + 0.5) * np.pi * j / ny), (2 * p + 1) * np.pi / (4 * ny)
        elif bc == ("dirichlet", "neumann"):
            v, t = np.sin((p + 0.5) * np.pi * j / ny), (2 * p + 1) * np.pi / (4 * ny)
        else:
            v, t = np.sin((p + 1) * np.pi * j / ny), (p + 1) * np.pi / (2 * ny)
        out.append((-(4 / dy ** 2) * np.sin(t) ** 2, v))
    return out


@pytest.mark.parametrize("bc", BCS)
def test_dirichlet_uniform_closed_form(bc):
    nx, ny, nz = 8, 12, 6
    Lx, Lz = 2.0, 3.0
    yf = synth.tanh_faces(ny, 0.0)
    g = geometry(nx, ny, nz, Lx, Lz, yf, bc=bc)
    dy = 2.0 / ny
    pairs = closed_form_y(bc, ny, dy)
    x = (np.arange(nx) + 0.5) * (Lx / nx)
    z = (np.arange(nz) + 0.5) * (Lz / nz)
    rng = np.random.default_rng(3)
    phi = np.zeros((ny, nz, nx))
    f = np.zeros((ny, nz, nx))
    for kx, kz, p in [(0, 0, 0), (1, 2, 3), (3, 0, 1), (2, 5, 11), (4, 3, 6)]:
        amp, th = rng.standard_normal(), rng.uniform(0, 2 * np.pi)
        mu, v = pairs[p]
        lam = -(4 / (Lx / nx) ** 2) * np.sin(np.pi * kx / nx) ** 2 - (4 / (Lz / nz) ** 2) * np.sin(np.pi * kz / nz) ** 2
        wave = np.cos(2 * np.pi * kx * x[None, :] / Lx + 2 * np.pi * kz * z[:, None] / Lz + th)
        phi += amp * v[:, None, None] * wave[None]
        f += amp * (lam + mu) * v[:, None, None] * wave[None]
    assert rel(laplacian(phi, g), f) <= 1e-12          # the closed form is an eigen-solution of L_h
    sol, m = oracle.solve(f, Lx, Lz, yf, bc=bc)
    assert m == 0.0
    assert rel(sol, phi) <= 1e-12


@pytest.mark.parametrize("bc", BCS)
def test_dirichlet_manufactured_stretched(bc):
    nx, ny, nz = 16, 40, 12
    yf = synth.tanh_faces(ny, 2.5)
    g = geometry(nx, ny, nz, 2 * np.pi, 1.3, yf, bc=bc)
    mu, V = oracle.y_eigenpairs(g)
    for p in (0, 1, 7, ny - 1):   # eigen-relation through the oracle's operator
        e = np.zeros((ny, 1, 1))
        e[:, 0, 0] = V[:, p]
        assert np.abs(laplacian(e, geometry(1, ny, 1, 1.0, 1.0, yf, bc=bc))[:, 0, 0] - mu[p] * V[:, p]).max() \
            <= 1e-9 * abs(mu).max()
    modes = [(0, 0, 0, 1.0, 0.3), (1, 1, 2, -0.7, 1.1), (3, -2, 5, 0.4, 2.0), (8, 6, ny - 1, 0.2, 0.5)]
    phi, f = oracle.manufactured_field(nx, ny, nz, 2 * np.pi, 1.3, yf, modes, bc=bc)
    sol, m = oracle.solve(f, 2 * np.pi, 1.3, yf, bc=bc)
    assert m == 0.0
    assert rel(sol, phi) <= 1e-11


def test_dirichlet_pins_catch_planted_mistakes(monkeypatch):
    """Plausible mistakes in the Dirichlet variant must fail the pins."""
    bc = ("dirichlet", "neumann")
    nx, ny, nz = 3, 6, 2
    yf = synth.tanh_faces(ny, 2.0)
    f = np.random.default_rng(5).standard_normal((ny, nz, nx))
    ref, _ = oracle.dense_solve(f, 1.0, 1.0, yf, bc=bc)

    # 1. elimination started with eps_{-1} = 0 (ignores the lower wall term)
    orig = op.thomas_modes

    def thomas_eps0(a, c, L, F):
        a2 = a.copy()
        a2[0] = 0.0
        return orig(a2, c, L, F)
    with monkeypatch.context() as m, np.errstate(divide="ignore", invalid="ignore"):
        m.setattr(op, "thomas_modes", thomas_eps0)
        assert not rel(op.solve(f, 1.0, 1.0, yf, bc=bc)[0], ref) <= 1e-6   # NaN (singular) also caught

    # 2. wall coefficient with a full-cell distance (1 / dyf^2 instead of 2 / dyf^2)
    import oracle.grid as og
    geo = og.geometry

    def geometry_full_cell(*args, **kw):
        g = geo(*args, **kw)
        if g.bc[0] == "dirichlet":
            g.a[0] *= 0.5
            g.b[0] = -(g.a[0] + g.c[0])
        return g
    with monkeypatch.context() as m:
        m.setattr(op, "geometry", geometry_full_cell)
        assert not rel(op.solve(f, 1.0, 1.0, yf, bc=bc)[0], ref) <= 1e-6   # NaN (singular) also caught

    # 3. the mean removed as if the problem were singular
    def solve_mean_removed(f, Lx, Lz, yf, bc):
        phi, _ = op.solve(f - f.mean(), Lx, Lz, yf, bc=bc)
        return phi
    assert rel(solve_mean_removed(f + 1.0, 1.0, 1.0, yf, bc), oracle.dense_solve(f + 1.0, 1.0, 1.0, yf, bc=bc)[0]) > 1e-6


@pytest.mark.parametrize("bc", [("neumann", "neumann")] + BCS)
def test_fractional_step_invariants(bc):
    """One projection substep with mass sources q (eqs. ``velsolen``,
    ``elliptic``, ``pressure``): after phi solves lap(phi) = (D u* - q)/(alpha dt),
    the projected velocity satisfies D u_{n+1} = q (plus alpha dt m when a
    Neumann-Neumann solve removes an incompatible mean m), and the pressure
    update is p + phi - visc L_h phi.  Holds because L_h = D G also at
    Dirichlet wall faces."""
    nx, ny, nz = 12, 10, 8
    yf = synth.tanh_faces(ny, 2.0)
    g = geometry(nx, ny, nz, 2 * np.pi, 1.5, yf, bc=bc)
    u, v, w = synth.uniform_velocity(nx, ny, nz, seed=21)
    q = np.random.default_rng(22).standard_normal((ny, nz, nx)) * 0.1
    alpha_dt, visc = 0.037, 0.002
    f = oracle.rhs_from_velocity(u, v, w, q, g, alpha_dt)
    phi, m = oracle.solve(f, 2 * np.pi, 1.5, yf, bc=bc)
    p = np.random.default_rng(23).standard_normal((ny, nz, nx))
    un, vn, wn, pn = oracle.projection_step(u, v, w, p, phi, g, alpha_dt, visc)
    div = oracle.divergence(un, vn, wn, g)
    assert np.abs(div - q - alpha_dt * m).max() <= 1e-12 * np.abs(oracle.divergence(u, v, w, g)).max()
    if bc[0] == "neumann":
        assert np.array_equal(vn[0], v[0])
    if bc[1] == "neumann":
        assert np.array_equal(vn[ny], v[ny])
    assert np.allclose(pn, p + phi - visc * laplacian(phi, g), rtol=0, atol=1e-14)
