"""Pins of the oracle's factored implicit viscous solve (paper: eq.
``nstime_discr`` with Crank-Nicolson viscous terms; "Fluid domain"
parallelisation subsection: direction-wise tridiagonal solves, cyclic in the
two periodic directions).

The oracle solves each direction with a dense matrix; these tests pin it to
(1) the textbook eigenvalues of the periodic second difference, (2) the
already pinned staggered stencils of ``oracle.operators`` (L_h's wall-normal
part at cell centres, G D across the y faces), (3) closed-form eigenvectors
of the uniform-grid wall-normal operators, (4) separability and the
commutation of the three solves, (5) a brute-force solve of the assembled
three-dimensional operator, and (6) planted mistakes that the pins catch."""

import numpy as np
import pytest

import oracle.helmholtz as oh
from oracle.grid import geometry
from oracle.operators import divergence, gradient, laplacian
from paper_2609_19130_amd import synth

PRESSURE_BCS = [("neumann", "neumann"), ("neumann", "dirichlet"), ("dirichlet", "neumann"),
                ("dirichlet", "dirichlet")]


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def grid(nx, ny, nz, beta_s=2.0, bc=("neumann", "neumann")):
    return geometry(nx, ny, nz, 1.7, 0.9, synth.tanh_faces(ny, beta_s), bc=bc)


def periodic_closed_form_ok(A, n, h, beta):
    """A (n x n) must map each Fourier mode cos(2 pi m i / n + th) to itself
    times 1 + (4 beta / h^2) sin^2(pi m / n)."""
    i = np.arange(n)
    worst = 0.0
    for m in range(n):
        for th in (0.0, 0.7):
            v = np.cos(2 * np.pi * m * i / n + th)
            if np.abs(v).max() < 1e-6:
                continue
            mu = 1 + (4 * beta / h ** 2) * np.sin(np.pi * m / n) ** 2
            x = np.linalg.solve(A, v)
            worst = max(worst, rel(x, v / mu))
    return worst


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 12])
@pytest.mark.parametrize("beta", [0.0, 0.01, 0.3, 40.0])
def test_periodic_fourier_closed_form(n, beta):
    h = 0.37
    assert periodic_closed_form_ok(oh.periodic_matrix(n, h, beta), n, h, beta) <= 1e-12


@pytest.mark.parametrize("bc", PRESSURE_BCS)
@pytest.mark.parametrize("beta", [0.002, 0.05, 3.0])
def test_cell_y_against_pinned_stencil(bc, beta):
    """du - beta L_y du = f for a field constant in x and z, with L_y taken
    from the pinned L_h stencil under the velocity wall conditions."""
    g = grid(3, 11, 2, bc=bc)
    gv = geometry(g.nx, g.ny, g.nz, g.Lx, g.Lz, g.yf, bc=oh.velocity_bc(g))
    yprof = np.random.default_rng(5).standard_normal(g.ny) + 0.4
    f = np.broadcast_to(yprof.reshape(-1, 1, 1), (g.ny, g.nz, g.nx)).copy()
    du = oh.factored_solve(f, g, beta)
    assert np.allclose(du, du[:, :1, :1], rtol=0, atol=1e-13 * np.abs(du).max())
    back = du - beta * laplacian(du, gv)
    assert rel(back, f) <= 1e-12


@pytest.mark.parametrize("beta", [0.002, 0.05, 3.0])
def test_face_y_against_pinned_stencils(beta):
    """Across interior faces L_y v = G_y (D_y v) with zero wall rows: the
    pinned divergence and gradient of the projection step."""
    g = grid(2, 9, 3)
    rng = np.random.default_rng(6)
    v = np.zeros((g.ny + 1, g.nz, g.nx))
    prof = rng.standard_normal(g.ny - 1) + 0.2
    v[1:g.ny] = prof.reshape(-1, 1, 1)
    dv = oh.factored_solve(v, g, beta, where="yfaces")
    assert np.all(dv[0] == 0) and np.all(dv[g.ny] == 0)
    z = np.zeros((g.ny, g.nz, g.nx))
    d = divergence(z, dv, z, g)           # (dv[j+1] - dv[j]) / dyf[j]
    gy = gradient(d, g)[1]                # (d[j] - d[j-1]) / dyc[j] at faces 1..ny-1
    back = dv[1:g.ny] - beta * gy[1:g.ny]
    assert rel(back, v[1:g.ny]) <= 1e-12


def uniform_y_modes(vbc, ny, dy):
    """Textbook eigenpairs of the uniform cell-centred second difference:
    Dirichlet-Dirichlet sin((p+1) pi (j+1/2)/ny), mu = -(4/dy^2) sin^2((p+1) pi/(2 ny));
    Dirichlet-Neumann sin((p+1/2) pi (j+1/2)/ny) and Neumann-Dirichlet
    cos((p+1/2) pi (j+1/2)/ny), mu = -(4/dy^2) sin^2((2p+1) pi/(4 ny));
    Neumann-Neumann cos(p pi (j+1/2)/ny), mu = -(4/dy^2) sin^2(p pi/(2 ny))."""
    j = np.arange(ny) + 0.5
    out = []
    for p in range(ny):
        if vbc == ("dirichlet", "dirichlet"):
            v, t = np.sin((p + 1) * np.pi * j / ny), (p + 1) * np.pi / (2 * ny)
        elif vbc == ("dirichlet", "neumann"):
            v, t = np.sin((p + 0.5) * np.pi * j / ny), (2 * p + 1) * np.pi / (4 * ny)
        elif vbc == ("neumann", "dirichlet"):
            v, t = np.cos((p + 0.5) * np.pi * j / ny), (2 * p + 1) * np.pi / (4 * ny)
        else:
            v, t = np.cos(p * np.pi * j / ny), p * np.pi / (2 * ny)
        out.append((-(4 / dy ** 2) * np.sin(t) ** 2, v))
    return out


@pytest.mark.parametrize("bc", PRESSURE_BCS)
def test_uniform_cell_y_closed_form(bc):
    ny, beta = 10, 0.013
    g = grid(1, ny, 1, beta_s=0.0, bc=bc)
    dy = 2.0 / ny
    for mu, v in uniform_y_modes(oh.velocity_bc(g), ny, dy):
        x = np.linalg.solve(oh.cell_y_matrix(g, beta), v)
        assert rel(x, v / (1 - beta * mu)) <= 1e-12


def test_uniform_face_y_closed_form():
    """Interior faces of a uniform grid, zero wall values: sin(m pi j/ny),
    j = 1..ny-1, mu = -(4/dy^2) sin^2(m pi/(2 ny)), m = 1..ny-1."""
    ny, beta = 9, 0.021
    g = grid(1, ny, 1, beta_s=0.0)
    dy = 2.0 / ny
    j = np.arange(1, ny)
    for m in range(1, ny):
        v = np.sin(m * np.pi * j / ny)
        mu = -(4 / dy ** 2) * np.sin(m * np.pi / (2 * ny)) ** 2
        x = np.linalg.solve(oh.face_y_matrix(g, beta), v)
        assert rel(x, v / (1 - beta * mu)) <= 1e-12


@pytest.mark.parametrize("where", ["cells", "yfaces"])
def test_separable_fields(where):
    """Periodic Fourier modes in x and z times any y profile: the x and z
    solves divide by their closed-form factors, the y solve acts on the
    profile alone."""
    g = grid(6, 7, 5)
    beta = 0.04
    ny_ = g.ny if where == "cells" else g.ny + 1
    prof = np.random.default_rng(7).standard_normal(ny_)
    if where == "yfaces":
        prof[0] = prof[-1] = 0.0
    i, k = np.arange(g.nx), np.arange(g.nz)
    for mx, mz in [(0, 0), (1, 2), (3, 4), (2, 0)]:
        cx = np.cos(2 * np.pi * mx * i / g.nx + 0.3)
        cz = np.cos(2 * np.pi * mz * k / g.nz - 1.1)
        f = prof.reshape(-1, 1, 1) * cz.reshape(1, -1, 1) * cx.reshape(1, 1, -1)
        yonly = oh.factored_solve(np.broadcast_to(prof.reshape(-1, 1, 1), f.shape).copy(), g, beta, where)[:, 0, 0]
        mux = 1 + (4 * beta / g.dx ** 2) * np.sin(np.pi * mx / g.nx) ** 2
        muz = 1 + (4 * beta / g.dz ** 2) * np.sin(np.pi * mz / g.nz) ** 2
        want = yonly.reshape(-1, 1, 1) * cz.reshape(1, -1, 1) * cx.reshape(1, 1, -1) / (mux * muz)
        assert rel(oh.factored_solve(f, g, beta, where), want) <= 1e-12


@pytest.mark.parametrize("where", ["cells", "yfaces"])
@pytest.mark.parametrize("bc", [("neumann", "neumann"), ("neumann", "dirichlet")])
def test_solves_commute(where, bc):
    if where == "yfaces" and bc != ("neumann", "neumann"):
        pytest.skip("y-face component defined for prescribed-velocity walls only")
    g = grid(5, 8, 4, bc=bc)
    shape = (g.ny if where == "cells" else g.ny + 1, g.nz, g.nx)
    f = np.random.default_rng(8).standard_normal(shape)
    a = oh.factored_solve(f, g, 0.07, where, order="xzy")
    for order in ("yzx", "zyx", "yxz"):
        assert rel(oh.factored_solve(f, g, 0.07, where, order=order), a) <= 1e-13


@pytest.mark.parametrize("where", ["cells", "yfaces"])
def test_beta_zero_is_identity(where):
    g = grid(4, 6, 3)
    shape = (g.ny if where == "cells" else g.ny + 1, g.nz, g.nx)
    f = np.random.default_rng(9).standard_normal(shape)
    out = oh.factored_solve(f, g, 0.0, where)
    want = f.copy()
    if where == "yfaces":
        want[0] = want[-1] = 0.0
    np.testing.assert_array_equal(out, want)


def forward_matrix(g, beta, where):
    """The assembled 3-D factored operator, column by column, from forward
    stencils: periodic second differences by rolls (their eigenvalues are
    pinned above) and the pinned L_h / G D stencils for y."""
    shape = (g.ny if where == "cells" else g.ny - 1, g.nz, g.nx)
    gv = geometry(g.nx, g.ny, g.nz, g.Lx, g.Lz, g.yf, bc=oh.velocity_bc(g))
    gn = geometry(g.nx, g.ny, g.nz, g.Lx, g.Lz, g.yf)

    def ax(f):
        return f - beta * (np.roll(f, -1, 2) - 2 * f + np.roll(f, 1, 2)) / g.dx ** 2

    def az(f):
        return f - beta * (np.roll(f, -1, 1) - 2 * f + np.roll(f, 1, 1)) / g.dz ** 2

    def ay(f):
        if where == "cells":
            # laplacian of a field minus its x and z parts = the y part
            return f - beta * (laplacian(f, gv) - (ax(f) - f) / -beta - (az(f) - f) / -beta)
        v = np.zeros((g.ny + 1, g.nz, g.nx))
        v[1:g.ny] = f
        z = np.zeros((g.ny, g.nz, g.nx))
        return f - beta * gradient(divergence(z, v, z, gn), gn)[1][1:g.ny]

    n = int(np.prod(shape))
    M = np.zeros((n, n))
    for c in range(n):
        e = np.zeros(n)
        e[c] = 1.0
        M[:, c] = ax(az(ay(e.reshape(shape)))).ravel()
    return M, shape


@pytest.mark.parametrize("where", ["cells", "yfaces"])
@pytest.mark.parametrize("bc", [("neumann", "neumann"), ("dirichlet", "neumann")])
def test_bruteforce_3d_operator(where, bc):
    if where == "yfaces" and bc != ("neumann", "neumann"):
        pytest.skip("y-face component defined for prescribed-velocity walls only")
    g = grid(3, 5, 4, bc=bc)
    beta = 0.09
    M, shape = forward_matrix(g, beta, where)
    f = np.random.default_rng(10).standard_normal(shape)
    want = np.linalg.solve(M, f.ravel()).reshape(shape)
    if where == "cells":
        got = oh.factored_solve(f, g, beta)
    else:
        full = np.zeros((g.ny + 1, g.nz, g.nx))
        full[1:g.ny] = f
        got = oh.factored_solve(full, g, beta, "yfaces")[1:g.ny]
    assert rel(got, want) <= 1e-12


def test_face_component_needs_prescribed_walls():
    g = grid(2, 5, 2, bc=("neumann", "dirichlet"))
    with pytest.raises(ValueError):
        oh.factored_solve(np.zeros((6, 2, 2)), g, 0.1, "yfaces")


def test_planted_mistakes_are_caught():
    """Mistakes planted in copies of the oracle's matrices fail the pins."""
    n, h, beta = 8, 0.37, 0.3
    no_corners = oh.periodic_matrix(n, h, beta)
    no_corners[0, n - 1] = no_corners[n - 1, 0] = 0.0
    assert periodic_closed_form_ok(no_corners, n, h, beta) > 1e-3
    wrong_sign = oh.periodic_matrix(n, h, beta)
    wrong_sign -= 2 * np.diag(np.diag(wrong_sign)) - 2 * np.eye(n)   # 1 - 2r on the diagonal
    assert periodic_closed_form_ok(wrong_sign, n, h, beta) > 1e-3
    # pressure walls instead of velocity walls in y
    g = grid(1, 9, 1)
    gv = geometry(1, 9, 1, g.Lx, g.Lz, g.yf, bc=oh.velocity_bc(g))
    gp_ = geometry(1, 9, 1, g.Lx, g.Lz, g.yf, bc=g.bc)
    yprof = np.random.default_rng(11).standard_normal(9) + 0.4
    A_wrong = np.eye(9) - 0.05 * np.diag(-(gp_.a + gp_.c)) - 0.05 * (np.diag(gp_.a[1:], -1) + np.diag(gp_.c[:-1], 1))
    du = np.linalg.solve(A_wrong, yprof).reshape(-1, 1, 1)
    assert rel(du - 0.05 * laplacian(du, gv), yprof.reshape(-1, 1, 1)) > 1e-3
