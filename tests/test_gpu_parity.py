"""GPU parity of libibpoisson against the CPU oracle (run on an MI355X).

FP64: ||phi_gpu - phi_oracle|| / ||phi_oracle|| <= 1e-12 (both carry zero
volume-weighted mean, so no constant is removed before comparing).
Mixed forms: relative residual ||f - m - L_h phi|| / ||f - m|| <= 1e-10,
recomputed here on the CPU with the oracle's FP64 operator.
"""

import numpy as np
import pytest
import torch

import oracle
from oracle.grid import geometry
from oracle.operators import divergence, gradient, laplacian, weighted_mean
from paper_2609_19130_amd import ibpoisson as ibp
from paper_2609_19130_amd import synth

from gpu_helpers import gpu_solve, rel, require_gpu, to_dev

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
RTOL_MIXED = 1e-10


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def residual(f, phi, Lx, Lz, yf):
    ny, nz, nx = f.shape
    g = geometry(nx, ny, nz, Lx, Lz, yf)
    m = weighted_mean(f, g)
    r = (f - m) - laplacian(phi, g)
    return float(np.linalg.norm(r.ravel()) / np.linalg.norm((f - m).ravel()))


def residual_vw_and_eta(f, phi, Lx, Lz, yf):
    """Volume-weighted relative residual ||V r|| / ||V (f - m)|| and the
    normwise backward error ||r||_inf / (||L_h||_inf ||phi||_inf + ||f - m||_inf),
    with the oracle's operator; ||L_h||_inf is the largest absolute row sum
    of the stencil, 4/dx^2 + 4/dz^2 + max_j 2 (a_j + c_j)."""
    ny, nz, nx = f.shape
    g = geometry(nx, ny, nz, Lx, Lz, yf)
    m = weighted_mean(f, g)
    r = (f - m) - laplacian(phi, g)
    w = g.dyf.reshape(-1, 1, 1)
    rvw = float(np.linalg.norm((w * r).ravel()) / np.linalg.norm((w * (f - m)).ravel()))
    lnorm = (4 / g.dx ** 2 if nx > 1 else 0.0) + (4 / g.dz ** 2 if nz > 1 else 0.0) + float(np.max(2 * (g.a + g.c)))
    eta = float(np.abs(r).max() / (lnorm * np.abs(phi).max() + np.abs(f - m).max()))
    return rvw, eta


# ---------------------------------------------------------------- FP64 parity
SHAPES = [  # (nx, ny, nz, beta): several tiles, ragged tails, every radix
    (2, 2, 1, 1.0), (4, 3, 2, 2.0), (6, 5, 3, 2.0), (8, 7, 5, 2.5), (12, 9, 6, 3.0),
    (16, 17, 10, 2.0), (22, 33, 11, 2.0), (32, 40, 24, 1.5), (40, 100, 14, 2.5),
    (176, 20, 30, 2.0), (112, 45, 7, 3.0), (96, 130, 9, 2.0), (30, 400, 18, 3.0),
    (20, 777, 4, 3.0),
    # power-of-two lengths take the register-FFT kernels (x, z or both)
    (64, 20, 32, 2.0), (128, 33, 64, 2.5), (256, 17, 128, 2.0), (512, 9, 512, 3.0),
    (1024, 6, 1024, 2.0), (32, 50, 20, 2.0), (48, 30, 256, 2.0), (64, 3, 1024, 1.0),
    # nz = nx with register-FFT lengths: fused persistent x/z passes
    (32, 5, 32, 2.0), (64, 19, 64, 2.5), (128, 40, 128, 2.0), (256, 11, 256, 3.0),
]

# every line-solve shape the dispatcher picks (lanes x rows per lane): 32 x 12
# for 257 <= ny <= 384 (the 512x384x512 benchmark's instance, FP64 8 and FP32
# 16 columns per block), 64 x 12 for 513..768 (the 1024x768x1024 one), 64 x 16
# and 64 x 24 up to the 1536-row limit, each at the bottom and the top of its
# range
LINE_SHAPES = [
    (64, 300, 48, 2.0), (48, 384, 40, 2.5), (32, 600, 16, 3.0), (16, 768, 24, 2.0),
    (12, 1024, 10, 2.0), (10, 1100, 6, 3.0), (8, 1536, 4, 2.0),
]


@pytest.mark.parametrize("nx,ny,nz,beta", SHAPES + LINE_SHAPES)
def test_fp64_matches_oracle(nx, ny, nz, beta):
    rng = np.random.default_rng(nx * 1000 + ny * 10 + nz)
    Lx, Lz = 2 * np.pi, 1.7
    yf = synth.tanh_faces(ny, beta)
    f = rng.uniform(-1, 1, (ny, nz, nx)) + 0.25      # incompatible: mean removed and reported
    phi, info = gpu_solve(f, Lx, Lz, yf)
    ref, m = oracle.solve(f, Lx, Lz, yf)
    assert rel(phi, ref) <= TOL64, rel(phi, ref)
    assert abs(info["removed_mean"] - m) <= 1e-14 * max(1.0, abs(m))
    assert info["converged"] == 1 and info["iterations"] == 0 and info["nonfinite_input"] == 0


def test_c1_divergence_rhs_and_projection():
    nx = ny = nz = 64
    Lx = Lz = 2 * np.pi
    yf = synth.tanh_faces(ny, 2.0)
    g = geometry(nx, ny, nz, Lx, Lz, yf)
    u, v, w = synth.uniform_velocity(nx, ny, nz, seed=1)
    f = divergence(u, v, w, g)
    plan = ibp.Plan(nx, ny, nz, Lx, Lz, yf)
    fd = plan.divergence(to_dev(u), to_dev(v), to_dev(w))
    f_gpu = fd.cpu().numpy()
    assert np.max(np.abs(f_gpu - f)) <= 1e-13 * np.max(np.abs(f))
    phi = plan.solve(to_dev(f)).cpu().numpy()
    ref, _ = oracle.solve(f, Lx, Lz, yf)
    assert rel(phi, ref) <= TOL64
    gx, gy, gz = gradient(phi, g)
    d = divergence(u - gx, v - gy, w - gz, g)
    assert np.max(np.abs(d)) / np.max(np.abs(f)) <= 1e-12


def test_c2_manufactured_256():
    n = 256
    Lx = Lz = 2 * np.pi
    yf = synth.tanh_faces(n, 2.5)
    modes = synth.eigen_modes(seed=2, count=32, kmax=16, pmax=16)
    phis, f = oracle.manufactured_field(n, n, n, Lx, Lz, yf, modes)
    phi, info = gpu_solve(f, Lx, Lz, yf)
    assert rel(phi, phis) <= TOL64, rel(phi, phis)
    ref, _ = oracle.solve(f, Lx, Lz, yf)
    assert rel(phi, ref) <= TOL64


def test_in_place_and_determinism():
    nx, ny, nz = 48, 37, 20
    Lx, Lz = 3.0, 2.0
    yf = synth.tanh_faces(ny, 2.0)
    f = np.random.default_rng(3).standard_normal((ny, nz, nx))
    plan = ibp.Plan(nx, ny, nz, Lx, Lz, yf)
    fd = to_dev(f)
    a = plan.solve(fd).clone()
    b = plan.solve(fd).clone()
    assert torch.equal(a, b), "two solves of the same input differ"
    x = fd.clone()
    plan.solve(x, x)                     # phi aliases rhs
    assert torch.equal(x, a)
    assert np.array_equal(fd.cpu().numpy(), f)   # rhs untouched by out-of-place solves


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("nx,ny,nz,chunk", [(64, 40, 32, 3), (48, 37, 24, 5), (128, 21, 64, 7)])
def test_plane_chunking_is_bitwise_neutral(monkeypatch, precision, nx, ny, nz, chunk):
    """x/z passes run chunk by chunk of y planes on two streams: results are
    bitwise those of whole-grid launches (ragged last chunk included)."""
    Lx, Lz = 2 * np.pi, 1.3
    yf = synth.tanh_faces(ny, 2.5)
    f = np.random.default_rng(nx + ny + nz).standard_normal((ny, nz, nx))
    monkeypatch.setenv("IBP_CHUNK", "0")
    a, _ = gpu_solve(f, Lx, Lz, yf, precision=precision, max_iters=3)
    monkeypatch.setenv("IBP_CHUNK", str(chunk))
    b, info = gpu_solve(f, Lx, Lz, yf, precision=precision, max_iters=3)
    assert np.array_equal(a, b)
    if precision == "fp64":
        ref, _ = oracle.solve(f, Lx, Lz, yf)
        assert rel(b, ref) <= TOL64


FUSED_CASES = [(128, 19, 128), (256, 11, 256), (512, 9, 512), (1024, 3, 1024)]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("nx,ny,nz", FUSED_CASES)
def test_fused_xz_matches_separate_passes(monkeypatch, precision, nx, ny, nz):
    """The fused persistent x/z passes against the separate x and z kernels:
    bitwise for FP64; the mixed form differs only in the order of its norm
    partial sums, so it is held to the refinement's own accuracy."""
    Lx, Lz = 2 * np.pi, 1.1
    yf = synth.tanh_faces(ny, 2.0)
    f = np.random.default_rng(nx + 7 * ny).standard_normal((ny, nz, nx))
    monkeypatch.setenv("IBP_FUSED", "0")
    a, _ = gpu_solve(f, Lx, Lz, yf, precision=precision, max_iters=3)
    monkeypatch.setenv("IBP_FUSED", "1")
    b, info = gpu_solve(f, Lx, Lz, yf, precision=precision, max_iters=3)
    ref, _ = oracle.solve(f, Lx, Lz, yf)
    if precision == "fp64":
        assert np.array_equal(a, b)
        assert rel(b, ref) <= TOL64
    else:
        assert info["converged"] == 1 and info["rel_residual"] <= 1e-10
        assert rel(b, ref) <= 1e-8


@pytest.mark.parametrize("lag,bpcu", [("1", "1"), ("1", ""), ("2", "1"), ("1000", "")])
def test_fused_schedule_is_bitwise_neutral(monkeypatch, lag, bpcu):
    """Any lag between a plane's first- and second-stage items and any
    persistent grid size give the same bits (lag 1 makes most second-stage
    items wait on their plane's counter; lag >= ny runs the stages apart)."""
    nx = nz = 256
    ny = 13
    Lx, Lz = 2 * np.pi, 2.0
    yf = synth.tanh_faces(ny, 2.0)
    f = np.random.default_rng(11).standard_normal((ny, nz, nx))
    monkeypatch.setenv("IBP_FUSED", "0")
    a, _ = gpu_solve(f, Lx, Lz, yf)
    monkeypatch.setenv("IBP_FUSED", "1")
    monkeypatch.setenv("IBP_FUSED_LAG", lag)
    monkeypatch.setenv("IBP_FUSED_BPCU", bpcu)
    for _ in range(3):   # the counters re-arm between launches
        b, _ = gpu_solve(f, Lx, Lz, yf)
        assert np.array_equal(a, b)


def test_caller_workspace():
    nx, ny, nz = 32, 24, 16
    Lx, Lz = 1.0, 1.0
    yf = synth.tanh_faces(ny, 2.0)
    f = np.random.default_rng(4).standard_normal((ny, nz, nx))
    plan = ibp.Plan(nx, ny, nz, Lx, Lz, yf)
    a = plan.solve(to_dev(f)).clone()
    ws = torch.empty(plan.workspace_size() + 256, dtype=torch.uint8, device="cuda")
    off = (-ws.data_ptr()) % 256
    plan.set_workspace(ws[off:off + plan.workspace_size()])
    b = plan.solve(to_dev(f))
    assert torch.equal(a, b)
    with pytest.raises(ibp.IbpError):
        plan.set_workspace(ws[off:off + 1024])


def test_nonfinite_input_flagged():
    nx, ny, nz = 16, 12, 8
    yf = synth.tanh_faces(ny, 2.0)
    f = np.random.default_rng(5).standard_normal((ny, nz, nx))
    f[3, 2, 5] = np.nan
    _, info = gpu_solve(f, 1.0, 1.0, yf)
    assert info["nonfinite_input"] == 1


# ---------------------------------------------------------------- mixed forms
# Mixed against FP64 at the same input: the refinement's target is the
# residual (<= 1e-10); the error it leaves depends on where the residual sits
# in the spectrum.  Read as for the paper-scale sequence, mixed agrees with
# FP64 to 1e-10 relative.  Measured on MI355X: at most 6.7e-11 (32x600x16,
# beta 3, the most stretched small grid), 2.8e-15 to 6.3e-15 at 512x384x512,
# where the FP64 tolerance 1e-12 is held as well.
TOL_MIXED_VS_FP64 = 1e-10
TOL_MIXED_VS_FP64_C3 = 1e-12


MIXED_FORMS = ["mixed", "mixed_f64sweep", "mixed_f64inv"]


@pytest.mark.parametrize("precision", MIXED_FORMS)
@pytest.mark.parametrize("nx,ny,nz,beta", [(64, 64, 64, 2.0), (40, 100, 14, 3.0), (176, 33, 30, 2.5),
                                           (96, 40, 1, 2.0), (26, 50, 22, 2.0), (30, 60, 263, 2.0),
                                           (64, 300, 48, 2.0), (48, 384, 40, 2.5), (32, 600, 16, 3.0),
                                           (16, 768, 24, 2.0)])
def test_mixed_refinement(precision, nx, ny, nz, beta):
    Lx = Lz = 2 * np.pi
    yf = synth.tanh_faces(ny, beta)
    g = geometry(nx, ny, nz, Lx, Lz, yf)
    u, v, w = synth.uniform_velocity(nx, ny, nz, seed=7)
    f = divergence(u, v, w, g)
    phi, info = gpu_solve(f, Lx, Lz, yf, precision=precision, rtol=RTOL_MIXED, max_iters=6)
    r = residual(f, phi, Lx, Lz, yf)
    assert info["converged"] == 1, info
    assert r <= RTOL_MIXED, (r, info)
    assert abs(info["rel_residual"] - r) <= 0.05 * r + 1e-14
    assert 1 <= info["iterations"] <= 6
    assert len(info["residual_history"]) == info["iterations"] + 1
    assert abs(info["residual_history"][-1] - info["rel_residual"]) <= 1e-15 + 1e-12 * r
    rvw, eta = residual_vw_and_eta(f, phi, Lx, Lz, yf)
    assert abs(info["rel_residual_vw"] - rvw) <= 0.05 * rvw + 1e-15, (info["rel_residual_vw"], rvw)
    assert abs(info["backward_error"] - eta) <= 0.05 * eta + 1e-18, (info["backward_error"], eta)
    ref, _ = oracle.solve(f, Lx, Lz, yf)
    phi64, _ = gpu_solve(f, Lx, Lz, yf)
    print(f"mixed vs fp64 {rel(phi, phi64):.3e}, vs oracle {rel(phi, ref):.3e}, residual {r:.3e}, "
          f"history {info['residual_history']}")
    assert rel(phi, phi64) <= TOL_MIXED_VS_FP64, rel(phi, phi64)
    assert rel(phi, ref) <= TOL_MIXED_VS_FP64


@pytest.mark.parametrize("precision", MIXED_FORMS)
@pytest.mark.parametrize("nx,ny,nz", [(2304, 6, 5), (4096, 4, 3)])
def test_mixed_refinement_wide_rows(precision, nx, ny, nz):
    """Rows wider than 2048 (the residual-only pass's 4096-cell tiles).  The
    wide x spectrum leaves a larger error per unit residual (2304 x 6 x 5:
    1.6e-10 from FP64 at a 6.0e-11 residual), so the refinement runs to 1e-11
    here and the solution is held to the same 1e-10 agreement."""
    Lx = Lz = 2 * np.pi
    rtol = 1e-11
    yf = synth.tanh_faces(ny, 2.0)
    g = geometry(nx, ny, nz, Lx, Lz, yf)
    u, v, w = synth.uniform_velocity(nx, ny, nz, seed=17)
    f = divergence(u, v, w, g)
    phi, info = gpu_solve(f, Lx, Lz, yf, precision=precision, rtol=rtol, max_iters=6)
    r = residual(f, phi, Lx, Lz, yf)
    assert info["converged"] == 1, info
    assert r <= rtol, (r, info)
    assert abs(info["rel_residual"] - r) <= 0.05 * r + 1e-14
    ref, _ = oracle.solve(f, Lx, Lz, yf)
    phi64, _ = gpu_solve(f, Lx, Lz, yf)
    assert rel(phi, phi64) <= TOL_MIXED_VS_FP64, rel(phi, phi64)
    assert rel(phi, ref) <= TOL_MIXED_VS_FP64


@pytest.mark.parametrize("precision", MIXED_FORMS)
def test_mixed_tight_rtol_reaches_fp64_accuracy(precision):
    nx, ny, nz = 176, 33, 30
    Lx = Lz = 2 * np.pi
    yf = synth.tanh_faces(ny, 2.5)
    g = geometry(nx, ny, nz, Lx, Lz, yf)
    u, v, w = synth.uniform_velocity(nx, ny, nz, seed=7)
    f = divergence(u, v, w, g)
    phi, info = gpu_solve(f, Lx, Lz, yf, precision=precision, rtol=1e-14, max_iters=8)
    ref, _ = oracle.solve(f, Lx, Lz, yf)
    assert info["rel_residual"] <= 1e-13, info
    assert rel(phi, ref) <= 1e-11
    # below the FP64 floor of this grid the refinement stops there (backward
    # error <= 8 unit roundoffs) instead of running to max_iters
    assert info["converged"] in (1, 2) and info["iterations"] < 8, info
    if info["converged"] == 2:
        assert info["backward_error"] <= 8 * 2.0 ** -53


@pytest.mark.parametrize("nx,ny,nz,bc", [(64, 64, 64, ("neumann", "neumann")),
                                         (128, 48, 64, ("dirichlet", "neumann")),
                                         (512, 40, 512, ("neumann", "neumann")),
                                         (256, 24, 1024, ("neumann", "dirichlet"))])
def test_f64inv_first_correction_without_initial_iterate(nx, ny, nz, bc):
    """IBP_MIXED_F64INV on power-of-two grids solves its first correction
    from the FP32 forward transform's rounding, r0 = f - IFFT64(FFT32(f))
    (minus the exact plane means when the problem is singular), and inverts
    the sum of the two spectral solutions once.  The result matches the FP64
    solve and the oracle, one correction suffices, and the recorded initial
    residual is the FP32 transform's (~1e-7 relative)."""
    Lx, Lz = 2 * np.pi, 1.7
    yf = synth.tanh_faces(ny, 2.5)
    g = geometry(nx, ny, nz, Lx, Lz, yf, bc=bc)
    rng = np.random.default_rng(nx + 3 * ny + nz)
    f = rng.standard_normal((ny, nz, nx)) + 0.3
    phi, info = gpu_solve(f, Lx, Lz, yf, precision="mixed_f64inv", rtol=1e-10, max_iters=3, bc=bc)
    phi64, _ = gpu_solve(f, Lx, Lz, yf, bc=bc)
    ref, _ = oracle.solve(f, Lx, Lz, yf, bc=bc)
    assert info["converged"] == 1 and info["iterations"] == 1, info
    hist = info["residual_history"]
    assert len(hist) == 2 and 1e-10 < hist[0] < 1e-5 and hist[1] <= 1e-10, hist
    assert rel(phi, phi64) <= 1e-11, rel(phi, phi64)
    assert rel(phi, ref) <= 1e-11, rel(phi, ref)
    m = weighted_mean(f, g) if bc == ("neumann", "neumann") else 0.0
    r = float(np.linalg.norm(((f - m) - laplacian(phi, g)).ravel()) / np.linalg.norm((f - m).ravel()))
    assert abs(info["rel_residual"] - r) <= 0.05 * r + 1e-14, (info["rel_residual"], r)


def test_mixed_rejects_aliasing():
    nx, ny, nz = 16, 12, 8
    yf = synth.tanh_faces(ny, 2.0)
    plan = ibp.Plan(nx, ny, nz, 1.0, 1.0, yf, precision="mixed")
    x = to_dev(np.ones((ny, nz, nx)))
    with pytest.raises(ibp.IbpError) as e:
        plan.solve(x, x)
    assert e.value.status == ibp.INVALID_VALUE


def test_mixed_nonconvergence_reported():
    nx = ny = nz = 32
    yf = synth.tanh_faces(ny, 2.0)
    f = np.random.default_rng(8).standard_normal((ny, nz, nx))
    _, info = gpu_solve(f, 1.0, 1.0, yf, precision="mixed", rtol=1e-30, max_iters=1)
    assert info["converged"] == 0 and info["iterations"] == 1
    assert info["rel_residual"] > 0


# ---------------------------------------------------------------- full size
def cdft(a, ex, ez):
    """sum_{k,i} a[:, k, i] ex[i] ez[k] with real matrix-vector products only
    (no complex copy of a full field)."""
    ar = a @ ex.real
    ai = a @ ex.imag
    return (ar @ ez.real - ai @ ez.imag) + 1j * (ar @ ez.imag + ai @ ez.real)


def sampled_modes(f, phi, Lx, Lz, yf, modes):
    """For each (kx, kz): the oracle's 1-D y solve of the mode's DFT of f,
    against the same DFT of the GPU phi (O(N) per mode, so any size works).
    The error of a mode is measured against the larger of its own norm and
    the RMS norm of all modes (= ||phi||_F by Parseval), so that modes the
    input leaves empty (pure rounding) are held to the solve's absolute
    accuracy rather than to a relative one they cannot have."""
    ny, nz, nx = f.shape
    g = geometry(nx, ny, nz, Lx, Lz, yf)
    m = weighted_mean(f, g)
    from oracle.grid import lambda_x, lambda_z
    from oracle.poisson import thomas_modes, zero_mode_flux_integration
    lx, lz = lambda_x(g), lambda_z(g)
    scale = float(np.linalg.norm(phi))
    worst = 0.0
    for kx, kz in modes:
        ex = np.exp(-2j * np.pi * kx * np.arange(nx) / nx)
        ez = np.exp(-2j * np.pi * kz * np.arange(nz) / nz)
        F = cdft(f - m, ex, ez)
        P = cdft(phi, ex, ez)
        if kx == 0 and kz == 0:
            X, _ = zero_mode_flux_integration(g, F.real)
        else:
            X = thomas_modes(g.a, g.c, -np.array(lx[kx] + lz[kz]), F)
        worst = max(worst, float(np.linalg.norm(P - X) / max(np.linalg.norm(X), scale)))
    return worst


@pytest.fixture(scope="module")
def c3_case():
    nx, ny, nz = 512, 384, 512
    Lx = Lz = 2 * np.pi
    yf = synth.tanh_faces(ny, 2.0)
    g = geometry(nx, ny, nz, Lx, Lz, yf)
    u, v, w = synth.kolmogorov_velocity(nx, ny, nz, seed=3, kmax=64)
    f = divergence(u, v, w, g)
    del u, v, w
    return f, Lx, Lz, yf


# low modes, modes with content near the cut-off |k| = 64 (kz = 500 is -12),
# and modes the k^-5/3 input leaves empty, including both Nyquist lines
MODES = [(0, 0), (1, 0), (0, 1), (1, 1), (3, 7), (40, 5), (7, 500), (64, 0), (17, 250), (255, 511),
         (256, 0), (256, 256)]


def test_c3_fullsize_fp64_and_mixed(c3_case):
    """512 x 384 x 512 in the benchmark's launch configuration (its line solve
    is the 32-lane, 12-row instance): the whole FP64 field against the
    oracle's full solve, each sampled mode against the oracle's 1-D solve,
    and both mixed forms' residuals recomputed here."""
    f, Lx, Lz, yf = c3_case
    ny, nz, nx = f.shape
    ref, m = oracle.solve(f, Lx, Lz, yf)
    plan = ibp.Plan(nx, ny, nz, Lx, Lz, yf)
    fd = to_dev(f)
    phi64 = plan.solve(fd)
    info64 = plan.info()
    p64 = phi64.cpu().numpy()
    err64 = rel(p64, ref)
    print(f"c3 fp64 vs oracle {err64:.3e}")
    assert err64 <= TOL64, err64
    assert abs(info64["removed_mean"] - m) <= 1e-14 * max(1.0, abs(m))
    assert sampled_modes(f, p64, Lx, Lz, yf, MODES) <= 1e-11
    for form in MIXED_FORMS:
        plan.set_precision(form, RTOL_MIXED, 6)
        phim = plan.solve(fd)
        info = plan.info()
        pm = phim.cpu().numpy()
        r = residual(f, pm, Lx, Lz, yf)
        d = rel(pm, p64)
        print(f"c3 {form}: residual {r:.3e} (reported {info['rel_residual']:.3e}), vs fp64 {d:.3e}, "
              f"vs oracle {rel(pm, ref):.3e}, history {info['residual_history']}")
        assert info["converged"] == 1 and r <= RTOL_MIXED, (r, info)
        assert abs(info["rel_residual"] - r) <= 0.05 * r + 1e-15
        assert d <= TOL_MIXED_VS_FP64_C3, d
        assert rel(pm, ref) <= TOL_MIXED_VS_FP64_C3
        if form == "mixed_f64inv":   # FP64 inverse passes: one correction reaches 1e-10 here
            assert info["iterations"] == 1, info
