"""Graph capture of solves (hipGraph through torch.cuda.graph) and the
one-GPU paper-scale sequence: 1024 x 768 x 1024, beta = 3, right-hand sides
an AR(1) blend of divergences of k^-5/3 velocity fields.  GPU only."""

import numpy as np
import pytest
import torch

import oracle
from oracle.grid import geometry
from oracle.operators import weighted_mean
from paper_2609_19130_amd import ibpoisson as ibp
from paper_2609_19130_amd import synth

from gpu_helpers import rel, require_gpu, to_dev
from test_gpu_parity import cdft, sampled_modes

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


@pytest.mark.parametrize("precision", ["fp64", "mixed", "mixed_f64inv"])
@pytest.mark.parametrize("nx,ny,nz", [(64, 33, 64), (48, 20, 40)])
def test_graph_replay_matches_eager(precision, nx, ny, nz):
    """A captured solve replayed on new inputs (written into the captured rhs
    between replays, with eager solves in between) gives bitwise the eager
    result on every replay, not only the first."""
    Lx, Lz = 2 * np.pi, 1.5
    yf = synth.tanh_faces(ny, 2.5)
    rng = np.random.default_rng(nx + ny + nz)
    inputs = [to_dev(rng.standard_normal((ny, nz, nx))) for _ in range(4)]
    cap = ibp.Plan(nx, ny, nz, Lx, Lz, yf, precision=precision, max_iters=4)
    ref = ibp.Plan(nx, ny, nz, Lx, Lz, yf, precision=precision, max_iters=4)
    f = inputs[0].clone()
    phi = torch.empty_like(f)
    cap.solve(f, phi)                   # eager warm-up on the capturing plan
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        cap.solve(f, phi)
    for k in range(1, 4):
        f.copy_(inputs[k])
        expect = ref.solve(inputs[k])
        other = cap.solve(inputs[(k + 1) % 4])   # eager work on the same plan between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(phi, expect), f"replay {k}"
        del other
    if precision != "fp64":
        assert cap.info()["converged"] == 1


C5 = dict(nx=1024, ny=768, nz=1024, beta=3.0, seed=5, bank=4, steps=100)


@pytest.fixture(scope="module")
def c5_bank():
    nx, ny, nz = C5["nx"], C5["ny"], C5["nz"]
    yf = synth.tanh_faces(ny, C5["beta"])
    plan = ibp.Plan(nx, ny, nz, 2 * np.pi, 2 * np.pi, yf)
    bank = []
    for b in range(C5["bank"]):
        u, v, w = synth.kolmogorov_velocity_device(nx, ny, nz, seed=1000 * C5["seed"] + b)
        bank.append(plan.divergence(u, v, w))
        del u, v, w
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    plan.close()
    return yf, bank


def test_c5_graph_sequence(c5_bank):
    """The benchmark's sequence of 100 AR(1) steps captured as one graph
    (advance the rhs, solve), FP64 and mixed: graph replay is bitwise the
    eager sequence; the final mixed solution is within 1e-10 of the FP64 one;
    the final FP64 solution matches the oracle's 1-D solves on sampled
    modes."""
    yf, bank = c5_bank
    nx, ny, nz = C5["nx"], C5["ny"], C5["nz"]
    Lx = Lz = 2 * np.pi
    sched = synth.ar1_schedule(C5["seed"], C5["steps"], nx, nz, C5["bank"])
    f0 = bank[0] * sched[0][3]
    f = torch.empty_like(f0)
    gbuf = torch.empty_like(f0)
    finals = {}
    for precision in ("fp64", "mixed"):
        plan = ibp.Plan(nx, ny, nz, Lx, Lz, yf, precision=precision, max_iters=6)
        phi = torch.empty_like(f0)
        # eager sequence
        f.copy_(f0)
        for t in range(C5["steps"]):
            plan.solve(f, phi)
            if t + 1 < C5["steps"]:
                synth.ar1_advance(f, gbuf, bank, sched[t + 1])
        torch.cuda.synchronize()
        eager = phi.clone()
        f_last = f.clone() if precision == "fp64" else None
        # captured sequence, replayed twice
        f.copy_(f0)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for t in range(C5["steps"]):
                plan.solve(f, phi)
                if t + 1 < C5["steps"]:
                    synth.ar1_advance(f, gbuf, bank, sched[t + 1])
        for rep in range(2):
            f.copy_(f0)
            phi.zero_()
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(phi, eager), (precision, rep)
        info = plan.info()
        finals[precision] = (eager, info)
        if precision == "fp64":
            fh = f_last.cpu().numpy()
        del g
        plan.close()
    p64, _ = finals["fp64"]
    pm, info = finals["mixed"]
    assert info["converged"] == 1 and info["rel_residual"] <= 1e-10, info
    d = float(torch.linalg.vector_norm(pm - p64) / torch.linalg.vector_norm(p64))
    assert d <= 1e-10, d
    modes = [(0, 0), (1, 0), (0, 1), (5, 1000), (64, 3), (300, 200)]
    assert sampled_modes(fh, p64.cpu().numpy(), Lx, Lz, yf, modes) <= 1e-11


def residual_torch(f, phi, Lx, Lz, yf):
    """||f - m - L_h phi|| / ||f - m|| on the GPU with plain torch float64
    array operations (the oracle's stencil: periodic second differences in x
    and z, the difference of the two face fluxes in y, no wall flux), for
    grids too large for a CPU pass within a test's time."""
    ny = phi.shape[0]
    yf = np.asarray(yf, dtype=np.float64)
    dyf = np.diff(yf)
    yc = 0.5 * (yf[1:] + yf[:-1])
    a = np.zeros(ny)
    c = np.zeros(ny)
    a[1:] = 1.0 / (dyf[1:] * (yc[1:] - yc[:-1]))
    c[:-1] = 1.0 / (dyf[:-1] * (yc[1:] - yc[:-1]))
    dx, dz = Lx / phi.shape[2], Lz / phi.shape[1]
    w = torch.from_numpy(dyf).to(phi.device).view(-1, 1, 1)
    m = float((f * w).sum() / (w.sum() * phi.shape[1] * phi.shape[2]))
    num = 0.0
    den = 0.0
    for j in range(ny):   # plane by plane keeps the temporaries small
        p = phi[j]
        lap = (torch.roll(p, -1, 1) - 2 * p + torch.roll(p, 1, 1)) / (dx * dx)
        lap += (torch.roll(p, -1, 0) - 2 * p + torch.roll(p, 1, 0)) / (dz * dz)
        if j > 0:
            lap += a[j] * (phi[j - 1] - p)
        if j < ny - 1:
            lap += c[j] * (phi[j + 1] - p)
        r = (f[j] - m) - lap
        num += float((r * r).sum())
        den += float(((f[j] - m) ** 2).sum())
    return (num / den) ** 0.5


def test_c5_scalar_field_innovations():
    """The paper-scale share with the innovations read literally: an AR(1)
    blend (rho 0.95) of four scalar k^-5/3 fields (rolled, sign-flipped),
    not of divergences.  On this input (beta = 3, ny = 768) the FP64 direct
    solve's own relative residual is ~1e-8: a 1e-10 residual target is below
    the FP64 floor.  Accepted when the mixed form stops at that floor
    (converged = 1 or 2, backward error <= 8 unit roundoffs), its residual is
    at most max(1e-10, 2 x the FP64 solve's residual), and its solution is
    within 1e-10 of the FP64 one; the FP64 solution also matches the
    oracle's 1-D solves on sampled modes."""
    nx, ny, nz, beta, seed = C5["nx"], C5["ny"], C5["nz"], C5["beta"], C5["seed"]
    Lx = Lz = 2 * np.pi
    yf = synth.tanh_faces(ny, beta)
    bank = [synth.kolmogorov_scalar_device(nx, ny, nz, seed=7000 + b) for b in range(C5["bank"])]
    steps = 4
    sched = synth.ar1_schedule(seed + 1, steps, nx, nz, C5["bank"])
    f = bank[0] * sched[0][3]
    gbuf = torch.empty_like(f)
    for t in range(1, steps):
        synth.ar1_advance(f, gbuf, bank, sched[t])
    del bank, gbuf
    torch.cuda.empty_cache()
    plan = ibp.Plan(nx, ny, nz, Lx, Lz, yf)
    phi64 = plan.solve(f)
    plan.set_precision("mixed", 1e-10, 8)
    phim = plan.solve(f)
    info = plan.info()
    torch.cuda.synchronize()
    d = float(torch.linalg.vector_norm(phim - phi64) / torch.linalg.vector_norm(phi64))
    r64 = residual_torch(f, phi64, Lx, Lz, yf)
    rm = residual_torch(f, phim, Lx, Lz, yf)
    print(f"c5 scalar: fp64 residual {r64:.3e}, mixed residual {rm:.3e} (reported {info['rel_residual']:.3e}), "
          f"mixed vs fp64 {d:.3e}, info {info}")
    assert info["converged"] in (1, 2), info
    assert info["backward_error"] <= 8 * 2.0 ** -53 or info["rel_residual"] <= 1e-10, info
    assert abs(info["rel_residual"] - rm) <= 0.05 * rm, (rm, info)
    assert rm <= max(1e-10, 2 * r64), (rm, r64)
    assert d <= 1e-10, d
    fh = f.cpu().numpy()
    modes = [(0, 0), (1, 0), (0, 1), (3, 2), (64, 3), (300, 200)]
    assert sampled_modes(fh, phi64.cpu().numpy(), Lx, Lz, yf, modes) <= 1e-11
    plan.close()
