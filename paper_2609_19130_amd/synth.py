"""Seeded synthetic inputs for the Poisson solver (shared by tests and bench).

This module draws random numbers and lays out grids; it holds none of the
solver's arithmetic (no discrete operator, transform or tridiagonal step).
Every host generator uses ``numpy.random.default_rng`` (PCG64) seeded
explicitly and draws in the order documented on each function, so any caller
reproduces the same inputs.  The ``*_device`` generators (for grids too
large to draw on the host) use a seeded ``torch.Generator`` on the GPU.

The workloads mirror the paper's setting (periodic uniform x and z, a
wall-bounded stretched wall-normal direction, a right-hand side that is the
divergence of a provisional velocity field, eq. ``elliptic``); the paper
uses no public dataset for this path.
"""

import numpy as np


def tanh_faces(ny, beta):
    """ny+1 wall-normal face coordinates on [-1, 1], clustered at both walls:
    y_j = tanh(beta (2j/ny - 1)) / tanh(beta); beta -> 0 gives uniform faces."""
    s = 2.0 * np.arange(ny + 1, dtype=np.float64) / ny - 1.0
    if beta == 0:
        y = s
    else:
        y = np.tanh(beta * s) / np.tanh(beta)
    y[0], y[-1] = -1.0, 1.0
    return y


def uniform_velocity(nx, ny, nz, seed):
    """Staggered velocity with i.i.d. U[-1, 1] components.

    Draw order: u (ny, nz, nx) on x faces, then the interior wall-normal
    component v (ny-1, nz, nx) on faces 1..ny-1, then w (ny, nz, nx) on z
    faces.  The two wall rows of v are zero."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(-1.0, 1.0, size=(ny, nz, nx))
    v = np.zeros((ny + 1, nz, nx))
    v[1:ny] = rng.uniform(-1.0, 1.0, size=(ny - 1, nz, nx))
    w = rng.uniform(-1.0, 1.0, size=(ny, nz, nx))
    return u, v, w


def eigen_modes(seed, count=32, kmax=16, pmax=16):
    """Random (kx, kz, p, amplitude, phase) tuples for manufactured fields.

    (kx, kz) is uniform over integer points with kx > 0, or kx = 0 and
    kz >= 0, and kx^2 + kz^2 <= kmax^2; p is uniform in {0..pmax-1} (p >= 1
    when kx = kz = 0); amplitude ~ N(0, 1); phase ~ U[0, 2 pi).  Draw order
    per mode: point index, p, amplitude, phase.  kz may be negative."""
    pts = [(kx, kz) for kx in range(0, kmax + 1) for kz in range(-kmax, kmax + 1)
           if kx * kx + kz * kz <= kmax * kmax and (kx > 0 or kz >= 0)]
    rng = np.random.default_rng(seed)
    modes = []
    for _ in range(count):
        kx, kz = pts[int(rng.integers(len(pts)))]
        lo = 1 if (kx == 0 and kz == 0) else 0
        p = int(rng.integers(lo, pmax))
        amp = float(rng.standard_normal())
        th = float(rng.uniform(0.0, 2 * np.pi))
        modes.append((kx, kz, p, amp, th))
    return modes


def _spectral_scalar(shape, rng, kmax, workers):
    """One real field on an index grid with shell spectrum E(k) ~ k^(-5/3):
    white N(0,1) noise, real FFT, multiply by |k|^(-11/6) for 1 <= |k| <= kmax
    (integer index wavenumbers), inverse FFT, normalise to unit RMS."""
    import scipy.fft as sfft
    noise = rng.standard_normal(size=shape)
    spec = sfft.rfftn(noise, workers=workers)
    del noise
    n0, n1, n2 = shape
    k0 = np.fft.fftfreq(n0, 1.0 / n0).reshape(-1, 1, 1)
    k1 = np.fft.fftfreq(n1, 1.0 / n1).reshape(1, -1, 1)
    k2 = np.arange(n2 // 2 + 1, dtype=np.float64).reshape(1, 1, -1)
    for s0 in range(n0):             # plane by plane keeps the temporaries small
        kk = np.sqrt(k0[s0] ** 2 + k1[0] ** 2 + k2[0] ** 2)
        filt = np.where((kk >= 1.0) & (kk <= kmax), np.power(np.maximum(kk, 1.0), -11.0 / 6.0), 0.0)
        spec[s0] *= filt
    field = sfft.irfftn(spec, s=shape, workers=workers)
    del spec
    field /= np.sqrt(np.mean(field * field))
    return field


def kolmogorov_velocity(nx, ny, nz, seed, kmax=64, workers=-1):
    """Staggered velocity whose components have a k^(-5/3) spectrum up to
    kmax.  Draw order: u, then v, then w, each from the same generator.  The
    wall rows of v are set to zero (v has ny+1 rows: the ny interior/lower
    rows come from the field, the upper wall row is appended)."""
    rng = np.random.default_rng(seed)
    u = _spectral_scalar((ny, nz, nx), rng, kmax, workers)
    vf = _spectral_scalar((ny, nz, nx), rng, kmax, workers)
    v = np.empty((ny + 1, nz, nx))
    v[:ny] = vf
    del vf
    v[0] = 0.0
    v[ny] = 0.0
    w = _spectral_scalar((ny, nz, nx), rng, kmax, workers)
    return u, v, w


BATCH_DIMS = tuple(range(32, 193, 16))


def batch_grids(seed=4, count=64):
    """Uneven grids for batched solves: each of nx, ny, nz uniform in
    {32, 48, ..., 192}, beta ~ U[1.5, 3], Lx = Lz = 2 pi; grid g draws from
    ``SeedSequence(seed).spawn(count)[g]`` (order nx, ny, nz, beta) and
    carries that child's integer seed for its right-hand side."""
    children = np.random.SeedSequence(seed).spawn(count)
    out = []
    for g, ss in enumerate(children):
        rng = np.random.default_rng(ss)
        nx, ny, nz = (int(BATCH_DIMS[rng.integers(len(BATCH_DIMS))]) for _ in range(3))
        beta = float(rng.uniform(1.5, 3.0))
        out.append(dict(nx=nx, ny=ny, nz=nz, beta=beta, Lx=2 * np.pi, Lz=2 * np.pi,
                        seed=int(ss.generate_state(1)[0])))
    return out


# ---------------------------------------------------------------- device-side inputs
# Grids of ~1e9 cells are too large to draw on the host in reasonable time;
# these generators follow the same spectral recipe with torch on the GPU
# (torch.Generator on the device, seeded explicitly).  They are input
# synthesis only: the solver's own arithmetic never runs here.

def _spectral_scalar_device(shape, gen, kmax, device, chunk=64):
    import torch
    noise = torch.randn(shape, generator=gen, device=device, dtype=torch.float64)
    spec = torch.fft.rfftn(noise)
    del noise
    n0, n1, n2 = shape
    k1 = torch.fft.fftfreq(n1, 1.0 / n1, device=device, dtype=torch.float64).view(1, -1, 1)
    k2 = torch.arange(n2 // 2 + 1, device=device, dtype=torch.float64).view(1, 1, -1)
    k0all = torch.fft.fftfreq(n0, 1.0 / n0, device=device, dtype=torch.float64)
    for s0 in range(0, n0, chunk):   # chunks of planes keep the temporaries small
        k0 = k0all[s0:s0 + chunk].view(-1, 1, 1)
        kk = torch.sqrt(k0 * k0 + k1 * k1 + k2 * k2)
        filt = torch.where((kk >= 1.0) & (kk <= kmax), torch.clamp(kk, min=1.0).pow(-11.0 / 6.0),
                           torch.zeros((), device=device, dtype=torch.float64))
        spec[s0:s0 + chunk] *= filt
    field = torch.fft.irfftn(spec, s=shape)
    del spec
    field /= torch.sqrt(torch.mean(field * field))
    return field


def kolmogorov_velocity_device(nx, ny, nz, seed, kmax=64, device="cuda"):
    """kolmogorov_velocity's recipe drawn on the GPU: torch.Generator seeded
    with `seed`, draw order u, v, w; v gets ny+1 rows with zero wall rows.
    Returns contiguous float64 device tensors."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    u = _spectral_scalar_device((ny, nz, nx), gen, kmax, device)
    vf = _spectral_scalar_device((ny, nz, nx), gen, kmax, device)
    v = torch.zeros((ny + 1, nz, nx), device=device, dtype=torch.float64)
    v[1:ny] = vf[1:ny]
    del vf
    w = _spectral_scalar_device((ny, nz, nx), gen, kmax, device)
    return u, v, w


def kolmogorov_scalar_device(nx, ny, nz, seed, kmax=64, device="cuda"):
    """One scalar field [ny][nz][nx] with the same k^(-5/3) recipe, drawn on
    the GPU (torch.Generator seeded with `seed`); unit RMS, not mean-free."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    return _spectral_scalar_device((ny, nz, nx), gen, kmax, device)


def ar1_schedule(seed, steps, nx, nz, bank=4):
    """Per-step innovation draws for an AR(1) sequence of right-hand sides:
    step t uses bank member t mod `bank`, rolled by (dz, dx) planes/columns
    in z and x (uniform integers) and multiplied by a sign (+1 or -1).  Draw
    order per step: dx, dz, sign."""
    rng = np.random.default_rng(seed)
    out = []
    for t in range(steps):
        dx = int(rng.integers(nx))
        dz = int(rng.integers(nz))
        sign = 1.0 if rng.integers(2) == 0 else -1.0
        out.append((t % bank, dx, dz, sign))
    return out


def roll_into(dst, src, dz, dx):
    """dst = src rolled by dz along axis 1 (z) and dx along axis 2 (x),
    periodic, written in place with slice copies (no allocation, so it can be
    captured in a graph)."""
    nz, nx = src.shape[1], src.shape[2]
    dz %= nz
    dx %= nx
    parts_z = [(slice(dz, nz), slice(0, nz - dz)), (slice(0, dz), slice(nz - dz, nz))]
    parts_x = [(slice(dx, nx), slice(0, nx - dx)), (slice(0, dx), slice(nx - dx, nx))]
    for dzs, szs in parts_z:
        if dzs.start == dzs.stop:
            continue
        for dxs, sxs in parts_x:
            if dxs.start == dxs.stop:
                continue
            dst[:, dzs, dxs].copy_(src[:, szs, sxs])


def ar1_advance(f, g, bank, step, rho=0.95):
    """f <- rho f + sqrt(1 - rho^2) * sign * roll(bank[k]), for one entry
    (k, dx, dz, sign) of ar1_schedule; g is a scratch field of f's shape."""
    k, dx, dz, sign = step
    roll_into(g, bank[k], dz, dx)
    f.mul_(rho).add_(g, alpha=sign * float(np.sqrt(1.0 - rho * rho)))
