"""Shared helpers of the GPU tests: device transfer and comparisons."""

import numpy as np
import torch

from paper_2609_19130_amd import ibpoisson as ibp


def require_gpu():
    assert torch.cuda.is_available(), "GPU test run without a visible GPU"
    ibp.lib()   # raises if the HIP library is missing


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def gpu_solve(f, Lx, Lz, yf, precision="fp64", rtol=1e-10, max_iters=4, plan=None, bc=("neumann", "neumann")):
    ny, nz, nx = f.shape
    own = plan is None
    if own:
        plan = ibp.Plan(nx, ny, nz, Lx, Lz, yf, precision=precision, rtol=rtol, max_iters=max_iters, bc=bc)
    fd = to_dev(f)
    phi = plan.solve(fd)
    info = plan.info()
    out = phi.cpu().numpy()
    if own:
        plan.close()
    return out, info


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))
