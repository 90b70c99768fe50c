"""The allocation-free solve (ibp_solve_scratch): its workspace is the
library's static per-GPU array.  Called through the C ABI (ctypes), it must
give ibp_solve's results bitwise, on consecutive calls whose second input is
smaller than the first (the array keeps the previous call's contents), in
the FP64 and mixed forms, and refuse grids whose workspace exceeds it."""

import ctypes

import numpy as np
import pytest
import torch

from paper_2609_19130_amd import ibpoisson as ibp
from paper_2609_19130_amd import synth

from gpu_helpers import require_gpu, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def _scratch_solve(plan, rhs, phi):
    st = ibp.lib().ibp_solve_scratch(plan.handle, ctypes.c_void_p(rhs.data_ptr()), ctypes.c_void_p(phi.data_ptr()),
                                     ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_scratch_solve_matches_plan_workspace(precision):
    shapes = [(96, 70, 48, 2.5), (32, 24, 16, 2.0)]   # the second call's grid is smaller
    for call, (nx, ny, nz, beta) in enumerate(shapes):
        yf = synth.tanh_faces(ny, beta)
        f = np.random.default_rng(100 + call).standard_normal((ny, nz, nx)) + 0.1
        plan = ibp.Plan(nx, ny, nz, 2 * np.pi, 1.3, yf, precision=precision, max_iters=6)
        fd = to_dev(f)
        ref = plan.solve(fd).clone()
        ref_info = plan.info()
        out = torch.full_like(fd, float("nan"))
        assert _scratch_solve(plan, fd, out) == ibp.SUCCESS
        info = plan.info()
        torch.cuda.synchronize()
        assert torch.equal(out, ref), (precision, call)
        assert info["converged"] == ref_info["converged"] and info["iterations"] == ref_info["iterations"]
        assert info["removed_mean"] == ref_info["removed_mean"]
        if precision == "mixed":
            assert info["rel_residual"] == ref_info["rel_residual"]
        # the plan's own workspace still gives the same bits afterwards
        again = plan.solve(fd)
        torch.cuda.synchronize()
        assert torch.equal(again, ref)
        plan.close()


def test_scratch_solve_refuses_large_grids():
    nx = ny = nz = 256
    yf = synth.tanh_faces(ny, 2.0)
    plan = ibp.Plan(nx, ny, nz, 1.0, 1.0, yf)
    assert plan.workspace_size() > 32 << 20
    x = torch.zeros((ny, nz, nx), dtype=torch.float64, device="cuda")
    assert _scratch_solve(plan, x, x) == ibp.UNSUPPORTED_SIZE
    plan.close()
