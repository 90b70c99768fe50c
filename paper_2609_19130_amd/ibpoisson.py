"""ctypes binding of libibpoisson (argument marshalling only).

Every step of the solve runs in the HIP kernels of ``libibpoisson.so``; this
module checks tensor shapes, dtypes and devices, passes raw device pointers
and the current HIP stream, and maps status codes to exceptions.  PyTorch
provides device memory and streams.  If the shared library is missing the
first call raises: there is no fallback implementation.
"""

import ctypes
import os

FP64, MIXED, MIXED_F64SWEEP, MIXED_F64INV = 0, 1, 2, 3
PRECISIONS = {"fp64": FP64, "mixed": MIXED, "mixed_f64sweep": MIXED_F64SWEEP, "mixed_f64inv": MIXED_F64INV}
LOCATIONS = {"cells": 0, "yfaces": 1}   # ibp_location_t

SUCCESS, INVALID_VALUE, UNSUPPORTED_SIZE, OUT_OF_MEMORY, HIP_ERROR, INTERNAL = range(6)

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libibpoisson.so")

_lib = None


class IbpError(RuntimeError):
    def __init__(self, status, what):
        self.status = status
        super().__init__(f"{what}: {status_string(status)} ({status})")


HISTORY_MAX = 16


class Info(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("converged", ctypes.c_int),
                ("nonfinite_input", ctypes.c_int), ("reserved", ctypes.c_int),
                ("rel_residual", ctypes.c_double), ("removed_mean", ctypes.c_double),
                ("rhs_norm", ctypes.c_double), ("residual_norm", ctypes.c_double),
                ("rel_residual_vw", ctypes.c_double), ("backward_error", ctypes.c_double),
                ("history_len", ctypes.c_int), ("reserved2", ctypes.c_int),
                ("residual_history", ctypes.c_double * HISTORY_MAX)]

    def as_dict(self):
        d = {name: getattr(self, name) for name, _ in self._fields_
             if name not in ("reserved", "reserved2", "residual_history", "history_len")}
        d["residual_history"] = [float(self.residual_history[k]) for k in range(self.history_len)]
        return d


class PassStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int), ("reserved", ctypes.c_int),
                ("total_ms", ctypes.c_double), ("bytes_per_launch", ctypes.c_double)]


class Tune(ctypes.Structure):
    _fields_ = [("xdiv", ctypes.c_int), ("zdiv", ctypes.c_int), ("ycols", ctypes.c_int), ("tried", ctypes.c_int),
                ("ms", ctypes.c_double), ("ms_before", ctypes.c_double), ("persistent", ctypes.c_int),
                ("lag", ctypes.c_int), ("chunk", ctypes.c_int), ("xsmall", ctypes.c_int), ("zsmall", ctypes.c_int),
                ("reserved", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


def lib():
    """Load libibpoisson.so (once) and declare its signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2609_19130_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, ci, cd, cs = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    sig = {
        "ibp_check_dims": (ci, [ci, ci, ci]),
        "ibp_plan_create": (ci, [ctypes.POINTER(vp), ci, ci, ci, cd, cd, ctypes.POINTER(cd)]),
        "ibp_plan_destroy": (ci, [vp]),
        "ibp_plan_set_precision": (ci, [vp, ci, cd, ci]),
        "ibp_plan_set_bc": (ci, [vp, ci, ci]),
        "ibp_plan_workspace_size": (ci, [vp, ctypes.POINTER(cs)]),
        "ibp_plan_set_workspace": (ci, [vp, vp, cs]),
        "ibp_solve": (ci, [vp, vp, vp, vp]),
        "ibp_solve_scratch": (ci, [vp, vp, vp, vp]),
        "ibp_solve_batched": (ci, [ctypes.POINTER(vp), ci, ctypes.POINTER(vp), ctypes.POINTER(vp), vp]),
        "ibp_get_info": (ci, [vp, ctypes.POINTER(Info)]),
        "ibp_divergence": (ci, [vp, vp, vp, vp, vp, vp]),
        "ibp_solve_divergence": (ci, [vp, vp, vp, vp, vp, cd, vp, vp, vp]),
        "ibp_project": (ci, [vp, vp, cd, cd, vp, vp, vp, vp, vp]),
        "ibp_helmholtz_set": (ci, [vp, cd]),
        "ibp_helmholtz": (ci, [vp, vp, ci, vp]),
        "ibp_plan_set_profiling": (ci, [vp, ci]),
        "ibp_plan_get_profile": (ci, [vp, ci, ctypes.POINTER(ci), ctypes.POINTER(PassStat)]),
        "ibp_batch_create": (ci, [ctypes.POINTER(vp), ci, ctypes.POINTER(vp)]),
        "ibp_batch_solve": (ci, [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), vp]),
        "ibp_batch_set_ycols": (ci, [vp, ci]),
        "ibp_batch_set_persistent": (ci, [vp, ci]),
        "ibp_batch_destroy": (ci, [vp]),
        "ibp_plan_autotune": (ci, [vp, vp, vp, vp, ctypes.POINTER(Tune)]),
        "ibp_batch_autotune": (ci, [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), vp, ctypes.POINTER(Tune)]),
        "ibp_status_string": (ctypes.c_char_p, [ci]),
        "ibp_version": (ci, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def status_string(status):
    return lib().ibp_status_string(int(status)).decode()


def check_dims(nx, ny, nz):
    """Host-only size check; returns a status code."""
    return lib().ibp_check_dims(int(nx), int(ny), int(nz))


def _check(status, what):
    if status != SUCCESS:
        raise IbpError(status, what)


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _field(t, shape, name):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda" or t.dtype != torch.float64 or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float64 CUDA tensor")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return ctypes.c_void_p(t.data_ptr())


class Plan:
    """One grid: nx, ny, nz pressure cells, periodic lengths Lx, Lz and the
    ny+1 wall-normal face coordinates ``y_nodes`` (host array)."""

    def __init__(self, nx, ny, nz, Lx, Lz, y_nodes, precision="fp64", rtol=1e-10, max_iters=4,
                 bc=("neumann", "neumann")):
        L = lib()
        y = [float(v) for v in y_nodes]
        if len(y) != ny + 1:
            raise ValueError(f"y_nodes must have ny+1 = {ny + 1} entries")
        arr = (ctypes.c_double * len(y))(*y)
        h = ctypes.c_void_p()
        _check(L.ibp_plan_create(ctypes.byref(h), int(nx), int(ny), int(nz), float(Lx), float(Lz), arr),
               "ibp_plan_create")
        self._h = h
        self.shape = (int(ny), int(nz), int(nx))
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.bc = ("neumann", "neumann")
        if tuple(bc) != self.bc:
            self.set_bc(*bc)
        self.set_precision(precision, rtol, max_iters)

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("plan destroyed")
        return self._h

    def set_bc(self, lower="neumann", upper="neumann"):
        """Wall conditions of the pressure correction ("neumann" or "dirichlet")."""
        code = {"neumann": 0, "dirichlet": 1}
        _check(lib().ibp_plan_set_bc(self.handle, code[lower], code[upper]), "ibp_plan_set_bc")
        self.bc = (lower, upper)

    def set_precision(self, precision, rtol=1e-10, max_iters=4):
        code = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        _check(lib().ibp_plan_set_precision(self.handle, code, float(rtol), int(max_iters)),
               "ibp_plan_set_precision")
        self.precision = code

    def workspace_size(self):
        n = ctypes.c_size_t()
        _check(lib().ibp_plan_workspace_size(self.handle, ctypes.byref(n)), "ibp_plan_workspace_size")
        return n.value

    def set_workspace(self, tensor):
        """Use a caller-owned device buffer (e.g. a torch uint8 tensor) as workspace;
        the tensor must stay alive while the plan uses it.  None re-allocates."""
        if tensor is None:
            _check(lib().ibp_plan_set_workspace(self.handle, None, 0), "ibp_plan_set_workspace")
            self._ws = None
            return
        nbytes = tensor.numel() * tensor.element_size()
        _check(lib().ibp_plan_set_workspace(self.handle, ctypes.c_void_p(tensor.data_ptr()), nbytes),
               "ibp_plan_set_workspace")
        self._ws = tensor

    def solve(self, rhs, phi=None, stream=None):
        """Enqueue a solve; returns phi (allocated if not given)."""
        import torch
        r = _field(rhs, self.shape, "rhs")
        if phi is None:
            phi = torch.empty(self.shape, dtype=torch.float64, device=rhs.device)
        p = _field(phi, self.shape, "phi")
        _check(lib().ibp_solve(self.handle, r, p, _stream_ptr(stream)), "ibp_solve")
        return phi

    def solve_scratch(self, rhs, phi, stream=None):
        """Enqueue a solve whose workspace is the library's static per-GPU
        array (ibp_solve_scratch; allocates nothing, phi must be given)."""
        r = _field(rhs, self.shape, "rhs")
        p = _field(phi, self.shape, "phi")
        _check(lib().ibp_solve_scratch(self.handle, r, p, _stream_ptr(stream)), "ibp_solve_scratch")
        return phi

    def autotune(self, rhs, phi=None, stream=None):
        """Time the plan's work splits on this input and keep the fastest
        (synchronises; phi receives the solution).  Returns the choice."""
        import torch
        r = _field(rhs, self.shape, "rhs")
        if phi is None:
            phi = torch.empty(self.shape, dtype=torch.float64, device=rhs.device)
        t = Tune()
        _check(lib().ibp_plan_autotune(self.handle, r, _field(phi, self.shape, "phi"), _stream_ptr(stream),
                                       ctypes.byref(t)), "ibp_plan_autotune")
        return t.as_dict()

    def info(self):
        inf = Info()
        _check(lib().ibp_get_info(self.handle, ctypes.byref(inf)), "ibp_get_info")
        return inf.as_dict()

    def set_profiling(self, enable=True):
        _check(lib().ibp_plan_set_profiling(self.handle, 1 if enable else 0), "ibp_plan_set_profiling")

    def profile(self):
        """Per-pass launch counts, summed event times and algorithmic bytes
        since profiling was enabled or last queried (synchronises)."""
        arr = (PassStat * 32)()
        n = ctypes.c_int()
        _check(lib().ibp_plan_get_profile(self.handle, 32, ctypes.byref(n), arr), "ibp_plan_get_profile")
        return {arr[i].name.decode(): dict(launches=arr[i].launches, total_ms=arr[i].total_ms,
                                           bytes_per_launch=arr[i].bytes_per_launch) for i in range(n.value)}

    def divergence(self, u, v, w, f=None, stream=None):
        import torch
        ny, nz, nx = self.shape
        pu = _field(u, self.shape, "u")
        pv = _field(v, (ny + 1, nz, nx), "v")
        pw = _field(w, self.shape, "w")
        if f is None:
            f = torch.empty(self.shape, dtype=torch.float64, device=u.device)
        pf = _field(f, self.shape, "f")
        _check(lib().ibp_divergence(self.handle, pu, pv, pw, pf, _stream_ptr(stream)), "ibp_divergence")
        return f

    def solve_divergence(self, u, v, w, alpha_dt, q=None, rhs_out=None, phi=None, stream=None):
        """Solve lap(phi) = (div u* - q) / alpha_dt (ibp_solve_divergence)."""
        import torch
        ny, nz, nx = self.shape
        pu = _field(u, self.shape, "u")
        pv = _field(v, (ny + 1, nz, nx), "v")
        pw = _field(w, self.shape, "w")
        pq = _field(q, self.shape, "q") if q is not None else None
        pr = _field(rhs_out, self.shape, "rhs_out") if rhs_out is not None else None
        if phi is None:
            phi = torch.empty(self.shape, dtype=torch.float64, device=u.device)
        _check(lib().ibp_solve_divergence(self.handle, pu, pv, pw, pq, float(alpha_dt), pr,
                                          _field(phi, self.shape, "phi"), _stream_ptr(stream)),
               "ibp_solve_divergence")
        return phi

    def project(self, phi, alpha_dt, u, v, w, p=None, visc=0.0, stream=None):
        """u -= alpha_dt G phi and p += phi - visc L_h phi, in place (ibp_project)."""
        ny, nz, nx = self.shape
        _check(lib().ibp_project(self.handle, _field(phi, self.shape, "phi"), float(alpha_dt), float(visc),
                                 _field(u, self.shape, "u"), _field(v, (ny + 1, nz, nx), "v"),
                                 _field(w, self.shape, "w"),
                                 _field(p, self.shape, "p") if p is not None else None, _stream_ptr(stream)),
               "ibp_project")

    def helmholtz_set(self, beta):
        """Factor the three directions' line operators for beta (ibp_helmholtz_set)."""
        _check(lib().ibp_helmholtz_set(self.handle, float(beta)), "ibp_helmholtz_set")

    def helmholtz(self, field, where="cells", stream=None):
        """In place: field <- (1 - beta L_y)^-1 (1 - beta L_z)^-1 (1 - beta L_x)^-1 field
        (ibp_helmholtz); where = "cells" ([ny][nz][nx]) or "yfaces" ([ny+1][nz][nx])."""
        ny, nz, nx = self.shape
        if where not in LOCATIONS:
            raise ValueError("where must be 'cells' or 'yfaces'")
        shape = self.shape if where == "cells" else (ny + 1, nz, nx)
        _check(lib().ibp_helmholtz(self.handle, _field(field, shape, "field"), LOCATIONS[where],
                                   _stream_ptr(stream)), "ibp_helmholtz")
        return field

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().ibp_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_batched(plans, rhs, phi, stream=None):
    """Enqueue len(plans) independent solves in one call."""
    n = len(plans)
    if len(rhs) != n or len(phi) != n:
        raise ValueError("plans, rhs and phi must have the same length")
    H = (ctypes.c_void_p * n)(*[p.handle for p in plans])
    R = (ctypes.c_void_p * n)(*[_field(r, p.shape, "rhs").value for r, p in zip(rhs, plans)])
    P = (ctypes.c_void_p * n)(*[_field(q, p.shape, "phi").value for q, p in zip(phi, plans)])
    _check(lib().ibp_solve_batched(H, n, R, P, _stream_ptr(stream)), "ibp_solve_batched")
    return phi


BATCH_MAX = 64


class Batch:
    """Grids solved together, one launch per solve stage (ibp_batch_*).  The
    plans must outlive the batch."""

    def __init__(self, plans):
        self.plans = list(plans)
        n = len(self.plans)
        H = (ctypes.c_void_p * n)(*[p.handle for p in self.plans])
        h = ctypes.c_void_p()
        _check(lib().ibp_batch_create(H, n, ctypes.byref(h)), "ibp_batch_create")
        self._h = h

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("batch is closed")
        return self._h

    def set_ycols(self, cols):
        _check(lib().ibp_batch_set_ycols(self.handle, int(cols)), "ibp_batch_set_ycols")

    def set_persistent(self, enable=True):
        """One persistent launch for the whole batched solve (True) or one
        launch per stage (False); ibp_batch_set_persistent."""
        _check(lib().ibp_batch_set_persistent(self.handle, 1 if enable else 0), "ibp_batch_set_persistent")

    def _ptrs(self, rhs, phi):
        n = len(self.plans)
        if len(rhs) != n or len(phi) != n:
            raise ValueError("one right-hand side and one solution per plan")
        R = (ctypes.c_void_p * n)(*[_field(r, p.shape, "rhs").value for r, p in zip(rhs, self.plans)])
        P = (ctypes.c_void_p * n)(*[_field(q, p.shape, "phi").value for q, p in zip(phi, self.plans)])
        return R, P

    def autotune(self, rhs, phi=None, stream=None):
        """Time the batch's work splits on these inputs and keep the fastest
        (synchronises; phi receives the solutions).  Returns the choice."""
        import torch
        if phi is None:
            phi = [torch.empty(p.shape, dtype=torch.float64, device=r.device) for p, r in zip(self.plans, rhs)]
        R, P = self._ptrs(rhs, phi)
        t = Tune()
        _check(lib().ibp_batch_autotune(self.handle, R, P, _stream_ptr(stream), ctypes.byref(t)),
               "ibp_batch_autotune")
        return t.as_dict()

    def solve(self, rhs, phi=None, stream=None):
        import torch
        n = len(self.plans)
        if len(rhs) != n:
            raise ValueError("one right-hand side per plan")
        if phi is None:
            phi = [torch.empty(p.shape, dtype=torch.float64, device=r.device) for p, r in zip(self.plans, rhs)]
        R, P = self._ptrs(rhs, phi)
        _check(lib().ibp_batch_solve(self.handle, R, P, _stream_ptr(stream)), "ibp_batch_solve")
        return phi

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().ibp_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
