"""Recursive-regularised lattice Boltzmann on MI355X (gfx950).

Python side of the HIP library ``liblbrr.so`` (C ABI in include/lbrr.h):

* the C entry points under their own names (``lb_create``, ``lb_step``, ...),
  taking plain integers / pointers;
* ``Simulation``: a thin object over one handle that passes torch tensors'
  device pointers and torch's current HIP stream.  PyTorch provides device
  memory and streams only; every step of the update runs in the library's
  kernels.  There is no CPU fallback: importing this package fails if the
  library has not been built.
"""
from __future__ import annotations

import ctypes

from . import _lib
from ._lib import (LB_D2Q9, LB_D3Q19, LB_D3Q27, LB_ERR_HIP, LB_ERR_INVALID_ARG, LB_ERR_OOM, LB_ERR_STATE,
                   LB_ERR_UNSTABLE, LB_ERR_UNSUPPORTED, LB_F32, LB_F64, LB_OK, LB_STORE_FP16, LB_STORE_FP32,
                   LB_STORE_FP64, LBError)

_L = _lib.load()

# C entry points, same names as in include/lbrr.h
lb_create = _L.lb_create
lb_config = _L.lb_config
lb_set_stream = _L.lb_set_stream
lb_init_fields = _L.lb_init_fields
lb_step = _L.lb_step
lb_set_check_interval = _L.lb_set_check_interval
lb_moments = _L.lb_moments
lb_reduce = _L.lb_reduce
lb_enstrophy = _L.lb_enstrophy
lb_get_populations = _L.lb_get_populations
lb_set_populations = _L.lb_set_populations
lb_step_count = _L.lb_step_count
lb_bytes_per_update = _L.lb_bytes_per_update
lb_destroy = _L.lb_destroy
lb_last_error = _L.lb_last_error
lb_probe_copy = _L.lb_probe_copy

LATTICES = {"D2Q9": LB_D2Q9, "D3Q19": LB_D3Q19, "D3Q27": LB_D3Q27}
Q = {"D2Q9": 9, "D3Q19": 19, "D3Q27": 27}
DIM = {"D2Q9": 2, "D3Q19": 3, "D3Q27": 3}
STORAGE = {"fp64": LB_STORE_FP64, "fp32": LB_STORE_FP32, "fp16": LB_STORE_FP16}

check = _lib.check


def _torch():
    import torch

    return torch


class Simulation:
    """One periodic lattice advanced by the library.

    lattice: "D2Q9" | "D3Q19" | "D3Q27"; shape (nz, ny, nx) with nz = 1 in 2D;
    tau: shifted relaxation time (nu = (tau - 1/2)/3); order: Hermite truncation;
    storage: "fp64" | "fp32" | "fp16" (deviations f - w rho0).
    """

    def __init__(self, lattice, shape, tau, order, storage="fp32", rho0=1.0, stream=None):
        torch = _torch()
        self.lattice = lattice
        self.nz, self.ny, self.nx = shape
        self.shape = tuple(shape)
        self.q = Q[lattice]
        self.d = DIM[lattice]
        self.tau = tau
        self.order = order
        self.storage = storage
        self.handle = lb_create(LATTICES[lattice], self.nx, self.ny, self.nz, float(tau), int(order))
        if not self.handle:
            raise LBError(LB_ERR_INVALID_ARG, _lib.last_error())
        check(lb_config(self.handle, STORAGE[storage], float(rho0)))
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        check(lb_set_stream(self.handle, ctypes.c_void_p(self.stream.cuda_stream)))

    # -- helpers ---------------------------------------------------------
    def _dev(self, t, dtype):
        torch = _torch()
        t = torch.as_tensor(t)
        if t.dtype not in (torch.float64, torch.float32):
            t = t.to(torch.float64)
        return t.to(device="cuda", dtype=dtype).contiguous()

    @property
    def storage_dtype(self):
        torch = _torch()
        return {"fp64": torch.float64, "fp32": torch.float32, "fp16": torch.float16}[self.storage]

    # -- API -------------------------------------------------------------
    def init_fields(self, rho, u, pi1=None, dtype=None):
        """rho (nz,ny,nx), u (d,nz,ny,nx), pi1 packed (d(d+1)/2,nz,ny,nx) or None."""
        torch = _torch()
        dtype = dtype or torch.float64
        r = self._dev(rho, dtype).reshape(self.shape)
        v = self._dev(u, dtype).reshape((self.d,) + self.shape)
        p = None if pi1 is None else self._dev(pi1, dtype).reshape((self.d * (self.d + 1) // 2,) + self.shape)
        code = LB_F64 if dtype == torch.float64 else LB_F32
        check(lb_init_fields(self.handle, r.data_ptr(), v.data_ptr(), 0 if p is None else p.data_ptr(), code, 1))
        self._keep = (r, v, p)  # alive until the stream has consumed them
        return self

    def step(self, n=1):
        check(lb_step(self.handle, int(n)))
        return self

    def set_check_interval(self, k):
        check(lb_set_check_interval(self.handle, int(k)))

    def moments(self, dtype=None, pi1=False):
        torch = _torch()
        dtype = dtype or torch.float64
        rho = torch.empty(self.shape, device="cuda", dtype=dtype)
        u = torch.empty((self.d,) + self.shape, device="cuda", dtype=dtype)
        p = torch.empty((self.d * (self.d + 1) // 2,) + self.shape, device="cuda", dtype=dtype) if pi1 else None
        code = LB_F64 if dtype == torch.float64 else LB_F32
        check(lb_moments(self.handle, rho.data_ptr(), u.data_ptr(), 0 if p is None else p.data_ptr(), code, 1))
        return (rho, u, p) if pi1 else (rho, u)

    def reduce(self):
        out = (ctypes.c_double * 5)()
        check(lb_reduce(self.handle, out))
        return tuple(out)

    def enstrophy(self):
        out = ctypes.c_double()
        check(lb_enstrophy(self.handle, ctypes.byref(out)))
        return out.value

    def get_populations(self):
        torch = _torch()
        t = torch.empty((self.q,) + self.shape, device="cuda", dtype=self.storage_dtype)
        check(lb_get_populations(self.handle, t.data_ptr(), 1))
        return t

    def set_populations(self, t):
        torch = _torch()
        t = torch.as_tensor(t).to(device="cuda", dtype=self.storage_dtype).contiguous()
        assert tuple(t.shape) == (self.q,) + self.shape
        check(lb_set_populations(self.handle, t.data_ptr(), 1))
        self._keep = (t,)

    @property
    def steps(self):
        return lb_step_count(self.handle)

    @property
    def bytes_per_update(self):
        return lb_bytes_per_update(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            lb_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
