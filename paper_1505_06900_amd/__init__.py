"""Recursive-regularised lattice Boltzmann on MI355X (gfx950).

Python side of the HIP library ``liblbrr.so`` (C ABI in include/lbrr.h):

* the C entry points under their own names (``lb_create``, ``lb_step``, ...),
  taking plain integers / pointers;
* ``Simulation``: a thin object over one handle that passes torch tensors'
  device pointers and torch's current HIP stream.  PyTorch provides device
  memory and streams only; every step of the update runs in the library's
  kernels.  There is no CPU fallback: the first use of any entry point
  raises if the library has not been built.
"""
from __future__ import annotations

import ctypes

from . import _lib
from ._lib import (LB_D2Q9, LB_D3Q19, LB_D3Q27, LB_ERR_HIP, LB_ERR_INVALID_ARG, LB_ERR_OOM, LB_ERR_STATE,
                   LB_ERR_UNSTABLE, LB_ERR_UNSUPPORTED, LB_F32, LB_F64, LB_OK, LB_STORE_FP16, LB_STORE_FP32,
                   LB_STORE_FP64, LB_STORE_MOM_FP32, LB_STORE_MOM_FP64, LBError)


def __getattr__(name):
    """C entry points under their own names (``lb_create``, ...), loaded on first use.

    The library is loaded lazily so that ``paper_1505_06900_amd.build`` can run
    (and rebuild it) without loading a stale or missing ``liblbrr.so``."""
    if name in _lib.SIGNATURES:
        return getattr(_lib.load(), name)
    if name in ("LB_MLP_NPARAM", "LB_MLP_NNORM", "LB_MLP_NIN"):
        return getattr(_lib, name)
    raise AttributeError(name)


def load():
    """Load liblbrr.so now (raises if it is missing or lacks a declared symbol)."""
    return _lib.load()


LATTICES = {"D2Q9": LB_D2Q9, "D3Q19": LB_D3Q19, "D3Q27": LB_D3Q27}
Q = {"D2Q9": 9, "D3Q19": 19, "D3Q27": 27}
DIM = {"D2Q9": 2, "D3Q19": 3, "D3Q27": 3}
STORAGE = {"fp64": LB_STORE_FP64, "fp32": LB_STORE_FP32, "fp16": LB_STORE_FP16,
           "mom_fp64": LB_STORE_MOM_FP64, "mom_fp32": LB_STORE_MOM_FP32}

check = _lib.check


def _torch():
    import torch

    return torch


class Simulation:
    """One periodic lattice advanced by the library.

    lattice: "D2Q9" | "D3Q19" | "D3Q27"; shape (nz, ny, nx) with nz = 1 in 2D;
    tau: shifted relaxation time (nu = (tau - 1/2)/3); order: Hermite truncation;
    storage: "fp64" | "fp32" | "fp16" (populations as deviations f - w rho0), or
             "mom_fp64" | "mom_fp32" (per-node moments rho - rho0, rho u, a1^(2)).
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
        self.handle = _lib.load().lb_create(LATTICES[lattice], self.nx, self.ny, self.nz, float(tau), int(order))
        if not self.handle:
            raise LBError(LB_ERR_INVALID_ARG, _lib.last_error())
        check(_lib.load().lb_config(self.handle, STORAGE[storage], float(rho0)))
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        check(_lib.load().lb_set_stream(self.handle, ctypes.c_void_p(self.stream.cuda_stream)))

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
        return {"fp64": torch.float64, "fp32": torch.float32, "fp16": torch.float16, "mom_fp64": torch.float64,
                "mom_fp32": torch.float32}[self.storage]

    # -- API -------------------------------------------------------------
    def init_fields(self, rho, u, pi1=None, dtype=None):
        """rho (nz,ny,nx), u (d,nz,ny,nx), pi1 packed (d(d+1)/2,nz,ny,nx) or None."""
        torch = _torch()
        dtype = dtype or torch.float64
        r = self._dev(rho, dtype).reshape(self.shape)
        v = self._dev(u, dtype).reshape((self.d,) + self.shape)
        p = None if pi1 is None else self._dev(pi1, dtype).reshape((self.d * (self.d + 1) // 2,) + self.shape)
        code = LB_F64 if dtype == torch.float64 else LB_F32
        check(_lib.load().lb_init_fields(self.handle, r.data_ptr(), v.data_ptr(), 0 if p is None else p.data_ptr(), code, 1))
        self._keep = (r, v, p)  # alive until the stream has consumed them
        return self

    def step(self, n=1):
        check(_lib.load().lb_step(self.handle, int(n)))
        return self

    def set_walls(self, x=False, y=False, z=False):
        """Resting no-slip walls on the first and last node of the flagged axes (lb_set_walls)."""
        mask = (1 if x else 0) | (2 if y else 0) | (4 if z else 0)
        check(_lib.load().lb_set_walls(self.handle, mask))
        self.walls = (bool(x), bool(y), bool(z))
        return self

    def set_check_interval(self, k):
        check(_lib.load().lb_set_check_interval(self.handle, int(k)))

    def moments(self, dtype=None, pi1=False):
        torch = _torch()
        dtype = dtype or torch.float64
        rho = torch.empty(self.shape, device="cuda", dtype=dtype)
        u = torch.empty((self.d,) + self.shape, device="cuda", dtype=dtype)
        p = torch.empty((self.d * (self.d + 1) // 2,) + self.shape, device="cuda", dtype=dtype) if pi1 else None
        code = LB_F64 if dtype == torch.float64 else LB_F32
        check(_lib.load().lb_moments(self.handle, rho.data_ptr(), u.data_ptr(), 0 if p is None else p.data_ptr(), code, 1))
        return (rho, u, p) if pi1 else (rho, u)

    def reduce(self):
        out = (ctypes.c_double * 5)()
        check(_lib.load().lb_reduce(self.handle, out))
        return tuple(out)

    def enstrophy(self):
        out = ctypes.c_double()
        check(_lib.load().lb_enstrophy(self.handle, ctypes.byref(out)))
        return out.value

    def get_populations(self):
        torch = _torch()
        t = torch.empty((self.q,) + self.shape, device="cuda", dtype=self.storage_dtype)
        check(_lib.load().lb_get_populations(self.handle, t.data_ptr(), 1))
        return t

    def set_populations(self, t):
        torch = _torch()
        t = torch.as_tensor(t).to(device="cuda", dtype=self.storage_dtype).contiguous()
        assert tuple(t.shape) == (self.q,) + self.shape
        check(_lib.load().lb_set_populations(self.handle, t.data_ptr(), 1))
        self._keep = (t,)

    def set_closure(self, params=None, norm=None, enable=True):
        """Enable the learned a1^(2) closure (D2Q9) with FP32 params (6723) and norm (78) tensors."""
        torch = _torch()
        if not enable:
            check(_lib.load().lb_set_closure(self.handle, None, None, 0))
            return
        p = torch.as_tensor(params).to(device="cuda", dtype=torch.float32).contiguous()
        n = torch.as_tensor(norm).to(device="cuda", dtype=torch.float32).contiguous()
        check(_lib.load().lb_set_closure(self.handle, p.data_ptr(), n.data_ptr(), 1))
        self._keep_closure = (p, n)

    def closure_features(self, a_target=None, plain_weight=1.0):
        """(features [nodes, 36], labels [nodes, 3]) of the next step;
        labels = a_target - plain_weight * plain a1^(2)."""
        torch = _torch()
        nodes = self.nx * self.ny * self.nz
        feat = torch.empty((nodes, 36), device="cuda", dtype=torch.float32)
        lab = torch.empty((nodes, 3), device="cuda", dtype=torch.float32)
        at = None if a_target is None else torch.as_tensor(a_target).to(device="cuda", dtype=torch.float64).contiguous()
        check(_lib.load().lb_closure_features(self.handle, 0 if at is None else at.data_ptr(), float(plain_weight),
                                              feat.data_ptr(), lab.data_ptr()))
        self._keep_target = at
        return feat, lab

    @property
    def steps(self):
        return _lib.load().lb_step_count(self.handle)

    @property
    def bytes_per_update(self):
        return _lib.load().lb_bytes_per_update(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            _lib.load().lb_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
