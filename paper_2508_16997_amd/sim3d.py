"""Three-dimensional (D3Q19 / D3Q27) simulation object over libvlb.so (include/vlb3d.h).

Argument marshalling only: every step runs in the library's HIP kernels; PyTorch
provides the device workspace, the stream and the field tensors.
"""
from __future__ import annotations

import ctypes as C
import sys
from typing import Optional

import numpy as np
import torch

from . import _lib as L

FIELDS3 = ("rho", "ux", "uy", "uz", "axx", "axy", "axz", "ayy", "ayz", "azz")


class Simulation3D:
    """One D3Q19 (q = 19) or D3Q27 (q = 27) simulation: x and z periodic, y periodic or
    half-way walls."""

    def __init__(self, nx: int, ny: int, nz: int, ymode: str = "periodic",
                 precision: str = "fp32", device: Optional[torch.device] = None,
                 stream: Optional[torch.cuda.Stream] = None, q: int = 19):
        self.lib = L.load()
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.precision = precision
        self.dtype = torch.float32 if precision == "fp32" else torch.float64
        prec = L.VLB_FP32 if precision == "fp32" else L.VLB_FP64
        h = C.c_void_p()
        self.q = int(q)
        L.check(self.lib.vlb3_create(self.nx, self.ny, self.nz, self.q, prec, L.MODES[ymode],
                                     C.byref(h)), "vlb3_create")
        self._h = h
        self.device = device or torch.device("cuda", torch.cuda.current_device())
        v = C.c_size_t()
        L.check(self.lib.vlb3_workspace_bytes(self._h, C.byref(v)), "vlb3_workspace_bytes")
        self.workspace_bytes = int(v.value)
        self._ws = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=self.device)
        self._ws_ptr = (self._ws.data_ptr() + 255) // 256 * 256
        self.stream = stream or torch.cuda.current_stream(self.device)
        L.check(self.lib.vlb3_bind(self._h, C.c_void_p(self._ws_ptr), self.workspace_bytes,
                                   C.c_void_p(self.stream.cuda_stream)), "vlb3_bind")

    @classmethod
    def from_problem(cls, prob, precision: Optional[str] = None, **kw) -> "Simulation3D":
        """Build, parameterise and initialise from a synth.Problem3D."""
        kw.setdefault("q", prob.q)
        sim = cls(prob.nx, prob.ny, prob.nz, prob.ymode, precision or prob.precision, **kw)
        if getattr(prob, "solid", None) is not None:
            sim.set_solid(prob.solid)
        sim.set_params(prob.nu_s, prob.eta_p, prob.lam, prob.kappa, prob.Lambda_s,
                       prob.Lambda_p, *prob.F, model=getattr(prob, "model", "oldroyd_b"),
                       model_param=getattr(prob, "model_param", 0.0))
        sim.init(**prob.init_arrays())
        return sim

    def _order_after_torch(self):
        cur = torch.cuda.current_stream(self.device)
        if cur.cuda_stream != self.stream.cuda_stream:
            self.stream.wait_stream(cur)

    def _order_before_torch(self):
        cur = torch.cuda.current_stream(self.device)
        if cur.cuda_stream != self.stream.cuda_stream:
            cur.wait_stream(self.stream)

    def set_solid(self, mask):
        """Solid nodes from a [nz][ny][nx] mask (nonzero = solid), or None for none; call
        before init()."""
        if mask is None:
            L.check(self.lib.vlb3_set_solid(self._h, None), "vlb3_set_solid")
            return
        m = np.ascontiguousarray(np.asarray(mask).reshape(self.nz, self.ny, self.nx) != 0,
                                 dtype=np.uint8)
        L.check(self.lib.vlb3_set_solid(self._h, m.ctypes.data), "vlb3_set_solid")

    def set_params(self, nu_s, eta_p, lam, kappa, Lambda_s=0.25, Lambda_p=1e-6, Fx=0.0, Fy=0.0,
                   Fz=0.0, flags=0, model="oldroyd_b", model_param=0.0):
        """Lattice-unit parameters and the constitutive closure ('oldroyd_b', 'giesekus'
        with model_param = alpha, 'lptt' / 'eptt' with epsilon, 'fene_p' with L^2 > 3)."""
        if model not in L.MODELS:
            raise ValueError(f"unknown constitutive model {model!r}")
        L.check(self.lib.vlb3_set_params(self._h, float(nu_s), float(eta_p), float(lam),
                                         float(kappa), float(Lambda_s), float(Lambda_p),
                                         float(Fx), float(Fy), float(Fz), int(flags)),
                "vlb3_set_params")
        L.check(self.lib.vlb3_set_closure(self._h, L.MODELS[model], float(model_param)),
                "vlb3_set_closure")

    def init(self, **fields):
        shape = (self.nz, self.ny, self.nx)
        keep = []
        ptrs = (C.c_void_p * 10)()
        for c, name in enumerate(FIELDS3):
            a = fields.get(name)
            if a is None:
                ptrs[c] = None
                continue
            t = torch.as_tensor(np.ascontiguousarray(np.broadcast_to(np.asarray(a), shape))
                                if not torch.is_tensor(a) else a)
            t = t.to(device=self.device, dtype=self.dtype).contiguous()
            keep.append(t)
            ptrs[c] = t.data_ptr()
        self._order_after_torch()
        L.check(self.lib.vlb3_init_equilibrium(self._h, ptrs), "vlb3_init_equilibrium")

    def step(self, n: int = 1):
        L.check(self.lib.vlb3_step(self._h, int(n)), "vlb3_step")

    @property
    def time(self) -> int:
        v = C.c_int64()
        L.check(self.lib.vlb3_get_step(self._h, C.byref(v)), "vlb3_get_step")
        return int(v.value)

    def read(self) -> dict:
        """rho, u (half-force shift) and the six conformation components, [nz][ny][nx]."""
        out = {k: torch.empty((self.nz, self.ny, self.nx), dtype=self.dtype, device=self.device)
               for k in FIELDS3}
        ptrs = (C.c_void_p * 10)(*[out[k].data_ptr() for k in FIELDS3])
        self._order_after_torch()
        L.check(self.lib.vlb3_read_fields(self._h, ptrs), "vlb3_read_fields")
        self._order_before_torch()
        return out

    def close(self):
        if getattr(self, "_h", None):
            self.lib.vlb3_destroy(self._h)
            self._h = None

    def __del__(self):
        if sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass
