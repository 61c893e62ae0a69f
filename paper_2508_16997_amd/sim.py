"""Python face of the HIP library: one :class:`Simulation` per lattice.

PyTorch provides the device memory (workspace and field tensors) and the stream; every
step of the method runs in the library's kernels.  Nothing here computes physics.
"""
from __future__ import annotations

import ctypes as C
import sys
from typing import Optional

import numpy as np
import torch

from . import _lib as L

_DT = {"fp32": torch.float32, "fp64": torch.float64}


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


class Simulation:
    """A coupled viscoelastic LB simulation on one GPU (see include/vlb.h)."""

    def __init__(self, nx: int, ny: int, xmode: str = "periodic", ymode: str = "periodic",
                 precision: str = "fp32", solid: Optional[np.ndarray] = None, circles=(),
                 device: str = "cuda", stream: Optional[torch.cuda.Stream] = None,
                 tile: Optional[int] = None, graph_chunk: int = 0):
        self.lib = L.load()
        if precision not in _DT:
            raise ValueError("precision must be 'fp32' or 'fp64'")
        self.nx, self.ny, self.precision = int(nx), int(ny), precision
        self.xmode, self.ymode = xmode, ymode
        self.dtype = _DT[precision]
        self.device = torch.device(device)
        self._mask = None if solid is None else np.ascontiguousarray(solid, dtype=np.uint8)
        self._circ = np.ascontiguousarray(np.asarray(circles, dtype=np.float64).reshape(-1))
        grid = L.VlbGrid(self.nx, self.ny, L.MODES[xmode], L.MODES[ymode],
                         L.VLB_FP32 if precision == "fp32" else L.VLB_FP64,
                         None if self._mask is None else self._mask.ctypes.data,
                         self._circ.ctypes.data_as(C.POINTER(C.c_double)) if self._circ.size else None,
                         self._circ.size // 3)
        h = C.c_void_p()
        L.check(self.lib.vlb_create(C.byref(grid), C.byref(h)), "vlb_create")
        self._h = h
        nbytes = C.c_size_t()
        L.check(self.lib.vlb_workspace_bytes(h, C.byref(nbytes)), "vlb_workspace_bytes")
        self.workspace_bytes = int(nbytes.value)
        self._ws = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self._ws.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        if stream is None:
            # graph capture needs a stream other than the legacy null stream
            stream = (torch.cuda.Stream(self.device) if graph_chunk
                      else torch.cuda.current_stream(self.device))
        self.stream = stream
        if tile is not None:
            L.check(self.lib.vlb_set_tile(h, int(tile)), "vlb_set_tile")
        L.check(self.lib.vlb_bind(h, C.c_void_p(self._ws_ptr), self.workspace_bytes,
                                  C.c_void_p(self.stream.cuda_stream)), "vlb_bind")
        if graph_chunk:
            L.check(self.lib.vlb_set_graph_chunk(h, int(graph_chunk)), "vlb_set_graph_chunk")
        self._force = None

    # ------------------------------------------------------------------ set-up
    @classmethod
    def from_problem(cls, prob, precision: Optional[str] = None, **kw) -> "Simulation":
        """Build, parameterise and initialise from a problem description (synth.Problem)."""
        sim = cls(prob.nx, prob.ny, prob.xmode, prob.ymode, precision or prob.precision,
                  solid=prob.solid, circles=prob.circles, **kw)
        curved = getattr(prob, "curved", "bouzidi")
        if curved not in ("bouzidi", "ylw"):
            raise ValueError(f"unknown curved-wall scheme {curved!r}")
        ends = getattr(prob, "open_ends", "neqe")
        if ends not in ("neqe", "nebb"):
            raise ValueError(f"unknown open-end scheme {ends!r}")
        flags = (L.VLB_FLAG_CURVED_YLW if curved == "ylw" else 0) | \
            (L.VLB_FLAG_OPEN_NEBB if ends == "nebb" else 0)
        sim.set_params(prob.nu_s, prob.eta_p, prob.lam, prob.kappa, prob.Lambda_s, prob.Lambda_p,
                       *(((float(prob.Fx), float(prob.Fy)) if prob.uniform_force() else (0.0, 0.0))),
                       flags=flags,
                       model=getattr(prob, "model", "oldroyd_b"),
                       model_param=getattr(prob, "model_param", 0.0))
        if not prob.uniform_force():
            fx, fy = prob.force_arrays()
            sim.set_force_field(fx, fy)
        if prob.inlet is not None:
            sim.set_inlet(**{k: prob.inlet[k] for k in ("ux", "axx", "axy", "ayy")})
        sim.init(**prob.init_arrays())
        return sim

    def _order_after_torch(self):
        """Make the library's stream wait for work queued on torch's current stream."""
        cur = torch.cuda.current_stream(self.device)
        if cur.cuda_stream != self.stream.cuda_stream:
            self.stream.wait_stream(cur)

    def _order_before_torch(self):
        """Make torch's current stream wait for the library's stream."""
        cur = torch.cuda.current_stream(self.device)
        if cur.cuda_stream != self.stream.cuda_stream:
            cur.wait_stream(self.stream)

    def _dev(self, a) -> Optional[torch.Tensor]:
        if a is None:
            return None
        t = torch.as_tensor(np.asarray(a) if not torch.is_tensor(a) else a)
        t = t.to(device=self.device, dtype=self.dtype)
        t = torch.broadcast_to(t, (self.ny, self.nx)).contiguous()
        return t

    def set_params(self, nu_s, eta_p, lam, kappa, Lambda_s=0.25, Lambda_p=1e-6, Fx=0.0, Fy=0.0,
                   flags=0, model="oldroyd_b", model_param=0.0):
        """Lattice-unit parameters; ``model`` names the constitutive closure ('oldroyd_b',
        'giesekus' with model_param = alpha, 'lptt' / 'eptt' with epsilon, 'fene_p' with
        L^2)."""
        if model not in L.MODELS:
            raise ValueError(f"unknown constitutive model {model!r}")
        p = L.VlbParams(float(nu_s), float(eta_p), float(lam), float(kappa), float(Lambda_s),
                        float(Lambda_p), float(Fx), float(Fy), int(flags), L.MODELS[model],
                        float(model_param))
        L.check(self.lib.vlb_set_params(self._h, C.byref(p)), "vlb_set_params")
        self.params = dict(nu_s=float(nu_s), eta_p=float(eta_p), lam=float(lam),
                           kappa=float(kappa), Lambda_s=float(Lambda_s),
                           Lambda_p=float(Lambda_p), Fx=float(Fx), Fy=float(Fy), flags=int(flags),
                           model=model, model_param=float(model_param))

    def set_force_field(self, fx, fy):
        if fx is None and fy is None:
            L.check(self.lib.vlb_set_force_field(self._h, None, None), "vlb_set_force_field")
            self._force = None
            return
        tx, ty = self._dev(fx), self._dev(fy)
        self._order_after_torch()
        L.check(self.lib.vlb_set_force_field(self._h, _ptr(tx), _ptr(ty)), "vlb_set_force_field")
        self._force = (tx, ty)  # keep alive until the copy has run

    def set_inlet(self, ux, axx, axy, ayy):
        arrs = [np.ascontiguousarray(np.asarray(a, np.float64).reshape(self.ny))
                for a in (ux, axx, axy, ayy)]
        L.check(self.lib.vlb_set_inlet(self._h, *[a.ctypes.data for a in arrs]), "vlb_set_inlet")

    def init(self, rho=None, ux=None, uy=None, axx=None, axy=None, ayy=None):
        ts = [self._dev(a) for a in (rho, ux, uy, axx, axy, ayy)]
        self._order_after_torch()
        L.check(self.lib.vlb_init_equilibrium(self._h, *[_ptr(t) for t in ts]),
                "vlb_init_equilibrium")
        self._init_keep = ts

    # ------------------------------------------------------------------ run
    def step(self, n: int = 1):
        L.check(self.lib.vlb_step(self._h, int(n)), "vlb_step")

    @property
    def time(self) -> int:
        v = C.c_int64()
        L.check(self.lib.vlb_get_step(self._h, C.byref(v)), "vlb_get_step")
        return int(v.value)

    def read(self) -> dict:
        out = {k: torch.empty((self.ny, self.nx), dtype=self.dtype, device=self.device)
               for k in ("rho", "ux", "uy", "axx", "axy", "ayy")}
        self._order_after_torch()
        L.check(self.lib.vlb_read_fields(self._h, *[_ptr(out[k]) for k in
                                                    ("rho", "ux", "uy", "axx", "axy", "ayy")]),
                "vlb_read_fields")
        self._order_before_torch()
        return out

    def history(self) -> dict:
        out = {k: torch.empty((self.ny, self.nx), dtype=self.dtype, device=self.device)
               for k in ("sxx", "sxy", "syy", "uxp", "uyp")}
        self._order_after_torch()
        L.check(self.lib.vlb_read_history(self._h, *[_ptr(out[k]) for k in
                                                     ("sxx", "sxy", "syy", "uxp", "uyp")]),
                "vlb_read_history")
        self._order_before_torch()
        return out

    def monitors(self, raise_on_nonfinite: bool = True) -> dict:
        m = L.VlbMonitor()
        st = self.lib.vlb_monitors(self._h, C.byref(m))
        if st != L.VLB_E_NONFINITE or raise_on_nonfinite:
            L.check(st, "vlb_monitors")
        return dict(mass=list(m.mass), residual=m.residual, umax=m.umax, step=m.step,
                    nonfinite=m.nonfinite, spd_violations=m.spd_violations)

    def drag(self, circle: int = 0):
        """Momentum-exchange force (F_x, F_y) on a circle (all solids if circle < 0)."""
        fx, fy = C.c_double(), C.c_double()
        self._order_after_torch()
        L.check(self.lib.vlb_drag(self._h, int(circle), C.byref(fx), C.byref(fy)), "vlb_drag")
        return fx.value, fy.value

    def geometry(self):
        """(node_class (ny, nx) uint8, link nodes, dirs, q) -- host only."""
        cls = np.zeros((self.ny, self.nx), dtype=np.uint8)
        n = C.c_int()
        L.check(self.lib.vlb_geometry(self._h, cls.ctypes.data, None, None, None, 0, C.byref(n)),
                "vlb_geometry")
        cnt = n.value
        node = np.zeros(cnt, np.int32)
        d = np.zeros(cnt, np.int8)
        q = np.zeros(cnt, np.float64)
        L.check(self.lib.vlb_geometry(self._h, cls.ctypes.data, node.ctypes.data, d.ctypes.data,
                                      q.ctypes.data, cnt, C.byref(n)), "vlb_geometry")
        return cls, node, d, q

    def state_bytes(self) -> int:
        v = C.c_size_t()
        L.check(self.lib.vlb_state_bytes(self._h, C.byref(v)), "vlb_state_bytes")
        return int(v.value)

    def save_state(self, buf: Optional[torch.Tensor] = None) -> torch.Tensor:
        n = self.state_bytes()
        if buf is None:
            buf = torch.empty(n, dtype=torch.uint8, device=self.device)
        self._order_after_torch()
        L.check(self.lib.vlb_save_state(self._h, _ptr(buf), buf.numel()), "vlb_save_state")
        return buf

    def load_state(self, buf: torch.Tensor):
        self._order_after_torch()
        L.check(self.lib.vlb_load_state(self._h, _ptr(buf), buf.numel()), "vlb_load_state")

    def set_tile(self, ty: int):
        L.check(self.lib.vlb_set_tile(self._h, int(ty)), "vlb_set_tile")

    def set_store_mode(self, mode: int):
        """0 automatic, 1 cached, 2 non-temporal stores of the post-collision state."""
        L.check(self.lib.vlb_set_store_mode(self._h, int(mode)), "vlb_set_store_mode")

    def set_schedule(self, tile_order: int = 0, waves: int = 0):
        """Tile order (0 auto, 1 XCD bands, 2 row-major, 3 column strips) and register budget of the
        single-precision step kernel (0 auto, 3 or 4 waves per SIMD)."""
        L.check(self.lib.vlb_set_schedule(self._h, int(tile_order), int(waves)),
                "vlb_set_schedule")

    def set_graph_chunk(self, chunk: int):
        L.check(self.lib.vlb_set_graph_chunk(self._h, int(chunk)), "vlb_set_graph_chunk")

    # ------------------------------------------------------------------ adjoint
    @staticmethod
    def default_stride(nsteps: int) -> int:
        """Checkpoint stride ceil(sqrt(nsteps)): O(sqrt N) states held at once."""
        return max(1, int(np.ceil(np.sqrt(max(1, int(nsteps))))))

    def adjoint_workspace_bytes(self, nsteps: int, stride: Optional[int] = None) -> int:
        stride = stride or self.default_stride(nsteps)
        v = C.c_size_t()
        L.check(self.lib.vlb_adjoint_workspace_bytes(self._h, int(nsteps), int(stride),
                                                     C.byref(v)), "vlb_adjoint_workspace_bytes")
        return int(v.value)

    def _adjoint_ws(self, nsteps, stride):
        need = self.adjoint_workspace_bytes(nsteps, stride)
        buf = getattr(self, "_adj_buf", None)
        if buf is None or buf.numel() < need + 256:
            self._adj_buf = buf = torch.empty(need + 256, dtype=torch.uint8, device=self.device)
        ptr = (buf.data_ptr() + 255) // 256 * 256
        return ptr, buf.numel() - (ptr - buf.data_ptr())

    def adjoint_forward(self, nsteps: int, stride: Optional[int] = None):
        """Advance nsteps steps, saving checkpoints for :meth:`adjoint_backward`."""
        stride = stride or self.default_stride(nsteps)
        ptr, nbytes = self._adjoint_ws(nsteps, stride)
        self._order_after_torch()
        L.check(self.lib.vlb_adjoint_forward(self._h, int(nsteps), int(stride), C.c_void_p(ptr),
                                             nbytes), "vlb_adjoint_forward")
        self._adj_rec = (ptr, nbytes)

    def adjoint_backward(self, dL_dux, dL_duy) -> dict:
        """Gradients of L given dL/du of the last readout: dlambda, deta_p, dFx, dFy."""
        if getattr(self, "_adj_rec", None) is None:
            raise RuntimeError("adjoint_backward needs adjoint_forward first")
        ptr, nbytes = self._adj_rec
        gx, gy = self._dev(dL_dux), self._dev(dL_duy)
        out = {k: torch.empty((self.ny, self.nx), dtype=torch.float64, device=self.device)
               for k in ("dFx", "dFy")}
        dl, de = C.c_double(), C.c_double()
        self._order_after_torch()
        L.check(self.lib.vlb_adjoint_backward(self._h, _ptr(gx), _ptr(gy), C.byref(dl), C.byref(de),
                                              _ptr(out["dFx"]), _ptr(out["dFy"]), C.c_void_p(ptr),
                                              nbytes), "vlb_adjoint_backward")
        self._order_before_torch()
        out["dlambda"] = dl.value
        out["deta_p"] = de.value
        return out

    def adjoint(self, nsteps: int, ux_target, uy_target, stride: Optional[int] = None) -> dict:
        """Loss (1/2N) sum |u(T) - u*|^2 after nsteps steps and its gradients."""
        stride = stride or self.default_stride(nsteps)
        ptr, nbytes = self._adjoint_ws(nsteps, stride)
        tx, ty = self._dev(ux_target), self._dev(uy_target)
        out = {k: torch.empty((self.ny, self.nx), dtype=torch.float64, device=self.device)
               for k in ("dFx", "dFy")}
        loss, dl, de = C.c_double(), C.c_double(), C.c_double()
        self._order_after_torch()
        L.check(self.lib.vlb_adjoint(self._h, int(nsteps), int(stride), _ptr(tx), _ptr(ty),
                                     C.byref(loss), C.byref(dl), C.byref(de), _ptr(out["dFx"]),
                                     _ptr(out["dFy"]), C.c_void_p(ptr), nbytes), "vlb_adjoint")
        self._order_before_torch()
        self._adj_rec = (ptr, nbytes)
        out.update(loss=loss.value, dlambda=dl.value, deta_p=de.value)
        return out

    def close(self):
        if getattr(self, "_h", None):
            self.stream.synchronize()
            self.lib.vlb_destroy(self._h)
            self._h = None

    def __del__(self):
        # during interpreter shutdown the HIP runtime (and a profiler's hooks) may already
        # be torn down: leave the handle to process exit instead of calling into it
        if sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many simulations advanced together by one step and one boundary launch per step.

    The members must share one stream, one precision and one step count and be fully
    set up (parameters, force, inlet, initial state) before the batch is made; the batch
    takes their descriptors at creation.  Each member stays readable through its own
    :class:`Simulation` methods.
    """

    def __init__(self, sims, tile: int = 4, graph_chunk: int = 0, persistent: bool = False,
                 noalloc: bool = False, schedule=None):
        """``noalloc``: build the batch with vlb_batch_create_noalloc (lists in the
        library's static per-device scratch, no workspace tensor; one such batch per
        device at a time)."""
        self.lib = L.load()
        self.sims = list(sims)
        if not self.sims:
            raise ValueError("a batch needs at least one simulation")
        self.stream = self.sims[0].stream
        self.device = self.sims[0].device
        arr = (C.c_void_p * len(self.sims))(*[s._h.value for s in self.sims])
        h = C.c_void_p()
        if noalloc:
            self.workspace_bytes, self._ws = 0, None
            self.sims[0]._order_after_torch()
            with torch.cuda.device(self.device):
                L.check(self.lib.vlb_batch_create_noalloc(arr, len(self.sims), int(tile),
                                                          C.byref(h)), "vlb_batch_create_noalloc")
        else:
            nbytes = C.c_size_t()
            L.check(self.lib.vlb_batch_workspace_bytes(arr, len(self.sims), int(tile),
                                                       C.byref(nbytes)),
                    "vlb_batch_workspace_bytes")
            self.workspace_bytes = int(nbytes.value)
            self._ws = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8,
                                   device=self.device)
            ptr = (self._ws.data_ptr() + 255) // 256 * 256
            self.sims[0]._order_after_torch()
            L.check(self.lib.vlb_batch_create(arr, len(self.sims), int(tile), C.c_void_p(ptr),
                                              self.workspace_bytes, C.byref(h)),
                    "vlb_batch_create")
        self._h = h
        if graph_chunk:
            L.check(self.lib.vlb_batch_set_graph_chunk(h, int(graph_chunk)),
                    "vlb_batch_set_graph_chunk")
        if persistent:
            L.check(self.lib.vlb_batch_set_persistent(h, 1), "vlb_batch_set_persistent")
        if schedule:
            self.set_schedule(*schedule)

    def set_schedule(self, tile_order: int = 0, waves: int = 0):
        """As :meth:`Simulation.set_schedule`, for the batch's launches."""
        self.sims[0]._order_after_torch()
        L.check(self.lib.vlb_batch_set_schedule(self._h, int(tile_order), int(waves)),
                "vlb_batch_set_schedule")

    def step(self, n: int = 1):
        self.sims[0]._order_after_torch()
        L.check(self.lib.vlb_batch_step(self._h, int(n)), "vlb_batch_step")
        self.sims[0]._order_before_torch()

    def read(self, run: int) -> dict:
        """Fields of member ``run`` through the batch (vlb_batch_read_fields)."""
        s = self.sims[run]
        out = {k: torch.empty((s.ny, s.nx), dtype=s.dtype, device=s.device)
               for k in ("rho", "ux", "uy", "axx", "axy", "ayy")}
        s._order_after_torch()
        L.check(self.lib.vlb_batch_read_fields(self._h, int(run), *[_ptr(out[k]) for k in
                                               ("rho", "ux", "uy", "axx", "axy", "ayy")]),
                "vlb_batch_read_fields")
        s._order_before_torch()
        return out

    def close(self):
        if getattr(self, "_h", None):
            self.stream.synchronize()
            self.lib.vlb_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        # during interpreter shutdown the HIP runtime (and a profiler's hooks) may already
        # be torn down: leave the handle to process exit instead of calling into it
        if sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


def params_from_groups(Re, Wi, beta, Sc, Ma, Lc, Lambda_s=0.25, Lambda_p=1e-6) -> dict:
    """Lattice-unit parameters from the dimensionless groups (library host routine)."""
    lib = L.load()
    p = L.VlbParams()
    uc = C.c_double()
    L.check(lib.vlb_params_from_groups(float(Re), float(Wi), float(beta), float(Sc), float(Ma),
                                       float(Lc), float(Lambda_s), float(Lambda_p), C.byref(p),
                                       C.byref(uc)), "vlb_params_from_groups")
    return dict(nu_s=p.nu_s, eta_p=p.eta_p, lam=p.lambda_, kappa=p.kappa, Lambda_s=p.Lambda_s,
                Lambda_p=p.Lambda_p, Uc=uc.value)


def host_geometry(nx, ny, xmode="periodic", ymode="periodic", solid=None, circles=()):
    """Node classes and boundary links from the library's host builder (no GPU needed)."""
    lib = L.load()
    mask = None if solid is None else np.ascontiguousarray(solid, dtype=np.uint8)
    circ = np.ascontiguousarray(np.asarray(circles, dtype=np.float64).reshape(-1))
    grid = L.VlbGrid(int(nx), int(ny), L.MODES[xmode], L.MODES[ymode], L.VLB_FP64,
                     None if mask is None else mask.ctypes.data,
                     circ.ctypes.data_as(C.POINTER(C.c_double)) if circ.size else None,
                     circ.size // 3)
    h = C.c_void_p()
    L.check(lib.vlb_create(C.byref(grid), C.byref(h)), "vlb_create")
    try:
        cls = np.zeros((ny, nx), dtype=np.uint8)
        n = C.c_int()
        L.check(lib.vlb_geometry(h, cls.ctypes.data, None, None, None, 0, C.byref(n)), "geometry")
        cnt = n.value
        node = np.zeros(cnt, np.int32)
        d = np.zeros(cnt, np.int8)
        q = np.zeros(cnt, np.float64)
        L.check(lib.vlb_geometry(h, cls.ctypes.data, node.ctypes.data, d.ctypes.data,
                                 q.ctypes.data, cnt, C.byref(n)), "geometry")
        return cls, node, d, q
    finally:
        lib.vlb_destroy(h)
