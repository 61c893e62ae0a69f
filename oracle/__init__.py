"""FP64 CPU oracle of the coupled viscoelastic lattice Boltzmann step -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (``paper_2508_16997_amd``)
never imports, links or calls anything here, and the oracle shares no code with it.

The arithmetic lives in ``vlb_oracle.cpp`` (plain C++17, double precision, no
fast-math, FMA contraction off); this module only builds it with g++ and marshals
arguments through ctypes.  Functions whose result is pinned only by other oracle code
are listed in the design notes as "parity unpinned".
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vlb_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None
# the three-dimensional (D3Q19) oracle: a separate library, vlb_oracle3d.cpp
_SRC3 = os.path.join(_HERE, "vlb_oracle3d.cpp")
_LIB3 = os.path.join(_HERE, "liboracle3d.so")
_lib3 = None

MODES = {"periodic": 0, "wall": 1, "open": 2, "wet": 3}
# constitutive closures (model function F(A), Sec. 2.2) and the meaning of model_param
MODELS = {"oldroyd_b": 0, "giesekus": 1, "lptt": 2, "eptt": 3, "fene_p": 4}
FLAG_NO_SOURCE = 1
FLAG_NO_GTILDE = 2  # planted mistake for sensitivity checks: drop G~_i
# alternative readings of the CNEBB scheme (Sec. 3.3), for sensitivity measurements only:
FLAG_CNEBB_UB_ZERO = 4  # zero wall velocity in the CNEBB equilibrium (reading A11's alternative)
FLAG_CNEBB_PAIR_NEQ = 8  # both-unknown pairs keep a non-equilibrium part (A12's alternative)
# the curved-wall scheme of the paper's cylinder for f (Sec. 4.3, reading A30); set from
# Problem.curved == "ylw"
FLAG_CURVED_YLW = 16
# wet-node NEBB open ends for f (Sec. 4.3, reading A31); set from Problem.open_ends == "nebb"
FLAG_OPEN_NEBB = 32


def build(force: bool = True) -> str:
    """Compile the oracles into ``oracle/liboracle.so`` and ``oracle/liboracle3d.so``
    (g++, -O2, no fast-math)."""
    for src, lib in ((_SRC, _LIB), (_SRC3, _LIB3)):
        if force or not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(src):
            tmp = lib + ".tmp"
            cmd = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math",
                   "-fopenmp", "-shared", "-fPIC", "-o", tmp, src]
            subprocess.run(cmd, check=True)
            os.replace(tmp, lib)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    path = os.environ.get("ORACLE_LIBRARY")  # an instrumented build (sanitizer tests)
    if not path:
        if not os.path.exists(_LIB):
            build(force=True)
        path = _LIB
    lib = C.CDLL(path)
    P = C.c_void_p
    D = C.c_double
    DP = C.POINTER(C.c_double)
    lib.orc_create.restype = P
    lib.orc_create.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_void_p, DP, C.c_int, C.c_int]
    lib.orc_destroy.argtypes = [P]
    lib.orc_set_threads.argtypes = [C.c_int]
    lib.orc_max_threads.restype = C.c_int
    lib.orc_set_params.argtypes = [P, D, D, D, D, D, D, C.c_int]
    lib.orc_set_force.argtypes = [P, D, D, DP, DP]
    lib.orc_set_tangent.argtypes = [P, D, D, DP, DP]
    lib.orc_set_inlet.argtypes = [P, DP, DP, DP, DP]
    lib.orc_init.argtypes = [P, DP, DP, DP, DP, DP, DP]
    lib.orc_step.argtypes = [P, C.c_longlong]
    lib.orc_get_step.restype = C.c_longlong
    lib.orc_get_step.argtypes = [P]
    lib.orc_read.argtypes = [P, DP, DP, DP, DP, DP, DP]
    lib.orc_read_tangent.argtypes = [P, DP, DP, DP, DP, DP, DP]
    lib.orc_read_history.argtypes = [P, DP, DP, DP, DP, DP]
    lib.orc_read_populations.argtypes = [P, DP, DP]
    lib.orc_drag.argtypes = [P, C.c_int, DP]
    lib.orc_geometry.argtypes = [P, C.c_void_p, C.c_void_p, C.c_void_p, DP, C.c_int]
    lib.orc_lattice.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, DP]
    lib.orc_node_feq.argtypes = [D, D, D, DP]
    lib.orc_node_geq.argtypes = [D, D, D, DP]
    lib.orc_node_hydro.argtypes = [DP, D, D, D, D, D, D, D, D, D, DP]
    lib.orc_node_cde.argtypes = [DP, D, D, D, D, D, D, D, D, D, D, D, DP]
    lib.orc_node_source.argtypes = [DP, DP, D, DP]
    lib.orc_node_source_model.argtypes = [DP, DP, D, C.c_int, D, DP]
    lib.orc_set_model.argtypes = [P, C.c_int, D]
    lib.orc_node_fd.restype = D
    lib.orc_node_fd.argtypes = [C.c_int, D, D, D, C.c_int, D, D]
    _lib = lib
    return lib


def _dp(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _c64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def set_threads(n: int) -> None:
    _load().orc_set_threads(int(n))


def max_threads() -> int:
    return int(_load().orc_max_threads())


class OracleSim:
    """One oracle simulation built from a :class:`synth.Problem`."""

    def __init__(self, prob, dual: bool = False, flags: int = 0):
        lib = _load()
        self.prob = prob
        self.nx, self.ny = prob.nx, prob.ny
        self.dual = dual
        mask = None
        if prob.solid is not None:
            mask = np.ascontiguousarray(prob.solid, dtype=np.uint8)
        circ = np.ascontiguousarray(np.array(prob.circles, dtype=np.float64).reshape(-1))
        self._keep = [mask, circ]
        self.h = lib.orc_create(prob.nx, prob.ny, MODES[prob.xmode], MODES[prob.ymode],
                                None if mask is None else mask.ctypes.data,
                                _dp(circ) if circ.size else None, len(prob.circles),
                                1 if dual else 0)
        if not self.h:
            raise ValueError("oracle: invalid grid")
        if getattr(prob, "curved", "bouzidi") == "ylw":
            flags |= FLAG_CURVED_YLW
        if getattr(prob, "open_ends", "neqe") == "nebb":
            flags |= FLAG_OPEN_NEBB
        rc = lib.orc_set_params(self.h, prob.nu_s, prob.eta_p, prob.lam, prob.kappa,
                                prob.Lambda_s, prob.Lambda_p, flags)
        if rc != 0:
            raise ValueError("oracle: invalid parameters")
        model = getattr(prob, "model", "oldroyd_b")
        if lib.orc_set_model(self.h, MODELS[model], float(getattr(prob, "model_param", 0.0))) != 0:
            raise ValueError(f"oracle: invalid model parameter for {model}")
        self.set_force(prob.Fx, prob.Fy)
        if prob.inlet is not None:
            i = prob.inlet
            arrs = [_c64(i[k]) for k in ("ux", "axx", "axy", "ayy")]
            lib.orc_set_inlet(self.h, *[_dp(a) for a in arrs])
        self.init()

    def __del__(self):
        if getattr(self, "h", None):
            _load().orc_destroy(self.h)
            self.h = None

    def set_force(self, Fx, Fy):
        lib = _load()
        if np.ndim(Fx) == 0 and np.ndim(Fy) == 0:
            lib.orc_set_force(self.h, float(Fx), float(Fy), None, None)
        else:
            fx = _c64(np.broadcast_to(np.asarray(Fx, np.float64), (self.ny, self.nx)))
            fy = _c64(np.broadcast_to(np.asarray(Fy, np.float64), (self.ny, self.nx)))
            lib.orc_set_force(self.h, 0.0, 0.0, _dp(fx), _dp(fy))

    def set_tangent(self, dlam=0.0, deta=0.0, dFx=None, dFy=None):
        fx = None if dFx is None else _c64(np.broadcast_to(dFx, (self.ny, self.nx)))
        fy = None if dFy is None else _c64(np.broadcast_to(dFy, (self.ny, self.nx)))
        rc = _load().orc_set_tangent(self.h, float(dlam), float(deta), _dp(fx), _dp(fy))
        if rc != 0:
            raise ValueError("oracle: tangent needs a dual-number simulation")

    def init(self, fields: Optional[dict] = None):
        f = self.prob.init_arrays() if fields is None else fields
        arrs = [_c64(f[k]) for k in ("rho", "ux", "uy", "axx", "axy", "ayy")]
        _load().orc_init(self.h, *[_dp(a) for a in arrs])

    def step(self, n: int = 1):
        _load().orc_step(self.h, int(n))

    @property
    def time(self) -> int:
        return int(_load().orc_get_step(self.h))

    def read(self) -> dict:
        out = {k: np.zeros((self.ny, self.nx)) for k in ("rho", "ux", "uy", "axx", "axy", "ayy")}
        _load().orc_read(self.h, *[_dp(out[k]) for k in ("rho", "ux", "uy", "axx", "axy", "ayy")])
        return out

    def read_tangent(self) -> dict:
        out = {k: np.zeros((self.ny, self.nx)) for k in ("rho", "ux", "uy", "axx", "axy", "ayy")}
        rc = _load().orc_read_tangent(self.h, *[_dp(out[k]) for k in
                                                ("rho", "ux", "uy", "axx", "axy", "ayy")])
        if rc != 0:
            raise ValueError("oracle: tangents need a dual-number simulation")
        return out

    def history(self):
        out = {k: np.zeros((self.ny, self.nx)) for k in ("sxx", "sxy", "syy", "uxp", "uyp")}
        first = _load().orc_read_history(self.h, *[_dp(out[k]) for k in
                                                   ("sxx", "sxy", "syy", "uxp", "uyp")])
        return out, bool(first)

    def drag(self, circle: int = 0):
        """Momentum-exchange force (F_x, F_y) on a circle (all solids if circle < 0)."""
        out = np.zeros(2)
        if _load().orc_drag(self.h, int(circle), _dp(out)) != 0:
            raise ValueError("oracle: drag needs at least one step")
        return float(out[0]), float(out[1])

    def populations(self):
        n = self.nx * self.ny
        f = np.zeros((9, n))
        g = np.zeros((3, 9, n))
        _load().orc_read_populations(self.h, _dp(f), _dp(g))
        return f.reshape(9, self.ny, self.nx), g.reshape(3, 9, self.ny, self.nx)

    def geometry(self):
        """(node_class (ny, nx) uint8, links structured array of (node, dir, q))."""
        lib = _load()
        cls = np.zeros((self.ny, self.nx), dtype=np.uint8)
        cnt = lib.orc_geometry(self.h, cls.ctypes.data, None, None, None, 0)
        node = np.zeros(cnt, dtype=np.int32)
        d = np.zeros(cnt, dtype=np.int8)
        q = np.zeros(cnt, dtype=np.float64)
        lib.orc_geometry(self.h, cls.ctypes.data, node.ctypes.data, d.ctypes.data, _dp(q), cnt)
        return cls, node, d, q


def lattice():
    lib = _load()
    ex = np.zeros(9, np.int32)
    ey = np.zeros(9, np.int32)
    opp = np.zeros(9, np.int32)
    w = np.zeros(9)
    lib.orc_lattice(ex.ctypes.data, ey.ctypes.data, opp.ctypes.data, _dp(w))
    return ex, ey, opp, w


def node_feq(rho, ux, uy):
    out = np.zeros(9)
    _load().orc_node_feq(rho, ux, uy, _dp(out))
    return out


def node_geq(phi, ux, uy):
    out = np.zeros(9)
    _load().orc_node_geq(phi, ux, uy, _dp(out))
    return out


def node_hydro(f9, Fx, Fy, tau_s1, tau_s2, tau_ab=(0.0, 0.0, 0.0), D=(0.0, 0.0)):
    f9 = _c64(f9)
    out = np.zeros(9)
    _load().orc_node_hydro(_dp(f9), Fx, Fy, tau_s1, tau_s2, tau_ab[0], tau_ab[1], tau_ab[2],
                           D[0], D[1], _dp(out))
    return out


def node_cde(g9, rho, ux, uy, Fx, Fy, S, Sp, uxp, uyp, tau_p1, tau_p2):
    g9 = _c64(g9)
    out = np.zeros(9)
    _load().orc_node_cde(_dp(g9), rho, ux, uy, Fx, Fy, S, Sp, uxp, uyp, tau_p1, tau_p2, _dp(out))
    return out


def node_source(A3, L4, lam, model=None, mpar=0.0):
    """Constitutive source (S_xx, S_xy, S_yy) at one node; L4 = (d_x u_x, d_x u_y,
    d_y u_x, d_y u_y).  Without a model: the Oldroyd-B entry point."""
    A3 = _c64(A3)
    L4 = _c64(L4)
    out = np.zeros(3)
    if model is None:
        _load().orc_node_source(_dp(A3), _dp(L4), lam, _dp(out))
    else:
        _load().orc_node_source_model(_dp(A3), _dp(L4), lam, MODELS[model], float(mpar),
                                      _dp(out))
    return out


def node_fd(lo_solid, qlo, plo, p0, hi_solid, qhi, phi):
    return float(_load().orc_node_fd(int(lo_solid), qlo, plo, p0, int(hi_solid), qhi, phi))


# ------------------------------------------------------------------------------------
# Three-dimensional (D3Q19 / D3Q27) oracle
# ------------------------------------------------------------------------------------
FIELDS3 = ("rho", "ux", "uy", "uz", "axx", "axy", "axz", "ayy", "ayz", "azz")


def _load3():
    global _lib3
    if _lib3 is not None:
        return _lib3
    path = os.environ.get("ORACLE3D_LIBRARY")
    if not path:
        if not os.path.exists(_LIB3) or os.path.getmtime(_LIB3) < os.path.getmtime(_SRC3):
            build(force=False)
        path = _LIB3
    lib = C.CDLL(path)
    P, D, DP = C.c_void_p, C.c_double, C.POINTER(C.c_double)
    lib.o3_create.restype = P
    lib.o3_create.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int]
    lib.o3_destroy.argtypes = [P]
    lib.o3_set_solid.argtypes = [P, C.c_void_p]
    lib.o3_set_params.argtypes = [P, D, D, D, D, D, D, D, D, D, C.c_int]
    lib.o3_init.argtypes = [P] + [DP] * 10
    lib.o3_step.argtypes = [P, C.c_longlong]
    lib.o3_read.argtypes = [P] + [DP] * 10
    lib.o3_collide_hydro.restype = C.c_int
    lib.o3_collide_hydro.argtypes = [C.c_int, DP, D, DP, DP, DP, DP, D, D, DP]
    lib.o3_collide_cde.restype = C.c_int
    lib.o3_collide_cde.argtypes = [C.c_int, DP, D, D, DP, DP, D, D, DP, D, D, DP]
    lib.o3_source.argtypes = [DP, DP, D, DP]
    lib.o3_source_model.argtypes = [DP, DP, D, C.c_int, D, DP]
    lib.o3_set_model.restype = C.c_int
    lib.o3_set_model.argtypes = [P, C.c_int, D]
    lib.o3_lattice.restype = C.c_int
    lib.o3_lattice.argtypes = [C.c_int, C.c_void_p, DP, C.c_void_p, DP]
    _lib3 = lib
    return lib


class OracleSim3D:
    """One three-dimensional oracle simulation built from a :class:`synth.Problem3D`."""

    def __init__(self, prob, no_source: bool = False):
        lib = _load3()
        self.prob = prob
        self.shape = (prob.nz, prob.ny, prob.nx)
        self.h = lib.o3_create(prob.nx, prob.ny, prob.nz, 1 if prob.ymode == "wall" else 0,
                               int(prob.q))
        if not self.h:
            raise ValueError("oracle3d: invalid grid")
        if getattr(prob, "solid", None) is not None:
            self._mask = np.ascontiguousarray(prob.solid, dtype=np.uint8).reshape(self.shape)
            lib.o3_set_solid(self.h, self._mask.ctypes.data)
        Fx, Fy, Fz = (float(v) for v in prob.F)
        if lib.o3_set_params(self.h, prob.nu_s, prob.eta_p, prob.lam, prob.kappa, prob.Lambda_s,
                             prob.Lambda_p, Fx, Fy, Fz, 1 if no_source else 0) != 0:
            raise ValueError("oracle3d: invalid parameters")
        model = getattr(prob, "model", "oldroyd_b")
        if lib.o3_set_model(self.h, MODELS[model], float(getattr(prob, "model_param", 0.0))) != 0:
            raise ValueError(f"oracle3d: invalid model parameter for {model}")
        f = prob.init_arrays()
        arrs = [_c64(f[k]) for k in FIELDS3]
        lib.o3_init(self.h, *[_dp(a) for a in arrs])

    def __del__(self):
        if getattr(self, "h", None):
            _load3().o3_destroy(self.h)
            self.h = None

    def step(self, n: int = 1):
        _load3().o3_step(self.h, int(n))

    def read(self) -> dict:
        out = {k: np.zeros(self.shape) for k in FIELDS3}
        _load3().o3_read(self.h, *[_dp(out[k]) for k in FIELDS3])
        return out


def collide_hydro3d(q, f, rho, u, F=(0.0, 0.0, 0.0), tau=None, D=(0.0, 0.0, 0.0), tau_s1=1.0,
                    tau_s2=1.0):
    """One hydrodynamic collision of the three-dimensional step at a single node (q
    populations in, q out); tau is the 3 x 3 polymer stress, D the diagonal defects."""
    f = _c64(np.asarray(f, float))
    out = np.zeros(int(q))
    t = _c64(np.zeros((3, 3)) if tau is None else np.asarray(tau, float))
    a = [_c64(np.asarray(v, float)) for v in (u, F, D)]
    if _load3().o3_collide_hydro(int(q), _dp(f), float(rho), _dp(a[0]), _dp(a[1]), _dp(t),
                                 _dp(a[2]), float(tau_s1), float(tau_s2), _dp(out)) != 0:
        raise ValueError("oracle3d: q must be 19 or 27")
    return out


def collide_cde3d(q, g, phi, rho, u, F=(0.0, 0.0, 0.0), S=0.0, Sp=0.0, up=None, tau_p1=1.0,
                  tau_p2=1.0):
    """One convection-diffusion collision of the three-dimensional step at a single node."""
    g = _c64(np.asarray(g, float))
    out = np.zeros(int(q))
    a = [_c64(np.asarray(v, float)) for v in (u, F, u if up is None else up)]
    if _load3().o3_collide_cde(int(q), _dp(g), float(phi), float(rho), _dp(a[0]), _dp(a[1]),
                               float(S), float(Sp), _dp(a[2]), float(tau_p1), float(tau_p2),
                               _dp(out)) != 0:
        raise ValueError("oracle3d: q must be 19 or 27")
    return out


def source3d(A, L, lam, model=None, mpar=0.0):
    """The three-dimensional constitutive source for the conformation A and the velocity
    gradient L[g][b] = d_g u_b (3 x 3 each), relaxation time lam; model names a closure
    as in synth.Problem (None: the Oldroyd-B entry point)."""
    a, l = _c64(np.asarray(A, float)), _c64(np.asarray(L, float))
    out = np.zeros((3, 3))
    if model is None:
        _load3().o3_source(_dp(a), _dp(l), float(lam), _dp(out))
    else:
        _load3().o3_source_model(_dp(a), _dp(l), float(lam), MODELS[model], float(mpar), _dp(out))
    return out


def lattice3d(q: int = 19):
    """Velocities (q, 3), weights, opposites and the third-order basis at every velocity
    (q, nb3) of D3Q19 (q = 19: the combinations h_{c,+}, h_{c,-} for c = 0, 1, 2) or
    D3Q27 (q = 27: H_xxy, H_xxz, H_yyx, H_yyz, H_zzx, H_zzy, H_xyz)."""
    e = np.zeros((27, 3), np.int32)
    w = np.zeros(27)
    opp = np.zeros(27, np.int32)
    h3 = np.zeros(27 * 7)
    nb3 = _load3().o3_lattice(int(q), e.ctypes.data, _dp(w), opp.ctypes.data, _dp(h3))
    if nb3 < 0:
        raise ValueError("oracle3d: q must be 19 or 27")
    return e[:q], w[:q], opp[:q], h3[:q * nb3].reshape(q, nb3)
