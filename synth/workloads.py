"""Problem set-ups of the paper's benchmarks, in lattice units, with seeded draws.

Every quantity here is either a grid/boundary description, a dimensionless group
converted to lattice units through the definitions of Sec. 2.4 (Re, Wi, beta, Sc, Ma),
or an analytic initial / forcing field that the paper prescribes for a benchmark
(Sec. 4.1 four-roll mill forcing, Sec. 4.2 Poiseuille forcing, Sec. 4.3 inlet profile).
No lattice Boltzmann arithmetic (relaxation times, equilibria, collisions, boundary
schemes) lives here.

Index convention for every 2-D array: ``a[y, x]`` (x fastest), shape ``(ny, nx)``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

# Lattice speed of sound of the D2Q9 velocity set used throughout the paper (Sec. 3.1),
# needed only to turn a Mach number into a characteristic velocity (Sec. 2.5).
C_S = 1.0 / math.sqrt(3.0)


@dataclass
class Problem:
    """One simulation: grid, boundaries, lattice-unit parameters and fields."""

    name: str
    nx: int
    ny: int
    xmode: str  # 'periodic' | 'wall' | 'open' (open: inlet at x = -1, outlet at x = nx)
    ymode: str  # 'periodic' | 'wall' | 'wet' (wet: rows 0 and ny - 1 are wall nodes)
    nu_s: float  # solvent kinematic viscosity (lattice units)
    eta_p: float  # polymer viscosity (rho0 = 1)
    lam: float  # polymer relaxation time lambda
    kappa: float  # centre-of-mass diffusion coefficient
    Lambda_s: float = 0.25
    Lambda_p: float = 1e-6
    Fx: object = 0.0  # float (uniform) or ndarray (ny, nx)
    Fy: object = 0.0
    init: Optional[dict] = None  # rho, ux, uy, axx, axy, ayy arrays (ny, nx) or None
    solid: Optional[np.ndarray] = None  # uint8 (ny, nx): 1 = solid
    circles: list = field(default_factory=list)  # (xc, yc, R)
    inlet: Optional[dict] = None  # ux, axx, axy, ayy arrays of length ny
    steps: int = 0
    precision: str = "fp32"
    meta: dict = field(default_factory=dict)
    # constitutive closure: 'oldroyd_b' (the paper's), 'giesekus' (model_param = alpha),
    # 'lptt' / 'eptt' (linear / exponential Phan-Thien-Tanner, model_param = epsilon),
    # 'fene_p' (model_param = L^2)
    model: str = "oldroyd_b"
    model_param: float = 0.0
    # hydrodynamic scheme on curved (circle) links: 'bouzidi' (linear interpolated
    # bounce-back) or 'ylw' (the curved-wall scheme of the paper's cylinder)
    curved: str = "bouzidi"
    # hydrodynamic open ends (xmode 'open'): 'neqe' (non-equilibrium extrapolation ghosts)
    # or 'nebb' (the first and last columns as wet nodes, the paper's cylinder set-up)
    open_ends: str = "neqe"

    @property
    def nodes(self) -> int:
        return self.nx * self.ny

    def force_arrays(self):
        """Body force as two (ny, nx) float64 arrays."""
        fx = np.broadcast_to(np.asarray(self.Fx, dtype=np.float64), (self.ny, self.nx))
        fy = np.broadcast_to(np.asarray(self.Fy, dtype=np.float64), (self.ny, self.nx))
        return np.ascontiguousarray(fx), np.ascontiguousarray(fy)

    def uniform_force(self) -> bool:
        return np.ndim(self.Fx) == 0 and np.ndim(self.Fy) == 0

    def init_arrays(self):
        """Initial rho, ux, uy, axx, axy, ayy as (ny, nx) float64 arrays."""
        shape = (self.ny, self.nx)
        d = dict(self.init or {})
        out = {}
        for key, default in (("rho", 1.0), ("ux", 0.0), ("uy", 0.0),
                             ("axx", 1.0), ("axy", 0.0), ("ayy", 1.0)):
            v = d.get(key, default)
            out[key] = np.ascontiguousarray(np.broadcast_to(np.asarray(v, np.float64), shape))
        return out

    def fluid_mask(self) -> np.ndarray:
        """Boolean (ny, nx): True where the node is fluid (mask and circles)."""
        m = np.ones((self.ny, self.nx), dtype=bool)
        if self.solid is not None:
            m &= self.solid == 0
        yy, xx = np.mgrid[0:self.ny, 0:self.nx]
        for (xc, yc, r) in self.circles:
            dx = xx.astype(np.float64) - xc
            dy = yy.astype(np.float64) - yc
            m &= ~(dx * dx + dy * dy <= r * r)
        return m

    def with_(self, **kw) -> "Problem":
        d = dict(self.__dict__)
        d.update(kw)
        return Problem(**d)


def lattice_units(Re: float, Wi: float, beta: float, Sc: float, Ma: float, Lc: float):
    """Dimensionless groups of Sec. 2.4-2.5 -> lattice-unit quantities (rho0 = 1).

    Ma = U_c / c_s, Re = U_c L_c / nu_0, beta = nu_s / nu_0, Wi = lambda U_c / L_c,
    Sc = nu_s / kappa, with nu_0 = nu_s + nu_p.
    """
    Uc = Ma * C_S
    nu0 = Uc * Lc / Re
    nu_s = beta * nu0
    eta_p = (1.0 - beta) * nu0
    lam = Wi * Lc / Uc
    kappa = nu_s / Sc
    return dict(Uc=Uc, nu0=nu0, nu_s=nu_s, eta_p=eta_p, lam=lam, kappa=kappa)


def poiseuille(nx=64, ny=32, Re=1.0, Wi=1.0, beta=0.5, Ma=0.1, Sc=1e6,
               Lambda_s=0.25, Lambda_p=1e-6, steps=10000, precision="fp64",
               wet=False) -> Problem:
    """Force-driven plane Poiseuille flow (Sec. 4.2).

    Periodic in x, no-slip walls half a spacing outside rows 0 and ny-1 (channel height
    H = L_c = ny), or with ``wet`` on rows 0 and ny - 1 themselves (wet-node walls,
    H = L_c = ny - 1).  Driving force F_x = 8 (nu_s + nu_p) U_c / L_c^2; start from unit
    density, zero velocity and identity conformation.
    """
    Lc = float(ny - 1 if wet else ny)
    p = lattice_units(Re, Wi, beta, Sc, Ma, Lc)
    Fx = 8.0 * p["nu0"] * p["Uc"] / (Lc * Lc)
    return Problem(
        name=f"poiseuille_{nx}x{ny}_Wi{Wi:g}{'_wet' if wet else ''}", nx=nx, ny=ny,
        xmode="periodic", ymode="wet" if wet else "wall",
        nu_s=p["nu_s"], eta_p=p["eta_p"], lam=p["lam"], kappa=p["kappa"],
        Lambda_s=Lambda_s, Lambda_p=Lambda_p, Fx=Fx, Fy=0.0, steps=steps,
        precision=precision,
        meta=dict(Re=Re, Wi=Wi, beta=beta, Sc=Sc, Ma=Ma, Uc=p["Uc"], Lc=Lc, H=Lc,
                  Tc=Lc / p["Uc"]))


def four_roll_mill(N=512, Re=1.0, Wi=5.0, beta=0.5, Ma=0.01, Sc=1e5, Lambda_s=0.25,
                   Lambda_p=1e-6, steps=20000, precision="fp32", newtonian_start=True,
                   eta_p_override=None) -> Problem:
    """Simplified four-roll mill on the periodic square [0, 2 pi]^2 (Sec. 4.1).

    Grid N x N with period N (x~ = 2 pi x / N), L_c = N / (2 pi).  Force
    F = F0 (-sin x~ cos y~, cos x~ sin y~), F0 = 2 mu_s U_c (2 pi / N)^2.  When
    ``newtonian_start`` the velocity starts from the steady Newtonian field
    U_c (-sin x~ cos y~, cos x~ sin y~); the conformation starts at the identity.
    """
    Lc = N / (2.0 * math.pi)
    p = lattice_units(Re, Wi, beta, Sc, Ma, Lc)
    eta_p = p["eta_p"] if eta_p_override is None else eta_p_override
    k = 2.0 * math.pi / N
    F0 = 2.0 * p["nu_s"] * p["Uc"] * k * k
    xs = k * np.arange(N, dtype=np.float64)
    X, Y = np.meshgrid(xs, xs, indexing="xy")  # X[y, x] = x~, Y[y, x] = y~
    Fx = -F0 * np.sin(X) * np.cos(Y)
    Fy = F0 * np.cos(X) * np.sin(Y)
    init = None
    if newtonian_start:
        init = dict(ux=-p["Uc"] * np.sin(X) * np.cos(Y), uy=p["Uc"] * np.cos(X) * np.sin(Y))
    return Problem(
        name=f"four_roll_{N}_Wi{Wi:g}", nx=N, ny=N, xmode="periodic", ymode="periodic",
        nu_s=p["nu_s"], eta_p=eta_p, lam=p["lam"], kappa=p["kappa"],
        Lambda_s=Lambda_s, Lambda_p=Lambda_p, Fx=Fx, Fy=Fy, init=init, steps=steps,
        precision=precision,
        meta=dict(Re=Re, Wi=Wi, beta=beta, Sc=Sc, Ma=Ma, Uc=p["Uc"], Lc=Lc, F0=F0,
                  Tc=Lc / p["Uc"]))


def cylinder(nx=4096, ny=1024, R=128.0, xc=2048.0, yc=512.0, Wi=1.0, beta=0.59, Re=1.0,
             Ma=0.01, Sc=1e6, Lambda_s=0.25, Lambda_p=2.5e-7, steps=2000,
             precision="fp32", wet=False) -> Problem:
    """Channel flow past a circular cylinder (Sec. 4.3), L_c = R.

    Half-way no-slip walls outside rows 0 and ny-1 (H = ny; with ``wet``, wet-node walls
    on rows 0 and ny - 1, H = ny - 1); inlet column at x = -1 carries the fully developed
    profile u_x = 1.5 * 4 U_c y'(H - y')/H^2 (y' = y + 1/2, wet: y' = y) with the steady
    Oldroyd-B conformation of that shear, A_xy = lambda u', A_xx = 1 + 2 (lambda u')^2,
    A_yy = 1; zero-gradient outlet at x = nx.  The flow starts from the inlet profile
    everywhere (zero inside the cylinder).
    """
    Lc = float(R)
    p = lattice_units(Re, Wi, beta, Sc, Ma, Lc)
    H = float(ny - 1 if wet else ny)
    yp = np.arange(ny, dtype=np.float64) + (0.0 if wet else 0.5)
    Umax_scale = 1.5 * 4.0 * p["Uc"] / (H * H)
    ux_in = Umax_scale * yp * (H - yp)
    dudy = Umax_scale * (H - 2.0 * yp)
    lam = p["lam"]
    axy_in = lam * dudy
    axx_in = 1.0 + 2.0 * (lam * dudy) ** 2
    ayy_in = np.ones(ny)
    prob = Problem(
        name=f"cylinder_{nx}x{ny}_R{R:g}_Wi{Wi:g}", nx=nx, ny=ny, xmode="open",
        ymode="wet" if wet else "wall",
        nu_s=p["nu_s"], eta_p=p["eta_p"], lam=lam, kappa=p["kappa"],
        Lambda_s=Lambda_s, Lambda_p=Lambda_p, Fx=0.0, Fy=0.0, circles=[(xc, yc, R)],
        inlet=dict(ux=ux_in, axx=axx_in, axy=axy_in, ayy=ayy_in), steps=steps,
        precision=precision,
        meta=dict(Re=Re, Wi=Wi, beta=beta, Sc=Sc, Ma=Ma, Uc=p["Uc"], Lc=Lc,
                  Tc=Lc / p["Uc"], blockage=2 * R / H))
    fluid = prob.fluid_mask()
    ux0 = np.where(fluid, ux_in[:, None], 0.0)
    prob.init = dict(ux=ux0, axx=np.where(fluid, axx_in[:, None], 1.0),
                     axy=np.where(fluid, axy_in[:, None], 0.0))
    return prob


def cylinder_channel(R=20, Wi=0.1, beta=0.59, Sc=1e6, Lambda_p=2.5e-7, precision="fp64",
                     steps=0, wet=False) -> Problem:
    """The paper's confined cylinder (Sec. 4.3): a 30R x 4R channel with the cylinder at
    (15R, 2R), i.e. midway between the half-way walls (node coordinates shifted by 1/2;
    with ``wet``, between wet-node walls on rows 0 and 4R, cylinder centre on row 2R),
    L_c = R, Re = 1, Ma = 0.01; inlet, outlet and start as in :func:`cylinder`."""
    R = int(R)
    pr = cylinder(nx=30 * R, ny=4 * R + (1 if wet else 0), R=float(R), xc=15 * R - 0.5,
                  yc=2 * R - (0.0 if wet else 0.5), Wi=Wi, beta=beta, Sc=Sc,
                  Lambda_p=Lambda_p, steps=steps, precision=precision, wet=wet)
    pr.name = f"cylinder_channel_R{R}_Wi{Wi:g}{'_wet' if wet else ''}"
    return pr


def batch_c4(seed=16997, nruns=256, steps=5000, nmin=32, nmax=512):
    """256 independent runs: half Poiseuille, half four-roll mill, uneven sizes.

    Run r is a Poiseuille channel when r < nruns/2, else a four-roll mill.  Its side
    N ~ U{nmin..nmax}, Wi = 10^U(-1, 2), beta ~ U(0.1, 0.9) drawn in that order from
    ``numpy.random.default_rng(seed)``.  Other groups per family as the single-run
    set-ups, with L_c taken from the grid.
    """
    rng = np.random.default_rng(seed)
    runs = []
    for r in range(nruns):
        n = int(rng.integers(nmin, nmax + 1))
        wi = float(10.0 ** rng.uniform(-1.0, 2.0))
        beta = float(rng.uniform(0.1, 0.9))
        if r < nruns // 2:
            pr = poiseuille(nx=n, ny=n, Wi=wi, beta=beta, steps=steps, precision="fp32")
        else:
            pr = four_roll_mill(N=n, Wi=wi, beta=beta, steps=steps, precision="fp32")
        pr.name = f"run{r:03d}_" + pr.name
        runs.append(pr)
    return runs


def smooth_force_perturbation(N, F0, seed, amp=0.1, kmax=4):
    """Seeded smooth periodic field: sum of Fourier modes 1 <= |k| <= kmax, rms ~ amp*F0."""
    rng = np.random.default_rng(seed)
    xs = 2.0 * math.pi * np.arange(N, dtype=np.float64) / N
    X, Y = np.meshgrid(xs, xs, indexing="xy")
    modes = [(kx, ky) for kx in range(0, kmax + 1) for ky in range(-kmax, kmax + 1)
             if 1 <= kx * kx + ky * ky <= kmax * kmax and (kx > 0 or ky > 0)]
    out = []
    for _comp in range(2):
        f = np.zeros((N, N))
        for (kx, ky) in modes:
            a, b = rng.standard_normal(2)
            ph = kx * X + ky * Y
            f += a * np.cos(ph) + b * np.sin(ph)
        f *= amp * F0 / math.sqrt(len(modes))
        out.append(f)
    return out[0], out[1]


def adjoint_c5(seed=16998, N=512, steps=2000, Wi=5.0, beta=0.5, precision="fp32"):
    """Adjoint workload: four-roll mill plus a hidden target.

    Returns ``(problem, target)`` where ``target`` holds lambda* = lambda (1 + 0.2 xi1),
    eta_p* = eta_p (1 + 0.2 xi2) with xi ~ U(-1, 1), and the force F* = F + dF with dF a
    seeded smooth field of amplitude 0.1 F0, all drawn from default_rng(seed).
    """
    pr = four_roll_mill(N=N, Wi=Wi, beta=beta, steps=steps, precision=precision)
    rng = np.random.default_rng(seed)
    xi1, xi2 = rng.uniform(-1.0, 1.0, size=2)
    dfx, dfy = smooth_force_perturbation(N, pr.meta["F0"], int(rng.integers(1 << 31)))
    target = dict(lam=pr.lam * (1.0 + 0.2 * xi1), eta_p=pr.eta_p * (1.0 + 0.2 * xi2),
                  Fx=pr.Fx + dfx, Fy=pr.Fy + dfy)
    return pr, target


def rest_state(nx=24, ny=16, xmode="periodic", ymode="wall", circles=(), solid=None,
               nu_s=0.1, eta_p=0.1, lam=50.0, kappa=1e-3) -> Problem:
    """Fluid at rest: rho = 1, u = 0, F = 0, A = I (any grid and wall set)."""
    return Problem(name="rest", nx=nx, ny=ny, xmode=xmode, ymode=ymode, nu_s=nu_s,
                   eta_p=eta_p, lam=lam, kappa=kappa, circles=list(circles), solid=solid,
                   steps=0, precision="fp64")


def random_periodic(nx, ny, seed, amp_u=0.02, amp_rho=0.01, amp_a=0.2, xmode="periodic",
                    ymode="periodic", nu_s=0.1, eta_p=0.07, lam=40.0, kappa=0.02,
                    Lambda_s=0.25, Lambda_p=0.05, force_amp=1e-4, solid=None,
                    circles=(), steps=0, precision="fp64") -> Problem:
    """Seeded random smooth-ish state for parity and invariant checks.

    Density, velocity and a symmetric positive-definite conformation are drawn
    node by node from ``default_rng(seed)``; a per-node body force of amplitude
    ``force_amp`` is drawn as well.
    """
    rng = np.random.default_rng(seed)
    shape = (ny, nx)
    rho = 1.0 + amp_rho * rng.uniform(-1, 1, shape)
    ux = amp_u * rng.uniform(-1, 1, shape)
    uy = amp_u * rng.uniform(-1, 1, shape)
    l1 = 1.0 + amp_a * rng.uniform(-1, 1, shape)
    l2 = 1.0 + amp_a * rng.uniform(-1, 1, shape)
    th = rng.uniform(0, math.pi, shape)
    c, s = np.cos(th), np.sin(th)
    axx = l1 * c * c + l2 * s * s
    ayy = l1 * s * s + l2 * c * c
    axy = (l1 - l2) * c * s
    fx = force_amp * rng.uniform(-1, 1, shape)
    fy = force_amp * rng.uniform(-1, 1, shape)
    pr = Problem(name=f"random_{nx}x{ny}_s{seed}", nx=nx, ny=ny, xmode=xmode, ymode=ymode,
                 nu_s=nu_s, eta_p=eta_p, lam=lam, kappa=kappa, Lambda_s=Lambda_s,
                 Lambda_p=Lambda_p, Fx=fx, Fy=fy, solid=solid, circles=list(circles),
                 steps=steps, precision=precision)
    fluid = pr.fluid_mask()
    pr.init = dict(rho=np.where(fluid, rho, 1.0), ux=np.where(fluid, ux, 0.0),
                   uy=np.where(fluid, uy, 0.0), axx=np.where(fluid, axx, 1.0),
                   axy=np.where(fluid, axy, 0.0), ayy=np.where(fluid, ayy, 1.0))
    if xmode == "open":
        yp = np.arange(ny) + 0.5
        pr.inlet = dict(ux=0.02 * 4 * yp * (ny - yp) / ny ** 2, axx=1.0 + 0.1 * np.sin(yp),
                        axy=0.05 * np.cos(yp), ayy=np.ones(ny))
    return pr


def waves(kind, n=64, amp=1e-3, nu_s=0.1, kappa=0.1, lam=1e12, eta_p=0.0, U=0.0,
          Lambda_s=0.25, Lambda_p=0.25, mode=1) -> Problem:
    """Single-mode periodic set-ups for transport-coefficient checks.

    kind='shear': u_y = amp sin(k x) on a uniform background u_x = U (n x 4 grid);
    kind='conformation': A_xx = 1 + amp sin(k x) at rest (n x 4 grid);
    kind='sound': rho = 1 + amp sin(k x), background u_x = U (n x 4 grid).
    """
    k = 2.0 * math.pi * mode / n
    x = np.arange(n, dtype=np.float64)
    shape = (4, n)
    s = np.broadcast_to(np.sin(k * x), shape)
    init = dict(ux=np.full(shape, U))
    if kind == "shear":
        init["uy"] = amp * s
    elif kind == "conformation":
        init["axx"] = 1.0 + amp * s
    elif kind == "sound":
        init["rho"] = 1.0 + amp * s
    else:
        raise ValueError(kind)
    return Problem(name=f"wave_{kind}", nx=n, ny=4, xmode="periodic", ymode="periodic",
                   nu_s=nu_s, eta_p=eta_p, lam=lam, kappa=kappa, Lambda_s=Lambda_s,
                   Lambda_p=Lambda_p, init={k2: np.ascontiguousarray(v) for k2, v in init.items()},
                   precision="fp64", meta=dict(k=k))


# ------------------------------------------------------------------------------------
# Three-dimensional (D3Q19) problems
# ------------------------------------------------------------------------------------
@dataclass
class Problem3D:
    """One three-dimensional simulation: x and z periodic, y periodic or bounded by
    half-way walls; uniform body force; fields indexed [z][y][x]."""

    name: str
    nx: int
    ny: int
    nz: int
    ymode: str  # 'periodic' | 'wall'
    nu_s: float
    eta_p: float
    lam: float
    kappa: float
    Lambda_s: float = 0.25
    Lambda_p: float = 1e-6
    F: tuple = (0.0, 0.0, 0.0)
    init: Optional[dict] = None  # rho, ux, uy, uz, axx, axy, axz, ayy, ayz, azz
    steps: int = 0
    precision: str = "fp32"
    meta: dict = field(default_factory=dict)
    q: int = 19  # lattice: 19 (D3Q19) or 27 (D3Q27)
    solid: Optional[np.ndarray] = None  # [nz][ny][nx] uint8, 1 = solid node
    model: str = "oldroyd_b"  # constitutive closure, as for Problem (FENE-P: L^2 > 3)
    model_param: float = 0.0

    @property
    def nodes(self) -> int:
        return self.nx * self.ny * self.nz

    def init_arrays(self):
        shape = (self.nz, self.ny, self.nx)
        d = dict(self.init or {})
        out = {}
        for key, default in (("rho", 1.0), ("ux", 0.0), ("uy", 0.0), ("uz", 0.0),
                             ("axx", 1.0), ("axy", 0.0), ("axz", 0.0), ("ayy", 1.0),
                             ("ayz", 0.0), ("azz", 1.0)):
            v = d.get(key, default)
            out[key] = np.ascontiguousarray(np.broadcast_to(np.asarray(v, np.float64), shape))
        return out

    def with_(self, **kw) -> "Problem3D":
        d = dict(self.__dict__)
        d.update(kw)
        return Problem3D(**d)


def random3d(nx, ny, nz, seed, ymode="periodic", amp_u=0.02, amp_rho=0.01, amp_a=0.2,
             nu_s=0.1, eta_p=0.07, lam=40.0, kappa=0.02, Lambda_s=0.25, Lambda_p=0.05,
             F=(1e-5, -2e-5, 1.5e-5), precision="fp64", q=19) -> Problem3D:
    """Seeded random state: density, velocity and a symmetric positive-definite
    conformation (A = R diag(l) R^T with a random rotation R and eigenvalues l drawn near
    1) node by node from default_rng(seed)."""
    rng = np.random.default_rng(seed)
    shape = (nz, ny, nx)
    rho = 1.0 + amp_rho * rng.uniform(-1, 1, shape)
    u = [amp_u * rng.uniform(-1, 1, shape) for _ in range(3)]
    lam_e = 1.0 + amp_a * rng.uniform(-1, 1, shape + (3,))
    M = rng.normal(size=shape + (3, 3))
    Qm, _ = np.linalg.qr(M)
    A = np.einsum("...ij,...j,...kj->...ik", Qm, lam_e, Qm)
    init = dict(rho=rho, ux=u[0], uy=u[1], uz=u[2], axx=A[..., 0, 0], axy=A[..., 0, 1],
                axz=A[..., 0, 2], ayy=A[..., 1, 1], ayz=A[..., 1, 2], azz=A[..., 2, 2])
    init = {k: np.ascontiguousarray(v) for k, v in init.items()}
    return Problem3D(name=f"random3d_q{q}_{nx}x{ny}x{nz}_s{seed}", nx=nx, ny=ny, nz=nz, ymode=ymode,
                     nu_s=nu_s, eta_p=eta_p, lam=lam, kappa=kappa, Lambda_s=Lambda_s,
                     Lambda_p=Lambda_p, F=tuple(F), init=init, precision=precision, q=q)


def channel3d(nx=4, ny=32, nz=4, Re=1.0, Wi=1.0, beta=0.5, Ma=0.1, Sc=1e6, Lambda_s=0.25,
              Lambda_p=1e-6, axis="x", steps=10000, precision="fp64", q=19) -> Problem3D:
    """Force-driven plane Poiseuille flow between half-way walls normal to y (the
    channel of Sec. 4.2 with a third, periodic direction), driven along x or z:
    H = L_c = ny, F = 8 (nu_s + nu_p) U_c / L_c^2, start from rest with A = I."""
    Lc = float(ny)
    p = lattice_units(Re, Wi, beta, Sc, Ma, Lc)
    Fm = 8.0 * p["nu0"] * p["Uc"] / (Lc * Lc)
    F = (Fm, 0.0, 0.0) if axis == "x" else (0.0, 0.0, Fm)
    return Problem3D(name=f"channel3d_q{q}_{nx}x{ny}x{nz}_{axis}_Wi{Wi:g}", nx=nx, ny=ny, nz=nz,
                     ymode="wall", nu_s=p["nu_s"], eta_p=p["eta_p"], lam=p["lam"],
                     kappa=p["kappa"], Lambda_s=Lambda_s, Lambda_p=Lambda_p, F=F, steps=steps,
                     precision=precision, q=q,
                     meta=dict(Re=Re, Wi=Wi, beta=beta, Sc=Sc, Ma=Ma, Uc=p["Uc"], Lc=Lc, H=Lc,
                               Tc=Lc / p["Uc"]))
