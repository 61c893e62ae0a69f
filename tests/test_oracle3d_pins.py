"""Pins of the three-dimensional (D3Q19 and D3Q27) oracle (test infrastructure) against facts that
do not come from the oracle itself: lattice quadrature identities, the moments its
equilibria must carry, the closed-form steady channel of Sec. 4.2 driven along x and
along z, the viscous decay of a shear wave along z, exact conservation and the rest
state.  Readings of the three-dimensional extension: A32 in the design notes."""
import numpy as np
import pytest

import synth

CS2 = 1.0 / 3.0


@pytest.fixture(scope="module")
def o3():
    import oracle

    oracle.build(force=False)
    oracle.set_threads(min(8, oracle.max_threads()))
    return oracle


def test_d3q19_quadrature_and_third_order_basis(o3):
    """Weights, isotropy to fourth order, opposites; the six third-order combinations
    H_aab -+ H_bcc are orthogonal to each other and to orders 0-2 on the lattice, with
    norms 2 c_s^6 and 6 c_s^6 (the continuous norm would be 4 c_s^6 for both)."""
    e, w, opp, h3 = o3.lattice3d()
    assert abs(w.sum() - 1) < 1e-15
    assert sorted(np.round(w * 36).astype(int).tolist()) == [1] * 12 + [2] * 6 + [12]
    d = np.eye(3)
    m2 = np.einsum("i,ia,ib->ab", w, e, e)
    assert np.allclose(m2, CS2 * d, atol=1e-15)
    m4 = np.einsum("i,ia,ib,ic,id->abcd", w, e, e, e, e)
    iso = CS2 ** 2 * (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
                      + np.einsum("ad,bc->abcd", d, d))
    assert np.allclose(m4, iso, atol=1e-15)
    assert np.array_equal(e[opp], -e)
    # third-order combinations: explicit formula from the Hermite polynomials
    def H3(a, b, c):
        return (e[:, a] * e[:, b] * e[:, c]
                - CS2 * (e[:, a] * d[b, c] + e[:, b] * d[a, c] + e[:, c] * d[a, b]))
    X, Y, Z = 0, 1, 2
    ref = np.stack([H3(X, X, Y) + H3(Y, Z, Z), H3(X, X, Y) - H3(Y, Z, Z),
                    H3(Z, Z, X) + H3(X, Y, Y), H3(Z, Z, X) - H3(X, Y, Y),
                    H3(Y, Y, Z) + H3(Z, X, X), H3(Y, Y, Z) - H3(Z, X, X)], axis=1)
    assert np.allclose(h3, ref, atol=1e-15)
    G = np.einsum("i,ip,iq->pq", w, h3, h3)
    assert np.allclose(G, np.diag([2, 6, 2, 6, 2, 6]) * CS2 ** 3, atol=1e-15)
    low = np.column_stack([np.ones(19), e, np.einsum("ia,ib->iab", e, e).reshape(19, 9)])
    assert np.abs(np.einsum("i,ip,iq->pq", w, h3, low)).max() < 1e-15


def test_d3q27_quadrature_and_third_order_basis(o3):
    """D3Q27 is the tensor product of D1Q3: weights 8/27, 2/27, 1/54, 1/216 (1, 6, 12 and
    8 velocities), isotropy to fourth order, opposites; H_aaa vanishes at every velocity;
    the seven third-order polynomials H_aab (a != b) and H_xyz are orthogonal to each
    other and to orders 0-2 with their continuous norms 2 c_s^6 and c_s^6."""
    e, w, opp, h3 = o3.lattice3d(27)
    assert e.shape == (27, 3) and h3.shape == (27, 7)
    assert abs(w.sum() - 1) < 1e-15
    assert sorted(np.round(w * 216).astype(int).tolist()) == [1] * 8 + [4] * 12 + [16] * 6 + [64]
    n2 = (e * e).sum(1)
    for k, wk in ((0, 8 / 27), (1, 2 / 27), (2, 1 / 54), (3, 1 / 216)):
        assert np.allclose(w[n2 == k], wk, rtol=0, atol=1e-16)
    d = np.eye(3)
    assert np.allclose(np.einsum("i,ia,ib->ab", w, e, e), CS2 * d, atol=1e-15)
    m4 = np.einsum("i,ia,ib,ic,id->abcd", w, e, e, e, e)
    iso = CS2 ** 2 * (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
                      + np.einsum("ad,bc->abcd", d, d))
    assert np.allclose(m4, iso, atol=1e-15)
    assert np.array_equal(e[opp], -e)

    def H3(a, b, c):
        return (e[:, a] * e[:, b] * e[:, c]
                - CS2 * (e[:, a] * d[b, c] + e[:, b] * d[a, c] + e[:, c] * d[a, b]))
    for a in range(3):
        assert np.abs(H3(a, a, a)).max() < 1e-15
    ref = np.stack([H3(0, 0, 1), H3(0, 0, 2), H3(1, 1, 0), H3(1, 1, 2), H3(2, 2, 0),
                    H3(2, 2, 1), H3(0, 1, 2)], axis=1)
    assert np.allclose(h3, ref, atol=1e-15)
    G = np.einsum("i,ip,iq->pq", w, h3, h3)
    assert np.allclose(G, np.diag([2, 2, 2, 2, 2, 2, 1]) * CS2 ** 3, atol=1e-15)
    low = np.column_stack([np.ones(27), e, np.einsum("ia,ib->iab", e, e).reshape(27, 9)])
    assert np.abs(np.einsum("i,ip,iq->pq", w, h3, low)).max() < 1e-15


def _channel(o3, ny, axis, q):
    pr = synth.channel3d(ny=ny, axis=axis, Ma=0.1, q=q)
    o = o3.OracleSim3D(pr)
    o.step(int(round(30 * pr.meta["Tc"])))
    return pr, o.read()


def _gre(a, b):
    return float(np.sqrt(((a - b) ** 2).sum() / (b ** 2).sum()))


@pytest.mark.parametrize("q", [19, 27])
def test_channel_closed_form_along_x_and_z(o3, q):
    """Force-driven Oldroyd-B channel between half-way walls normal to y (Wi = 1,
    beta = 0.5, Sc = 1e6; 30 T_c): the closed form u = 4 U y (H - y) / H^2,
    A_xy = lambda u', A_xx = 1 + 2 (lambda u')^2, every other component at rest, at
    second order in H for u; the same channel driven along z is the same solution with
    x and z exchanged, to round-off."""
    err = {}
    for ny in (16, 32):
        res = {}
        for axis in ("x", "z"):
            pr, r = _channel(o3, ny, axis, q)
            res[axis] = r
        rx, rz = res["x"], res["z"]
        for a, b in (("ux", "uz"), ("uz", "ux"), ("uy", "uy"), ("axy", "ayz"), ("axx", "azz"),
                     ("azz", "axx"), ("axz", "axz"), ("ayy", "ayy"), ("rho", "rho")):
            assert np.abs(rx[a] - rz[b]).max() < 1e-11, (a, b)
        y = np.arange(ny) + 0.5
        lam, Uc = pr.lam, pr.meta["Uc"]
        ex_u = 4 * Uc * y * (ny - y) / ny ** 2
        du = 4 * Uc * (ny - 2 * y) / ny ** 2
        err[ny] = (_gre(rx["ux"][0, :, 0], ex_u), _gre(rx["axy"][0, :, 0], lam * du),
                   _gre(rx["axx"][0, :, 0] - 1, 2 * (lam * du) ** 2))
        # x-invariant, z-invariant, no transverse flow, the untouched components at rest
        assert np.ptp(rx["ux"], axis=(0, 2)).max() < 1e-12
        assert np.abs(rx["uy"]).max() < 1e-12 and np.abs(rx["uz"]).max() < 1e-12
        for c, one in (("axz", 0.0), ("ayz", 0.0), ("azz", 1.0)):
            assert np.abs(rx[c] - one).max() < 1e-11, c
    assert err[32][0] < 1e-3 and err[16][0] / err[32][0] > 3.5, err
    assert err[32][1] < 6e-3 and err[32][2] < 1.5e-2, err
    assert all(a / b > 2.3 for a, b in zip(err[16], err[32])), err


def _wave(o3, eta, q, N=32, nu=0.05, lam=1.0, U=1e-4, steps=400):
    pr = synth.Problem3D(name="wave_z", nx=4, ny=4, nz=N, ymode="periodic", nu_s=nu, q=q,
                         eta_p=eta, lam=lam, kappa=0.05, Lambda_s=0.25, Lambda_p=0.25)
    z = np.indices((N, 4, 4))[0].astype(float)
    k = 2 * np.pi / N
    s = np.sin(k * z)
    pr.init = {"ux": U * s}
    o = o3.OracleSim3D(pr)
    amp = []
    for _ in range(2):
        o.step(steps)
        amp.append((o.read()["ux"] * s).sum() / (s * s).sum())
    return np.log(amp[0] / amp[1]) / steps / k ** 2


@pytest.mark.parametrize("q", [19, 27])
def test_shear_wave_along_z_decays_viscously(o3, q):
    """u_x = U sin(k z) decays at nu k^2: with the solvent alone nu = nu_s (0.3 % at
    N = 32), and with a polymer that relaxes fast against the decay (lambda = 1 step,
    decay time 260 steps) at nu_s + eta_p (0.7 %): the z components of the velocity
    gradient, the source and the polymer stress all take part."""
    nu0 = _wave(o3, 0.0, q)
    assert abs(nu0 / 0.05 - 1) < 5e-3, nu0
    nu1 = _wave(o3, 0.05, q)
    assert abs(nu1 / 0.10 - 1) < 1.5e-2, nu1


@pytest.mark.parametrize("q", [19, 27])
@pytest.mark.parametrize("ymode", ["periodic", "wall"])
def test_mass_and_conformation_budget_exact(o3, ymode, q):
    """Total mass exact (periodic streaming, half-way walls); with the constitutive source
    off every conformation component's total is exact too (CNEBB at the walls, Sec. 3.3)."""
    pr = synth.random3d(10, 8, 6, seed=4, ymode=ymode, q=q)
    o = o3.OracleSim3D(pr, no_source=True)
    r0 = o.read()
    o.step(30)
    r1 = o.read()
    assert abs(r1["rho"].sum() / r0["rho"].sum() - 1) < 1e-13
    for c in ("axx", "axy", "axz", "ayy", "ayz", "azz"):
        assert abs(r1[c].sum() - r0[c].sum()) < 1e-12 * np.abs(r0[c]).sum(), c


@pytest.mark.parametrize("q", [19, 27])
def test_rest_state_is_exact(o3, q):
    """rho = 1, u = 0, A = I, no force: every step leaves it unchanged (walls included)."""
    pr = synth.Problem3D(name="rest", nx=6, ny=7, nz=5, ymode="wall", nu_s=0.1, eta_p=0.1, q=q,
                         lam=50.0, kappa=1e-3)
    o = o3.OracleSim3D(pr)
    o.step(40)
    r = o.read()
    assert np.abs(r["rho"] - 1).max() < 1e-14
    for c in ("ux", "uy", "uz", "axy", "axz", "ayz"):
        assert np.abs(r[c]).max() < 1e-14, c
    for c in ("axx", "ayy", "azz"):
        assert np.abs(r[c] - 1).max() < 1e-14, c


@pytest.mark.parametrize("q", [19, 27])
def test_collision_relaxes_each_hermite_order_and_drops_the_rest(o3, q):
    """Per-node check of the hydrodynamic TRT regularized collision (Sec. 3.1) at fixed
    rho and u: a non-equilibrium perturbation along a second-order Hermite direction comes
    out scaled by 1 - 1/tau_s1, one along each third-order basis function of the lattice
    by 1 - 1/tau_s2, and one orthogonal (in the lattice's weighted inner product) to every
    Hermite polynomial up to third order is removed.  Catches a basis function left out
    of the third-order projection (H_xyz on D3Q27, say), a wrong norm, the two relaxation
    times exchanged, and an unregularized collision."""
    e, w, opp, h3 = o3.lattice3d(q)
    ef = e.astype(float)
    rho, u = 1.02, np.array([0.03, -0.02, 0.015])
    f0 = w * (1.0 + 0.05 * ef[:, 0] - 0.02 * ef[:, 2])  # any state: rho, u are inputs
    ts1, ts2 = 0.7, 0.8
    c1, c2 = 1 - 1 / ts1, 1 - 1 / ts2
    base = o3.collide_hydro3d(q, f0, rho, u, tau_s1=ts1, tau_s2=ts2)

    def resp(d):
        return o3.collide_hydro3d(q, f0 + d, rho, u, tau_s1=ts1, tau_s2=ts2) - base

    def H2(a, b):
        return ef[:, a] * ef[:, b] - CS2 * (a == b)

    eps = 1e-3
    tol = 1e-12 * eps
    for d in (w * H2(0, 1), w * H2(1, 2), w * (H2(0, 0) - H2(1, 1)), w * (H2(0, 0) + H2(1, 1) + H2(2, 2))):
        assert np.abs(resp(eps * d) - c1 * eps * d).max() < tol
    for m in range(h3.shape[1]):
        d = eps * w * h3[:, m]
        assert np.abs(d).max() > 1e-6
        assert np.abs(resp(d) - c2 * d).max() < tol, m
    # the content beyond third order: a random vector made orthogonal to 1, e, H2, h3
    B = np.column_stack([np.ones(q), ef] + [H2(a, b) for a in range(3) for b in range(a, 3)]
                        + [h3])
    v = np.random.default_rng(3).normal(size=q)
    coef = np.linalg.solve(B.T @ (w[:, None] * B), B.T @ (w * v))
    g = eps * w * (v - B @ coef)
    assert np.abs(g).max() > 1e-6
    assert np.abs(resp(g)).max() < tol


@pytest.mark.parametrize("q", [19, 27])
def test_conformation_collision_relaxes_orders_one_and_two(o3, q):
    """Per-node check of the convection-diffusion TRT regularized collision (Sec. 3.2) at
    fixed phi, rho and u without source: a non-equilibrium perturbation along e_a comes out
    scaled by 1 - 1/tau_p1, one along a second-order Hermite direction by 1 - 1/tau_p2,
    and anything orthogonal to orders 0-2 is removed; the source enters the zeroth moment
    as 1.5 S - 0.5 S_prev.  Catches the two relaxation times exchanged, an unregularized
    collision and a wrong source time difference."""
    e, w, opp, h3 = o3.lattice3d(q)
    ef = e.astype(float)
    phi, rho, u = 1.3, 1.01, np.array([0.02, 0.01, -0.03])
    g0 = w * (1.2 + 0.04 * ef[:, 1])
    tp1, tp2 = 0.75, 0.6
    c1, c2 = 1 - 1 / tp1, 1 - 1 / tp2
    base = o3.collide_cde3d(q, g0, phi, rho, u, tau_p1=tp1, tau_p2=tp2)

    def resp(d):
        return o3.collide_cde3d(q, g0 + d, phi, rho, u, tau_p1=tp1, tau_p2=tp2) - base

    def H2(a, b):
        return ef[:, a] * ef[:, b] - CS2 * (a == b)

    eps = 1e-3
    tol = 1e-12 * eps
    for a in range(3):
        d = eps * w * ef[:, a]
        assert np.abs(resp(d) - c1 * d).max() < tol, a
    for d in (w * H2(0, 2), w * (H2(1, 1) - H2(2, 2)), w * (H2(0, 0) + H2(1, 1) + H2(2, 2))):
        assert np.abs(resp(eps * d) - c2 * eps * d).max() < tol
    B = np.column_stack([np.ones(q), ef] + [H2(a, b) for a in range(3) for b in range(a, 3)])
    v = np.random.default_rng(5).normal(size=q)
    coef = np.linalg.solve(B.T @ (w[:, None] * B), B.T @ (w * v))
    g = eps * w * (v - B @ coef)
    assert np.abs(g).max() > 1e-6
    assert np.abs(resp(g)).max() < tol
    # source: the zeroth moment of the output grows by 1.5 S - 0.5 S_prev
    S, Sp = 2e-3, 5e-4
    out = o3.collide_cde3d(q, g0, phi, rho, u, S=S, Sp=Sp, tau_p1=tp1, tau_p2=tp2)
    assert abs((out - base).sum() - (1.5 * S - 0.5 * Sp)) < 1e-15


def test_source_vanishes_on_the_steady_states_of_three_dimensional_flows(o3):
    """The constitutive source (Sec. 3.2, Oldroyd-B with every index over x, y, z) is zero
    on the closed-form steady conformations: uniaxial extension u = e (x, -y/2, -z/2),
    A = diag(1/(1 - 2 Wi), 1/(1 + Wi), 1/(1 + Wi)) with Wi = lambda e; simple shear
    u_x = g z in the x-z plane, A_xz = lambda g, A_xx = 1 + 2 (lambda g)^2; and A = I
    under a rigid rotation.  A uniform dilation L = d I at A = I gives (2 + 3) d I (the
    upper-convected terms and A tr L).  Catches a transposed gradient, a dropped or
    doubled upper-convected term, a wrong z index and the A tr L term left out."""
    lam = 3.0
    for e in (0.02, -0.05, 0.1):
        L = np.diag([e, -e / 2, -e / 2])
        Wi = lam * e
        A = np.diag([1 / (1 - 2 * Wi), 1 / (1 + Wi), 1 / (1 + Wi)])
        assert np.abs(o3.source3d(A, L, lam)).max() < 1e-15, e
    for g in (0.01, 0.2):
        L = np.zeros((3, 3))
        L[2, 0] = g  # d_z u_x
        A = np.eye(3)
        A[0, 2] = A[2, 0] = lam * g
        A[0, 0] = 1 + 2 * (lam * g) ** 2
        assert np.abs(o3.source3d(A, L, lam)).max() < 1e-15, g
        # the transposed arrangement (u_z = g x) is a different flow: not steady here
        assert np.abs(o3.source3d(A, L.T, lam)).max() > 1e-3 * g
    W = np.array([[0.0, 0.03, -0.02], [-0.03, 0.0, 0.05], [0.02, -0.05, 0.0]])
    assert np.abs(o3.source3d(np.eye(3), W, lam)).max() < 1e-16
    d = 0.01
    assert np.abs(o3.source3d(np.eye(3), d * np.eye(3), lam) - 5 * d * np.eye(3)).max() < 1e-16


def _sound_decay_z(o3, U, q, n=64, steps=600):
    """Damping rate of a sound wave along z in a frame moving at U along z."""
    pr = synth.Problem3D(name="sound_z", nx=2, ny=2, nz=n, ymode="periodic", nu_s=0.05,
                         eta_p=0.0, lam=1.0, kappa=0.05, Lambda_s=0.25, Lambda_p=0.25, q=q)
    k = 2 * np.pi / n
    z = np.arange(n)
    shape = (n, 2, 2)
    rho = 1.0 + 1e-4 * np.cos(k * z)[:, None, None] * np.ones(shape)
    pr.init = {"rho": rho, "uz": np.full(shape, U)}
    o = o3.OracleSim3D(pr)
    E = []
    for _ in range(steps):
        r = o.read()
        a = ((r["rho"][:, 0, 0] - 1) * np.exp(-1j * k * z)).sum()
        b = ((r["uz"][:, 0, 0] - U) * np.exp(-1j * k * z)).sum()
        E.append(abs(a) ** 2 / 3 + abs(b) ** 2)
        o.step(1)
    t = np.arange(steps)
    return -np.polyfit(t[100:], np.log(np.array(E)[100:]), 1)[0] / 2


@pytest.mark.parametrize("q", [19, 27])
def test_galilean_invariant_sound_damping_along_z(o3, q):
    """Acoustic damping along z is the same in a frame moving at U = 0.1 along z (Sec. 3.1,
    G_i): neither lattice's equilibrium carries rho u_z^3, and the correction G_i, with
    the defect d_z(rho u_z^3) differenced along z, removes that error from the viscous
    stress.  Catches a dropped or mis-indexed z component of G_i and a wrong sign."""
    r0 = _sound_decay_z(o3, 0.0, q)
    r1 = _sound_decay_z(o3, 0.1, q)
    assert r0 > 0
    assert abs(r1 / r0 - 1) < 5e-3, (r0, r1)


def _mask_channel(o3, q, H=16, steps=2000, axis="y"):
    """The Oldroyd-B channel driven along x between walls normal to `axis`: half-way walls
    of the domain (axis y) or two planes of solid nodes (axis z)."""
    base = synth.channel3d(nx=4, ny=H, nz=4, Ma=0.1, q=q)
    if axis == "y":
        pr = base
    else:
        solid = np.zeros((H + 2, 4, 4), np.uint8)
        solid[0] = solid[-1] = 1
        pr = base.with_(ny=4, nz=H + 2, ymode="periodic", solid=solid)
    o = o3.OracleSim3D(pr)
    o.step(steps)
    return o.read()


@pytest.mark.parametrize("q", [19, 27])
def test_solid_planes_act_as_the_walls(o3, q):
    """Two planes of solid nodes normal to z bound the same channel as the half-way walls
    normal to y (half-way bounce-back at the solid faces, CNEBB at the adjacent nodes,
    the wall rule of the differences): after 2,000 steps of the Oldroyd-B channel the two
    agree with y and z exchanged, to round-off.  Catches a solid neighbour missed by the
    pull, by CNEBB or by the differences."""
    ry = _mask_channel(o3, q, axis="y")
    rz = _mask_channel(o3, q, axis="z")
    pairs = (("ux", "ux"), ("uy", "uz"), ("uz", "uy"), ("axx", "axx"), ("axy", "axz"),
             ("axz", "axy"), ("ayy", "azz"), ("azz", "ayy"), ("ayz", "ayz"), ("rho", "rho"))
    for a, b in pairs:
        fy = ry[a][0, :, 0]                # [z][y][x] -> profile along y
        fz = rz[b][1:-1, 0, 0]             # fluid rows along z
        assert np.abs(fy - fz).max() < 1e-11 * max(1.0, np.abs(fy).max()), (a, b)
    assert np.abs(rz["ux"][0]).max() == 0.0 and np.all(rz["axx"][-1] == 1.0)  # solid: at rest


def _duct_series(H, F, mu, n_terms=60):
    """Steady Poiseuille flow in the square duct 0 < y, z < H: u, du/dy, du/dz at the
    node centres (the classical Fourier series, terms n = 1, 3, 5, ...)."""
    a = H / 2.0
    c = (np.arange(H) + 0.5) - a
    Y, Z = np.meshgrid(c, c, indexing="ij")
    u = np.zeros_like(Y)
    uy = np.zeros_like(Y)
    uz = np.zeros_like(Y)
    for m in range(n_terms):
        n = 2 * m + 1
        kk = n * np.pi / (2 * a)
        s = (-1) ** m / n ** 3
        ch = np.cosh(kk * Z) / np.cosh(kk * a)
        u += s * (1 - ch) * np.cos(kk * Y)
        uy += s * (1 - ch) * (-kk) * np.sin(kk * Y)
        uz += s * (-kk * np.sinh(kk * Z) / np.cosh(kk * a)) * np.cos(kk * Y)
    pref = 16 * a * a * F / (mu * np.pi ** 3)
    return pref * u, pref * uy, pref * uz  # indexed [y][z]


@pytest.mark.parametrize("q", [19, 27])
def test_square_duct_oldroyd_b_closed_form(o3, q):
    """Steady Oldroyd-B flow in a square duct (half-way walls normal to y, solid planes
    normal to z; Wi = 1, beta = 0.5): the velocity is the Newtonian duct series with the
    total viscosity, and the conformation A_xy = lambda du/dy, A_xz = lambda du/dz,
    A_xx = 1 + 2 lambda^2 |grad u|^2, with A_yy = A_zz = 1, A_yz = 0 and no secondary flow
    (Oldroyd-B has no second normal-stress difference).  Exercises every term of the 3-D
    source with two shear components at once and the corners where both kinds of wall
    meet.  Measured: the velocity converges at second order (GRE 3.9 % -> 1.4 % from
    H = 12 to 24); the conformation away from the walls (outside H/6 of them) too (A_xy
    1.5 % -> 0.5 %), while next to the walls, where the wall-parallel gradient varies,
    it converges at first order (all nodes: 15 % -> 8 %).  D3Q19 carries a spurious
    secondary flow of 0.3 % -> 0.16 % of the axial peak (its lattice lacks part of the
    isotropy the stress divergence needs); D3Q27 has none."""
    err, sec = {}, {}
    for H in (12, 24):
        base = synth.channel3d(nx=2, ny=H, nz=2, Ma=0.1, q=q)
        solid = np.zeros((H + 2, H, 2), np.uint8)
        solid[0] = solid[-1] = 1
        pr = base.with_(nz=H + 2, solid=solid)
        o = o3.OracleSim3D(pr)
        o.step(int(round(15 * pr.meta["Tc"])))
        r = o.read()
        mu = pr.nu_s + pr.eta_p
        u, uy, uz = _duct_series(H, pr.F[0], mu)
        lam = pr.lam
        g = {k: r[k][1:-1, :, 0].T for k in r}  # fluid [z][y] -> [y][z]
        k = H // 6
        c = (slice(k, -k), slice(k, -k))
        err[H] = (_gre(g["ux"], u), _gre(g["axy"][c], lam * uy[c]), _gre(g["axz"][c], lam * uz[c]),
                  _gre(g["axx"][c] - 1, 2 * lam ** 2 * (uy[c] ** 2 + uz[c] ** 2)))
        sec[H] = max(np.abs(g["uy"]).max(), np.abs(g["uz"]).max()) / u.max()
        axx1 = np.abs(g["axx"] - 1).max()
        for name, one in (("ayy", 1.0), ("azz", 1.0), ("ayz", 0.0)):
            assert np.abs(g[name] - one).max() < 3e-3 * axx1, name
    assert err[24][0] < 2e-2 and max(err[24][1:3]) < 1e-2 and err[24][3] < 1.5e-2, err
    assert all(e12 / e24 > 2.3 for e12, e24 in zip(err[12], err[24])), err
    if q == 27:
        assert max(sec.values()) < 1e-10, sec
    else:
        assert sec[24] < 2e-3 and sec[24] < 0.7 * sec[12], sec


CLOSURES = [("giesekus", 0.3), ("lptt", 0.25), ("eptt", 0.25), ("fene_p", 30.0)]


@pytest.mark.parametrize("model,mp", CLOSURES)
def test_closures_reduce_to_the_planar_ones(o3, model, mp):
    """Reading A28 in three dimensions: on a planar state (A_zz = 1, A_xz = A_yz = 0, an
    in-plane velocity gradient) each closure's 3-D source equals the 2-D oracle's source
    of the same closure (tr A - 3 in 3-D is tr A - 2 in the plane; FENE-P with L^2 - 1 in
    the plane), whose closures the two-dimensional pins tie to Giesekus' steady shear
    solution and the scalar equations of PTT and FENE-P; S_xz, S_yz vanish and (but for
    FENE-P) S_zz is the divergence term tr L.  Also
    the 3-D closures are isotropic: S(R A R^T, R L R^T) = R S(A, L) R^T for a rotation R.
    Catches a wrong trace offset, a transposed or mis-indexed B B and a closure applied
    to the wrong components."""
    rng = np.random.default_rng(11)
    lam = 7.0
    for _ in range(5):
        a = np.array([[1.4, 0.3], [0.3, 0.8]]) + 0.1 * rng.normal(size=(2, 2))
        a = 0.5 * (a + a.T)
        Lp = 0.05 * rng.normal(size=(2, 2))
        A = np.eye(3)
        A[:2, :2] = a
        L = np.zeros((3, 3))
        L[:2, :2] = Lp
        S3 = o3.source3d(A, L, lam, model, mp)
        mp2 = mp - 1.0 if model == "fene_p" else mp
        S2 = o3.node_source(np.array([a[0, 0], a[0, 1], a[1, 1]]),
                            np.array([Lp[0, 0], Lp[0, 1], Lp[1, 0], Lp[1, 1]]), lam, model, mp2)
        assert np.allclose([S3[0, 0], S3[0, 1], S3[1, 1]], S2, rtol=1e-12, atol=1e-15), (S3, S2)
        assert abs(S3[0, 2]) < 1e-15 and abs(S3[1, 2]) < 1e-15
        if model != "fene_p":  # B_zz = 0 leaves only the divergence term A_zz tr L
            assert abs(S3[2, 2] - np.trace(L)) < 1e-15
    # isotropy
    M = rng.normal(size=(3, 3))
    A = np.eye(3) + 0.2 * (M @ M.T) / 3
    L = 0.04 * rng.normal(size=(3, 3))
    Qr, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    S = o3.source3d(A, L, lam, model, mp)
    Sr = o3.source3d(Qr @ A @ Qr.T, Qr @ L @ Qr.T, lam, model, mp)
    assert np.allclose(Sr, Qr @ S @ Qr.T, rtol=1e-11, atol=1e-14)
