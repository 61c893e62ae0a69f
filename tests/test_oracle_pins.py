"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test names the plausible mistakes it is built to catch.  None of them compares the
oracle with itself: they use closed forms stated by the paper (Poiseuille steady state,
Waters-King transient, four-roll steady field, planar-extension conformation), textbook
results of the model equations (Oldroyd-B simple shear, diffusion and viscous decay
rates, Gauss-Hermite quadrature moments), exact invariants of the scheme (mass,
momentum, the conservation property of CNEBB, the rest state, mirror symmetry) and
sensitivity-checked physical effects of single terms (Galilean invariance for G_i,
second-order source integration for the time derivative of F~_i).
"""
import math

import numpy as np
import pytest

import synth
from analytic import (four_roll_newtonian, gre, poiseuille_steady, poiseuille_steady_model,
                      shear_conformation, waters_king_u)

CS2 = 1.0 / 3.0


# ---------------------------------------------------------------------------------
# Lattice and equilibria
# ---------------------------------------------------------------------------------
def test_lattice_tables(oracle_lib):
    """D2Q9 directions in the paper's order, weights, opposites, quadrature moments."""
    ex, ey, opp, w = oracle_lib.lattice()
    assert list(ex) == [0, 1, 0, -1, 0, 1, -1, -1, 1]
    assert list(ey) == [0, 0, 1, 0, -1, 1, 1, -1, -1]
    assert list(opp) == [0, 3, 4, 1, 2, 7, 8, 5, 6]
    np.testing.assert_allclose(w, [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4, rtol=0, atol=1e-16)
    e = np.stack([ex, ey], 1).astype(float)
    assert abs(w.sum() - 1) < 1e-15
    np.testing.assert_allclose(np.einsum("i,ia->a", w, e), 0, atol=1e-16)
    np.testing.assert_allclose(np.einsum("i,ia,ib->ab", w, e, e), CS2 * np.eye(2), atol=1e-16)
    d = np.eye(2)
    m4 = np.einsum("i,ia,ib,ic,id->abcd", w, e, e, e, e)
    iso = CS2 ** 2 * (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
                      + np.einsum("ad,bc->abcd", d, d))
    np.testing.assert_allclose(m4, iso, atol=1e-16)
    # third-order Hermite H_xxx vanishes identically on D2Q9 (e_x^3 = e_x)
    assert np.all(e[:, 0] ** 3 - 3 * CS2 * e[:, 0] == 0)


@pytest.mark.parametrize("rho,ux,uy", [(1.0, 0.0, 0.0), (1.03, 0.07, -0.04), (0.97, -0.1, 0.12)])
def test_equilibrium_moments(oracle_lib, rho, ux, uy):
    """Hermite equilibria reproduce their defining moments (catches wrong coefficients).

    f^eq: density, momentum, momentum flux rho(cs2 I + uu) and the off-diagonal third
    moments rho ux^2 uy, rho ux uy^2; g^eq: phi, phi u, phi(cs2 I + uu).
    """
    ex, ey, _, _ = oracle_lib.lattice()
    f = oracle_lib.node_feq(rho, ux, uy)
    assert abs(f.sum() - rho) < 1e-15
    assert abs((ex * f).sum() - rho * ux) < 1e-15 and abs((ey * f).sum() - rho * uy) < 1e-15
    assert abs((ex * ex * f).sum() - rho * (CS2 + ux * ux)) < 1e-15
    assert abs((ex * ey * f).sum() - rho * ux * uy) < 1e-15
    assert abs((ey * ey * f).sum() - rho * (CS2 + uy * uy)) < 1e-15
    hxxy = (ex * ex - CS2) * ey
    hxyy = (ey * ey - CS2) * ex
    assert abs((hxxy * f).sum() - rho * ux * ux * uy) < 1e-15
    assert abs((hxyy * f).sum() - rho * ux * uy * uy) < 1e-15
    phi = 1.7
    g = oracle_lib.node_geq(phi, ux, uy)
    assert abs(g.sum() - phi) < 1e-15
    assert abs((ex * g).sum() - phi * ux) < 1e-15
    assert abs((ex * ey * g).sum() - phi * ux * uy) < 1e-15
    assert abs((ey * ey * g).sum() - phi * (CS2 + uy * uy)) < 1e-15


def test_collision_invariants(oracle_lib):
    """Per-node conservation of the collisions on random states (pin P5).

    Hydro: mass kept, momentum gains exactly F (catches a zeroed A_alpha, a wrong F_i
    prefactor, mass/momentum leaking from T_i or G_i).  T_i injects -tau/tau_s1 into the
    second moment, so the momentum equation gets +div(tau).  CDE: sum g+ = phi + S +
    (S - S_prev)/2 (catches a wrong F~ or time-difference weight).
    """
    rng = np.random.default_rng(7)
    ex, ey, _, _ = oracle_lib.lattice()
    for _ in range(20):
        f = oracle_lib.node_feq(1 + 0.02 * rng.standard_normal(), 0.05 * rng.standard_normal(),
                                0.05 * rng.standard_normal()) + 1e-3 * rng.standard_normal(9)
        Fx, Fy = 1e-3 * rng.standard_normal(2)
        t1, t2 = rng.uniform(0.51, 2.0, 2)
        tau = 1e-3 * rng.standard_normal(3)
        D = 1e-4 * rng.standard_normal(2)
        out = oracle_lib.node_hydro(f, Fx, Fy, t1, t2, tau, D)
        assert abs(out.sum() - f.sum()) < 1e-14
        assert abs((ex * out).sum() - (ex * f).sum() - Fx) < 1e-14
        assert abs((ey * out).sum() - (ey * f).sum() - Fy) < 1e-14
        # T_i alone: difference of two collisions that differ only in tau
        out0 = oracle_lib.node_hydro(f, Fx, Fy, t1, t2, (0, 0, 0), D)
        dT = out - out0
        assert abs(dT.sum()) < 1e-15 and abs((ex * dT).sum()) < 1e-15
        assert abs((ex * ey * dT).sum() + tau[1] / t1) < 1e-15
        assert abs(((ex * ex - CS2) * dT).sum() + tau[0] / t1) < 1e-15
        # G_i alone: no mass, no momentum; removes (1 - 1/2tau) dPhi from Pi_xx, Pi_yy
        outG = oracle_lib.node_hydro(f, Fx, Fy, t1, t2, tau, (0, 0))
        dG = out - outG
        assert abs(dG.sum()) < 1e-15 and abs((ex * dG).sum()) < 1e-15
        h1 = 1 - 1 / (2 * t1)
        assert abs(((ex * ex - CS2) * dG).sum() + h1 * D[0]) < 1e-15
        g = oracle_lib.node_geq(1.3, 0.03, -0.02) + 1e-3 * rng.standard_normal(9)
        S, Sp = 1e-3 * rng.standard_normal(2)
        p1, p2 = rng.uniform(0.5001, 1.5, 2)
        og = oracle_lib.node_cde(g, 1.01, 0.03, -0.02, Fx, Fy, S, Sp, 0.02, 0.01, p1, p2)
        assert abs(og.sum() - (g.sum() + S + 0.5 * (S - Sp))) < 1e-14


# ---------------------------------------------------------------------------------
# Constitutive source: homogeneous flows with closed-form Oldroyd-B conformations
# ---------------------------------------------------------------------------------
def _steady_A(oracle_lib, L, lam):
    """Solve Phi(A) = 0 for the symmetric A (Phi is affine in A)."""
    b = oracle_lib.node_source([0.0, 0.0, 0.0], L, lam)
    M = np.zeros((3, 3))
    for j in range(3):
        e = np.zeros(3)
        e[j] = 1.0
        M[:, j] = oracle_lib.node_source(e, L, lam) - b
    return np.linalg.solve(M, -b)


def test_source_simple_shear(oracle_lib):
    """u_x = gdot y: A_xy = lam gdot, A_xx = 1 + 2 (lam gdot)^2, A_yy = 1 (Sec. 4.2).

    The transposed flow u_y = gdot x swaps the roles of xx and yy: catches a transposed
    velocity gradient in the upper-convected terms.
    """
    lam, gd = 7.0, 0.13
    A = _steady_A(oracle_lib, [0.0, 0.0, gd, 0.0], lam)  # L = [[Lxx, Lxy], [Lyx, Lyy]]
    np.testing.assert_allclose(A, [1 + 2 * (lam * gd) ** 2, lam * gd, 1.0], rtol=1e-13)
    A = _steady_A(oracle_lib, [0.0, gd, 0.0, 0.0], lam)
    np.testing.assert_allclose(A, [1.0, lam * gd, 1 + 2 * (lam * gd) ** 2], rtol=1e-13)


def test_source_planar_extension(oracle_lib):
    """u = eps (x, -y): A_xx = 1/(1 - 2 Wi_eff), A_yy = 1/(1 + 2 Wi_eff), A_xy = 0.

    These are the stagnation-point values the paper quotes for the four-roll mill
    (Sec. 4.1) with Wi_eff = lambda eps.  A uniform dilation u = eps (x, y) checks the
    A div(u) term: A_xx = A_yy = 1/(1 - 4 lambda eps).
    """
    lam, eps = 3.0, 0.07
    A = _steady_A(oracle_lib, [eps, 0.0, 0.0, -eps], lam)
    np.testing.assert_allclose(A, [1 / (1 - 2 * lam * eps), 0.0, 1 / (1 + 2 * lam * eps)],
                               rtol=1e-13, atol=1e-15)
    A = _steady_A(oracle_lib, [eps, 0.0, 0.0, eps], lam)
    np.testing.assert_allclose(A, [1 / (1 - 4 * lam * eps), 0.0, 1 / (1 - 4 * lam * eps)],
                               rtol=1e-13, atol=1e-15)


MODEL_CASES = [("giesekus", 0.2), ("giesekus", 0.5), ("lptt", 0.25), ("eptt", 0.25),
               ("fene_p", 20.0), ("fene_p", 100.0)]


@pytest.mark.parametrize("model,mp", MODEL_CASES)
def test_source_simple_shear_closures(oracle_lib, model, mp):
    """Other closures through the model function F(A) (Sec. 2.2): the steady conformation
    of simple shear (Giesekus' analytic solution; the PTT and FENE-P scalar equations)
    zeroes the oracle's constitutive source, for both shear directions and several Wi.
    The planar solution of a transposed flow u_y = gdot x swaps xx and yy."""
    lam = 5.0
    for Wi in (0.3, 1.5, -1.5, 4.0):
        gd = Wi / lam
        A = np.array(shear_conformation(model, mp, Wi))
        S = oracle_lib.node_source(A, [0.0, 0.0, gd, 0.0], lam, model, mp)
        assert np.abs(S).max() < 1e-14 * max(1.0, np.abs(A).max()), (Wi, A, S)
        At = A[[2, 1, 0]]
        S = oracle_lib.node_source(At, [0.0, gd, 0.0, 0.0], lam, model, mp)
        assert np.abs(S).max() < 1e-14 * max(1.0, np.abs(A).max()), (Wi, At, S)
        # and it is not the Oldroyd-B state
        assert np.abs(A - shear_conformation("oldroyd_b", 0.0, Wi)).max() > 1e-3


def test_closures_reduce_to_oldroyd_b(oracle_lib):
    """alpha = 0, eps = 0 and L^2 -> infinity give the Oldroyd-B source."""
    rng = np.random.default_rng(4)
    for _ in range(20):
        A = np.array([1.3, 0.2, 0.9]) + 0.1 * rng.standard_normal(3)
        L = 0.05 * rng.standard_normal(4)
        ob = oracle_lib.node_source(A, L, 7.0)
        for model, mp, tol in (("giesekus", 0.0, 0.0), ("lptt", 0.0, 0.0), ("eptt", 0.0, 0.0),
                               ("fene_p", 1e12, 1e-11)):
            S = oracle_lib.node_source(A, L, 7.0, model, mp)
            assert np.abs(S - ob).max() <= tol * np.abs(ob).max(), model


@pytest.mark.parametrize("model,mp", [("giesekus", 0.2), ("lptt", 0.25), ("eptt", 0.25),
                                      ("fene_p", 20.0)])
def test_poiseuille_closures_second_order(oracle_lib, model, mp):
    """Steady channel flow of each closure (Wi = 1, beta = 0.5 as Sec. 4.2) against the
    semi-analytic solution (the local simple-shear stress balances G (H/2 - y)): u and
    A converge at second order from Ny = 16 to 32 to profiles that differ from the
    Oldroyd-B ones by 19-48 % in u."""
    oracle_lib.set_threads(min(8, oracle_lib.max_threads()))
    err = {}
    for ny, steps in ((16, 24000), (32, 40000)):
        pr = synth.poiseuille(nx=4, ny=ny).with_(model=model, model_param=mp)
        ref = poiseuille_steady_model(ny, pr.Fx, pr.nu_s, pr.eta_p, pr.lam, model, mp)
        o = oracle_lib.OracleSim(pr)
        o.step(steps)
        r = o.read()
        err[ny] = (gre(r["ux"][:, 0], ref["ux"]), gre(r["axy"][:, 0], ref["axy"]),
                   gre(r["axx"][:, 0] - 1, ref["axx"] - 1))
    assert err[32][0] < 1.2e-3 and err[32][1] < 2e-3 and err[32][2] < 2.5e-3, err
    assert err[16][0] / err[32][0] > 3.5, err


def test_finite_difference_exact_on_quadratics(oracle_lib):
    """Central and wall-aware derivatives are exact for quadratics vanishing at the wall."""
    rng = np.random.default_rng(3)
    for _ in range(50):
        a, b, c = rng.standard_normal(3)
        p = lambda t: a * t * t + b * t + c  # noqa: E731
        assert abs(oracle_lib.node_fd(0, 0.5, p(-1), p(0), 0, 0.5, p(1)) - b) < 1e-13
        q = rng.uniform(0.05, 1.0)
        # wall at -q: quadratic through (-q, 0)
        pw = lambda t: (t + q) * (a * t + b)  # noqa: E731
        d0 = q * a + b
        assert abs(oracle_lib.node_fd(1, q, 0.0, pw(0), 0, 0.5, pw(1)) - d0) < 1e-12
        pw2 = lambda t: (t - q) * (a * t + b)  # noqa: E731
        d0 = -q * a + b
        assert abs(oracle_lib.node_fd(0, 0.5, pw2(-1), pw2(0), 1, q, 0.0) - d0) < 1e-12
        q2 = rng.uniform(0.05, 1.0)
        pb = lambda t: a * (t + q) * (t - q2)  # noqa: E731
        d0 = a * (q - q2)
        assert abs(oracle_lib.node_fd(1, q, 0.0, pb(0), 1, q2, 0.0) - d0) < 1e-12


# ---------------------------------------------------------------------------------
# Whole-step invariants
# ---------------------------------------------------------------------------------
def _wall_cases():
    return [
        dict(xmode="periodic", ymode="wall"),
        dict(xmode="wall", ymode="periodic"),
        dict(xmode="periodic", ymode="periodic", circles=[(11.5, 8.0, 3.7)]),
        dict(xmode="periodic", ymode="wall", circles=[(10.0, 7.5, 4.2)]),
        dict(xmode="periodic", ymode="wet"),
        dict(xmode="periodic", ymode="wet", circles=[(10.0, 7.5, 3.2)]),
    ]


@pytest.mark.parametrize("case", _wall_cases())
def test_rest_state_is_exact(oracle_lib, case):
    """rho = 1, u = 0, F = 0, A = I stays put on any wall set (pin P4)."""
    pr = synth.rest_state(nx=24, ny=16, **case)
    o = oracle_lib.OracleSim(pr)
    o.step(60)
    r = o.read()
    fl = pr.fluid_mask()
    for k, ref in (("rho", 1.0), ("ux", 0.0), ("uy", 0.0), ("axx", 1.0), ("axy", 0.0),
                   ("ayy", 1.0)):
        assert np.abs(r[k][fl] - ref).max() < 1e-13, k


def test_rest_state_open_boundaries(oracle_lib):
    pr = synth.rest_state(nx=24, ny=12, xmode="open", ymode="wall", circles=[(12.0, 6.0, 2.5)])
    pr.inlet = dict(ux=np.zeros(12), axx=np.ones(12), axy=np.zeros(12), ayy=np.ones(12))
    o = oracle_lib.OracleSim(pr)
    o.step(40)
    r = o.read()
    fl = pr.fluid_mask()
    assert np.abs(r["rho"][fl] - 1).max() < 1e-13
    assert np.abs(r["ux"][fl]).max() < 1e-13 and np.abs(r["axx"][fl] - 1).max() < 1e-13


def _open_channel_steady(oracle_lib, ny, nu, umax):
    """Newtonian channel 3*ny x ny with half-way walls, the parabolic inlet profile of
    peak umax (node centres, walls at y = 0 and ny) and the outlet; run to steady state."""
    nx = 3 * ny
    pr = synth.random_periodic(nx, ny, seed=0, amp_u=0, amp_rho=0, amp_a=0, xmode="open",
                               ymode="wall", nu_s=nu, eta_p=0.0, force_amp=0.0)
    yp = np.arange(ny) + 0.5
    pr.inlet["ux"] = umax * 4 * yp * (ny - yp) / ny ** 2
    o = oracle_lib.OracleSim(pr)
    prev = None
    for _ in range(60):
        o.step(1000)
        r = o.read()
        if prev is not None and np.abs(r["ux"] - prev).max() < 1e-9 * umax:
            return pr, r
        prev = r["ux"].copy()
    raise AssertionError("open channel not steady")


def _shifted_wall_channel(oracle_lib, H, qb, qt, steps, curved="bouzidi"):
    """Oldroyd-B channel (Wi = 1, beta = 0.5 as Sec. 4.2) whose walls are two circles of
    radius 1e6: flat to 2e-6 over the 4-node period, at y_b = 1 - qb below fluid row 1
    and y_t = H + qt above row H, so every wall link has fraction qb or qt."""
    nx, ny, R = 4, H + 2, 1e6
    yb, yt = 1.0 - qb, H + qt
    base = synth.poiseuille(nx=nx, ny=H)
    G = base.Fx * (H / (yt - yb)) ** 2
    pr = base.with_(ny=ny, ymode="periodic", Fx=G, name="shifted_walls",
                    circles=[(nx / 2, yb - R, R), (nx / 2, yt + R, R)], curved=curved)
    fl = pr.fluid_mask()
    assert fl[1:H + 1].all() and not fl[0].any() and not fl[H + 1].any()
    o = oracle_lib.OracleSim(pr)
    o.step(steps)
    r = o.read()
    y = np.arange(1, H + 1, dtype=float)
    k = G / (2 * (pr.nu_s + pr.eta_p))
    du = k * (yb + yt - 2 * y)
    ref = dict(ux=k * (y - yb) * (yt - y), axy=pr.lam * du, axx=2 * (pr.lam * du) ** 2)
    err = (gre(r["ux"][1:H + 1, 0], ref["ux"]), gre(r["axy"][1:H + 1, 0], ref["axy"]),
           gre(r["axx"][1:H + 1, 0] - 1, ref["axx"]))
    c = np.polyfit(y, r["ux"][1:H + 1, 0], 2)
    walls = np.sort(np.roots(c).real)
    return err, walls, (yb, yt)


@pytest.mark.parametrize("qb,qt", [(0.5, 0.5), (0.3, 0.7), (0.2, 0.25), (0.8, 0.65)])
def test_curved_links_shifted_wall_poiseuille(oracle_lib, qb, qt):
    """Curved-link machinery (wall fractions q from the circle, interpolated bounce-back
    on both sides of q = 1/2, wall-aware differences at fraction q, CNEBB at curved links)
    against the steady closed form for walls at arbitrary positions: the fitted walls of
    the velocity profile lie within 0.08 of the true ones and every error falls from
    H = 16 to 32.  With q = 1/2 it is the half-way channel (second order); otherwise the
    conformation wall stays at the link midpoint (CNEBB treats curved walls as a
    staircase, Sec. 3.3), which makes u and A converge at about first order."""
    oracle_lib.set_threads(min(8, oracle_lib.max_threads()))
    e16, _, _ = _shifted_wall_channel(oracle_lib, 16, qb, qt, 12000)
    e32, walls, true = _shifted_wall_channel(oracle_lib, 32, qb, qt, 40000)
    assert np.abs(walls - np.array(true)).max() < 0.08, (walls, true)
    assert e32[0] < 1e-2 and e32[1] < 6e-2 and e32[2] < 0.16, e32
    assert all(a / b > 1.7 for a, b in zip(e16, e32)), (e16, e32)
    if qb == qt == 0.5:
        assert e32[0] < 1.2e-3 and e16[0] / e32[0] > 3.5


def _newtonian_shifted_channel(oracle_lib, H, qb, qt, curved):
    """Steady Newtonian Poiseuille flow between the two flat circle walls of
    _shifted_wall_channel (fractions qb below row 1, qt above row H); returns the largest
    velocity error relative to the closed form's maximum and the walls fitted to the
    profile."""
    nx, ny, R = 4, H + 2, 1e6
    yb, yt = 1.0 - qb, H + qt
    nu, F = 0.1, 1e-6 * (16.0 / H) ** 2
    pr = synth.random_periodic(nx, ny, seed=1, circles=[(nx / 2, yb - R, R), (nx / 2, yt + R, R)],
                               amp_u=0, amp_rho=0, amp_a=0, force_amp=0, nu_s=nu, eta_p=0.0,
                               lam=10.0, kappa=0.1, Lambda_s=3.0 / 16.0, Lambda_p=0.25)
    pr = pr.with_(Fx=F, Fy=0.0, curved=curved)
    o = oracle_lib.OracleSim(pr)
    o.step(int(8 * (yt - yb) ** 2 / nu))
    u = o.read()["ux"][1:H + 1, 0]
    y = np.arange(1, H + 1, dtype=float)
    exact = F / (2 * nu) * (y - yb) * (yt - y)
    walls = np.sort(np.roots(np.polyfit(y, u, 2)).real)
    return float(np.abs(u - exact).max() / exact.max()), walls, (yb, yt)


@pytest.mark.parametrize("qb,qt", [(0.3, 0.7), (0.2, 0.25), (0.8, 0.65)])
def test_ylw_curved_wall_newtonian_poiseuille_second_order(oracle_lib, qb, qt):
    """The cylinder's curved-wall scheme for f (Sec. 4.3, reading A30: the unified
    interpolation of Yu, Mei, Luo and Shyy with the mass restore) against the closed form
    for walls at arbitrary fractions: second order (error ratio above 3.5 from H = 16 to
    32, below 2.5e-3 at H = 32) with the fitted walls within 0.03 of the true ones.  A
    swapped interpolation weight, a dropped term of the back interpolation or the wrong
    direction at the far node each miss by an order of magnitude and converge at first
    order."""
    oracle_lib.set_threads(min(8, oracle_lib.max_threads()))
    e16, _, _ = _newtonian_shifted_channel(oracle_lib, 16, qb, qt, "ylw")
    e32, walls, true = _newtonian_shifted_channel(oracle_lib, 32, qb, qt, "ylw")
    assert e32 < 2.5e-3 and e16 / e32 > 3.5, (e16, e32)
    assert np.abs(walls - np.array(true)).max() < 0.03, (walls, true)


def test_ylw_conserves_mass_exactly(oracle_lib):
    """With the mass restore of reading A30 the total mass of a periodic box with a
    circle is conserved to round-off; linear interpolated bounce-back alone, or the
    unified interpolation without the restore, change it by about 5e-5 in 25 steps."""
    out = {}
    for curved in ("bouzidi", "ylw"):
        pr = synth.random_periodic(24, 20, seed=12, circles=[(11.3, 9.6, 4.3)]).with_(curved=curved)
        o = oracle_lib.OracleSim(pr)
        m0 = o.read()["rho"].sum()
        o.step(25)
        out[curved] = (o.read()["rho"].sum() - m0) / m0
    assert abs(out["ylw"]) < 1e-13, out
    assert abs(out["bouzidi"]) > 1e-6, out


def test_open_channel_poiseuille_second_order(oracle_lib):
    """Open ends (Sec. 4.3: prescribed inlet profile, zero-gradient outlet) on a straight
    channel: far from the ends the flow is plane Poiseuille with the inlet's flow rate,
    dp/dx = -8 mu U_max / H^2 with p = c_s^2 rho, and the pressure extrapolates to the
    reference density at the outlet ghost column; the error to the closed form falls at
    second order from H = 16 to H = 32 (2.0 % -> 0.47 % of U_max at nu = 0.5; the
    extrapolated non-equilibrium part carries an O(tau dx^2) error).
    """
    oracle_lib.set_threads(min(8, oracle_lib.max_threads()))
    nu, umax = 0.5, 0.002
    err = {}
    for ny in (16, 32):
        pr, r = _open_channel_steady(oracle_lib, ny, nu, umax)
        nx = pr.nx
        yp = np.arange(ny) + 0.5
        exact = umax * 4 * yp * (ny - yp) / ny ** 2
        mid = r["ux"][:, nx // 2]
        err[ny] = np.abs(mid - exact).max() / umax
        assert np.abs(r["uy"][:, nx // 4: 3 * nx // 4]).max() < 1e-3 * umax
        rho = r["rho"].mean(0)
        x = np.arange(nx)
        slope, icpt = np.polyfit(x[nx // 4: 3 * nx // 4], rho[nx // 4: 3 * nx // 4], 1)
        ref = -8 * nu * umax / ny ** 2 / CS2
        assert abs(slope / ref - 1) < (0.025 if ny == 16 else 0.005), (ny, slope, ref)
        # reference density at the outlet ghost column x = nx (linear part of p)
        assert abs(slope * nx + icpt - 1.0) < 1e-3 * abs(slope) * nx, (ny, slope * nx + icpt)
        assert np.ptp(r["rho"][:, nx // 4: 3 * nx // 4], axis=0).max() < 1e-2 * abs(slope) * nx
    assert err[32] < 6e-3 and err[16] / err[32] > 3.5, err


def _open_channel_oldroyd_b(oracle_lib, ny, steps, open_ends="neqe"):
    """Oldroyd-B channel 3*ny x ny between half-way walls at Wi = 1, beta = 0.5, Ma = 0.01
    (the Sec. 4.2 groups), driven only through its open ends: the inlet carries the
    parabolic velocity and the conformation of the steady channel solution, the outlet
    is the zero-gradient column.  Starts from that solution everywhere."""
    base = synth.poiseuille(nx=3 * ny, ny=ny, Wi=1.0, Ma=0.01)
    lam, Uc = base.lam, base.meta["Uc"]
    yp = np.arange(ny) + 0.5
    ux = 4 * Uc * yp * (ny - yp) / ny ** 2
    du = 4 * Uc * (ny - 2 * yp) / ny ** 2
    axy, axx = lam * du, 1 + 2 * (lam * du) ** 2
    pr = base.with_(xmode="open", Fx=0.0, name="open_oldroyd_b", open_ends=open_ends,
                    inlet=dict(ux=ux, axx=axx, axy=axy, ayy=np.ones(ny)))
    full = lambda v: np.ascontiguousarray(np.broadcast_to(v[:, None], (ny, pr.nx)))
    pr.init = dict(ux=full(ux), axx=full(axx), axy=full(axy))
    o = oracle_lib.OracleSim(pr)
    o.step(steps)
    return pr, o.read(), dict(ux=ux, axy=axy, axx=axx)


def test_open_channel_oldroyd_b_conformation_at_every_column(oracle_lib):
    """The open ends carry the conformation of the channel solution (Sec. 4.3 set-up;
    reading A21 with the inlet profile of reading A19): in an Oldroyd-B channel driven
    only through its inlet and outlet, every column -- the first and the last included --
    holds the steady closed form A_xy = lambda u', A_xx = 1 + 2 (lambda u')^2, A_yy = 1
    within the discretisation error of the same channel with periodic ends (the same
    walls, the same H).

    Catches an inlet conformation ghost extrapolated around A = I instead of the
    prescribed profile (first column off by about 85 %), an outlet ghost set to the rest
    equilibrium instead of the zero-gradient copy (last column off by about 90 %), and a
    velocity profile that does not carry through the inlet.
    """
    oracle_lib.set_threads(min(8, oracle_lib.max_threads()))
    ny = 16
    pr, r, ex = _open_channel_oldroyd_b(oracle_lib, ny, 30000)
    # the periodic channel with the same groups, to its steady state: the error budget
    per = synth.poiseuille(nx=2, ny=ny, Wi=1.0, Ma=0.01)
    op = oracle_lib.OracleSim(per)
    op.step(int(round(18 * per.meta["Tc"])))
    rp = op.read()
    bud_xy = np.abs(rp["axy"][:, 0] - ex["axy"]).max() / np.abs(ex["axy"]).max()
    bud_xx = np.abs(rp["axx"][:, 0] - ex["axx"]).max() / np.abs(ex["axx"] - 1).max()
    assert 1e-3 < bud_xy < 5e-2 and 1e-3 < bud_xx < 5e-2, (bud_xy, bud_xx)
    e_xy = np.abs(r["axy"] - ex["axy"][:, None]).max(axis=0) / np.abs(ex["axy"]).max()
    e_xx = np.abs(r["axx"] - ex["axx"][:, None]).max(axis=0) / np.abs(ex["axx"] - 1).max()
    e_u = np.abs(r["ux"] - ex["ux"][:, None]).max(axis=0) / pr.meta["Uc"]
    for c in (0, 1, pr.nx // 2, pr.nx - 2, pr.nx - 1):
        assert e_xy[c] < 1.25 * bud_xy, (c, e_xy[c], bud_xy)
        assert e_xx[c] < 1.25 * bud_xx, (c, e_xx[c], bud_xx)
    assert e_xy.max() < 1.25 * bud_xy and e_xx.max() < 1.25 * bud_xx
    assert e_u.max() < 1e-2, e_u.max()
    assert np.abs(r["ayy"] - 1).max() < 1e-3 * np.abs(ex["axx"] - 1).max()


def test_nebb_open_ends_hold_their_boundary_state(oracle_lib):
    """Wet-node NEBB open ends (Sec. 4.3, reading A31): from a random state with a
    per-node body force, after every step the first column carries exactly the inlet
    velocity (u_in(y), 0) and the last column the reference density 1 with u_y = 0 (read
    out with the half-force shift).  A wrong density closure, a dropped half-force term
    or a wrong diagonal weight breaks one of the four at 1e-6 or more."""
    pr = synth.random_periodic(40, 18, seed=5, xmode="open", ymode="wall",
                               circles=[(20.3, 9.1, 3.3)]).with_(open_ends="nebb")
    o = oracle_lib.OracleSim(pr)
    for n in (1, 1, 5):
        o.step(n)
        r = o.read()
        assert np.abs(r["ux"][:, 0] - pr.inlet["ux"]).max() < 1e-15
        assert np.abs(r["uy"][:, 0]).max() < 1e-15
        assert np.abs(r["rho"][:, -1] - 1.0).max() < 1e-14
        assert np.abs(r["uy"][:, -1]).max() < 1e-15
    # the conformation open ends are still the extrapolation ghosts: A is not pinned there
    assert np.abs(r["axx"][:, 0] - pr.inlet["axx"]).max() > 1e-6


def _nebb_channel(oracle_lib, ny, nu=0.5, umax=2e-4):
    nx = 3 * ny
    pr = synth.random_periodic(nx, ny, seed=0, amp_u=0, amp_rho=0, amp_a=0, xmode="open",
                               ymode="wall", nu_s=nu, eta_p=0.0,
                               force_amp=0.0).with_(open_ends="nebb")
    yp = np.arange(ny) + 0.5
    exact = umax * 4 * yp * (ny - yp) / ny ** 2
    pr.inlet["ux"] = exact
    o = oracle_lib.OracleSim(pr)
    prev = None
    for _ in range(80):
        o.step(1000)
        r = o.read()
        if prev is not None and np.abs(r["ux"] - prev).max() < 1e-9 * umax:
            return pr, r, exact
        prev = r["ux"].copy()
    raise AssertionError("open channel not steady")


def test_nebb_open_channel_poiseuille_second_order(oracle_lib):
    """Newtonian channel with wet-node NEBB open ends (reading A31): the mass flux of the
    inlet passes unchanged, the pressure falls at dp/dx = -8 mu U_max / H^2 to the
    reference density at the outlet column, and mid-channel the profile is the inlet's
    parabola scaled by the density ratio (the flux is rho u), with an error falling at
    second order from H = 16 (0.11 % of U_max) to H = 32 (0.03 %)."""
    oracle_lib.set_threads(min(8, oracle_lib.max_threads()))
    nu, umax = 0.5, 2e-4
    err = {}
    for ny in (16, 32):
        pr, r, exact = _nebb_channel(oracle_lib, ny, nu, umax)
        nx = pr.nx
        flux = (r["rho"] * r["ux"]).sum(axis=0)
        assert np.abs(flux / flux[0] - 1).max() < 1e-8
        rho = r["rho"].mean(0)
        x = np.arange(nx)
        slope, icpt = np.polyfit(x[nx // 4: 3 * nx // 4], rho[nx // 4: 3 * nx // 4], 1)
        ref = -8 * nu * umax / ny ** 2 / CS2
        assert abs(slope / ref - 1) < (3e-3 if ny == 16 else 1e-3), (ny, slope, ref)
        assert abs(slope * (nx - 1) + icpt - 1.0) < 1e-6, (ny, slope * (nx - 1) + icpt)
        scaled = exact * r["rho"][:, 0].mean() / r["rho"][:, nx // 2].mean()
        err[ny] = np.abs(r["ux"][:, nx // 2] - scaled).max() / umax
    assert err[16] < 1.3e-3 and err[32] < 3.5e-4 and err[16] / err[32] > 3.3, err


def test_nebb_open_channel_oldroyd_b_conformation_at_every_column(oracle_lib):
    """The Oldroyd-B channel driven only through its open ends, with the hydrodynamic
    ends as wet NEBB nodes (reading A31) and the conformation ends as the extrapolation
    ghosts: every column holds the steady closed form A_xy = lambda u',
    A_xx = 1 + 2 (lambda u')^2 within 1.25 times the error of the periodic channel."""
    oracle_lib.set_threads(min(8, oracle_lib.max_threads()))
    ny = 16
    pr, r, ex = _open_channel_oldroyd_b(oracle_lib, ny, 30000, open_ends="nebb")
    per = synth.poiseuille(nx=2, ny=ny, Wi=1.0, Ma=0.01)
    op = oracle_lib.OracleSim(per)
    op.step(int(round(18 * per.meta["Tc"])))
    rp = op.read()
    bud_xy = np.abs(rp["axy"][:, 0] - ex["axy"]).max() / np.abs(ex["axy"]).max()
    bud_xx = np.abs(rp["axx"][:, 0] - ex["axx"]).max() / np.abs(ex["axx"] - 1).max()
    e_xy = np.abs(r["axy"] - ex["axy"][:, None]).max(axis=0) / np.abs(ex["axy"]).max()
    e_xx = np.abs(r["axx"] - ex["axx"][:, None]).max(axis=0) / np.abs(ex["axx"] - 1).max()
    e_u = np.abs(r["ux"] - ex["ux"][:, None]).max(axis=0) / pr.meta["Uc"]
    assert e_xy.max() < 1.25 * bud_xy and e_xx.max() < 1.25 * bud_xx, (e_xy.max(), e_xx.max(),
                                                                        bud_xy, bud_xx)
    assert e_u[0] < 1e-14 and e_u.max() < 1e-2, e_u


@pytest.mark.parametrize("walls", ["y", "x"])
def test_hydrostatic_channel_keeps_the_conformation_at_rest(oracle_lib, walls):
    """A body force normal to half-way walls settles into hydrostatic equilibrium: the
    velocity with the half-force shift (Sec. 3.1) is zero to round-off, the pressure
    gradient balances the force density, c_s^2 d rho / dn = F, and the conformation stays
    A = I: the only residue is the (tau_p1 - 1/2) F phi / rho first moment that G~_i
    leaves in a forced fluid at rest, here lambda (tau_p1 - 1/2) |F| = 6e-9.

    Catches a CNEBB equilibrium taken at the unshifted velocity j / rho (Sec. 3.3 uses the
    fluid velocity, which in a forced fluid includes F / 2): the wall nodes then see a
    spurious normal velocity -F / (2 rho), and the conformation near the walls moves off
    I by 1e-5 here.
    """
    F, lam, kappa = 1e-4, 20.0, 1e-6
    tp = 3 * kappa  # tau_p1 - 1/2
    if walls == "y":
        pr = synth.random_periodic(4, 16, seed=0, amp_u=0, amp_rho=0, amp_a=0, ymode="wall",
                                   nu_s=0.5, eta_p=0.1, lam=lam, kappa=kappa, Lambda_p=1e-6,
                                   force_amp=0.0)
        pr.Fx, pr.Fy = 0.0, F
    else:
        pr = synth.random_periodic(16, 4, seed=0, amp_u=0, amp_rho=0, amp_a=0, xmode="wall",
                                   nu_s=0.5, eta_p=0.1, lam=lam, kappa=kappa, Lambda_p=1e-6,
                                   force_amp=0.0)
        pr.Fx, pr.Fy = F, 0.0
    o = oracle_lib.OracleSim(pr)
    o.step(3000)
    r = o.read()
    assert np.abs(r["ux"]).max() < 1e-13 and np.abs(r["uy"]).max() < 1e-13
    rho = r["rho"][:, 0] if walls == "y" else r["rho"][0, :]
    assert np.abs(np.diff(rho) / (F / CS2) - 1).max() < 1e-6, np.diff(rho)
    bound = 10 * lam * tp * F
    for c, one in (("axx", 1.0), ("axy", 0.0), ("ayy", 1.0)):
        assert np.abs(r[c] - one).max() < bound, (c, np.abs(r[c] - one).max(), bound)


@pytest.mark.parametrize("case", [dict(xmode="periodic", ymode="wall"),
                                  dict(xmode="periodic", ymode="periodic")])
def test_hydro_mass_is_exact(oracle_lib, case):
    """Periodic + half-way bounce-back conserve total mass to round-off (pin P6)."""
    pr = synth.random_periodic(20, 14, seed=11, **case)
    o = oracle_lib.OracleSim(pr)
    m0 = o.read()["rho"].sum()
    o.step(25)
    assert abs(o.read()["rho"].sum() - m0) < 1e-12 * m0


@pytest.mark.parametrize("case", _wall_cases())
def test_cnebb_conformation_budget(oracle_lib, case):
    """CNEBB conserves every conformation component exactly (Sec. 3.3; pin P6).

    With walls, staircase and curved obstacles: sum phi(n+1) = sum [phi + S + (S -
    S_prev)/2](n) to round-off, and with the source switched off sum phi is constant.
    Catches a wrong phi_b (missing post-collision wall-bound populations), a missing
    g_0 fix-up, or a streaming index error.
    """
    pr = synth.random_periodic(22, 16, seed=5, **case)
    o = oracle_lib.OracleSim(pr)
    fl = pr.fluid_mask()
    o.step(3)
    for _ in range(4):
        before = o.read()
        h0, first0 = o.history()
        o.step(1)
        after = o.read()
        h1, _ = o.history()  # S(n) and u(n) of the step just taken
        for comp, s in (("axx", "sxx"), ("axy", "sxy"), ("ayy", "syy")):
            sp = h0[s] if not first0 else h1[s]
            budget = (before[comp] + h1[s] + 0.5 * (h1[s] - sp))[fl].sum()
            assert abs(after[comp][fl].sum() - budget) < 1e-12 * max(1.0, abs(budget))
    o2 = oracle_lib.OracleSim(pr, flags=oracle_lib.FLAG_NO_SOURCE)
    tot0 = {c: o2.read()[c][fl].sum() for c in ("axx", "axy", "ayy")}
    o2.step(20)
    r = o2.read()
    for c in ("axx", "axy", "ayy"):
        assert abs(r[c][fl].sum() - tot0[c]) < 1e-12 * max(1.0, abs(tot0[c]))


def test_poiseuille_mirror_symmetry(oracle_lib):
    """Channel flow is mirror symmetric about the centre line (pin P7)."""
    pr = synth.poiseuille(nx=8, ny=32, steps=0)
    o = oracle_lib.OracleSim(pr)
    o.step(1500)
    r = o.read()
    for k in ("ux", "axx", "ayy", "rho"):
        assert np.abs(r[k] - r[k][::-1]).max() < 1e-12 * max(1.0, np.abs(r[k]).max())
    for k in ("uy", "axy"):
        assert np.abs(r[k] + r[k][::-1]).max() < 1e-12 * max(1.0, np.abs(r[k]).max())


# ---------------------------------------------------------------------------------
# Closed forms of the paper's benchmarks
# ---------------------------------------------------------------------------------
def test_poiseuille_steady_closed_form(oracle_lib):
    """Steady Oldroyd-B Poiseuille at Wi = 1, beta = 0.5, Ny = 32 (Sec. 4.2; pin P1).

    Catches a dropped or mis-scaled T_i (u would change by a factor 2), a wrong
    upper-convected term (A_xx, A_xy), a wrong CNEBB reconstruction near the walls.
    """
    pr = synth.poiseuille(nx=4, ny=32)
    o = oracle_lib.OracleSim(pr)
    o.step(10000)
    r = o.read()
    ref = poiseuille_steady(32, pr.meta["Uc"], pr.lam)
    assert gre(r["ux"][:, 0], ref["ux"]) < 2e-3
    assert gre(r["axy"][:, 0], ref["axy"]) < 6e-3
    assert gre(r["axx"][:, 0], ref["axx"]) < 1.5e-2
    assert np.abs(r["ayy"] - 1).max() < 1e-10
    assert np.abs(r["uy"]).max() < 1e-14


def test_poiseuille_second_order(oracle_lib):
    """Global relative error falls at second order for Ny = 16, 32, 64 (Sec. 4.2)."""
    errs = []
    for ny in (16, 32, 64):
        pr = synth.poiseuille(nx=2, ny=ny)
        o = oracle_lib.OracleSim(pr)
        o.step(int(round(18 * pr.meta["Tc"])))
        r = o.read()
        ref = poiseuille_steady(ny, pr.meta["Uc"], pr.lam)
        errs.append([gre(r["ux"][:, 0], ref["ux"]), gre(r["axy"][:, 0], ref["axy"]),
                     gre(r["axx"][:, 0], ref["axx"])])
    errs = np.array(errs)
    order = np.log2(errs[0] / errs[2]) / 2
    assert np.all(order > 1.8), order


# ---------------------------------------------------------------------------------
# Wet-node walls (non-equilibrium bounce-back at the wall nodes, reading A29)
# ---------------------------------------------------------------------------------
@pytest.mark.parametrize("ny", [9, 17])
def test_wet_walls_newtonian_poiseuille_is_exact(oracle_lib, ny):
    """Newtonian channel flow between wet-node walls reaches the parabola
    u = 4 U_c y (H - y) / H^2, H = ny - 1, to round-off (pin P12).

    A closed form the scheme reproduces exactly: non-equilibrium bounce-back with the
    half-force momentum and a second-order collision hold the wall nodes at u = 0 and
    the interior on the parabola.  A missing -F/2 in the wall momentum (slip F/2),
    a wrong sign or weight of the tangential correction or of the normal term, or a
    wrong wall row, each leave an O(1e-3) error or more.
    """
    pr = synth.poiseuille(nx=2, ny=ny, beta=1.0, wet=True)
    o = oracle_lib.OracleSim(pr)
    o.step(int(30 * pr.meta["Tc"]))
    r = o.read()
    ref = poiseuille_steady(ny, pr.meta["Uc"], pr.lam, wet=True)
    assert np.abs(r["ux"][:, 0] - ref["ux"]).max() < 1e-12 * ref["ux"].max()
    assert np.abs(r["uy"]).max() < 1e-14
    # the populations the wall nodes hold carry zero velocity: sum e f + F/2 = 0
    f, _ = o.populations()
    ex = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
    jx = np.tensordot(ex, f, axes=1) + 0.5 * pr.Fx
    assert np.abs(jx[[0, -1], :]).max() < 1e-15


def test_wet_walls_oldroyd_b_poiseuille(oracle_lib):
    """Steady Oldroyd-B channel flow between wet-node walls (Wi = 1, beta = 0.5, Sec. 4.2):
    the closed form at H = 16, 32, 64 with errors falling at close to second order.

    The wall nodes take their wall-normal velocity gradient from the one-sided
    second-order difference; a first-order difference there would leave A_xy and A_xx
    at first order.
    """
    errs = []
    for ny in (17, 33, 65):
        pr = synth.poiseuille(nx=2, ny=ny, wet=True)
        o = oracle_lib.OracleSim(pr)
        o.step(int(round(18 * pr.meta["Tc"])))
        r = o.read()
        ref = poiseuille_steady(ny, pr.meta["Uc"], pr.lam, wet=True)
        errs.append([gre(r["ux"][:, 0], ref["ux"]), gre(r["axy"][:, 0], ref["axy"]),
                     gre(r["axx"][:, 0], ref["axx"])])
        assert np.abs(r["ayy"] - 1).max() < 1e-10
    errs = np.array(errs)
    assert errs[1, 0] < 1e-4 and errs[1, 1] < 3e-3 and errs[1, 2] < 8e-3, errs
    order = np.log2(errs[0] / errs[2]) / 2
    assert np.all(order > 1.6), order


def test_wet_walls_reject_solids_next_to_the_wall(oracle_lib):
    """The one-sided differences at wall nodes need two fluid rows: solids there are
    refused (as by the library)."""
    mask = np.zeros((12, 10), np.uint8)
    mask[2, 4] = 1
    pr = synth.random_periodic(10, 12, seed=1, ymode="wet", solid=mask)
    with pytest.raises(Exception):
        oracle_lib.OracleSim(pr)


def test_waters_king_transient(oracle_lib):
    """Centre-line start-up velocity vs the Waters-King series (Sec. 4.2; pin P2).

    Tolerance 3 % of U_c covers Ma = 0.1 compressibility and the half-step start; the
    overshoot to 1.56 U_c at t* = 0.5 is elastic, so a missing polymer stress, a wrong
    lambda or a wrong time difference of F~ fails by far more.
    """
    pr = synth.poiseuille(nx=2, ny=32)
    o = oracle_lib.OracleSim(pr)
    Tc, Uc = pr.meta["Tc"], pr.meta["Uc"]
    ys = (np.arange(32) + 0.5) / 32
    done = 0
    for ts in (0.25, 0.5, 1.0, 2.0, 5.0):
        n = int(round(ts * Tc))
        o.step(n - done)
        done = n
        u = o.read()["ux"][:, 0] / Uc
        ref = waters_king_u(ys, n / Tc, 1.0, 0.5)
        assert np.abs(u - ref).max() < 0.03, (ts, np.abs(u - ref).max())


def test_four_roll_newtonian_steady(oracle_lib):
    """Newtonian four-roll mill converges to U_c(-sin cos, cos sin) at second order (P3)."""
    errs = []
    for N in (16, 32):
        pr = synth.four_roll_mill(N=N, beta=1.0, Wi=1.0, steps=0, precision="fp64")
        assert pr.eta_p == 0.0
        o = oracle_lib.OracleSim(pr)
        o.step(int(6 / (pr.nu_s * (2 * math.pi / N) ** 2)))
        r = o.read()
        ux, uy = four_roll_newtonian(N, pr.meta["Uc"])
        errs.append(math.sqrt(((r["ux"] - ux) ** 2 + (r["uy"] - uy) ** 2).mean()) / pr.meta["Uc"])
    assert errs[1] < 3e-3
    assert math.log2(errs[0] / errs[1]) > 1.8


# ---------------------------------------------------------------------------------
# Transport coefficients and single-term effects
# ---------------------------------------------------------------------------------
def _mode_amp(field, k):
    x = np.arange(field.shape[-1])
    return abs((field[0] * np.exp(-1j * k * x)).sum())


@pytest.mark.parametrize("U", [0.0, 0.05])
def test_shear_wave_viscosity(oracle_lib, U):
    """Shear wave decays at nu_s k^2, nu_s = c_s^2 (tau_s1 - 1/2) (Sec. 3.1; P3)."""
    pr = synth.waves("shear", n=64, amp=1e-4, nu_s=0.05, U=U)
    o = oracle_lib.OracleSim(pr)
    k = pr.meta["k"]
    o.step(50)
    a0 = _mode_amp(o.read()["uy"], k)
    o.step(500)
    a1 = _mode_amp(o.read()["uy"], k)
    rate = -math.log(a1 / a0) / 500
    assert abs(rate / (pr.nu_s * k * k) - 1) < 2e-3


@pytest.mark.parametrize("lam", [1e12, 2000.0])
def test_conformation_diffusion(oracle_lib, lam):
    """A_xx mode at rest decays at kappa k^2 + 1/lambda, kappa = c_s^2 (tau_p1 - 1/2) (P10)."""
    pr = synth.waves("conformation", n=64, amp=1e-3, kappa=0.1, lam=lam)
    o = oracle_lib.OracleSim(pr)
    k = pr.meta["k"]
    o.step(20)
    a0 = _mode_amp(o.read()["axx"] - 1, k)
    o.step(400)
    a1 = _mode_amp(o.read()["axx"] - 1, k)
    rate = -math.log(a1 / a0) / 400
    assert abs(rate / (pr.kappa * k * k + 1 / lam) - 1) < 2e-3


@pytest.mark.parametrize("kappa", [0.1, 0.02])
def test_auxiliary_term_cancels_the_accelerated_flux_error(oracle_lib, kappa):
    """G~_i against the Chapman-Enskog error of the convection-diffusion scheme (Sec. 3.2).

    A conformation wave A_xx = 1 + a sin(k x) carried by a uniform flow that a body force
    F accelerates from rest.  Without G~_i the scheme's first-order error flux
    (tau_p1 - 1/2) d_t(phi u) = (tau_p1 - 1/2) phi F / rho slows the pattern by
    (tau_p1 - 1/2) F per step; G~_i must give back exactly that displacement.  The
    displacement with and without it (the latter a mistake planted in the oracle) must
    differ by (tau_p1 - 1/2) F T to 0.5 %: a prefactor 1 - 1/tau instead of
    1 - 1/(2 tau), a flipped sign or a missing phi fails.
    """
    n, T, F = 128, 400, 1e-5
    k = 2 * np.pi / n
    x = np.arange(n)
    disp = []
    for flags in (0, oracle_lib.FLAG_NO_GTILDE):
        pr = synth.waves("conformation", n=n, amp=1e-3, kappa=kappa).with_(Fx=F)
        o = oracle_lib.OracleSim(pr, flags=flags)

        def phase():
            a = o.read()["axx"][0] - 1
            return np.angle((a * np.exp(-1j * k * x)).sum())

        p0 = phase()
        o.step(T)
        disp.append(-np.angle(np.exp(1j * (phase() - p0))) / k)
    ref = 3.0 * kappa * F * T  # (tau_p1 - 1/2) F T with tau_p1 = 3 kappa + 1/2
    assert abs((disp[0] - disp[1]) / ref - 1) < 5e-3, (disp, ref)
    # and the pattern moves with the flow: sum of u_n = F (n + 1/2) over the steps, to
    # within a few 1e-3
    assert abs(disp[0] / (F * T * T / 2) - 1) < 3e-3, disp


def _sound_decay(oracle_lib, U):
    pr = synth.waves("sound", n=64, amp=1e-4, nu_s=0.05, U=U)
    o = oracle_lib.OracleSim(pr)
    k = pr.meta["k"]
    x = np.arange(64)
    E = []
    for _ in range(600):
        r = o.read()
        a = ((r["rho"][0] - 1) * np.exp(-1j * k * x)).sum()
        b = ((r["ux"][0] - U) * np.exp(-1j * k * x)).sum()
        E.append(abs(a) ** 2 / 3 + abs(b) ** 2)
        o.step(1)
    t = np.arange(600)
    return -np.polyfit(t[100:], np.log(np.array(E)[100:]), 1)[0] / 2


def test_galilean_invariant_sound_damping(oracle_lib):
    """Acoustic damping is the same in a frame moving at U = 0.1 (Sec. 3.1, G_i).

    The D2Q9 equilibrium lacks rho u_x^3; the correction G_i removes that defect.
    With G_i the two damping rates agree to ~1e-5; a dropped G_i changes the moving
    frame's rate by 4.5 % and a sign error by about as much the other way.
    """
    r0 = _sound_decay(oracle_lib, 0.0)
    r1 = _sound_decay(oracle_lib, 0.1)
    assert abs(r1 / r0 - 1) < 5e-3


def test_source_time_integration_second_order(oracle_lib):
    """Uniform A relaxes as exp(-t/lambda) to second order (Sec. 3.2, d_t F~ term).

    With lambda = 10 the half time-difference of F~ makes the source integration
    second order (error 0.3 % after 20 steps); without it the error is 10 %.
    """
    pr = synth.waves("conformation", n=8, amp=0.0, lam=10.0, kappa=0.1)
    pr.init["axx"] = np.full((4, 8), 1.5)
    o = oracle_lib.OracleSim(pr)
    o.step(20)
    a = o.read()["axx"][0, 0] - 1
    assert abs(a / (0.5 * math.exp(-2.0)) - 1) < 1e-2


# ---------------------------------------------------------------------------------
# Geometry
# ---------------------------------------------------------------------------------
def test_geometry_channel_links(oracle_lib):
    """Channel: 3 links per wall node, q = 1/2, sorted by (node, dir)."""
    pr = synth.poiseuille(nx=64, ny=32, steps=0)
    o = oracle_lib.OracleSim(pr)
    cls, node, d, q = o.geometry()
    assert len(node) == 2 * 64 * 3
    assert np.all(q == 0.5)
    assert np.all(np.diff(node.astype(np.int64) * 16 + d) > 0)
    assert set(np.unique(d[node < 64])) == {4, 7, 8}
    assert (cls == 2).sum() == 128 and (cls == 1).sum() == 0


def test_geometry_circle_fractions(oracle_lib):
    """Circle links: 0 < q <= 1 and the cut point lies on the circle."""
    xc, yc, R = 20.0, 15.0, 6.5
    pr = synth.rest_state(nx=40, ny=30, xmode="periodic", ymode="periodic", circles=[(xc, yc, R)])
    o = oracle_lib.OracleSim(pr)
    cls, node, d, q = o.geometry()
    ex, ey, _, _ = oracle_lib.lattice()
    assert len(node) > 0 and np.all(q > 0) and np.all(q <= 1)
    x = node % 40
    y = node // 40
    px = x + q * ex[d] - xc
    py = y + q * ey[d] - yc
    np.testing.assert_allclose(np.hypot(px, py), R, rtol=1e-12)
    fl = pr.fluid_mask()
    assert np.array_equal(cls == 1, ~fl)


def test_waters_king_series_limits():
    """The start-up series used by the transient pins (Sec. 4.2) in its known limits.

    beta = 1 (no polymer) must equal the textbook Newtonian start-up series
    u* = 4y(1-y) - 32 sum sin(N y)/N^3 exp(-N^2 t*/Re); long times give the steady
    parabola; and the centre-line values at Wi = 1 (t* = 0.25, 0.5, 1, 2, 5) and at
    Wi = 10^4 (t* = 18.04), beta = 0.5, are reproduced.
    """
    ys = np.linspace(0.05, 0.95, 7)
    n = np.arange(1, 4001, dtype=float)
    N = (2 * n - 1) * math.pi
    for t in (0.01, 0.1, 0.5):
        newt = 4 * ys * (1 - ys) - 32 * (np.sin(np.multiply.outer(ys, N)) / N ** 3 *
                                         np.exp(-N ** 2 * t)).sum(-1)
        np.testing.assert_allclose(waters_king_u(ys, t, 3.0, 1.0), newt, atol=1e-10)
    np.testing.assert_allclose(waters_king_u(ys, 200.0, 1.0, 0.5), 4 * ys * (1 - ys), atol=1e-9)
    for t, v in ((0.25, 1.34216), (0.5, 1.55606), (1.0, 1.27296), (2.0, 1.01680),
                 (5.0, 0.999996)):
        assert abs(float(waters_king_u(0.5, t, 1.0, 0.5)) - v) < 1e-5, t
    assert abs(float(waters_king_u(0.5, 18.04, 1e4, 0.5)) - 1.99648) < 1e-5


def test_momentum_exchange_balance(oracle_lib):
    """Momentum-exchange force (Sec. 4.3) against the exact momentum budget.

    Every collision adds the body force F to a node's momentum and every boundary link
    removes e_i (f_i^post + f_opp(i)) from the fluid, whatever rule fills the returning
    population; in a domain closed by periodicity and solids the total momentum
    P = sum(rho u - F/2) therefore obeys P(t+1) - P(t) = sum F - D at every step, with
    D the drag on all solids (walls, a staircase block and a curved cylinder here).
    """
    mask = np.zeros((30, 60), np.uint8)
    mask[12:16, 10:14] = 1
    pr = synth.random_periodic(60, 30, seed=5, ymode="wall", solid=mask,
                               circles=[(40.0, 15.0, 6.3)])
    o = oracle_lib.OracleSim(pr)
    fx, fy = pr.force_arrays()
    fl = pr.fluid_mask()

    def momentum():
        r = o.read()
        return np.array([((r["rho"] * r["ux"] - 0.5 * fx)[fl]).sum(),
                         ((r["rho"] * r["uy"] - 0.5 * fy)[fl]).sum()])

    with pytest.raises(ValueError):
        o.drag(-1)  # no step taken yet
    o.step(3)
    fsum = np.array([fx[fl].sum(), fy[fl].sum()])
    for _ in range(3):
        p0 = momentum()
        o.step(1)
        d = np.array(o.drag(-1))
        assert np.abs(d).max() > 1e-2
        assert np.abs(momentum() - p0 - (fsum - d)).max() < 1e-12
        # the cylinder's share is part of it and is not the whole
        dc = np.array(o.drag(0))
        assert 0 < np.abs(dc).max() < np.abs(d).max()
