"""Closed-form solutions the paper states or that follow from its model equations.

These are independent of both the oracle and the HIP library: they are evaluated
directly from the formulas, in numpy.
"""
from __future__ import annotations

import math

import numpy as np


def waters_king_u(ystar, tstar, Wi, beta, Re=1.0, nterms=20000):
    """Start-up of Oldroyd-B plane Poiseuille flow (Sec. 4.2, Waters and King).

    u*(y*, t*) = 4 y*(1 - y*) - 32 sum_n sin(N y*) / N^3 G_N(E, t*), N = (2n - 1) pi,
    E = Wi/Re, alpha_N = 1 + beta E N^2, beta_N^2 = alpha_N^2 - 4 N^2 E,
    gamma_N = 1 + (beta - 2) N^2 E, G_N = exp(-alpha_N t*/(2 Wi)) {cosh | cos}(...).
    """
    ystar = np.asarray(ystar, dtype=np.float64)
    E = Wi / Re
    n = np.arange(1, nterms + 1, dtype=np.float64)
    N = (2.0 * n - 1.0) * math.pi
    alpha = 1.0 + beta * E * N * N
    b2 = alpha * alpha - 4.0 * N * N * E
    bN = np.sqrt(np.abs(b2))
    gamma = 1.0 + (beta - 2.0) * N * N * E
    arg = bN * tstar / (2.0 * Wi)
    decay = np.exp(-alpha * tstar / (2.0 * Wi))
    with np.errstate(over="ignore", invalid="ignore"):
        # growing cosh/sinh branch written as a difference of decaying exponentials
        ep = np.exp((-alpha + bN) * tstar / (2.0 * Wi))
        em = np.exp((-alpha - bN) * tstar / (2.0 * Wi))
        g_real = 0.5 * (ep + em) + gamma / np.where(bN > 0, bN, 1.0) * 0.5 * (ep - em)
        g_osc = decay * (np.cos(arg) + gamma / np.where(bN > 0, bN, 1.0) * np.sin(arg))
    G = np.where(b2 >= 0.0, g_real, g_osc)
    out = 4.0 * ystar * (1.0 - ystar)
    terms = np.sin(np.multiply.outer(ystar, N)) / N ** 3 * G
    return out - 32.0 * terms.sum(axis=-1)


def poiseuille_steady(ny, Uc, lam, wet=False):
    """Steady Oldroyd-B Poiseuille flow between half-way walls, height H = ny (Sec. 4.2),
    or between wet-node walls on rows 0 and ny - 1, height H = ny - 1.

    u = 4 U_c y'(H - y')/H^2 at y' = j + 1/2 (wet: y' = j); A_xy = lambda u',
    A_xx = 1 + 2 (lambda u')^2, A_yy = 1 (Kramers relation with tau_xy = eta_p u',
    tau_xx = 2 lambda eta_p u'^2).
    """
    H = float(ny - 1 if wet else ny)
    yp = np.arange(ny, dtype=np.float64) + (0.0 if wet else 0.5)
    u = 4.0 * Uc * yp * (H - yp) / H ** 2
    du = 4.0 * Uc * (H - 2.0 * yp) / H ** 2
    return dict(ux=u, axy=lam * du, axx=1.0 + 2.0 * (lam * du) ** 2, ayy=np.ones(ny), dudy=du)


def gre(a, b):
    """Global relative error sum|a - b| / sum|b| (Sec. 4.2)."""
    return float(np.abs(np.asarray(a) - np.asarray(b)).sum() / np.abs(np.asarray(b)).sum())


def four_roll_newtonian(N, Uc):
    """Steady Newtonian four-roll-mill field for the forcing F0(-sin x cos y, cos x sin y).

    Same field as the paper's steady solution shifted by pi in x (Sec. 4.1):
    u = U_c (-sin x~ cos y~, cos x~ sin y~).
    """
    xs = 2.0 * math.pi * np.arange(N) / N
    X, Y = np.meshgrid(xs, xs, indexing="xy")
    return -Uc * np.sin(X) * np.cos(Y), Uc * np.cos(X) * np.sin(Y)


# ---------------------------------------------------------------------------------
# Steady homogeneous simple shear u_x = gdot y of the constitutive closures (model
# function F(A), Sec. 2.2), Wi = lambda gdot.  With B = A - I the steady conformation
# equation reads, component by component,
#   F_r,xx = 2 Wi A_xy,   F_r,xy = Wi A_yy,   F_r,yy = 0,
# solved here in closed form or as one scalar equation per closure.
# ---------------------------------------------------------------------------------
def shear_conformation(model, mp, Wi):
    """(A_xx, A_xy, A_yy) of steady simple shear at Weissenberg number Wi (any sign)."""
    from scipy.optimize import brentq

    s = 1.0 if Wi >= 0 else -1.0
    W = abs(Wi)
    if W == 0.0:
        return 1.0, 0.0, 1.0
    if model == "oldroyd_b":
        axx, axy, ayy = 1 + 2 * W * W, W, 1.0
    elif model == "giesekus":
        # Giesekus' analytic solution: chi^2 = [sqrt(1 + 16 a (1 - a) Wi^2) - 1] /
        # [8 a (1 - a) Wi^2], f = (1 - chi) / (1 + (1 - 2a) chi); A_yy = 1 - f,
        # A_xy = Wi (1 - f)^2 / (1 + (1 - 2a) f), A_xx - A_yy = 2 f (1 - a f) / (a (1 - f)).
        a = mp
        if a == 0.0:
            return shear_conformation("oldroyd_b", 0.0, Wi)
        chi = math.sqrt((math.sqrt(1 + 16 * a * (1 - a) * W * W) - 1) / (8 * a * (1 - a) * W * W))
        f = (1 - chi) / (1 + (1 - 2 * a) * chi)
        ayy = 1 - f
        axy = W * (1 - f) ** 2 / (1 + (1 - 2 * a) * f)
        axx = ayy + 2 * f * (1 - a * f) / (a * (1 - f))
    elif model in ("lptt", "eptt"):
        # F_r = Y(tr A - 2) B: B_yy = 0, B_xy = Wi / Y, B_xx = 2 Wi^2 / Y^2 and
        # Y = 1 + eps B_xx (linear) or exp(eps B_xx) (exponential).
        e = mp

        def g(Y):
            bxx = 2 * W * W / (Y * Y)
            return (1 + e * bxx if model == "lptt" else math.exp(e * bxx)) - Y

        Y = brentq(g, 1.0, 1.0 + 2 * e * W * W + 1.0, xtol=1e-15, rtol=1e-15)
        axx, axy, ayy = 1 + 2 * W * W / (Y * Y), W / Y, 1.0
    elif model == "fene_p":
        # F_r = f A - I: A_yy = 1/f, A_xy = Wi / f^2, A_xx = (1 + 2 Wi^2 / f^2) / f with
        # f = (L^2 - 2) / (L^2 - tr A).
        L2 = mp

        def g(f):
            tr = (1 + 2 * W * W / (f * f)) / f + 1 / f
            return f * (L2 - tr) - (L2 - 2)

        f = brentq(g, 1.0, 1e6, xtol=1e-15, rtol=1e-15)
        axx, axy, ayy = (1 + 2 * W * W / (f * f)) / f, W / (f * f), 1 / f
    else:
        raise ValueError(model)
    return axx, s * axy, ayy


def shear_stress_function(model, mp, Wi):
    """F_s,xy of steady simple shear: the polymer shear stress is (eta_p / lambda) F_s,xy."""
    axx, axy, ayy = shear_conformation(model, mp, Wi)
    if model == "fene_p":
        f = (mp - 2) / (mp - axx - ayy)
        return f * axy
    return axy


def poiseuille_steady_model(ny, G, nu_s, eta_p, lam, model, mp):
    """Steady force-driven channel flow of a closure at the node centres y = j + 1/2
    between walls at y = 0 and y = ny (body force G along x, rho0 = 1, no diffusion of
    A).  The flow is locally simple shear, so the total shear stress
    nu_s gdot + (eta_p / lambda) F_s,xy(lambda gdot) = G (ny/2 - y) fixes gdot(y);
    u(y) is its integral from the wall and A(y) the shear conformation at gdot(y)."""
    from scipy.integrate import quad
    from scipy.optimize import brentq

    H = float(ny)

    def gdot(y):
        sig = G * (H / 2 - y)
        if sig == 0.0:
            return 0.0
        h = lambda g: nu_s * g + eta_p / lam * shear_stress_function(model, mp, lam * g) - sig  # noqa: E731
        hi = sig / nu_s
        return brentq(h, 0.0, hi, xtol=1e-17, rtol=1e-15) if sig > 0 else \
            brentq(h, hi, 0.0, xtol=1e-17, rtol=1e-15)

    ys = np.arange(ny) + 0.5
    u = np.array([quad(gdot, 0.0, y, epsabs=1e-14, epsrel=1e-12, limit=200)[0] for y in ys])
    A = np.array([shear_conformation(model, mp, lam * gdot(y)) for y in ys])
    return dict(ux=u, axx=A[:, 0], axy=A[:, 1], ayy=A[:, 2])
