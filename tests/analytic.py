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


def poiseuille_steady(ny, Uc, lam):
    """Steady Oldroyd-B Poiseuille flow between half-way walls, height H = ny (Sec. 4.2).

    u = 4 U_c y'(H - y')/H^2 at y' = j + 1/2; A_xy = lambda u', A_xx = 1 + 2 (lambda u')^2,
    A_yy = 1 (Kramers relation with tau_xy = eta_p u', tau_xx = 2 lambda eta_p u'^2).
    """
    H = float(ny)
    yp = np.arange(ny, dtype=np.float64) + 0.5
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
