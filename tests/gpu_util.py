"""Helpers shared by the GPU tests: run the HIP path and the oracle on one problem."""
from __future__ import annotations

import sys

import numpy as np

FIELDS = ("rho", "ux", "uy", "axx", "axy", "ayy")


def say(*a):
    """Name the case before a GPU step, flushed, so a fault still tells which it was."""
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def gpu_fields(sim) -> dict:
    import torch

    r = sim.read()
    torch.cuda.synchronize()
    return {k: v.double().cpu().numpy() for k, v in r.items()}


def rel_l2(a, b, mask):
    """||a - b||_2 / ||b||_2 over fluid nodes (0 when both vanish)."""
    d = np.sqrt(((a - b)[mask] ** 2).sum())
    n = np.sqrt((b[mask] ** 2).sum())
    if n == 0.0:
        return float(d)
    return float(d / n)


def parity(g: dict, o: dict, mask) -> dict:
    """Relative L2 errors: u as a vector, each conformation component, rho - 1."""
    du = np.sqrt(((g["ux"] - o["ux"]) ** 2 + (g["uy"] - o["uy"]) ** 2)[mask].sum())
    nu = np.sqrt((o["ux"] ** 2 + o["uy"] ** 2)[mask].sum())
    out = {"u": float(du / nu) if nu > 0 else float(du)}
    for k in ("axx", "axy", "ayy"):
        out[k] = rel_l2(g[k], o[k], mask)
    out["rho"] = rel_l2(g["rho"] - 1.0, o["rho"] - 1.0, mask)
    return out


def run_pair(prob, steps, precision=None, dual_chunks=None, sim_kw=None):
    """Run the HIP path and the oracle for ``steps`` steps; return both field dicts."""
    import oracle
    from paper_2508_16997_amd import Simulation

    sim = Simulation.from_problem(prob, precision=precision, **(sim_kw or {}))
    o = oracle.OracleSim(prob)
    chunks = dual_chunks or [steps]
    for c in chunks:
        sim.step(c)
        o.step(c)
    g = gpu_fields(sim)
    r = o.read()
    sim.close()
    return g, r
