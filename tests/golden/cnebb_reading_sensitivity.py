"""How much the confined-cylinder drag depends on two readings of the CNEBB scheme.

The boundary scheme (Sec. 3.3) leaves two points open that no closed form separates:
the velocity in the CNEBB equilibrium at a boundary node next to a half-way or curved
wall (reading A11: the node's own velocity with the half-force shift; alternative: the
wall's, zero) and the rebuild of an unknown population whose opposite is unknown too
(reading A12: the equilibrium alone; alternative: plus the non-equilibrium part of the
population that left in its own direction).  This script runs the FP64 oracle on the
paper's 30R x 4R cylinder channel (Sec. 4.3; Re = 1, beta = 0.59, Sc = 1e6) to the
steady criterion max |u(t + T_c) - u(t)| / U_c < 1e-8 under each reading and prints
C_d = F_x / (rho U_c^2 R) and its relative change.  It calls only the oracle.

    python tests/golden/cnebb_reading_sensitivity.py [R Wi ...]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402


def steady_cd(pr, flags, max_tstar=1000):
    o = oracle.OracleSim(pr, flags=flags)
    uc, tc = pr.meta["Uc"], pr.meta["Tc"]
    step = int(round(tc))
    prev = o.read()
    while o.time < max_tstar * tc:
        o.step(step)
        r = o.read()
        res = max(np.abs(r["ux"] - prev["ux"]).max(), np.abs(r["uy"] - prev["uy"]).max()) / uc
        prev = r
        if res < 1e-8:
            fx, fy = o.drag(0)
            return fx / (uc * uc * pr.meta["Lc"]), o.time / tc
        if not np.isfinite(res):
            return float("nan"), o.time / tc
    return float("nan"), o.time / tc


def main(cases):
    oracle.build(force=False)
    oracle.set_threads(min(16, oracle.max_threads()))
    readings = [("A11, A12 (used)", 0), ("A11 alternative: u_b = 0", oracle.FLAG_CNEBB_UB_ZERO),
                ("A12 alternative: pair keeps neq", oracle.FLAG_CNEBB_PAIR_NEQ)]
    for R, wi in cases:
        pr = synth.cylinder_channel(R=R, Wi=wi, Sc=1e6)
        ref = None
        for name, flags in readings:
            t0 = time.time()
            cd, ts = steady_cd(pr, flags)
            ref = cd if ref is None else ref
            print(f"R = {R:3d}  Wi = {wi:4.2f}  {name:34s} C_d = {cd:9.4f}  "
                  f"rel. change {cd / ref - 1:+.2e}  (steady at t* = {ts:.0f}, {time.time() - t0:.0f} s)",
                  flush=True)


if __name__ == "__main__":
    args = [float(a) for a in sys.argv[1:]]
    cases = [(int(args[i]), args[i + 1]) for i in range(0, len(args), 2)] or [(5, 0.5), (10, 0.1)]
    main(cases)
