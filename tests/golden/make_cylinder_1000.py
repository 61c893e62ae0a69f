"""Writes cylinder_1000.npz (Wi = 1) or cylinder_1000_wi<Wi>.npz: oracle fields of the
4096 x 1024 cylinder after 1,000 steps.

Calls only the FP64 oracle (oracle/) on the seeded workload of synth.cylinder (R = 128 at
(2048, 512), Wi in {0.5, 1, 2}, beta = 0.59, Sc = 1e6; the FP32 configuration of the
benchmark, run in FP64 by the oracle).  Stores the fields at a sample of nodes: every 32nd node in x and
y, every fluid node within two lattice units of the cylinder surface (curved links and
CNEBB), every 8th node of the first and last fluid rows (channel walls) and of the first
and last columns (inlet and outlet).
Run from the repository root: python tests/golden/make_cylinder_1000.py [threads] [Wi]
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

STEPS = 1000


def sample_nodes(pr):
    ny, nx = pr.ny, pr.nx
    fluid = pr.fluid_mask()
    yy, xx = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    pick = (yy % 32 == 0) & (xx % 32 == 0)
    xc, yc, R = pr.circles[0]
    d = np.sqrt((xx - xc) ** 2 + (yy - yc) ** 2)
    pick |= (d <= R + 2.0)
    pick |= ((yy == 0) | (yy == ny - 1)) & (xx % 8 == 0)
    pick |= ((xx == 0) | (xx == nx - 1)) & (yy % 8 == 0)
    pick &= fluid
    ys, xs = np.nonzero(pick)
    return ys.astype(np.int32), xs.astype(np.int32)


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else os.cpu_count()
    WI = float(sys.argv[2]) if len(sys.argv) > 2 else 1.0
    oracle.build(force=False)
    oracle.set_threads(threads)
    pr = synth.cylinder(Wi=WI)
    ys, xs = sample_nodes(pr)
    o = oracle.OracleSim(pr)
    t0 = time.time()
    done = 0
    while done < STEPS:
        n = min(50, STEPS - done)
        o.step(n)
        done += n
        print(f"{done} steps, {time.time() - t0:.0f} s", flush=True)
    r = o.read()
    out = {k: v[ys, xs].copy() for k, v in r.items()}
    name = "cylinder_1000.npz" if WI == 1.0 else f"cylinder_1000_wi{WI:g}.npz"
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), name)
    np.savez_compressed(path, steps=STEPS, wi=WI, ys=ys, xs=xs, **out)
    print("wrote", path, len(ys), "nodes")


if __name__ == "__main__":
    main()
