"""Writes batch_5000.npz: oracle fields of eight runs of the batched workload after 5,000
steps (the step count of the batched configuration).

Calls only the FP64 oracle (oracle/) on runs of synth.batch_c4() (seed 16997: 256 runs,
sides N ~ U{32..512}, half Poiseuille channels and half four-roll mills, Wi = 10^U(-1, 2),
beta ~ U(0.1, 0.9)): eight runs with Wi <= 10 drawn with default_rng(7), the same draw
as the 500-step batch test.  Stores, per run, the fields at every 8th node in x and y plus
every 4th node of the first and last rows (the channel walls).
Run from the repository root: python tests/golden/make_batch_5000.py [threads]
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

STEPS = 5000
FIELDS = ("rho", "ux", "uy", "axx", "axy", "ayy")


def pick_runs():
    runs = synth.batch_c4()
    ok = [i for i, r in enumerate(runs) if r.meta["Wi"] <= 10.0]
    rng = np.random.default_rng(7)
    return sorted(rng.choice(ok, size=8, replace=False).tolist()), runs


def sample_nodes(pr):
    yy, xx = np.meshgrid(np.arange(pr.ny), np.arange(pr.nx), indexing="ij")
    pick = ((yy % 8 == 0) & (xx % 8 == 0)) | (((yy == 0) | (yy == pr.ny - 1)) & (xx % 4 == 0))
    ys, xs = np.nonzero(pick & pr.fluid_mask())
    return ys.astype(np.int32), xs.astype(np.int32)


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else os.cpu_count()
    oracle.build(force=False)
    oracle.set_threads(threads)
    pick, runs = pick_runs()
    out = {"steps": STEPS, "runs": np.array(pick, np.int32)}
    t0 = time.time()
    for i in pick:
        pr = runs[i]
        ys, xs = sample_nodes(pr)
        o = oracle.OracleSim(pr)
        for done in range(0, STEPS, 500):
            o.step(500)
            print(f"run {i} ({pr.nx}x{pr.ny}) {done + 500} steps, {time.time() - t0:.0f} s", flush=True)
        r = o.read()
        out[f"r{i}_ys"], out[f"r{i}_xs"] = ys, xs
        for k in FIELDS:
            out[f"r{i}_{k}"] = r[k][ys, xs].copy()
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "batch_5000.npz")
    np.savez_compressed(path, **out)
    print("wrote", path, pick)


if __name__ == "__main__":
    main()
