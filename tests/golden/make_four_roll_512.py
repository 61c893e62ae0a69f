"""Writes four_roll_512_20k.npz: oracle fields of the 512^2 four-roll mill after 20k steps.

Calls only the FP64 oracle (oracle/) on the seeded workload of synth.four_roll_mill
(Wi = 5, beta = 0.5, FP32 configuration of the benchmark; the oracle runs in FP64).
Stores every 8th node in x and y (64 x 64 samples per field) to keep the file small.
Run from the repository root: python tests/golden/make_four_roll_512.py [threads]
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

STRIDE = 8
STEPS = 20000


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else os.cpu_count()
    oracle.build(force=False)
    oracle.set_threads(threads)
    pr = synth.four_roll_mill(N=512, steps=STEPS)
    o = oracle.OracleSim(pr)
    t0 = time.time()
    done = 0
    while done < STEPS:
        n = min(1000, STEPS - done)
        o.step(n)
        done += n
        print(f"{done} steps, {time.time() - t0:.0f} s", flush=True)
    r = o.read()
    out = {k: v[::STRIDE, ::STRIDE].copy() for k, v in r.items()}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "four_roll_512_20k.npz")
    np.savez_compressed(path, stride=STRIDE, steps=STEPS, **out)
    print("wrote", path)


if __name__ == "__main__":
    main()
