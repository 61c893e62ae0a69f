"""Build ``libvlb.so`` (the HIP library behind include/vlb.h) for gfx950 with hipcc.

Run ``python -m paper_2508_16997_amd.build`` or call :func:`build`.  The library is
written next to this file so that it travels with the source tree.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libvlb.so")
SOURCES = ["vlb_kernels.hip", "vlb_batch.hip", "vlb_fill.hip", "vlb_aux.hip", "vlb_adjoint.hip",
           "vlb3d.hip", "vlb3d_f64.hip", "vlb_api.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("VLB_OFFLOAD_ARCH", "gfx950")
ROCM_LIB = os.path.join(os.path.dirname(os.path.dirname(HIPCC)), "lib")

COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # packed FP32 instructions are kept out of every kernel on this platform
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]
PER_FILE = {
    # host geometry must be bit-reproducible: no fused multiply-add contraction
    "vlb_api.cpp": ["-x", "hip", "-ffp-contract=off"],
    # contraction decided per source expression, so every inlined copy of a device
    # function rounds identically (results independent of the tiling)
    "vlb_kernels.hip": ["-ffp-contract=on"],
    # machine-level loop-invariant code motion would hoist the FP64 constants of the
    # tile body out of the persistent tile loop and keep them live across it (spills)
    "vlb_batch.hip": ["-ffp-contract=on", "-mllvm", "-disable-machine-licm"],
    "vlb_fill.hip": ["-ffp-contract=on"],
    "vlb_adjoint.hip": ["-ffp-contract=on"],
    "vlb3d.hip": ["-ffp-contract=on", "-mllvm", "-pragma-unroll-threshold=1000000"],
    "vlb3d_f64.hip": ["-ffp-contract=on", "-mllvm", "-pragma-unroll-threshold=1000000"],
    "vlb_aux.hip": ["-ffp-contract=on"],
}


def compile_all(cmds, verbose: bool = False) -> None:
    """Run the per-source compiler commands side by side (each is its own process)."""
    workers = max(1, min(len(cmds), os.cpu_count() or 1, 8))
    with ThreadPoolExecutor(max_workers=workers) as pool:
        futs = []
        for cmd in cmds:
            if verbose:
                print(" ".join(cmd), flush=True)
            futs.append(pool.submit(subprocess.run, cmd, check=True))
        for f in futs:
            f.result()


def build(verbose: bool = False, out: str = LIB, defines=()) -> str:
    """Compile every source and link ``libvlb.so`` (or ``out``); returns its path.

    ``defines`` are extra -D tuning knobs of the kernels (e.g. VLB_WAVES_PER_EU=4).
    """
    if not os.path.exists(HIPCC) and shutil.which("hipcc") is None:
        raise RuntimeError("hipcc not found; the HIP library cannot be built")
    hipcc = HIPCC if os.path.exists(HIPCC) else shutil.which("hipcc")
    objdir = os.path.join(PKG, "_build", os.path.basename(out).replace(".so", ""))
    os.makedirs(objdir, exist_ok=True)
    objs, cmds = [], []
    for src in SOURCES:
        obj = os.path.join(objdir, src.replace(".", "_") + ".o")
        cmds.append([hipcc, *COMMON, *[f"-D{d}" for d in defines], *PER_FILE.get(src, []), "-c",
                     os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    compile_all(cmds, verbose)
    tmp = out + ".tmp"
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs,
           # roctx ranges around the entry points that enqueue device work
           f"-L{ROCM_LIB}", "-lrocprofiler-sdk-roctx", f"-Wl,-rpath,{ROCM_LIB}"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
