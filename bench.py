#!/usr/bin/env python3
"""Throughput of the coupled viscoelastic LB step on one MI355X.

Workload (default): simplified four-roll mill, 512 x 512 periodic, FP32, Wi = 5,
beta = 0.5, Stokes-Oldroyd-B set-up of the paper's Sec. 4.1 with synthetic (analytic)
fields.  One "step" is one coupled update: 1 hydrodynamic + 3 conformation D2Q9
lattices, every step of the hot path on the GPU.

Prints one JSON line with the metric (coupled MLUPS), the roofline of the step kernel
(algorithmic bytes per launch / average launch time from HIP events on the launch
stream, against the 8 TB/s HBM peak) and the FP64 oracle timed on the host's cores on
a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "coupled MLUPS (FP32) & % HBM roofline; batched vs single; adjoint/forward cost"
HBM_PEAK_GBS = 8000.0
ORDER_NAMES = {0: "automatic", 1: "xcd bands", 2: "row-major", 3: "column strips"}

# HBM bytes per k_step launch on a workload, from rocprofv3 counters (per dispatch, KiB):
# FETCH_SIZE counts half of the bytes a plain 1 GiB copy reads and WRITE_SIZE all it
# writes, so traffic = 2 * FETCH + WRITE.  Valid only for the kernel sources they were
# taken with (hash below) and the launch shape (tile height, store mode) the bench
# times; otherwise the bench reports null.
MEASURED_TRAFFIC = {
    "four_roll_512": [
        {"sources": "fe274e1098cea5b8", "tile": 8, "store_mode": "streaming",
         "tile_order": "xcd bands", "fetch_KiB": 25532.4, "write_KiB": 42147.2,
         "profile": "profiles/k_step_four_roll_512_cylinder_4096x1024_fp32_fetch_write.md"},
        {"sources": "fe274e1098cea5b8", "tile": 8, "store_mode": "cached",
         "tile_order": "xcd bands", "fetch_KiB": 25923.2, "write_KiB": 42128.0,
         "profile": "profiles/k_step_four_roll_512_cylinder_4096x1024_fp32_fetch_write.md"},
        {"sources": "fe274e1098cea5b8", "tile": 8, "store_mode": "streaming",
         "tile_order": "row-major", "fetch_KiB": 30198.8, "write_KiB": 42150.6,
         "profile": "profiles/k_step_four_roll_512_cylinder_4096x1024_fp32_fetch_write.md"},
        {"sources": "fe274e1098cea5b8", "tile": 8, "store_mode": "streaming",
         "tile_order": "column strips", "fetch_KiB": 30186.9, "write_KiB": 42150.6,
         "profile": "profiles/k_step_four_roll_512_cylinder_4096x1024_fp32_fetch_write.md"},
    ],
    "cylinder_4096x1024": [
        {"sources": "fe274e1098cea5b8", "tile": 4, "store_mode": "streaming",
         "tile_order": "row-major", "fetch_KiB": 440269.9, "write_KiB": 663801.3,
         "profile": "profiles/k_step_four_roll_512_cylinder_4096x1024_fp32_fetch_write.md"},
    ],
}
KERNEL_SOURCES = ("vlb_device.h", "vlb_internal.h", "vlb_step.h", "vlb_kernels.hip")


def kernel_sources_hash():
    import hashlib

    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2508_16997_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def auto_store_mode(pr, esz):
    """The library's automatic choice: streaming (non-temporal) stores once the two
    population buffers exceed 192 MiB, cached stores below."""
    return "streaming" if 2.0 * 36 * pr.nx * pr.ny * esz > 192.0 * 1024 * 1024 else "cached"


def autotuned_tile(sim):
    """Tile height picked (and applied, with its store mode) by the library's autotuner
    for this simulation: a sweep of tile heights and store modes outside any timed
    region, state saved and restored."""
    import tempfile

    from paper_2508_16997_amd.autotune import tune

    with tempfile.TemporaryDirectory() as d:
        rec = tune(sim, cache=os.path.join(d, "autotune.json"), force=True)
    sim.store_mode_name = "cached" if rec["store_mode"] == 1 else "streaming"
    sim.schedule_desc = {"tile_order": ORDER_NAMES[rec["tile_order"]],
                         "waves_per_simd": rec["waves"] or 3}
    return int(rec["tile"])


def measured_traffic(workload_name, tile, store_mode, tile_order):
    for rec in MEASURED_TRAFFIC.get(workload_name, []):
        if (rec["sources"] == kernel_sources_hash() and rec["tile"] == tile
                and rec["store_mode"] == store_mode and rec["tile_order"] == tile_order):
            return int(round((2.0 * rec["fetch_KiB"] + rec["write_KiB"]) * 1024))
    return None


def workload(name):
    import synth

    if name == "four_roll_512":
        pr = synth.four_roll_mill(N=512, steps=20000)
        desc = "four-roll mill 512x512 periodic, FP32, Wi=5, beta=0.5, Re=1, Sc=1e5"
    elif name == "cylinder_4096x1024":
        pr = synth.cylinder(Wi=1.0)
        desc = "channel flow past cylinder 4096x1024, R=128, FP32, Wi=1, beta=0.59, Sc=1e6"
    elif name == "poiseuille_64x32_fp64":
        pr = synth.poiseuille()
        desc = "Oldroyd-B Poiseuille 64x32, FP64, Wi=1, beta=0.5"
    else:
        raise SystemExit(f"unknown workload {name}")
    return pr, desc


def bytes_per_node(esz):
    """Algorithmic HBM bytes of one coupled node update: one read and one write of the 36
    populations and of the 5 history values (S and u of the previous step), 328 B in
    FP32 storage and 656 B in FP64."""
    return 2 * 36 * esz + 2 * 5 * esz


def extra_bytes_per_node(pr, esz):
    """Bytes a node update also reads on some workloads, kept out of the roofline figure:
    the per-node body force (four-roll mill) and the 2-byte geometry word of walled or
    obstructed grids."""
    return {"force": 0 if pr.uniform_force() else 2 * esz,
            "geometry": 2 if (pr.ymode in ("wall", "wet") or pr.xmode == "wall" or pr.circles
                              or pr.solid is not None) else 0}


def copy_bandwidth(nbytes=1 << 30, reps=20):
    """Achievable HBM bandwidth: a plain device-to-device copy of nbytes (GB/s)."""
    import torch

    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    s = e0.elapsed_time(e1) / 1e3 / reps
    return 2.0 * nbytes / s / 1e9


def cylinder_leg(steps, warmup, tile, chunk, cpu_steps=0):
    """Channel flow past a cylinder, 4096 x 1024, FP32 storage: a working set (1.4 GB)
    far beyond the last-level cache, so its rate is an HBM rate."""
    import torch
    import synth
    from paper_2508_16997_amd import Simulation

    pr = synth.cylinder(Wi=1.0)
    stream = torch.cuda.Stream()
    sim = Simulation.from_problem(pr, stream=stream, tile=tile or 4, graph_chunk=chunk)
    tile = tile or autotuned_tile(sim)
    nodes = int(pr.fluid_mask().sum())
    sim.step(warmup)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    sim.step(steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_s = ev0.elapsed_time(ev1) / 1e3 / steps
    bad = sim.monitors(raise_on_nonfinite=False)["nonfinite"]
    sim.close()
    bpn = bytes_per_node(4)
    achieved = bpn * nodes / step_s / 1e9
    out = {"workload": "channel flow past a cylinder 4096x1024, R=128, FP32 storage, Wi=1",
           "fluid_nodes": nodes, "steps": steps, "MLUPS": round(nodes * steps / wall / 1e6, 2),
           "us_per_step": round(step_s * 1e6, 3), "bytes_per_node": bpn,
           "extra_bytes_per_node": extra_bytes_per_node(pr, 4),
           "achieved_GBs": round(achieved, 1), "frac": round(achieved / HBM_PEAK_GBS, 4),
           "frac_basis": "328 B per fluid node over the whole step (k_step + k_fill, HIP "
                         "events on the launch stream); the working set (1.4 GB) is HBM "
                         "resident, so this is the gating HBM fraction",
           "tile": f"64x{tile}", **getattr(sim, "schedule_desc", {}),
           "traffic": measured_traffic("cylinder_4096x1024", tile,
                                       getattr(sim, "store_mode_name", None) or auto_store_mode(pr, 4),
                                       getattr(sim, "schedule_desc", {}).get("tile_order")),
           "nonfinite": int(bad)}
    if cpu_steps:
        out["cpu_baseline"] = cpu_baseline_steps([pr], cpu_steps, "the same 4096x1024 workload")
    return out


def batched_leg(steps, warmup, tile, chunk, forms=(False, True), cpu_steps=0):
    """Batched workload (256 uneven runs advanced together) vs the same runs one by one.

    The batch is timed in both forms (one step launch and one fill launch per step under
    hipGraph replay, or the persistent cooperative launch of up to 256 steps), each at
    its autotuned tile; the faster is the batched figure.  The sequential leg steps each
    run alone for the same number of steps, back to back, with hipGraph replay.
    ``forms`` limits the forms (a kernel trace of the per-step form alone, say).
    """
    import torch
    import synth
    from paper_2508_16997_amd import Batch, Simulation

    runs = synth.batch_c4()
    stream = torch.cuda.Stream()
    sims = [Simulation.from_problem(r, stream=stream, tile=tile or 4, graph_chunk=chunk)
            for r in runs]
    nodes = sum(int(r.fluid_mask().sum()) for r in runs)
    from paper_2508_16997_amd.autotune import tune_batch

    # both batched forms, each at its fastest tile (or the tile given); the faster one
    # is the batched figure, the other is reported beside it
    best, tuned = tune_batch(sims, tiles=(tile,) if tile else (2, 4, 8), graph_chunk=chunk,
                             forms=tuple(forms))
    tile, pers = best[0], best[1]

    def timed_batch(ty, persistent, order, waves):
        b = Batch(sims, tile=ty, graph_chunk=0 if persistent else chunk, persistent=persistent,
                  schedule=(order, waves))
        b.step(warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.step(steps)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        b.close()
        return t

    t_batch = timed_batch(*best)
    others = [k for k in tuned if k[1] != pers]
    other = min(others, key=tuned.get) if others else None
    t_other = timed_batch(*other) if other else None
    for s in sims:  # warm the per-run graphs
        s.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in sims:
        s.step(steps)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    bad = sum(s.monitors(raise_on_nonfinite=False)["nonfinite"] > 0 for s in sims)
    step_bytes = bytes_per_node(4) * nodes
    for s in sims:
        s.close()
    out = {"runs": len(runs), "nodes": nodes, "steps": steps,
            "batched_MLUPS": round(nodes * steps / t_batch / 1e6, 2),
            "sequential_MLUPS": round(nodes * steps / t_seq / 1e6, 2),
            "batched_vs_sequential": round(t_seq / t_batch, 3),
            "batched_GBs": round(step_bytes * steps / t_batch / 1e9, 1),
            "batched_frac": round(step_bytes * steps / t_batch / 1e9 / HBM_PEAK_GBS, 4),
            "tile": f"64x{tile}", "form": "persistent" if pers else "per-step launches",
            "tile_order": ORDER_NAMES[best[2]],
            "waves_per_simd": best[3] or 3,
            "other_form": None if other is None else {
                "form": "persistent" if other[1] else "per-step launches",
                "tile": f"64x{other[0]}", "tile_order": ORDER_NAMES[other[2]],
                "MLUPS": round(nodes * steps / t_other / 1e6, 2)},
            "runs_nonfinite": int(bad)}
    if cpu_steps:
        import numpy as np

        pick = sorted(np.random.default_rng(7).choice(len(runs), size=8, replace=False).tolist())
        out["cpu_baseline"] = cpu_baseline_steps(
            [runs[i] for i in pick], cpu_steps,
            f"8 runs of the batched set (indices {pick}, drawn with default_rng(7))")
    return out


def adjoint_leg(steps, stride, tile, chunk):
    """Adjoint workload: gradients of the velocity misfit after `steps` steps.

    Times the plain forward, the checkpointed forward and the backward pass (seed,
    segment recompute, reverse sweep).  The per-step adjoint cost is the backward time
    less the recompute (steps - segments forward steps at the measured forward rate).
    """
    import math

    import torch
    import synth
    from paper_2508_16997_amd import Simulation

    pr, hidden = synth.adjoint_c5(steps=steps)
    stream = torch.cuda.Stream()
    tgt_sim = Simulation.from_problem(
        pr.with_(lam=hidden["lam"], eta_p=hidden["eta_p"], Fx=hidden["Fx"], Fy=hidden["Fy"]),
        stream=stream, tile=tile, graph_chunk=chunk)
    tgt_sim.step(steps)
    tgt = tgt_sim.read()
    tx, ty = tgt["ux"].clone(), tgt["uy"].clone()
    tgt_sim.close()
    sim = Simulation.from_problem(pr, stream=stream, tile=tile, graph_chunk=chunk)
    s0 = sim.save_state()
    sim.adjoint(min(steps, 2 * stride), tx, ty, stride=stride)  # warm-up (graphs, workspace)
    torch.cuda.synchronize()

    def timed(fn):
        sim.load_state(s0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0, r

    t_fwd, _ = timed(lambda: sim.step(steps))
    t_afwd, _ = timed(lambda: sim.adjoint_forward(steps, stride))
    t_all, g = timed(lambda: sim.adjoint(steps, tx, ty, stride=stride))
    nseg = math.ceil(steps / stride)
    step_s = t_fwd / steps
    t_bwd = t_all - t_afwd
    recompute = (steps - nseg) * step_s
    adj_step = (t_bwd - recompute) / steps
    ws = sim.adjoint_workspace_bytes(steps, stride)
    sim.close()
    return {"workload": f"four-roll mill {pr.nx}x{pr.ny} FP32, hidden-parameter target",
            "steps": steps, "stride": stride, "workspace_GB": round(ws / 1e9, 3),
            "forward_ms": round(t_fwd * 1e3, 3),
            "checkpointed_forward_ms": round(t_afwd * 1e3, 3),
            "backward_ms": round(t_bwd * 1e3, 3),
            "forward_step_us": round(step_s * 1e6, 3),
            "adjoint_step_us": round(adj_step * 1e6, 3),
            "adjoint_vs_forward": round(adj_step / step_s, 3),
            "recompute_fraction_of_backward": round(recompute / t_bwd, 3),
            "gradient_vs_forward_wall": round((t_afwd + t_bwd) / t_fwd, 3),
            "loss": g["loss"], "dL_dlambda": g["dlambda"], "dL_deta_p": g["deta_p"]}


def _oracle_rate(pr, seconds, threads):
    import oracle

    oracle.set_threads(threads)
    o = oracle.OracleSim(pr)
    t0 = time.perf_counter()
    o.step(1)
    t1 = time.perf_counter() - t0
    n = max(1, int(seconds / max(t1, 1e-6)))
    t0 = time.perf_counter()
    o.step(n)
    dt = time.perf_counter() - t0
    nodes = int(pr.fluid_mask().sum())
    return nodes * n / dt / 1e6, n, dt, oracle.max_threads()


def cpu_baseline_steps(problems, steps, what):
    """The FP64 oracle on all host cores (up to 16) for a fixed number of steps of each
    problem, one after another: the coupled MLUPS of that sample."""
    import oracle

    oracle.build(force=False)
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    oracle.set_threads(max(1, min(cores, 16)))
    node_steps, dt = 0, 0.0
    for pr in problems:
        o = oracle.OracleSim(pr)
        t0 = time.perf_counter()
        o.step(steps)
        dt += time.perf_counter() - t0
        node_steps += int(pr.fluid_mask().sum()) * steps
        del o
    return {"value": node_steps / dt / 1e6, "unit": "MLUPS", "cores": oracle.max_threads(),
            "kind": "oracle",
            "sample": f"{steps} coupled FP64 steps of {what}, {dt:.1f} s"}


def cpu_baseline(pr, seconds):
    """The FP64 oracle as it stands, on all host cores (up to 16) and on one core."""
    import oracle

    oracle.build(force=False)
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    cores = max(1, min(cores, 16))
    v, n, dt, used = _oracle_rate(pr, seconds, cores)
    v1, n1, dt1, _ = _oracle_rate(pr, seconds / 3.0, 1)
    return {"value": v, "unit": "MLUPS", "cores": used, "kind": "oracle",
            "sample": f"{n} coupled FP64 steps of the same {pr.nx}x{pr.ny} workload "
                      f"(after 1 untimed step), {dt:.1f} s; one core: {n1} steps, {dt1:.1f} s",
            "value_1_core": v1}


def d3_leg(steps, warmup, cpu_steps=0, q=19):
    """Three-dimensional form on D3Q19 (q = 19) or D3Q27 (q = 27): force-driven Oldroyd-B
    channel 256 x 64 x 256 (4.2 M nodes, half-way walls normal to y), FP32 storage.
    Algorithmic bytes per node and step: 7 q populations read and written (7 lattices)
    and the history of S (6) and u (3) read and written: 2 x (7 q + 9) x 4 = 1,136 B on
    D3Q19, 1,584 B on D3Q27; the rho/u planes of the neighbour differences (16 B written,
    16 B read) and the 4 q B of hydrodynamic pulls of the rho/u launch are reported beside
    it.  HIP events on the simulation's stream bracket both launches of every step."""
    import torch
    import synth
    from paper_2508_16997_amd.sim3d import Simulation3D

    pr = synth.channel3d(nx=256, ny=64, nz=256, Ma=0.1, precision="fp32", q=q)
    stream = torch.cuda.Stream()
    sim = Simulation3D.from_problem(pr, stream=stream)
    sim.step(warmup)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    sim.step(steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_s = ev0.elapsed_time(ev1) / 1e3 / steps
    r = sim.read()
    torch.cuda.synchronize()
    finite = bool(torch.isfinite(r["ux"]).all())
    sim.close()
    nodes = pr.nx * pr.ny * pr.nz
    bpn = 2 * (7 * q + 9) * 4
    achieved = bpn * nodes / step_s / 1e9
    out = {"workload": f"D3Q{q} Oldroyd-B channel 256x64x256, half-way walls in y, FP32 storage, "
                       "Wi=1, beta=0.5",
           "nodes": nodes, "steps": steps, "MLUPS": round(nodes * steps / wall / 1e6, 2),
           "us_per_step": round(step_s * 1e6, 3), "bytes_per_node": bpn,
           "extra_bytes_per_node": {"rho_u_planes": 32, "rho_u_launch_pulls": 4 * q},
           "achieved_GBs": round(achieved, 1), "frac": round(achieved / HBM_PEAK_GBS, 4),
           "kernels": "k3_macro + k3_step", "finite": finite}
    if cpu_steps:
        import oracle

        oracle.build(force=False)
        oracle.set_threads(os.cpu_count() or 1)
        o = oracle.OracleSim3D(pr)
        t = time.perf_counter()
        o.step(cpu_steps)
        dt = time.perf_counter() - t
        out["cpu_baseline"] = {"value": round(nodes * cpu_steps / dt / 1e6, 3), "unit": "MLUPS",
                               "cores": os.cpu_count() or 1, "kind": "oracle",
                               "sample": f"{cpu_steps} coupled FP64 steps of the same "
                                         f"256x64x256 D3Q{q} channel, {dt:.1f} s"}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", default="four_roll_512",
                    choices=["four_roll_512", "cylinder_4096x1024", "poiseuille_64x32_fp64"])
    ap.add_argument("--tile", type=int, default=0,
                    help="tile height of the step kernel (64 x TY threads); 0 = autotune "
                         "each leg before its timed region")
    ap.add_argument("--store-mode", choices=["auto", "cached", "streaming"], default="auto",
                    help="stores of the step kernel when --tile is fixed (the autotuner picks "
                         "its own)")
    ap.add_argument("--schedule", default="",
                    help="ORDER,WAVES of the step kernel when --tile is fixed (tile order 1 = "
                         "XCD bands, 2 = row-major, 3 = column strips; 3 or 4 waves per SIMD); "
                         "default automatic")
    ap.add_argument("--graph-chunk", type=int, default=50)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-cylinder-steps", type=int, default=50,
                    help="oracle steps of the cylinder for its CPU baseline (0: none)")
    ap.add_argument("--cpu-batched-steps", type=int, default=500,
                    help="oracle steps of each of 8 sampled batched runs (0: none)")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched-vs-sequential leg (256 uneven runs)")
    ap.add_argument("--batched-steps", type=int, default=200)
    ap.add_argument("--batched-form", choices=["both", "per-step", "persistent"],
                    default="both", help="batched forms to time (default both)")
    ap.add_argument("--no-cylinder", action="store_true",
                    help="skip the 4096x1024 cylinder leg")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the adjoint leg (512x512, gradient of a velocity misfit)")
    ap.add_argument("--adjoint-steps", type=int, default=2000)
    ap.add_argument("--adjoint-stride", type=int, default=45)
    ap.add_argument("--no-3d", action="store_true",
                    help="skip the three-dimensional (D3Q19) leg")
    ap.add_argument("--d3-steps", type=int, default=200)
    ap.add_argument("--cpu-3d-steps", type=int, default=2,
                    help="oracle steps of the 3-D channel for its CPU baseline (0: none)")
    ap.add_argument("--copy-only", action="store_true",
                    help="only time a plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (asked for {max(args.gpus, world)}): the "
              "coupled step runs on a single GPU; a slab decomposition across GPUs is not "
              "implemented", file=sys.stderr)
        return 2

    import torch

    if args.copy_only:
        print(json.dumps({"copy_GBs": round(copy_bandwidth(), 1), "bytes": 2 * (1 << 30)}))
        return 0

    from paper_2508_16997_amd import Simulation

    pr, desc = workload(args.workload)
    prec = pr.precision
    esz = 4 if prec == "fp32" else 8
    stream = torch.cuda.Stream()
    sim = Simulation.from_problem(pr, stream=stream, tile=args.tile or 4,
                                  graph_chunk=args.graph_chunk)
    tile = args.tile or autotuned_tile(sim)
    if args.tile and args.store_mode != "auto":
        sim.set_store_mode(1 if args.store_mode == "cached" else 2)
        sim.store_mode_name = args.store_mode
    if args.tile and args.schedule:
        order, waves = (int(v) for v in args.schedule.split(","))
        sim.set_schedule(order, waves)
        sim.schedule_desc = {"tile_order": ORDER_NAMES[order],
                             "waves_per_simd": waves}
    store_mode = getattr(sim, "store_mode_name", None) or auto_store_mode(pr, esz)
    nodes = int(pr.fluid_mask().sum())
    sim.step(args.warmup)
    torch.cuda.synchronize()

    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    sim.step(args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)

    mon = sim.monitors()
    if mon["nonfinite"]:
        print("non-finite fields after the timed steps", file=sys.stderr)
        return 3
    copy_gbs = copy_bandwidth()

    mlups = nodes * args.steps / wall / 1e6
    bpn = bytes_per_node(esz)
    extra = extra_bytes_per_node(pr, esz)
    launch_s = gpu_ms / 1e3 / args.steps
    bytes_launch = bpn * nodes
    achieved = bytes_launch / launch_s / 1e9
    achieved_all = (bpn + sum(extra.values())) * nodes / launch_s / 1e9
    out = {
        "metric": METRIC,
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",  # arithmetic type; storage below

        "data": "synthetic",
        "config": {"workload": desc, "storage": "f32" if prec == "fp32" else "f64",
                   "nx": pr.nx, "ny": pr.ny, "fluid_nodes": nodes,
                   "bytes_per_node": bpn, "extra_bytes_per_node": extra, "tile": f"64x{tile}",
                   "store_mode": store_mode,
                   "tile_choice": "fixed" if args.tile else "autotuned",
                   **getattr(sim, "schedule_desc", {}),
                   "graph_chunk_steps": 2 * args.graph_chunk},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(args.workload, tile, store_mode,
                                                 getattr(sim, "schedule_desc", {}).get("tile_order")),
                     "kernel": "k_step",
                     "avg_launch_us": round(launch_s * 1e6, 3),
                     "bytes_per_launch": bytes_launch,
                     "achieved_with_extra_reads": round(achieved_all, 1),
                     "copy_ceiling_GBs": round(copy_gbs, 1),
                     "frac_of_copy": round(achieved / copy_gbs, 4)},
    }
    sim.close()
    if not args.no_cylinder:
        out["cylinder"] = cylinder_leg(1000, 100, args.tile, args.graph_chunk,
                                       0 if args.no_cpu_baseline else args.cpu_cylinder_steps)
    if not args.no_batched:
        forms = {"both": (False, True), "per-step": (False,), "persistent": (True,)}
        out["batched"] = batched_leg(args.batched_steps, 2 * args.graph_chunk + 1, args.tile,
                                     args.graph_chunk, forms[args.batched_form],
                                     0 if args.no_cpu_baseline else args.cpu_batched_steps)
    if not args.no_adjoint:
        out["adjoint"] = adjoint_leg(args.adjoint_steps, args.adjoint_stride, tile,
                                     args.graph_chunk)
    if not args.no_3d:
        out["d3q19"] = d3_leg(args.d3_steps, 20, 0 if args.no_cpu_baseline else args.cpu_3d_steps)
        out["d3q27"] = d3_leg(args.d3_steps, 20, 0, q=27)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(pr, args.cpu_seconds)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
