"""Launch-shape autotuner for the step kernel.

For a simulation it times every tile height (64 x TY threads, TY in 1, 2, 4, 8), both
store modes (cached, non-temporal), the three tile orders (XCD bands, row-major, column
strips) and, for
single-precision storage, both register budgets of the step kernel (three or four
waves per SIMD) with HIP events on the simulation's stream, times the few fastest
again (interleaved repetitions, median), keeps the fastest, and caches the choice per size class in a JSON file (``VLB_AUTOTUNE_CACHE`` or
``~/.cache/paper_2508_16997_amd/autotune.json``).  The simulation's state is saved
before and restored after the sweep, so tuning does not advance it.  Results do not
depend on any of these choices (bit-identical by test).
"""
from __future__ import annotations

import json
import os
from typing import Optional

import torch

TILES = (1, 2, 4, 8)
STORE_MODES = {1: "cached", 2: "streaming"}
ORDERS = {1: "xcd", 2: "rows", 3: "strips"}
CACHE_VERSION = "v3"  # records of an earlier search or decision rule are not reused


def waves_for(precision) -> tuple:
    """Register budgets worth sweeping: FP32 storage has two, FP64 one."""
    return (3, 4) if precision == "fp32" else (0,)


def cache_path() -> str:
    p = os.environ.get("VLB_AUTOTUNE_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "paper_2508_16997_amd", "autotune.json")


def size_class(sim) -> str:
    """Key of the cache: precision, grid, boundary kinds, solids."""
    solid = "solid" if (sim._mask is not None and sim._mask.any()) or sim._circ.size else "open"
    return f"{CACHE_VERSION}:{sim.precision}:{sim.nx}x{sim.ny}:{sim.xmode}/{sim.ymode}:{solid}"


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path, data):
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def time_step(sim, steps: int) -> float:
    """Average device time of one step (seconds) over ``steps`` steps."""
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(sim.stream)
    sim.step(steps)
    e1.record(sim.stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / 1e3 / steps


def tune(sim, steps: int = 60, warmup: int = 10, cache: Optional[str] = None,
         force: bool = False, refine: int = 4) -> dict:
    """Pick and apply the fastest (tile, store mode, tile order, waves) for ``sim``;
    returns the record.  The ``refine`` fastest of the sweep are timed again (three
    interleaved repetitions of 4 x ``steps`` steps) and the lowest median wins."""
    path = cache or cache_path()
    data = _load(path)
    key = size_class(sim)
    if not force and key in data:
        rec = data[key]
        sim.set_tile(rec["tile"])
        sim.set_store_mode(rec["store_mode"])
        sim.set_schedule(rec["tile_order"], rec["waves"])
        return rec
    state = sim.save_state()
    timings = {}
    for ty in TILES:
        for mode in STORE_MODES:
            for order in ORDERS:
                for waves in waves_for(sim.precision):
                    sim.load_state(state)
                    sim.set_tile(ty)
                    sim.set_store_mode(mode)
                    sim.set_schedule(order, waves)
                    sim.step(warmup)
                    timings[(ty, mode, order, waves)] = time_step(sim, steps)
    # the few fastest of the sweep again, interleaved and longer, so that one noisy
    # timing does not decide: the lowest median of three repetitions wins
    finalists = sorted(timings, key=timings.get)[:refine]
    reps = {c: [] for c in finalists}
    for _ in range(3):
        for c in finalists:
            sim.load_state(state)
            sim.set_tile(c[0])
            sim.set_store_mode(c[1])
            sim.set_schedule(c[2], c[3])
            sim.step(warmup)
            reps[c].append(time_step(sim, 4 * steps))
    med = {c: sorted(v)[1] for c, v in reps.items()}
    (ty, mode, order, waves), best = min(med.items(), key=lambda kv: kv[1])
    sim.load_state(state)
    sim.set_tile(ty)
    sim.set_store_mode(mode)
    sim.set_schedule(order, waves)
    rec = {"tile": ty, "store_mode": mode, "tile_order": order, "waves": waves,
           "us_per_step": round(best * 1e6, 3),
           "sweep_us": {f"{t}/{STORE_MODES[m]}/{ORDERS[o]}/w{w}": round(v * 1e6, 3)
                        for (t, m, o, w), v in timings.items()},
           "refine_us": {f"{t}/{STORE_MODES[m]}/{ORDERS[o]}/w{w}": round(v * 1e6, 3)
                         for (t, m, o, w), v in med.items()}}
    data[key] = rec
    _store(path, data)
    return rec


def tune_batch(sims, tiles=TILES, steps: int = 20, warmup: int = 5, graph_chunk: int = 0,
               forms=(False,)):
    """Time one batch per (tile height, form, tile order, waves) over the same members and
    return (fastest (tile, persistent, order, waves), {that key: seconds per step}).
    ``forms`` lists the forms to try: False = one step launch and one fill launch per step
    (hipGraph replay when graph_chunk > 0), True = the persistent cooperative launch
    (its register budget is fixed, so waves is not swept for it).  The members advance by
    warmup + steps steps per configuration; results do not depend on the choice."""
    from .sim import Batch

    timings = {}
    for ty in tiles:
        for pers in forms:
            for order in ORDERS:
                for waves in ((0,) if pers else waves_for(sims[0].precision)):
                    b = Batch(sims, tile=ty, graph_chunk=0 if pers else graph_chunk,
                              persistent=pers, schedule=(order, waves))
                    b.step(warmup)
                    e0 = torch.cuda.Event(enable_timing=True)
                    e1 = torch.cuda.Event(enable_timing=True)
                    e0.record(b.stream)
                    b.step(steps)
                    e1.record(b.stream)
                    e1.synchronize()
                    timings[(ty, bool(pers), order, waves)] = e0.elapsed_time(e1) / 1e3 / steps
                    b.close()
    best = min(timings, key=timings.get)
    return best, timings
