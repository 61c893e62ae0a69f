"""Autotuner: sweeps tile height, store mode, tile order and register budget, leaves the
state untouched, caches."""
import json

import numpy as np
import pytest

import synth
from gpu_util import FIELDS, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _exact(sim):
    import torch

    r = sim.read()
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in r.items()}


def test_autotune_sweeps_restores_and_caches(tmp_path):
    from paper_2508_16997_amd import Simulation
    from paper_2508_16997_amd.autotune import ORDERS, STORE_MODES, size_class, tune

    pr = synth.random_periodic(150, 70, seed=9, ymode="wall", precision="fp32")
    say("autotune", pr.nx, pr.ny)
    sim = Simulation.from_problem(pr, graph_chunk=10)
    ref = Simulation.from_problem(pr, graph_chunk=10)
    sim.step(7)
    ref.step(7)
    before = _exact(sim)
    cache = str(tmp_path / "tune.json")
    rec = tune(sim, steps=20, warmup=3, cache=cache)
    assert rec["tile"] in (1, 2, 4, 8) and rec["store_mode"] in (1, 2)
    assert rec["tile_order"] in (1, 2, 3) and rec["waves"] in (3, 4)
    assert len(rec["sweep_us"]) == 48 and len(rec["refine_us"]) == 4
    # the refined candidates are the sweep's four fastest; the lowest median wins
    fastest = sorted(rec["sweep_us"], key=rec["sweep_us"].get)[:4]
    assert set(rec["refine_us"]) == set(fastest)
    assert min(rec["refine_us"].values()) == rec["us_per_step"]
    key = f"{rec['tile']}/{STORE_MODES[rec['store_mode']]}/{ORDERS[rec['tile_order']]}/w{rec['waves']}"
    assert rec["refine_us"][key] == rec["us_per_step"]
    after = _exact(sim)
    for k in FIELDS:
        assert np.array_equal(before[k], after[k]), k
    assert sim.time == 7
    # tuned and untuned runs agree bit for bit
    sim.step(33)
    ref.step(33)
    a, b = _exact(sim), _exact(ref)
    for k in FIELDS:
        assert np.array_equal(a[k], b[k]), k
    data = json.load(open(cache))
    assert data[size_class(sim)]["tile"] == rec["tile"]
    # a cached class is applied without a sweep
    again = tune(sim, cache=cache)
    assert again == data[size_class(sim)]
    sim.close()
    ref.close()


def test_tune_batch_picks_a_tile_and_members_stay_exact():
    """tune_batch times one batch per tile height and form over the same members; the
    members then continue in a batch of the chosen shape bit-identically to runs stepped
    alone."""
    import torch
    from paper_2508_16997_amd import Batch, Simulation
    from paper_2508_16997_amd.autotune import tune_batch

    runs = [synth.random_periodic(70, 37, seed=3, ymode="wall", precision="fp32"),
            synth.random_periodic(40, 24, seed=4, precision="fp32")]
    stream = torch.cuda.Stream()
    say("tune_batch")
    members = [Simulation.from_problem(r, stream=stream) for r in runs]
    alone = [Simulation.from_problem(r, stream=stream) for r in runs]
    best, timings = tune_batch(members, tiles=(2, 4, 8), steps=6, warmup=2, graph_chunk=2,
                               forms=(False, True))
    ty, pers, order, waves = best
    expect = {(t, False, o, w) for t in (2, 4, 8) for o in (1, 2, 3) for w in (3, 4)}
    expect |= {(t, True, o, 0) for t in (2, 4, 8) for o in (1, 2, 3)}
    assert set(timings) == expect
    assert timings[best] == min(timings.values())
    done = len(expect) * (2 + 6)
    b = Batch(members, tile=ty, graph_chunk=2, persistent=pers, schedule=(order, waves))
    b.step(11)
    for s in alone:
        s.step(done + 11)
    stream.synchronize()
    for sb, ss in zip(members, alone):
        assert sb.time == ss.time == done + 11
        gb, gs = _exact(sb), _exact(ss)
        for k in FIELDS:
            assert np.array_equal(gb[k], gs[k]), k
    b.close()
    for s in members + alone:
        s.close()
