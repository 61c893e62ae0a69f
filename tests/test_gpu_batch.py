"""Batched form: many runs advanced by one step launch and one boundary launch per step.

Every batched run must be bit-identical to the same run stepped alone (the kernels are
the same; only the work list differs), and a sample of runs is checked against the FP64
oracle at the FP32 bar (relative L2 <= 1e-5).  The run set follows the batched workload:
half Poiseuille channels, half four-roll mills, side N ~ U{32..512}, Wi = 10^U(-1, 2),
beta ~ U(0.1, 0.9), all drawn from one seeded generator.
"""
import numpy as np
import pytest

import synth
from gpu_util import FIELDS, gpu_fields, parity, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle

    oracle.build(force=False)
    oracle.set_threads(min(16, oracle.max_threads()))


def _mixed_set(precision):
    """Small uneven runs of every boundary kind the step supports."""
    mask = np.zeros((37, 70), np.uint8)
    mask[10:15, 20:24] = 1
    runs = [r.with_(precision=precision)
            for r in synth.batch_c4(seed=5, nruns=8, steps=0, nmin=20, nmax=140)]
    runs += [
        synth.random_periodic(40, 24, seed=1, precision=precision),
        synth.random_periodic(70, 37, seed=2, ymode="wall", solid=mask, precision=precision),
        synth.random_periodic(90, 30, seed=3, xmode="wall", circles=[(45.0, 15.0, 6.7)],
                              precision=precision),
        synth.random_periodic(75, 33, seed=4, ymode="wall", circles=[(30.2, 16.3, 5.9)],
                              precision=precision).with_(curved="ylw"),
        synth.random_periodic(130, 33, seed=4, xmode="open", ymode="wall",
                              circles=[(50.0, 16.0, 7.2)], precision=precision),
        synth.random_periodic(100, 29, seed=6, xmode="open", ymode="wall",
                              circles=[(40.0, 14.2, 6.1)],
                              precision=precision).with_(curved="ylw", open_ends="nebb"),
    ]
    return runs


def _make(runs, stream, **kw):
    from paper_2508_16997_amd import Simulation

    return [Simulation.from_problem(r, stream=stream, **kw) for r in runs]


def _read_exact(sim):
    import torch

    r = sim.read()
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in r.items()}


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("ty,chunk,schedule", [(4, 20, (0, 0)), (2, 0, (2, 3)), (8, 20, (3, 4))])
def test_batch_bit_identical_to_single(precision, ty, chunk, schedule):
    import torch
    from paper_2508_16997_amd import Batch

    runs = _mixed_set(precision)
    stream = torch.cuda.Stream()
    say("batch bit-identity", precision, "ty", ty, "chunk", chunk, "schedule", schedule,
        "runs", len(runs))
    batched = _make(runs, stream)
    single = _make(runs, stream)
    b = Batch(batched, tile=ty, graph_chunk=chunk, schedule=schedule)
    for n in (1, 129):  # first step, then graph replays and an eager tail
        b.step(n)
        for s in single:
            s.step(n)
    stream.synchronize()
    for r, sb, ss in zip(runs, batched, single):
        assert sb.time == ss.time == 130
        gb, gs = _read_exact(sb), _read_exact(ss)
        for k in FIELDS:
            assert np.array_equal(gb[k], gs[k]), (r.name, k)
        hb, hs = sb.history(), ss.history()
        for k in hb:
            assert torch.equal(hb[k], hs[k]), (r.name, "history", k)
    b.close()
    for s in batched + single:
        s.close()


@pytest.mark.parametrize("precision,ty,order", [("fp32", 4, 3), ("fp32", 8, 2), ("fp64", 2, 1)])
def test_persistent_batch_bit_identical(precision, ty, order):
    """One cooperative launch per chunk of at most 256 steps, grid-wide barriers between
    the tiles and the fills: same bits as the runs stepped alone, across the first step
    and a chunk boundary (1 + 300 steps = launches of 1, 256 and 44 steps)."""
    import torch
    from paper_2508_16997_amd import Batch

    runs = _mixed_set(precision)
    stream = torch.cuda.Stream()
    say("persistent batch", precision, "ty", ty, "runs", len(runs))
    batched = _make(runs, stream)
    single = _make(runs, stream)
    b = Batch(batched, tile=ty, persistent=True, schedule=(order, 0))
    for n in (1, 300):
        b.step(n)
        for s in single:
            s.step(n)
    stream.synchronize()
    for r, sb, ss in zip(runs, batched, single):
        assert sb.time == ss.time == 301
        gb, gs = _read_exact(sb), _read_exact(ss)
        for k in FIELDS:
            assert np.array_equal(gb[k], gs[k]), (r.name, k)
        hb, hs = sb.history(), ss.history()
        for k in hb:
            assert torch.equal(hb[k], hs[k]), (r.name, "history", k)
    b.close()
    for s in batched + single:
        s.close()


def test_persistent_batch_full_set_matches_per_step():
    """The 256-run batched workload: persistent and per-step batches agree bit for bit."""
    import torch
    from paper_2508_16997_amd import Batch

    runs = synth.batch_c4()
    stream = torch.cuda.Stream()
    say("persistent batch full set", len(runs))
    a, p = _make(runs, stream), _make(runs, stream)
    ba = Batch(a, graph_chunk=5)
    bp = Batch(p, persistent=True)
    ba.step(21)
    bp.step(21)
    stream.synchronize()
    for r, sa, sp in zip(runs, a, p):
        ga, gp = _read_exact(sa), _read_exact(sp)
        for k in FIELDS:
            assert np.array_equal(ga[k], gp[k]), (r.name, k)
    ba.close()
    bp.close()
    for s in a + p:
        s.close()


def test_batch_oracle_sample():
    """Eight runs of the full-size batched set (Wi <= 10) against the oracle."""
    import torch
    import oracle
    from paper_2508_16997_amd import Batch

    runs = synth.batch_c4()
    pick = [i for i, r in enumerate(runs) if r.meta["Wi"] <= 10.0]
    rng = np.random.default_rng(7)
    pick = sorted(rng.choice(pick, size=8, replace=False).tolist())
    sample = [runs[i] for i in pick]
    stream = torch.cuda.Stream()
    say("batch oracle sample", pick, [r.nx for r in sample])
    sims = _make(sample, stream)
    b = Batch(sims, graph_chunk=50)
    steps = 500
    b.step(steps)
    stream.synchronize()
    for i, r, s in zip(pick, sample, sims):
        o = oracle.OracleSim(r)
        o.step(steps)
        err = parity(gpu_fields(s), o.read(), r.fluid_mask())
        assert max(err["u"], err["axx"], err["axy"], err["ayy"]) < 1e-5, (i, r.name, err)
    b.close()
    for s in sims:
        s.close()


def test_batch_full_set_5000_steps_golden():
    """The whole 256-run batched workload for its 5,000 steps in the launch
    configuration the benchmark times (per-step graphs, 64 x 8 tiles), then eight runs
    (Wi <= 10, the draw of the 500-step sample) at a sample of nodes against oracle
    values written by tests/golden/make_batch_5000.py (oracle only)."""
    import os

    import torch
    from paper_2508_16997_amd import Batch

    path = os.path.join(os.path.dirname(__file__), "golden", "batch_5000.npz")
    if not os.path.exists(path):
        pytest.skip("golden file not generated")
    ref = np.load(path)
    steps = int(ref["steps"])
    runs = synth.batch_c4()
    stream = torch.cuda.Stream()
    say("batch 5000-step golden", len(runs), "runs", steps, "steps")
    sims = _make(runs, stream)
    b = Batch(sims, tile=8, graph_chunk=50)
    b.step(steps)
    stream.synchronize()
    for i in ref["runs"].tolist():
        ys, xs = ref[f"r{i}_ys"], ref[f"r{i}_xs"]
        g = {k: v[ys, xs] for k, v in gpu_fields(sims[i]).items()}
        o = {k: ref[f"r{i}_{k}"] for k in FIELDS}
        err = parity(g, o, np.ones(len(ys), dtype=bool))
        assert max(err["u"], err["axx"], err["axy"], err["ayy"]) < 1e-5, (i, runs[i].name, err)
    b.close()
    for s in sims:
        s.close()


def test_batch_full_set_bit_identical():
    """All 256 runs of the batched workload at full size, 20 steps, batched vs alone."""
    import torch
    from paper_2508_16997_amd import Batch

    runs = synth.batch_c4()
    stream = torch.cuda.Stream()
    say("batch full set", len(runs), "runs", sum(r.nx * r.ny for r in runs), "nodes")
    batched = _make(runs, stream)
    b = Batch(batched, graph_chunk=5)
    b.step(21)
    stream.synchronize()
    for r, sb in zip(runs, batched):
        ss = _make([r], stream)[0]
        ss.step(21)
        gb, gs = _read_exact(sb), _read_exact(ss)
        for k in FIELDS:
            assert np.array_equal(gb[k], gs[k]), (r.name, k)
        assert np.isfinite(gb["ux"]).all(), r.name
        ss.close()
    b.close()
    for s in batched:
        s.close()


def test_batch_picks_up_new_parameters():
    """set_params / set_force_field on a member between batch steps reach the batch."""
    import torch
    from paper_2508_16997_amd import Batch

    runs = [synth.random_periodic(70, 37, seed=8, ymode="wall", precision="fp32"),
            synth.random_periodic(40, 24, seed=9, precision="fp32")]
    stream = torch.cuda.Stream()
    say("batch parameter refresh")
    batched = _make(runs, stream)
    single = _make(runs, stream)
    b = Batch(batched, graph_chunk=4)
    b.step(11)
    for s in single:
        s.step(11)
    for s in (batched[0], single[0]):
        s.set_params(0.12, 0.05, 30.0, 0.02, 0.25, 0.05, 1e-5, -2e-6)
        s.set_force_field(None, None)
    b.step(20)
    for s in single:
        s.step(20)
    stream.synchronize()
    for i, (sb, ss) in enumerate(zip(batched, single)):
        gb, gs = _read_exact(sb), _read_exact(ss)
        rb = {k: v.cpu().numpy() for k, v in b.read(i).items()}
        for k in FIELDS:
            assert np.array_equal(gb[k], gs[k]), k
            assert np.array_equal(rb[k], gs[k]), ("batch read", k)
    b.close()
    for s in batched + single:
        s.close()


def test_batch_rejects_mismatched_members():
    import torch
    from paper_2508_16997_amd import Batch, VlbError

    stream = torch.cuda.Stream()
    a = _make([synth.random_periodic(40, 24, seed=1, precision="fp32")], stream)[0]
    c = _make([synth.random_periodic(40, 24, seed=1, precision="fp64")], stream)[0]
    say("batch errors")
    with pytest.raises(VlbError):
        Batch([a, c])  # mixed precisions
    d = _make([synth.random_periodic(40, 24, seed=2, precision="fp32")], stream)[0]
    d.step(3)
    with pytest.raises(VlbError):
        Batch([a, d])  # different step counts
    e = _make([synth.random_periodic(40, 24, seed=3, precision="fp32")], torch.cuda.Stream())[0]
    with pytest.raises(VlbError):
        Batch([a, e])  # different streams
    with pytest.raises(VlbError):
        Batch([a], tile=3)
    b = Batch([a])
    b.step(2)
    a.step(1)  # stepped outside the batch: the batch refuses to continue
    with pytest.raises(VlbError):
        b.step(1)
    b.close()
    for s in (a, c, d, e):
        s.close()
