"""Momentum-exchange force on solids (Sec. 4.3) through vlb_drag.

The force is summed over boundary links from the post-collision populations of the last
step and the populations the boundary rules returned.  Checked against the FP64 oracle
(all solids, one circle; periodic channel with walls, a staircase block and a curved
cylinder, and an open channel whose ends use non-equilibrium extrapolation), against
the exact momentum budget of a closed domain on the GPU itself, and for its errors.
"""
import os

import numpy as np
import pytest

import synth
from gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle

    oracle.build(force=False)
    oracle.set_threads(min(16, oracle.max_threads()))


def _closed(precision):
    mask = np.zeros((30, 60), np.uint8)
    mask[12:16, 10:14] = 1
    return synth.random_periodic(60, 30, seed=5, ymode="wall", solid=mask,
                                 circles=[(40.0, 15.0, 6.3)], precision=precision)


def _open(precision):
    return synth.random_periodic(130, 33, seed=11, xmode="open", ymode="wall",
                                 circles=[(50.0, 16.0, 7.2)], precision=precision)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
@pytest.mark.parametrize("make", [_closed, _open], ids=["closed", "open"])
def test_drag_matches_oracle(make, precision, tol):
    import oracle
    from paper_2508_16997_amd import Simulation

    pr = make(precision)
    say("drag vs oracle", pr.name, precision)
    sim = Simulation.from_problem(pr)
    o = oracle.OracleSim(pr)
    for n in (1, 40):
        sim.step(n)
        o.step(n)
        for c in (-1, 0):
            g = np.array(sim.drag(c))
            r = np.array(o.drag(c))
            assert np.abs(r).max() > 1e-3, (c, r)
            err = np.abs(g - r).max() / np.abs(r).max()
            assert err < tol, (pr.name, n, c, g, r, err)
    sim.close()


def test_drag_momentum_balance_fp64():
    """P(t+1) - P(t) = sum F - D in a closed domain, P = sum over fluid of (rho u - F/2)."""
    from paper_2508_16997_amd import Simulation

    pr = _closed("fp64")
    fx, fy = pr.force_arrays()
    fl = pr.fluid_mask()
    say("drag momentum balance")
    sim = Simulation.from_problem(pr)

    def momentum():
        import torch

        r = sim.read()
        torch.cuda.synchronize()
        r = {k: v.cpu().numpy() for k, v in r.items()}
        return np.array([((r["rho"] * r["ux"] - 0.5 * fx)[fl]).sum(),
                         ((r["rho"] * r["uy"] - 0.5 * fy)[fl]).sum()])

    sim.step(5)
    fsum = np.array([fx[fl].sum(), fy[fl].sum()])
    for _ in range(3):
        p0 = momentum()
        sim.step(1)
        d = np.array(sim.drag(-1))
        assert np.abs(d).max() > 1e-2
        assert np.abs(momentum() - p0 - (fsum - d)).max() < 1e-12
    sim.close()


def test_drag_errors():
    from paper_2508_16997_amd import Simulation, VlbError

    say("drag errors")
    sim = Simulation.from_problem(_closed("fp32"))
    with pytest.raises(VlbError):
        sim.drag(0)  # no step yet
    sim.step(1)
    with pytest.raises(VlbError):
        sim.drag(1)  # one circle only
    sim.drag(0)
    sim.close()
    per = Simulation.from_problem(synth.random_periodic(40, 24, seed=1, precision="fp32"))
    per.step(1)
    assert per.drag(-1) == (0.0, 0.0)  # no solid links
    per.close()


def _paper_cd():
    import os

    path = os.path.join(os.path.dirname(__file__), "golden", "cylinder_cd_table.txt")
    rows = np.loadtxt(path, comments="#")
    return {(r[0], int(r[1])): {0.1: r[2], 0.5: r[3], 1.0: r[4]} for r in rows}


@pytest.mark.parametrize("Sc,wis", [(1e6, (0.1, 0.5)), (1e4, (0.1, 0.5, 1.0))])
def test_cylinder_drag_coefficient_vs_paper(Sc, wis):
    """Steady C_d of the confined cylinder (R = 10, 20; FP64) against the paper's CNEBB
    values at the same Sc.

    The paper's hydrodynamic walls, inlet and outlet are wet-node (NEBB) and its cylinder
    rule for f is YLW; here the walls are half-way bounce-back, the cylinder interpolated
    bounce-back and the open ends non-equilibrium extrapolation, so the coarse-grid error
    differs: the bar is 3 % at R = 10 and 1.2 % at R = 20 for Wi <= 0.5, plus the paper's
    trends (C_d grows with R from 10 to 20 and falls from Wi = 0.1 to 0.5).  At Wi = 1 the
    paper's values still move by 15 % between R = 10 and 40; here they lie 6-9 % above
    them at R = 10 and 20 (bar 10 %), with the same steep rise over Wi = 0.5.
    """
    from paper_2508_16997_amd import Batch, Simulation
    import torch

    paper = _paper_cd()
    cases = [(R, wi) for R in (10, 20) for wi in wis]
    probs = [synth.cylinder_channel(R=R, Wi=wi, Sc=Sc) for R, wi in cases]
    stream = torch.cuda.Stream()
    say("cylinder C_d", Sc, cases)
    sims = [Simulation.from_problem(p, stream=stream) for p in probs]
    b = Batch(sims, tile=4, graph_chunk=100)
    tcs = [p.meta["Tc"] for p in probs]
    ucs = [p.meta["Uc"] for p in probs]
    b.step(1)
    for s in sims:
        s.monitors()
    n, last, cd = 1, [1] * len(sims), [None] * len(sims)
    step = int(round(min(tcs)))
    while any(c is None for c in cd):
        assert n < 1000 * max(tcs), ("no steady state by t* = 1000", cd)
        b.step(step)
        n += step
        for i, s in enumerate(sims):
            if cd[i] is None and n - last[i] >= tcs[i]:
                m = s.monitors()
                last[i] = n
                if m["residual"] / ucs[i] < 1e-8:
                    R = cases[i][0]
                    fx, fy = s.drag(0)
                    cd[i] = fx / (0.5 * ucs[i] ** 2 * 2 * R)
                    assert abs(fy) < 1e-6 * abs(fx), (cases[i], fx, fy)
    say("C_d", dict(zip(cases, cd)))
    got = dict(zip(cases, cd))
    for (R, wi), c in got.items():
        tol = 0.10 if wi == 1.0 else (0.03 if R == 10 else 0.012)
        ref = paper[(Sc, R)][wi]
        assert abs(c / ref - 1) < tol, (R, wi, c, ref)
    for R in (10, 20):
        assert got[(R, 0.5)] < got[(R, 0.1)]
        if 1.0 in wis:
            assert got[(R, 1.0)] > 1.25 * got[(R, 0.5)]
    for wi in (0.1, 0.5):
        assert got[(20, wi)] > got[(10, wi)]
    b.close()
    for s in sims:
        s.close()


def _steady_cd(probs, cases, stream):
    """Run a batch of cylinder channels to the steady criterion; C_d per case (None for a
    run that is not steady by t* = 1000)."""
    from paper_2508_16997_amd import Batch, Simulation

    sims = [Simulation.from_problem(p, stream=stream) for p in probs]
    b = Batch(sims, tile=4, graph_chunk=100)
    tcs = [p.meta["Tc"] for p in probs]
    ucs = [p.meta["Uc"] for p in probs]
    b.step(1)
    for s in sims:
        s.monitors()
    n, last, cd, done = 1, [1] * len(sims), [None] * len(sims), [False] * len(sims)
    step = int(round(min(tcs)))
    while not all(done):
        b.step(step)
        n += step
        for i, s in enumerate(sims):
            if not done[i] and n - last[i] >= tcs[i]:
                m = s.monitors(raise_on_nonfinite=False)
                last[i] = n
                assert m["nonfinite"] == 0, ("breakdown", cases[i], n / tcs[i])
                if m["residual"] / ucs[i] < 1e-8:
                    fx, _ = s.drag(0)
                    cd[i] = fx / (0.5 * ucs[i] ** 2 * 2 * cases[i][0])
                    done[i] = True
                elif n / tcs[i] > 1000:
                    done[i] = True
    b.close()
    for s in sims:
        s.close()
    return cd


def test_cylinder_drag_paper_boundary_set():
    """The paper's boundary set for f on the cylinder (Sec. 4.3): wet-node NEBB inlet and
    outlet and the curved-wall scheme YLW on the circle (readings A30, A31), half-way
    channel walls; Sc = 1e6, R = 20, Wi = 0.1 and 0.5, FP64.  Both runs become steady,
    within 1.5 % and 2 % of the paper's CNEBB values, with C_d falling from Wi = 0.1 to
    0.5 as in the paper."""
    import torch

    paper = _paper_cd()
    cases = [(20, 0.1), (20, 0.5)]
    probs = [synth.cylinder_channel(R=R, Wi=wi, Sc=1e6).with_(open_ends="nebb", curved="ylw")
             for R, wi in cases]
    say("cylinder C_d, NEBB ends + YLW", cases)
    cd = _steady_cd(probs, cases, torch.cuda.Stream())
    say("C_d", dict(zip(cases, cd)))
    assert all(c is not None for c in cd), cd
    for (R, wi), c, tol in zip(cases, cd, (0.015, 0.02)):
        ref = paper[(1e6, R)][wi]
        assert abs(c / ref - 1) < tol, (R, wi, c, ref)
    assert cd[1] < cd[0]


@pytest.mark.parametrize("Sc", [
    1e4, 1e5,  # about 2 GPU-minutes each
    pytest.param(1e6, marks=pytest.mark.skipif(
        not os.environ.get("VLB_LONG_TESTS"),
        reason="about 13 minutes of GPU time; set VLB_LONG_TESTS=1"))])
def test_cylinder_drag_full_table(Sc):
    """All 24 cells of the paper's CNEBB column at one Schmidt number (R = 5 ... 40,
    Wi = 0.1, 0.5, 1.0; FP64, batched, to the criterion or t* = 1000).

    Every run reaches a steady state.  Wi <= 0.5: within 1.5 % of the paper from R = 15
    on, within 17 % on the coarse grids R = 5, 10 (the link-wise hydrodynamic boundaries
    against the paper's wet-node/YLW set-up).  Wi = 1: within 11 % from R = 20 where the
    paper is steady (4 % from R = 25 at Sc = 1e6), falling monotonically from R = 15 to
    40 as the paper's column does.
    """
    import torch
    from paper_2508_16997_amd import Batch, Simulation

    paper = _paper_cd()
    Rs = (5, 10, 15, 20, 25, 30, 35, 40)
    cases = [(R, wi) for R in Rs for wi in (0.1, 0.5, 1.0)]
    probs = [synth.cylinder_channel(R=R, Wi=wi, Sc=Sc) for R, wi in cases]
    stream = torch.cuda.Stream()
    say("cylinder C_d full table", Sc)
    sims = [Simulation.from_problem(p, stream=stream) for p in probs]
    b = Batch(sims, tile=4, graph_chunk=100)
    tcs = [p.meta["Tc"] for p in probs]
    ucs = [p.meta["Uc"] for p in probs]
    b.step(1)
    for s in sims:
        s.monitors()
    n, last, cd, it = 1, [1] * len(sims), [None] * len(sims), 0
    step = int(round(min(tcs)))
    while any(c is None for c in cd):
        b.step(step)
        n += step
        it += 1
        for i, s in enumerate(sims):
            if cd[i] is None and n - last[i] >= tcs[i]:
                m = s.monitors(raise_on_nonfinite=False)
                last[i] = n
                assert m["nonfinite"] == 0, ("breakdown", cases[i], n / tcs[i])
                if m["residual"] / ucs[i] < 1e-8:
                    fx, _ = s.drag(0)
                    cd[i] = fx / (0.5 * ucs[i] ** 2 * 2 * cases[i][0])
                else:
                    assert n / tcs[i] < 1000, ("no steady state by t* = 1000", cases[i])
        if it % 500 == 0:
            say("step", n, "open", [c for c, v in zip(cases, cd) if v is None])
    got = dict(zip(cases, cd))
    say("C_d", got)
    for (R, wi), c in got.items():
        ref = paper[(Sc, R)][wi]
        if np.isnan(ref):
            continue
        if wi <= 0.5:
            tol = 0.015 if R >= 15 else 0.17
        elif R >= 20:
            tol = 0.04 if (Sc == 1e6 and R >= 25) else 0.11
        else:
            continue
        assert abs(c / ref - 1) < tol, (R, wi, c, ref)
    w1 = [got[(R, 1.0)] for R in Rs if R >= 15]
    assert all(a > b2 for a, b2 in zip(w1, w1[1:])), w1
    b.close()
    for s in sims:
        s.close()
