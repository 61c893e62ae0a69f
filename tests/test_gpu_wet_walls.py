"""Wet-node walls on the HIP path (VLB_WET): rows 0 and ny - 1 are wall nodes, f rebuilt
there by non-equilibrium bounce-back, CNEBB for the conformation lattices at the wall
nodes, one-sided second-order wall-normal differences (the wall setting of the paper's
channel flows, Sec. 4.2-4.3).

Parity with the FP64 oracle on random states (FP64 1e-10, FP32 1e-5 relative L2) with a
curved obstacle, a staircase block and open ends; the Newtonian channel exact to
round-off and the Oldroyd-B closed form in FP64; bit-identical results for every tile
height and in both batched forms; the argument checks of the library.
"""
import numpy as np
import pytest

import synth
from analytic import gre, poiseuille_steady
from gpu_util import FIELDS, gpu_fields, parity, run_pair, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle

    oracle.build(force=False)
    oracle.set_threads(min(16, oracle.max_threads()))


def _cases(precision):
    mask = np.zeros((33, 70), np.uint8)
    mask[12:17, 20:24] = 1
    return {
        "plain": synth.random_periodic(70, 21, seed=31, ymode="wet", precision=precision),
        "obstacles": synth.random_periodic(70, 33, seed=32, ymode="wet", solid=mask,
                                           circles=[(48.0, 16.0, 6.6)], precision=precision),
        "open_ends": synth.random_periodic(130, 33, seed=33, xmode="open", ymode="wet",
                                           circles=[(50.0, 16.0, 7.2)], precision=precision),
    }


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
@pytest.mark.parametrize("case", ["plain", "obstacles", "open_ends"])
def test_wet_walls_parity(case, precision, tol):
    pr = _cases(precision)[case]
    say("wet walls parity", case, precision)
    g, o = run_pair(pr, 60, dual_chunks=[1, 59], sim_kw=dict(tile=4))
    e = parity(g, o, pr.fluid_mask())
    # the velocity and conformation fields at the bar; rho - 1 (of order 1e-2 here) in
    # FP64 too
    keys = ("u", "axx", "axy", "ayy") + (("rho",) if precision == "fp64" else ())
    assert max(e[k] for k in keys) < tol, e
    # the wall nodes hold the wall velocity exactly
    assert np.abs(g["ux"][[0, -1], :]).max() == 0.0 and np.abs(g["uy"][[0, -1], :]).max() == 0.0


def test_wet_walls_drag_on_a_circle_matches_oracle():
    import oracle
    from paper_2508_16997_amd import Simulation, VlbError

    pr = _cases("fp64")["open_ends"]
    say("wet walls drag")
    sim = Simulation.from_problem(pr)
    o = oracle.OracleSim(pr)
    sim.step(40)
    o.step(40)
    fg = np.array(sim.drag(0))
    fo = np.array(o.drag(0))
    assert np.abs(fg - fo).max() < 1e-10 * np.abs(fo).max(), (fg, fo)
    with pytest.raises(VlbError):
        sim.drag(-1)  # wall links of wet-node walls: not built
    sim.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_wet_walls_independent_of_tiling(prec):
    """Every tile height (the wall rows' neighbours come from the tile, the ring or the
    two-rows-in recompute) gives the same bits; so do graph replays."""
    from paper_2508_16997_amd import Simulation

    pr = _cases("fp64")["obstacles"]
    say("wet walls tiling", prec)
    ref = None
    for ty, chunk in ((4, 0), (1, 0), (2, 0), (8, 0), (4, 3)):
        sim = Simulation.from_problem(pr, precision=prec, tile=ty, graph_chunk=chunk)
        sim.step(15)
        g = gpu_fields(sim)
        sim.close()
        if ref is None:
            ref = g
        else:
            for k in FIELDS:
                assert np.array_equal(g[k], ref[k]), (ty, chunk, k)


@pytest.mark.parametrize("ny", [9, 17])
def test_wet_walls_newtonian_channel_exact(ny):
    from paper_2508_16997_amd import Simulation

    pr = synth.poiseuille(nx=4, ny=ny, beta=1.0, wet=True)
    ref = poiseuille_steady(ny, pr.meta["Uc"], pr.lam, wet=True)
    say("wet walls newtonian", ny)
    sim = Simulation.from_problem(pr, graph_chunk=100)
    sim.step(int(30 * pr.meta["Tc"]))
    r = gpu_fields(sim)
    sim.close()
    assert np.abs(r["ux"][:, 0] - ref["ux"]).max() < 1e-12 * ref["ux"].max()


def test_wet_walls_oldroyd_b_channel_fp64():
    """Wi = 1, beta = 0.5, H = 32: the bars of the oracle's own pin."""
    from paper_2508_16997_amd import Simulation

    pr = synth.poiseuille(nx=4, ny=33, wet=True)
    ref = poiseuille_steady(33, pr.meta["Uc"], pr.lam, wet=True)
    say("wet walls oldroyd-b channel")
    sim = Simulation.from_problem(pr, graph_chunk=100)
    sim.step(int(round(18 * pr.meta["Tc"])))
    r = gpu_fields(sim)
    sim.close()
    assert gre(r["ux"][:, 0], ref["ux"]) < 1e-4
    assert gre(r["axy"][:, 0], ref["axy"]) < 3e-3
    assert gre(r["axx"][:, 0], ref["axx"]) < 8e-3


@pytest.mark.parametrize("persistent", [False, True])
def test_wet_walls_in_a_batch_bit_identical(persistent):
    import torch
    from paper_2508_16997_amd import Batch, Simulation

    runs = list(_cases("fp32").values()) + [synth.random_periodic(40, 24, seed=34)
                                            .with_(precision="fp32")]
    stream = torch.cuda.Stream()
    say("wet walls batch", persistent)
    batched = [Simulation.from_problem(r, stream=stream) for r in runs]
    single = [Simulation.from_problem(r, stream=stream) for r in runs]
    b = Batch(batched, tile=4, graph_chunk=0 if persistent else 5, persistent=persistent)
    b.step(1)
    b.step(30)
    for s in single:
        s.step(31)
    stream.synchronize()
    for r, sb, ss in zip(runs, batched, single):
        gb, gs = sb.read(), ss.read()
        torch.cuda.synchronize()
        for k in FIELDS:
            assert torch.equal(gb[k], gs[k]), (r.name, k)
    b.close()
    for s in batched + single:
        s.close()


def test_wet_walls_argument_checks():
    from paper_2508_16997_amd import Simulation, VlbError

    say("wet walls argument checks")
    mask = np.zeros((12, 10), np.uint8)
    mask[2, 4] = 1  # a solid two rows from the wall
    with pytest.raises(VlbError):
        Simulation.from_problem(synth.random_periodic(10, 12, seed=1, ymode="wet", solid=mask))
    with pytest.raises(VlbError):
        Simulation.from_problem(synth.random_periodic(10, 4, seed=1, ymode="wet"))
    with pytest.raises(VlbError):
        Simulation.from_problem(synth.random_periodic(10, 12, seed=1, xmode="wet"))
