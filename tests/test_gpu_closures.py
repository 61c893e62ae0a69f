"""Constitutive closures other than Oldroyd-B (model function F(A), Sec. 2.2) on the
HIP path: Giesekus, linear and exponential Phan-Thien-Tanner, FENE-P.

Parity with the FP64 oracle on random states with walls, a staircase block and a curved
cylinder (FP64 1e-10, FP32 1e-5 relative L2); steady channel flow of each closure against
the semi-analytic profile (local simple shear balancing the body force); a batch that
mixes closures is bit-identical to its members stepped alone (the adjoint of every
closure is checked in test_gpu_adjoint.py).
"""
import numpy as np
import pytest

import synth
from analytic import gre, poiseuille_steady_model
from gpu_util import FIELDS, gpu_fields, parity, run_pair, say

pytestmark = pytest.mark.gpu

CLOSURES = [("giesekus", 0.3), ("lptt", 0.25), ("eptt", 0.25), ("fene_p", 20.0)]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle

    oracle.build(force=False)
    oracle.set_threads(min(16, oracle.max_threads()))


def _walled(model, mp, precision, seed=3):
    mask = np.zeros((33, 70), np.uint8)
    mask[10:15, 20:24] = 1
    pr = synth.random_periodic(70, 33, seed=seed, ymode="wall", solid=mask,
                               circles=[(48.0, 17.0, 6.6)], precision=precision, lam=12.0)
    return pr.with_(model=model, model_param=mp)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
@pytest.mark.parametrize("model,mp", CLOSURES)
def test_closure_parity(model, mp, precision, tol):
    pr = _walled(model, mp, precision)
    say("closure parity", model, mp, precision)
    g, o = run_pair(pr, 60, dual_chunks=[1, 59])
    e = parity(g, o, pr.fluid_mask())
    assert max(e["u"], e["axx"], e["axy"], e["ayy"]) < tol, e


@pytest.mark.parametrize("model,mp", CLOSURES)
def test_closure_poiseuille_fp64(model, mp):
    """Wi = 1, beta = 0.5, Ny = 32: the same bars as the oracle's own pin."""
    from paper_2508_16997_amd import Simulation

    pr = synth.poiseuille(nx=4, ny=32).with_(model=model, model_param=mp)
    ref = poiseuille_steady_model(32, pr.Fx, pr.nu_s, pr.eta_p, pr.lam, model, mp)
    say("closure poiseuille", model, mp)
    sim = Simulation.from_problem(pr, graph_chunk=100)
    sim.step(40000)
    r = gpu_fields(sim)
    sim.close()
    assert gre(r["ux"][:, 0], ref["ux"]) < 1.2e-3
    assert gre(r["axy"][:, 0], ref["axy"]) < 2e-3
    assert gre(r["axx"][:, 0] - 1, ref["axx"] - 1) < 2.5e-3


def test_batch_mixing_closures_bit_identical():
    import torch
    from paper_2508_16997_amd import Batch, Simulation

    runs = [_walled(m, p, "fp32", seed=10 + i) for i, (m, p) in enumerate(CLOSURES)]
    runs.append(_walled("oldroyd_b", 0.0, "fp32", seed=20))
    stream = torch.cuda.Stream()
    say("batch of closures")
    batched = [Simulation.from_problem(r, stream=stream) for r in runs]
    single = [Simulation.from_problem(r, stream=stream) for r in runs]
    b = Batch(batched, graph_chunk=10)
    b.step(45)
    for s in single:
        s.step(45)
    stream.synchronize()
    for r, sb, ss in zip(runs, batched, single):
        gb, gs = sb.read(), ss.read()
        torch.cuda.synchronize()
        for k in FIELDS:
            assert torch.equal(gb[k], gs[k]), (r.model, k)
    b.close()
    for s in batched + single:
        s.close()


def test_closure_parameter_limits_match_oldroyd_b():
    """alpha = 0 and eps = 0 take the closure branch and equal Oldroyd-B bit for bit."""
    from paper_2508_16997_amd import Simulation

    ob = _walled("oldroyd_b", 0.0, "fp32")
    say("closure limits")
    ref = Simulation.from_problem(ob)
    ref.step(30)
    gr = gpu_fields(ref)
    ref.close()
    for m in ("giesekus", "lptt", "eptt"):
        sim = Simulation.from_problem(ob.with_(model=m, model_param=0.0))
        sim.step(30)
        g = gpu_fields(sim)
        sim.close()
        for k in FIELDS:
            assert np.array_equal(g[k], gr[k]), (m, k)
