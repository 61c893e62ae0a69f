"""vlb_batch_create_noalloc: the batch whose lists live in the library's static scratch.

Checked against vlb_batch_create (the workspace form) on identical member sets: after
the same steps every member's fields are bit-identical (the same kernels run on the same
lists; only where the lists live differs).  Two batches in a row, the second smaller,
so the second reuses scratch that still holds the first's lists; each in the per-step
form and the persistent form.  While a noalloc batch lives, a second one on the device
is refused.
"""
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


def _runs(n, seed, precision="fp32"):
    mask = np.zeros((37, 70), np.uint8)
    mask[10:15, 20:24] = 1
    runs = [r.with_(precision=precision)
            for r in synth.batch_c4(seed=seed, nruns=n, steps=0, nmin=20, nmax=160)]
    runs += [
        synth.random_periodic(70, 37, seed=seed, ymode="wall", solid=mask, precision=precision),
        synth.random_periodic(130, 33, seed=seed + 1, xmode="open", ymode="wall",
                              circles=[(50.0, 16.0, 7.2)], precision=precision),
    ]
    return runs


def _make(runs, stream):
    from paper_2508_16997_amd import Simulation

    return [Simulation.from_problem(r, stream=stream) for r in runs]


def _fields(sim):
    import torch

    r = sim.read()
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in r.items()}


@pytest.mark.parametrize("persistent", [False, True])
def test_noalloc_batch_matches_workspace_batch(persistent):
    import torch
    from paper_2508_16997_amd import Batch, VlbError
    from paper_2508_16997_amd import _lib as L

    stream = torch.cuda.Stream()
    for call, (n, seed, tile, steps) in enumerate(((10, 21, 2, 23), (3, 22, 4, 17))):
        runs = _runs(n, seed)
        say("noalloc batch", "persistent" if persistent else "per-step", "call", call,
            len(runs), "runs", tile, steps)
        ref_sims, na_sims = _make(runs, stream), _make(runs, stream)
        ref = Batch(ref_sims, tile=tile, graph_chunk=5, persistent=persistent)
        na = Batch(na_sims, tile=tile, graph_chunk=5, persistent=persistent, noalloc=True)
        assert na.workspace_bytes == 0 and na._ws is None
        if call == 0:
            # the device's scratch is held: a second noalloc batch is refused
            with pytest.raises(VlbError) as e:
                Batch(na_sims[:1], tile=tile, noalloc=True)
            assert e.value.status == L.VLB_E_STATE
        ref.step(steps)
        na.step(steps)
        stream.synchronize()
        for r, a, b in zip(runs, ref_sims, na_sims):
            ga, gb = _fields(a), _fields(b)
            for k in FIELDS:
                assert np.array_equal(ga[k], gb[k]), (call, r.name, k)
            assert np.isfinite(gb["ux"]).all()
        ref.close()
        na.close()  # releases the scratch for the next call
        for s in ref_sims + na_sims:
            s.close()
