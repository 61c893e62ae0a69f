"""Discrete adjoint (HIP) against derivatives computed without it.

* 8 x 8 periodic, FP64: the full gradient (lambda, eta_p and all 128 force components)
  against central differences of the FP64 oracle, for Oldroyd-B and the other closures.
* 128 x 128, 200 steps: directional derivatives along lambda, eta_p and a random smooth
  force direction against the oracle's forward-mode (dual-number) derivatives.
* The adjoint workload at full size (512 x 512, FP32, 2000 steps, checkpoint stride 45,
  hidden target from its seeded generator): against central differences of the FP64
  HIP forward path (relative step 1e-6) along the same three directions.
* Checkpoint stride does not change the result (bit for bit), the autograd face agrees
  with the C entry point, and misuse is rejected.
"""
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


def _loss(u, t, n):
    return 0.5 * float(((u[0] - t[0]) ** 2 + (u[1] - t[1]) ** 2).sum()) / n


def _oracle_loss(pr, steps, target):
    import oracle

    o = oracle.OracleSim(pr)
    o.step(steps)
    r = o.read()
    return _loss((r["ux"], r["uy"]), target, pr.nx * pr.ny)


def _gpu_adjoint(pr, steps, target, precision, stride=None):
    import torch
    from paper_2508_16997_amd import Simulation

    sim = Simulation.from_problem(pr, precision=precision)
    dt = torch.float32 if precision == "fp32" else torch.float64
    tx = torch.as_tensor(np.ascontiguousarray(target[0]), dtype=dt, device="cuda")
    ty = torch.as_tensor(np.ascontiguousarray(target[1]), dtype=dt, device="cuda")
    g = sim.adjoint(steps, tx, ty, stride=stride)
    out = dict(loss=g["loss"], dlambda=g["dlambda"], deta_p=g["deta_p"],
               dFx=g["dFx"].cpu().numpy(), dFy=g["dFy"].cpu().numpy())
    sim.close()
    return out


def _target(pr, seed, amp=0.02):
    rng = np.random.default_rng(seed)
    return (amp * rng.uniform(-1, 1, (pr.ny, pr.nx)), amp * rng.uniform(-1, 1, (pr.ny, pr.nx)))


def _rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("model,mp", [("oldroyd_b", 0.0), ("giesekus", 0.3), ("lptt", 0.25),
                                      ("eptt", 0.25), ("fene_p", 20.0)])
def test_adjoint_bruteforce_8x8_fp64(model, mp):
    """All 130 gradient components against oracle central differences, for every
    constitutive closure (the transpose of each closure's Jacobian)."""
    pr = synth.random_periodic(8, 8, seed=3, precision="fp64").with_(model=model,
                                                                     model_param=mp)
    steps, stride = 12, 5  # three segments, the last one partial
    tgt = _target(pr, 11)
    say("adjoint 8x8 brute force", model, steps, stride)
    g = _gpu_adjoint(pr, steps, tgt, "fp64", stride)
    assert abs(g["loss"] - _oracle_loss(pr, steps, tgt)) < 1e-12 * abs(g["loss"]) + 1e-18

    def fd(make, h):
        return (_oracle_loss(make(+h), steps, tgt) - _oracle_loss(make(-h), steps, tgt)) / (2 * h)

    hl = 1e-6 * pr.lam
    dl = fd(lambda d: pr.with_(lam=pr.lam + d), hl)
    he = 1e-6 * pr.eta_p
    de = fd(lambda d: pr.with_(eta_p=pr.eta_p + d), he)
    assert abs(g["dlambda"] - dl) < 1e-6 * abs(dl), (g["dlambda"], dl)
    assert abs(g["deta_p"] - de) < 1e-6 * abs(de), (g["deta_p"], de)
    # the force enters almost linearly: a larger step keeps rounding (eps L / h) small
    hF = 1e-3 * float(np.abs(pr.Fx).max())
    dFx = np.zeros((8, 8))
    dFy = np.zeros((8, 8))
    for y in range(8):
        for x in range(8):
            def mkx(d, x=x, y=y):
                F = np.array(pr.Fx, dtype=float)
                F[y, x] += d
                return pr.with_(Fx=F)

            def mky(d, x=x, y=y):
                F = np.array(pr.Fy, dtype=float)
                F[y, x] += d
                return pr.with_(Fy=F)

            dFx[y, x] = fd(mkx, hF)
            dFy[y, x] = fd(mky, hF)
    assert _rel(g["dFx"], dFx) < 1e-6, _rel(g["dFx"], dFx)
    assert _rel(g["dFy"], dFy) < 1e-6, _rel(g["dFy"], dFy)


def _smooth_dir(n, seed):
    fx, fy = synth.smooth_force_perturbation(n, 1.0, seed)
    return fx, fy


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-8), ("fp32", 1e-4)])
def test_adjoint_vs_oracle_forward_mode_128(precision, tol):
    """Directional derivatives along lambda, eta_p and a smooth force field."""
    import oracle

    pr = synth.four_roll_mill(N=128, Wi=5.0, beta=0.5, steps=200)
    n = pr.nx * pr.ny
    steps = 200
    # target: the same flow with other parameters (a hidden-parameter fit)
    tgt_pr = pr.with_(lam=pr.lam * 1.1, eta_p=pr.eta_p * 0.9)
    o = oracle.OracleSim(tgt_pr)
    o.step(steps)
    r = o.read()
    tgt = (r["ux"], r["uy"])
    vx, vy = _smooth_dir(128, 5)
    say("adjoint 128 forward-mode", precision)
    g = _gpu_adjoint(pr, steps, tgt, precision)
    checks = []
    for name, kw in (("lambda", dict(dlam=1.0)), ("eta_p", dict(deta=1.0)),
                     ("force", dict(dFx=vx, dFy=vy))):
        od = oracle.OracleSim(pr, dual=True)
        od.set_tangent(**kw)
        od.step(steps)
        u = od.read()
        t = od.read_tangent()
        dd = float(((u["ux"] - tgt[0]) * t["ux"] + (u["uy"] - tgt[1]) * t["uy"]).sum()) / n
        if name == "lambda":
            ad = g["dlambda"]
        elif name == "eta_p":
            ad = g["deta_p"]
        else:
            ad = float((g["dFx"] * vx + g["dFy"] * vy).sum())
        checks.append((name, ad, dd))
    for name, ad, dd in checks:
        assert abs(ad - dd) <= tol * abs(dd), (name, ad, dd, checks)


def test_adjoint_full_size_vs_fp64_central_differences():
    """512 x 512 FP32 adjoint, 2000 steps, stride 45, vs FP64 GPU central differences."""
    import torch
    from paper_2508_16997_amd import Simulation

    pr, hidden = synth.adjoint_c5()
    steps, stride = pr.steps, 45
    n = pr.nx * pr.ny
    say("adjoint full size: target run", pr.nx, steps)

    def run64(p):
        sim = Simulation.from_problem(p, precision="fp64", graph_chunk=50)
        sim.step(steps)
        r = sim.read()
        torch.cuda.synchronize()
        out = (r["ux"].cpu().numpy(), r["uy"].cpu().numpy())
        sim.close()
        return out

    tgt = run64(pr.with_(lam=hidden["lam"], eta_p=hidden["eta_p"], Fx=hidden["Fx"],
                         Fy=hidden["Fy"]))
    say("adjoint full size: FP32 adjoint")
    g = _gpu_adjoint(pr, steps, tgt, "fp32", stride)
    vx, vy = _smooth_dir(pr.nx, 77)
    Fx = np.broadcast_to(np.asarray(pr.Fx, float), (pr.ny, pr.nx))
    Fy = np.broadcast_to(np.asarray(pr.Fy, float), (pr.ny, pr.nx))
    say("adjoint full size: FP64 central differences")

    def L(p):
        return _loss(run64(p), tgt, n)

    res = {}
    h = 1e-6 * pr.lam
    res["lambda"] = (g["dlambda"], (L(pr.with_(lam=pr.lam + h)) - L(pr.with_(lam=pr.lam - h))) / (2 * h))
    h = 1e-6 * pr.eta_p
    res["eta_p"] = (g["deta_p"], (L(pr.with_(eta_p=pr.eta_p + h)) - L(pr.with_(eta_p=pr.eta_p - h))) / (2 * h))
    s = 1e-6 * float(np.abs(Fx).max()) / float(np.abs(vx).max())
    fd = (L(pr.with_(Fx=Fx + s * vx, Fy=Fy + s * vy)) - L(pr.with_(Fx=Fx - s * vx, Fy=Fy - s * vy))) / (2 * s)
    res["force"] = (float((g["dFx"] * vx + g["dFy"] * vy).sum()), fd)
    for name, (ad, dd) in res.items():
        assert abs(ad - dd) <= 1e-4 * abs(dd), (name, ad, dd, res)


def test_adjoint_stride_invariance():
    """Recompute is the same arithmetic: any checkpoint stride gives the same bits."""
    pr = synth.random_periodic(100, 70, seed=4, precision="fp32")
    tgt = _target(pr, 12)
    say("adjoint stride invariance")
    ref = _gpu_adjoint(pr, 50, tgt, "fp32", stride=50)
    for stride in (1, 7):
        g = _gpu_adjoint(pr, 50, tgt, "fp32", stride=stride)
        assert g["dlambda"] == ref["dlambda"] and g["deta_p"] == ref["deta_p"], stride
        assert np.array_equal(g["dFx"], ref["dFx"]) and np.array_equal(g["dFy"], ref["dFy"]), stride


def test_adjoint_autograd_matches_entry_point():
    import torch
    from paper_2508_16997_amd import Simulation
    from paper_2508_16997_amd.adjoint import velocity_after

    pr = synth.random_periodic(70, 40, seed=6, precision="fp64")
    tgt = _target(pr, 13)
    steps = 30
    say("adjoint autograd")
    ref = _gpu_adjoint(pr, steps, tgt, "fp64", stride=6)
    sim = Simulation.from_problem(pr)
    lam = torch.tensor(pr.lam, dtype=torch.float64, requires_grad=True)
    eta = torch.tensor(pr.eta_p, dtype=torch.float64, requires_grad=True)
    Fx = torch.tensor(np.asarray(pr.Fx, float), device="cuda", requires_grad=True)
    Fy = torch.tensor(np.asarray(pr.Fy, float), device="cuda", requires_grad=True)
    ux, uy = velocity_after(sim, steps, lam, eta, Fx, Fy, stride=6)
    tx = torch.as_tensor(tgt[0], device="cuda")
    ty = torch.as_tensor(tgt[1], device="cuda")
    loss = 0.5 * ((ux - tx) ** 2 + (uy - ty) ** 2).mean()
    loss.backward()
    assert abs(loss.item() - ref["loss"]) <= 1e-12 * ref["loss"]
    assert abs(lam.grad.item() - ref["dlambda"]) <= 1e-10 * abs(ref["dlambda"])
    assert abs(eta.grad.item() - ref["deta_p"]) <= 1e-10 * abs(ref["deta_p"])
    assert _rel(Fx.grad.cpu().numpy(), ref["dFx"]) < 1e-10
    assert _rel(Fy.grad.cpu().numpy(), ref["dFy"]) < 1e-10
    sim.close()


def test_adjoint_rejects_misuse():
    import torch
    from paper_2508_16997_amd import Simulation, VlbError

    say("adjoint errors")
    wall = synth.random_periodic(40, 24, seed=1, ymode="wall", precision="fp32")
    sim = Simulation.from_problem(wall)
    z = torch.zeros((24, 40), device="cuda")
    with pytest.raises(VlbError):
        sim.adjoint(5, z, z)  # walls: unsupported
    sim.close()
    per = synth.random_periodic(40, 24, seed=1, precision="fp32")
    sim = Simulation.from_problem(per)
    with pytest.raises(RuntimeError):
        sim.adjoint_backward(z, z)  # no forward pass yet
    sim.adjoint_forward(6, 3)
    sim.step(1)  # stepped after the recorded forward pass
    with pytest.raises(VlbError):
        sim.adjoint_backward(z, z)
    sim.adjoint_forward(4, 2)
    sim.set_tile(1)  # a different work list than the recorded forward pass
    with pytest.raises(VlbError):
        sim.adjoint_backward(z, z)
    sim.close()
