"""``torch.autograd`` face of the library's discrete adjoint.

:class:`VlbFunction` maps (lambda, eta_p, F_x(x), F_y(x)) to the velocity read out after
``nsteps`` coupled steps from a simulation's current state.  Its forward pass runs the
steps with checkpoints and its backward pass runs the hand-written adjoint kernels
(reverse sweep with segment recompute).  Both passes are HIP work; this module only
moves arguments.  Periodic axes, half-way walls, solid masks and circles; the library
reports open ends and wet-node walls as unsupported.
"""
from __future__ import annotations

from typing import Optional

import torch


class VlbFunction(torch.autograd.Function):
    """u(T) = step^T(state; lambda, eta_p, F) for one :class:`~.sim.Simulation`.

    ``lam`` and ``eta_p`` are 0-d tensors, ``Fx`` and ``Fy`` are [ny][nx] tensors; the
    other parameters are the simulation's current ones.  The simulation is left at step
    t0 + nsteps; reload a saved state before the next forward pass to repeat it.
    """

    @staticmethod
    def forward(ctx, sim, nsteps: int, stride: Optional[int], lam, eta_p, Fx, Fy):
        p = dict(sim.params)
        p.update(lam=float(lam), eta_p=float(eta_p))
        sim.set_params(p["nu_s"], p["eta_p"], p["lam"], p["kappa"], p["Lambda_s"], p["Lambda_p"],
                       0.0, 0.0, p["flags"], model=p.get("model", "oldroyd_b"),
                       model_param=p.get("model_param", 0.0))
        sim.set_force_field(Fx.detach(), Fy.detach())
        sim.adjoint_forward(int(nsteps), stride)
        r = sim.read()
        ctx.sim = sim
        ctx.dtypes = (lam.dtype, eta_p.dtype, Fx.dtype, Fy.dtype)
        return r["ux"], r["uy"]

    @staticmethod
    def backward(ctx, gux, guy):
        sim = ctx.sim
        if gux is None:
            gux = torch.zeros((sim.ny, sim.nx), dtype=sim.dtype, device=sim.device)
        if guy is None:
            guy = torch.zeros((sim.ny, sim.nx), dtype=sim.dtype, device=sim.device)
        g = sim.adjoint_backward(gux, guy)
        tl, te, tfx, tfy = ctx.dtypes
        dev = sim.device
        return (None, None, None, torch.tensor(g["dlambda"], dtype=tl, device=dev),
                torch.tensor(g["deta_p"], dtype=te, device=dev), g["dFx"].to(tfx),
                g["dFy"].to(tfy))


def velocity_after(sim, nsteps: int, lam, eta_p, Fx, Fy, stride: Optional[int] = None):
    """Differentiable (u_x, u_y) after ``nsteps`` steps; see :class:`VlbFunction`."""
    return VlbFunction.apply(sim, nsteps, stride, lam, eta_p, Fx, Fy)
