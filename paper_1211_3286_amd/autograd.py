"""``torch.autograd.Function`` over a whole run: (eps0, u0, tau) -> (u(T), eps(T)).

Forward: rlb_init + rlb_step(T) with a tape of g every ``ckpt_every`` steps,
then rlb_moments. Backward: rlb_grad, the hand-written adjoint in the HIP
library (checkpointed segments recomputed, reverse sweeps on the GPU).
"""

from __future__ import annotations

import copy

import torch


class RLBStep(torch.autograd.Function):
    """apply(eps0, u0, n0, tau, params, nsteps, precision, ckpt_every) -> (u_T, eps_T).

    eps0, n0: (nz, ny, nx) float64; u0: (3, nz, ny, nx) float64 (GPU tensors);
    tau: float64 tensor [tau_v, tau_e, tau_eps]; params: lattice description
    (nx, ny, nz, bc, tau_f, tau_q); returns device tensors shaped like eps0/u0.
    Gradients flow to eps0, u0 and tau.
    """

    @staticmethod
    def forward(ctx, eps0, u0, n0, tau, params, nsteps, precision, ckpt_every):
        from paper_1211_3286_amd import Simulation
        p = copy.copy(params)
        tv, te, tpe = [float(x) for x in tau.detach().cpu().tolist()]
        p.tau_v, p.tau_e, p.tau_eps = tv, te, tpe
        sim = Simulation([p], n0.detach(), eps0.detach(), u0.detach(), precision=precision,
                         ckpt_every=ckpt_every, tape_steps=max(int(nsteps), 1))
        sim.step(int(nsteps))
        m = sim.moments()
        ctx.sim = sim
        ctx.shape = tuple(eps0.shape)
        ctx.tau_device = tau.device
        return m["u"].reshape(u0.shape), m["eps"].reshape(eps0.shape)

    @staticmethod
    def backward(ctx, du, deps):
        sim = ctx.sim
        nc = sim.ncells
        if du is None:
            du = torch.zeros(3, nc, dtype=torch.float64, device=sim.device)
        if deps is None:
            deps = torch.zeros(nc, dtype=torch.float64, device=sim.device)
        dtau, de0, du0 = sim.grad(du.reshape(3, nc), deps.reshape(nc))
        sim.close()
        ctx.sim = None
        g_tau = torch.tensor(dtau, dtype=torch.float64, device=ctx.tau_device)
        return (de0.reshape(ctx.shape), du0.reshape((3,) + ctx.shape), None, g_tau, None, None,
                None, None)
