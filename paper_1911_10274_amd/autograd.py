"""``torch.autograd.Function`` over the simulator's adjoint.

``TitanRollout.apply(k, act_c, act_s, sim, nsteps, checkpoint_every,
spring_body)`` returns, per body b, J_b = -(x-displacement of body b's centre
of mass) after ``nsteps`` steps from the simulation's current state, and is
differentiable with respect to the per-spring stiffness ``k`` and actuation
phasor (``act_c`` = amp cos(phase), ``act_s`` = amp sin(phase)).

The forward pushes the parameters into the simulation (``titan_set_springs``)
and calls ``titan_rollout_grad``, which runs the rollout and its adjoint in
one launch and returns the per-spring gradients of every body's own loss.
Bodies do not interact, so the gradient of sum_b w_b J_b is the unit-weight
gradient of each spring scaled by the weight of its body: the backward is
that scaling, no second rollout.
"""
from __future__ import annotations

import numpy as np
import torch

from . import titan as T


class TitanRollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, k, act_c, act_s, sim, nsteps: int, checkpoint_every: int, spring_body):
        kk = k.detach().to("cpu", torch.float64).numpy()
        c = act_c.detach().to("cpu", torch.float64).numpy()
        s = act_s.detach().to("cpu", torch.float64).numpy()
        sim.set_springs(0, k=kk, amp=np.hypot(c, s), phase=np.arctan2(s, c))
        loss, gk, gc, gs = sim.rollout_grad(nsteps, checkpoint_every)
        ctx.save_for_backward(torch.from_numpy(gk), torch.from_numpy(gc), torch.from_numpy(gs),
                              spring_body.to("cpu", torch.int64))
        ctx.devices = (k.device, act_c.device, act_s.device)
        return torch.from_numpy(loss).to(k.device)

    @staticmethod
    def backward(ctx, grad_loss):
        gk, gc, gs, body = ctx.saved_tensors
        w = grad_loss.detach().to("cpu", torch.float32)[body]
        dk, dc, ds = ctx.devices
        return (gk * w).to(dk), (gc * w).to(dc), (gs * w).to(ds), None, None, None, None
