"""``torch.autograd.Function``s over the simulator's adjoint.

``TitanRollout.apply(k, act_c, act_s, sim, nsteps, checkpoint_every,
spring_body)`` returns, per body b, J_b = -(x-displacement of body b's centre
of mass) after ``nsteps`` steps from the simulation's current state, and is
differentiable with respect to the per-spring stiffness ``k`` and actuation
phasor (``act_c`` = amp cos(phase), ``act_s`` = amp sin(phase)); the phasors
go to the simulation as given (``titan_set_springs_phasor``). With the
parameters on the GPU the loss and gradients never leave GPU memory
(``titan_rollout_grad_device``).

``TitanVoxelRollout.apply(k, voxel_a, voxel_phi, sim, nsteps,
checkpoint_every, spring_body, sv_ptr, sv_idx)`` is the same loss with the
actuation given per voxel (``titan_set_voxel_actuation``: a spring's phasor is
the mean of its voxels' a (cos phi, sin phi)); its gradient with respect to
the voxel amplitudes and phases comes from the library
(``titan_rollout_grad_voxel``, mapped on the device).

Each forward pushes the parameters into the simulation and runs the rollout
and its adjoint once, keeping the gradients of every body's own loss.
Bodies do not interact, so the gradient of sum_b w_b J_b is each parameter's
unit-weight gradient scaled by the weight of its body: the backward is that
scaling, no second rollout.
"""
from __future__ import annotations

import numpy as np
import torch


def _np32(t):
    return t.detach().to("cpu", torch.float32).numpy()


class TitanRollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, k, act_c, act_s, sim, nsteps: int, checkpoint_every: int, spring_body):
        sim.set_springs(0, k=_np32(k))
        sim.set_springs_phasor(0, _np32(act_c), _np32(act_s))
        if k.is_cuda:
            # loss and gradients stay in GPU memory (titan_rollout_grad_device)
            loss, gk, gc, gs = sim.rollout_grad_device(nsteps, checkpoint_every)
        else:
            loss, gk, gc, gs = (torch.from_numpy(a) for a in sim.rollout_grad(nsteps, checkpoint_every))
        ctx.save_for_backward(gk, gc, gs, spring_body.to(gk.device, torch.int64))
        ctx.devices = (k.device, act_c.device, act_s.device)
        return loss.to(k.device)

    @staticmethod
    def backward(ctx, grad_loss):
        gk, gc, gs, body = ctx.saved_tensors
        w = grad_loss.detach().to(gk.device, torch.float32)[body]
        dk, dc, ds = ctx.devices
        return (gk * w).to(dk), (gc * w).to(dc), (gs * w).to(ds), None, None, None, None


class TitanVoxelRollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, k, voxel_a, voxel_phi, sim, nsteps: int, checkpoint_every: int, spring_body, sv_ptr, sv_idx):
        sim.set_springs(0, k=_np32(k))
        ptr = np.asarray(sv_ptr, np.int64)
        idx = np.asarray(sv_idx, np.int32)
        sim.set_voxel_actuation(_np32(voxel_a), _np32(voxel_phi), ptr, idx)
        loss, gk, ga, gp = sim.rollout_grad_voxel(nsteps, checkpoint_every, n_voxels=voxel_a.numel())
        sb = spring_body.to("cpu", torch.int64)
        # a voxel belongs to the body of any of its springs
        vbody = torch.zeros(voxel_a.numel(), dtype=torch.int64)
        seg = torch.from_numpy(np.repeat(np.arange(ptr.size - 1), np.diff(ptr)))
        vbody[torch.from_numpy(idx.astype(np.int64))] = sb[seg]
        ctx.save_for_backward(torch.from_numpy(gk), torch.from_numpy(ga), torch.from_numpy(gp), sb, vbody)
        ctx.devices = (k.device, voxel_a.device, voxel_phi.device)
        return torch.from_numpy(loss).to(k.device)

    @staticmethod
    def backward(ctx, grad_loss):
        gk, ga, gp, sb, vbody = ctx.saved_tensors
        g = grad_loss.detach().to("cpu", torch.float32)
        dk, da, dp = ctx.devices
        return ((gk * g[sb]).to(dk), (ga * g[vbody]).to(da), (gp * g[vbody]).to(dp), None, None, None, None, None,
                None)
