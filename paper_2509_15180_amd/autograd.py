"""torch.autograd bridge: the total tip-to-goal loss of a batch of rollouts as a
differentiable function of the sPAM pressures and end positions.

Forward: vine_sim_set_spams, vine_sim_reset, vine_sim_rollout, vine_sim_grad (the
adjoint runs with the forward, since it needs the same equilibria).  A trajectory
loss keeps a checkpoint every ``ckpt_every`` steps and lets vine_sim_grad recompute
the weighted states from them, instead of keeping every state.  Backward: the
stored gradients scaled by the incoming scalar.  The sides of the sPAMs are
discrete and are not differentiated.  A robot whose adjoint is flagged (a weighted
step that did not converge, or a singular adjoint system) raises VineError: its
derivative would be that of a branch the equilibrium conditions do not define.
"""
from __future__ import annotations

import numpy as np
import torch

from .vinesim import VINE_ESTATE, VineError, VineSim


class _RolloutLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pressure, s_start, s_end, sim: VineSim, side, goal, weights, ckpt_every):
        spam = np.stack([s_start.detach().cpu().numpy(), s_end.detach().cpu().numpy(),
                         np.asarray(side, np.float64), pressure.detach().cpu().numpy()], 1)
        stream = torch.cuda.current_stream()
        sim.set_spams(spam, stream=stream)
        sim.reset(stream=stream)
        sim.rollout(-1, ckpt_every=ckpt_every if weights is not None else 0, stream=stream)
        dP, d0, d1, loss, status = sim.grad(goal, weights, stream=stream)
        bad = torch.nonzero(status).flatten().tolist()
        if bad:
            raise VineError(VINE_ESTATE, f"adjoint flagged for robots {bad[:16]} (status "
                            f"{status[bad[:16]].tolist()}: bit 0 singular system, bit 1 a "
                            "weighted step that did not converge)")
        ctx.save_for_backward(dP, d0, d1)
        ctx.devices = (pressure.device, s_start.device, s_end.device)
        return loss.sum()

    @staticmethod
    def backward(ctx, g):
        dP, d0, d1 = ctx.saved_tensors
        dev = ctx.devices
        return ((g * dP).to(dev[0]), (g * d0).to(dev[1]), (g * d1).to(dev[2]),
                None, None, None, None, None)


def rollout_loss(sim: VineSim, pressure, s_start, s_end, side, goal, weights=None,
                 ckpt_every: int = 32):
    """L = sum_b sum_t w_t |tip_b(t) - goal_b|^2 after rolling every robot of ``sim``
    out to its target length with the given sPAM parameters (tensors [S], float64).
    ``weights`` None: the final state only; otherwise the weighted states are
    recomputed from checkpoints every ``ckpt_every`` steps."""
    return _RolloutLoss.apply(pressure, s_start, s_end, sim, side, goal, weights, ckpt_every)
