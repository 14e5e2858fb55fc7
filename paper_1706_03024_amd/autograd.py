"""torch.autograd front end of the path-replay adjoint.

theta = [conc per (medium, dye slot)] + [QY per dye] + [sigma_s per medium]
(the fpt_grad_param_count order).  forward() uploads theta into the scene and
renders the film; backward() replays the same paths (same random numbers)
through fpt_render_adjoint to get d<grad_film, film>/d theta.  No path state
is stored between the two passes.
"""
from __future__ import annotations

import numpy as np
import torch

from .renderer import Scene


def split_params(desc, theta):
    """Splits theta into (conc, qy, sigma_s) host arrays."""
    th = np.asarray(theta, dtype=np.float64)
    nc = sum(len(m["dyes"]) for m in desc["media"])
    nd = len(desc["dyes"])
    return th[:nc], th[nc:nc + nd], th[nc + nd:]


def params_of(desc):
    """theta of a scene dictionary."""
    conc = [c for m in desc["media"] for _, c in m["dyes"]]
    qy = [d["qy"] for d in desc["dyes"]]
    ss = [m["sigma_s"] for m in desc["media"]]
    return np.array(conc + qy + ss, dtype=np.float64)


class FluorRender(torch.autograd.Function):
    """film = render(scene; theta).  Gradients flow to theta only.

    The path-replay gradient is valid only with the parameters the forward
    pass rendered with, so backward() sets the scene to this forward's theta
    for the replay and restores whatever the scene held before (another
    forward may have run on the same scene in between)."""

    @staticmethod
    def forward(ctx, theta, scene: Scene, run: dict, adjoint_run: dict | None = None):
        th = theta.detach().cpu().numpy().astype(np.float64)
        scene.set_params(*split_params(scene.desc, th))
        film = scene.render(run)
        ctx.scene = scene
        ctx.theta = th
        ctx.run = adjoint_run if adjoint_run is not None else run
        ctx.theta_dtype = theta.dtype
        ctx.theta_device = theta.device
        return film

    @staticmethod
    def backward(ctx, grad_film):
        sc = ctx.scene
        held = sc.theta.copy()
        swap = not np.array_equal(held, ctx.theta)
        if swap:
            sc.set_params(*split_params(sc.desc, ctx.theta))
        g = sc.render_adjoint(ctx.run, grad_film.contiguous().float())
        if swap:
            sc.set_params(*split_params(sc.desc, held))
        return g.to(ctx.theta_device, ctx.theta_dtype), None, None, None


def render_differentiable(scene: Scene, theta, run: dict, adjoint_run: dict | None = None):
    """film as a differentiable function of theta (a 1-D tensor)."""
    return FluorRender.apply(theta, scene, run, adjoint_run)
