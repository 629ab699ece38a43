"""FWI gradients as torch.autograd.Functions over the HIP adjoint (fd3d_forward_ckpt /
fd3d_adjoint / fd3d_gradient).

``Traces.apply(lam, mu, rho, shot, opts)`` returns the traces of one shot; its backward
takes dL/dtraces as the residual and returns dL/dlam, dL/dmu, dL/drho.  The checkpoints
stay on the GPU between forward and backward.

``Misfit.apply(lam, mu, rho, shots, d_obs, opts)`` returns J = 1/2 sum over shots of
|d - d_obs|^2 and computes the gradient eagerly, one shot at a time through one
gradient workspace (memory stays at one shot's checkpoints); backward scales it.

A shot is a dict: src_pos, moment, force, wavelet, rec_pos.  opts: dx (one spacing or
(dx, dy, dz)), dt, nt, sponge, sponge_alpha, ckpt_every, dtype.
"""
from __future__ import annotations

from typing import Dict, List, Sequence

import torch

from .simulator import Simulator


def _sim(lam, mu, rho, opts) -> Simulator:
    return Simulator(lam.detach(), mu.detach(), rho.detach(), opts["dx"], opts["dt"], opts["nt"],
                     dtype=opts.get("dtype", torch.float32), sponge=opts.get("sponge", 20),
                     sponge_alpha=opts.get("sponge_alpha", 0.0), device=lam.device)


def _shot_args(shot: Dict):
    return dict(src_pos=shot["src_pos"], moment=shot.get("moment", (0.0,) * 6), force=shot.get("force", (0.0,) * 3),
                wavelet=shot["wavelet"], rec_pos=shot["rec_pos"])


class Traces(torch.autograd.Function):
    @staticmethod
    def forward(ctx, lam, mu, rho, shot, opts):
        sim = _sim(lam, mu, rho, opts)
        gws = sim.grad_workspace(opts.get("ckpt_every", 50))
        tr = sim.forward_ckpt(gws, **_shot_args(shot))
        ctx.sim, ctx.gws, ctx.shot = sim, gws, shot
        return tr

    @staticmethod
    def backward(ctx, grad_traces):
        sim, gws = ctx.sim, ctx.gws
        g = [torch.zeros_like(sim.lam) for _ in range(3)]
        sim.adjoint(gws, grad_traces.contiguous(), *g, **_shot_args(ctx.shot))
        ctx.sim = ctx.gws = None
        return g[0], g[1], g[2], None, None


class Misfit(torch.autograd.Function):
    @staticmethod
    def forward(ctx, lam, mu, rho, shots: Sequence[Dict], d_obs: List[torch.Tensor], opts):
        sim = _sim(lam, mu, rho, opts)
        gws = sim.grad_workspace(opts.get("ckpt_every", 50))
        g = [torch.zeros_like(sim.lam) for _ in range(3)]
        J = torch.zeros(1, dtype=sim.dtype, device=sim.device)
        for shot, obs in zip(shots, d_obs):
            _, j = sim.gradient(gws, obs, *g, **_shot_args(shot))
            J += j
        sim.close()
        ctx.save_for_backward(*g)
        return J[0]

    @staticmethod
    def backward(ctx, grad_J):
        gl, gm, gr = ctx.saved_tensors
        return grad_J * gl, grad_J * gm, grad_J * gr, None, None, None


def descent(lam, mu, rho, shots: Sequence[Dict], d_obs: List[torch.Tensor], opts, iters: int = 3,
            step: float = 0.02, shrink: float = 0.5, tries: int = 6):
    """A plain FWI loop: steepest descent on J = 1/2 sum |d - d_obs|^2 over (lam, mu, rho),
    each model array moved along its own gradient scaled so that the largest change is
    ``step`` times the array's largest value, with backtracking (step times ``shrink``, at
    most ``tries`` times) until J decreases.  Returns the final model and the misfit
    history [J0, J1, ...]."""
    model = [lam.detach().clone(), mu.detach().clone(), rho.detach().clone()]
    m = [a.clone().requires_grad_(True) for a in model]
    J = Misfit.apply(*m, shots, d_obs, opts)
    J.backward()
    hist = [float(J)]
    for _ in range(iters):
        g = [a.grad.detach() for a in m]
        a = step
        for _ in range(tries):
            trial = [x - a * float(x.abs().max()) * gx / max(float(gx.abs().max()), 1e-300)
                     for x, gx in zip(model, g)]
            Jt = float(Misfit.apply(*trial, shots, d_obs, opts))
            if Jt < hist[-1]:
                break
            a *= shrink
        else:
            break
        model = trial
        m = [x.clone().requires_grad_(True) for x in model]
        J = Misfit.apply(*m, shots, d_obs, opts)
        J.backward()
        hist.append(float(J))
    return model, hist
