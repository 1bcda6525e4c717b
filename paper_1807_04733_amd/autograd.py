"""torch.autograd binding of the particle-in-cell run and its likelihood-ratio adjoint.

theta = (ln tau0 scale of every channel, every transmission-table node).  forward(theta)
runs the whole simulation on the GPU and returns the binned density and current;
backward(g_dens, g_cur) replays it with the same random streams and returns the
gradient estimate of sum(g_dens * density) + sum(g_cur * current) with respect to theta.
"""
from __future__ import annotations

from dataclasses import replace

import numpy as np
import torch

from .sim import PicSim


def theta0(problem) -> np.ndarray:
    """theta at the problem's own parameters (log-scales 0, the tables as they are)."""
    it = problem.instances[0]
    return np.concatenate([np.zeros(it.n_channels), it.T.ravel()])


def with_theta(problem, theta) -> object:
    """Problem with tau0 of channel c scaled by exp(theta_c) in every instance and every
    instance's transmission tables replaced by the remaining entries of theta."""
    theta = np.asarray(theta, np.float64)
    it0 = problem.instances[0]
    C = it0.n_channels
    T = theta[C:].reshape(it0.T.shape)
    if np.any(T < 0) or np.any(T > 1):
        raise ValueError("transmission nodes must stay in [0, 1]")
    insts = [replace(it, inv_tau0=it.inv_tau0 * np.exp(-theta[:C]), T=T.copy())
             for it in problem.instances]
    return replace(problem, instances=insts)


class PicFunction(torch.autograd.Function):
    """(dens, cur) = PicFunction.apply(theta, problem, estimator, sim_kwargs)."""

    @staticmethod
    def forward(ctx, theta, problem, estimator=0, sim_kwargs=None):
        kw = dict(sim_kwargs or {})
        kw.setdefault("adjoint", 1 if estimator == 0 else 2)
        prob = with_theta(problem, theta.detach().cpu().numpy())
        sim = PicSim(prob, **kw)
        sim.step()
        sim.counters()                      # surfaces device-side errors
        dens, cur = sim.deposit()
        ctx.sim = sim
        ctx.estimator = estimator
        ctx.theta_meta = (theta.dtype, theta.device)
        d = torch.cat([x.reshape(-1) for x in dens])
        c = torch.cat([x.reshape(-1) for x in cur])
        return d, c

    @staticmethod
    def backward(ctx, g_dens, g_cur):
        sim = ctx.sim
        grad = sim.backward(g_dens.detach() if g_dens is not None else None,
                            g_cur.detach() if g_cur is not None else None, ctx.estimator)
        sim.close()
        dtype, device = ctx.theta_meta
        return torch.as_tensor(grad, dtype=dtype, device=device), None, None, None
