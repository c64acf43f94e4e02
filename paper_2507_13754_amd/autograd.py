"""Sound-speed misfit with an adjoint-series gradient, as a torch autograd op.

J(c) = 1/2 sum_{f, s} || R p_{f,s}(c) - p_obs_{f,s} ||^2, where p_{f,s} is the
L-term Born series at frequency f for source s and R samples receiver cells.
The gradient dJ/dc(x) = sum_f Re( sum_s g_V(x) dV/dc(x) ) comes from the
library's adjoint of the truncated series (tbs_adjoint: the series run with
conj(G^) and conj(V), paired with the forward partial sums), so the backward
pass costs about one forward series per (f, s) besides the forward replay.
"""
from __future__ import annotations

import math
from typing import List, Sequence

import torch

from . import Plan, TBS_ADJ_STORE, background_k0


class MisfitProblem:
    """Plans and data of one misfit: one plan (batch = number of sources) per
    frequency; all tensors live on one device."""

    def __init__(self, shape: Sequence[int], dx: float, freqs: Sequence[float], c0: float,
                 alpha0: float, y: float, sources: torch.Tensor, receivers: torch.Tensor,
                 p_obs: Sequence[torch.Tensor], nterms: int, dtype=torch.complex64,
                 adjoint_flags: int = TBS_ADJ_STORE):
        self.shape = tuple(shape)
        self.freqs = list(freqs)
        self.c0, self.alpha0, self.y = float(c0), float(alpha0), float(y)
        self.nterms = int(nterms)
        self.dtype = dtype
        self.flags = adjoint_flags
        self.sources = sources.to(dtype).contiguous()
        self.receivers = receivers.to(torch.int64).contiguous()     # flat spatial indices
        self.p_obs = [p.to(dtype).contiguous() for p in p_obs]
        nsrc = self.sources.shape[0]
        self.plans: List[Plan] = []
        for f in self.freqs:
            om = 2.0 * math.pi * f
            k0 = background_k0(om, self.c0, self.alpha0, self.y)
            self.plans.append(Plan(self.shape, dx, k0, dtype=dtype, batch=nsrc).tabulate())

    def close(self):
        for p in self.plans:
            p.close()
        self.plans = []


class TBSMisfit(torch.autograd.Function):
    """J = TBSMisfit.apply(c, problem); c: float64 [...grid] on the device."""

    @staticmethod
    def forward(ctx, c: torch.Tensor, problem: MisfitProblem):
        c = c.contiguous()
        saved = []
        J = torch.zeros((), dtype=torch.float64, device=c.device)
        for f, plan, pobs in zip(problem.freqs, problem.plans, problem.p_obs):
            om = 2.0 * math.pi * f
            V, dVdc = plan.potential(c, om, problem.c0, problem.alpha0, problem.y, with_derivative=True)
            p = plan.solve(problem.sources, V, problem.nterms)
            q, Jf = plan.misfit(p, problem.receivers, pobs)
            J = J + Jf[0]
            saved.append((V, dVdc, q))
        ctx.problem = problem
        ctx.saved = saved
        return J

    @staticmethod
    def backward(ctx, gJ):
        problem = ctx.problem
        grad = None
        for plan, (V, dVdc, q) in zip(problem.plans, ctx.saved):
            g = plan.adjoint(problem.sources, V, problem.nterms, q, flags=problem.flags)
            grad = plan.speed_gradient(g, dVdc, out=grad, accumulate=grad is not None)
        ctx.saved = None
        return grad * gJ, None
