"""torch.autograd glue over spock_solve / spock_backward (marshalling only).

SpockValue.apply(x0, q, problem, settings) returns (V*, u0) of the problem
with stage-cost diagonals q ([num_nodes][nx], FP64) and root state x0. When q
differs from the diagonals the problem was factored with, the forward pass
factors a problem with this q on the same tree (Alg. 1 runs again), so V*
and u0 are always functions of the q passed in. backward calls
spock_backward at that problem's solution with the incoming cotangents and
returns the gradients with respect to x0 and q."""
from __future__ import annotations

import numpy as np
import torch

from . import Problem, Settings, default_settings


class SpockValue(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x0: torch.Tensor, q: torch.Tensor, problem: Problem,
                settings: Settings | None = None):
        s = settings or default_settings(eps_abs=1e-10, eps_rel=1e-10, max_iters=400000)
        qh = q.detach().to("cpu", torch.float64).numpy()
        if problem.q is None:
            raise ValueError("the problem has dense cost matrices: no diagonal q to differentiate")
        if qh.shape != problem.q.shape:
            raise ValueError(f"q has shape {tuple(qh.shape)}, the problem {problem.q.shape}")
        if not np.array_equal(qh[1:], problem.q[1:]):
            problem = problem.refactor(q=qh)
        v = torch.zeros(problem.n_v, dtype=problem.torch_dtype, device=x0.device)
        x0c = x0.detach().to(torch.float64).contiguous()
        info = problem.solve(x0c, v, s)
        if info["status"] != "converged":
            raise RuntimeError(f"spock_solve did not converge: {info}")
        u_off = 1 + problem.tree.num_nodes * problem.nx
        V = v[0].to(torch.float64).clone()
        u0 = v[u_off: u_off + problem.nu].to(torch.float64).clone()
        ctx.save_for_backward(x0c, v)
        ctx.problem = problem
        return V, u0

    @staticmethod
    def backward(ctx, gV, gu0):
        x0c, v = ctx.saved_tensors
        gVv = float(gV) if gV is not None else 0.0
        gu = gu0.to(torch.float64).contiguous() if gu0 is not None else None
        gx, gq, _, info = ctx.problem.backward(v, x0c, gV=gVv, gu0=gu)
        if info["status"] != "converged":
            raise RuntimeError(f"spock_backward did not converge: {info}")
        return gx, gq, None, None
