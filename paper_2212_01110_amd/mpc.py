"""Closed-loop model predictive control with warm starts (section 6,
closed-loop simulation).

At every step the risk-averse problem is solved from the current state of
every realisation at once (one spock_solve_batched launch, or one
spock_solve per realisation), the first input u^0 is applied, and the
realised disturbance picks the next state x+ = A(w) x + B(w) u^0. The
primal-dual solution of each realisation warm-starts its next solve (the
problem data do not change between steps, only the root state). The plant
update is the experiment's own simulation; every step of the method runs in
the library.
"""
from __future__ import annotations

import time

import numpy as np

from . import Problem, default_settings, solve_batched


def closed_loop(problem: Problem, A_w: np.ndarray, B_w: np.ndarray, x0: np.ndarray, branches: np.ndarray,
                settings=None, warm: bool = True, batched: bool = True, progress=None) -> dict:
    """Runs the loop for R realisations over S steps.

    A_w [d, nx, nx], B_w [d, nx, nu]: the plant for each disturbance value
    (the branches of the tree, in child order); x0 [nx]: the first state of
    every realisation; branches [R, S]: the realised disturbance index of each
    realisation and step; warm: start each solve from the previous solution
    (else from v = 0). Returns states [R, S+1, nx], inputs [R, S, nu],
    iterations and T evaluations [R, S], the status of every solve and the
    wall time of every step [S]. progress(t, seconds) is called after each
    step when given."""
    import torch
    s = settings or default_settings(eps_abs=1e-3, eps_rel=1e-3, max_iters=200000)
    branches = np.asarray(branches, dtype=np.int64)
    R, S = branches.shape
    nx, nu = problem.nx, problem.nu
    dev = torch.device("cuda")
    u_off = 1 + problem.tree.num_nodes * nx
    xs = np.zeros((R, S + 1, nx))
    us = np.zeros((R, S, nu))
    iters = np.zeros((R, S), dtype=np.int64)
    tev = np.zeros((R, S), dtype=np.int64)
    status = [[None] * S for _ in range(R)]
    step_s = np.zeros(S)
    xs[:, 0] = np.asarray(x0, float)
    vs = [torch.zeros(problem.n_v, dtype=problem.torch_dtype, device=dev) for _ in range(R)]
    for t in range(S):
        x0s = [torch.as_tensor(xs[r, t], dtype=torch.float64, device=dev) for r in range(R)]
        if not warm:
            for v in vs:
                v.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if batched:
            infos = solve_batched([problem] * R, x0s, vs, s)
        else:
            infos = [problem.solve(x0s[r], vs[r], s) for r in range(R)]
        torch.cuda.synchronize()
        step_s[t] = time.perf_counter() - t0
        for r in range(R):
            u0 = vs[r][u_off: u_off + nu].double().cpu().numpy()
            us[r, t] = u0
            iters[r, t], tev[r, t], status[r][t] = infos[r]["iters"], infos[r]["t_evals"], infos[r]["status"]
            w = branches[r, t]
            xs[r, t + 1] = A_w[w] @ xs[r, t] + B_w[w] @ u0
        if progress:
            progress(t, step_s[t])
    return {"states": xs, "inputs": us, "iters": iters, "t_evals": tev, "status": status,
            "step_seconds": step_s}
