"""AV@R and the exact nested risk-averse cost of a policy (section 4.2 and
eq. original-problem).

AV@R_a[Z] = min_t { t + (1/a) E^p[Z - t]_+ } for a > 0 (t is a scalar) and
max Z for a = 0. The objective is convex and piecewise linear in t with
breakpoints at the values Z_c, so the minimum is attained at one of them and
is found exactly by evaluating every breakpoint.
"""
from __future__ import annotations

import numpy as np


def avar(Z: np.ndarray, p: np.ndarray, a: float) -> float:
    Z = np.asarray(Z, float)
    p = np.asarray(p, float)
    if a == 0.0:
        return float(np.max(Z))
    vals = [t + np.sum(p * np.maximum(Z - t, 0.0)) / a for t in Z]
    return float(min(vals))


def nested_cost(lay, inst, x: np.ndarray, u: np.ndarray) -> float:
    """Nested AV@R cost of the trajectory (x, u) on the tree: leaves carry
    x'Q_N x; each nonleaf i carries AV@R_{a_i} over its children c of
    (x^i'Q^c x^i + u^i'R^c u^i + V^c) with conditional probabilities."""
    V = np.zeros(lay.num_nodes)
    for j in lay.leaves:
        V[j] = x[j] @ (inst.qN[j] * x[j])
    for t in range(lay.N - 1, -1, -1):
        for i in lay.stage_nodes[t]:
            ch = lay.children[i]
            Z = np.array([x[i] @ (inst.q[c] * x[i]) + u[i] @ (inst.r[c] * u[i]) + V[c]
                          for c in ch])
            V[i] = avar(Z, lay.p[ch], inst.a_risk[i])
    return float(V[0])
