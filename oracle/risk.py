"""AV@R, general conic risk measures and the nested risk-averse cost of a
policy (sections 4.2, 4.3 and eq. original-problem).

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


def conic_risk(E, F, b, kpos, Z) -> float:
    """rho(Z) = max { mu'Z : E mu + F nu <=_K b } (section 4.3), K the first
    kpos rows nonnegative (<=), the rest zero (=); a linear program in
    (mu, nu), solved by scipy's HiGHS."""
    from scipy.optimize import linprog
    E = np.asarray(E, float)
    F = np.asarray(F, float).reshape(E.shape[0], -1)
    b = np.asarray(b, float)
    n, nnu = E.shape[1], F.shape[1]
    A = np.hstack([E, F])
    c = -np.concatenate([np.asarray(Z, float), np.zeros(nnu)])
    kw = {}
    if kpos > 0:
        kw.update(A_ub=A[:kpos], b_ub=b[:kpos])
    if kpos < A.shape[0]:
        kw.update(A_eq=A[kpos:], b_eq=b[kpos:])
    res = linprog(c, bounds=[(None, None)] * (n + nnu), method="highs",
                  options={"primal_feasibility_tolerance": 1e-10, "dual_feasibility_tolerance": 1e-10}, **kw)
    if res.status != 0:
        raise RuntimeError(f"risk LP failed: {res.message}")
    return float(-res.fun)


def node_risk(lay, inst, i, Z) -> float:
    """The risk measure of nonleaf node i applied to its children's values."""
    if lay.risk is None:
        return avar(Z, lay.p[lay.children[i]], inst.a_risk[i])
    return conic_risk(lay.E_matrix(i), lay.F_matrix(i), lay.b_vector(i), lay.kpos(i), Z)


def nested_cost(lay, inst, x: np.ndarray, u: np.ndarray) -> float:
    """Nested risk-averse cost of the trajectory (x, u) on the tree: leaves
    carry x'Q_N x; each nonleaf i carries its risk measure (AV@R_{a_i} with
    conditional probabilities, or the conic risk of section 4.3) over its
    children c of (x^i'Q^c x^i + u^i'R^c u^i + V^c)."""
    V = np.zeros(lay.num_nodes)
    for j in lay.leaves:
        V[j] = x[j] @ lay.cost_matrices(inst, j)[2] @ x[j]
    for t in range(lay.N - 1, -1, -1):
        for i in lay.stage_nodes[t]:
            ch = lay.children[i]
            Z = np.array([x[i] @ lay.cost_matrices(inst, c)[0] @ x[i] + u[i] @ lay.cost_matrices(inst, c)[1] @ u[i]
                          + V[c] for c in ch])
            V[i] = node_risk(lay, inst, i, Z)
    return float(V[0])
