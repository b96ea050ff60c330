"""Brute-force nested dynamic programming for single-input problems.

V^j(x) = x'Q_N x at leaves; V^i(x) = min_{u in [umin, umax]} AV@R_a over the
children c of (x'Q^c x + u'R^c u + V^c(A^c x + B^c u)) (eq. original-problem).
Every V^i is convex, so each one-dimensional minimisation is exact up to the
tolerance of the bounded scalar minimiser. AV@R is evaluated from its
definition (section 4.2) by scanning the breakpoints of the piecewise-linear
objective in t, written here independently of the oracle.
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import minimize_scalar

from .dense import tree_lists


def _avar(Z, p, a):
    if a == 0.0:
        return max(Z)
    best = np.inf
    for t in Z:
        val = t + sum(pk * max(zk - t, 0.0) for pk, zk in zip(p, Z)) / a
        best = min(best, val)
    return best


class NestedDP:
    """risk(i, Z): the risk measure of node i applied to its children's
    values (AV@R_a of the node, from its definition, when not given)."""

    def __init__(self, inst, xatol=1e-11, risk=None):
        assert inst.nu == 1
        self.inst = inst
        self.risk = risk
        self.ch, self.stage = tree_lists(inst.anc)
        self.xatol = xatol
        self.max_abs_x = 0.0

    def value(self, i, x):
        inst = self.inst
        self.max_abs_x = max(self.max_abs_x, float(np.max(np.abs(x))))
        if not self.ch[i]:
            if getattr(inst, "QNm", None) is not None:
                return float(x @ inst.QNm[i] @ x)
            return float(x @ (inst.qN[i] * x))
        p = [inst.prob[c] / inst.prob[i] for c in self.ch[i]]

        def obj(uu):
            Z = []
            for c in self.ch[i]:
                qx = inst.Qm[c] @ x if getattr(inst, "Qm", None) is not None else inst.q[c] * x
                rr = inst.Rm[c][0, 0] if getattr(inst, "Rm", None) is not None else inst.r[c][0]
                ell = float(x @ qx + rr * uu * uu)
                xc = inst.A[c] @ x + inst.B[c][:, 0] * uu
                Z.append(ell + self.value(c, xc))
            return self.risk(i, Z) if self.risk is not None else _avar(Z, p, inst.a_risk[i])

        res = minimize_scalar(obj, bounds=(inst.umin[i][0], inst.umax[i][0]),
                              method="bounded", options={"xatol": self.xatol, "maxiter": 500})
        if i == 0:
            self.u0 = res.x
        return float(res.fun)

    def solve(self):
        V = self.value(0, np.asarray(self.inst.x0, float))
        return V, self.u0
