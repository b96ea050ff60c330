"""Gradients of the optimal value V* from a converged primal-dual pair
(envelope theorem on the saddle form of the CP problem, section 3).

V*(theta) = min_z max_eta f(z) + <L z, eta> - g*(eta). The weights enter
only through L (the rows Q^{1/2} x^{anc} and Q_N^{1/2} x^j of the definition
of eta, section 5.2), so dV*/d sqrt(q) = <(dL/d sqrt(q)) z*, eta*>. The root
state enters through the affine set S1 = {D z1 = e(x0)}: with a multiplier
lam of D z1 = e, optimality in z1 reads D' lam = (L* eta*)_{z1} and
dV*/dx0 = lam on the rows x^0 = x0 (solved by least squares).
Parity pinned by central differences of oracle solves (tests).
"""
from __future__ import annotations

import numpy as np

from .operators import Lt_apply


def envelope_gradients(prob, v):
    lay, inst = prob.lay, prob.inst
    nx, nu = lay.nx, lay.nu
    z, eta = lay.split(v)
    # ---- diag Q (non-root c) and diag Q_N (leaves)
    gq = np.zeros((lay.num_nodes, nx))
    gqN = np.zeros((lay.num_nodes, nx))
    for c in range(1, lay.num_nodes):
        i = lay.anc[c]
        xi = z[lay.x_off[i]: lay.x_off[i] + nx]
        e = eta[lay.e2x[c]: lay.e2x[c] + nx]
        gq[c] = xi * e / (2.0 * np.sqrt(inst.q[c]))
    for j in lay.leaves:
        xj = z[lay.x_off[j]: lay.x_off[j] + nx]
        e = eta[lay.e3q[j]: lay.e3q[j] + nx]
        gqN[j] = xj * e / (2.0 * np.sqrt(inst.qN[j]))
    # ---- x0 through the multiplier of D z1 = e(x0)
    nonleaf = lay.nonleaf
    upos = {i: k for k, i in enumerate(nonleaf)}
    nn = lay.num_nodes
    nvar = nn * nx + len(nonleaf) * nu
    rows = []
    for k in range(nx):
        r = np.zeros(nvar)
        r[k] = 1.0
        rows.append(r)
    for c in range(1, nn):
        i = lay.anc[c]
        for k in range(nx):
            r = np.zeros(nvar)
            r[c * nx + k] = 1.0
            r[i * nx: i * nx + nx] -= inst.A[c][k]
            r[nn * nx + upos[i] * nu: nn * nx + upos[i] * nu + nu] -= inst.B[c][k]
            rows.append(r)
    D = np.array(rows)
    Lte = Lt_apply(lay, inst, eta)
    g1 = np.concatenate([np.concatenate([Lte[lay.x_off[i]: lay.x_off[i] + nx] for i in range(nn)]),
                         np.concatenate([Lte[lay.u_off[i]: lay.u_off[i] + nu] for i in nonleaf])])
    lam = np.linalg.lstsq(D.T, g1, rcond=None)[0]
    return {"x0": lam[:nx], "q": gq, "qN": gqN}
