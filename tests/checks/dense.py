"""Dense checkers written from textbook definitions (no oracle code).

* S1 projection: Euclidean projection on the affine set {D z1 = e} by the
  normal equations z - D'(DD')^{-1}(Dz - e), solved with lstsq.
* S2 projection: orthogonal projection on ker G via an orthonormal basis of the
  null space (scipy.linalg.null_space).
* Tree LQR: for a = 1 AV@R is the expectation (section 4.2), so with inactive
  boxes the problem is a risk-neutral LQR on the tree, solved by the Riccati
  recursion with probability-weighted children.
* Feasible conic point: from a trajectory, the epigraph variables of
  eq. min-s0-v1 are filled in with the optimal AV@R dual y of section 4.3.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg


def tree_lists(anc):
    nn = len(anc)
    ch = [[] for _ in range(nn)]
    for i in range(1, nn):
        ch[anc[i]].append(i)
    stage = np.zeros(nn, dtype=int)
    for i in range(1, nn):
        stage[i] = stage[anc[i]] + 1
    return ch, stage


def s1_dense_projection(inst, xbar, ubar, x0):
    """Projection of (xbar, ubar) on {x^0 = x0, x^c = A^c x^anc + B^c u^anc}."""
    anc = inst.anc
    nn, nx, nu = len(anc), inst.nx, inst.nu
    ch, _ = tree_lists(anc)
    nonleaf = [i for i in range(nn) if ch[i]]
    upos = {i: k for k, i in enumerate(nonleaf)}
    nvar = nn * nx + len(nonleaf) * nu
    rows = []
    rhs = []
    for k in range(nx):
        row = np.zeros(nvar)
        row[k] = 1.0
        rows.append(row)
        rhs.append(x0[k])
    for c in range(1, nn):
        i = anc[c]
        for k in range(nx):
            row = np.zeros(nvar)
            row[c * nx + k] = 1.0
            row[i * nx: i * nx + nx] -= inst.A[c][k]
            base = nn * nx + upos[i] * nu
            row[base: base + nu] -= inst.B[c][k]
            rows.append(row)
            rhs.append(0.0)
    D = np.array(rows)
    e = np.array(rhs)
    zb = np.concatenate([xbar.reshape(-1), np.concatenate([ubar[i] for i in nonleaf])])
    lam = np.linalg.lstsq(D @ D.T, D @ zb - e, rcond=None)[0]
    z = zb - D.T @ lam
    x = z[: nn * nx].reshape(nn, nx)
    u = np.zeros((nn, nu))
    for i in nonleaf:
        u[i] = z[nn * nx + upos[i] * nu: nn * nx + upos[i] * nu + nu]
    return x, u


def nullspace_projection(G, w):
    Z = scipy.linalg.null_space(G)
    return Z @ (Z.T @ w)


def tree_lqr(inst, x0):
    """Risk-neutral tree LQR (a = 1, boxes inactive): returns V* and u^0."""
    assert getattr(inst, "Qm", None) is None, "diagonal costs only"
    anc = inst.anc
    nn = len(anc)
    ch, stage = tree_lists(anc)
    N = stage.max()
    P = {}
    gains = {}
    for j in range(nn):
        if not ch[j]:
            P[j] = np.diag(inst.qN[j])
    for t in range(N - 1, -1, -1):
        for i in range(nn):
            if stage[i] != t:
                continue
            pc = {c: inst.prob[c] / inst.prob[i] for c in ch[i]}
            Rt = sum(pc[c] * (np.diag(inst.r[c]) + inst.B[c].T @ P[c] @ inst.B[c]) for c in ch[i])
            S = sum(pc[c] * (inst.B[c].T @ P[c] @ inst.A[c]) for c in ch[i])
            Qs = sum(pc[c] * (np.diag(inst.q[c]) + inst.A[c].T @ P[c] @ inst.A[c]) for c in ch[i])
            P[i] = Qs - S.T @ np.linalg.solve(Rt, S)
            gains[i] = -np.linalg.solve(Rt, S)
    return float(x0 @ P[0] @ x0), gains[0] @ x0


def feasible_conic_point(lay, inst, x, u):
    """z of eq. min-s0-v1 built from a trajectory (x, u): tau^c = l^c,
    s^j = l_N^j, s^i = AV@R of its children's (l^c + s^c) and y^i the optimal
    dual vector of that AV@R in the conic form (section 4.3): y_3 = t,
    y_1 = [Z - t]_+ / a, y_2 = [t - Z]_+ (a > 0); y_3 = max Z, y_2 = y_3 - Z,
    y_1 = 0 (a = 0). Offsets come from the layout object (pure bookkeeping)."""
    nn = lay.num_nodes
    z = np.zeros(lay.n_z)
    V = np.zeros(nn)
    for j in lay.leaves:
        V[j] = x[j] @ (inst.qN[j] * x[j])
    for i in range(nn):
        z[lay.x_off[i]: lay.x_off[i] + lay.nx] = x[i]
    for i in lay.nonleaf:
        z[lay.u_off[i]: lay.u_off[i] + lay.nu] = u[i]
    for t in range(lay.N - 1, -1, -1):
        for i in lay.stage_nodes[t]:
            chi = lay.children[i]
            n = len(chi)
            ell = np.array([x[i] @ (inst.q[c] * x[i]) + u[i] @ (inst.r[c] * u[i]) for c in chi])
            Z = ell + V[chi]
            p = inst.prob[chi] / inst.prob[i]
            a = inst.a_risk[i]
            if a == 0.0:
                tt = Z.max()
                y1 = np.zeros(n)
                y2 = tt - Z
            else:
                cands = [(tv + p @ np.maximum(Z - tv, 0.0) / a, tv) for tv in Z]
                tt = min(cands)[1]
                y1 = np.maximum(Z - tt, 0.0) / a
                y2 = np.maximum(tt - Z, 0.0)
            y = np.concatenate([y1, y2, [tt]])
            V[i] = p @ y1 + tt
            z[lay.y_off[i]: lay.y_off[i] + 2 * n + 1] = y
            for k, c in enumerate(chi):
                z[lay.tau_off[c]] = ell[k]
                z[lay.s_off[c]] = V[c]
    z[0] = V[0]
    return z, V


def cut_through(inst, x_star, u_star, rows_per_node=1):
    """Bounds of the polyhedral constraint rows placed between the value a
    solution gives them and the value of the zero-input trajectory (x from
    the dynamics with u = 0), so that the given solution becomes infeasible
    while the zero-input point stays strictly feasible (the first
    rows_per_node rows of every nonleaf node; the others keep their bounds).
    Returns a modified copy."""
    out = inst.copy()
    c = out.cons
    ch, _ = tree_lists(inst.anc)
    x0t = np.zeros((inst.num_nodes, inst.nx))
    x0t[0] = inst.x0
    for cc in range(1, inst.num_nodes):
        x0t[cc] = inst.A[cc] @ x0t[inst.anc[cc]]
    cmin, cmax = c.cmin.copy(), c.cmax.copy()
    for i in range(inst.num_nodes):
        if not ch[i]:
            continue
        r_star = c.Gx[i] @ x_star[i] + c.Gu[i] @ u_star[i]
        r_zero = c.Gx[i] @ x0t[i]
        for k in range(min(rows_per_node, r_star.shape[0])):
            mid = 0.5 * (r_star[k] + r_zero[k])
            if abs(r_star[k] - r_zero[k]) < 1e-6:
                continue
            if r_star[k] > r_zero[k]:
                cmax[i, k] = mid
            else:
                cmin[i, k] = mid
    out.cons = type(c)(c.Gx, c.Gu, cmin, cmax, c.GN, c.cNmin, c.cNmax)
    return out
