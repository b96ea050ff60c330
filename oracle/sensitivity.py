"""Gradients of the optimal value V* and of the first input u^0.

envelope_gradients: V* from a converged primal-dual pair (envelope theorem
on the saddle form of the CP problem, section 3).
fixed_point_tangent / implicit_gradients: V* and u^0 by differentiating the
fixed point v* = T(v*) (section 3) with the Jacobians of T written out (see
the block comment below).

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
    if lay.dense_costs:
        raise NotImplementedError("gradients with respect to diagonal cost weights need diagonal costs")
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


# ---------------------------------------------------------------- implicit tangents
# The fixed point v* = T(v*, theta) (section 3) moves with theta = (x0, diag Q,
# diag Q_N) along dv solving (I - J_v) dv = J_theta dtheta, with J_v and
# J_theta the derivatives of T written out below piece by piece: prox_f is
# affine (s^0 - alpha, the projection on the affine set S1 whose offset is
# linear in x0, the linear projection on S2), the weights enter only the rows
# Q^{1/2} x^{anc} and Q_N^{1/2} x^j of L, and prox of g* differentiates through
# the Jacobian of the projection on S3 at w / alpha (clip masks of the boxes
# and of K*, R_+, and the Jacobian of the projection on a second-order cone).
# The tangent of s^0 is dV*, that of u^0 is du^0.

def _soc_jacobian(v: np.ndarray) -> np.ndarray:
    """Jacobian of the projection on {(w, t): ||w|| <= t} at v = (w, t)."""
    w, t = v[:-1], v[-1]
    n = v.shape[0]
    nw = np.linalg.norm(w)
    if nw <= t:
        return np.eye(n)
    if nw <= -t:
        return np.zeros((n, n))
    wh = w / nw
    J = np.zeros((n, n))
    J[:-1, :-1] = 0.5 * ((1.0 + t / nw) * np.eye(n - 1) - (t / nw) * np.outer(wh, wh))
    J[:-1, -1] = 0.5 * wh
    J[-1, :-1] = 0.5 * wh
    J[-1, -1] = 0.5
    return J


def _S3_jvp(lay, inst, p: np.ndarray, dp: np.ndarray) -> np.ndarray:
    """Derivative of proj_S3 at p applied to dp (blocks as in proj_S3)."""
    out = np.zeros_like(dp)
    for i in lay.nonleaf:
        kp, ny = lay.kpos(i), lay.ny[i]
        sl = slice(lay.e1y[i], lay.e1y[i] + kp)
        out[sl] = (p[sl] > 0.0) * dp[sl]
        sl = slice(lay.e1y[i] + kp, lay.e1y[i] + ny)
        out[sl] = dp[sl]
        out[lay.e1s[i]] = (p[lay.e1s[i]] > 0.0) * dp[lay.e1s[i]]
        _, _, cmin, cmax = lay.gamma(inst, i)
        sl = slice(lay.e1c[i], lay.e1c[i] + lay.nc)
        out[sl] = ((p[sl] > cmin) & (p[sl] < cmax)) * dp[sl]
    shift_of = lambda m: np.concatenate([np.zeros(m - 2), [0.5, -0.5]])  # noqa: E731
    for c in range(1, lay.num_nodes):
        sl = slice(lay.e2x[c], lay.e2b[c] + 1)
        m = sl.stop - sl.start
        out[sl] = _soc_jacobian(p[sl] - shift_of(m)) @ dp[sl]
    for j in lay.leaves:
        _, cmin, cmax = lay.gamma_N(inst, j)
        sl = slice(lay.e3x[j], lay.e3x[j] + lay.ncN)
        out[sl] = ((p[sl] > cmin) & (p[sl] < cmax)) * dp[sl]
        sl = slice(lay.e3q[j], lay.e3b[j] + 1)
        m = sl.stop - sl.start
        out[sl] = _soc_jacobian(p[sl] - shift_of(m)) @ dp[sl]
    return out


def _dL(lay, dsq, dsqN, z):
    """Derivative of L z in the square roots of the weights (only the rows
    Q^{1/2} x^{anc} and Q_N^{1/2} x^j depend on them)."""
    out = np.zeros(lay.n_eta)
    for c in range(1, lay.num_nodes):
        i = lay.anc[c]
        out[lay.e2x[c]: lay.e2x[c] + lay.nx] = dsq[c] * z[lay.x_off[i]: lay.x_off[i] + lay.nx]
    for j in lay.leaves:
        out[lay.e3q[j]: lay.e3q[j] + lay.nx] = dsqN[j] * z[lay.x_off[j]: lay.x_off[j] + lay.nx]
    return out


def _dLt(lay, dsq, dsqN, eta):
    """Derivative of L* eta in the square roots of the weights."""
    out = np.zeros(lay.n_z)
    for c in range(1, lay.num_nodes):
        i = lay.anc[c]
        out[lay.x_off[i]: lay.x_off[i] + lay.nx] += dsq[c] * eta[lay.e2x[c]: lay.e2x[c] + lay.nx]
    for j in lay.leaves:
        out[lay.x_off[j]: lay.x_off[j] + lay.nx] += dsqN[j] * eta[lay.e3q[j]: lay.e3q[j] + lay.nx]
    return out


def T_point(prob, v, x0):
    """The quantities of T(v) its derivative depends on: z+ and the
    pre-prox point w = eta + alpha L (2 z+ - z) of the dual update."""
    from .cp import T_apply
    from .operators import L_apply
    lay = prob.lay
    z, eta = lay.split(v)
    zp, _ = lay.split(T_apply(prob, v, x0))
    return zp, eta + prob.alpha * L_apply(lay, prob.inst, 2.0 * zp - z)


def T_jvp(prob, v, x0, dv, dx0=None, dq=None, dqN=None, point=None):
    """Derivative of T at (v, theta) along (dv, dtheta); dq and dqN are
    perturbations of the weight diagonals [num_nodes][nx]; point is
    T_point(prob, v, x0) if already at hand."""
    if prob.lay.dense_costs:
        raise NotImplementedError("gradients with respect to diagonal cost weights need diagonal costs")
    from .operators import L_apply, Lt_apply
    from .prox import proj_S1, proj_S2
    lay, inst, a = prob.lay, prob.inst, prob.alpha
    nx = lay.nx
    z, eta = lay.split(v)
    dz, deta = lay.split(dv)
    zero = np.zeros((lay.num_nodes, nx))
    sq, sqN = np.sqrt(inst.q), np.sqrt(inst.qN)
    dsq = zero if dq is None else np.where(sq > 0, 0.5 * np.asarray(dq) / np.where(sq > 0, sq, 1), 0.0)
    dsqN = zero if dqN is None else np.where(sqN > 0, 0.5 * np.asarray(dqN) / np.where(sqN > 0, sqN, 1), 0.0)
    dx0 = np.zeros(nx) if dx0 is None else np.asarray(dx0, float)
    zp, w = T_point(prob, v, x0) if point is None else point
    # tangent of zhat, then of z+ = prox_f(zhat) (affine in zhat and x0)
    dzhat = dz - a * (Lt_apply(lay, inst, deta) + _dLt(lay, dsq, dsqN, eta))
    dzp = proj_S2(lay, inst, dzhat)
    dzp[0] = dzhat[0]
    dxb = np.stack([lay.x_of(dzhat, i) for i in range(lay.num_nodes)])
    dub = np.zeros((lay.num_nodes, lay.nu))
    for i in lay.nonleaf:
        dub[i] = lay.u_of(dzhat, i)
    xs, us = proj_S1(lay, inst, prob.fac, dxb, dub, dx0)
    for i in range(lay.num_nodes):
        dzp[lay.x_off[i]: lay.x_off[i] + nx] = xs[i]
    for i in lay.nonleaf:
        dzp[lay.u_off[i]: lay.u_off[i] + lay.nu] = us[i]
    # tangent of w and of eta+ = w - alpha proj_S3(w / alpha)
    dw = deta + a * (L_apply(lay, inst, 2.0 * dzp - dz) + _dL(lay, dsq, dsqN, 2.0 * zp - z))
    detap = dw - _S3_jvp(lay, inst, w / a, dw)
    return np.concatenate([dzp, detap])


def fixed_point_tangent(prob, v, x0, dx0=None, dq=None, dqN=None, dense_max=3000, tol=1e-13):
    """dv with (I - J_v) dv = J_theta dtheta at the fixed point v. Up to
    dense_max unknowns J_v is assembled column by column and the system is
    solved by least squares (the minimum-norm tangent where the fixed point
    is not unique); above, by GMRES on the same operator."""
    n = prob.lay.n_v
    pt = T_point(prob, v, x0)
    rhs = T_jvp(prob, v, x0, np.zeros(n), dx0, dq, dqN, point=pt)
    if n <= dense_max:
        J = np.zeros((n, n))
        e = np.zeros(n)
        for k in range(n):
            e[k] = 1.0
            J[:, k] = T_jvp(prob, v, x0, e, point=pt)
            e[k] = 0.0
        return np.linalg.lstsq(np.eye(n) - J, rhs, rcond=None)[0]
    import scipy.sparse.linalg as sla
    op = sla.LinearOperator((n, n), matvec=lambda d: d - T_jvp(prob, v, x0, d, point=pt), dtype=float)
    sol, info = sla.gmres(op, rhs, rtol=tol, atol=0.0, restart=200, maxiter=50)
    if info != 0:
        raise RuntimeError(f"GMRES did not reach {tol} (info {info})")
    return sol


def implicit_gradients(prob, v, x0):
    """Full Jacobians of V* (= s^0) and u^0 with respect to x0 and the weight
    diagonals at the fixed point v (tiny trees: one tangent per parameter).
    Returns {"V_x0": [nx], "V_q": [nn, nx], "V_qN": [nn, nx], "u0_x0": [nu, nx],
    "u0_q": [nu, nn, nx], "u0_qN": [nu, nn, nx]}."""
    lay = prob.lay
    nx, nu, nn = lay.nx, lay.nu, lay.num_nodes
    u0 = slice(lay.u_off[0], lay.u_off[0] + nu)
    out = {"V_x0": np.zeros(nx), "V_q": np.zeros((nn, nx)), "V_qN": np.zeros((nn, nx)),
           "u0_x0": np.zeros((nu, nx)), "u0_q": np.zeros((nu, nn, nx)), "u0_qN": np.zeros((nu, nn, nx))}
    n = lay.n_v
    pt = T_point(prob, v, x0)
    J = np.zeros((n, n))
    e = np.zeros(n)
    for k in range(n):
        e[k] = 1.0
        J[:, k] = T_jvp(prob, v, x0, e, point=pt)
        e[k] = 0.0
    A = np.eye(n) - J
    pinv_solve = lambda b: np.linalg.lstsq(A, b, rcond=None)[0]  # noqa: E731
    zero = np.zeros(n)
    for k in range(nx):
        d = np.zeros(nx)
        d[k] = 1.0
        dv = pinv_solve(T_jvp(prob, v, x0, zero, dx0=d, point=pt))
        out["V_x0"][k], out["u0_x0"][:, k] = dv[0], dv[u0]
    for c in range(1, nn):
        for k in range(nx):
            d = np.zeros((nn, nx))
            d[c, k] = 1.0
            dv = pinv_solve(T_jvp(prob, v, x0, zero, dq=d, point=pt))
            out["V_q"][c, k], out["u0_q"][:, c, k] = dv[0], dv[u0]
    for j in lay.leaves:
        for k in range(nx):
            d = np.zeros((nn, nx))
            d[j, k] = 1.0
            dv = pinv_solve(T_jvp(prob, v, x0, zero, dqN=d, point=pt))
            out["V_qN"][j, k], out["u0_qN"][:, j, k] = dv[0], dv[u0]
    return out
