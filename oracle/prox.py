"""Proximal maps of f and g* (sections 5.3 and 5.4).

prox_{alpha f} is separable (section 5.3): s^0 - alpha, the projection on the
dynamics set S1 (Alg. 1 offline, Alg. 2 online), and the projection on the
kernel set S2. prox_{alpha g*} uses the extended Moreau decomposition
(eq. prox:g) with the alpha that the printed formula drops:
prox_{alpha g*}(w) = w - alpha * proj_{S3}(w / alpha).
"""
from __future__ import annotations

import numpy as np

from .layout import Layout


# ---------------------------------------------------------------- S1 (Alg. 1)
def factor_s1(lay: Layout, inst):
    """Alg. 1: offline factorisation, stage N-1 down to 0.

    Returns per nonleaf node the matrix R~ (with its Cholesky factor) and K,
    per child A-bar = A + B K, and per node P."""
    nx, nu = lay.nx, lay.nu
    P, K, Rt, Rchol, Abar = {}, {}, {}, {}, {}
    for j in lay.leaves:
        P[j] = np.eye(nx)
    for t in range(lay.N - 1, -1, -1):
        for i in lay.stage_nodes[t]:
            ch = lay.children[i]
            Ptil = {c: inst.B[c].T @ P[c] for c in ch}
            Rt[i] = np.eye(nu) + sum(Ptil[c] @ inst.B[c] for c in ch)
            Rchol[i] = np.linalg.cholesky(Rt[i])
            rhs = sum(Ptil[c] @ inst.A[c] for c in ch)
            K[i] = -_chol_solve(Rchol[i], rhs)
            for c in ch:
                Abar[c] = inst.A[c] + inst.B[c] @ K[i]
            P[i] = np.eye(nx) + K[i].T @ K[i] + sum(Abar[c].T @ P[c] @ Abar[c] for c in ch)
    return {"P": P, "K": K, "Rt": Rt, "Rchol": Rchol, "Abar": Abar}


def _chol_solve(Lc, rhs):
    y = np.linalg.solve(Lc, rhs)
    return np.linalg.solve(Lc.T, y)


# ---------------------------------------------------------------- S1 (Alg. 2)
def proj_S1(lay: Layout, inst, fac, xbar: np.ndarray, ubar: np.ndarray, x0: np.ndarray):
    """Alg. 2: backward sweep for (d, q), then forward sweep for (u, x).

    xbar [nn, nx] and ubar [nn, nu] are the point to project; the root state is
    fixed to x0. The forward sweep uses the literal dynamics A x + B u."""
    nx, nu = lay.nx, lay.nu
    q = {j: -xbar[j] for j in lay.leaves}
    d = {}
    for t in range(lay.N - 1, -1, -1):
        for i in lay.stage_nodes[t]:
            ch = lay.children[i]
            d[i] = _chol_solve(fac["Rchol"][i], ubar[i] - sum(inst.B[c].T @ q[c] for c in ch))
            q[i] = (fac["K"][i].T @ (d[i] - ubar[i]) - xbar[i]
                    + sum(fac["Abar"][c].T @ (fac["P"][c] @ inst.B[c] @ d[i] + q[c]) for c in ch))
    x = np.zeros((lay.num_nodes, nx))
    u = np.zeros((lay.num_nodes, nu))
    x[0] = x0
    for t in range(lay.N):
        for i in lay.stage_nodes[t]:
            u[i] = fac["K"][i] @ x[i] + d[i]
            for c in lay.children[i]:
                x[c] = inst.A[c] @ x[i] + inst.B[c] @ u[i]
    return x, u


# ---------------------------------------------------------------- S2
def s2_matrix(lay: Layout, inst, i):
    """[E' -I -I; F' 0 0] of S2^i (section 5.2), acting on (y, tau^{[i]},
    s^{[i]}); for AV@R F is empty and E' y = a y_1 - y_2 + y_3 1."""
    n = len(lay.children[i])
    E = lay.E_matrix(i, inst.a_risk[i])
    F = lay.F_matrix(i)
    top = np.hstack([E.T, -np.eye(n), -np.eye(n)])
    if F.shape[1] == 0:
        return top
    return np.vstack([top, np.hstack([F.T, np.zeros((F.shape[1], 2 * n))])])


def proj_S2_block(G: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Projection of w on ker G: w - G' (G G')^+ G w (least squares, so that
    dependent rows of G are allowed)."""
    return w - G.T @ np.linalg.lstsq(G @ G.T, G @ w, rcond=None)[0]


def proj_S2(lay: Layout, inst, z: np.ndarray) -> np.ndarray:
    """Apply the S2 projection to every z_2 block of z (returns a copy)."""
    out = z.copy()
    for i in lay.nonleaf:
        idx = s2_indices(lay, i)
        out[idx] = proj_S2_block(s2_matrix(lay, inst, i), z[idx])
    return out


def s2_indices(lay: Layout, i):
    ch = lay.children[i]
    return np.concatenate([np.arange(lay.y_off[i], lay.y_off[i] + lay.ny[i]),
                           lay.tau_off[ch], lay.s_off[ch]]).astype(np.int64)


# ---------------------------------------------------------------- prox f
def prox_f(lay: Layout, inst, fac, zhat: np.ndarray, alpha: float, x0: np.ndarray):
    """prox_{alpha f}(zhat) with f = s^0 + delta_S1 + delta_S2 (eq. f)."""
    out = proj_S2(lay, inst, zhat)
    out[0] = zhat[0] - alpha
    xbar = np.zeros((lay.num_nodes, lay.nx))
    ubar = np.zeros((lay.num_nodes, lay.nu))
    for i in range(lay.num_nodes):
        xbar[i] = lay.x_of(zhat, i)
    for i in lay.nonleaf:
        ubar[i] = lay.u_of(zhat, i)
    x, u = proj_S1(lay, inst, fac, xbar, ubar, x0)
    for i in range(lay.num_nodes):
        out[lay.x_off[i]: lay.x_off[i] + lay.nx] = x[i]
    for i in lay.nonleaf:
        out[lay.u_off[i]: lay.u_off[i] + lay.nu] = u[i]
    return out


# ---------------------------------------------------------------- S3 and g*
def proj_soc(v: np.ndarray) -> np.ndarray:
    """Projection on SOC = {(w, t): ||w|| <= t}, last coordinate t."""
    w, t = v[:-1], v[-1]
    nw = np.linalg.norm(w)
    if nw <= t:
        return v.copy()
    if nw <= -t:
        return np.zeros_like(v)
    c = 0.5 * (nw + t)
    return np.concatenate([c * w / nw, [c]])


def _proj_translated_soc(v: np.ndarray) -> np.ndarray:
    """Projection on SOC + (0, ..., 0, 1/2, -1/2) (eq. S3-def)."""
    shift = np.zeros_like(v)
    shift[-2], shift[-1] = 0.5, -0.5
    return shift + proj_soc(v - shift)


def proj_S3(lay: Layout, inst, w: np.ndarray) -> np.ndarray:
    """Projection on S3 (eq. S3-def): y^i on K* = R^kpos_+ x R^{ny - kpos}
    (the dual of R^kpos_+ x {0}; for AV@R kpos = 2n), s^i - b'y^i on R_+, the
    constraint rows on C^i = [cmin, cmax] (the state/input box when Gamma is
    the identity), the SOC blocks, and the leaves' rows on C_N^j."""
    p = np.zeros_like(w)
    for i in lay.nonleaf:
        ny, kp = lay.ny[i], lay.kpos(i)
        y = w[lay.e1y[i]: lay.e1y[i] + ny]
        p[lay.e1y[i]: lay.e1y[i] + kp] = np.maximum(y[:kp], 0.0)
        p[lay.e1y[i] + kp: lay.e1y[i] + ny] = y[kp:]
        p[lay.e1s[i]] = max(w[lay.e1s[i]], 0.0)
        _, _, cmin, cmax = lay.gamma(inst, i)
        sl = slice(lay.e1c[i], lay.e1c[i] + lay.nc)
        p[sl] = np.clip(w[sl], cmin, cmax)
    for c in range(1, lay.num_nodes):
        sl = slice(lay.e2x[c], lay.e2b[c] + 1)
        p[sl] = _proj_translated_soc(w[sl])
    for j in lay.leaves:
        _, cmin, cmax = lay.gamma_N(inst, j)
        sl = slice(lay.e3x[j], lay.e3x[j] + lay.ncN)
        p[sl] = np.clip(w[sl], cmin, cmax)
        sl = slice(lay.e3q[j], lay.e3b[j] + 1)
        p[sl] = _proj_translated_soc(w[sl])
    return p


def prox_gstar(lay: Layout, inst, w: np.ndarray, alpha: float) -> np.ndarray:
    """prox_{alpha g*}(w) = w - alpha proj_S3(w / alpha), g = delta_S3."""
    return w - alpha * proj_S3(lay, inst, w / alpha)
