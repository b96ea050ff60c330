"""Canonical ordering of the primal vector z and the dual vector eta.

General problems (section 4.3 conic risk, section 4.1 constraints): when the
instance carries `risk` (per nonleaf node i: E^i [ny, n_i], F^i [ny, nnu],
b^i [ny] and kpos^i, the number of leading rows of the cone K = R^kpos_+ x
{0}) the block y^i has ny^i entries; when it carries `cons` (Gamma_x
[nn, nc, nx], Gamma_u [nn, nc, nu], bounds cmin, cmax [nn, nc] at nonleaf
nodes and Gamma_N [nn, ncN, nx], cNmin, cNmax at leaves) the constraint rows
of eta are Gamma_x x + Gamma_u u and Gamma_N x. Without them: AV@R_a
(ny = 2 n + 1, E = [a I, -I, 1]', b = (p, 0, 1), kpos = 2 n) and boxes
(Gamma = identity).

Follows section 5.2 ("Operator splitting"):
  z   = (s^0, z_1, z_2), z_1 = ((x^i) over all nodes, (u^i) over nonleaf nodes),
        z_2 = (y^i, tau^{[i]}, s^{[i]}) per nonleaf node i, where tau^{[i]} and
        s^{[i]} collect the slack of every child of i;
  eta = ((y^i, s^i - b^i'y^i, (x^i, u^i)) per nonleaf i,
         (Q^{1/2}x^{anc(i)}, R^{1/2}u^{anc(i)}, tau^i/2, tau^i/2) per non-root i,
         (x^j, (Q_N^{1/2}x^j, s^j/2, s^j/2)) per leaf j),
with nodes in breadth-first order (Fig. 1). The constraint maps Gamma are the
identity (box constraints), so the "(x^i, u^i)" and "x^j" parts are copies.
For AV@R (section 4.3) y^i has 2 n_i + 1 entries, n_i = |ch(i)|.

All offsets are built by walking the nodes in order and accumulating sizes.
"""
from __future__ import annotations

import numpy as np


class Layout:
    def __init__(self, inst):
        anc = np.asarray(inst.anc, dtype=np.int64)
        nn = anc.shape[0]
        nx, nu = int(inst.nx), int(inst.nu)
        self.nx, self.nu, self.num_nodes = nx, nu, nn
        self.anc = anc
        self.children = [[] for _ in range(nn)]
        for i in range(1, nn):
            if not (0 <= anc[i] < i):
                raise ValueError("ancestor must precede its child")
            self.children[anc[i]].append(i)
        self.stage = np.zeros(nn, dtype=np.int64)
        for i in range(1, nn):
            self.stage[i] = self.stage[anc[i]] + 1
        self.N = int(self.stage.max())
        self.nonleaf = [i for i in range(nn) if self.children[i]]
        self.leaves = [i for i in range(nn) if not self.children[i]]
        for j in self.leaves:
            if self.stage[j] != self.N:
                raise ValueError("every leaf must sit at the last stage")
        self.stage_nodes = [[i for i in range(nn) if self.stage[i] == t]
                            for t in range(self.N + 1)]
        self.risk = getattr(inst, "risk", None)
        self.cons = getattr(inst, "cons", None)
        # dense cost matrices (section 4.1 allows any Q, Q_N >= 0, R > 0)
        self.dense_costs = any(getattr(inst, k, None) is not None for k in ("Qm", "Rm", "QNm"))
        self.ny = np.zeros(nn, dtype=np.int64)
        for i in self.nonleaf:
            self.ny[i] = (len(self.risk.b[i]) if self.risk is not None else 2 * len(self.children[i]) + 1)
        self.nc = self.cons.Gx.shape[1] if self.cons is not None else nx + nu
        self.ncN = self.cons.GN.shape[1] if self.cons is not None else nx
        prob = np.asarray(inst.prob, dtype=float)
        # conditional probability of a child given its ancestor (the pi used
        # by the risk measure of the ancestor's node, section 4.4)
        self.p = np.ones(nn)
        for i in range(1, nn):
            self.p[i] = prob[i] / prob[anc[i]]

        # ---- z ----
        off = 0
        self.s_off = np.full(nn, -1, dtype=np.int64)
        self.s_off[0] = off
        off += 1
        self.x_off = np.zeros(nn, dtype=np.int64)
        for i in range(nn):
            self.x_off[i] = off
            off += nx
        self.u_off = np.full(nn, -1, dtype=np.int64)
        for i in self.nonleaf:
            self.u_off[i] = off
            off += nu
        self.y_off = np.full(nn, -1, dtype=np.int64)
        self.tau_off = np.full(nn, -1, dtype=np.int64)
        for i in self.nonleaf:
            self.y_off[i] = off
            off += self.ny[i]
            for c in self.children[i]:
                self.tau_off[c] = off
                off += 1
            for c in self.children[i]:
                self.s_off[c] = off
                off += 1
        self.n_z = off

        # ---- eta ----
        off = 0
        self.e1y = np.full(nn, -1, dtype=np.int64)
        self.e1s = np.full(nn, -1, dtype=np.int64)
        self.e1c = np.full(nn, -1, dtype=np.int64)
        for i in self.nonleaf:
            self.e1y[i] = off
            off += self.ny[i]
            self.e1s[i] = off
            off += 1
            self.e1c[i] = off
            off += self.nc
        # with boxes the constraint rows are (x^i, u^i)
        self.e1x = self.e1c
        self.e1u = np.where(self.e1c >= 0, self.e1c + nx, -1)
        self.e2x = np.full(nn, -1, dtype=np.int64)
        self.e2u = np.full(nn, -1, dtype=np.int64)
        self.e2a = np.full(nn, -1, dtype=np.int64)
        self.e2b = np.full(nn, -1, dtype=np.int64)
        for c in range(1, nn):
            self.e2x[c] = off
            off += nx
            self.e2u[c] = off
            off += nu
            self.e2a[c] = off
            off += 1
            self.e2b[c] = off
            off += 1
        self.e3x = np.full(nn, -1, dtype=np.int64)
        self.e3q = np.full(nn, -1, dtype=np.int64)
        self.e3a = np.full(nn, -1, dtype=np.int64)
        self.e3b = np.full(nn, -1, dtype=np.int64)
        for j in self.leaves:
            self.e3x[j] = off              # constraint rows (x^j itself with boxes)
            off += self.ncN
            self.e3q[j] = off
            off += nx
            self.e3a[j] = off
            off += 1
            self.e3b[j] = off
            off += 1
        self.n_eta = off
        self.n_v = self.n_z + self.n_eta

    # ---- the conic risk of each nonleaf node (section 4.3)
    def b_vector(self, i):
        """b^i; for AV@R (pi, 0_n, 1), pi the conditional probabilities of
        the children of i."""
        if self.risk is not None:
            return np.asarray(self.risk.b[i], float)
        ch = self.children[i]
        n = len(ch)
        return np.concatenate([self.p[ch], np.zeros(n), [1.0]])

    def E_matrix(self, i, a_risk=None):
        """E^i [ny, n_i]; for AV@R_a [a I; -I; 1']."""
        if self.risk is not None:
            return np.asarray(self.risk.E[i], float)
        n = len(self.children[i])
        return np.vstack([a_risk * np.eye(n), -np.eye(n), np.ones((1, n))])

    def F_matrix(self, i):
        """F^i [ny, nnu]; empty for AV@R."""
        if self.risk is not None:
            return np.asarray(self.risk.F[i], float).reshape(self.ny[i], -1)
        return np.zeros((self.ny[i], 0))

    def kpos(self, i):
        """rows of y^i in the nonnegative part of K* (the rest are free)."""
        if self.risk is not None:
            return int(self.risk.kpos[i])
        return 2 * len(self.children[i])

    # ---- constraint rows (section 4.1)
    def cost_matrices(self, inst, c):
        """(Q^c, R^c, Q_N^c) as matrices: the dense ones when the instance
        carries them, else the diagonals."""
        Q = inst.Qm[c] if getattr(inst, "Qm", None) is not None else np.diag(inst.q[c])
        R = inst.Rm[c] if getattr(inst, "Rm", None) is not None else np.diag(inst.r[c])
        QN = inst.QNm[c] if getattr(inst, "QNm", None) is not None else np.diag(inst.qN[c])
        return Q, R, QN

    def cost_roots(self, inst, c):
        """Symmetric positive semidefinite square roots of (Q^c, R^c, Q_N^c),
        the blocks that multiply x and u in the cost rows of eta (section
        5.2): V diag(sqrt(lambda)) V' from the eigendecomposition."""
        def root(M):
            lam, V = np.linalg.eigh(0.5 * (M + M.T))
            return (V * np.sqrt(np.maximum(lam, 0.0))) @ V.T
        cache = self.__dict__.setdefault("_roots", {})
        if c not in cache:
            cache[c] = tuple(root(M) for M in self.cost_matrices(inst, c))
        return cache[c]

    def gamma(self, inst, i):
        """(Gamma_x, Gamma_u, cmin, cmax) of nonleaf i."""
        if self.cons is not None:
            c = self.cons
            return c.Gx[i], c.Gu[i], c.cmin[i], c.cmax[i]
        nx, nu = self.nx, self.nu
        Gx = np.vstack([np.eye(nx), np.zeros((nu, nx))])
        Gu = np.vstack([np.zeros((nx, nu)), np.eye(nu)])
        return Gx, Gu, np.concatenate([inst.xmin[i], inst.umin[i]]), np.concatenate([inst.xmax[i], inst.umax[i]])

    def gamma_N(self, inst, j):
        """(Gamma_N, cmin, cmax) of leaf j."""
        if self.cons is not None:
            c = self.cons
            return c.GN[j], c.cNmin[j], c.cNmax[j]
        return np.eye(self.nx), inst.xmin[j], inst.xmax[j]

    def split(self, v):
        return v[: self.n_z], v[self.n_z:]

    def x_of(self, z, i):
        return z[self.x_off[i]: self.x_off[i] + self.nx]

    def u_of(self, z, i):
        return z[self.u_off[i]: self.u_off[i] + self.nu]

    def unpack_xu(self, z):
        x = np.stack([self.x_of(z, i) for i in range(self.num_nodes)])
        u = np.zeros((self.num_nodes, self.nu))
        for i in self.nonleaf:
            u[i] = self.u_of(z, i)
        return x, u
