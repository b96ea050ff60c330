"""Dense interior-point checker of the epigraph program (section 5.1,
eq. min-s0-v1), written from the program's statement, not from the oracle.

Variables (own indexing): x^i for every node, u^i for nonleaf nodes, per
nonleaf node i the conic dual y^i of its risk measure, the
stage-cost bound tau^c of every non-root node and the cost-to-go bound s^i of
every node; s^0 is the objective. Constraints:
  x^0 = x0,  x^c = A^c x^i + B^c u^i                       (dynamics)
  E^i'y = tau + s (one row per child), F^i'y = 0              (section 4.3)
  y in K* (its first kpos entries >= 0), b^i'y <= s^i
  AV@R_a (default): E = [a I; -I; 1'], F empty, b = (p, 0, 1), kpos = 2 n_i,
  with y3 >= -1 added (keeps the optimum; see below)
  cmin <= Gamma_x x^i + Gamma_u u^i <= cmax, cNmin <= Gamma_N x^j <= cNmax
  (the state/input boxes when the instance carries no constraint data)
  x^i'Q^c x^i + u^i'R^c u^i <= tau^c,  x^j'Q_N x^j <= s^j      (cost epigraphs)

Solved by the logarithmic barrier method with equality-constrained Newton
steps (Boyd & Vandenberghe, Convex Optimization, sections 10.2 and 11.3) from
a strictly feasible point built by hand, to a duality-gap bound m/t <= gap.
Derivatives are taken by central differences of such solves (the
centering point's own sensitivity converges too slowly where a constraint is
weakly active to serve as a pin).
"""
from __future__ import annotations

import numpy as np

from .dense import tree_lists


class EpigraphIPM:
    def __init__(self, inst, x0=None):
        assert getattr(inst, "Qm", None) is None and getattr(inst, "Rm", None) is None, "diagonal costs only"
        self.inst = inst
        self.x0 = np.asarray(inst.x0 if x0 is None else x0, float)
        anc = np.asarray(inst.anc)
        self.nn = nn = len(anc)
        self.nx, self.nu = nx, nu = inst.nx, inst.nu
        self.ch, self.stage = tree_lists(anc)
        self.nonleaf = [i for i in range(nn) if self.ch[i]]
        self.leaves = [i for i in range(nn) if not self.ch[i]]
        # ---- variable indices
        n = 0
        self.ix = {}
        for i in range(nn):
            self.ix[i] = np.arange(n, n + nx)
            n += nx
        self.iu = {}
        for i in self.nonleaf:
            self.iu[i] = np.arange(n, n + nu)
            n += nu
        # the conic risk of every nonleaf node (section 4.3): AV@R_a unless the
        # instance carries a general one
        self.risk = getattr(inst, "risk", None)
        self.cons = getattr(inst, "cons", None)
        self.E, self.Fr, self.b, self.kpos = {}, {}, {}, {}
        for i in self.nonleaf:
            k = len(self.ch[i])
            p = inst.prob[self.ch[i]] / inst.prob[i]
            if self.risk is None:
                self.E[i] = np.vstack([inst.a_risk[i] * np.eye(k), -np.eye(k), np.ones((1, k))])
                self.Fr[i] = np.zeros((2 * k + 1, 0))
                self.b[i] = np.concatenate([p, np.zeros(k), [1.0]])
                self.kpos[i] = 2 * k
            else:
                self.E[i] = np.asarray(self.risk.E[i], float)
                self.b[i] = np.asarray(self.risk.b[i], float)
                self.Fr[i] = np.asarray(self.risk.F[i], float).reshape(len(self.b[i]), -1)
                self.kpos[i] = int(self.risk.kpos[i])
        self.iy = {}
        for i in self.nonleaf:
            ny = len(self.b[i])
            self.iy[i] = np.arange(n, n + ny)
            n += ny
        self.itau = {}
        for c in range(1, nn):
            self.itau[c] = n
            n += 1
        self.isv = {}
        for i in range(nn):
            self.isv[i] = n
            n += 1
        self.n = n
        self._build()

    # ------------------------------------------------------------------ data
    def _build(self):
        inst, nx, nu, n = self.inst, self.nx, self.nu, self.n
        anc = inst.anc
        F, h = [], []
        for k in range(nx):                                   # x^0 = x0
            row = np.zeros(n)
            row[self.ix[0][k]] = 1.0
            F.append(row)
            h.append(self.x0[k])
        for c in range(1, self.nn):                           # dynamics
            i = anc[c]
            for k in range(nx):
                row = np.zeros(n)
                row[self.ix[c][k]] = 1.0
                row[self.ix[i]] -= inst.A[c][k]
                row[self.iu[i]] -= inst.B[c][k]
                F.append(row)
                h.append(0.0)
        for i in self.nonleaf:                                # E'y = tau + s, F'y = 0
            for k, c in enumerate(self.ch[i]):
                row = np.zeros(n)
                row[self.iy[i]] = self.E[i][:, k]
                row[self.itau[c]] = -1.0
                row[self.isv[c]] = -1.0
                F.append(row)
                h.append(0.0)
            for col in self.Fr[i].T:
                row = np.zeros(n)
                row[self.iy[i]] = col
                F.append(row)
                h.append(0.0)
        self.F, self.h = np.array(F), np.array(h)
        self.n_x0_rows = nx
        # linear inequalities G z <= g
        G, g = [], []

        def add(idx, coef, rhs):
            row = np.zeros(n)
            row[idx] = coef
            G.append(row)
            g.append(rhs)
        for i in self.nonleaf:
            for k in range(self.kpos[i]):                       # y in K*
                add(self.iy[i][k], -1.0, 0.0)
            row = np.zeros(n)                                   # b'y <= s
            row[self.iy[i]] = self.b[i]
            row[self.isv[i]] = -1.0
            G.append(row)
            g.append(0.0)
            if self.risk is None:
                # y3 >= -1: the AV@R minimiser t = y3 is one of the
                # (nonnegative) child values, or for a = 1 any t <= min of
                # them, so the optimum stays feasible; without it the
                # direction (y1 + d 1, y3 - d) leaves every constraint and s^0
                # unchanged when a = 1 and the barrier problem has no minimiser
                add(self.iy[i][-1], -1.0, 1.0)

        def rows(idx_x, Gx, idx_u, Gu, lo, hi):                 # lo <= Gx x + Gu u <= hi
            for r in range(Gx.shape[0]):
                row = np.zeros(n)
                row[idx_x] = Gx[r]
                if idx_u is not None:
                    row[idx_u] = Gu[r]
                G.append(row)
                g.append(hi[r])
                G.append(-row)
                g.append(-lo[r])
        c = self.cons
        for i in range(self.nn):
            if i in self.iu:                                    # nonleaf
                if c is None:
                    rows(self.ix[i], np.eye(nx), None, None, inst.xmin[i], inst.xmax[i])
                    rows(self.iu[i], np.eye(nu), None, None, inst.umin[i], inst.umax[i])
                else:
                    rows(self.ix[i], c.Gx[i], self.iu[i], c.Gu[i], c.cmin[i], c.cmax[i])
            elif c is None:
                rows(self.ix[i], np.eye(nx), None, None, inst.xmin[i], inst.xmax[i])
            else:
                rows(self.ix[i], c.GN[i], None, None, c.cNmin[i], c.cNmax[i])
        self.G, self.g = np.array(G), np.array(g)
        # quadratic inequalities sum_k w_k z_{idx_k}^2 - z_j <= 0
        self.quads = []
        for c in range(1, self.nn):
            i = anc[c]
            self.quads.append((np.concatenate([self.ix[i], self.iu[i]]),
                               np.concatenate([inst.q[c], inst.r[c]]), self.itau[c], ("q", c)))
        for j in self.leaves:
            self.quads.append((self.ix[j], np.asarray(inst.qN[j], float), self.isv[j], ("qN", j)))
        self.m = len(self.g) + len(self.quads)

    # ------------------------------------------------------------------ start
    def _strict_y(self, i, Z):
        """A y with E'y = Z, F'y = 0 and its cone rows at least a positive
        margin (a small linear program: maximise the margin, at most 1)."""
        from scipy.optimize import linprog
        E, F, kp = self.E[i], self.Fr[i], self.kpos[i]
        ny = E.shape[0]
        A_eq = np.hstack([np.vstack([E.T, F.T]), np.zeros((E.shape[1] + F.shape[1], 1))])
        b_eq = np.concatenate([Z, np.zeros(F.shape[1])])
        A_ub = np.zeros((kp, ny + 1))
        for k in range(kp):
            A_ub[k, k] = -1.0                                   # t - y_k <= 0
            A_ub[k, -1] = 1.0
        c = np.zeros(ny + 1)
        c[-1] = -1.0
        res = linprog(c, A_ub=A_ub if kp else None, b_ub=np.zeros(kp) if kp else None, A_eq=A_eq, b_eq=b_eq,
                      bounds=[(None, None)] * ny + [(None, 1.0)], method="highs")
        if res.status != 0 or res.x[-1] <= 0.0:
            raise ValueError("no strictly feasible conic dual point for the start")
        return res.x[:ny]

    def feasible_start(self):
        """u = 0, x from the dynamics, tau and s with a margin, y strictly
        inside its cone with E'y = tau + s and F'y = 0, s^i above b'y."""
        inst, z = self.inst, np.zeros(self.n)
        x = np.zeros((self.nn, self.nx))
        x[0] = self.x0
        for c in range(1, self.nn):
            x[c] = inst.A[c] @ x[inst.anc[c]]
        for i in range(self.nn):
            z[self.ix[i]] = x[i]
        for c in range(1, self.nn):
            i = inst.anc[c]
            z[self.itau[c]] = x[i] @ (inst.q[c] * x[i]) + 1.0
        for j in self.leaves:
            z[self.isv[j]] = x[j] @ (inst.qN[j] * x[j]) + 1.0
        for t in range(int(self.stage.max()) - 1, -1, -1):
            for i in self.nonleaf:
                if self.stage[i] != t:
                    continue
                ch = self.ch[i]
                Z = np.array([z[self.itau[c]] + z[self.isv[c]] for c in ch])
                if self.risk is None:                           # y1 = 1, y3 above every Z (y2 > 0)
                    k = len(ch)
                    y3 = max(Z.max(), 0.0) + 1.0
                    y = np.concatenate([np.ones(k), inst.a_risk[i] + y3 - Z, [y3]])
                else:
                    y = self._strict_y(i, Z)
                z[self.iy[i]] = y
                z[self.isv[i]] = self.b[i] @ y + 1.0
        if np.min(self.slacks(z)) <= 0.0:
            raise ValueError("hand-built start is not strictly feasible (box too tight for u = 0)")
        return z

    # ------------------------------------------------------------------ barrier
    def slacks(self, z):
        lin = self.g - self.G @ z
        quad = np.array([z[j] - w @ (z[idx] ** 2) for idx, w, j, _ in self.quads])
        return np.concatenate([lin, quad])

    def _phi(self, z, t):
        s = self.slacks(z)
        if np.min(s) <= 0.0:
            return np.inf
        return t * z[self.isv[0]] - np.sum(np.log(s))

    def _grad_hess(self, z, t):
        n = self.n
        grad = np.zeros(n)
        grad[self.isv[0]] = t
        sl = self.g - self.G @ z
        grad += self.G.T @ (1.0 / sl)
        H = (self.G.T * (1.0 / sl ** 2)) @ self.G
        for idx, w, j, _ in self.quads:
            sq = z[j] - w @ (z[idx] ** 2)                # -g > 0
            dg = np.zeros(n)
            dg[idx] = 2.0 * w * z[idx]
            dg[j] = -1.0
            grad += dg / sq
            H += np.outer(dg, dg) / sq ** 2
            H[idx, idx] += 2.0 * w / sq
        return grad, H

    def _reduced_solve(self, Hw, b):
        """Hw x = b for the symmetric positive (semi)definite reduced Hessian,
        by an eigendecomposition (directions of zero curvature dropped)."""
        lam, V = np.linalg.eigh(Hw)
        keep = lam > lam.max() * 1e-15
        return V[:, keep] @ ((V[:, keep].T @ b) / lam[keep])

    def solve(self, gap=1e-10, mu=8.0, t0=1.0, newton_tol=1e-10, max_newton=100):
        """Barrier method in the null space of the equality constraints:
        z = zp + Z w with F zp = h and Z an orthonormal basis of ker F, so
        every iterate satisfies the equalities exactly (up to rounding of
        zp + Z w) and each Newton step is unconstrained in w."""
        import scipy.linalg
        self.Z = scipy.linalg.null_space(self.F)
        self.Fpinv = np.linalg.pinv(self.F)
        z = self.feasible_start()
        zp = self.Fpinv @ self.h
        w = self.Z.T @ (z - zp)
        z = zp + self.Z @ w
        if np.min(self.slacks(z)) <= 0.0:
            raise ValueError("start lost strict feasibility on the null-space projection")
        t = t0
        Z = self.Z
        while True:
            for _ in range(max_newton):
                grad, H = self._grad_hess(z, t)
                gw = Z.T @ grad
                Hw = Z.T @ H @ Z
                dw = -self._reduced_solve(Hw, gw)
                lam2 = -gw @ dw                             # Newton decrement squared
                if lam2 / 2.0 <= newton_tol:
                    break
                dz = Z @ dw
                step, f0 = 1.0, self._phi(z, t)
                while True:
                    f1 = self._phi(z + step * dz, t)
                    if f1 <= f0 - 0.25 * step * lam2:
                        break
                    # phi's rounding at large t can hide a true decrease
                    if np.isfinite(f1) and step * lam2 < 1e-11 * max(1.0, abs(f0)):
                        break
                    step *= 0.5
                    if step < 1e-12:
                        break
                if step < 1e-12:
                    break
                w = w + step * dw
                z = zp + Z @ w
            if self.m / t <= gap * max(1.0, abs(z[self.isv[0]])):
                break
            t *= mu
        self.z, self.t = z, t
        return z

    # ------------------------------------------------------------------ results
    @property
    def V(self):
        return float(self.z[self.isv[0]])

    @property
    def u0(self):
        return self.z[self.iu[0]].copy()
