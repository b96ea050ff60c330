"""SPOCK: SuperMann with Chambolle-Pock and Anderson directions (section 6,
Alg. 3).

Readings taken where the printed algorithm is ambiguous:
  * the residual r^k at the current iterate is formed before the termination
    test and the Anderson step that need it (r^k is reused after a K1 step);
  * c^k of section 6 is that residual r^k = v^k - T(v^k), so the direction is
    d = -r - (M^P - M^R) gamma with gamma = argmin ||M^R gamma - r||;
  * the buffers hold m difference columns, fed by accepted iterates only, and
    the oldest column is dropped while sigma_min/sigma_max(M^R) < rank_tol;
  * in the K2 step rho = w~^2 - <r~, v~ - v>_M: the factor printed as 2 alpha
    is SuperMann's 2 x averagedness constant, which is 1 for a firmly
    nonexpansive T (the halfspace it projects on then contains Fix T);
  * backtracking stops after max_ls halvings with the plain KM step v - lam r;
  * w~ = 0 means v~ is a fixed point and is accepted as K1;
  * the returned point is T(v^k), for which the certificates of section 3 hold.
"""
from __future__ import annotations

import numpy as np

from .cp import (Problem, Settings, SolveResult, T_apply, residual_stats, M_apply,
                 finish)


class AndersonBuffer:
    """Difference buffers M^P (iterates) and M^R (residuals) of section 6.2."""

    def __init__(self, m: int, rank_tol: float = 1e-6):
        self.m = m
        self.rank_tol = rank_tol
        self.dV: list = []
        self.dR: list = []

    def push(self, dv, dr):
        if self.m <= 0:
            return
        self.dV.append(dv)
        self.dR.append(dr)
        if len(self.dV) > self.m:
            self.dV.pop(0)
            self.dR.pop(0)

    def _prune(self):
        while self.dR:
            s = np.linalg.svd(np.column_stack(self.dR), compute_uv=False)
            if s[0] > 0.0 and s[-1] / s[0] >= self.rank_tol:
                return
            self.dV.pop(0)
            self.dR.pop(0)

    def direction(self, r: np.ndarray) -> np.ndarray:
        self._prune()
        if not self.dR:
            return -r
        MR = np.column_stack(self.dR)
        MP = np.column_stack(self.dV)
        gamma = np.linalg.lstsq(MR, r, rcond=None)[0]
        return -r - (MP - MR) @ gamma


def spock_solve(prob: Problem, x0: np.ndarray, settings: Settings, v0=None,
                keep_history: bool = False, trace: list | None = None) -> SolveResult:
    """Alg. 3. With a list in trace, every K2 step appends
    (v, v~, T(v~), v_new): the iterate, the trial point, its image and the
    step's result (test instrumentation only)."""
    lay = prob.lay
    s = settings
    v = np.zeros(lay.n_v) if v0 is None else np.array(v0, dtype=float)
    Tv = T_apply(prob, v, x0)
    t_evals = 1
    r = v - Tv
    st = residual_stats(prob, r)
    xi0 = st["xi"]
    zeta = st["omega"]
    omega_safe = st["omega"]
    aa = AndersonBuffer(s.m, s.rank_tol)
    prev = None
    counts = {"K0": 0, "K1": 0, "K2": 0, "KM": 0, "backtracks": 0}
    hist = []
    k = 0
    while True:
        # r, Tv and st belong to the current iterate v
        if keep_history:
            hist.append((t_evals, st["xi"]))
        if st["xi"] <= max(s.eps_abs, s.eps_rel * xi0):
            return finish(prob, Tv, "converged", k, t_evals, xi0, st["xi"], counts, hist)
        if k >= s.max_iters:
            return finish(prob, Tv, "maxiter", k, t_evals, xi0, st["xi"], counts, hist)
        if prev is not None:
            aa.push(v - prev[0], r - prev[1])
        if s.direction == "zero":
            d = np.zeros_like(v)
        else:
            d = aa.direction(r)
        omega = st["omega"]
        prev = (v, r)
        if omega <= s.c0 * zeta:                                   # K0
            v = v + d
            zeta = omega
            counts["K0"] += 1
            Tv = T_apply(prob, v, x0)
            t_evals += 1
            r = v - Tv
            st = residual_stats(prob, r)
            k += 1
            continue
        Md = M_apply(prob, d)
        tau = 1.0
        accepted = False
        for _ in range(s.max_ls):
            vt = v + tau * d
            Tvt = T_apply(prob, vt, x0)
            t_evals += 1
            rt = vt - Tvt
            stt = residual_stats(prob, rt)
            om_t = stt["omega"]
            if om_t == 0.0 or (omega <= omega_safe and om_t <= s.c1 * omega):   # K1
                v, Tv, r, st = vt, Tvt, rt, stt
                omega_safe = om_t + s.c2 ** k
                counts["K1"] += 1
                accepted = True
                break
            rho = om_t ** 2 - s.k2_factor * tau * (rt @ Md)
            if rho >= s.sigma * om_t * omega:                              # K2
                v_new = v - s.lam * rho / om_t ** 2 * rt
                if trace is not None:
                    trace.append((v, vt, Tvt, v_new))
                v = v_new
                counts["K2"] += 1
                Tv = T_apply(prob, v, x0)
                t_evals += 1
                r = v - Tv
                st = residual_stats(prob, r)
                accepted = True
                break
            tau *= s.beta
            counts["backtracks"] += 1
        if not accepted:                                                   # KM fallback
            v = v - s.lam * r
            counts["KM"] += 1
            Tv = T_apply(prob, v, x0)
            t_evals += 1
            r = v - Tv
            st = residual_stats(prob, r)
        k += 1
