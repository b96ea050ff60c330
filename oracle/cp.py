"""The Chambolle-Pock operator T and the plain (vanilla) CP method (section 3).

T(z, eta) = (prox_{alpha f}(z - alpha L* eta),
             prox_{alpha g*}(eta + alpha L (2 z+ - z)))       (eq. chambolle-pock-operator)
R = id - T, r = (r_z, r_eta);
xi_p = r_z / alpha - L* r_eta, xi_d = r_eta / alpha - L r_z,
xi = max(||xi_p||_inf, ||xi_d||_inf), stop when xi <= max(eps_abs, eps_rel xi_0);
omega = (r_z'(r_z - alpha L* r_eta) + r_eta'(r_eta - alpha L r_z))^{1/2}, the
M-norm of r (Alg. 3).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .layout import Layout
from .operators import L_apply, Lt_apply
from .prox import prox_f, prox_gstar
from .risk import nested_cost


@dataclass
class Settings:
    eps_abs: float = 1e-4
    eps_rel: float = 1e-4
    max_iters: int = 20000
    # SuperMann / Anderson parameters (our defaults; the paper cites them)
    m: int = 3
    c0: float = 0.99
    c1: float = 0.99
    c2: float = 0.99
    beta: float = 0.5
    sigma: float = 0.1
    lam: float = 1.0
    max_ls: int = 20
    rank_tol: float = 1e-6
    direction: str = "anderson"      # "anderson" | "zero" (test switch)
    # factor of <r~, v~ - v>_M in the K2 step: 1 for a firmly nonexpansive T
    # (the reading taken); the printed 2 alpha only as a test switch
    k2_factor: float = 1.0


@dataclass
class SolveResult:
    v: np.ndarray                  # T(v^k) at termination
    status: str                    # "converged" | "maxiter"
    iters: int
    t_evals: int
    xi0: float
    xi: float
    V_s0: float
    V_nested: float
    u0: np.ndarray
    x: np.ndarray
    u: np.ndarray
    counts: dict = field(default_factory=dict)
    history: list = field(default_factory=list)


class Problem:
    """Bundles an instance with its layout, Alg. 1 factors and step size."""

    def __init__(self, inst, alpha: float | None = None, fac=None):
        from .operators import norm_L
        from .prox import factor_s1
        self.inst = inst
        self.lay = Layout(inst)
        self.fac = factor_s1(self.lay, inst) if fac is None else fac
        self.normL = norm_L(self.lay, inst)
        self.alpha = 0.99 / self.normL if alpha is None else float(alpha)


def T_apply(prob: "Problem", v: np.ndarray, x0: np.ndarray) -> np.ndarray:
    lay, inst, a = prob.lay, prob.inst, prob.alpha
    z, eta = lay.split(v)
    zp = prox_f(lay, inst, prob.fac, z - a * Lt_apply(lay, inst, eta), a, x0)
    ep = prox_gstar(lay, inst, eta + a * L_apply(lay, inst, 2.0 * zp - z), a)
    return np.concatenate([zp, ep])


def residual_stats(prob: "Problem", r: np.ndarray):
    """xi_p, xi_d, xi and omega of a residual r = v - T(v)."""
    lay, inst, a = prob.lay, prob.inst, prob.alpha
    rz, re = lay.split(r)
    Lrz = L_apply(lay, inst, rz)
    Ltre = Lt_apply(lay, inst, re)
    xi_p = rz / a - Ltre
    xi_d = re / a - Lrz
    xi = max(np.max(np.abs(xi_p), initial=0.0), np.max(np.abs(xi_d), initial=0.0))
    om2 = rz @ (rz - a * Ltre) + re @ (re - a * Lrz)
    return {"xi": float(xi), "omega": float(np.sqrt(max(om2, 0.0))),
            "xi_p": xi_p, "xi_d": xi_d}


def M_apply(prob: "Problem", d: np.ndarray) -> np.ndarray:
    """M d = (d_z - alpha L* d_eta, d_eta - alpha L d_z) (section 3)."""
    lay, inst, a = prob.lay, prob.inst, prob.alpha
    dz, de = lay.split(d)
    return np.concatenate([dz - a * Lt_apply(lay, inst, de), de - a * L_apply(lay, inst, dz)])


def finish(prob: "Problem", Tv: np.ndarray, status, iters, t_evals, xi0, xi, counts=None,
           history=None) -> SolveResult:
    lay = prob.lay
    z, _ = lay.split(Tv)
    x, u = lay.unpack_xu(z)
    return SolveResult(v=Tv, status=status, iters=iters, t_evals=t_evals, xi0=xi0, xi=xi,
                       V_s0=float(z[0]), V_nested=nested_cost(lay, prob.inst, x, u),
                       u0=u[0].copy(), x=x, u=u, counts=counts or {},
                       history=history or [])


def cp_solve(prob: "Problem", x0: np.ndarray, settings: Settings, v0=None,
             keep_history: bool = False) -> SolveResult:
    """Vanilla CP: v <- T(v) until the termination rule of section 3 holds."""
    lay = prob.lay
    v = np.zeros(lay.n_v) if v0 is None else np.array(v0, dtype=float)
    xi0 = None
    hist = []
    for k in range(settings.max_iters + 1):
        Tv = T_apply(prob, v, x0)
        st = residual_stats(prob, v - Tv)
        if xi0 is None:
            xi0 = st["xi"]
        if keep_history:
            hist.append(st["xi"])
        if st["xi"] <= max(settings.eps_abs, settings.eps_rel * xi0):
            return finish(prob, Tv, "converged", k, k + 1, xi0, st["xi"], history=hist)
        if k == settings.max_iters:
            return finish(prob, Tv, "maxiter", k, k + 1, xi0, st["xi"], history=hist)
        v = Tv
