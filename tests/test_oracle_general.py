"""Pins of the oracle on general problems: conic risk measures (E, F, b, K)
with nu != 0 (section 4.3) and polyhedral constraints Gamma x + Gamma u in C
(section 4.1)."""
import numpy as np
import pytest
import scipy.linalg

import oracle as O
import spock_gen as G
from tests.checks.bruteforce import NestedDP
from tests.checks.dense import cut_through
from tests.checks.kkt import EpigraphIPM

TIGHT = O.Settings(eps_abs=1e-12, eps_rel=1e-12, max_iters=900000)


def test_avar_and_boxes_written_generally_reproduce_the_special_form():
    # AV@R as (E, F, b, K) and the boxes as Gamma = I give the same layout
    # and the same operators, element by element
    inst = G.make_random_small(11, [3, 1, 2], 4, 3)
    gen = inst.copy()
    gen.risk = G.avar_as_conic(inst)
    gen.cons = G.boxes_as_constraints(inst)
    P, Pg = O.Problem(inst), O.Problem(gen)
    assert (P.lay.n_z, P.lay.n_eta) == (Pg.lay.n_z, Pg.lay.n_eta)
    assert abs(P.normL - Pg.normL) <= 1e-13 * P.normL
    rng = np.random.default_rng(1)
    v = rng.standard_normal(P.lay.n_v)
    z, e = P.lay.split(v)
    assert np.max(np.abs(O.L_apply(P.lay, inst, z) - O.L_apply(Pg.lay, gen, z))) <= 1e-14
    assert np.max(np.abs(O.Lt_apply(P.lay, inst, e) - O.Lt_apply(Pg.lay, gen, e))) <= 1e-14
    assert np.max(np.abs(O.prox_gstar(P.lay, inst, e, P.alpha) - O.prox_gstar(Pg.lay, gen, e, P.alpha))) <= 1e-14
    Pg.alpha = P.alpha
    assert np.max(np.abs(O.T_apply(P, v, inst.x0) - O.T_apply(Pg, v, inst.x0))) <= 1e-12


def _general(seed=82, br=(3, 1), nx=3, nu=2, nc=4, ncN=2):
    return G.make_general_small(seed, list(br), nx, nu, nc=nc, ncN=ncN)


def test_general_L_adjoint_identity():
    inst = _general()
    P = O.Problem(inst)
    rng = np.random.default_rng(2)
    for _ in range(5):
        z = rng.standard_normal(P.lay.n_z)
        e = rng.standard_normal(P.lay.n_eta)
        lhs = e @ O.L_apply(P.lay, inst, z)
        rhs = O.Lt_apply(P.lay, inst, e) @ z
        assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))


def test_general_S2_projection_is_nullspace_projection():
    # S2 of a risk with nu != 0: kernel of [E' -I -I; F' 0 0]
    inst = _general()
    P = O.Problem(inst)
    rng = np.random.default_rng(3)
    for i in P.lay.nonleaf:
        Gm = O.prox.s2_matrix(P.lay, inst, i)
        w = rng.standard_normal(Gm.shape[1])
        Zb = scipy.linalg.null_space(Gm)
        assert np.max(np.abs(O.proj_S2_block(Gm, w) - Zb @ (Zb.T @ w))) <= 1e-13


def test_general_prox_gstar_optimality():
    # p = prox_{alpha g*}(w): (w - p)/alpha lies in S3 and p is in its normal
    # cone there (Moreau), for the general cones and constraint rows
    inst = _general()
    P = O.Problem(inst)
    rng = np.random.default_rng(4)
    a = P.alpha
    for _ in range(5):
        w = 3 * rng.standard_normal(P.lay.n_eta)
        p = O.prox_gstar(P.lay, inst, w, a)
        q = (w - p) / a
        assert np.max(np.abs(O.proj_S3(P.lay, inst, q) - q)) <= 1e-12
        for _ in range(20):
            s = O.proj_S3(P.lay, inst, q + 2 * rng.standard_normal(P.lay.n_eta))
            assert p @ (s - q) <= 1e-10


def test_mixture_risk_value_has_its_closed_form():
    # the conic evaluation (an LP) of (1 - kappa) E^p[Z] + kappa max Z
    inst = _general()
    lay = O.Layout(inst)
    rng = np.random.default_rng(5)
    for i in lay.nonleaf:
        ch = lay.children[i]
        Z = rng.standard_normal(len(ch)) * 3
        want = 0.6 * lay.p[ch] @ Z + 0.4 * Z.max()
        got = O.risk.node_risk(lay, inst, i, Z)
        assert abs(got - want) <= 1e-9 * max(1.0, abs(want))


@pytest.mark.parametrize("seed,kappa", [(91, 0.4), (92, 0.8)])
def test_mixture_risk_solution_matches_bruteforce_dp(seed, kappa):
    # single input, boxes: nested dynamic programming with the closed-form
    # risk (1 - kappa) E^p[Z] + kappa max Z
    inst = G.make_random_small(seed, [2, 2], 2, 1, box=50.0, ubox=0.6)
    inst.risk = G.mixture_risk(inst, kappa)
    ch = [[] for _ in range(inst.num_nodes)]
    for c in range(1, inst.num_nodes):
        ch[inst.anc[c]].append(c)

    def risk(i, Z):
        p = inst.prob[ch[i]] / inst.prob[i]
        return (1 - kappa) * float(p @ np.asarray(Z)) + kappa * max(Z)
    Vdp, u0dp = NestedDP(inst, risk=risk).solve()
    res = O.spock_solve(O.Problem(inst), inst.x0, TIGHT)
    assert res.status == "converged"
    assert abs(res.V_nested - Vdp) <= 1e-8 * max(1.0, abs(Vdp))
    assert abs(res.V_s0 - Vdp) <= 1e-7 * max(1.0, abs(Vdp))
    assert abs(res.u0[0] - u0dp) <= 1e-5


def active_general(seed, br, nx, nu, nc):
    """A general instance whose constraint rows cut through the solution of
    the same instance with loose bounds (so some rows are active)."""
    loose = G.make_general_small(seed, br, nx, nu, nc=nc, ncN=2)
    res = O.spock_solve(O.Problem(loose), loose.x0, O.Settings(eps_abs=1e-8, eps_rel=1e-8, max_iters=900000))
    return cut_through(loose, res.x, res.u)


@pytest.mark.parametrize("seed,br,nx,nu,nc", [(81, [2, 2], 2, 1, 3), (82, [3, 1], 3, 2, 4),
                                              (84, [2, 2, 1], 2, 2, 5)])
def test_polyhedral_constraints_match_dense_ipm(seed, br, nx, nu, nc):
    # general constraint rows and the mixture risk against the dense
    # interior-point solve of the epigraph program
    inst = active_general(seed, br, nx, nu, nc)
    ipm = EpigraphIPM(inst)
    ipm.solve()
    res = O.spock_solve(O.Problem(inst), inst.x0, TIGHT)
    assert res.status == "converged"
    assert abs(res.V_nested - ipm.V) <= 1e-8 * max(1.0, abs(ipm.V))
    assert np.max(np.abs(res.u0 - ipm.u0)) <= 1e-7
    # a constraint row is active somewhere (the constraints matter)
    lay = O.Layout(inst)
    act = 0
    for i in lay.nonleaf:
        Gx, Gu, lo, hi = lay.gamma(inst, i)
        r = Gx @ res.x[i] + Gu @ res.u[i]
        act += np.sum(np.minimum(r - lo, hi - r) < 1e-6)
    assert act >= 1
