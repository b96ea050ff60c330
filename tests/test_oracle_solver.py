"""Whole-solver pins of the oracle: closed forms, brute force, invariants."""
import numpy as np
import pytest

import oracle as O
import spock_gen as G
from tests.checks.bruteforce import NestedDP
from tests.checks.dense import tree_lqr, s1_dense_projection, nullspace_projection

TIGHT = O.Settings(eps_abs=1e-11, eps_rel=1e-11, max_iters=200000)


def _unbox(inst):
    inst.xmin[:] = -1e6
    inst.xmax[:] = 1e6
    inst.umin[:] = -1e6
    inst.umax[:] = 1e6
    return inst


@pytest.mark.parametrize("seed,br,nx,nu", [(1, [2, 2], 2, 1), (2, [3, 1, 1], 3, 2),
                                          (3, [2, 2, 1], 2, 2)])
def test_risk_neutral_matches_tree_lqr(seed, br, nx, nu):
    # AV@R_1 is the expectation (section 4.2), so with inactive boxes the
    # nested problem is a tree LQR with a closed-form Riccati solution.
    inst = _unbox(G.make_random_small(seed, br, nx, nu, a=1.0))
    Vlqr, u0lqr = tree_lqr(inst, inst.x0)
    P = O.Problem(inst)
    res = O.spock_solve(P, inst.x0, TIGHT)
    assert res.status == "converged"
    assert abs(res.V_s0 - Vlqr) <= 1e-8 * max(1.0, Vlqr)
    assert abs(res.V_nested - Vlqr) <= 1e-8 * max(1.0, Vlqr)
    assert np.max(np.abs(res.u0 - u0lqr)) <= 1e-6 * max(1.0, np.max(np.abs(u0lqr)))


def test_config1_matches_bruteforce_dp():
    # config 1 (a = 0.5, n_u = 1, input box active somewhere) against nested DP
    inst = G.make_config(1)
    dp = NestedDP(inst)
    Vdp, u0dp = dp.solve()
    P = O.Problem(inst)
    res = O.spock_solve(P, inst.x0, TIGHT)
    assert res.status == "converged"
    assert np.max(np.abs(res.x)) < 5.0 - 1e-3          # state box inactive at the optimum
    assert abs(res.V_nested - Vdp) <= 1e-8 * max(1.0, abs(Vdp))
    assert abs(res.V_s0 - Vdp) <= 1e-8 * max(1.0, abs(Vdp))
    assert abs(res.u0[0] - u0dp) <= 1e-5


@pytest.mark.parametrize("seed,a", [(21, 0.0), (22, 0.4), (23, 0.9)])
def test_random_single_input_matches_bruteforce(seed, a):
    inst = G.make_random_small(seed, [2, 2], 2, 1, a=a, box=50.0, ubox=0.6)
    dp = NestedDP(inst)
    Vdp, u0dp = dp.solve()
    res = O.spock_solve(O.Problem(inst), inst.x0, TIGHT)
    assert res.status == "converged"
    assert abs(res.V_nested - Vdp) <= 1e-8 * max(1.0, abs(Vdp))
    assert abs(res.V_s0 - Vdp) <= 1e-7 * max(1.0, abs(Vdp))


def test_zero_direction_spock_is_vanilla_cp():
    # with d = 0, c0 = c1 = 0 and lambda = 1 every step is K2 with rho = omega^2,
    # i.e. v - r = T(v): SPOCK reproduces CP iterate for iterate.
    inst = G.make_config(1)
    P = O.Problem(inst)
    s = O.Settings(eps_abs=1e-6, eps_rel=1e-6, c0=0.0, c1=0.0, lam=1.0, direction="zero")
    a = O.spock_solve(P, inst.x0, s, keep_history=True)
    b = O.cp_solve(P, inst.x0, O.Settings(eps_abs=1e-6, eps_rel=1e-6), keep_history=True)
    assert a.counts["K2"] == a.iters and a.counts["K0"] == 0
    assert a.iters == b.iters
    assert np.max(np.abs(a.v - b.v)) <= 1e-12 * max(1.0, np.max(np.abs(b.v)))


def test_certificates_every_iterate():
    # section 3: xi_p in df(z+) + L* eta+, L z+ + xi_d in dg*(eta+), with
    # (z+, eta+) = T(z, eta) (holds for the corrected prox of g*)
    inst = G.make_random_small(31, [2, 2, 1], 2, 2)
    P = O.Problem(inst)
    lay = P.lay
    fac = P.fac
    rng = np.random.default_rng(0)
    v = rng.standard_normal(lay.n_v)
    for _ in range(5):
        Tv = O.T_apply(P, v, inst.x0)
        st = O.residual_stats(P, v - Tv)
        zp, ep = lay.split(Tv)
        # dual: w = L z+ + xi_d lies in S3 and eta+ is in its normal cone
        w = O.L_apply(lay, inst, zp) + st["xi_d"]
        assert np.max(np.abs(O.proj_S3(lay, inst, w) - w)) <= 1e-10 * max(1, np.max(np.abs(w)))
        for _ in range(20):
            s = O.proj_S3(lay, inst, w + rng.standard_normal(lay.n_eta))
            assert ep @ (s - w) <= 1e-9
        # primal: g = xi_p - L* eta+ is a subgradient of f at z+:
        # g[s0] = 1, g on z1 orthogonal to the dynamics directions, g on z2 orthogonal to S2
        g = st["xi_p"] - O.Lt_apply(lay, inst, ep)
        assert abs(g[0] - 1.0) <= 1e-10
        gx = np.stack([lay.x_of(g, i) for i in range(lay.num_nodes)])
        gu = np.zeros((lay.num_nodes, lay.nu))
        for i in lay.nonleaf:
            gu[i] = lay.u_of(g, i)
        px, pu = s1_dense_projection(inst, gx, gu, np.zeros(lay.nx))   # projection on dir S1
        assert np.max(np.abs(px)) + np.max(np.abs(pu[lay.nonleaf])) <= 1e-9
        for i in lay.nonleaf:
            idx = O.prox.s2_indices(lay, i)
            assert np.max(np.abs(nullspace_projection(O.prox.s2_matrix(lay, inst, i), g[idx]))) <= 1e-9
        v = Tv + 0.1 * rng.standard_normal(lay.n_v)


def test_T_firmly_nonexpansive_in_M_metric():
    inst = G.make_random_small(41, [3, 1], 3, 2)
    P = O.Problem(inst)
    rng = np.random.default_rng(2)
    for _ in range(30):
        v = 3 * rng.standard_normal(P.lay.n_v)
        w = 3 * rng.standard_normal(P.lay.n_v)
        dT = O.T_apply(P, v, inst.x0) - O.T_apply(P, w, inst.x0)
        lhs = dT @ O.M_apply(P, dT)
        rhs = dT @ O.M_apply(P, v - w)
        assert lhs <= rhs + 1e-10 * abs(rhs)
        assert (v - w) @ O.M_apply(P, v - w) > 0          # M positive definite (alpha ||L|| < 1)


def test_gap_bound_and_s0_multiplier():
    # at convergence: s0 of T(v) approaches V* and the s0-row multiplier -> -1
    inst = G.make_config(1)
    P = O.Problem(inst)
    ref = O.spock_solve(P, inst.x0, TIGHT)
    loose = O.spock_solve(P, inst.x0, O.Settings(eps_abs=1e-4, eps_rel=1e-4))
    zs, es = P.lay.split(ref.v)
    zl, el = P.lay.split(loose.v)
    r = loose.v - O.T_apply(P, loose.v, inst.x0)
    st = O.residual_stats(P, r)
    Tl = O.T_apply(P, loose.v, inst.x0)
    z1, e1 = P.lay.split(Tl)
    # gap bound derived from the certificates of section 3
    bound = np.max(np.abs(st["xi_p"])) * np.sum(np.abs(zs - z1)) + np.max(np.abs(st["xi_d"])) * np.sum(np.abs(e1))
    assert abs(z1[0] - ref.V_s0) <= bound + 1e-9
    assert abs(es[P.lay.e1s[0]] + 1.0) <= 1e-8


def test_anderson_buffer_rules():
    rng = np.random.default_rng(4)
    n = 40
    aa = O.AndersonBuffer(3)
    r = rng.standard_normal(n)
    assert np.array_equal(aa.direction(r), -r)                       # empty buffer
    dV = [rng.standard_normal(n) for _ in range(3)]
    dR = [rng.standard_normal(n) for _ in range(3)]
    for a, b in zip(dV, dR):
        aa.push(a, b)
    MR, MP = np.column_stack(dR), np.column_stack(dV)
    gam = np.linalg.solve(MR.T @ MR, MR.T @ r)                       # normal equations
    assert np.max(np.abs(aa.direction(r) - (-r - (MP - MR) @ gam))) <= 1e-12
    # exact recovery: r in span(M^R) => gamma reproduces r exactly
    g0 = np.array([0.3, -1.2, 2.0])
    r2 = MR @ g0
    assert np.max(np.abs(aa.direction(r2) - (-r2 - (MP - MR) @ g0))) <= 1e-12
    # memory m keeps the newest m columns
    aa.push(rng.standard_normal(n), rng.standard_normal(n))
    assert len(aa.dR) == 3 and aa.dR[0] is dR[1]
    # rank rule drops the oldest of dependent columns
    bb = O.AndersonBuffer(3)
    bb.push(dV[0], dR[0])
    bb.push(dV[1], 2.0 * dR[0])
    bb.direction(r)
    assert len(bb.dR) == 1 and bb.dR[0] is not dR[0]


def _dense_M(P):
    """M = [I, -alpha L*; -alpha L, I] (section 3) from the dense L."""
    Ld = O.dense_L(P.lay, P.inst)
    nz, ne = P.lay.n_z, P.lay.n_eta
    M = np.eye(nz + ne)
    M[:nz, nz:] = -P.alpha * Ld.T
    M[nz:, :nz] = -P.alpha * Ld
    return M


def test_M_apply_and_omega_match_dense_definition():
    # omega of the residual statistics is the M-norm of r: r'Mr with M built
    # densely from its definition (the column-by-column L is pinned by the
    # adjoint identity); a sign error in the cross term would show here
    inst = G.make_random_small(52, [3, 1], 3, 2)
    P = O.Problem(inst)
    M = _dense_M(P)
    rng = np.random.default_rng(9)
    for _ in range(10):
        r = rng.standard_normal(P.lay.n_v)
        assert np.max(np.abs(O.M_apply(P, r) - M @ r)) <= 1e-13 * max(1, np.max(np.abs(M @ r)))
        om = O.residual_stats(P, r)["omega"]
        assert abs(om ** 2 - r @ M @ r) <= 1e-12 * (r @ r)


def _K2_trace(inst, k2_factor=1.0, iters=400):
    P = O.Problem(inst)
    trace = []
    s = O.Settings(eps_abs=1e-12, eps_rel=1e-12, max_iters=iters, k2_factor=k2_factor)
    O.spock_solve(P, inst.x0, s, trace=trace)
    return P, trace


def test_K2_steps_project_on_a_halfspace_containing_the_fixed_points():
    # SPOCK's own K2 steps (Anderson directions, lambda = 1): for a firmly
    # nonexpansive T the halfspace {w : <r~, v~ - w>_M >= ||r~||_M^2}
    # contains Fix T, and the step lands on its boundary; hence Fejer
    # monotonicity in the M-norm towards any fixed point. This decides the
    # reading of the K2 factor (1, not the printed 2 alpha).
    inst = G.make_config(1)
    P, trace = _K2_trace(inst)
    assert len(trace) >= 20
    M = _dense_M(P)
    vstar = O.spock_solve(P, inst.x0, TIGHT).v
    for v, vt, Tvt, vn in trace:
        rt = vt - Tvt
        nr = rt @ M @ rt
        assert abs(rt @ M @ (vt - vn) - nr) <= 1e-9 * nr
        assert (vn - vstar) @ M @ (vn - vstar) <= (v - vstar) @ M @ (v - vstar) * (1 + 1e-12) + 1e-20
        # Fix T lies in the halfspace
        assert rt @ M @ (vt - vstar) >= nr * (1 - 1e-9) - 1e-14


def test_K2_printed_factor_leaves_the_halfspace_boundary():
    # the printed factor 2 alpha planted in the oracle: its K2 step does not
    # land on the boundary of that halfspace (alpha != 1/2 here)
    inst = G.make_config(1)
    P, _ = _K2_trace(inst, iters=1)
    assert abs(2 * P.alpha - 1.0) > 0.05
    P, trace = _K2_trace(inst, k2_factor=2 * P.alpha)
    assert trace
    M = _dense_M(P)
    v, vt, Tvt, vn = trace[0]
    rt = vt - Tvt
    nr = rt @ M @ rt
    assert abs(rt @ M @ (vt - vn) - nr) > 1e-6 * nr


def test_cp_and_spock_agree():
    inst = G.make_config(1)
    P = O.Problem(inst)
    s = O.Settings(eps_abs=1e-9, eps_rel=1e-9)
    a = O.cp_solve(P, inst.x0, s)
    b = O.spock_solve(P, inst.x0, s)
    assert abs(a.V_nested - b.V_nested) <= 1e-6
    assert b.t_evals < a.t_evals
