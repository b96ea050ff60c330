"""Pins of the oracle with dense cost matrices (section 4.1: any Q, Q_N >= 0
and R > 0; the cost rows of eta carry their symmetric square roots): the
diagonal case written densely, an orthogonal change of coordinates that maps
a diagonal problem onto a dense one with the same value, and brute-force
nested DP on single-input trees with active input boxes."""
import numpy as np
import pytest

import oracle as O
import spock_gen as G
from tests.checks.bruteforce import NestedDP

TIGHT = O.Settings(eps_abs=1e-10, eps_rel=1e-10, max_iters=400000)


def _as_dense(inst):
    d = inst.copy()
    d.Qm = np.stack([np.diag(q) for q in inst.q])
    d.Rm = np.stack([np.diag(r) for r in inst.r])
    d.QNm = np.stack([np.diag(q) for q in inst.qN])
    return d


def _orthogonal(rng, n):
    q, r = np.linalg.qr(rng.standard_normal((n, n)))
    return q * np.sign(np.diag(r))


def test_diagonal_written_dense_is_the_diagonal_problem():
    inst = G.make_random_small(11, [3, 1, 2], 4, 3)
    dense = _as_dense(inst)
    P, Pd = O.Problem(inst), O.Problem(dense, alpha=O.Problem(inst).alpha)
    assert abs(P.normL - Pd.normL) <= 1e-12 * P.normL
    rng = np.random.default_rng(3)
    z, e = rng.standard_normal(P.lay.n_z), rng.standard_normal(P.lay.n_eta)
    assert np.max(np.abs(O.L_apply(P.lay, inst, z) - O.L_apply(Pd.lay, dense, z))) <= 1e-14
    assert np.max(np.abs(O.Lt_apply(P.lay, inst, e) - O.Lt_apply(Pd.lay, dense, e))) <= 1e-14
    v = rng.standard_normal(P.lay.n_v)
    assert np.max(np.abs(O.T_apply(P, v, inst.x0) - O.T_apply(Pd, v, inst.x0))) <= 1e-13


def test_dense_L_adjoint_identity():
    inst = G.dense_costs(G.make_random_small(12, [2, 3], 3, 2), 5)
    P = O.Problem(inst)
    rng = np.random.default_rng(4)
    z, e = rng.standard_normal(P.lay.n_z), rng.standard_normal(P.lay.n_eta)
    lhs = O.L_apply(P.lay, inst, z) @ e
    assert abs(lhs - z @ O.Lt_apply(P.lay, inst, e)) <= 1e-12 * max(1.0, abs(lhs))


@pytest.mark.parametrize("a", [0.3])
def test_rotation_of_a_diagonal_problem(a):
    # x' = U x, u' = W u with U, W orthogonal maps the diagonal problem onto
    # one with dense Q' = U Q U', R' = W R W' and the same value; u0' = W u0
    # (boxes inactive)
    inst = G.make_random_small(41, [2, 2, 1], 3, 2, a=a, box=50.0, ubox=50.0)
    rng = np.random.default_rng(9)
    U, W = _orthogonal(rng, inst.nx), _orthogonal(rng, inst.nu)
    rot = G.rotate_states_inputs(inst, U, W)
    st = O.Settings(eps_abs=1e-9, eps_rel=1e-9, max_iters=100000)
    r1 = O.spock_solve(O.Problem(inst), inst.x0, st)
    r2 = O.spock_solve(O.Problem(rot), rot.x0, st)
    assert r1.status == r2.status == "converged"
    # both values within the residual's reach of the same optimum
    assert abs(r1.V_s0 - r2.V_s0) <= 1e-7 * max(1.0, abs(r1.V_s0))
    assert abs(r1.V_nested - r2.V_nested) <= 1e-7 * max(1.0, abs(r1.V_nested))
    assert np.max(np.abs(W @ r1.u0 - r2.u0)) <= 1e-5 * max(1.0, np.max(np.abs(r1.u0)))


@pytest.mark.parametrize("seed,a", [(51, 0.0), (52, 0.4), (55, 0.8)])
def test_dense_costs_match_bruteforce_dp(seed, a):
    inst = G.dense_costs(G.make_random_small(seed, [2, 2], 2, 1, a=a, box=50.0, ubox=0.6), seed)
    Vdp, u0dp = NestedDP(inst).solve()
    res = O.spock_solve(O.Problem(inst), inst.x0, TIGHT)
    assert res.status == "converged"
    assert abs(res.V_nested - Vdp) <= 1e-8 * max(1.0, abs(Vdp))
    assert abs(res.V_s0 - Vdp) <= 1e-7 * max(1.0, abs(Vdp))
    assert abs(res.u0[0] - u0dp) <= 1e-5
