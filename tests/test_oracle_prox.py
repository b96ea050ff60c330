"""Pins of Alg. 1 / Alg. 2 (projection on S1) against dense affine projection."""
import numpy as np
import pytest

import oracle as O
import spock_gen as G
from tests.checks.dense import s1_dense_projection

CASES = [([2, 2, 2], 2, 1), ([3, 1, 1], 3, 2), ([2, 3, 1], 4, 2), ([1, 1, 1, 1], 2, 3),
         ([4], 3, 1), ([2, 2], 5, 5)]


@pytest.mark.parametrize("k", range(len(CASES)))
def test_s1_projection_matches_dense(k):
    br, nx, nu = CASES[k]
    inst = G.make_random_small(200 + k, br, nx, nu)
    lay = O.Layout(inst)
    fac = O.factor_s1(lay, inst)
    rng = np.random.default_rng(k)
    xbar = rng.standard_normal((lay.num_nodes, nx))
    ubar = rng.standard_normal((lay.num_nodes, nu))
    x0 = rng.standard_normal(nx)
    x, u = O.proj_S1(lay, inst, fac, xbar, ubar, x0)
    xd, ud = s1_dense_projection(inst, xbar, ubar, x0)
    scale = max(1.0, np.max(np.abs(xd)))
    assert np.max(np.abs(x - xd)) <= 1e-11 * scale
    assert np.max(np.abs(u[lay.nonleaf] - ud[lay.nonleaf])) <= 1e-11 * scale
    # dynamics hold and the root is pinned
    assert np.max(np.abs(x[0] - x0)) == 0.0
    for c in range(1, lay.num_nodes):
        i = lay.anc[c]
        assert np.max(np.abs(x[c] - inst.A[c] @ x[i] - inst.B[c] @ u[i])) <= 1e-12 * scale
    # idempotent
    x2, u2 = O.proj_S1(lay, inst, fac, x, u, x0)
    assert np.max(np.abs(x2 - x)) <= 1e-11 * scale


def test_factor_matches_definitions():
    # R~ = I + sum B'PB, K = -R~^{-1} sum B'PA, P = I + K'K + sum Abar'P Abar (Alg. 1),
    # checked through the cost-to-go identity of the projection problem:
    # min over the subtree of 1/2 sum ||x-0||^2 + ||u||^2 from x at node i = 1/2 x'P^i x
    inst = G.make_random_small(300, [2, 1, 2], 3, 2)
    lay = O.Layout(inst)
    fac = O.factor_s1(lay, inst)
    rng = np.random.default_rng(1)
    x0 = rng.standard_normal(3)
    x, u = O.proj_S1(lay, inst, fac, np.zeros((lay.num_nodes, 3)), np.zeros((lay.num_nodes, 2)), x0)
    cost = 0.5 * (np.sum(x ** 2) + np.sum(u[lay.nonleaf] ** 2))
    assert abs(cost - 0.5 * x0 @ fac["P"][0] @ x0) <= 1e-12 * cost
