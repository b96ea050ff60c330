"""Pins of the oracle's L, L*, ||L||, S2 and S3 against the mathematics."""
import numpy as np
import pytest

import oracle as O
import spock_gen as G
from tests.checks.dense import feasible_conic_point, nullspace_projection, tree_lists

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")

SHAPES = [([2, 2, 2], 2, 1), ([3, 1], 3, 2), ([2, 3, 1, 1], 2, 2), ([1, 1], 1, 1),
          ([4, 2], 3, 3), ([2], 4, 1)]


def _inst(k, br, nx, nu, **kw):
    return G.make_random_small(100 + k, br, nx, nu, **kw)


@pytest.mark.parametrize("k", range(len(SHAPES)))
def test_adjoint_identity(k):
    br, nx, nu = SHAPES[k]
    inst = _inst(k, br, nx, nu)
    lay = O.Layout(inst)
    rng = np.random.default_rng(k)
    for _ in range(3):
        z = rng.standard_normal(lay.n_z)
        e = rng.standard_normal(lay.n_eta)
        lhs = e @ O.L_apply(lay, inst, z)
        rhs = z @ O.Lt_apply(lay, inst, e)
        assert abs(lhs - rhs) <= 1e-13 * max(1.0, abs(lhs))


def test_sizes_match_counting_formula():
    # n_z = 1 + |nodes| nx + |nonleaf| nu + 4(|nodes|-1) + |nonleaf|
    # n_eta = 2(|nodes|-1) + 2|nonleaf| + |nonleaf|(nx+nu) + (|nodes|-1)(nx+nu+2) + |leaves|(2nx+2)
    for k, (br, nx, nu) in enumerate(SHAPES):
        lay = O.Layout(_inst(k, br, nx, nu))
        nn, nl, lv = lay.num_nodes, len(lay.nonleaf), len(lay.leaves)
        assert lay.n_z == 1 + nn * nx + nl * nu + 4 * (nn - 1) + nl
        assert lay.n_eta == 2 * (nn - 1) + 2 * nl + nl * (nx + nu) + (nn - 1) * (nx + nu + 2) + lv * (2 * nx + 2)
    assert O.Layout(G.make_config(1)).n_v == 282


@pytest.mark.parametrize("k", range(len(SHAPES)))
def test_norm_blocks_vs_full_spectral_norm(k):
    br, nx, nu = SHAPES[k]
    inst = _inst(k, br, nx, nu)
    lay = O.Layout(inst)
    M = O.dense_L(lay, inst)
    full = np.linalg.norm(M, 2)
    # power iteration on L'L as a second, independent estimate
    rng = np.random.default_rng(0)
    v = rng.standard_normal(lay.n_z)
    for _ in range(3000):
        v = M.T @ (M @ v)
        v /= np.linalg.norm(v)
    pw = np.sqrt(v @ (M.T @ (M @ v)))
    nb = O.norm_L(lay, inst)
    assert abs(nb - full) <= 1e-12 * full
    assert abs(pw - full) <= 1e-6 * full


def test_norm_independent_of_horizon():
    # identical node data on horizons 2 and 6 (block-diagonal remark, section 5.2)
    vals = []
    for N in (2, 6):
        inst = G.make_random_small(7, [2] + [1] * (N - 1), 3, 2, q_kind="I", prob_kind="uniform")
        inst.r[:] = 0.3
        inst.qN[:] = 1.5
        vals.append(O.norm_L(O.Layout(inst), inst))
    assert abs(vals[0] - vals[1]) <= 1e-14 * vals[0]


@pytest.mark.parametrize("k", range(len(SHAPES)))
def test_s2_projection_vs_nullspace(k):
    br, nx, nu = SHAPES[k]
    inst = _inst(k, br, nx, nu)
    lay = O.Layout(inst)
    rng = np.random.default_rng(k + 10)
    for i in lay.nonleaf:
        Gm = O.prox.s2_matrix(lay, inst, i)
        w = rng.standard_normal(Gm.shape[1])
        p = O.proj_S2_block(Gm, w)
        assert np.max(np.abs(p - nullspace_projection(Gm, w))) <= 1e-13
        assert np.max(np.abs(Gm @ p)) <= 1e-13
        assert np.max(np.abs(O.proj_S2_block(Gm, p) - p)) <= 1e-13


def test_s2_matrix_encodes_avar_conic_form():
    # E'y = a y1 - y2 + y3 1 must equal tau + s on S2 (section 5.2, E of section 4.3)
    inst = _inst(0, [3, 1], 2, 1)
    lay = O.Layout(inst)
    i = 0
    n = len(lay.children[i])
    a = inst.a_risk[i]
    rng = np.random.default_rng(3)
    y = rng.standard_normal(2 * n + 1)
    tau = rng.standard_normal(n)
    s = a * y[:n] - y[n:2 * n] + y[2 * n] - tau
    w = np.concatenate([y, tau, s])
    assert np.max(np.abs(O.prox.s2_matrix(lay, inst, i) @ w)) <= 1e-14


@pytest.mark.parametrize("a", [0.0, 0.3, 1.0])
def test_feasible_point_maps_into_S3_and_s0_is_nested_cost(a):
    inst = _inst(5, [2, 2, 1], 2, 2, a=a)
    lay = O.Layout(inst)
    rng = np.random.default_rng(11)
    # any trajectory satisfying the dynamics, well inside the boxes
    x = np.zeros((lay.num_nodes, lay.nx))
    u = np.zeros((lay.num_nodes, lay.nu))
    x[0] = 0.3 * rng.standard_normal(lay.nx)
    for t in range(lay.N):
        for i in lay.stage_nodes[t]:
            u[i] = 0.2 * rng.standard_normal(lay.nu)
            for c in lay.children[i]:
                x[c] = inst.A[c] @ x[i] + inst.B[c] @ u[i]
    z, V = feasible_conic_point(lay, inst, x, u)
    eta = O.L_apply(lay, inst, z)
    assert np.max(np.abs(O.proj_S3(lay, inst, eta) - eta)) <= 1e-12
    for i in lay.nonleaf:
        idx = O.prox.s2_indices(lay, i)
        assert np.max(np.abs(O.prox.s2_matrix(lay, inst, i) @ z[idx])) <= 1e-12
    assert abs(z[0] - O.nested_cost(lay, inst, x, u)) <= 1e-12 * max(1, abs(z[0]))
    # lowering one epigraph slack below its stage cost leaves S3 (SOC orientation)
    z2 = z.copy()
    z2[lay.tau_off[1]] -= 0.05
    eta2 = O.L_apply(lay, inst, z2)
    assert np.max(np.abs(O.proj_S3(lay, inst, eta2) - eta2)) > 1e-3
    # raising it keeps the point inside
    z3 = z.copy()
    z3[lay.tau_off[1]] += 0.05
    eta3 = O.L_apply(lay, inst, z3)
    assert np.max(np.abs(O.proj_S3(lay, inst, eta3) - eta3)) <= 1e-12


def test_soc_projection_properties():
    rng = np.random.default_rng(5)
    for _ in range(200):
        v = rng.standard_normal(rng.integers(2, 8)) * 3
        p = O.proj_soc(v)
        assert np.linalg.norm(p[:-1]) <= p[-1] + 1e-12          # in the cone
        q = p - v                                                # in the polar = -SOC... (v - p) in -SOC
        assert np.linalg.norm(q[:-1]) <= q[-1] + 1e-12
        assert abs(p @ (v - p)) <= 1e-11 * max(1, v @ v)        # orthogonal


def test_prox_gstar_optimality():
    # p = prox_{alpha g*}(w): pi = (w - p)/alpha is in S3 and <p, s - pi> <= 0 for all s in S3
    inst = _inst(2, [2, 3, 1, 1], 2, 2)
    lay = O.Layout(inst)
    rng = np.random.default_rng(9)
    alpha = 0.37
    for _ in range(5):
        w = 3 * rng.standard_normal(lay.n_eta)
        p = O.prox_gstar(lay, inst, w, alpha)
        pi = (w - p) / alpha
        assert np.max(np.abs(O.proj_S3(lay, inst, pi) - pi)) <= 1e-12
        for _ in range(50):
            s = O.proj_S3(lay, inst, 4 * rng.standard_normal(lay.n_eta))
            assert p @ (s - pi) <= 1e-10


def test_prox_gstar_literal_formula_fails():
    # the printed eq. prox:g without the alpha factor is not the prox: its
    # projection residual is not in S3 for alpha != 1
    inst = _inst(2, [2, 3, 1, 1], 2, 2)
    lay = O.Layout(inst)
    rng = np.random.default_rng(9)
    alpha = 0.37
    w = 3 * rng.standard_normal(lay.n_eta)
    p_lit = w - O.proj_S3(lay, inst, w / alpha)
    pi = (w - p_lit) / alpha
    assert np.max(np.abs(O.proj_S3(lay, inst, pi) - pi)) > 1e-3
