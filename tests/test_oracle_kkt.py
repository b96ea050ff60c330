"""Pins of the oracle's whole-solver results and of its first-input
derivatives against a dense interior-point solve of the epigraph program
(tests/checks/kkt.py, written from the program's statement): tiny trees with
several inputs, active input boxes and a in {0, 0.3, 0.6, 1}."""
import numpy as np
import pytest

import oracle as O
import spock_gen as G
from tests.checks.kkt import EpigraphIPM

TIGHT = O.Settings(eps_abs=1e-12, eps_rel=1e-12, max_iters=500000)

CASES = [(71, [2, 2], 2, 2, 0.3), (72, [3, 1], 3, 2, 0.0), (73, [2, 1, 2], 2, 2, 1.0),
         (74, [2, 2], 2, 2, 0.6), (75, [3, 2], 2, 1, 0.3)]


def _inst(seed, br, nx, nu, a):
    return G.make_random_small(seed, br, nx, nu, a=a, box=5.0, ubox=0.6)


@pytest.mark.parametrize("seed,br,nx,nu,a", CASES)
def test_value_and_first_input_match_dense_ipm(seed, br, nx, nu, a):
    inst = _inst(seed, br, nx, nu, a)
    ipm = EpigraphIPM(inst)
    ipm.solve()
    P = O.Problem(inst)
    res = O.spock_solve(P, inst.x0, TIGHT)
    assert res.status == "converged"
    # the input box is active somewhere in every case but the last
    active = np.sum(np.abs(res.u[P.lay.nonleaf]) > 0.6 - 1e-9)
    assert active >= (0 if seed == 75 else 1)
    assert abs(res.V_nested - ipm.V) <= 1e-8 * max(1.0, abs(ipm.V))
    assert abs(res.V_s0 - ipm.V) <= 1e-8 * max(1.0, abs(ipm.V))
    assert np.max(np.abs(res.u0 - ipm.u0)) <= 1e-7


def _ipm_u0(inst, x0=None):
    ipm = EpigraphIPM(inst, x0=x0)
    ipm.solve()
    return ipm.u0, ipm.V


@pytest.mark.parametrize("seed,br,nx,nu,a", CASES[:4])
def test_implicit_first_input_gradients_match_ipm_differences(seed, br, nx, nu, a):
    # du^0/dx0 and du^0/d diag Q of the oracle (fixed-point tangents) against
    # central differences of dense IPM solves (h = 1e-5; the solves are exact
    # to about 1e-11, so the differences carry about 1e-6)
    inst = _inst(seed, br, nx, nu, a)
    P = O.Problem(inst)
    res = O.spock_solve(P, inst.x0, TIGHT)
    g = O.implicit_gradients(P, res.v, inst.x0)
    h = 1e-5
    for k in range(nx):
        xp, xm = inst.x0.copy(), inst.x0.copy()
        xp[k] += h
        xm[k] -= h
        (up, Vp), (um, Vm) = _ipm_u0(inst, xp), _ipm_u0(inst, xm)
        fd = (up - um) / (2 * h)
        assert np.max(np.abs(fd - g["u0_x0"][:, k])) <= 2e-5 * max(1.0, np.max(np.abs(fd))), (k, fd, g["u0_x0"][:, k])
        assert abs((Vp - Vm) / (2 * h) - g["V_x0"][k]) <= 2e-5 * max(1.0, abs(g["V_x0"][k]))
    for c, k in [(1, 0), (2, 1), (P.lay.leaves[0], 0)]:
        ip, im = inst.copy(), inst.copy()
        ip.q[c, k] += h
        im.q[c, k] -= h
        fd = (_ipm_u0(ip)[0] - _ipm_u0(im)[0]) / (2 * h)
        assert np.max(np.abs(fd - g["u0_q"][:, c, k])) <= 2e-5 * max(1.0, np.max(np.abs(fd))), (c, k)
    j = P.lay.leaves[-1]
    ip, im = inst.copy(), inst.copy()
    ip.qN[j, 1] += h
    im.qN[j, 1] -= h
    fd = (_ipm_u0(ip)[0] - _ipm_u0(im)[0]) / (2 * h)
    assert np.max(np.abs(fd - g["u0_qN"][:, j, 1])) <= 2e-5 * max(1.0, np.max(np.abs(fd)))


@pytest.mark.parametrize("seed,br,nx,nu,a", CASES[:3])
def test_implicit_value_gradients_match_envelope(seed, br, nx, nu, a):
    # two formulas for dV*/dtheta: the tangent of s^0 of the fixed point and
    # the envelope theorem on the saddle form
    inst = _inst(seed, br, nx, nu, a)
    P = O.Problem(inst)
    res = O.spock_solve(P, inst.x0, TIGHT)
    g = O.implicit_gradients(P, res.v, inst.x0)
    e = O.envelope_gradients(P, res.v)
    sc = max(1.0, np.max(np.abs(e["x0"])))
    assert np.max(np.abs(g["V_x0"] - e["x0"])) <= 1e-8 * sc
    assert np.max(np.abs(g["V_q"][1:] - e["q"][1:])) <= 1e-8 * max(1.0, np.max(np.abs(e["q"])))
    lv = P.lay.leaves
    assert np.max(np.abs(g["V_qN"][lv] - e["qN"][lv])) <= 1e-8 * max(1.0, np.max(np.abs(e["qN"])))
