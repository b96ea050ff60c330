"""Pins of the oracle's envelope gradients by central finite differences of
tight oracle solves (tiny trees)."""
import numpy as np
import pytest

import oracle as O
import spock_gen as G

TIGHT = O.Settings(eps_abs=1e-12, eps_rel=1e-12, max_iters=500000)


def _V(inst, alpha):
    P = O.Problem(inst, alpha=alpha)
    return O.spock_solve(P, inst.x0, TIGHT)


@pytest.mark.parametrize("seed,a", [(61, 0.5), (62, 1.0)])
def test_envelope_gradients_match_central_differences(seed, a):
    inst = G.make_random_small(seed, [2, 2], 2, 1, a=a, box=50.0, ubox=0.8)
    P = O.Problem(inst)
    res = O.spock_solve(P, inst.x0, TIGHT)
    g = O.envelope_gradients(P, res.v)
    h = 1e-5
    for k in range(inst.nx):
        ip, im = inst.copy(), inst.copy()
        ip.x0[k] += h
        im.x0[k] -= h
        fd = (_V(ip, P.alpha).V_s0 - _V(im, P.alpha).V_s0) / (2 * h)
        assert abs(fd - g["x0"][k]) <= 1e-5 * max(1, abs(fd)), (k, fd, g["x0"][k])
    for c, k in [(1, 0), (2, 1), (4, 0)]:
        ip, im = inst.copy(), inst.copy()
        ip.q[c, k] += h
        im.q[c, k] -= h
        fd = (_V(ip, P.alpha).V_s0 - _V(im, P.alpha).V_s0) / (2 * h)
        assert abs(fd - g["q"][c, k]) <= 1e-5 * max(1, abs(fd)), (c, k, fd, g["q"][c, k])
    j = P.lay.leaves[0]
    ip, im = inst.copy(), inst.copy()
    ip.qN[j, 1] += h
    im.qN[j, 1] -= h
    fd = (_V(ip, P.alpha).V_s0 - _V(im, P.alpha).V_s0) / (2 * h)
    assert abs(fd - g["qN"][j, 1]) <= 1e-5 * max(1, abs(fd))
