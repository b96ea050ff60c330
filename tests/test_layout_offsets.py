"""The closed-form offsets used by the HIP kernels (breadth-first sizes:
first child fc_i = 1 + sum_{k<i} n_k) against the oracle's accumulated
layout, on trees of every shape used by the tests and workloads."""
import numpy as np
import pytest

import oracle as O
import spock_gen as G


def closed_forms(anc, nx, nu):
    nn = len(anc)
    nch = np.zeros(nn, dtype=np.int64)
    fc = np.full(nn, -1, dtype=np.int64)
    for i in range(1, nn):
        if nch[anc[i]] == 0:
            fc[anc[i]] = i
        nch[anc[i]] += 1
    nl = int(np.sum(nch > 0))
    zU = 1 + nn * nx
    zZ2 = zU + nl * nu
    eE2 = 2 * (nn - 1) + nl * (2 + nx + nu)
    eE3 = eE2 + (nn - 1) * (nx + nu + 2)
    f = {}
    f["x"] = lambda i: 1 + i * nx
    f["u"] = lambda i: zU + i * nu
    f["z2"] = lambda i: zZ2 + 4 * (fc[i] - 1) + i
    f["s"] = lambda c: 0 if c == 0 else f["z2"](anc[c]) + 3 * nch[anc[c]] + 1 + (c - fc[anc[c]])
    f["tau"] = lambda c: f["z2"](anc[c]) + 2 * nch[anc[c]] + 1 + (c - fc[anc[c]])
    f["e1"] = lambda i: 2 * (fc[i] - 1) + i * (2 + nx + nu)
    f["e1s"] = lambda i: f["e1"](i) + 2 * nch[i] + 1
    f["e1x"] = lambda i: f["e1s"](i) + 1
    f["e1u"] = lambda i: f["e1x"](i) + nx
    f["e2"] = lambda c: eE2 + (c - 1) * (nx + nu + 2)
    f["e3"] = lambda j: eE3 + (j - nl) * (2 * nx + 2)
    nz = 1 + nn * nx + nl * nu + 4 * (nn - 1) + nl
    neta = eE3 + (nn - nl) * (2 * nx + 2)
    return f, nl, nz, neta


TREES = [([2, 2, 2], 2, 1), ([3, 1, 2], 4, 3), ([1, 1, 1, 1], 3, 2), ([5, 3], 6, 2),
         ([2, 2, 1], 1, 1), ([2, 2, 2, 2, 2, 1, 1, 1, 1, 1], 20, 10), ([4, 1, 3, 1], 5, 7)]


@pytest.mark.parametrize("br,nx,nu", TREES)
def test_closed_form_offsets(br, nx, nu):
    inst = G.make_random_small(0, br, nx, nu)
    lay = O.Layout(inst)
    f, nl, nz, neta = closed_forms(inst.anc, nx, nu)
    assert nl == len(lay.nonleaf) and lay.nonleaf == list(range(nl))
    assert (nz, neta) == (lay.n_z, lay.n_eta)
    for i in range(lay.num_nodes):
        assert f["x"](i) == lay.x_off[i]
        assert f["s"](i) == lay.s_off[i]
        if i > 0:
            assert f["tau"](i) == lay.tau_off[i]
            assert f["e2"](i) == lay.e2x[i]
    for i in lay.nonleaf:
        assert f["u"](i) == lay.u_off[i]
        assert f["z2"](i) == lay.y_off[i]
        assert f["e1"](i) == lay.e1y[i]
        assert f["e1s"](i) == lay.e1s[i]
        assert f["e1x"](i) == lay.e1x[i]
        assert f["e1u"](i) == lay.e1u[i]
    for j in lay.leaves:
        assert f["e3"](j) == lay.e3x[j]


def test_uneven_batch_trees():
    for inst in G.make_batch(4, count=6):
        lay = O.Layout(inst)
        f, nl, nz, neta = closed_forms(inst.anc, inst.nx, inst.nu)
        assert (nz, neta) == (lay.n_z, lay.n_eta)
        for i in lay.nonleaf:
            assert f["z2"](i) == lay.y_off[i] and f["e1"](i) == lay.e1y[i]
