"""C-ABI checks that need no GPU: symbol export and host-side validation."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2212_01110_amd as SP
import spock_gen as G

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "spock.h")).read()
    return sorted(set(re.findall(r"\b(spock_[A-Za-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(SP.LIB_PATH):
        pytest.fail("libspock.so is not built; run __graft_entry__.build()")
    return SP.lib()


def test_every_declared_symbol_is_exported(lib):
    names = _declared_symbols()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(SP.EXPORTED)


def test_version(lib):
    assert "gfx950" in SP.version()


def test_default_settings(lib):
    s = SP.default_settings()
    assert s.eps_abs == 1e-4 and s.m == 3 and s.method == SP.METHOD_SPOCK
    assert s.c0 == 0.99 and s.beta == 0.5 and s.sigma == 0.1 and s.lam == 1.0 and s.max_ls == 20


def _create(anc, prob):
    h = ctypes.c_void_p()
    a = np.ascontiguousarray(anc, dtype=np.int32)
    p = np.ascontiguousarray(prob, dtype=np.float64)
    rc = SP.lib().spock_tree_create(len(a), a.ctypes.data, p.ctypes.data, ctypes.byref(h))
    if rc == 0:
        SP.lib().spock_tree_destroy(h)
    return rc


def test_tree_validation(lib):
    inst = G.make_config(1)
    assert _create(inst.anc, inst.prob) == 0
    t = SP.Tree(inst.anc, inst.prob)
    assert (t.N, t.num_nonleaf, t.num_leaves) == (3, 7, 8)
    # not breadth-first: a child listed before its ancestor's earlier sibling's children
    anc = inst.anc.copy()
    anc[3], anc[5] = anc[5], anc[3]
    assert _create(anc, inst.prob) == -2
    # root must have anc -1
    bad = inst.anc.copy()
    bad[0] = 0
    assert _create(bad, inst.prob) == -2
    # a leaf above the last stage
    assert _create([-1, 0, 0, 1], [1, 0.5, 0.5, 0.5]) == -2
    # probabilities: nonpositive / children not summing to the parent
    p = inst.prob.copy()
    p[1] = 0.0
    assert _create(inst.anc, p) == -3
    p = inst.prob.copy()
    p[3] *= 1.01
    assert _create(inst.anc, p) == -3
    # too small / null
    assert _create([-1], [1.0]) == -1


def test_uneven_and_chain_trees_accepted(lib):
    for b in (0, 3, 7):
        inst = G.make_batch(4, count=b + 1)[b]
        assert _create(inst.anc, inst.prob) == 0
    inst = G.make_config(3)
    assert _create(inst.anc, inst.prob) == 0


def test_invalid_arguments_rejected_before_any_device_call(lib):
    L = SP.lib()
    s = SP.default_settings()
    infos = (SP.Info * 2)()
    arr = (ctypes.c_void_p * 2)()
    # no problem handle / no instances
    assert L.spock_backward_batched(None, 2, arr, arr, 1.0, None, arr, None, None, ctypes.byref(s), infos,
                                    None) == -1
    assert L.spock_backward(None, None, None, 1.0, None, None, None, None, ctypes.byref(s),
                            ctypes.byref(SP.Info()), None) == -1


def test_dense_costs_validated_by_factor(lib):
    # dense Q, R, Q_N (section 4.1) pass through the library's own checks:
    # an indefinite Q, a singular R and a non-symmetric Q_N are rejected with
    # SPOCK_EINVAL when the problem is factored
    inst = G.dense_costs(G.make_config(1), seed=3)
    tree = SP.Tree(inst.anc, inst.prob)
    for name, edit in (("Qm", lambda m: m.__setitem__(2, m[2] - 5.0 * np.eye(m.shape[1]))),
                       ("Rm", lambda m: m.__setitem__(1, 0.0 * m[1])),
                       ("QNm", lambda m: m.__setitem__((-1, 0, 1), m[-1, 0, 1] + 1e-3))):
        bad = inst.copy()
        m = getattr(inst, name).copy()
        edit(m)
        setattr(bad, name, m)
        with pytest.raises(SP.SpockError) as e:
            SP.Problem.from_instance(bad, tree=tree)
        assert e.value.code == -1, name
