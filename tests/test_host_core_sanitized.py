"""Host-only library code (tree validation, data checks, Alg. 1, ||L||,
nested AV@R cost, dataflow item list) built on the CPU with g++ under
AddressSanitizer and UndefinedBehaviorSanitizer (tests/native), run on
several trees, and compared with the oracle: K, Abar and P of Alg. 1, ||L||
and the nested cost; malformed trees and data must give their error codes."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle as O
import spock_gen as G

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = [os.path.join(ROOT, "tests", "native", "host_core_check.cpp"),
       os.path.join(ROOT, "paper_2212_01110_amd", "csrc", "host_core.cpp")]


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if not shutil.which("g++"):
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("hcc") / "host_core_check")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-pthread", *SRC, "-o", exe],
                   check=True)
    return exe


def _run(driver, tmp_path, inst, x=None, u=None, nc=1, anc=None, prob=None, dense=None):
    nn, nx, nu = inst.num_nodes, inst.nx, inst.nu
    anc = inst.anc if anc is None else anc
    prob = inst.prob if prob is None else prob
    nl = int(np.sum(np.bincount(np.asarray(anc)[1:], minlength=nn) > 0))
    x = np.zeros((nn, nx)) if x is None else x
    u = np.zeros((nl, nu)) if u is None else u
    parts = [np.array([nn, nx, nu]), np.asarray(anc), np.asarray(prob)]
    parts += [np.asarray(getattr(inst, k), float).ravel() for k in
              ("A", "B", "q", "r", "qN", "xmin", "xmax", "umin", "umax", "a_risk")]
    parts += [x.ravel(), u.ravel(), np.array([nc]), np.array([0 if dense is None else 1])]
    if dense is not None:
        parts += [np.asarray(m, float).ravel() for m in dense]
    path = tmp_path / "case.txt"
    with open(path, "w") as f:
        for p in parts:
            f.write(" ".join(repr(float(v)) if p.dtype.kind == "f" else str(int(v)) for v in p) + "\n")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    res = subprocess.run([driver, str(path)], capture_output=True, text=True, env=env)
    assert res.returncode == 0, res.stderr[-4000:]
    assert "runtime error" not in res.stderr and "AddressSanitizer" not in res.stderr, res.stderr[-4000:]
    out = {}
    for line in res.stdout.splitlines():
        k, *vals = line.split()
        out[k] = np.array([float(v) for v in vals])
    return out


CASES = [("config1", lambda: G.make_config(1), 1), ("b3-1-2", lambda: G.make_random_small(11, [3, 1, 2], 4, 3), 2),
         ("b5-wide", lambda: G.make_random_small(14, [5, 3], 6, 2), 2),
         ("config4-b3", lambda: G.make_batch(4, count=4)[3], 1),
         ("datacentre", lambda: G.make_datacentre(4, 3), 1)]


@pytest.mark.parametrize("name,mk,nc", CASES)
def test_host_core_matches_oracle_under_sanitizers(driver, tmp_path, name, mk, nc):
    inst = mk()
    P = O.Problem(inst)
    lay = P.lay
    rng = np.random.default_rng(3)
    x = rng.standard_normal((inst.num_nodes, inst.nx))
    u = rng.standard_normal((len(lay.nonleaf), inst.nu))
    out = _run(driver, tmp_path, inst, x, u, nc=nc)
    assert out["tree_rc"][0] == 0 and out["data_rc"][0] == 0 and out["factor_rc"][0] == 0
    assert tuple(out["shape"].astype(int)) == (lay.N, len(lay.nonleaf), len(lay.leaves))
    nx, nu = inst.nx, inst.nu
    K = out["K"].reshape(-1, nu, nx)
    Ab = out["Abar"].reshape(-1, nx, nx)
    Pm = out["P"].reshape(-1, nx, nx)
    fac = P.fac
    for i in lay.nonleaf:
        assert np.max(np.abs(K[i] - fac["K"][i])) <= 1e-10 * max(1, np.max(np.abs(fac["K"][i])))
    for c in range(1, inst.num_nodes):
        assert np.max(np.abs(Ab[c] - fac["Abar"][c])) <= 1e-10 * max(1, np.max(np.abs(fac["Abar"][c])))
    for i in range(inst.num_nodes):
        assert np.max(np.abs(Pm[i] - fac["P"][i])) <= 1e-10 * max(1, np.max(np.abs(fac["P"][i])))
    assert abs(out["normL"][0] - P.normL) <= 1e-12 * P.normL
    uu = np.zeros((inst.num_nodes, nu))
    uu[lay.nonleaf] = u
    ref = O.nested_cost(lay, inst, x, uu)
    assert abs(out["nested"][0] - ref) <= 1e-12 * max(1, abs(ref))
    # item list: every backward item of a family comes after those of its
    # nonleaf children; forward items of a parent before its children's
    rc, nbwd, _ = out["items_rc"].astype(int)
    assert rc == 0
    items = out["items"].astype(int)
    fam = items // 64
    pos_b = {f: k for k, f in enumerate(fam[:nbwd])}
    pos_f = {}
    for k, f in enumerate(fam[nbwd:]):
        pos_f.setdefault(f, k)
    for c in lay.nonleaf[1:]:
        i = lay.anc[c]
        assert pos_b[c] < pos_b[i] and pos_f[i] < pos_f[c]
    assert sorted(set(fam[:nbwd])) == list(lay.nonleaf)
    # post-pass blocks: consecutive runs of families covering all of them,
    # each with at most cap children (the children of a run are contiguous)
    nch = np.bincount(np.asarray(lay.anc[1:]), minlength=inst.num_nodes)
    for tpb in (32, 16, 8, 4):
        nb, cap = out[f"pblk{tpb}"].astype(int)
        bf = out[f"pblk{tpb}_f"].astype(int)
        assert len(bf) == nb + 1 and bf[0] == 0 and bf[-1] == len(lay.nonleaf)
        assert np.all(np.diff(bf) >= 1)
        for k in range(nb):
            assert nch[bf[k]:bf[k + 1]].sum() <= cap


def test_malformed_trees_and_data_under_sanitizers(driver, tmp_path):
    inst = G.make_config(1)
    anc = inst.anc.copy()
    anc[3], anc[5] = anc[5], anc[3]                     # not breadth-first
    assert _run(driver, tmp_path, inst, anc=anc)["tree_rc"][0] == -2
    p = inst.prob.copy()
    p[3] *= 1.01                                        # children do not sum to the parent
    assert _run(driver, tmp_path, inst, prob=p)["tree_rc"][0] == -3
    bad = inst.copy()
    bad.q[2, 0] = -1.0                                  # nonpositive weight
    assert _run(driver, tmp_path, bad)["data_rc"][0] == -1
    bad = inst.copy()
    bad.xmin[4, 1], bad.xmax[4, 1] = 1.0, -1.0           # empty box
    assert _run(driver, tmp_path, bad)["data_rc"][0] == -4
    bad = inst.copy()
    bad.A[5, 0, 0] = np.nan                             # non-finite dynamics
    assert _run(driver, tmp_path, bad)["data_rc"][0] == -1


def _sym_root_ok(M, H):
    # H symmetric, positive semidefinite, H @ H == M
    assert np.max(np.abs(H - np.swapaxes(H, -1, -2))) <= 1e-13 * max(1.0, np.max(np.abs(H)))
    assert np.min(np.linalg.eigvalsh(H)) >= -1e-12
    assert np.max(np.abs(H @ H - M)) <= 1e-12 * max(1.0, np.max(np.abs(M)))


@pytest.mark.parametrize("name,mk", [("config1", lambda: G.make_config(1)),
                                      ("b5-wide", lambda: G.make_random_small(14, [5, 3], 6, 2))])
def test_dense_costs_under_sanitizers(driver, tmp_path, name, mk):
    # dense costs (section 4.1: Q, Q_N positive semidefinite, R positive
    # definite): their symmetric roots and ||L|| of the general layout
    # against the oracle's L, which uses the same roots
    inst = G.dense_costs(mk(), seed=7)
    nn, nx, nu = inst.num_nodes, inst.nx, inst.nu
    Q = inst.Qm.copy()
    Q[3] = Q[3] - (np.min(np.linalg.eigvalsh(Q[3]))) * np.eye(nx)  # singular: allowed
    inst.Qm = Q
    out = _run(driver, tmp_path, inst, dense=(inst.Qm, inst.Rm, inst.QNm))
    assert out["data_rc"][0] == 0 and out["general_rc"][0] == 0
    lay = O.Problem(inst).lay
    for key, M, n, nodes in (("Qh", inst.Qm, nx, range(1, nn)), ("Rh", inst.Rm, nu, range(1, nn)),
                             ("QNh", inst.QNm, nx, lay.leaves)):
        H = out[key].reshape(nn, n, n)
        for c in nodes:
            _sym_root_ok(M[c], H[c])
    ref = O.Problem(inst).normL
    assert abs(out["normL"][0] - ref) <= 1e-12 * ref


def test_dense_costs_rejected_under_sanitizers(driver, tmp_path):
    inst = G.dense_costs(G.make_config(1), seed=8)
    nx, nu = inst.nx, inst.nu

    def rc(Qm=None, Rm=None, QNm=None):
        m = (inst.Qm if Qm is None else Qm, inst.Rm if Rm is None else Rm, inst.QNm if QNm is None else QNm)
        return _run(driver, tmp_path, inst, dense=m)["data_rc"][0]

    assert rc() == 0
    Q = inst.Qm.copy()
    Q[2, 0, 1] += 1e-3                                  # not symmetric
    assert rc(Qm=Q) == -1
    Q = inst.Qm.copy()
    Q[4] -= 3.0 * np.eye(nx)                            # indefinite
    assert rc(Qm=Q) == -1
    R = inst.Rm.copy()
    R[1] = np.zeros((nu, nu))                           # R must be definite
    assert rc(Rm=R) == -1
    QN = inst.QNm.copy()
    QN[-1, 0, 0] = np.inf                               # non-finite
    assert rc(QNm=QN) == -1
