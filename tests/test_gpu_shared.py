"""GPU parity of the shared-tree batched form (instances of one problem that
differ in x0 and iterate; the sweeps of Alg. 2 as 16-instance matrix-core
tiles): one evaluation of T per instance against the oracle element by
element, converged solutions against the oracle's stored references, and the
decisions of Alg. 3 against the single-instance solver step by step."""
import json
import os

import numpy as np
import pytest

import oracle as O
import paper_2212_01110_amd as SP
import spock_gen as G
from tests.gpu_util import check, dev, host, relerr, seeded

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

FP = {"fp64": (SP.FP64, 1e-12), "fp32": (SP.FP32, 5e-6)}
STAT = {"fp64": 1e-12, "fp32": 2e-6}
SHARED = 1024  # mapping reported by the shared-tree form


def _golden(key):
    path = os.path.join(os.path.dirname(__file__), "golden", "oracle_refs.json")
    refs = json.load(open(path)) if os.path.exists(path) else {}
    if key not in refs:
        pytest.skip(f"golden reference {key} not generated (tests/golden/make_golden.py)")
    return refs[key]


def _with_x0s(inst, B, seed, scale=1.0):
    """B copies of one instance with their own x0 (inside the root box)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(B):
        c = inst.copy()
        c.x0 = np.clip(scale * rng.standard_normal(inst.nx), 0.9 * inst.xmin[0], 0.9 * inst.xmax[0])
        out.append(c)
    return out


# (instances, why): n_x, n_u across 1..4 tiles of 16 rows, uneven families,
# batches that are not a multiple of 16
CASES = {
    "config5x64": lambda: G.make_batch(5),
    "b5-wide-x5": lambda: _with_x0s(G.make_random_small(14, [5, 3], 6, 2), 5, 1),
    "nx37-nu21-x20": lambda: _with_x0s(G.make_random_small(18, [3, 1], 37, 21), 20, 2),
    "nx64-x17": lambda: _with_x0s(G.make_random_small(13, [2, 2, 2], 64, 64), 17, 3),
    "nx1-x3": lambda: _with_x0s(G.make_random_small(15, [2, 2, 1], 1, 1), 3, 4),
}


@pytest.mark.parametrize("cut", ["auto", "0", "1"])
@pytest.mark.parametrize("prec", list(FP))
@pytest.mark.parametrize("name", list(CASES))
def test_shared_T_matches_oracle(name, prec, cut, monkeypatch):
    # max_iters = 0: the call evaluates T once at the given point of every
    # instance and returns it (status maxiter), with xi0 of that point. The
    # sweeps in one launch (cut 0), or split at stage 1 (subtree workgroups
    # below it) or at the automatic cut
    if cut != "auto":
        monkeypatch.setenv("SPOCK_SH_CUT", cut)
    insts = CASES[name]()
    op = O.Problem(insts[0])
    gp = SP.Problem.from_instance(insts[0], precision=FP[prec][0], alpha=op.alpha)
    dt = gp.torch_dtype
    rng = seeded(f"shared:{name}:{prec}")
    vins = [rng.standard_normal(op.lay.n_v) for _ in insts]
    vs = [dev(v, dt) for v in vins]
    vin_used = [host(v) for v in vs]
    x0s = [dev(i.x0, torch.float64) for i in insts]
    infos = SP.solve_batched([gp] * len(insts), x0s, vs, SP.default_settings(max_iters=0, eps_abs=0, eps_rel=0))
    worst, worst_xi = 0.0, 0.0
    for b, inst in enumerate(insts):
        assert infos[b]["mapping"] == SHARED and infos[b]["status"] == "maxiter", infos[b]
        assert infos[b]["t_evals"] == 1
        op.inst = inst
        ref = O.T_apply(op, vin_used[b], inst.x0)
        worst = max(worst, relerr(host(vs[b]), ref))
        rs = O.residual_stats(op, vin_used[b] - ref)
        xi = max(np.max(np.abs(rs["xi_p"])), np.max(np.abs(rs["xi_d"])))
        worst_xi = max(worst_xi, abs(infos[b]["xi0"] - xi) / max(1.0, xi))
    check(f"shared_T:{name}:{prec}:{cut}", worst, FP[prec][1])
    check(f"shared_xi0:{name}:{prec}:{cut}", worst_xi, STAT[prec])


@pytest.mark.parametrize("method", ["spock", "cp"])
def test_shared_follows_single_instance_solver(method):
    # FP64, 40 iterations: every instance takes the decisions of spock_solve
    # (K0 / K1 / K2 / backtracks / KM counts equal) and lands on its iterate
    insts = G.make_batch(5, count=6)
    op = O.Problem(insts[0])
    gp = SP.Problem.from_instance(insts[0], precision=SP.FP64, alpha=op.alpha)
    st = SP.default_settings(max_iters=40, eps_abs=0, eps_rel=0, method=method)
    x0s = [dev(i.x0, torch.float64) for i in insts]
    vs = [torch.zeros(gp.n_v, dtype=torch.float64, device="cuda") for _ in insts]
    infos = SP.solve_batched([gp] * len(insts), x0s, vs, st)
    for b in range(len(insts)):
        v1 = torch.zeros(gp.n_v, dtype=torch.float64, device="cuda")
        one = gp.solve(x0s[b], v1, st)
        for k in ("iters", "t_evals", "n_k0", "n_k1", "n_k2", "n_km", "n_backtracks"):
            assert infos[b][k] == one[k], (b, k, infos[b], one)
        check(f"shared_vs_single:{method}:{b}", relerr(host(vs[b]), host(v1)), 1e-9)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_shared_solve_matches_oracle_references(prec):
    # the 64-instance workload; instances 0 and 37 against the oracle's
    # solutions at 1e-11, every instance converged
    insts = G.make_batch(5)
    refs = {0: _golden("config5b0_tangents_1e-11"), 37: _golden("config5b37_tangents_1e-11")}
    gp = SP.Problem.from_instance(insts[0], precision=FP[prec][0], alpha=refs[0]["alpha"])
    eps = 1e-10 if prec == "fp64" else 1e-5
    x0s = [dev(i.x0, torch.float64) for i in insts]
    vs = [torch.zeros(gp.n_v, dtype=gp.torch_dtype, device="cuda") for _ in insts]
    infos = SP.solve_batched([gp] * len(insts), x0s, vs,
                             SP.default_settings(eps_abs=eps, eps_rel=eps, max_iters=400000))
    assert all(i["status"] == "converged" and i["mapping"] == SHARED for i in infos), \
        [(i["status"], i["mapping"]) for i in infos]
    lay = O.Problem(insts[0]).lay
    # FP64: residual 1e-10 times a modest condition number (measured 1e-10);
    # FP32: the 1e-5 residual (measured 3e-6; the FP32 floor of this tree
    # is below it)
    tol = 1e-9 if prec == "fp64" else 3e-5
    for b, r in refs.items():
        check(f"shared_V:{b}:{prec}", abs(infos[b]["V_s0"] - r["V_s0"]) / max(1.0, abs(r["V_s0"])), tol)
        u0 = host(vs[b])[lay.u_off[0]: lay.u_off[0] + lay.nu]
        check(f"shared_u0:{b}:{prec}", np.max(np.abs(u0 - np.array(r["u0"]))) / max(1.0, np.max(np.abs(r["u0"]))), tol)


def test_shared_and_block_engines_agree(monkeypatch):
    # the same 20 instances through the per-instance block engine
    # (SPOCK_SHARED=0): converged values agree to the solve tolerance
    # (measured 1.6e-9 at eps 1e-9)
    insts = G.make_batch(5, count=20)
    gp = SP.Problem.from_instance(insts[0], precision=SP.FP64)
    st = SP.default_settings(eps_abs=1e-9, eps_rel=1e-9, max_iters=200000)
    x0s = [dev(i.x0, torch.float64) for i in insts]
    va = [torch.zeros(gp.n_v, dtype=torch.float64, device="cuda") for _ in insts]
    ia = SP.solve_batched([gp] * len(insts), x0s, va, st)
    monkeypatch.setenv("SPOCK_SHARED", "0")
    vb = [torch.zeros(gp.n_v, dtype=torch.float64, device="cuda") for _ in insts]
    ib = SP.solve_batched([gp] * len(insts), x0s, vb, st)
    assert all(i["mapping"] == SHARED for i in ia) and all(i["mapping"] != SHARED for i in ib)
    for b in range(len(insts)):
        assert ia[b]["status"] == ib[b]["status"] == "converged"
        check(f"shared_vs_block:{b}", abs(ia[b]["V_s0"] - ib[b]["V_s0"]) / max(1.0, abs(ib[b]["V_s0"])), 1e-8)


def test_shared_rejects_x0_outside_box():
    insts = G.make_batch(5, count=3)
    gp = SP.Problem.from_instance(insts[0], precision=SP.FP64)
    x0s = [dev(i.x0, torch.float64) for i in insts]
    x0s[1] = dev(np.full(insts[0].nx, 2.0 * insts[0].xmax[0].max()), torch.float64)
    vs = [torch.full((gp.n_v,), 7.0, dtype=torch.float64, device="cuda") for _ in insts]
    infos = SP.solve_batched([gp] * 3, x0s, vs, SP.default_settings(max_iters=50))
    assert infos[1]["status"] == "rejected"
    assert float(host(vs[1]).min()) == 7.0 == float(host(vs[1]).max())
    assert infos[0]["status"] in ("converged", "maxiter") and infos[2]["status"] in ("converged", "maxiter")
