"""The paper's section-6 experiments on the GPU, against the oracle: the
data-centre model (tridiagonal A(w), B = I, Q = I, R = 10 I, |x| <= 1,
|u| <= 1.5, AV@R 0.95, binary tree with probabilities (0.3, 0.7)).

The paper's own counts (571 SPOCK vs 3159 CP calls of L at 1e-5) depend on a
step size and SuperMann parameters it does not print, so they are context,
not parity: parity is with the oracle run with the same alpha and
parameters (tests/golden)."""
import json
import os

import numpy as np
import pytest

import oracle as O
import paper_2212_01110_amd as SP
import spock_gen as G
from tests.gpu_util import check, dev, host

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _golden(key):
    path = os.path.join(os.path.dirname(__file__), "golden", "oracle_refs.json")
    refs = json.load(open(path)) if os.path.exists(path) else {}
    if key not in refs:
        pytest.skip(f"golden reference {key} not generated (tests/golden/make_golden.py)")
    return refs[key]


def test_datacentre_cp_vs_spock_counts_match_oracle(monkeypatch):
    # section 6, first experiment (N 7, n_x 5): CP is deterministic up to
    # rounding, so its T-evaluation count matches the oracle's to a couple of
    # iterations; SPOCK's decisions can flip after long runs (the FP64
    # trajectories separate like any chaotic iteration, and the mapping's
    # rounding differs from the oracle's), so its count is compared within
    # 25% and its value at the tolerance. The mapping is fixed so that the
    # run is repeatable.
    monkeypatch.setenv("SPOCK_TEAM", "16")
    inst = G.make_datacentre(7, 5)
    cp_ref = _golden("datacentre_N7_nx5_cp_1e-5")
    sp_ref = _golden("datacentre_N7_nx5_spock_1e-5")
    gp = SP.Problem.from_instance(inst, precision=SP.FP64, alpha=cp_ref["alpha"])
    x0 = dev(inst.x0, torch.float64)
    out = {}
    for method in ("cp", "spock"):
        v = torch.zeros(gp.n_v, dtype=torch.float64, device="cuda")
        out[method] = gp.solve(x0, v, SP.default_settings(eps_abs=1e-5, eps_rel=1e-5, max_iters=200000,
                                                          method=method, compute_nested=1))
        assert out[method]["status"] == "converged", out[method]
    assert abs(out["cp"]["t_evals"] - cp_ref["t_evals"]) <= 2, (out["cp"], cp_ref["t_evals"])
    assert abs(out["spock"]["t_evals"] - sp_ref["t_evals"]) <= 0.25 * sp_ref["t_evals"], (out["spock"],
                                                                                        sp_ref["t_evals"])
    for m, ref in (("cp", cp_ref), ("spock", sp_ref)):
        check(f"datacentre_V:{m}", abs(out[m]["V_nested"] - ref["V_nested"]) / abs(ref["V_nested"]), 1e-4)
    # the acceleration the experiment is about: SPOCK needs fewer T evaluations
    assert out["spock"]["t_evals"] * 2 < out["cp"]["t_evals"]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_datacentre_nx50_short_horizon_matches_oracle(prec):
    # the open-loop series at n_x = n_u = 50 (here N = 3, 15 nodes): the
    # solution against the oracle solved tight
    inst = G.make_datacentre(3, 50)
    op = O.Problem(inst)
    ref = O.spock_solve(op, inst.x0, O.Settings(eps_abs=1e-9, eps_rel=1e-9))
    gp = SP.Problem.from_instance(inst, precision=SP.FP64 if prec == "fp64" else SP.FP32, alpha=op.alpha)
    x0 = dev(inst.x0, torch.float64)
    v = torch.zeros(gp.n_v, dtype=gp.torch_dtype, device="cuda")
    eps = 1e-8 if prec == "fp64" else 1e-5
    info = gp.solve(x0, v, SP.default_settings(eps_abs=eps, eps_rel=eps, max_iters=200000, compute_nested=1))
    assert info["status"] == "converged", info
    check(f"dc50_V:{prec}", abs(info["V_nested"] - ref.V_nested) / max(1, abs(ref.V_nested)), 1e-4)
    out = host(v)
    u0 = out[op.lay.u_off[0]: op.lay.u_off[0] + op.lay.nu]
    check(f"dc50_u0:{prec}", np.max(np.abs(u0 - ref.u0)) / max(1, np.max(np.abs(ref.u0))), 1e-4)
