"""GPU parity of spock_backward (implicit differentiation at the fixed point)
against the oracle: envelope gradients of V*, fixed-point tangents of V* and
u^0 (oracle.implicit_gradients on tiny trees; stored tangents of the 95-node
tree from tests/golden), and central finite differences of FP64 solves at
h = 1e-6."""
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

TIGHT = O.Settings(eps_abs=1e-12, eps_rel=1e-12, max_iters=500000)


def _gpu_solve(gp, inst, x0=None, eps=1e-11):
    x0t = dev(inst.x0 if x0 is None else x0, torch.float64)
    v = torch.zeros(gp.n_v, dtype=gp.torch_dtype, device="cuda")
    info = gp.solve(x0t, v, SP.default_settings(eps_abs=eps, eps_rel=eps, max_iters=400000))
    return v, x0t, info


def _golden(key):
    path = os.path.join(os.path.dirname(__file__), "golden", "oracle_refs.json")
    refs = json.load(open(path)) if os.path.exists(path) else {}
    if key not in refs:
        pytest.skip(f"golden reference {key} not generated (tests/golden/make_golden.py)")
    return refs[key]


CASES = [("config1", lambda: G.make_config(1)),
         ("small-a05", lambda: G.make_random_small(61, [2, 2], 2, 1, a=0.5, box=50.0, ubox=0.8)),
         ("small-a1", lambda: G.make_random_small(62, [2, 2], 2, 1, a=1.0, box=50.0, ubox=0.8)),
         ("small-b3", lambda: G.make_random_small(63, [3, 1], 3, 2, a=0.3, box=50.0))]


@pytest.mark.parametrize("name,mk", CASES)
def test_value_gradients_match_oracle_envelope(name, mk):
    inst = mk()
    op = O.Problem(inst)
    ref = O.spock_solve(op, inst.x0, TIGHT)
    g = O.envelope_gradients(op, ref.v)
    gp = SP.Problem.from_instance(inst, precision=SP.FP64, alpha=op.alpha)
    v, x0t, info = _gpu_solve(gp, inst)
    assert info["status"] == "converged"
    gx, gq, gqN, binfo = gp.backward(v, x0t, gV=1.0)
    assert binfo["status"] == "converged", binfo
    check(f"bwd_Vx0:{name}", np.max(np.abs(host(gx) - g["x0"])) / max(1.0, np.max(np.abs(g["x0"]))), 1e-6)
    check(f"bwd_Vq:{name}", np.max(np.abs(host(gq)[1:] - g["q"][1:])) / max(1.0, np.max(np.abs(g["q"]))), 1e-6)
    lv = op.lay.leaves
    check(f"bwd_VqN:{name}", np.max(np.abs(host(gqN)[lv] - g["qN"][lv])) / max(1.0, np.max(np.abs(g["qN"]))),
          1e-6)


# several inputs, active input boxes, a in {0, 0.3, 0.6}
U0_CASES = [(71, [2, 2], 2, 2, 0.3), (72, [3, 1], 3, 2, 0.0), (74, [2, 2], 2, 2, 0.6)]


@pytest.mark.parametrize("seed,br,nx,nu,a", U0_CASES)
def test_first_input_gradients_match_oracle(seed, br, nx, nu, a):
    # du^0/dx0, du^0/d diag Q and du^0/d diag Q_N: one adjoint per component
    # of u^0 (cotangent e_j) against the oracle's fixed-point tangents, which
    # are pinned by central differences of a dense interior-point solver
    inst = G.make_random_small(seed, br, nx, nu, a=a, box=5.0, ubox=0.6)
    op = O.Problem(inst)
    ref = O.spock_solve(op, inst.x0, TIGHT)
    g = O.implicit_gradients(op, ref.v, inst.x0)
    gp = SP.Problem.from_instance(inst, precision=SP.FP64, alpha=op.alpha)
    v, x0t, info = _gpu_solve(gp, inst)
    assert info["status"] == "converged"
    lv = op.lay.leaves
    for j in range(nu):
        e = np.zeros(nu)
        e[j] = 1.0
        gx, gq, gqN, binfo = gp.backward(v, x0t, gV=0.0, gu0=dev(e, torch.float64))
        assert binfo["status"] == "converged", binfo
        sc = max(1.0, np.max(np.abs(g["u0_x0"][j])), np.max(np.abs(g["u0_q"][j])))
        check(f"bwd_u0x0:{seed}:{j}", np.max(np.abs(host(gx) - g["u0_x0"][j])) / sc, 1e-6)
        check(f"bwd_u0q:{seed}:{j}", np.max(np.abs(host(gq)[1:] - g["u0_q"][j][1:])) / sc, 1e-6)
        check(f"bwd_u0qN:{seed}:{j}", np.max(np.abs(host(gqN)[lv] - g["u0_qN"][j][lv])) / sc, 1e-6)


def _direction(kind, seed, inst):
    # the same seeded directions as tests/golden/make_golden.py
    rng = np.random.default_rng(seed)
    if kind == "x0":
        return rng.standard_normal(inst.nx)
    d = rng.standard_normal((inst.num_nodes, inst.nx))
    d[0] = 0.0
    return d


# FP64: solve and adjoint in FP64; FP32: FP32 storage forward and adjoint
# (its forward solve stops at 1e-6, above its residual floor)
PREC = {"fp64": (SP.FP64, 1e-11, 1e-12, 1e-6), "fp32": (SP.FP32, 1e-6, 1e-7, 1e-4)}


@pytest.mark.parametrize("prec", list(PREC))
@pytest.mark.parametrize("key,mk", [("config5_tangents_1e-11", lambda: G.make_config(5)),
                                    ("config5b0_tangents_1e-11", lambda: G.make_batch(5, count=1)[0]),
                                    ("config5b37_tangents_1e-11", lambda: G.make_batch(5, count=38)[37])])
def test_95_node_gradients_match_oracle_tangents(key, mk, prec):
    # gradients of V* + g.u^0 (g seeded) along the stored directions of x0
    # and diag Q, from one adjoint solve
    ref = _golden(key)
    inst = mk()
    pr, eps, beps, tol = PREC[prec]
    gp = SP.Problem.from_instance(inst, precision=pr, alpha=ref["alpha"])
    v, x0t, info = _gpu_solve(gp, inst, eps=eps)
    assert info["status"] == "converged", info
    gu = np.random.default_rng(7).standard_normal(inst.nu)
    gx, gq, _, binfo = gp.backward(v, x0t, gV=1.0, gu0=dev(gu, torch.float64),
                                   settings=SP.default_settings(eps_abs=beps, max_iters=400000))
    assert binfo["status"] == "converged", binfo
    for d in ref["dirs"]:
        dirv = _direction(d["kind"], d["seed"], inst)
        want = d["dV"] + gu @ np.array(d["du0"])
        got = host(gx) @ dirv if d["kind"] == "x0" else float(np.sum(host(gq)[1:] * dirv[1:]))
        check(f"bwd95:{key}:{d['kind']}{d['seed']}:{prec}", abs(got - want) / max(1.0, abs(want)), tol)


def test_95_node_value_gradient_matches_central_differences():
    # central differences of FP64 GPU solves at h = 1e-6 (solves to 1e-12)
    inst = G.make_config(5)
    gp = SP.Problem.from_instance(inst, precision=SP.FP64)
    v, x0t, info = _gpu_solve(gp, inst, eps=1e-12)
    gx, _, _, binfo = gp.backward(v, x0t, gV=1.0)
    assert binfo["status"] == "converged"
    d = np.random.default_rng(5).standard_normal(inst.nx)
    h = 1e-6
    Vp = _gpu_solve(gp, inst, x0=inst.x0 + h * d, eps=1e-12)[2]["V_s0"]
    Vm = _gpu_solve(gp, inst, x0=inst.x0 - h * d, eps=1e-12)[2]["V_s0"]
    fd = (Vp - Vm) / (2 * h)
    # the difference is as exact as its two solves: |error| <~ 1e-12 * cond / h
    check("bwd95_fd", abs(fd - host(gx) @ d) / max(1.0, abs(fd)), 1e-5)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_64_instances_batched_forward_and_adjoints(prec):
    # the differentiation workload: 64 instances of the 95-node tree (shared
    # data, own x0) solved in one batched call (the shared-tree form), then
    # adjoints of instances 0 and 37 against the oracle's stored tangents and
    # of six more with converged, finite gradients (the bench times all 64)
    pr, eps, beps, tol = PREC[prec]
    insts = G.make_batch(5)
    refs = {0: _golden("config5b0_tangents_1e-11"), 37: _golden("config5b37_tangents_1e-11")}
    gp = SP.Problem.from_instance(insts[0], precision=pr, alpha=refs[0]["alpha"])
    x0s = [dev(i.x0, torch.float64) for i in insts]
    vs = [torch.zeros(gp.n_v, dtype=gp.torch_dtype, device="cuda") for _ in insts]
    infos = SP.solve_batched([gp] * len(insts), x0s, vs,
                             SP.default_settings(eps_abs=eps, eps_rel=eps, max_iters=400000))
    assert all(i["status"] == "converged" for i in infos), [i["status"] for i in infos]
    gu = np.random.default_rng(7).standard_normal(insts[0].nu)
    assert all(i["mapping"] == 1024 for i in infos)
    for b, inst in enumerate(insts):
        if b not in (0, 5, 13, 21, 37, 44, 52, 63):
            continue
        gx, gq, _, binfo = gp.backward(vs[b], x0s[b], gV=1.0, gu0=dev(gu, torch.float64),
                                       settings=SP.default_settings(eps_abs=beps, max_iters=400000))
        assert binfo["status"] == "converged", (b, binfo)
        assert np.all(np.isfinite(host(gx))) and np.all(np.isfinite(host(gq)))
        if b in refs:
            for d in refs[b]["dirs"]:
                dirv = _direction(d["kind"], d["seed"], inst)
                want = d["dV"] + gu @ np.array(d["du0"])
                got = host(gx) @ dirv if d["kind"] == "x0" else float(np.sum(host(gq)[1:] * dirv[1:]))
                check(f"bwd64:{b}:{d['kind']}:{prec}", abs(got - want) / max(1.0, abs(want)), tol)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_64_instances_batched_adjoint(prec):
    # spock_backward_batched: all 64 adjoints of the differentiation workload
    # at once (shared-tree sweeps, lockstep GMRES); instances 0 and 37 against
    # the oracle's stored tangents, every instance converged and finite, and
    # eight of them against spock_backward one by one (both converge to the
    # same adjoint: agreement within the adjoint tolerance)
    pr, eps, beps, tol = PREC[prec]
    insts = G.make_batch(5)
    refs = {0: _golden("config5b0_tangents_1e-11"), 37: _golden("config5b37_tangents_1e-11")}
    gp = SP.Problem.from_instance(insts[0], precision=pr, alpha=refs[0]["alpha"])
    x0s = [dev(i.x0, torch.float64) for i in insts]
    vs = [torch.zeros(gp.n_v, dtype=gp.torch_dtype, device="cuda") for _ in insts]
    infos = SP.solve_batched([gp] * len(insts), x0s, vs,
                             SP.default_settings(eps_abs=eps, eps_rel=eps, max_iters=400000))
    assert all(i["status"] == "converged" for i in infos)
    gu = np.random.default_rng(7).standard_normal(insts[0].nu)
    gut = dev(gu, torch.float64)
    st = SP.default_settings(eps_abs=beps, max_iters=400000)
    out = SP.backward_batched(gp, vs, x0s, gV=1.0, gu0s=[gut] * len(insts), settings=st)
    for b, (gx, gq, gqN, bi) in enumerate(out):
        assert bi["status"] == "converged" and bi["mapping"] == 1024, (b, bi)
        assert np.all(np.isfinite(host(gx))) and np.all(np.isfinite(host(gq))) and np.all(np.isfinite(host(gqN)))
    for b, r in refs.items():
        gx, gq = host(out[b][0]), host(out[b][1])
        for d in r["dirs"]:
            dirv = _direction(d["kind"], d["seed"], insts[b])
            want = d["dV"] + gu @ np.array(d["du0"])
            got = gx @ dirv if d["kind"] == "x0" else float(np.sum(gq[1:] * dirv[1:]))
            check(f"bwdb64:{b}:{d['kind']}:{prec}", abs(got - want) / max(1.0, abs(want)), tol)
    for b in (0, 5, 13, 21, 37, 44, 52, 63):
        gx1, gq1, _, bi = gp.backward(vs[b], x0s[b], gV=1.0, gu0=gut, settings=st)
        assert bi["status"] == "converged"
        scale = max(1.0, float(np.max(np.abs(host(gx1)))))
        check(f"bwdb64_vs_single_x0:{b}:{prec}", float(np.max(np.abs(host(out[b][0]) - host(gx1)))) / scale, tol)
        scale = max(1.0, float(np.max(np.abs(host(gq1)))))
        check(f"bwdb64_vs_single_q:{b}:{prec}", float(np.max(np.abs(host(out[b][1]) - host(gq1)))) / scale, tol)


def test_adjoint_falls_back_when_a_dataflow_wait_gives_up(monkeypatch):
    # every bounded wait of the dataflow sweeps gives up at once: the adjoint
    # is redone with the per-stage form and the gradients stay exact
    inst = G.make_random_small(63, [3, 1], 3, 2, a=0.3, box=50.0)
    op = O.Problem(inst)
    ref = O.spock_solve(op, inst.x0, TIGHT)
    g = O.envelope_gradients(op, ref.v)
    gp = SP.Problem.from_instance(inst, precision=SP.FP64, alpha=op.alpha)
    v, x0t, info = _gpu_solve(gp, inst)
    monkeypatch.setenv("SPOCK_TEAM", "512")
    monkeypatch.setenv("SPOCK_FLOW_SPIN", "0")
    gp2 = SP.Problem.from_instance(inst, precision=SP.FP64, alpha=op.alpha)
    gx, _, _, binfo = gp2.backward(v, x0t, gV=1.0)
    assert binfo["flow_fallback"] == 1 and binfo["status"] == "converged", binfo
    check("bwd_giveup", np.max(np.abs(host(gx) - g["x0"])) / max(1.0, np.max(np.abs(g["x0"]))), 1e-6)


def test_autograd_function():
    from paper_2212_01110_amd.autograd import SpockValue
    inst = G.make_random_small(61, [2, 2], 2, 1, a=0.5, box=50.0, ubox=0.8)
    op = O.Problem(inst)
    ref = O.spock_solve(op, inst.x0, TIGHT)
    g = O.envelope_gradients(op, ref.v)
    gp = SP.Problem.from_instance(inst, precision=SP.FP64, alpha=op.alpha)
    x0 = torch.tensor(inst.x0, dtype=torch.float64, device="cuda", requires_grad=True)
    q = torch.tensor(inst.q, dtype=torch.float64, device="cuda", requires_grad=True)
    V, u0 = SpockValue.apply(x0, q, gp)
    assert abs(V.item() - ref.V_s0) <= 1e-8 * max(1, abs(ref.V_s0))
    (V + 0.0 * u0.sum()).backward()
    assert np.max(np.abs(x0.grad.cpu().numpy() - g["x0"])) <= 1e-6 * max(1, np.max(np.abs(g["x0"])))
    assert np.max(np.abs(q.grad.cpu().numpy()[1:] - g["q"][1:])) <= 1e-6 * max(1, np.max(np.abs(g["q"])))


def test_autograd_forward_follows_a_changed_q():
    # the forward pass is a function of the q passed in: after an update of q
    # (as an optimiser step would make) V* and its gradients are those of the
    # new weights, against the oracle factored with them
    from paper_2212_01110_amd.autograd import SpockValue
    inst = G.make_random_small(61, [2, 2], 2, 1, a=0.5, box=50.0, ubox=0.8)
    gp = SP.Problem.from_instance(inst, precision=SP.FP64)
    x0 = torch.tensor(inst.x0, dtype=torch.float64, device="cuda", requires_grad=True)
    q1 = torch.tensor(inst.q, dtype=torch.float64, device="cuda", requires_grad=True)
    V1, _ = SpockValue.apply(x0, q1, gp)
    inst2 = inst.copy()
    inst2.q[1:] *= 1.7
    q2 = torch.tensor(inst2.q, dtype=torch.float64, device="cuda", requires_grad=True)
    V2, u02 = SpockValue.apply(x0, q2, gp)
    op2 = O.Problem(inst2)
    ref2 = O.spock_solve(op2, inst2.x0, TIGHT)
    g2 = O.envelope_gradients(op2, ref2.v)
    assert abs(V2.item() - ref2.V_s0) <= 1e-8 * max(1, abs(ref2.V_s0))
    assert abs(V1.item() - V2.item()) > 1e-3
    V2.backward()
    assert np.max(np.abs(q2.grad.cpu().numpy()[1:] - g2["q"][1:])) <= 1e-6 * max(1, np.max(np.abs(g2["q"])))
    assert np.max(np.abs(x0.grad.cpu().numpy() - g2["x0"])) <= 1e-6 * max(1, np.max(np.abs(g2["x0"])))
