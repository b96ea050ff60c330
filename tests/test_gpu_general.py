"""GPU parity of general problems: conic risk measures (E, F, b, K) with
nu != 0 (section 4.3), polyhedral constraints and dense cost matrices
(section 4.1), through the C ABI against the oracle: every operator on
identical inputs, ||L||, and converged solutions."""
import numpy as np
import pytest

import oracle as O
import paper_2212_01110_amd as SP
import spock_gen as G
from tests.checks.dense import cut_through
from tests.gpu_util import check, dev, host, relerr, seeded

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

FP = {"fp64": (SP.FP64, 1e-12), "fp32": (SP.FP32, 5e-6)}
STAT = {"fp64": 1e-12, "fp32": 2e-6}


def _active(seed, br, nx, nu, nc):
    loose = G.make_general_small(seed, br, nx, nu, nc=nc, ncN=2)
    res = O.spock_solve(O.Problem(loose), loose.x0, O.Settings(eps_abs=1e-8, eps_rel=1e-8, max_iters=900000))
    return cut_through(loose, res.x, res.u)


def _avar_written_generally():
    inst = G.make_random_small(11, [3, 1, 2], 4, 3)
    gen = inst.copy()
    gen.risk = G.avar_as_conic(inst)
    gen.cons = G.boxes_as_constraints(inst)
    return gen


CASES = {
    "mixture-box": lambda: G.make_general_small(85, [3, 2], 3, 2),
    "mixture-poly": lambda: _active(82, [3, 1], 3, 2, 4),
    "mixture-poly-deep": lambda: _active(84, [2, 2, 1], 2, 2, 5),
    "avar-as-general": _avar_written_generally,
    "mixture-nx20": lambda: G.make_general_small(86, [2, 2, 1, 1], 20, 10, nc=12, ncN=6, bound=3.0),
    # dense Q, R, Q_N (AV@R and boxes otherwise; with general risk and
    # polyhedral rows; n_x = 20 so the roots span several lanes' rows)
    "dense-avar": lambda: G.dense_costs(G.make_random_small(11, [3, 1, 2], 4, 3), seed=21),
    "dense-mixture-poly": lambda: G.dense_costs(_active(82, [3, 1], 3, 2, 4), seed=22),
    "dense-nx20": lambda: G.dense_costs(G.make_random_small(18, [2, 2, 1], 20, 10), seed=23),
}
_INST = {}
_REF = {}


def _inst(name):
    if name not in _INST:
        _INST[name] = CASES[name]()
    return _INST[name]


def _build(inst, prec, alpha=None):
    op = O.Problem(inst) if alpha is None else O.Problem(inst, alpha=alpha)
    gp = SP.Problem.from_instance(inst, precision=FP[prec][0], alpha=op.alpha)
    return gp, op


@pytest.mark.parametrize("prec", list(FP))
@pytest.mark.parametrize("name", list(CASES))
def test_general_operators_match_oracle(name, prec):
    inst = _inst(name)
    gp, op = _build(inst, prec)
    tol = FP[prec][1]
    assert (gp.n_z, gp.n_eta) == (op.lay.n_z, op.lay.n_eta)
    if prec == "fp64":
        check(f"gen_normL:{name}", abs(gp.norm_L - op.normL) / op.normL, 1e-12)
    dt = gp.torch_dtype
    rng = seeded(name + prec)
    z, e = rng.standard_normal(op.lay.n_z), rng.standard_normal(op.lay.n_eta)
    zt, et = dev(z, dt), dev(e, dt)
    eo = torch.zeros(op.lay.n_eta, dtype=dt, device="cuda")
    zo = torch.zeros(op.lay.n_z, dtype=dt, device="cuda")
    gp.apply_L(zt, eo)
    gp.apply_Lt(et, zo)
    check(f"gen_L:{name}:{prec}", relerr(host(eo), O.L_apply(op.lay, inst, host(zt))), tol)
    check(f"gen_Lt:{name}:{prec}", relerr(host(zo), O.Lt_apply(op.lay, inst, host(et))), tol)
    w = dev(3 * rng.standard_normal(op.lay.n_eta), dt)
    out = torch.zeros_like(w)
    gp.prox_gstar(w, out)
    check(f"gen_prox_gstar:{name}:{prec}", relerr(host(out), O.prox_gstar(op.lay, inst, host(w), op.alpha)), tol)
    x0 = dev(inst.x0, torch.float64)
    zf = torch.zeros_like(zt)
    gp.prox_f(zt, x0, zf)
    check(f"gen_prox_f:{name}:{prec}",
          relerr(host(zf), O.prox_f(op.lay, inst, op.fac, host(zt), op.alpha, inst.x0)), tol)
    vt = dev(rng.standard_normal(op.lay.n_v), dt)
    Tv = torch.zeros_like(vt)
    st = gp.T(vt, x0, Tv)
    vin = host(vt)
    ref = O.T_apply(op, vin, inst.x0)
    check(f"gen_T:{name}:{prec}", relerr(host(Tv), ref), tol)
    r = vin - ref
    rs = O.residual_stats(op, r)
    rz, re = op.lay.split(r)
    srel = STAT[prec]
    xp, xd = np.max(np.abs(rs["xi_p"])), np.max(np.abs(rs["xi_d"]))
    check(f"gen_xi_p:{name}:{prec}", abs(st["xi_p"] - xp) / max(1, xp), srel)
    check(f"gen_xi_d:{name}:{prec}", abs(st["xi_d"] - xd) / max(1, xd), srel)
    check(f"gen_omega2:{name}:{prec}", abs(st["omega2"] - r @ O.M_apply(op, r)) / max(1, r @ r), srel)


@pytest.mark.parametrize("mapping", ["8", "256", "512"])
@pytest.mark.parametrize("name", ["mixture-poly", "mixture-nx20"])
def test_general_T_every_sweep_mapping(name, mapping, monkeypatch):
    # the general pre/post passes with each form of the shared sweeps
    monkeypatch.setenv("SPOCK_TEAM", mapping)
    inst = _inst(name)
    gp, op = _build(inst, "fp64")
    vt = dev(seeded(name + mapping).standard_normal(op.lay.n_v), torch.float64)
    x0 = dev(inst.x0, torch.float64)
    Tv = torch.zeros_like(vt)
    gp.T(vt, x0, Tv)
    check(f"gen_T_map:{name}:{mapping}", relerr(host(Tv), O.T_apply(op, host(vt), inst.x0)), 1e-12)


@pytest.mark.parametrize("prec", list(FP))
@pytest.mark.parametrize("name", ["mixture-box", "mixture-poly", "mixture-poly-deep", "dense-avar",
                                  "dense-mixture-poly"])
def test_general_solve_matches_oracle(name, prec):
    inst = _inst(name)
    gp, op = _build(inst, prec)
    if name not in _REF:
        _REF[name] = O.spock_solve(op, inst.x0, O.Settings(eps_abs=1e-10, eps_rel=1e-10, max_iters=900000))
    ref = _REF[name]
    x0 = dev(inst.x0, torch.float64)
    v = torch.zeros(gp.n_v, dtype=gp.torch_dtype, device="cuda")
    eps = 1e-9 if prec == "fp64" else 1e-5
    # FP64: the residual bound times a modest condition number; FP32 stops at
    # a 1e-5 residual, and the polyhedral cases are ill-conditioned (the
    # oracle itself needs ~1e4 iterations), so the solution error is ~1e-4
    tol = 1e-6 if prec == "fp64" else 5e-4
    info = gp.solve(x0, v, SP.default_settings(eps_abs=eps, eps_rel=eps, max_iters=900000))
    assert info["status"] == "converged", info
    check(f"gen_solve_V:{name}:{prec}", abs(info["V_s0"] - ref.V_s0) / max(1, abs(ref.V_s0)), tol)
    out = host(v)
    u0 = out[op.lay.u_off[0]: op.lay.u_off[0] + op.lay.nu]
    check(f"gen_solve_u0:{name}:{prec}", np.max(np.abs(u0 - ref.u0)) / max(1, np.max(np.abs(ref.u0))), tol)


def test_dense_costs_rotation_invariance():
    # x' = U x, u' = W u with U, W orthogonal maps a problem with diagonal
    # costs onto one with dense costs and the same optimal value, u0' = W u0
    # (inactive boxes: they are not invariant); the diagonal problem runs
    # the special-form kernels, the rotated one the general kernels
    base = G.make_random_small(17, [3, 2], 5, 3)
    big = 1e6
    base.xmin[:], base.xmax[:], base.umin[:], base.umax[:] = -big, big, -big, big
    rng = np.random.default_rng(5)
    U = np.linalg.qr(rng.standard_normal((base.nx, base.nx)))[0]
    W = np.linalg.qr(rng.standard_normal((base.nu, base.nu)))[0]
    rot = G.rotate_states_inputs(base, U, W)
    st = SP.default_settings(eps_abs=1e-10, eps_rel=1e-10, max_iters=900000)
    out = {}
    for name, inst in (("diag", base), ("rot", rot)):
        gp = SP.Problem.from_instance(inst, precision=SP.FP64)
        v = torch.zeros(gp.n_v, dtype=torch.float64, device="cuda")
        info = gp.solve(dev(inst.x0, torch.float64), v, st)
        assert info["status"] == "converged", (name, info)
        lay = O.Problem(inst).lay
        out[name] = (info["V_s0"], host(v)[lay.u_off[0]: lay.u_off[0] + lay.nu])
    (Vd, ud), (Vr, ur) = out["diag"], out["rot"]
    check("dense_rot_V", abs(Vr - Vd) / max(1, abs(Vd)), 1e-7)
    check("dense_rot_u0", np.max(np.abs(ur - W @ ud)) / max(1, np.max(np.abs(ud))), 1e-5)


def test_dense_costs_rejected_by_factor():
    inst = G.dense_costs(G.make_random_small(11, [3, 1, 2], 4, 3), seed=21)
    bad = inst.copy()
    bad.Qm = inst.Qm.copy()
    bad.Qm[2] -= 3.0 * np.eye(inst.nx)              # indefinite
    with pytest.raises(SP.SpockError) as e:
        SP.Problem.from_instance(bad)
    assert e.value.code == -1


def test_general_problems_rejected_where_unsupported():
    inst = _inst("mixture-box")
    gp, _ = _build(inst, "fp64")
    x0 = dev(inst.x0, torch.float64)
    v = torch.zeros(gp.n_v, dtype=torch.float64, device="cuda")
    with pytest.raises(SP.SpockError) as e:
        SP.solve_batched([gp], [x0], [v], SP.default_settings())
    assert e.value.code == -8
    with pytest.raises(SP.SpockError) as e:
        gp.backward(v, x0, gV=1.0)
    assert e.value.code == -8
