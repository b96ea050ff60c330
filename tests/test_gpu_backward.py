"""GPU parity of spock_backward (implicit differentiation at the fixed point)
against the oracle's envelope gradients and central finite differences."""
import numpy as np
import pytest

import oracle as O
import paper_2212_01110_amd as SP
import spock_gen as G
from tests.gpu_util import dev, host

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TIGHT = O.Settings(eps_abs=1e-12, eps_rel=1e-12, max_iters=500000)


def _gpu_solve(gp, inst, x0=None, eps=1e-11, prec=SP.FP64):
    x0t = dev(inst.x0 if x0 is None else x0, torch.float64)
    v = torch.zeros(gp.n_v, dtype=gp.torch_dtype, device="cuda")
    info = gp.solve(x0t, v, SP.default_settings(eps_abs=eps, eps_rel=eps, max_iters=400000))
    return v, x0t, info


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
    sc = max(1.0, np.max(np.abs(g["x0"])))
    assert np.max(np.abs(host(gx) - g["x0"])) <= 1e-6 * sc, (host(gx), g["x0"])
    sq = max(1.0, np.max(np.abs(g["q"])))
    assert np.max(np.abs(host(gq)[1:] - g["q"][1:])) <= 1e-6 * sq
    lv = op.lay.leaves
    assert np.max(np.abs(host(gqN)[lv] - g["qN"][lv])) <= 1e-6 * max(1.0, np.max(np.abs(g["qN"])))


def test_first_input_gradient_matches_finite_differences():
    inst = G.make_random_small(61, [2, 2], 2, 1, a=0.5, box=50.0, ubox=0.8)
    op = O.Problem(inst)
    gp = SP.Problem.from_instance(inst, precision=SP.FP64, alpha=op.alpha)
    v, x0t, _ = _gpu_solve(gp, inst)
    lay = op.lay
    gu0 = dev(np.ones(inst.nu), torch.float64)
    gx, gq, _, binfo = gp.backward(v, x0t, gV=0.0, gu0=gu0)
    assert binfo["status"] == "converged"
    rng = np.random.default_rng(3)
    d = rng.standard_normal(inst.nx)
    h = 1e-5

    def u0_at(x0):
        vv, _, _ = _gpu_solve(gp, inst, x0=x0, eps=1e-12)
        out = host(vv)
        return out[lay.u_off[0]: lay.u_off[0] + lay.nu].sum()

    fd = (u0_at(inst.x0 + h * d) - u0_at(inst.x0 - h * d)) / (2 * h)
    assert abs(fd - host(gx) @ d) <= 1e-4 * max(1, abs(fd)), (fd, host(gx) @ d)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_config5_gradients_directional_fd(prec):
    inst = G.make_config(5)
    gp64 = SP.Problem.from_instance(inst, precision=SP.FP64)
    gp = gp64 if prec == "fp64" else SP.Problem.from_instance(inst, precision=SP.FP32)
    v, x0t, info = _gpu_solve(gp, inst, eps=1e-10 if prec == "fp64" else 1e-6)
    gx, gq, _, binfo = gp.backward(v, x0t, gV=1.0, settings=SP.default_settings(
        eps_abs=1e-12 if prec == "fp64" else 1e-7, max_iters=400000))
    rng = np.random.default_rng(5)
    d = rng.standard_normal(inst.nx)
    h = 1e-5

    def V_at(x0):
        _, _, inf = _gpu_solve(gp64, inst, x0=x0, eps=1e-11)
        return inf["V_s0"]

    fd = (V_at(inst.x0 + h * d) - V_at(inst.x0 - h * d)) / (2 * h)
    # the central difference itself is only as exact as its two solves:
    # |error| <= eps_V / h with eps_V ~ 1e-11 * cond (xi <= 1e-11), i.e. a few
    # 1e-6 relative at h = 1e-5; the bound below leaves that margin
    tol = 3e-5 if prec == "fp64" else 2e-3
    assert abs(fd - host(gx) @ d) <= tol * max(1, abs(fd)), (fd, host(gx) @ d, binfo)
    # one cost weight (child 3, component 2)
    i3 = inst.copy()
    i4 = inst.copy()
    i3.q[3, 2] += h
    i4.q[3, 2] -= h
    gpa = SP.Problem.from_instance(i3, precision=SP.FP64, alpha=gp64.alpha)
    gpb = SP.Problem.from_instance(i4, precision=SP.FP64, alpha=gp64.alpha)
    fdq = (_gpu_solve(gpa, i3, eps=1e-11)[2]["V_s0"] - _gpu_solve(gpb, i4, eps=1e-11)[2]["V_s0"]) / (2 * h)
    assert abs(fdq - host(gq)[3, 2]) <= tol * max(1, abs(fdq)), (fdq, host(gq)[3, 2])


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
