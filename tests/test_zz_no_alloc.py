"""The allocation-free entry point spock_T_noalloc (fixed device scratch)
against spock_T, through the C ABI: two calls in a row on one GPU, the
second on a smaller problem, so the shared scratch array is reused with
different sizes; both compared element by element and on the residual
statistics."""
import numpy as np
import pytest

import paper_2212_01110_amd as SP
import spock_gen as G
from tests.gpu_util import check, dev, host, relerr, seeded

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL = {"fp64": (SP.FP64, 1e-12), "fp32": (SP.FP32, 5e-6)}


@pytest.mark.parametrize("team", ["default", "512"])
@pytest.mark.parametrize("prec", list(TOL))
def test_T_noalloc_matches_T_on_two_calls(prec, team, monkeypatch):
    if team != "default":
        monkeypatch.setenv("SPOCK_TEAM", team)
    pr, tol = TOL[prec]
    # the 223-node tree, then the 15-node tree (a smaller input)
    for cfg in (2, 1):
        inst = G.make_config(cfg)
        gp = SP.Problem.from_instance(inst, precision=pr)
        vt = dev(seeded(f"noalloc{cfg}").standard_normal(gp.n_v), gp.torch_dtype)
        x0 = dev(inst.x0, torch.float64)
        Ta = torch.zeros_like(vt)
        sa = gp.T(vt, x0, Ta)
        Tb = torch.full_like(vt, float("nan"))
        sb = gp.T_noalloc(vt, x0, Tb)
        ref = host(Ta)
        check(f"T_noalloc:{cfg}:{prec}:{team}", relerr(host(Tb), ref), tol)
        for k in ("xi_p", "xi_d", "omega2", "rz2", "re2", "cross"):
            check(f"T_noalloc_stats:{cfg}:{prec}:{team}:{k}", abs(sb[k] - sa[k]) / max(1.0, abs(sa[k])),
                  tol if prec == "fp64" else 2e-6)
