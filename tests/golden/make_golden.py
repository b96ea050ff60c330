"""Writes tests/golden/oracle_refs.json: reference solutions of the seeded
workloads computed by the CPU oracle only (nothing here touches the GPU
path). Run: OMP_NUM_THREADS=1 python tests/golden/make_golden.py [names...]

Entries: V* as s^0 of the returned point and as the exact nested AV@R cost
of its trajectory (eq. original-problem), the first input u^0 (unique since
R > 0), the iteration counts, and the settings used.
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402
import spock_gen as G  # noqa: E402

OUT = os.environ.get("SPOCK_GOLDEN_OUT",
                     os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_refs.json"))


def _entry(res, method, eps, op, dt, **extra):
    out = {"method": method, "eps": eps, "status": res.status, "iters": res.iters,
           "t_evals": res.t_evals, "V_s0": res.V_s0, "V_nested": res.V_nested,
           "u0": res.u0.tolist(), "alpha": op.alpha, "norm_L": op.normL,
           "xi0": res.xi0, "xi": res.xi, "seconds": dt, "counts": res.counts}
    out.update(extra)
    return out


def run(name, inst, method, eps, max_iters=200000):
    op = O.Problem(inst)
    s = O.Settings(eps_abs=eps, eps_rel=eps, max_iters=max_iters)
    t = time.time()
    res = (O.cp_solve if method == "cp" else O.spock_solve)(op, inst.x0, s)
    dt = time.time() - t
    print(f"{name}: {method} eps={eps} {res.status} iters={res.iters} t_evals={res.t_evals} "
          f"V={res.V_nested:.12g} {dt:.1f}s", flush=True)
    return _entry(res, method, eps, op, dt)


def run_chain(name, inst, levels, max_iters=400000):
    """SPOCK to the first tolerance from v = 0, then continued from the
    returned point to each tighter absolute tolerance in turn (a fresh
    Anderson memory at each restart). Returns one entry per level."""
    op = O.Problem(inst)
    out, v0, t0 = {}, None, time.time()
    for k, eps in enumerate(levels):
        s = O.Settings(eps_abs=eps, eps_rel=eps if k == 0 else 0.0, max_iters=max_iters)
        res = O.spock_solve(op, inst.x0, s, v0=v0)
        dt = time.time() - t0
        print(f"{name}: spock chain eps={eps} {res.status} iters={res.iters} V={res.V_nested:.12g} "
              f"{dt:.1f}s", flush=True)
        out[eps] = _entry(res, "spock", eps, op, dt, start="continued" if k else "v=0",
                          chain=[float(e) for e in levels[: k + 1]])
        v0 = res.v
    return out


JOBS = {
    "config1_spock_1e-10": lambda: run("config1", G.make_config(1), "spock", 1e-10),
    "config1_cp_1e-6": lambda: run("config1", G.make_config(1), "cp", 1e-6),
    "config5_spock_1e-5": lambda: run("config5", G.make_config(5), "spock", 1e-5),
    "config2_spock_1e-4": lambda: run("config2", G.make_config(2), "spock", 1e-4),
    "config2_spock_1e-5": lambda: run("config2", G.make_config(2), "spock", 1e-5),
    "config4_b7_spock_1e-6": lambda: run("config4[7]", G.make_batch(4, count=8)[7], "spock", 1e-6),
    "config4_b2_spock_1e-6": lambda: run("config4[2]", G.make_batch(4, count=8)[2], "spock", 1e-6),
    "config4_b5_spock_1e-6": lambda: run("config4[5]", G.make_batch(4, count=8)[5], "spock", 1e-6),
    "datacentre_N7_nx5_cp_1e-5": lambda: run("datacentre", G.make_datacentre(7, 5), "cp", 1e-5),
    "datacentre_N7_nx5_spock_1e-5": lambda: run("datacentre", G.make_datacentre(7, 5), "spock", 1e-5),
}


def tangent_direction(kind, seed, inst):
    """Seeded parameter direction: x0 [nx] or diag Q [nn, nx] (row 0 zero)."""
    rng = np.random.default_rng(seed)
    if kind == "x0":
        return rng.standard_normal(inst.nx)
    d = rng.standard_normal((inst.num_nodes, inst.nx))
    d[0] = 0.0
    return d


def run_tangents(name, inst, eps, dirs):
    """Tight oracle solve, then the fixed-point tangents of V* (= s^0) and
    u^0 along seeded directions of x0 and diag Q (oracle.fixed_point_tangent,
    GMRES on the derivative of T)."""
    op = O.Problem(inst)
    t = time.time()
    res = O.spock_solve(op, inst.x0, O.Settings(eps_abs=eps, eps_rel=eps, max_iters=900000))
    out = {"eps": eps, "alpha": op.alpha, "status": res.status, "xi": res.xi, "V_s0": res.V_s0,
           "u0": res.u0.tolist(), "dirs": []}
    lay = op.lay
    for kind, seed in dirs:
        d = tangent_direction(kind, seed, inst)
        dv = O.fixed_point_tangent(op, res.v, inst.x0, **({"dx0": d} if kind == "x0" else {"dq": d}), tol=1e-11)
        out["dirs"].append({"kind": kind, "seed": seed, "dV": float(dv[0]),
                            "du0": dv[lay.u_off[0]: lay.u_off[0] + lay.nu].tolist()})
        print(f"{name}: tangent {kind} seed {seed} dV={dv[0]:.10g} {time.time() - t:.1f}s", flush=True)
    out["seconds"] = time.time() - t
    return out


JOBS["config5_tangents_1e-11"] = lambda: run_tangents(
    "config5", G.make_config(5), 1e-11, [("x0", 501), ("x0", 502), ("q", 503), ("q", 504)])
# two of the 64 instances of the batched form (same tree and data, own x0)
JOBS["config5b0_tangents_1e-11"] = lambda: run_tangents(
    "config5[0]", G.make_batch(5, count=1)[0], 1e-11, [("x0", 511), ("q", 512)])
JOBS["config5b37_tangents_1e-11"] = lambda: run_tangents(
    "config5[37]", G.make_batch(5, count=38)[37], 1e-11, [("x0", 513), ("q", 514)])

# jobs that write several entries: name -> (function, {key: level})
CHAINS = {
    "config2_chain": (lambda: run_chain("config2", G.make_config(2), [1e-5, 1e-6, 1e-7]),
                      {1e-6: "config2_spock_1e-6", 1e-7: "config2_spock_1e-7"}),
    "config5_chain": (lambda: run_chain("config5", G.make_config(5), [1e-5, 1e-6, 1e-7, 1e-8]),
                      {1e-7: "config5_spock_1e-7", 1e-8: "config5_spock_1e-8"}),
}


def main(names):
    refs = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for n in names or JOBS:
        if n in CHAINS:
            fn, keys = CHAINS[n]
            res = fn()
            for lvl, key in keys.items():
                refs[key] = res[lvl]
        else:
            refs[n] = JOBS[n]()
        with open(OUT, "w") as f:
            json.dump(refs, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:])
