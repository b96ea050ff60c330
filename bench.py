"""Benchmark of the SPOCK hot path on one MI355X.

Headline workload: the 20 776-node scenario tree (n_x = 50, n_u = 20,
N = 15, branching 3 for 7 stages, 2187 scenarios), FP32 bulk iterations with
FP64 factorisation, Anderson solve and residual statistics. A step is one
SPOCK iteration (Alg. 3): the evaluations of the CP operator T (pre-pass,
both Alg. 2 sweeps, dual update, residual statistics), the Anderson
Gram/direction kernels and the SuperMann line search. K steps are timed as
one solve capped at K iterations from a cold start (v = 0); value = T
evaluations per second (= CP iterations = calls of L, the paper's count).

roofline: the dominant kernel (the sweeps of T, one launch per evaluation in
the dataflow form) timed with HIP events recorded by the library on its own
stream, against the algorithmic bytes of the sweeps as the method states them
(every factor matrix once per sweep that uses it, q and d written and read
once); the whole T (those plus v read and T(v) written) beside it.
cpu_baseline: the FP64 oracle, single-threaded, on a bounded number of T
evaluations of the same workload.

The same JSON line carries the other legs of the metric, each measured:
  tree20776_fp64            the headline workload in FP64 bulk
  tree20776_residual_budget ξ reached from a cold start within a stated
                            iteration budget (FP32 and FP64), with ξ0
  time_to_residual_223node  SPOCK to ξ <= max(1e-4, 1e-4 ξ0), FP64 and FP32
  time_to_residual_512batch 512 uneven trees from perturbed warm starts:
                            batched FP32 and FP64 launches against the plain
                            FP64 path solving every instance one by one
  fp32_error_vs_oracle      FP32 bulk against stored oracle solutions (V*, u^0)
                            and its residual floor
  datacentre_cp_vs_spock    the paper's section-6 comparison (N 7, n_x 5,
                            eps 1e-5): T evaluations of CP and SPOCK on the GPU
  datacentre_scaling        the paper's open-loop series (n_x = n_u = 50,
                            N = 3..15, eps 1e-3), SPOCK in FP32 and FP64
  datacentre_closed_loop_mpc the paper's closed-loop simulation (N 10,
                            n_x = n_u = 20, 20 steps, 15 realisations), warm
                            against cold starts
  differentiation_64_instances 64 instances of the 95-node tree sharing its
                            data: forward by the shared-tree (MFMA) form and
                            all 64 adjoint gradients in one batched call (by
                            default); with --legs diff64 (or all) also the
                            block engine, the forward one by one and the
                            adjoints one by one
  shared_forward_64_instances (only when asked: --legs shared64) one FP32
                            forward of that workload by the shared-tree form
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "time-to-residual-1e-4 & CP iters/s, batched FP32 vs plain FP64; achieved HBM GB/s"
HBM_PEAK_GBS = 8000.0
NAMES = {1: "15-node binary tree nx2 nu1 N3 (AV@R a=0.5)",
         2: "223-node tree nx20 nu10 N10 (branching 2 for 5 stages)",
         3: "20776-node tree nx50 nu20 N15 (branching 3 for 7 stages, 2187 scenarios)",
         5: "95-node tree nx20 nu10 N8 (branching 2 for 4 stages)"}
# the paper's own figures (sequential Julia, CPU and precision not stated), as context
PAPER_SCALING_S = {3: 0.0299, 6: 0.285, 9: 2.43, 12: 22.9, 14: 78.3, 15: 151.5}
PAPER_SCALING_ITERS = {3: 105, 6: 128, 9: 110, 12: 109, 15: 105}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def tree_counts(inst):
    anc = np.asarray(inst.anc)
    nn = anc.shape[0]
    nch = np.bincount(anc[1:], minlength=nn)
    nl = int(np.sum(nch > 0))
    return nn, nl, nn - nl


def sizes(inst):
    nn, nl, nleaf = tree_counts(inst)
    nx, nu = inst.nx, inst.nu
    n_z = 1 + nn * nx + nl * nu + 4 * (nn - 1) + nl
    n_eta = 2 * (nn - 1) + 2 * nl + nl * (nx + nu) + (nn - 1) * (nx + nu + 2) + nleaf * (2 * nx + 2)
    return n_z, n_eta


def algorithmic_elems_sweeps(inst):
    """Elements both Alg. 2 sweeps must move as the method states them: every
    factor matrix once per sweep that uses it (Abar and B per child in both
    sweeps, K per family in both, R~^{-1} and W per family in the backward
    sweep), and q and d written once and read once."""
    nn, nl, _ = tree_counts(inst)
    nx, nu = inst.nx, inst.nu
    mats = (nn - 1) * (2 * nx * nx + 2 * nx * nu) + nl * (2 * nu * nx + nu * nu + nx * nu)
    return int(mats + 2 * (nn * nx + nl * nu))


def algorithmic_elems_sweeps_regrouped(inst):
    """The same for the regrouped backward step the sweeps kernel computes
    (At, Bt per child and R~^{-1}, P1 per family backward; Abar, B per child
    and K per family forward) with its vector traffic."""
    nn, nl, _ = tree_counts(inst)
    nx, nu = inst.nx, inst.nu
    mats = 2 * (nn - 1) * (nx * nx + nx * nu) + nl * (2 * nx * nu + nu * nu)
    bwd_vec = nl * (nx + nu) + nl * (nx + nu) + (nn - 1) * nx
    fwd_vec = nl * (nu + nx) + nl * nu + (nn - 1) * nx
    return int(mats + bwd_vec + fwd_vec)


def algorithmic_elems_T(inst):
    """One whole T: the sweeps plus v read once and T(v) written once."""
    n_z, n_eta = sizes(inst)
    return algorithmic_elems_sweeps(inst) + 2 * (n_z + n_eta)


def measured_traffic():
    """HBM bytes per launch of the sweeps kernel from the committed counter
    summary (rocprofv3 FETCH_SIZE / WRITE_SIZE, scaled by a plain copy), or
    None when the kernel sources differ from those the counters were taken
    on."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "k_T_flow_20776node_fp32_traffic.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    b = re.search(r"traffic_bytes_per_launch: (\d+)", txt)
    h = re.search(r"kernel_sources_sha256_16: ([0-9a-f]+)", txt)
    if not b or not h:
        return None
    sha = hashlib.sha256()
    for f in ("flow.hip", "device_common.h", "spock_internal.h"):
        sha.update(open(os.path.join(ROOT, "paper_2212_01110_amd", "csrc", f), "rb").read())
    return int(b.group(1)) if sha.hexdigest()[:16] == h.group(1) else None


def cpu_baseline(inst, alpha, budget_s):
    """FP64 oracle: T evaluations with residual statistics from v = 0 until
    the time budget is spent, on one thread (the oracle walks the tree node
    by node; BLAS is limited to one thread for its small products)."""
    import oracle as O
    from oracle.layout import Layout
    from threadpoolctl import threadpool_limits

    class _P:
        pass
    p = _P()
    p.inst, p.lay = inst, Layout(inst)
    with threadpool_limits(limits=1):
        p.fac = O.factor_s1(p.lay, inst)
        p.alpha = alpha
        v = np.zeros(p.lay.n_v)
        n = 0
        t0 = time.perf_counter()
        while True:
            Tv = O.T_apply(p, v, inst.x0)
            O.residual_stats(p, v - Tv)
            v = Tv
            n += 1
            el = time.perf_counter() - t0
            if el >= budget_s or n >= 1000:
                break
    return {"value": round(n / el, 4), "unit": "CP iters/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} evaluations of T with residual statistics (FP64 numpy, one thread) on the "
                      f"same workload from v=0, {el:.1f} s"}


def timed_solve(torch, gp, x0, v, settings):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = gp.solve(x0, v, settings)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, info


def roofline_of(prof, inst, itemsize):
    e_sw = algorithmic_elems_sweeps(inst)
    e_T = algorithmic_elems_T(inst)
    ach = e_sw * itemsize / (prof["sweeps"] * 1e-6) / 1e9
    ach_T = e_T * itemsize / (prof["total"] * 1e-6) / 1e9
    return {"achieved": round(ach, 1), "frac": round(ach / HBM_PEAK_GBS, 4),
            "bytes_per_launch": e_sw * itemsize, "us_per_launch": round(prof["sweeps"], 2),
            "T_phases_us": {k: round(x, 2) for k, x in prof.items()},
            "T_whole_algorithmic_bytes": e_T * itemsize,
            "T_whole_GBps": round(ach_T, 1), "T_whole_frac": round(ach_T / HBM_PEAK_GBS, 4),
            "regrouped_bytes_per_launch": algorithmic_elems_sweeps_regrouped(inst) * itemsize}


def leg_fp64(torch, SP, inst, steps, reps):
    """The headline workload in FP64 bulk: T evaluations/s over the same
    capped solve and the phase timing."""
    gp = SP.Problem.from_instance(inst, precision=SP.FP64)
    x0 = torch.as_tensor(inst.x0, dtype=torch.float64, device="cuda")
    v = torch.zeros(gp.n_v, dtype=torch.float64, device="cuda")
    gp.solve(x0, v, SP.default_settings(max_iters=5))
    v.zero_()
    sec, info = timed_solve(torch, gp, x0, v, SP.default_settings(max_iters=steps))
    prof = gp.profile_T(v, x0, torch.empty_like(v), reps=reps)
    out = {"value": round(info["t_evals"] / sec, 2), "unit": "CP iters/s", "steps": info["iters"],
           "t_evals": info["t_evals"], "seconds": round(sec, 4), "mapping": info["mapping"]}
    out.update(roofline_of(prof, inst, 8))
    log(f"20776-node FP64: {out['value']} T/s, sweeps {out['achieved']} GB/s")
    return out, gp


def leg_budget(torch, SP, inst, gps, iters):
    """SPOCK from v = 0 for at most `iters` iterations, FP32 and FP64: the
    residual reached against the target max(1e-4, 1e-4 xi0)."""
    out = {"workload": NAMES[3], "iteration_budget": iters}
    x0 = torch.as_tensor(inst.x0, dtype=torch.float64, device="cuda")
    for name, gp in gps.items():
        v = torch.zeros(gp.n_v, dtype=gp.torch_dtype, device="cuda")
        sec, info = timed_solve(torch, gp, x0, v, SP.default_settings(max_iters=iters))
        tgt = max(1e-4, 1e-4 * info["xi0"])
        out[name] = {"seconds": round(sec, 3), "iters": info["iters"], "t_evals": info["t_evals"],
                     "xi0": info["xi0"], "xi": info["xi"], "target": tgt,
                     "reached": info["status"] == "converged", "V_s0": info["V_s0"],
                     "counts": {k: info[k] for k in ("n_k0", "n_k1", "n_k2", "n_km", "n_backtracks")}}
        log(f"20776-node {name} budget: xi {info['xi0']:.4g} -> {info['xi']:.4g} in {sec:.2f}s")
    # Anderson memory within the paper's range (section 6.2: 3 to 10), FP32
    gp = gps.get("fp32")
    if gp is not None:
        out["fp32_by_memory"] = {}
        for m in (5, 10):
            v = torch.zeros(gp.n_v, dtype=gp.torch_dtype, device="cuda")
            sec, info = timed_solve(torch, gp, x0, v, SP.default_settings(max_iters=iters, m=m))
            its = max(1, info["iters"])
            out["fp32_by_memory"][m] = {"seconds": round(sec, 3), "iters": info["iters"],
                                        "t_evals": info["t_evals"], "xi": info["xi"],
                                        "k2_share": round(info["n_k2"] / its, 3)}
            log(f"20776-node fp32 budget m={m}: xi -> {info['xi']:.4g} in {sec:.2f}s")
    return out


def ttr_single(torch, SP, G):
    """223-node tree: SPOCK to xi <= 1e-4 from v = 0, FP64 and FP32 bulk."""
    inst = G.make_config(2)
    out = {"workload": NAMES[2]}
    x0 = torch.as_tensor(inst.x0, dtype=torch.float64, device="cuda")
    s = SP.default_settings(max_iters=200000)
    ref_V = None
    for name, prec in (("fp64", SP.FP64), ("fp32", SP.FP32)):
        gp = SP.Problem.from_instance(inst, precision=prec)
        v = torch.zeros(gp.n_v, dtype=gp.torch_dtype, device="cuda")
        gp.solve(x0, v, SP.default_settings(max_iters=5))  # mapping autotuned outside the timing
        v.zero_()
        sec, info = timed_solve(torch, gp, x0, v, s)
        if ref_V is None:
            ref_V = info["V_s0"]
        out[name] = {"seconds": round(sec, 4), "iters": info["iters"], "t_evals": info["t_evals"],
                     "status": info["status"], "xi": info["xi"], "V_s0": info["V_s0"],
                     "V_rel_err_vs_fp64": abs(info["V_s0"] - ref_V) / max(1.0, abs(ref_V)),
                     "mapping": info["mapping"]}
        log(f"223-node {name}: {info['status']} {info['iters']} iters {sec:.3f}s")
        if name == "fp64":  # Anderson memory within the paper's range (section 6.2)
            out["fp64_by_memory"] = {}
            for m in (5, 10):
                v.zero_()
                sec, info = timed_solve(torch, gp, x0, v, SP.default_settings(max_iters=200000, m=m))
                its = max(1, info["iters"])
                out["fp64_by_memory"][m] = {"seconds": round(sec, 4), "iters": info["iters"],
                                            "t_evals": info["t_evals"], "status": info["status"],
                                            "k2_share": round(info["n_k2"] / its, 3)}
                log(f"223-node fp64 m={m}: {info['status']} {info['iters']} iters {sec:.3f}s")
    return out


def ttr_batched(torch, SP, G, keep=None):
    """512 uneven instances: warm start = FP64 solution + N(0, 0.05^2) on
    every entry (seeded); batched FP32 and FP64 (one persistent graph-captured
    launch each), and mixed (FP32 to 1e-3, then FP64 from there), vs the
    plain FP64 path solving every instance one by one from the same warm
    starts."""
    insts = G.make_batch(4, count=512)
    x0s = [torch.as_tensor(i.x0, dtype=torch.float64, device="cuda") for i in insts]
    p64 = [SP.Problem.from_instance(i, precision=SP.FP64) for i in insts]
    p32 = [SP.Problem.from_instance(i, precision=SP.FP32) for i in insts]
    if keep is not None:
        keep["p32_512"] = p32
    v64 = [torch.zeros(p.n_v, dtype=torch.float64, device="cuda") for p in p64]
    log("512-batch problems factored")
    t0 = time.perf_counter()
    SP.solve_batched(p64, x0s, v64, SP.default_settings(eps_abs=1e-5, eps_rel=1e-5, max_iters=5000))
    torch.cuda.synchronize()
    log(f"512-batch FP64 previous solutions {time.perf_counter() - t0:.2f}s")
    rng = np.random.default_rng(2024)
    warm = [v + torch.as_tensor(rng.normal(0.0, 0.05, v.numel()), device="cuda") for v in v64]
    s = SP.default_settings(max_iters=200000)
    res = {}
    for name, probs, dt in (("fp32", p32, torch.float32), ("fp64", p64, torch.float64)):
        vb = [w.to(dt, copy=True) for w in warm]  # the solves overwrite their starts
        SP.solve_batched(probs, x0s, [x.clone() for x in vb], SP.default_settings(max_iters=5))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = SP.solve_batched(probs, x0s, vb, s)
        torch.cuda.synchronize()
        res[name] = (time.perf_counter() - t0, infos)
        log(f"512-batch {name} warm {res[name][0]:.3f}s")
    # mixed precision: the FP32 batch to a loose 1e-3 (at most 3000
    # iterations, above the FP32 residual floor of most trees), then the
    # FP64 batch from those points to the target
    vb = [w.to(torch.float32, copy=True) for w in warm]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    i_lo = SP.solve_batched(p32, x0s, vb, SP.default_settings(eps_abs=1e-3, eps_rel=1e-3, max_iters=3000))
    vb = [x.to(torch.float64) for x in vb]
    i_mix = SP.solve_batched(p64, x0s, vb, s)
    torch.cuda.synchronize()
    t_mix = time.perf_counter() - t0
    log(f"512-batch mixed FP32 -> FP64 {t_mix:.3f}s")
    # plain FP64, every instance one by one from the same warm starts
    t_plain, iters_plain, infos_plain = 0.0, [], []
    for b in range(512):
        p64[b].solve(x0s[b], warm[b].clone(), SP.default_settings(max_iters=3))  # mapping tuned, untimed
        sec, info = timed_solve(torch, p64[b], x0s[b], warm[b].clone(), s)
        t_plain += sec
        iters_plain.append(info["iters"])
        infos_plain.append(info)
        if b % 128 == 127:
            log(f"plain FP64: {b + 1} of 512 instances, {t_plain:.2f}s")
    log(f"plain FP64 all 512 {t_plain:.3f}s")
    # reference values on a sample of 16 instances: plain FP64 solved to 1e-8
    sample = np.linspace(0, 511, 16).astype(int)
    tight = {}
    for k, b in enumerate(sample):
        tight[b] = p64[b].solve(x0s[b], warm[b].clone(), SP.default_settings(eps_abs=1e-8, eps_rel=1e-8,
                                                                             max_iters=200000))
        if k % 8 == 7:
            log(f"512-batch FP64 references to 1e-8: {k + 1} of 16")
    i32, i64 = res["fp32"][1], res["fp64"][1]
    rel = lambda a, b: abs(a["V_s0"] - b["V_s0"]) / max(1.0, abs(b["V_s0"]))  # noqa: E731
    return {"workload": "512 uneven trees nx10 nu5 N 5..12 (warm start, sigma 0.05)",
            "batched_fp32_seconds": round(res["fp32"][0], 4),
            "batched_fp32_converged": sum(i["status"] == "converged" for i in i32),
            "batched_fp32_iters_median_max": [int(np.median([i["iters"] for i in i32])), max(i["iters"] for i in i32)],
            "batched_fp64_seconds": round(res["fp64"][0], 4),
            "batched_fp64_iters_median_max": [int(np.median([i["iters"] for i in i64])), max(i["iters"] for i in i64)],
            "plain_fp64_seconds": round(t_plain, 3),
            "plain_fp64_iters_median_max": [int(np.median(iters_plain)), max(iters_plain)],
            "plain_fp64_converged": sum(i["status"] == "converged" for i in infos_plain),
            "V_rel_err_reference": "16 of the 512 instances (evenly spaced) solved by the plain FP64 path to 1e-8",
            "V_max_rel_err_batched_fp32": max(rel(i32[b], tight[b]) for b in sample),
            "V_max_rel_err_batched_fp64": max(rel(i64[b], tight[b]) for b in sample),
            "V_max_rel_err_plain_fp64": max(rel(infos_plain[b], tight[b]) for b in sample),
            "batched_mixed_seconds": round(t_mix, 4),
            "batched_mixed_fp32_iters_median_max": [int(np.median([i["iters"] for i in i_lo])),
                                                    max(i["iters"] for i in i_lo)],
            "batched_mixed_fp64_iters_median_max": [int(np.median([i["iters"] for i in i_mix])),
                                                    max(i["iters"] for i in i_mix)],
            "batched_mixed_converged": sum(i["status"] == "converged" for i in i_mix),
            "V_max_rel_err_batched_mixed": max(rel(i_mix[b], tight[b]) for b in sample),
            "speedup_batched_fp32_vs_plain_fp64": round(t_plain / res["fp32"][0], 2),
            "speedup_batched_fp64_vs_plain_fp64": round(t_plain / res["fp64"][0], 2),
            "speedup_batched_mixed_vs_plain_fp64": round(t_plain / t_mix, 2)}


def _golden():
    path = os.path.join(ROOT, "tests", "golden", "oracle_refs.json")
    return json.load(open(path)) if os.path.exists(path) else {}


def leg_fp32_error(torch, SP, G, keep=None):
    """FP32 bulk against the FP64 oracle per result (stored oracle solutions,
    tests/golden): V* and u^0 of the 223-node tree and of three of the 512
    trees, each solved in FP32 to 1e-5; and the FP32 residual floor: the
    smallest xi an FP32 solve reaches when asked for 1e-9 (223-node tree;
    the 512 trees in one batched launch)."""
    refs = _golden()
    out = {}
    rel = lambda a, b: abs(a - b) / max(1.0, abs(b))  # noqa: E731

    def u0_of(v, inst):
        h = v.detach().double().cpu().numpy()
        off = 1 + inst.num_nodes * inst.nx
        return h[off: off + inst.nu]
    key2 = "config2_spock_1e-7" if "config2_spock_1e-7" in refs else "config2_spock_1e-5"
    inst = G.make_config(2)
    x0 = torch.as_tensor(inst.x0, dtype=torch.float64, device="cuda")
    gp = SP.Problem.from_instance(inst, precision=SP.FP32, alpha=refs[key2]["alpha"])
    v = torch.zeros(gp.n_v, dtype=torch.float32, device="cuda")
    info = gp.solve(x0, v, SP.default_settings(eps_abs=1e-5, eps_rel=1e-5, max_iters=400000, compute_nested=1))
    u0r = np.array(refs[key2]["u0"])
    out["tree223"] = {"reference": key2, "status": info["status"],
                      "V_rel_err": rel(info["V_nested"], refs[key2]["V_nested"]),
                      "u0_rel_err": float(np.max(np.abs(u0_of(v, inst) - u0r)) / max(1.0, np.max(np.abs(u0r))))}
    v.zero_()
    info = gp.solve(x0, v, SP.default_settings(eps_abs=1e-9, eps_rel=1e-9, max_iters=40000))
    out["tree223"]["fp32_floor_xi"] = info["xi"]
    out["tree223"]["fp32_floor_iters"] = info["iters"]
    insts = G.make_batch(4, count=8)
    rows = {}
    for b in (2, 5, 7):
        key = f"config4_b{b}_spock_1e-6"
        if key not in refs:
            continue
        gpb = SP.Problem.from_instance(insts[b], precision=SP.FP32, alpha=refs[key]["alpha"])
        xb = torch.as_tensor(insts[b].x0, dtype=torch.float64, device="cuda")
        vb = torch.zeros(gpb.n_v, dtype=torch.float32, device="cuda")
        ib = gpb.solve(xb, vb, SP.default_settings(eps_abs=1e-5, eps_rel=1e-5, max_iters=400000,
                                                   compute_nested=1))
        u0r = np.array(refs[key]["u0"])
        rows[b] = {"V_rel_err": rel(ib["V_nested"], refs[key]["V_nested"]),
                   "u0_rel_err": float(np.max(np.abs(u0_of(vb, insts[b]) - u0r)) / max(1.0, np.max(np.abs(u0r))))}
    out["trees512_sample"] = rows
    # floor of the batch: FP32 batched launch asked for 1e-9 from v = 0
    insts = G.make_batch(4, count=512)
    p32 = (keep or {}).get("p32_512") or [SP.Problem.from_instance(i, precision=SP.FP32) for i in insts]
    x0s = [torch.as_tensor(i.x0, dtype=torch.float64, device="cuda") for i in insts]
    vs = [torch.zeros(p.n_v, dtype=torch.float32, device="cuda") for p in p32]
    infos = SP.solve_batched(p32, x0s, vs, SP.default_settings(eps_abs=1e-9, eps_rel=1e-9, max_iters=4000))
    xs = np.array([i["xi"] for i in infos])
    out["trees512_fp32_floor_xi"] = {"median": float(np.median(xs)), "p90": float(np.percentile(xs, 90)),
                                     "max": float(xs.max()), "iteration_cap": 4000}
    log(f"FP32 errors: {out}")
    return out


def leg_datacentre(torch, SP, G):
    """Section 6 first experiment: the data-centre model (N 7, n_x 5, binary
    tree, a 0.95), CP and SPOCK in FP64 to eps_abs = eps_rel = 1e-5."""
    inst = G.make_datacentre(7, 5)
    gp = SP.Problem.from_instance(inst, precision=SP.FP64)
    x0 = torch.as_tensor(inst.x0, dtype=torch.float64, device="cuda")
    out = {"workload": "data-centre model N7 nx5 (255 nodes), eps 1e-5, FP64",
           "paper_L_calls": {"cp": 3159, "spock": 571}}
    for method in ("cp", "spock"):
        v = torch.zeros(gp.n_v, dtype=torch.float64, device="cuda")
        gp.solve(x0, v.clone(), SP.default_settings(max_iters=3, method=method))
        sec, info = timed_solve(torch, gp, x0, v, SP.default_settings(eps_abs=1e-5, eps_rel=1e-5,
                                                                      max_iters=200000, method=method))
        out[method] = {"t_evals": info["t_evals"], "iters": info["iters"], "seconds": round(sec, 4),
                       "status": info["status"], "V_s0": info["V_s0"]}
    out["t_evals_ratio_cp_over_spock"] = round(out["cp"]["t_evals"] / out["spock"]["t_evals"], 3)
    # Anderson memory within the paper's range (3 to 10; QR-updated above 4)
    out["spock_by_memory"] = {}
    for m in (1, 3, 5, 10):
        v = torch.zeros(gp.n_v, dtype=torch.float64, device="cuda")
        sec, info = timed_solve(torch, gp, x0, v, SP.default_settings(eps_abs=1e-5, eps_rel=1e-5,
                                                                      max_iters=200000, m=m))
        out["spock_by_memory"][m] = {"t_evals": info["t_evals"], "iters": info["iters"],
                                     "k2_share": round(info["n_k2"] / max(1, info["iters"]), 3),
                                     "seconds": round(sec, 4), "status": info["status"]}
    log(f"datacentre N7: CP {out['cp']['t_evals']} vs SPOCK {out['spock']['t_evals']} T evaluations")
    return out


def leg_scaling(torch, SP, G, horizons):
    """Section 6 open-loop series: data-centre model with n_x = n_u = 50,
    binary tree of horizon N, SPOCK to eps 1e-3 from v = 0, FP32 and FP64."""
    out = {"workload": "data-centre model nx=nu=50, binary tree, N = " + ",".join(map(str, horizons)) +
           ", SPOCK eps 1e-3 from v=0",
           "paper_seconds_context": PAPER_SCALING_S, "paper_iters_context": PAPER_SCALING_ITERS,
           "paper_hardware": "sequential Julia, CPU and precision not stated", "runs": []}
    for N in horizons:
        inst = G.make_datacentre(N, 50)
        x0 = torch.as_tensor(inst.x0, dtype=torch.float64, device="cuda")
        row = {"N": N, "nodes": int(inst.num_nodes)}
        for name, prec in (("fp32", SP.FP32), ("fp64", SP.FP64)):
            gp = SP.Problem.from_instance(inst, precision=prec)
            v = torch.zeros(gp.n_v, dtype=gp.torch_dtype, device="cuda")
            gp.solve(x0, v, SP.default_settings(max_iters=3))
            v.zero_()
            sec, info = timed_solve(torch, gp, x0, v, SP.default_settings(eps_abs=1e-3, eps_rel=1e-3,
                                                                          max_iters=20000))
            row[name] = {"seconds": round(sec, 4), "iters": info["iters"], "t_evals": info["t_evals"],
                         "status": info["status"], "V_s0": info["V_s0"], "mapping": info["mapping"]}
            del gp, v
            torch.cuda.empty_cache()
        log(f"datacentre N{N}: fp32 {row['fp32']['seconds']}s ({row['fp32']['iters']} it), "
            f"fp64 {row['fp64']['seconds']}s ({row['fp64']['iters']} it)")
        out["runs"].append(row)
    return out


def leg_mpc(torch, SP, G, steps=20, realisations=15):
    """Section 6 closed-loop simulation: data-centre model N 10,
    n_x = n_u = 20 (2047 nodes), x0 = 0.1 * 1, eps 1e-3, 20 steps for 15
    seeded realisations of the disturbance (branch w = 2 with probability
    0.7), all realisations in one batched launch per step; warm starts from
    the previous step's solution against cold starts."""
    from paper_2212_01110_amd.mpc import closed_loop
    inst = G.make_datacentre(10, 20)
    out = {"workload": "data-centre model N10 nx=nu=20 (2047 nodes), eps 1e-3, "
                       f"{steps} steps x {realisations} realisations, FP64, batched per step"}
    gp = SP.Problem.from_instance(inst, precision=SP.FP64)
    branches = (np.random.default_rng(2023).random((realisations, steps)) < 0.7).astype(int)
    s = SP.default_settings(eps_abs=1e-3, eps_rel=1e-3, max_iters=200000)
    for name, warm in (("warm", True), ("cold", False)):
        res = closed_loop(gp, inst.A[1:3], inst.B[1:3], inst.x0, branches, s, warm=warm,
                          progress=lambda t, sec: log(f"mpc {name} step {t}: {sec:.3f}s"))
        out[name] = {"seconds_per_step": [round(x, 4) for x in res["step_seconds"]],
                     "mean_t_evals_per_step": [round(float(x), 1) for x in res["t_evals"].mean(axis=0)],
                     "total_seconds": round(float(res["step_seconds"].sum()), 3),
                     "all_converged": all(st == "converged" for row in res["status"] for st in row)}
        log(f"mpc {name}: {out[name]['total_seconds']}s, T evals per step {out[name]['mean_t_evals_per_step'][:4]}")
    return out


def leg_diff64(torch, SP, G, full=True):
    """The differentiation workload: 64 instances of the 95-node tree (n_x 20,
    n_u 10, N 8, branching 2 for 4 stages; shared tree and data, own x0).
    Forward in FP32 to eps 1e-5 three ways: the shared-tree form (one call,
    instances in lockstep, Alg. 2 sweeps as 16-instance MFMA tiles), the
    per-instance block engine (SPOCK_SHARED=0) and spock_solve instance by
    instance; FP64 forward to 1e-10 by the first two. Then the adjoint
    gradients d(V*, u^0)/d(x0, diag Q) one instance at a time (all 64 in
    FP32 to 1e-6, 8 in FP64 to 1e-10), and of all 64 in one batched call in
    both precisions. full=False (the default leg diff64b): the shared-tree
    forward and the batched adjoints only."""
    insts = G.make_batch(5)
    out = {"workload": "64 instances of the 95-node tree nx20 nu10 N8 (shared tree and data, own x0)"}
    gu = np.random.default_rng(7).standard_normal(insts[0].nu)
    for pname, prec, eps, beps, nadj in (("fp32", SP.FP32, 1e-5, 1e-6, 64), ("fp64", SP.FP64, 1e-10, 1e-10, 8)):
        gp = SP.Problem.from_instance(insts[0], precision=prec)
        dt = gp.torch_dtype
        x0s = [torch.as_tensor(i.x0, dtype=torch.float64, device="cuda") for i in insts]
        s = SP.default_settings(eps_abs=eps, eps_rel=eps, max_iters=400000)
        res = {}
        forms = [("shared_mfma", "1"), ("block_engine", "0")] if full else [("shared_mfma", "1")]
        for form, env in forms:
            os.environ["SPOCK_SHARED"] = env
            vs = [torch.zeros(gp.n_v, dtype=dt, device="cuda") for _ in insts]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            infos = SP.solve_batched([gp] * len(insts), x0s, vs, s)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            res[form] = {"seconds": round(el, 4), "all_converged": all(i["status"] == "converged" for i in infos),
                         "t_evals_total": int(sum(i["t_evals"] for i in infos)),
                         "max_iters": int(max(i["iters"] for i in infos)), "mapping": infos[0]["mapping"]}
            if form == "shared_mfma":
                res[form]["rounds"] = int(max(i["t_evals"] for i in infos))
                res[form]["ms_per_round"] = round(el / res[form]["rounds"] * 1e3, 4)
                sol = vs
            log(f"diff64 {pname} forward {form}: {el:.3f}s {res[form]}")
        os.environ.pop("SPOCK_SHARED", None)
        if pname == "fp32" and full:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ok = True
            for b in range(len(insts)):
                v1 = torch.zeros(gp.n_v, dtype=dt, device="cuda")
                ok = gp.solve(x0s[b], v1, s)["status"] == "converged" and ok
            torch.cuda.synchronize()
            res["per_instance_spock_solve"] = {"seconds": round(time.perf_counter() - t0, 4), "all_converged": ok}
            log(f"diff64 {pname} forward one by one: {res['per_instance_spock_solve']}")
        gut = torch.as_tensor(gu, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its, ok = [], True
        for b in range(nadj if full else 0):
            _, _, _, bi = gp.backward(sol[b], x0s[b], gV=1.0, gu0=gut,
                                      settings=SP.default_settings(eps_abs=beps, max_iters=200000))
            its.append(bi["iters"])
            ok = ok and bi["status"] == "converged"
        torch.cuda.synchronize()
        if full:
            res["adjoint"] = {"instances": nadj, "eps": beps, "seconds": round(time.perf_counter() - t0, 4),
                              "all_converged": ok, "J_T_applications_mean": round(float(np.mean(its)), 1),
                              "J_T_applications_max": int(np.max(its))}
            log(f"diff64 {pname} adjoint: {res['adjoint']}")
        # all 64 adjoints in one spock_backward_batched call
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        outb = SP.backward_batched(gp, sol, x0s, gV=1.0, gu0s=[gut] * len(insts),
                                   settings=SP.default_settings(eps_abs=beps, max_iters=400000))
        torch.cuda.synchronize()
        itb = [o[3]["iters"] for o in outb]
        res["adjoint_batched"] = {"instances": len(insts), "eps": beps,
                                  "seconds": round(time.perf_counter() - t0, 4),
                                  "all_converged": all(o[3]["status"] == "converged" for o in outb),
                                  "J_T_applications_mean": round(float(np.mean(itb)), 1),
                                  "J_T_applications_max": int(np.max(itb))}
        log(f"diff64 {pname} adjoint batched: {res['adjoint_batched']}")
        out[pname] = res
        gp.close()
    return out


def leg_shared64(torch, SP, G):
    """One FP32 forward of the 64-instance workload by the shared-tree form
    alone (eps 1e-5), for kernel profiles of that form."""
    insts = G.make_batch(5)
    gp = SP.Problem.from_instance(insts[0], precision=SP.FP32)
    x0s = [torch.as_tensor(i.x0, dtype=torch.float64, device="cuda") for i in insts]
    vs = [torch.zeros(gp.n_v, dtype=torch.float32, device="cuda") for _ in insts]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = SP.solve_batched([gp] * len(insts), x0s, vs, SP.default_settings(eps_abs=1e-5, eps_rel=1e-5))
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    rounds = int(max(i["t_evals"] for i in infos))
    out = {"seconds": round(el, 4), "rounds": rounds, "ms_per_round": round(el / rounds * 1e3, 4),
           "all_converged": all(i["status"] == "converged" for i in infos), "mapping": infos[0]["mapping"]}
    log(f"shared64: {out}")
    gp.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--config", type=int, default=3, choices=[1, 2, 3, 5])
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--method", default="spock", choices=["spock", "cp"])
    ap.add_argument("--t-reps", type=int, default=30)
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--budget-iters", type=int, default=3000)
    ap.add_argument("--horizons", default="3,6,9,12,15")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--legs", default="fp64,budget,223,512,fp32err,datacentre,scaling,diff64b",
                    help="comma-separated extra legs to run (see the module docstring); 'all' adds "
                         "the closed-loop simulation (mpc) and the 64-instance differentiation (diff64)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one plain device copy of 512 MiB (reference for the memory-traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: the solver runs on one GPU only (--gpus 1); sharding the tree over several GPUs "
              "is a design, not implemented", file=sys.stderr)
        raise SystemExit(2)

    import torch
    import paper_2212_01110_amd as SP
    import spock_gen as G

    torch.cuda.set_device(0)
    t_setup = time.perf_counter()
    inst = G.make_config(args.config)
    prec = SP.FP32 if args.precision == "fp32" else SP.FP64
    gp = SP.Problem.from_instance(inst, precision=prec)
    dt = gp.torch_dtype
    x0 = torch.as_tensor(inst.x0, dtype=torch.float64, device="cuda")
    v = torch.zeros(gp.n_v, dtype=dt, device="cuda")
    log(f"config {args.config} n_v={gp.n_v} alpha={gp.alpha:.6g} setup {time.perf_counter() - t_setup:.1f}s")

    # warm-up steps (the first solve also autotunes the family-to-lane mapping)
    if args.warmup > 0:
        info = gp.solve(x0, v, SP.default_settings(method=args.method, max_iters=args.warmup))
        log(f"warmup: {info['iters']} iters {info['t_evals']} T-evals map={info['mapping']} {info['seconds']:.3f}s")
    # timed: exactly K steps from a cold start
    v.zero_()
    s = SP.default_settings(method=args.method, max_iters=args.steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = gp.solve(x0, v, s)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    steps = info["iters"]
    log(f"timed: {info['status']} {steps} iters {info['t_evals']} T-evals xi={info['xi']:.4g} "
        f"V_s0={info['V_s0']:.8g} map={info['mapping']} {el:.3f}s")

    if args.calibrate_copy:
        a = torch.empty(512 << 20, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1)
        b.copy_(a)
        torch.cuda.synchronize()
        log("calibration copy: 536870912 bytes read, 536870912 bytes written")
        del a, b
    # roofline of the sweeps kernel: HIP events recorded by the library
    Tv = torch.empty_like(v)
    prof = gp.profile_T(v, x0, Tv, reps=args.t_reps)
    itemsize = 4 if prec == SP.FP32 else 8
    kname = "k_T_flow (both Alg. 2 sweeps, one launch)" if info["mapping"] == 512 else \
        "per-stage backward/forward sweep launches"
    traffic = measured_traffic() if (args.config == 3 and prec == SP.FP32 and info["mapping"] == 512) else None
    roof = {"bound": "hbm", "peak": HBM_PEAK_GBS, "unit": "GB/s", "traffic": traffic, "kernel": kname}
    roof.update(roofline_of(prof, inst, itemsize))
    log(f"T phases (us): {prof}; sweeps {roof['achieved']} GB/s ({roof['frac']}), whole T {roof['T_whole_frac']}")

    extras = {}
    legs = set(args.legs.split(",")) if not args.no_extras else set()
    if "all" in legs:
        legs |= {"fp64", "budget", "223", "512", "fp32err", "datacentre", "scaling", "mpc", "diff64"}
    keep = {}
    leg_seconds = {}

    def timed_leg(name, fn):
        t = time.perf_counter()
        r = fn()
        leg_seconds[name] = round(time.perf_counter() - t, 1)
        log(f"leg {name}: {leg_seconds[name]}s")
        return r
    if args.config == 3 and ({"fp64", "budget"} & legs):
        gps = {args.precision: gp}
        if "fp64" in legs and prec == SP.FP32:
            extras["tree20776_fp64"], gps["fp64"] = timed_leg(
                "fp64", lambda: leg_fp64(torch, SP, inst, args.steps, args.t_reps))
        if "budget" in legs:
            extras["tree20776_residual_budget"] = timed_leg(
                "budget", lambda: leg_budget(torch, SP, inst, gps, args.budget_iters))
        gps.clear()
    if "223" in legs:
        extras["time_to_residual_223node"] = timed_leg("223", lambda: ttr_single(torch, SP, G))
    if "512" in legs:
        extras["time_to_residual_512batch"] = timed_leg("512", lambda: ttr_batched(torch, SP, G, keep))
    if "fp32err" in legs:
        extras["fp32_error_vs_oracle"] = timed_leg("fp32err", lambda: leg_fp32_error(torch, SP, G, keep))
    keep.clear()
    if "datacentre" in legs:
        extras["datacentre_cp_vs_spock"] = timed_leg("datacentre", lambda: leg_datacentre(torch, SP, G))
    if "mpc" in legs:
        extras["datacentre_closed_loop_mpc"] = timed_leg("mpc", lambda: leg_mpc(torch, SP, G))
    if "diff64b" in legs and "diff64" not in legs:
        extras["differentiation_64_instances"] = timed_leg("diff64b", lambda: leg_diff64(torch, SP, G, full=False))
    if "diff64" in legs:
        extras["differentiation_64_instances"] = timed_leg("diff64", lambda: leg_diff64(torch, SP, G))
    if "shared64" in legs:
        extras["shared_forward_64_instances"] = timed_leg("shared64", lambda: leg_shared64(torch, SP, G))
    if "scaling" in legs:
        extras["datacentre_scaling"] = timed_leg(
            "scaling", lambda: leg_scaling(torch, SP, G, [int(n) for n in args.horizons.split(",")]))
    cpu = None
    if not args.no_cpu_baseline:
        cpu = timed_leg("cpu_baseline", lambda: cpu_baseline(inst, gp.alpha, args.cpu_budget))
        log(f"cpu baseline {cpu['value']} CP iters/s")

    out = {
        "metric": METRIC,
        "value": round(info["t_evals"] / el, 2),
        "unit": "CP iters/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": round(el / max(1, steps) * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == SP.FP32 else "f64",
        "data": "synthetic",
        "config": {"workload": NAMES[args.config], "method": args.method, "bulk_precision": args.precision,
                   "factor_and_residual_precision": "f64", "n_v": gp.n_v, "start": "cold (v=0)",
                   "t_evals": info["t_evals"], "xi_after_steps": info["xi"],
                   "residual_1e-4_reached": info["status"] == "converged"},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    out.update(extras)
    out["leg_seconds"] = leg_seconds
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
