"""Benchmark of the SPOCK hot path on one MI355X.

A step is one full solve of the workload to xi <= max(1e-4, 1e-4 xi_0)
(section 3 termination) from a cold start: every evaluation of the CP
operator T (stage sweeps with fused L, L*, proximal maps and residual
statistics), the Anderson Gram/direction kernels and the SuperMann line
search. value = evaluations of T (= CP iterations = calls of L) per second
over the timed solves; ms_per_step = time to residual.

roofline: the CP operator T (its backward and forward stage kernels) timed
with HIP events on the library's stream, against the algorithmic bytes of one
T; cpu_baseline: the FP64 CPU oracle on a bounded number of T evaluations of
the same workload.
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

METRIC = ("time-to-residual-1e-4 & CP iters/s, batched FP32 vs plain FP64; achieved HBM GB/s")
HBM_PEAK_GBS = 8000.0


def algorithmic_bytes_T(inst, itemsize):
    """Bytes one evaluation of T must move: every per-edge and per-node
    factor matrix once per sweep that uses it (Abar and B in both sweeps, K in
    both, R~^{-1} and W in the backward sweep), v read once, T(v) written
    once, the sweep intermediates q and d written and read once, and the
    per-node data of L and the boxes read once."""
    anc = np.asarray(inst.anc)
    nn = anc.shape[0]
    nx, nu = inst.nx, inst.nu
    nch = np.bincount(anc[1:], minlength=nn)
    nl = int(np.sum(nch > 0))
    nleaf = nn - nl
    n_z = 1 + nn * nx + nl * nu + 4 * (nn - 1) + nl
    n_eta = 2 * (nn - 1) + 2 * nl + nl * (nx + nu) + (nn - 1) * (nx + nu + 2) + nleaf * (2 * nx + 2)
    mats = (nn - 1) * (2 * nx * nx + 2 * nx * nu) + nl * (3 * nx * nu + nu * nu)
    vecs = 2 * (n_z + n_eta) + 2 * nl * (nx + nu)
    node = (nn - 1) * (nx + nu) + nleaf * nx + nn * 2 * nx + nl * 2 * nu + 2 * nn
    return int((mats + vecs + node) * itemsize), int(mats + vecs + node)


def build_workload(cfg):
    import spock_gen as G
    if cfg in (1, 2, 3, 5):
        return G.make_config(cfg)
    raise SystemExit(f"bench: config {cfg} is not a single-instance workload")


def cpu_baseline(inst, budget_s=20.0):
    """FP64 oracle T evaluations (+ residual statistics) on the same workload
    until the time budget is spent; returns CP iterations per second."""
    import oracle as O
    from oracle.layout import Layout
    lay = Layout(inst)
    fac = O.factor_s1(lay, inst)
    nl = O.norm_L(lay, inst)

    class _P:
        pass
    p = _P()
    p.inst, p.lay, p.fac, p.alpha, p.normL = inst, lay, fac, 0.99 / nl, nl
    v = np.zeros(lay.n_v)
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
    try:
        cores = len(os.sched_getaffinity(0))
    except Exception:
        cores = os.cpu_count()
    threads = int(os.environ.get("OMP_NUM_THREADS", cores))
    return {"value": n / el, "unit": "CP iters/s", "cores": min(cores, threads), "kind": "oracle",
            "sample": f"{n} CP iterations (T + residual statistics, FP64 numpy) of the same "
                      f"workload from v=0, {el:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=3)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--method", default="spock", choices=["spock", "cp"])
    ap.add_argument("--max-iters", type=int, default=20000)
    ap.add_argument("--t-reps", type=int, default=50)
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on one GPU only; --gpus must be 1", file=sys.stderr)
        raise SystemExit(2)

    import torch
    import paper_2212_01110_amd as SP

    torch.cuda.set_device(0)
    t_setup = time.perf_counter()
    inst = build_workload(args.config)
    prec = SP.FP32 if args.precision == "fp32" else SP.FP64
    gp = SP.Problem.from_instance(inst, precision=prec)
    dt = gp.torch_dtype
    x0 = torch.as_tensor(inst.x0, dtype=torch.float64, device="cuda")
    v = torch.zeros(gp.n_v, dtype=dt, device="cuda")
    s = SP.default_settings(method=args.method, max_iters=args.max_iters)
    print(f"[bench] config {args.config} n_v={gp.n_v} alpha={gp.alpha:.6g} setup "
          f"{time.perf_counter() - t_setup:.1f}s", file=sys.stderr, flush=True)

    for w in range(args.warmup):
        v.zero_()
        info = gp.solve(x0, v, s)
        print(f"[bench] warmup {w}: {info['status']} iters={info['iters']} "
              f"t_evals={info['t_evals']} {info['seconds']:.3f}s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        v.zero_()
        infos.append(gp.solve(x0, v, s))
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    t_evals = sum(i["t_evals"] for i in infos)
    for k, i in enumerate(infos):
        print(f"[bench] step {k}: {i['status']} iters={i['iters']} t_evals={i['t_evals']} "
              f"xi={i['xi']:.3g} V_s0={i['V_s0']:.8g} map={i['mapping']} {i['seconds']:.3f}s", file=sys.stderr,
              flush=True)

    # ---- roofline of T: HIP events on the library's stream (torch current stream)
    vt = torch.zeros(gp.n_v, dtype=dt, device="cuda")
    Tv = torch.empty_like(vt)
    gp.T(v, x0, Tv, want_stats=False)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(args.t_reps):
        gp.T(v, x0, Tv, want_stats=False)
    ev1.record()
    ev1.synchronize()
    t_T = ev0.elapsed_time(ev1) / 1e3 / args.t_reps
    itemsize = 4 if prec == SP.FP32 else 8
    abytes, _ = algorithmic_bytes_T(inst, itemsize)
    achieved = abytes / t_T / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "kernel": "CP operator T (k_bwd + k_fwd stage launches + k_reduce_stats)",
            "bytes_per_launch": abytes, "us_per_launch": round(t_T * 1e6, 2)}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(inst, args.cpu_budget)

    names = {1: "15-node binary tree nx2 nu1 N3 (AV@R a=0.5)",
             2: "223-node tree nx20 nu10 N10 (branching 2 for 5 stages)",
             3: "20776-node tree nx50 nu20 N15 (branching 3 for 7 stages, 2187 scenarios)",
             5: "95-node tree nx20 nu10 N8"}
    out = {
        "metric": METRIC,
        "value": round(t_evals / el, 2),
        "unit": "CP iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(el / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == SP.FP32 else "f64",
        "data": "synthetic",
        "config": {"workload": names.get(args.config, str(args.config)), "method": args.method,
                   "bulk_precision": args.precision, "eps_abs": 1e-4, "eps_rel": 1e-4,
                   "n_v": gp.n_v, "start": "cold (v=0)"},
        "time_to_residual_s": round(el / args.steps, 4),
        "t_evals_per_solve": t_evals / args.steps,
        "iters_per_solve": sum(i["iters"] for i in infos) / args.steps,
        "status": [i["status"] for i in infos],
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
