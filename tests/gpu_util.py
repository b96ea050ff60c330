"""Helpers for the GPU parity tests (device tensors, oracle comparison)."""
import json
import os
import zlib

import numpy as np

import oracle as O
import paper_2212_01110_amd as SP


def dev(a, dtype):
    import torch
    return torch.as_tensor(np.asarray(a, dtype=np.float64), device="cuda").to(dtype).contiguous()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().to("cpu").double().numpy()


def build(inst, precision=SP.FP64, alpha=None):
    """GPU problem and oracle problem with the same step size (the oracle
    computes its own ||L||; the two are compared in a test)."""
    op = O.Problem(inst) if alpha is None else O.Problem(inst, alpha=alpha)
    gp = SP.Problem.from_instance(inst, precision=precision, alpha=op.alpha)
    return gp, op


def relerr(a, b):
    return float(np.max(np.abs(a - b)) / max(1.0, np.max(np.abs(b))))


def seeded(name: str) -> np.random.Generator:
    """Generator seeded from the case name (stable across processes)."""
    return np.random.default_rng(zlib.crc32(name.encode()))


def check(tag: str, err: float, tol: float):
    """Asserts err <= tol; with SPOCK_ERRLOG set, also appends the measured
    error to that file (one JSON object per line) so the margins can be read
    after a run."""
    path = os.environ.get("SPOCK_ERRLOG")
    if path:
        with open(path, "a") as f:
            f.write(json.dumps({"case": tag, "err": float(err), "tol": float(tol)}) + "\n")
    assert err <= tol, f"{tag}: error {err:.3e} above {tol:.1e}"
