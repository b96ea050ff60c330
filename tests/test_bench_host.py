"""Host-side logic of bench.py (no GPU): the algorithmic byte count behind
the roofline figure, the vector sizes it is built from, the refusal of more
than one GPU, and the committed HBM-traffic summary it reads."""
import importlib.util
import os
import re
import subprocess
import sys

import pytest

import spock_gen as G
from oracle.layout import Layout

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_sweeps_bytes_of_the_20776_node_tree(bench):
    # both Alg. 2 sweeps in FP32 on the n_x 50, n_u 20, N 15 tree: every
    # factor matrix once per sweep that uses it, q and d written and read once
    inst = G.make_config(3)
    assert bench.algorithmic_elems_sweeps(inst) * 4 == 845_795_040
    assert bench.algorithmic_elems_sweeps_regrouped(inst) * 4 == 785_566_280


@pytest.mark.parametrize("cfg", [1, 2, 3])
def test_vector_sizes_match_the_oracle_layout(bench, cfg):
    inst = G.make_config(cfg)
    lay = Layout(inst)
    assert bench.sizes(inst) == (lay.n_z, lay.n_eta)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""


def test_traffic_summary_is_well_formed(bench):
    path = os.path.join(ROOT, "profiles", "k_T_flow_20776node_fp32_traffic.md")
    txt = open(path).read()
    b = int(re.search(r"traffic_bytes_per_launch: (\d+)", txt).group(1))
    assert re.search(r"kernel_sources_sha256_16: [0-9a-f]{16}", txt)
    # measured against algorithmic bytes of the same launch: within 1%
    assert abs(b / 845_795_040 - 1.0) < 0.01
    got = bench.measured_traffic()
    assert got is None or got == b
