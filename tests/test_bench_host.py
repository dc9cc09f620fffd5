"""bench.py's host logic (no GPU): the output contract's refusal of several GPUs, the algorithmic byte and flop
counts behind the roofline, the roofline's choice of bound, and the reading of the committed counter lines."""

import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from workloads import make_config  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_json_line():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=60)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def test_level_bytes_by_hand_on_the_tiny_graph():
    # tiny: widths [1, 3, 4, 3, 1], edges per level [3, 8, 6, 3]; interior launches are levels 1..L-1
    g, _ = make_config("tiny")
    assert list(g.widths) == [1, 3, 4, 3, 1] and list(g.epl) == [3, 8, 6, 3]
    S_pad = 1024
    got = bench.level_bytes(g, S_pad, "fp64")
    rec, x = 4 + 6 * 8, 3 * 8 * S_pad
    want = [(0 + 3) * S_pad * 8 + 3 * rec + 4 * (3 + 1) + x,   # level 1 reads only the root's constant
            (3 + 4) * S_pad * 8 + 8 * rec + 4 * (4 + 1) + x,
            (4 + 3) * S_pad * 8 + 6 * rec + 4 * (3 + 1) + x]
    assert got == want
    # binary32 records (src + a, b, k0..k2) and 2-byte storage
    got16 = bench.level_bytes(g, S_pad, "fp16r")
    assert got16[1] == (3 + 4) * S_pad * 2 + 8 * (4 + 5 * 4) + 4 * 5 + x


def test_lookup_entry_bytes_follow_the_table_copy():
    g, _ = make_config("tiny", factor="lookup")
    n = g.n_inputs
    assert bench.input_bytes(g, 256, "fp64") == 8 * n * 256
    for p in ("fp32", "fp32r", "bf16r"):  # binary32 paths read the binary32 copy of the tables
        assert bench.input_bytes(g, 256, p) == 4 * n * 256
    assert bench.record_bytes(g, "fp64") == 16 and bench.record_bytes(g, "fp32r") == 12
    assert bench.flops_per_edge_sample(g) == 2
    r, _ = make_config("tiny")
    assert bench.input_bytes(r, 256, "fp32r") == 3 * 8 * 256 and bench.flops_per_edge_sample(r) == 13


def test_roofline_names_the_binding_term():
    g, _ = make_config("tiny")
    S_pad, steps = 1024, 4
    bytes_step = sum(bench.level_bytes(g, S_pad, "fp64"))
    # a level time that makes the byte rate 4 TB/s: HBM-bound at half the peak
    t_step = bytes_step / 4e12
    kern = {"level": {"total_ms": t_step * steps * 1e3, "launches": 3 * steps, "avg_us": t_step / 3 * 1e6}}
    r = bench.roofline(g, S_pad, "fp64", kern, steps, "tiny")
    assert r["bound"] == "hbm" and r["frac"] == pytest.approx(0.5) and r["kernel"] == "level_gather_kernel"
    assert r["traffic"] is None  # no counter line for this workload
    # whole-graph launches are priced against the vector peak of their precision
    kern = {"fused": {"total_ms": 1.0 * steps, "launches": steps, "avg_us": 1000.0}}
    r = bench.roofline(g, S_pad, "fp32r", kern, steps, "tiny")
    es = float(g.n_edges) * S_pad
    assert r["bound"] == "alu" and r["peak"] == 157.3
    assert r["achieved"] == pytest.approx(es * 13 / 1e-3 / 1e12)


def test_counter_lines_are_read_only_for_the_current_sources():
    src = bench.kernel_source_id("fused_sweep_kernel")
    assert src is not None and len(src) == 16
    lines = [l for f in sorted(os.listdir(os.path.join(ROOT, "profiles"))) if f.endswith(".md")
             for l in open(os.path.join(ROOT, "profiles", f)) if l.startswith("pmc:")]
    assert lines, "committed counter lines"
    parsed = [dict(item.split("=", 1) for item in line[4:].split()) for line in lines]

    def traffic(kv):
        return 1024.0 * (float(kv["fetch_kib"]) * float(kv["fetch_scale"])
                         + float(kv["write_kib"]) * float(kv["write_scale"]))

    # lines taken on the current sources are the ones read; a stale line never is
    current = {(kv["kernel"], kv["workload"], kv["precision"]): traffic(kv) for kv in parsed
               if kv["src_id"] == bench.kernel_source_id(kv["kernel"])}
    assert current, "counter lines for the current kernel sources"
    for kv in parsed:
        key = (kv["kernel"], kv["workload"], kv["precision"])
        got = bench.profiled_traffic(*key)
        if key in current:
            assert got == pytest.approx(current[key])
        else:
            assert got is None
    assert bench.profiled_traffic("no_such_kernel", "mid", "fp64") is None
    assert bench.profiled_traffic("fused_sweep_kernel", "no_such_workload", "fp64") is None


def test_error_stats_against_a_known_reference():
    V = np.array([1.0, -2.0, 4.0, 0.5])
    Q = np.array([1.0, 4.0, 16.0, 100.0])  # sqrt(Q) = 10 dominates the last sample's scale
    y = V + np.array([1e-13, -2e-13, 0.0, 1e-12])
    e = bench.error_stats(y, V, Q, "fp64")
    assert e["scaled_max"] == pytest.approx(1e-13, rel=1e-6) and e["pass"] is True
    assert e["plain_rel_max"] == pytest.approx(2e-12, rel=1e-6)
    assert bench.error_stats(y, V, Q, "fp16r")["pass"] is None  # 16-bit: bar checked by the parity tests
