"""Benchmark: edge-sample updates/s of the leveled-DAG level sweep on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload mid] [--precision fp64] [--no-serving] [--no-mc]

One step = one full evaluation (every level, the final-node reduction, and for
the rescaled FP32 path the exponent bookkeeping) of the workload's graph for
all S samples, with the graph, the samples and the workspace already resident
in HBM.  Prints one JSON line.  The CPU-baseline leg times the plain FP64
oracle on the host cores; its outputs are also the reference for the reported
error of the GPU results (every oracle call of this script happens in that leg,
on outputs the other legs sampled).  The lookup leg ("lookup") times the same
workload with the paper's own edge factor, a per-sample table entry times a
sign.  The Monte Carlo leg ("mc") runs one Metropolis walker per sample on the
workload's graph and reports its step rate beside a plain evaluation.  The
serving leg ("serving" in the JSON) replays the
serving request stream through the continuous-batching server and through
one-at-a-time evaluation, and reports p50/p99 request latency beside
throughput.
"""

from __future__ import annotations

import argparse
import glob
import json
import os
import platform
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "edge-sample updates/s (FP64 vs FP32) at stated rel err; p50/p99 request latency"
UNIT = "edge-sample updates/s"
HBM_PEAK_GBS = 8000.0
VALU_PEAK_TFLOPS = {"fp64": 78.6, "fp32r": 157.3, "fp32": 157.3, "fp16r": 157.3, "bf16r": 157.3}
# algorithmic flops per edge-sample of the fused factor + accumulate:
# 3 sub, |.|^2 = 1 mul + 2 fma (5), 1 + b r^2 = fma (2), divide (1), acc fma (2)
FLOPS_PER_EDGE_SAMPLE = 13
# 16-bit storage has no fixed tolerance: its bar is a per-sample bound derived from the
# arithmetic, checked by the parity tests; the bench reports its errors only
TOL = {"fp64": 1e-12, "fp32r": 1e-5, "fp32": 1e-5, "fp16r": None, "bf16r": None}
# arithmetic type of the path, and the type the level values are stored in between levels
DTYPE = {"fp64": "f64", "fp32r": "f32", "fp32": "f32", "fp16r": "f32", "bf16r": "f32"}
STORAGE = {"fp64": "f64", "fp32r": "f32", "fp32": "f32", "fp16r": "f16", "bf16r": "bf16"}
VALUE_BYTES = {"fp64": 8, "fp32r": 4, "fp32": 4, "fp16r": 2, "bf16r": 2}
WORKLOAD_TEXT = {
    "tiny": "tiny: L=4, widths [1,3,4,3,1], in-degree 2, S=1024, x~U[-1,1]^3",
    "mid": "mid: L=12, interior width 256, in-degree 4, S=65536, x~N(0,I3)",
    "precision": "precision: L=24, interior width 4096, in-degree 8, S=4096, x~U[-1,1]^3, b~U[0.1,4]",
    "large": "large: L=32, interior width 65536, in-degree 6, S=1024, x~N(0,I3), b~U[0.1,4]",
}


def record_bytes(g, precision: str) -> int:
    """Record fields a level needs per edge: rational binary64 src (4 B) + c0, cb, g0, g1, g2, a (6 x 8 B);
    rational binary32 src + a, b, k0, k1, k2 (5 x 4 B); lookup src + slot (2 x 4 B) + the constant
    (8 B binary64, 4 B binary32)."""
    if g.kind == "lookup":
        return 8 + (8 if precision == "fp64" else 4)
    return 4 + 6 * 8 if precision == "fp64" else 4 + 5 * 4


def table_entry_bytes(g, precision: str) -> int:
    """Bytes of a per-sample input as the interior levels read it: binary64 coordinates or table entries,
    except the binary32 paths of a lookup graph, which read a binary32 copy of the tables."""
    return 8 if g.kind != "lookup" or precision == "fp64" else 4


def input_bytes(g, S_pad: int, precision: str) -> int:
    """Per-sample inputs read once: 3 coordinates, or the table (n_slots entries)."""
    return table_entry_bytes(g, precision) * g.n_inputs * S_pad


def level_bytes(g, S_pad: int, precision: str) -> list:
    """Algorithmic bytes of each interior-level launch: read the previous level's
    rows once, write this level's rows once, read the edge records and row
    pointers once, read the per-sample inputs once."""
    B = VALUE_BYTES[precision]
    rec = record_bytes(g, precision)
    out = []
    for l in range(1, g.L):
        w_prev = 0 if l == 1 else int(g.widths[l - 1])  # level 1 reads the root's constant 1
        out.append((w_prev + int(g.widths[l])) * S_pad * B + int(g.epl[l - 1]) * rec
                   + 4 * (int(g.widths[l]) + 1) + input_bytes(g, S_pad, precision))
    return out


def flops_per_edge_sample(g) -> int:
    """Algorithmic flops per edge-sample: the rational factor and accumulate (13), or the
    lookup factor's product with the constant and the accumulate (2)."""
    return 2 if g.kind == "lookup" else FLOPS_PER_EDGE_SAMPLE


def cpu_info() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            m = re.search(r"model name\s*:\s*(.*)", f.read())
            return m.group(1).strip() if m else platform.processor()
    except OSError:
        return platform.processor()


def _oracle_rate(g, xs, threads, target_s):
    """Sweep xs with the oracle repeatedly for about target_s seconds: (edge-sample updates/s, threads used,
    passes, seconds)."""
    import oracle

    reps, t0 = 0, time.perf_counter()
    while True:
        _, used = oracle.sweep(g, xs, threads=threads, return_threads=True)
        reps += 1
        t = time.perf_counter() - t0
        if t >= 0.9 * target_s or reps >= 10000:
            break
    return g.n_edges * xs.shape[1] * reps / t, int(used), reps, t


def _oracle_sample(g, x, threads, target_s):
    """Samples the oracle sweeps in about target_s seconds at the given thread count (calibrated on a small
    slice), at most all of them."""
    import oracle

    S = x.shape[1]
    cal = min(S, 256)
    t0 = time.perf_counter()
    oracle.sweep(g, np.ascontiguousarray(x[:, :cal]), threads=threads)
    dt = max(time.perf_counter() - t0, 1e-6)
    return int(min(S, max(cal, cal * target_s / dt)))


def cpu_baseline_leg(g, x, idx_ref, target_s: float = 12.0):
    """Time the FP64 oracle on the host cores (every core, then one thread) on a bounded sample of the same
    workload; also return its values on idx_ref, the reference for the GPU results' error."""
    import oracle

    S = x.shape[1]
    E = g.n_edges
    n = _oracle_sample(g, x, 0, target_s)
    rate, used, reps, t = _oracle_rate(g, np.ascontiguousarray(x[:, :n]), 0, target_s)
    n1 = _oracle_sample(g, x, 1, target_s / 3)
    rate1, _, reps1, t1 = _oracle_rate(g, np.ascontiguousarray(x[:, :n1]), 1, target_s / 3)
    xr = np.ascontiguousarray(x[:, idx_ref])
    V = oracle.sweep(g, xr, "value")
    Q = oracle.sweep(g, xr, "square")
    base = {"value": rate, "unit": UNIT, "cores": used, "kind": "oracle",
            "sample": f"first {n} of {S} samples of the same graph ({E} edges), FP64 level sweep, "
                      f"{reps} pass(es), {t:.1f} s on {cpu_info()}",
            "single_thread": {"value": rate1, "unit": UNIT, "cores": 1,
                              "sample": f"first {n1} of {S} samples, {reps1} pass(es), {t1:.1f} s"},
            "parallel_speedup": rate / rate1}
    return base, V, Q


def error_stats(y, V, Q, precision):
    import oracle

    scaled = oracle.scaled_error(y, V, Q)
    with np.errstate(divide="ignore", invalid="ignore"):
        plain = np.abs(y - V) / np.abs(V)
    plain = plain[np.isfinite(plain)]
    tol = TOL[precision]
    return {"scaled_max": float(scaled.max()), "tol": tol,
            "pass": bool(np.all(scaled <= tol)) if tol is not None else None,
            "plain_rel_p50": float(np.percentile(plain, 50)), "plain_rel_p99": float(np.percentile(plain, 99)),
            "plain_rel_max": float(plain.max()), "samples_checked": int(len(y)),
            "definition": "|y-r|/max(|r|,sqrt(Q)), r = FP64 oracle, Q = sum over paths of prod w^2"}


def run_timed(P, G, xd, precision, steps, warmup):
    import torch

    S = xd.shape[1]
    ws = torch.empty(G.workspace_bytes(S, precision), dtype=torch.uint8, device=xd.device)
    out = torch.empty(S, dtype=torch.float64, device=xd.device)
    for _ in range(warmup):
        G.evaluate(xd, precision, out=out, workspace=ws)
    torch.cuda.synchronize()
    for k in ("level", "fused", "final_partial", "final_combine", "fill", "hub"):
        P.timing_read(k)
    P.timing_enable(True)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(steps):
        G.evaluate(xd, precision, out=out, workspace=ws)
    stop.record()
    torch.cuda.synchronize()
    P.timing_enable(False)
    ms = start.elapsed_time(stop) / steps
    kern = {}
    for k in ("level", "fused", "final_partial", "final_combine", "fill", "hub"):
        t, n = P.timing_read(k)
        if n:
            kern[k] = {"total_ms": t, "launches": n, "avg_us": 1000.0 * t / n}
    return ms, kern, out


def level_kernel_name(G, precision):
    """The kernel the interior levels run on: row panels over narrow sample tiles where the library's panel
    plan applies (binary32 and 16-bit storage precisions of wide graphs), else the row-streamed gather."""
    from paper_2501_00675_amd._lib import PRECISIONS

    code = PRECISIONS[precision]
    return "level_panel_kernel" if (G.info()["panel_mask"] >> code) & 1 else "level_gather_kernel"


def roofline(g, S_pad, precision, kern, steps, workload, copy_gbs=None, level_kernel="level_gather_kernel"):
    """Roofline of the dominant kernel class, from its live HIP-event timings.  copy_gbs: the bandwidth a plain
    device copy reaches on this GPU, reported beside the nominal peak for HBM-bound kernels; level_kernel: the
    kernel the interior levels run on."""
    dom = max(kern, key=lambda k: kern[k]["total_ms"])
    if dom == "level":
        per_launch = level_bytes(g, S_pad, precision)
        n_launch = len(per_launch)
        bytes_step = float(sum(per_launch))
        es_step = float(sum(int(g.epl[l - 1]) for l in range(1, g.L))) * S_pad
        t_step = kern[dom]["total_ms"] / 1000.0 / steps
        hbm = bytes_step / t_step / 1e9
        alu = es_step * flops_per_edge_sample(g) / t_step / 1e12
        f_h, f_a = hbm / HBM_PEAK_GBS, alu / VALU_PEAK_TFLOPS[precision]
        if f_h >= f_a:
            r = {"bound": "hbm", "achieved": hbm, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": f_h}
        else:
            r = {"bound": "alu", "achieved": alu, "peak": VALU_PEAK_TFLOPS[precision], "unit": "TFLOP/s",
                 "frac": f_a}
        r.update({"kernel": level_kernel, "avg_launch_us": kern[dom]["avg_us"],
                  "launches_per_step": n_launch, "algorithmic_bytes_per_launch": bytes_step / n_launch,
                  "other_term": ({"alu_tflops": alu, "alu_frac": f_a} if r["bound"] == "hbm"
                                 else {"hbm_gbs": hbm, "hbm_frac": f_h})})
    elif dom == "fused":
        # whole graph per launch with levels in LDS: every edge-sample of every level
        es_step = float(g.n_edges) * S_pad
        t_launch = kern[dom]["total_ms"] / 1000.0 / kern[dom]["launches"]
        n_launch = kern[dom]["launches"] / steps
        fl = flops_per_edge_sample(g)
        alu = es_step / n_launch * fl / t_launch / 1e12
        # compulsory HBM bytes: per-sample inputs in, out written, edge records once per 64-sample workgroup
        hbm_bytes = input_bytes(g, S_pad, precision) + 8 * S_pad + g.n_edges * record_bytes(g, precision) * (S_pad // 64)
        r = {"bound": "alu", "achieved": alu, "peak": VALU_PEAK_TFLOPS[precision], "unit": "TFLOP/s",
             "frac": alu / VALU_PEAK_TFLOPS[precision], "kernel": "fused_sweep_kernel",
             "avg_launch_us": kern[dom]["avg_us"], "launches_per_step": n_launch,
             "algorithmic_flops_per_launch": es_step / n_launch * fl,
             "other_term": {"hbm_gbs_compulsory": hbm_bytes / t_launch / 1e9}}
        if g.kind == "lookup":
            # the binding stream is the table entry each edge-sample reads (from L1/L2)
            r["other_term"]["table_gbs_read"] = es_step / n_launch * table_entry_bytes(g, precision) / t_launch / 1e9
    else:
        r = {"bound": "alu", "achieved": None, "peak": None, "unit": None, "frac": None, "kernel": dom}
    if r.get("bound") == "hbm" and copy_gbs:
        r["copy_GBps"] = copy_gbs
        r["frac_of_copy"] = r["achieved"] / copy_gbs
    r["traffic"] = profiled_traffic(r.get("kernel"), workload, precision)
    r["kernel_src_id"] = kernel_source_id(r.get("kernel"))
    return r


# sources that define each timed kernel and its launch (device code, launcher, planner, build flags)
KERNEL_SOURCES = {
    "level_gather_kernel": ["kernels_level.hip", "sweep_device.h", "kernels_common.h", "cos_internal.h",
                            "evaluate.cpp", "../_build.py"],
    "level_panel_kernel": ["kernels_panel.hip", "sweep_device.h", "kernels_common.h", "cos_internal.h",
                           "evaluate.cpp", "graph.cpp", "../_build.py"],
    "fused_sweep_kernel": ["kernels_fused.hip", "fused_plan.h", "sweep_device.h", "kernels_common.h",
                           "cos_internal.h", "evaluate.cpp", "../_build.py"],
}


def kernel_source_id(kernel):
    """Hash of the sources a kernel is built and launched from (changes whenever the kernel can change)."""
    import hashlib

    files = KERNEL_SOURCES.get(kernel)
    if not files:
        return None
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2501_00675_amd", "csrc", f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def profiled_traffic(kernel, workload, precision):
    """HBM bytes per launch from the committed rocprofv3 --pmc summaries (FETCH_SIZE and WRITE_SIZE in KiB
    per dispatch, scaled by the factors a plain copy kernel gives), or None when no summary exists for this
    kernel and workload or the kernel's sources changed since the counters were taken."""
    src = kernel_source_id(kernel)
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        for line in open(path):
            if not line.startswith("pmc:"):
                continue
            kv = dict(item.split("=", 1) for item in line[4:].split())
            if (kv.get("kernel") == kernel and kv.get("workload") == workload and kv.get("precision") == precision
                    and src is not None and kv.get("src_id") == src):
                return 1024.0 * (float(kv["fetch_kib"]) * float(kv["fetch_scale"])
                                 + float(kv["write_kib"]) * float(kv["write_scale"]))
    return None


def calibrate_copy(steps: int, nbytes: int = 1 << 30) -> dict:
    """A plain device-to-device copy of nbytes: reads nbytes and writes nbytes per launch."""
    import torch

    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    del src, dst
    torch.cuda.empty_cache()
    return {"calibration": "device copy", "bytes_read_per_launch": nbytes, "bytes_written_per_launch": nbytes,
            "ms_per_launch": ms, "copy_GBps": 2 * nbytes / (ms / 1000) / 1e9}


FACTOR_TEXT = {"rational": "; w_e = a_e/(1+b_e|x-k_e|^2), x in R^3 per sample",
               "lookup": "; w_e = c_e*T_s[slot_e], c_e = +-1, T_s ~ U[-1,1]^{n} per sample"}


def lookup_leg(P, args):
    """The same workload with lookup factors (the paper's Green's-function-per-vertex-pair form):
    FP64 and FP32-rescaled throughput and roofline terms.  Returns the results and the sampled
    outputs the CPU-baseline leg checks against the oracle."""
    import torch

    from workloads import make_config

    g, T = make_config(args.workload, factor="lookup")
    S = T.shape[1]
    S_pad = (S + 255) // 256 * 256
    G = P.Graph.from_leveled(g)
    Td = torch.from_numpy(T).to("cuda:0")
    idx = np.unique(np.concatenate([[0, S - 1], np.random.default_rng(1).choice(S, min(S, 256) - 2,
                                                                                 replace=False)]))
    res = {"workload": WORKLOAD_TEXT[args.workload] + FACTOR_TEXT["lookup"].format(n=g.n_inputs)}
    check = {"graph": g, "x": np.ascontiguousarray(T[:, idx]), "y": {}, "into": res}
    for p in ("fp64", "fp32r"):
        print(f"# lookup {p}", file=sys.stderr, flush=True)
        ms, kern, out = run_timed(P, G, Td, p, args.steps, args.warmup)
        res[p] = {"value": g.n_edges * S / (ms / 1000.0), "ms_per_step": ms, "kernels": kern,
                  "roofline": roofline(g, S_pad, p, kern, args.steps, args.workload + "_lookup",
                                       level_kernel=level_kernel_name(G, p))}
        check["y"][p] = out.cpu().numpy()[idx]
    return res, [check]


MC_TEXT = ("Metropolis walkers for |V| (one per sample of the workload), uniform box proposals of half-width "
           "{sigma}, Philox4x64-10 on the device; a step = propose + level sweep + accept")


def mc_leg(P, args, workload, eval_ms):
    """Monte Carlo walkers on the workload's graph: one walker per sample, steps/s and edge-sample updates/s
    including proposal and acceptance, against a plain evaluation of the same samples (eval_ms).  The oracle
    re-runs the first walkers' chains in the CPU-baseline leg."""
    import torch

    from workloads import make_config

    g, x = make_config(workload)
    C, sigma, seed = x.shape[1], 0.5, 1
    G = P.Graph.from_leveled(g)
    res = {"workload": WORKLOAD_TEXT[workload] + "; " + MC_TEXT.format(sigma=sigma), "walkers": C}
    n_check = min(C, 64)
    check_steps = 8
    for p in ("fp64", "fp32r"):
        print(f"# mc {p}", file=sys.stderr, flush=True)
        W = P.Walkers(G, torch.from_numpy(x).to("cuda:0"), p, seed=seed, sigma=sigma)
        W.run(check_steps)  # also the warm-up; its state is what the oracle re-runs
        torch.cuda.synchronize()
        state = [t.cpu().numpy() for t in (W.x, W.accepted)] if p == "fp64" else None
        W.reset_sums()
        st = torch.cuda.current_stream()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record(st)
        W.run(args.steps)
        b.record(st)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / args.steps
        e = W.estimates()
        res[p] = {"ms_per_step": ms, "value": g.n_edges * C / (ms / 1000.0), "steps_per_s": 1000.0 / ms,
                  "walker_steps_per_s": C * 1000.0 / ms, "acceptance": e["acceptance"], "sign": e["sign"],
                  "sign_se": e["sign_se"]}
        if p in eval_ms:
            res[p]["overhead_vs_evaluate"] = ms / eval_ms[p] - 1.0
        if state is not None:
            res["check"] = {"walkers": n_check, "steps": check_steps, "x": state[0][:, :n_check],
                            "accepted": state[1][:n_check]}
    # a small graph is where launches would dominate: one launch for the whole run (fused plan) against
    # three per step (the same chain on the streamed plan)
    gt, xt = make_config("tiny", S=C)
    small = {}
    for path in ("auto", "streamed"):
        Gt = P.Graph.from_leveled(gt).set_path(path)
        W = P.Walkers(Gt, torch.from_numpy(xt).to("cuda:0"), "fp64", seed=seed, sigma=1.0)
        W.run(10)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        W.run(200)
        b.record()
        torch.cuda.synchronize()
        small[path] = a.elapsed_time(b) / 200
    res["tiny_graph"] = {"walkers": C, "steps": 200, "ms_per_step_one_launch": small["auto"],
                         "ms_per_step_three_launches": small["streamed"],
                         "walker_steps_per_s": C * 1000.0 / small["auto"]}
    chk = {"graph": g, "mc": True, "x0": np.ascontiguousarray(x[:, :n_check]), "seed": seed, "sigma": sigma,
           "into": res}
    return res, [chk]


def reference_checks(checks):
    """Part of the CPU-baseline leg: the oracle's values on the sampled outputs of the other legs, and
    the resulting error statistics (written into each check's result dict)."""
    import oracle

    for c in checks:
        if c.get("mc"):  # the oracle's chain for the first walkers: same positions and acceptances
            from oracle import mc

            ref = c["into"].pop("check")
            xo, _, no, _ = mc.run(c["graph"], c["x0"], oracle.sweep(c["graph"], c["x0"]), 0, ref["steps"],
                                  c["seed"], c["sigma"])
            c["into"]["oracle_chain"] = {"walkers": ref["walkers"], "steps": ref["steps"],
                                         "positions_bit_identical": bool(np.array_equal(xo, ref["x"])),
                                         "accepted_equal": bool(np.array_equal(no, ref["accepted"]))}
            continue
        V = oracle.sweep(c["graph"], c["x"], "value")
        Q = oracle.sweep(c["graph"], c["x"], "square")
        for p, y in c["y"].items():
            if "requests" in c:  # serving: worst case over the checked requests
                acc = c["into"].setdefault("accuracy", {"requests_checked": c["requests"],
                                                        "samples_per_request": "<=128", "scaled_max": {},
                                                        "pass": True})
                e = float(oracle.scaled_error(y, V, Q).max())
                acc["scaled_max"][p] = max(acc["scaled_max"].get(p, 0.0), e)
                acc["pass"] = bool(acc["pass"] and e <= TOL[p])
            else:
                c["into"][p]["accuracy"] = error_stats(y, V, Q, p)


SERVING_TEXT = ("serving: 512 resident graphs, L~U{4..20}, interior width log-U[16,2048], in-degree U{2..8}; "
                "4096 requests, S~log-U[256,8192], x~U[-1,1]^3; t=0 burst and Poisson arrivals")


def _pct(v, q):
    return float(np.percentile(np.asarray(v, np.float64), q))


def serving_leg(P, args):
    """Continuous-batching server vs one-at-a-time cos_evaluate on the serving request stream.

    Runs: a t=0 burst of every request (batched FP64, FP32-rescaled, and the two 16-bit storage formats),
    then Poisson arrivals at load x the measured batched-FP64 capacity, each trace replayed by batched
    FP64, batched FP32-rescaled and single-request FP64 (cos_evaluate, one request at a time, in arrival order).  Latency of a request =
    completion - arrival; throughput = total edge-samples / (last completion - first arrival).
    """
    import torch

    from workloads import serving_mix

    dev = torch.device("cuda:0")
    t_gen = time.perf_counter()
    graphs, reqs = serving_mix()
    print(f"# serving: {len(graphs)} graphs, {len(reqs)} requests generated in {time.perf_counter() - t_gen:.1f} s",
          file=sys.stderr, flush=True)
    Gs = [P.Graph.from_leveled(g) for g in graphs]
    es = np.array([graphs[r["graph"]].n_edges * r["S"] for r in reqs], np.float64)
    total_es = float(es.sum())
    Ss = np.array([r["S"] for r in reqs])
    off = np.concatenate([[0], np.cumsum(Ss)])
    xs = [torch.from_numpy(r["x"]).to(dev) for r in reqs]
    outs = {k: torch.empty(int(off[-1]), dtype=torch.float64, device=dev)
            for k in ("fp64", "fp32r", "fp16r", "bf16r", "single")}

    def out_view(kind, i):
        return outs[kind][int(off[i]):int(off[i + 1])]

    ws = torch.empty(max(G.workspace_bytes(int(S), "fp64") for G, S in ((Gs[r["graph"]], r["S"]) for r in reqs)),
                     dtype=torch.uint8, device=dev)
    budget = int(args.serve_budget_gib * (1 << 30))
    srv = P.Server(budget, args.serve_slots)
    gids = [srv.add_graph(G) for G in Gs]
    torch.cuda.synchronize()

    def batched(precision, arrivals_ns, n=None):
        n = len(reqs) if n is None else n
        before = srv.stats()
        srv.read_steps()  # drop the trace of earlier runs
        P.timing_read("serve")
        P.timing_read("fill")
        P.timing_enable(True)
        t0 = time.monotonic_ns() + 1_000_000
        tickets = []
        for i in range(n):
            target = t0 + int(arrivals_ns[i])
            while time.monotonic_ns() < target:
                pass
            tickets.append(srv.submit(gids[reqs[i]["graph"]], xs[i], precision, out=out_view(precision, i),
                                      sync_inputs=False))
        st = [srv.wait(t) for t in tickets]
        after = srv.stats()
        P.timing_enable(False)
        step_ms, n_steps = P.timing_read("serve")
        trace = srv.read_steps()
        period = np.diff([r["t_done_ns"] for r in trace]) / 1e3  # completion-to-completion, µs
        per_step = [r["n_fused"] + r["n_streamed"] for r in trace]
        done = np.array([d["t_done_ns"] for d in st], np.float64)
        lat = (done - (t0 + np.asarray(arrivals_ns[:n], np.float64))) / 1e6
        span = (done.max() - t0) / 1e9
        return {"value": float(es[:n].sum()) / span, "makespan_ms": span * 1e3, "p50_ms": _pct(lat, 50),
                "p99_ms": _pct(lat, 99), "steps": after["steps"] - before["steps"],
                "step_graph_ms": step_ms, "mean_step_us": 1000.0 * step_ms / max(n_steps, 1),
                "max_step_requests": after["max_step_requests"], "max_active": after["max_active"],
                "peak_workspace_bytes": after["peak_bytes"],
                "step_trace": {"steps": len(trace),
                               "period_us_p50": _pct(period, 50) if len(period) else None,
                               "period_us_p99": _pct(period, 99) if len(period) else None,
                               "requests_per_step_p50": _pct(per_step, 50) if per_step else None}}

    def single(arrivals_ns, n=None):
        n = len(reqs) if n is None else n
        stream = torch.cuda.current_stream(dev)
        t0 = time.monotonic_ns() + 1_000_000
        done = np.empty(n)
        for i in range(n):
            target = t0 + int(arrivals_ns[i])
            while time.monotonic_ns() < target:
                pass
            Gs[reqs[i]["graph"]].evaluate(xs[i], "fp64", out=out_view("single", i), workspace=ws)
            stream.synchronize()
            done[i] = time.monotonic_ns()
        lat = (done - (t0 + np.asarray(arrivals_ns[:n], np.float64))) / 1e6
        span = (done.max() - t0) / 1e9
        return {"value": float(es[:n].sum()) / span, "makespan_ms": span * 1e3, "p50_ms": _pct(lat, 50),
                "p99_ms": _pct(lat, 99)}

    zeros = np.zeros(len(reqs))
    for p in ("fp64", "fp32r", "fp16r", "bf16r"):  # warm-up: code objects, first-touch of the arena
        batched(p, zeros, n=256)
    single(zeros, n=64)
    res = {"workload": SERVING_TEXT, "requests": len(reqs), "graphs": len(graphs), "total_edge_samples": total_es,
           "server": {"hbm_budget_bytes": budget, "max_slots": args.serve_slots}}
    res["burst"] = {p: batched(p, zeros) for p in ("fp64", "fp32r", "fp16r", "bf16r")}
    res["burst"]["fp64_single"] = single(zeros)
    cap_rps = len(reqs) / (res["burst"]["fp64"]["makespan_ms"] / 1e3)
    res["poisson"] = {}
    modes = {"fp64_batched": lambda a: batched("fp64", a), "fp32r_batched": lambda a: batched("fp32r", a),
             "fp64_single": single}
    for load in args.serve_loads:
        rate = load * cap_rps
        runs = {}
        for seed in args.serve_seeds:
            gaps = np.random.default_rng(seed).exponential(1.0, len(reqs))
            arr = np.cumsum(gaps) / rate * 1e9
            arr -= arr[0]
            print(f"# serving poisson load {load} seed {seed}: {rate:.0f} requests/s", file=sys.stderr, flush=True)
            runs[str(seed)] = {m: f(arr) for m, f in modes.items()}
        summary = {}
        for m in modes:
            for q in ("p50_ms", "p99_ms"):
                v = [runs[k][m][q] for k in runs]
                summary[f"{m}_{q}"] = {"median": _pct(v, 50), "min": float(min(v)), "max": float(max(v))}
        res["poisson"][str(load)] = {"rate_rps": rate, "seeds": runs, "across_seeds": summary}
    torch.cuda.synchronize()
    # results of the last trace: batched FP64 bit-identical to one-at-a-time FP64 for every request
    same = torch.eq(outs["fp64"].view(torch.int64), outs["single"].view(torch.int64))
    res["fp64_batched_bit_identical_to_single"] = bool(same.all().item())
    # sampled outputs of a seeded subset of requests (64 requests, up to 128 samples each), checked
    # against the oracle by the CPU-baseline leg
    checks = []
    for i in np.random.default_rng(5).choice(len(reqs), 64, replace=False):
        r = reqs[i]
        idx = np.unique(np.random.default_rng(int(i)).choice(r["S"], min(r["S"], 128), replace=False))
        checks.append({"graph": graphs[r["graph"]], "x": np.ascontiguousarray(r["x"][:, idx]), "requests": 64,
                       "into": res, "y": {p: out_view(p, i).cpu().numpy()[idx] for p in ("fp64", "fp32r")}})
    srv.close()
    return res, checks


def sampled_idx(S, n, seed):
    """Samples 0 and S-1 plus a seeded draw, n in all (at most S)."""
    return np.unique(np.concatenate([[0, S - 1], np.random.default_rng(seed).choice(S, min(S, n) - 2,
                                                                                    replace=False)]))


def extra_leg(P, name, precisions, args, copy_gbs):
    """Another workload timed at each precision (roofline, sampled outputs for the CPU-baseline leg's check,
    and the FP32-rescaled result against the GPU's own FP64 result on every sample)."""
    import torch

    from workloads import make_config

    g, x = make_config(name)
    S = x.shape[1]
    S_pad = (S + 255) // 256 * 256
    G = P.Graph.from_leveled(g)
    xd = torch.from_numpy(x).to("cuda:0")
    idx = sampled_idx(S, 1024, 0)
    res = {"workload": WORKLOAD_TEXT[name] + FACTOR_TEXT["rational"], "L": g.L, "edges": g.n_edges, "S": S}
    check = {"graph": g, "x": np.ascontiguousarray(x[:, idx]), "y": {}, "into": res, "full_x": x, "name": name}
    full = {}
    for p in precisions:
        print(f"# {name} {p}", file=sys.stderr, flush=True)
        ms, kern, out = run_timed(P, G, xd, p, args.steps, args.warmup)
        res[p] = {"value": g.n_edges * S / (ms / 1000.0), "ms_per_step": ms, "dtype": DTYPE[p],
                  "storage_dtype": STORAGE[p], "kernels": kern,
                  "roofline": roofline(g, S_pad, p, kern, args.steps, name, copy_gbs,
                                       level_kernel_name(G, p))}
        y = out.cpu().numpy()
        full[p] = y
        check["y"][p] = y[idx]
    if "fp64" in full:
        for p in [q for q in full if q != "fp64"]:
            with np.errstate(divide="ignore", invalid="ignore"):
                rel = np.abs(full[p] - full["fp64"]) / np.abs(full["fp64"])
            rel = rel[np.isfinite(rel)]
            res[p]["vs_gpu_fp64_plain_rel"] = {"p50": float(np.percentile(rel, 50)),
                                               "p99": float(np.percentile(rel, 99)), "max": float(rel.max()),
                                               "samples": int(len(rel))}
    G.close()
    return res, [check]


def oracle_full_pass(g, x):
    """One oracle pass over every sample of a workload on all host cores (edge-sample updates/s)."""
    import oracle

    t0 = time.perf_counter()
    _, used = oracle.sweep(g, np.ascontiguousarray(x), return_threads=True)
    t = time.perf_counter() - t0
    return {"value": g.n_edges * x.shape[1] / t, "unit": UNIT, "cores": int(used), "samples": int(x.shape[1]),
            "seconds": t}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="large", choices=sorted(WORKLOAD_TEXT))
    ap.add_argument("--precision", default="fp32r", choices=sorted(TOL))
    ap.add_argument("--variants", default="fp64,fp16r,bf16r",
                    help="comma list of extra precisions to time ('' for none; fp16r is skipped for lookup factors)")
    ap.add_argument("--extra", default="mid,precision",
                    help="comma list of other workloads timed at FP64 and FP32-rescaled ('' for none)")
    ap.add_argument("--mc-workload", default="mid", choices=sorted(WORKLOAD_TEXT))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only time a plain 1 GiB device copy (reference for HBM counters and bandwidth)")
    ap.add_argument("--factor", default="rational", choices=["rational", "lookup"],
                    help="edge-factor kind of the timed workload")
    ap.add_argument("--no-lookup", action="store_true", help="skip the lookup-factor block of the default run")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving leg")
    ap.add_argument("--no-mc", action="store_true", help="skip the Monte Carlo walkers leg")
    ap.add_argument("--serving-only", action="store_true", help="run only the serving leg")
    ap.add_argument("--serve-slots", type=int, default=256)
    ap.add_argument("--serve-budget-gib", type=float, default=24.0)
    ap.add_argument("--serve-loads", type=lambda v: [float(t) for t in v.split(",") if t], default=[0.5, 0.9])
    ap.add_argument("--serve-seeds", type=lambda v: [int(t) for t in v.split(",") if t], default=[4, 14, 24],
                    help="seeds of the Poisson arrival traces replayed at each load")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only: samples are independent, so the path "
                                   "would replicate the graph on every GPU and give each S/N samples with no "
                                   "per-level exchange, but no multi-GPU run is provided",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.calibrate_copy:
        print(json.dumps(calibrate_copy(args.steps)), flush=True)
        return

    import torch

    import paper_2501_00675_amd as P
    from workloads import make_config

    if args.serving_only:
        res, checks = serving_leg(P, args)
        if not args.no_cpu_baseline:
            reference_checks(checks)
        print(json.dumps({"serving": res}), flush=True)
        return
    copy = calibrate_copy(10)
    copy_gbs = copy["copy_GBps"]
    g, x = make_config(args.workload, factor=args.factor)
    S = x.shape[1]
    E = g.n_edges
    G = P.Graph.from_leveled(g)
    xd = torch.from_numpy(x).to("cuda:0")
    S_pad = (S + 255) // 256 * 256

    print(f"# bench {args.workload} S={S} E={E} precision={args.precision} steps={args.steps}", file=sys.stderr,
          flush=True)
    ms, kern, out = run_timed(P, G, xd, args.precision, args.steps, args.warmup)
    y = out.cpu().numpy()
    value = E * S / (ms / 1000.0)
    result = {
        "metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPE[args.precision], "data": "synthetic (seeded generator; stands in for the paper's CoS graphs)",
        "config": {"workload": WORKLOAD_TEXT[args.workload] + FACTOR_TEXT[args.factor].format(n=g.n_inputs),
                   "L": g.L, "edges": E, "nodes": g.n_nodes, "S": S, "precision": args.precision,
                   "storage_dtype": STORAGE[args.precision], "factor": args.factor, "seed": g.meta.get("seed")},
        "kernels": kern,
        "roofline": roofline(g, S_pad, args.precision, kern, args.steps, args.workload, copy_gbs,
                             level_kernel_name(G, args.precision)),
        "copy_calibration": copy,
    }
    variants = {}
    for pv in [v for v in args.variants.split(",") if v and v != args.precision
               and not (v == "fp16r" and g.kind == "lookup")]:
        print(f"# variant {pv}", file=sys.stderr, flush=True)
        msv, kv, outv = run_timed(P, G, xd, pv, args.steps, args.warmup)
        variants[pv] = {"value": E * S / (msv / 1000.0), "ms_per_step": msv, "dtype": DTYPE[pv],
                        "storage_dtype": STORAGE[pv], "kernels": kv,
                        "roofline": roofline(g, S_pad, pv, kv, args.steps, args.workload, copy_gbs,
                                             level_kernel_name(G, pv)),
                        "_y": outv.cpu().numpy()}
    if "fp64" in variants:
        variants["fp64"]["speed_ratio_headline_over_fp64"] = value / variants["fp64"]["value"]
    G.close()
    checks = []
    extras = {}
    for name in [w for w in args.extra.split(",") if w and w != args.workload]:
        extras[name], c = extra_leg(P, name, ["fp64", "fp32r"], args, copy_gbs)
        checks += c
    if args.factor == "rational" and not args.no_mc:
        eval_ms = {}
        if args.mc_workload == args.workload:
            eval_ms = {args.precision: ms, **{k: v["ms_per_step"] for k, v in variants.items()}}
        elif args.mc_workload in extras:
            eval_ms = {p: extras[args.mc_workload][p]["ms_per_step"] for p in ("fp64", "fp32r")}
        result["mc"], c = mc_leg(P, args, args.mc_workload, eval_ms)
        checks += c
    if args.factor == "rational" and not args.no_lookup:
        result["lookup"], c = lookup_leg(P, args)
        checks += c
    if not args.no_serving:
        result["serving"], c = serving_leg(P, args)
        checks += c
    if not args.no_cpu_baseline:
        print("# cpu baseline (oracle)", file=sys.stderr, flush=True)
        idx = sampled_idx(S, 1024, 0)
        base, V, Q = cpu_baseline_leg(g, x, idx, args.cpu_seconds)
        result["cpu_baseline"] = base
        result["accuracy"] = error_stats(y[idx], V, Q, args.precision)
        for pv, d in variants.items():
            d["accuracy"] = error_stats(d["_y"][idx], V, Q, pv)
        # the oracle over every sample of each workload, one pass on all cores
        result["oracle_full_S"] = {args.workload: oracle_full_pass(g, x)}
        for c in checks:
            if "full_x" in c:
                result["oracle_full_S"][c["name"]] = oracle_full_pass(c["graph"], c.pop("full_x"))
        reference_checks(checks)
    else:
        result["cpu_baseline"] = None
        if "mc" in result:
            result["mc"].pop("check", None)  # host copies kept for the oracle's chain, not reported
    for d in variants.values():
        d.pop("_y", None)
    result["variants"] = variants
    result["extra_workloads"] = extras
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
