"""The five synthetic workloads and the serving request stream.

Shapes follow the paper's description of CoS graphs (2n+2 levels, edge count
growing exponentially with order n; Sec. III) at orders of magnitude only: the
paper's real graphs come from an external construction and are not available.

  tiny       L=4,  widths [1,3,4,3,1], d=2, S=1024, x~U[-1,1]^3, b~U[0.5,2]
  mid        L=12, interior width 256, d=4, S=65536, x~N(0,I3), b~U[0.5,2]
  precision  L=24, interior width 4096, d=8, S=4096, x~U[-1,1]^3, b~U[0.1,4]
  large      L=32, interior width 65536, d=6, S=1024, x~N(0,I3), b~U[0.1,4]
  serving    512 graphs, L~U{4..20}, width log-U[16,2048], d~U{2..8},
             requests S~log-U[256,8192], x~U[-1,1]^3, b~U[0.5,2]

a ~ U[-1,1] and k ~ U[-1,1]^3 everywhere.  Level 1 has in-degree 1 (the
root is its only possible source); the final node takes all of level L-1.
Each config has a fixed seed (tiny 1, mid 2, precision 3, serving 4, large 5),
fanned out with SeedSequence.spawn into structure / parameter / sample streams.
"""

from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from .graphs import LeveledGraph, draw_lookup, draw_params, draw_samples, draw_table, layered_graph

CONFIGS = {
    "tiny": dict(widths=[1, 3, 4, 3, 1], degree=2, S=1024, x="uniform", b=(0.5, 2.0), seed=1),
    "mid": dict(L=12, width=256, degree=4, S=65536, x="normal", b=(0.5, 2.0), seed=2),
    "precision": dict(L=24, width=4096, degree=8, S=4096, x="uniform", b=(0.1, 4.0), seed=3),
    "large": dict(L=32, width=65536, degree=6, S=1024, x="normal", b=(0.1, 4.0), seed=5),
}

SERVING = dict(n_graphs=512, L=(4, 20), width=(16, 2048), degree=(2, 8), S=(256, 8192),
               n_requests=4096, x="uniform", b=(0.5, 2.0), seed=4)


def _widths(cfg) -> list:
    if "widths" in cfg:
        return list(cfg["widths"])
    return [1] + [cfg["width"]] * (cfg["L"] - 1) + [1]


def lookup_slots(L: int) -> int:
    """Table entries per sample for a graph of L edge levels: read as order n with
    L = 2n + 2 levels and 2n vertices, one entry per ordered vertex pair, (L - 2)^2
    (at least 4)."""
    return max(4, (L - 2) ** 2)


def make_config(name: str, S: int | None = None, seed: int | None = None,
                order: str = "src", factor: str = "rational", **over) -> tuple[LeveledGraph, np.ndarray]:
    """Build (graph, per-sample input) for a named config.  S / seed / shape keys may be overridden.

    factor "rational": a, b, k per edge and x[3, S] coordinates;
    factor "lookup": the same structure with a table entry and a fermion sign per
    edge and per-sample tables T[n_slots, S] (n_slots = lookup_slots(L)).
    """
    cfg = dict(CONFIGS[name])
    cfg.update(over)
    if S is not None:
        cfg["S"] = S
    sd = cfg["seed"] if seed is None else seed
    ss_struct, ss_par, ss_x = np.random.SeedSequence(sd).spawn(3)
    g = layered_graph(_widths(cfg), cfg["degree"], np.random.Generator(np.random.PCG64(ss_struct)),
                      order=order)
    if factor == "lookup":
        n_slots = int(cfg.get("n_slots", lookup_slots(g.L)))
        g = draw_lookup(g, np.random.Generator(np.random.PCG64(ss_par)), n_slots)
        x = draw_table(n_slots, int(cfg["S"]), np.random.Generator(np.random.PCG64(ss_x)))
    elif factor == "rational":
        draw_params(g, np.random.Generator(np.random.PCG64(ss_par)), b_range=cfg["b"])
        x = draw_samples(int(cfg["S"]), cfg["x"], np.random.Generator(np.random.PCG64(ss_x)))
    else:
        raise ValueError(factor)
    g.meta = dict(config=name, seed=sd, factor=factor, **{k: v for k, v in cfg.items() if k != "seed"})
    return g, x


def _log_uniform_int(rng, lo, hi, size=None):
    return np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), size))).astype(np.int64)


def serving_mix(n_graphs: int | None = None, n_requests: int | None = None, seed: int | None = None,
                max_width: int | None = None, max_S: int | None = None):
    """Graphs and request stream of the serving workload.

    Returns (graphs, requests) where requests is a list of dicts
    {graph: index, S: samples, x: float64[3,S], seed: int}; arrival times are
    drawn by the caller (they depend on the measured capacity).
    """
    cfg = dict(SERVING)
    if n_graphs is not None:
        cfg["n_graphs"] = n_graphs
    if n_requests is not None:
        cfg["n_requests"] = n_requests
    sd = cfg["seed"] if seed is None else seed
    ss_g, ss_r = np.random.SeedSequence(sd).spawn(2)

    def one_graph(i, ss):
        rng = np.random.Generator(np.random.PCG64(ss))
        L = int(rng.integers(cfg["L"][0], cfg["L"][1] + 1))
        W = int(_log_uniform_int(rng, *cfg["width"]))
        if max_width is not None:
            W = min(W, max_width)
        d = int(rng.integers(cfg["degree"][0], cfg["degree"][1] + 1))
        g = layered_graph([1] + [W] * (L - 1) + [1], d, rng)
        draw_params(g, rng, b_range=cfg["b"])
        g.meta = dict(config="serving", graph=i, L=L, width=W, degree=d)
        return g

    # every graph has its own seed stream, so building them in threads changes nothing
    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        graphs = list(ex.map(one_graph, range(cfg["n_graphs"]), ss_g.spawn(cfg["n_graphs"])))
    rng = np.random.Generator(np.random.PCG64(ss_r))
    reqs = []
    for r in range(cfg["n_requests"]):
        gi = int(rng.integers(len(graphs)))
        S = int(_log_uniform_int(rng, *cfg["S"]))
        if max_S is not None:
            S = min(S, max_S)
        xs = int(rng.integers(1 << 62))
        x = draw_samples(S, cfg["x"], np.random.Generator(np.random.PCG64(xs)))
        reqs.append(dict(graph=gi, S=S, x=x, seed=xs))
    return graphs, reqs
