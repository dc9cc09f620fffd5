"""Leveled-DAG diagram summation on AMD Instinct MI355X (gfx950).

Evaluates the combinatorial-summation graph of Sturt & Kozik (arXiv
2501.00675, Sec. II): the root holds 1, each edge multiplies its source value
by an edge factor and adds it into its destination, and the final node holds
the sum over all root-to-final paths of the products of their factors -- for
many sample points at once.  The work runs in hand-written HIP kernels behind
the C ABI of include/cos.h (libcosdag.so); this package only marshals
arguments.  There is no CPU fallback: importing fails if the library is not
built.

Usage (device tensors from torch; every call is queued on the current stream):

    import torch, paper_2501_00675_amd as cos
    G = cos.Graph(L, widths, edges_per_level, src, dst, a, b, k)   # or slot=, coef=, n_slots=
    y = G.evaluate(x)                        # x: float64 [3, S] on the device -> V per sample
    y32 = G.evaluate(x, "fp32r")             # also "fp32", "fp16r", "bf16r"
    G.save("g.npz"); G = cos.Graph.load("g.npz")

    with cos.Server(hbm_budget=8 << 30, max_slots=64) as srv:   # continuous batching
        gid = srv.add_graph(G)
        t = srv.submit(gid, x, "fp64")       # t.out holds the result once srv.wait(t) returns
        stats = srv.wait(t)                  # latency stamps, steps

    W = cos.Walkers(G, x0, "fp64", seed=1, sigma=0.5)   # Metropolis walkers for |V(x)|
    W.run(200).reset_sums().run(1000)
    W.estimates()                            # <sign V>, <|x|^2>, standard errors, acceptance
"""

from ._lib import LIB, PRECISIONS, CosError  # noqa: F401
from .graph import Graph, timing_enable, timing_read  # noqa: F401
from .mc import Walkers  # noqa: F401
from .server import Server, Ticket  # noqa: F401

__all__ = ["Graph", "Server", "Ticket", "Walkers", "CosError", "PRECISIONS", "timing_enable", "timing_read", "LIB"]
