"""Leveled-DAG container and seeded structure / parameter / sample draws.

Layout follows the flattened representation of the paper (Sec. II.C "Graph
flattening", Fig. ``combinedgraphflat``): levels l = 0..L of node widths
W_0..W_L with W_0 = W_L = 1; node ids are global and contiguous level by level;
edge level l (l = 1..L) holds the edges whose destination lies in node level l
(the figure names an edge box by its destination level).  Edges are stored
level-major as flat (src, dst) arrays plus per-edge parameters (a, b, k) of the
synthetic edge factor w_e(x) = a_e / (1 + b_e |x - k_e|^2).
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class LeveledGraph:
    """Per-level flattened edge lists of a leveled DAG.

    widths  int64[L+1]  node count of each level (widths[0] = widths[L] = 1)
    epl     int64[L]    edges per edge level l = 1..L (epl[l-1])
    src,dst int32[E]    global node ids, level-major
    a, b    float64[E]  edge-factor parameters (rational factor)
    k       float64[E,3]
    slot    int32[E]    lookup factor: table entry of each edge (None: rational factor)
    coef    float64[E]  lookup factor: constant of each edge (fermion-loop sign)
    n_slots int         lookup factor: entries per sample table
    """

    widths: np.ndarray
    epl: np.ndarray
    src: np.ndarray
    dst: np.ndarray
    a: np.ndarray
    b: np.ndarray
    k: np.ndarray
    meta: dict = field(default_factory=dict)
    slot: np.ndarray | None = None
    coef: np.ndarray | None = None
    n_slots: int = 0

    @property
    def kind(self) -> str:
        return "lookup" if self.slot is not None else "rational"

    @property
    def n_inputs(self) -> int:
        """Rows of the per-sample input: 3 coordinates, or the table entries."""
        return int(self.n_slots) if self.slot is not None else 3

    @property
    def L(self) -> int:
        return int(len(self.widths) - 1)

    @property
    def n_nodes(self) -> int:
        return int(self.widths.sum())

    @property
    def n_edges(self) -> int:
        return int(self.epl.sum())

    @property
    def final_node(self) -> int:
        return self.n_nodes - 1

    def level_slices(self):
        off = np.concatenate([[0], np.cumsum(self.epl)])
        return [slice(int(off[i]), int(off[i + 1])) for i in range(self.L)]

    def copy(self) -> "LeveledGraph":
        return LeveledGraph(self.widths.copy(), self.epl.copy(), self.src.copy(),
                            self.dst.copy(), self.a.copy(), self.b.copy(),
                            self.k.copy(), dict(self.meta),
                            None if self.slot is None else self.slot.copy(),
                            None if self.coef is None else self.coef.copy(), self.n_slots)

    def with_lookup(self, slot, coef, n_slots: int) -> "LeveledGraph":
        """The same structure with lookup factors w_e = coef_e * T[slot_e]."""
        g = self.copy()
        g.slot = np.array(np.broadcast_to(slot, (g.n_edges,)), dtype=np.int32)
        g.coef = np.array(np.broadcast_to(coef, (g.n_edges,)), dtype=np.float64)
        g.n_slots = int(n_slots)
        return g

    def with_params(self, a=None, b=None, k=None) -> "LeveledGraph":
        g = self.copy()
        if a is not None:
            g.a = np.ascontiguousarray(np.broadcast_to(a, g.a.shape), dtype=np.float64)
        if b is not None:
            g.b = np.ascontiguousarray(np.broadcast_to(b, g.b.shape), dtype=np.float64)
        if k is not None:
            g.k = np.ascontiguousarray(np.broadcast_to(k, g.k.shape), dtype=np.float64)
        return g


def level_offsets(widths: np.ndarray) -> np.ndarray:
    """First global node id of each level (length L+2; last entry = node count)."""
    return np.concatenate([[0], np.cumsum(np.asarray(widths, dtype=np.int64))])


def _draw_distinct(rng: np.random.Generator, n_dst: int, n_src: int, d: int) -> np.ndarray:
    """Each of n_dst rows draws d distinct values uniformly from range(n_src)."""
    if d > n_src:
        raise ValueError(f"in-degree {d} exceeds previous width {n_src}")
    if n_dst * n_src <= (1 << 22):
        keys = rng.random((n_dst, n_src))
        # the d smallest keys per row, in key order (same result as a full argsort, in linear time)
        part = np.argpartition(keys, d - 1, axis=1)[:, :d] if d < n_src else np.tile(np.arange(n_src), (n_dst, 1))
        order = np.argsort(np.take_along_axis(keys, part, axis=1), axis=1)
        return np.take_along_axis(part, order, axis=1).astype(np.int64)
    out = rng.integers(0, n_src, size=(n_dst, d))
    while True:
        s = np.sort(out, axis=1)
        bad = np.any(s[:, 1:] == s[:, :-1], axis=1) if d > 1 else np.zeros(n_dst, bool)
        nb = int(bad.sum())
        if nb == 0:
            return out.astype(np.int64)
        out[bad] = rng.integers(0, n_src, size=(nb, d))


def _repair_coverage(rng: np.random.Generator, srcs: np.ndarray, n_src: int) -> None:
    """Give every previous-level node at least one out-edge, keeping in-degrees.

    Each uncovered source u (ascending id) replaces, in the list of a uniformly
    drawn destination that holds some source of out-degree >= 2, the source of
    largest out-degree (ties -> smallest id).  Feasible iff rows*d >= n_src.
    """
    n_dst, d = srcs.shape
    if n_dst * d < n_src:
        raise ValueError("W_l * d < W_{l-1}: cannot cover every source")
    outdeg = np.bincount(srcs.ravel(), minlength=n_src)
    for u in np.flatnonzero(outdeg == 0):
        while True:
            j = int(rng.integers(n_dst))
            row = srcs[j]
            od = outdeg[row]
            if od.max() >= 2:
                break
        victim = int(row[od == od.max()].min())
        pos = int(np.flatnonzero(row == victim)[0])
        row[pos] = u
        outdeg[victim] -= 1
        outdeg[u] += 1


def layered_graph(widths, degree, rng: np.random.Generator, order: str = "src",
                  cover: bool = True) -> LeveledGraph:
    """Random leveled DAG structure (parameters zero-filled).

    degree: int or per-edge-level sequence of interior in-degrees.  Each node of
    level l draws min(d_l, W_{l-1}) distinct sources from level l-1; the final
    node takes every node of level L-1 as a source (each previous-level node
    must have an out-edge and there is a single destination).  After the draw,
    uncovered sources are repaired (see _repair_coverage) unless cover=False,
    which leaves dead-end nodes in place.

    order: "src"  -> within a level, edges sorted by (src, dst) as in the
                     flattened arrays of the paper's figure;
           "shuffle" -> random order within each level.
    """
    widths = np.asarray(widths, dtype=np.int64)
    L = len(widths) - 1
    if L < 1 or widths[0] != 1 or widths[-1] != 1 or (widths < 1).any():
        raise ValueError("widths must be >= 1 with widths[0] = widths[L] = 1")
    degs = np.broadcast_to(np.asarray(degree, dtype=np.int64), (L,))
    off = level_offsets(widths)
    src_all, dst_all, epl = [], [], []
    for l in range(1, L + 1):
        n_src, n_dst = int(widths[l - 1]), int(widths[l])
        if l == L:
            d = n_src
            srcs = np.tile(np.arange(n_src, dtype=np.int64), (n_dst, 1))
        else:
            d = int(min(degs[l - 1], n_src))
            srcs = _draw_distinct(rng, n_dst, n_src, d)
            if cover:
                _repair_coverage(rng, srcs, n_src)
        dl = np.repeat(np.arange(n_dst, dtype=np.int64), d)
        sl = srcs.reshape(-1)
        if order == "src":
            perm = np.lexsort((dl, sl))
        elif order == "shuffle":
            perm = rng.permutation(len(sl))
        else:
            raise ValueError(order)
        src_all.append((sl[perm] + off[l - 1]).astype(np.int32))
        dst_all.append((dl[perm] + off[l]).astype(np.int32))
        epl.append(len(sl))
    src = np.concatenate(src_all)
    dst = np.concatenate(dst_all)
    E = len(src)
    return LeveledGraph(widths, np.asarray(epl, dtype=np.int64), src, dst,
                        np.zeros(E), np.zeros(E), np.zeros((E, 3)))


def draw_params(g: LeveledGraph, rng: np.random.Generator, a_range=(-1.0, 1.0),
                b_range=(0.5, 2.0), k_range=(-1.0, 1.0)) -> LeveledGraph:
    """Fill a ~ U[a_range], b ~ U[b_range], k ~ U[k_range]^3 in edge order."""
    E = g.n_edges
    g.a = rng.uniform(a_range[0], a_range[1], E)
    g.b = rng.uniform(b_range[0], b_range[1], E)
    g.k = rng.uniform(k_range[0], k_range[1], (E, 3))
    return g


def draw_lookup(g: LeveledGraph, rng: np.random.Generator, n_slots: int, p_minus: float = 0.5) -> LeveledGraph:
    """Lookup factors: each edge reads a uniformly drawn table entry (a vertex
    pair) and carries a sign, -1 with probability p_minus (closing a fermion
    loop), in edge order."""
    E = g.n_edges
    slot = rng.integers(0, n_slots, E)
    coef = np.where(rng.random(E) < p_minus, -1.0, 1.0)
    return g.with_lookup(slot, coef, n_slots)


def draw_table(n_slots: int, S: int, rng: np.random.Generator) -> np.ndarray:
    """Per-sample tables as structure-of-arrays float64[n_slots, S], entries U[-1, 1]
    (standing in for the Green's functions between the sample's vertices)."""
    return rng.uniform(-1.0, 1.0, (n_slots, S))


def draw_samples(S: int, dist: str, rng: np.random.Generator) -> np.ndarray:
    """Sample points x as structure-of-arrays float64[3, S]."""
    if dist == "uniform":
        return rng.uniform(-1.0, 1.0, (3, S))
    if dist == "normal":
        return rng.standard_normal((3, S))
    raise ValueError(dist)


def transpose(g: LeveledGraph) -> LeveledGraph:
    """Reverse every edge and swap root and final node.

    Node (level l, local i) maps to (level L-l, local i); an edge of edge level
    l becomes an edge of edge level L-l+1.  Root-to-final paths map one to one
    onto the reversed graph's paths with the same edge set, so the path sum is
    unchanged while the level recursion sums in a different structure.
    """
    L = g.L
    widths_t = g.widths[::-1].copy()
    off = level_offsets(g.widths)
    off_t = level_offsets(widths_t)
    level_of = np.repeat(np.arange(L + 1), g.widths)
    out_src, out_dst, out_idx, epl = [], [], [], []
    sl = g.level_slices()
    for lt in range(1, L + 1):
        l = L - lt + 1  # original edge level
        s = sl[l - 1]
        u, v = g.src[s].astype(np.int64), g.dst[s].astype(np.int64)
        lu, lv = level_of[u], level_of[v]
        nu = (v - off[lv]) + off_t[L - lv]
        nv = (u - off[lu]) + off_t[L - lu]
        out_src.append(nu.astype(np.int32))
        out_dst.append(nv.astype(np.int32))
        out_idx.append(np.arange(s.start, s.stop))
        epl.append(s.stop - s.start)
    idx = np.concatenate(out_idx)
    return LeveledGraph(widths_t, np.asarray(epl, dtype=np.int64),
                        np.concatenate(out_src), np.concatenate(out_dst),
                        g.a[idx].copy(), g.b[idx].copy(), g.k[idx].copy(), dict(g.meta),
                        None if g.slot is None else g.slot[idx].copy(),
                        None if g.coef is None else g.coef[idx].copy(), g.n_slots)
