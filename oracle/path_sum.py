"""Exact path-sum definition of the diagram sum -- TEST INFRASTRUCTURE ONLY.

The value at the final node is, by definition, the sum over every path from the
root to the final node of the product of the edge factors along it (paper Sec.
II.B: each unique path through the graph is one diagram; caption of Fig.
``diagrams-graph``).  This module writes that definition out literally, in
exact rational arithmetic, by enumerating every path.  It is exponential in
the depth and is meant for graphs with at most ~1e4 paths.

Inputs given as binary64 are converted exactly (every finite double is a
dyadic rational), so the result is the exact value of the sum for those inputs.
"""

from __future__ import annotations

from fractions import Fraction


def edge_factor_exact(a, b, k, x) -> Fraction:
    """w(x) = a / (1 + b |x - k|^2) in exact rationals."""
    r2 = sum((Fraction(float(x[c])) - Fraction(float(k[c]))) ** 2 for c in range(3))
    return Fraction(float(a)) / (1 + Fraction(float(b)) * r2)


def lookup_factor_exact(coef, slot, table_col) -> Fraction:
    """w = c * T[slot] (the sample's table entry for the edge's vertex pair) in exact rationals."""
    return Fraction(float(coef)) * Fraction(float(table_col[int(slot)]))


def enumerate_paths(g):
    """All root-to-final paths as lists of edge indices (depth-first)."""
    out_edges = {}
    for e in range(g.n_edges):
        out_edges.setdefault(int(g.src[e]), []).append(e)
    final = g.final_node
    paths = []
    stack = [(0, [])]
    while stack:
        node, path = stack.pop()
        if node == final:
            paths.append(path)
            continue
        for e in out_edges.get(node, []):
            stack.append((int(g.dst[e]), path + [e]))
    return paths


def path_sum(g, x_col, weight=None):
    """Exact V = sum over paths of prod_e w_e for one sample: x_col = (x0, x1, x2)
    for rational factors, or the sample's table column (n_slots values) for
    lookup factors.

    weight: optional function Fraction -> Fraction applied to each factor
    (abs for the 1-norm, square for the squared 2-norm).
    """
    if getattr(g, "slot", None) is not None:
        w = [lookup_factor_exact(g.coef[e], g.slot[e], x_col) for e in range(g.n_edges)]
    else:
        w = [edge_factor_exact(g.a[e], g.b[e], g.k[e], x_col) for e in range(g.n_edges)]
    if weight is not None:
        w = [weight(v) for v in w]
    total = Fraction(0)
    for path in enumerate_paths(g):
        term = Fraction(1)
        for e in path:
            term *= w[e]
        total += term
    return total


def path_count(g) -> int:
    return len(enumerate_paths(g))
