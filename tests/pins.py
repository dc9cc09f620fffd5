"""Pins for the CPU oracle: facts fixed independently of the oracle itself.

Each pin takes a loaded oracle library (so that deliberately broken builds of
the oracle can be run through the same checks) and raises AssertionError when
the oracle disagrees with:

  * the path count of the paper's flattening figure (golden fixture),
  * the exact rational sum over every path (the definition, Sec. II.B),
  * the closed form of level-constant factors on in-regular graphs,
  * exact path counts Prod_l d_l of in-regular graphs with unit factors,
  * transpose invariance V(G) = V(G^T),
  * exact power-of-two scaling and negation of one level;

and the same facts for lookup factors w_e = c_e T[slot_e] (the paper's Green's
function per vertex pair times a fermion-loop sign), plus exact invariance
under a relabelling of the table entries.

Error bounds use the standard model fl(a op b) = (a op b)(1 + d), |d| <= u:
the factor takes <= 8 roundings and a level adds one product and at most d_l
summands, so |V_oracle - V| <= gamma_K * A with K = sum_l (9 + d_l) and A the
exact 1-norm of the path terms.
"""

from __future__ import annotations

import math
import os
from fractions import Fraction

import numpy as np

import oracle
from oracle.path_sum import path_count, path_sum
from workloads import LeveledGraph, layered_graph, level_offsets, make_config, transpose

U = 2.0 ** -53
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def gamma(K: int) -> float:
    return K * U / (1 - K * U)


def load_figure_graph():
    """The L=4 instantiation of Fig. combinedgraphflat and its stated path count."""
    widths, edges, expect = None, {}, None
    with open(os.path.join(GOLDEN, "paper_figure_L4.txt")) as f:
        for line in f:
            line = line.split("#", 1)[0].split()
            if not line:
                continue
            if line[0] == "widths":
                widths = [int(v) for v in line[1:]]
            elif line[0] == "edges":
                vals = [int(v) for v in line[2:]]
                edges[int(line[1])] = list(zip(vals[0::2], vals[1::2]))
            elif line[0] == "expect_paths":
                expect = int(line[1])
    L = len(widths) - 1
    pairs = [p for l in range(1, L + 1) for p in edges[l]]
    E = len(pairs)
    g = LeveledGraph(np.array(widths, dtype=np.int64),
                     np.array([len(edges[l]) for l in range(1, L + 1)], dtype=np.int64),
                     np.array([p[0] for p in pairs], dtype=np.int32),
                     np.array([p[1] for p in pairs], dtype=np.int32),
                     np.ones(E), np.zeros(E), np.zeros((E, 3)))
    return g, expect


def max_in_degrees(g) -> list:
    out = []
    for sl in g.level_slices():
        d = g.dst[sl]
        out.append(int(np.bincount(d - d.min()).max()) if len(d) else 0)
    return out


def error_K(g) -> int:
    return sum(9 + d for d in max_in_degrees(g))


def dyadic(rng, shape, lo, hi, bits=6):
    """Uniform multiples of 2^-bits in [lo, hi] (exact in binary64)."""
    q = 2 ** bits
    return rng.integers(int(lo * q), int(hi * q) + 1, shape).astype(np.float64) / q


def dyadic_params(g, rng):
    E = g.n_edges
    return g.with_params(a=dyadic(rng, E, -1, 1), b=dyadic(rng, E, 0, 2), k=dyadic(rng, (E, 3), -1, 1))


def random_small_graph(rng, max_paths=4000):
    """Random leveled DAG (random widths, in-degrees, parallel-free) with few paths."""
    while True:
        L = int(rng.integers(1, 7))
        widths = [1] + [int(v) for v in rng.integers(1, 5, L - 1)] + [1]
        deg = [int(v) for v in rng.integers(1, 4, L)]
        cover = bool(rng.random() < 0.7)
        if cover:  # every previous-level node needs room for an out-edge
            deg = [max(d, -(-widths[l] // widths[l + 1])) for l, d in enumerate(deg)]
        g = layered_graph(widths, deg, rng, order="shuffle", cover=cover)
        if path_count(g) <= max_paths:
            return dyadic_params(g, rng)


# ---------------------------------------------------------------- the pins


def pin_paper_figure(lib):
    g, expect = load_figure_graph()
    assert expect == 6
    assert path_count(g) == expect
    x = np.random.default_rng(0).uniform(-1, 1, (3, 5))
    v = oracle.sweep(g, x, lib=lib)
    assert np.all(v == expect), v


def pin_exact_path_sum(lib, n_random=12, n_samples=3, seed=11):
    rng = np.random.default_rng(seed)
    fig, _ = load_figure_graph()
    tiny, _ = make_config("tiny", S=4)
    graphs = [dyadic_params(fig, rng), dyadic_params(tiny, rng)]
    graphs += [random_small_graph(rng) for _ in range(n_random)]
    for g in graphs:
        x = dyadic(rng, (3, n_samples), -1, 1)
        V = oracle.sweep(g, x, "value", lib=lib)
        A = oracle.sweep(g, x, "abs", lib=lib)
        Q = oracle.sweep(g, x, "square", lib=lib)
        tol = gamma(error_K(g))
        for j in range(n_samples):
            ex_v = path_sum(g, x[:, j])
            ex_a = path_sum(g, x[:, j], weight=abs)
            ex_q = path_sum(g, x[:, j], weight=lambda w: w * w)
            bound = Fraction(tol) * ex_a
            assert abs(Fraction(float(V[j])) - ex_v) <= bound, (g.widths, j, V[j], float(ex_v))
            assert abs(Fraction(float(A[j])) - ex_a) <= bound, (g.widths, j, A[j], float(ex_a))
            assert abs(Fraction(float(Q[j])) - ex_q) <= Fraction(tol) * ex_q, (g.widths, j, Q[j], float(ex_q))


def level_constant_graph(g, rng):
    """Same structure, every edge of level l gets the level's (a_l, b_l, k_l)."""
    L = g.L
    al = rng.uniform(-1, 1, L)
    bl = rng.uniform(0.1, 4.0, L)
    kl = rng.uniform(-1, 1, (L, 3))
    lev = np.repeat(np.arange(L), g.epl)
    return g.with_params(a=al[lev], b=bl[lev], k=kl[lev]), (al, bl, kl)


def in_degrees(g) -> list:
    """Per-level in-degree of an in-regular graph (asserts regularity)."""
    out = []
    for sl in g.level_slices():
        c = np.bincount(g.dst[sl] - g.dst[sl].min())
        assert c.min() == c.max(), "not in-regular"
        out.append(int(c[0]))
    return out


def pin_level_constant_closed_form(lib, seed=21):
    rng = np.random.default_rng(seed)
    for name, S in (("tiny", 64), ("mid", 64), ("precision", 8)):
        g, x = make_config(name, S=S)
        d = in_degrees(g)
        gc, (al, bl, kl) = level_constant_graph(g, rng)
        v = oracle.sweep(gc, x, lib=lib)
        # V(x) = prod_l d_l a_l / (1 + b_l |x - k_l|^2)
        cf = np.ones(S)
        for l in range(g.L):
            r2 = ((x - kl[l][:, None]) ** 2).sum(axis=0)
            cf = cf * (d[l] * al[l] / (1.0 + bl[l] * r2))
        tol = gamma(error_K(g)) + gamma(10 * g.L)
        rel = np.abs(v - cf) / np.abs(cf)
        assert rel.max() <= tol, (name, rel.max(), tol)


def pin_all_ones_counts(lib, include_large=False):
    names = ["tiny", "mid", "precision"] + (["large"] if include_large else [])
    expect = {"tiny": 1 * 2 * 2 * 3, "mid": 4 ** 10 * 256, "precision": 8 ** 22 * 4096,
              "large": 6 ** 30 * 65536}
    for name in names:
        g, x = make_config(name, S=2)
        g1 = g.with_params(a=1.0, b=0.0, k=0.0)
        assert math.prod(in_degrees(g)) == expect[name]
        v = oracle.sweep(g1, x, lib=lib)
        if name == "large":
            # partial sums m * 6^30 of the final 65536-way sum exceed 53 bits
            err = np.abs(v - float(expect[name])) / float(expect[name])
            assert err.max() <= gamma(error_K(g)), (name, v, expect[name])
        else:
            assert np.all(v == float(expect[name])), (name, v, expect[name])


def pin_transpose(lib, seed=31):
    for name, S in (("tiny", 32), ("mid", 32)):
        g, x = make_config(name, S=S, seed=seed)
        gt = transpose(g)
        assert gt.n_edges == g.n_edges and list(gt.widths) == list(g.widths[::-1])
        v, q = oracle.sweep(g, x, lib=lib), oracle.sweep(g, x, "square", lib=lib)
        vt, qt = oracle.sweep(gt, x, lib=lib), oracle.sweep(gt, x, "square", lib=lib)
        err = oracle.scaled_error(vt, v, q)
        assert err.max() <= 1e-13, (name, err.max())
        assert np.abs(qt - q).max() <= 1e-13 * q.max()


def pin_pow2_scaling(lib, seed=41):
    g, x = make_config("mid", S=16, seed=seed)
    v = oracle.sweep(g, x, lib=lib)
    lev = np.repeat(np.arange(g.L), g.epl)
    for l, f in ((3, 8.0), (g.L - 1, 0.25), (0, -1.0)):
        a = g.a.copy()
        a[lev == l] *= f
        vs = oracle.sweep(g.with_params(a=a), x, lib=lib)
        assert np.array_equal(vs, v * f), (l, f)


# ---------------------------------------------------------------- lookup factors
# w_e = c_e * T[slot_e]: one rounding per factor, so the rational bound
# gamma_K (K = sum_l (9 + d_l)) holds with room to spare.


def dyadic_lookup(g, rng, n_slots):
    """Lookup factors with dyadic constants (signs and halves) on g's structure."""
    E = g.n_edges
    coef = dyadic(rng, E, -1, 1, bits=1)
    coef[coef == 0] = 1.0
    return g.with_lookup(rng.integers(0, n_slots, E), coef, n_slots)


def pin_lookup_exact_path_sum(lib, n_random=10, n_samples=3, seed=51):
    rng = np.random.default_rng(seed)
    fig, _ = load_figure_graph()
    tiny, _ = make_config("tiny", S=4)
    graphs = [dyadic_lookup(fig, rng, 5), dyadic_lookup(tiny, rng, 4)]
    graphs += [dyadic_lookup(random_small_graph(rng), rng, int(rng.integers(1, 9))) for _ in range(n_random)]
    for g in graphs:
        T = dyadic(rng, (g.n_slots, n_samples), -1, 1)
        V = oracle.sweep(g, T, "value", lib=lib)
        A = oracle.sweep(g, T, "abs", lib=lib)
        Q = oracle.sweep(g, T, "square", lib=lib)
        tol = gamma(error_K(g))
        for j in range(n_samples):
            ex_v = path_sum(g, T[:, j])
            ex_a = path_sum(g, T[:, j], weight=abs)
            ex_q = path_sum(g, T[:, j], weight=lambda w: w * w)
            bound = Fraction(tol) * ex_a
            assert abs(Fraction(float(V[j])) - ex_v) <= bound, (g.widths, j, V[j], float(ex_v))
            assert abs(Fraction(float(A[j])) - ex_a) <= bound, (g.widths, j, A[j], float(ex_a))
            assert abs(Fraction(float(Q[j])) - ex_q) <= Fraction(tol) * ex_q, (g.widths, j, Q[j], float(ex_q))


def pin_lookup_level_constant(lib, seed=61):
    """Every edge of level l reads slot s_l with constant c_l: V = prod_l d_l c_l T[s_l]."""
    rng = np.random.default_rng(seed)
    for name, S in (("tiny", 64), ("mid", 64), ("precision", 8)):
        g, _ = make_config(name, S=S)
        d = in_degrees(g)
        n_slots = 7
        sl = rng.integers(0, n_slots, g.L)
        cl = rng.uniform(-2, 2, g.L)
        lev = np.repeat(np.arange(g.L), g.epl)
        gl = g.with_lookup(sl[lev], cl[lev], n_slots)
        T = rng.uniform(-1, 1, (n_slots, S))
        v = oracle.sweep(gl, T, lib=lib)
        cf = np.ones(S)
        for l in range(g.L):
            cf = cf * (d[l] * cl[l] * T[sl[l]])
        tol = gamma(error_K(g)) + gamma(2 * g.L)
        rel = np.abs(v - cf) / np.abs(cf)
        assert rel.max() <= tol, (name, rel.max(), tol)


def pin_lookup_all_ones(lib):
    expect = {"tiny": 12, "mid": 4 ** 10 * 256, "precision": 8 ** 22 * 4096}
    for name, count in expect.items():
        g, _ = make_config(name, S=2)
        g1 = g.with_lookup(0, 1.0, 3)
        T = np.array([[1.0, 1.0], [5.0, -3.0], [0.0, 7.0]])  # only slot 0 is read
        v = oracle.sweep(g1, T, lib=lib)
        assert np.all(v == float(count)), (name, v, count)


def pin_lookup_sign_and_scale(lib, seed=71):
    """Negating or scaling by 2^k the constants of one level does the same to V, exactly;
    permuting the table rows along with the slots leaves V unchanged, exactly."""
    g, _ = make_config("mid", S=16, seed=seed, factor="lookup")
    rng = np.random.default_rng(seed)
    T = rng.uniform(-1, 1, (g.n_slots, 16))
    v = oracle.sweep(g, T, lib=lib)
    lev = np.repeat(np.arange(g.L), g.epl)
    for l, f in ((2, -1.0), (g.L - 1, 4.0), (0, 0.5)):
        c = g.coef.copy()
        c[lev == l] *= f
        vs = oracle.sweep(g.with_lookup(g.slot, c, g.n_slots), T, lib=lib)
        assert np.array_equal(vs, v * f), (l, f)
    perm = rng.permutation(g.n_slots)
    inv = np.argsort(perm)
    vp = oracle.sweep(g.with_lookup(inv[g.slot], g.coef, g.n_slots), T[perm], lib=lib)
    assert np.array_equal(vp, v)


def pin_lookup_transpose(lib, seed=81):
    for name, S in (("tiny", 32), ("mid", 32)):
        g, T = make_config(name, S=S, seed=seed, factor="lookup")
        gt = transpose(g)
        v, q = oracle.sweep(g, T, lib=lib), oracle.sweep(g, T, "square", lib=lib)
        vt = oracle.sweep(gt, T, lib=lib)
        err = oracle.scaled_error(vt, v, q)
        assert err.max() <= 1e-13, (name, err.max())


ALL_PINS = [pin_paper_figure, pin_exact_path_sum, pin_level_constant_closed_form,
            pin_all_ones_counts, pin_transpose, pin_pow2_scaling, pin_lookup_exact_path_sum,
            pin_lookup_level_constant, pin_lookup_all_ones, pin_lookup_sign_and_scale, pin_lookup_transpose]
