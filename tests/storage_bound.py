"""Error bound of the 16-bit level storage precisions (fp16r, bf16r), from the oracle.

The library's 16-bit paths compute every interior level in binary32 (edge
factors from binary32 parameters, sums by fused multiply-add in canonical
edge order), scale the level by a power of two, round it to the storage
format and widen it again on read; the final node is summed in binary64.

An error e_n made at interior node n reaches the final node multiplied by
G_n, the (signed) sum over the paths from n to the final node; to first order
y - V = sum_n e_n G_n.  With v_n the node's value (sum over root-to-n paths),
the errors at node n of level l are bounded by

  storage       b_n = u |v_n| + (s/2) 2^h_l M_{l-1}     (s/2: half the smallest
                subnormal spacing, 2^h_l M_{l-1} a bound on the level's scale:
                h_l the binary16 headroom, M_{l-1} the largest |v| of level l-1)
  accumulation  c_n = d_n 2^-24 R_n                     (d_n in-edges, R_n = sum_e |w_e v_src|)
  factors       f_n = eps_w R_n                         (eps_w: one binary32 factor)

u is the storage format's unit roundoff (2^-11 binary16, 2^-8 bfloat16).
Rounding to nearest makes b_n and c_n mean-zero errors; modelled as
independent (the probabilistic rounding-error model of Higham and Mary, SIAM
J. Sci. Comput. 41 (2019)), Hoeffding's inequality gives

  |y - V| <= lambda sqrt(sum_n (b_n + c_n)^2 G_n^2) + sum_n f_n |G_n|

except with probability 2 exp(-lambda^2 / 2) per sample (2e-14 at lambda = 8).
The factor errors may be systematic (the reciprocal's bias, the rounding of
x shared by all edges) and are summed linearly.  The worst-case first-order
bound sum_n (b_n + c_n + f_n) |G_n| is reported beside it.  Both carry a
factor 1 + 2(L-1)u for higher-order terms.  v_n and G_n are the oracle's node
values of the graph and of its transpose.

eps_w for the rational factor a / (1 + b |x - k|^2): the binary32 roundings of
x and k perturb r = x - k by about (|x| + |k|) 2^-24 per component, which moves
D = 1 + b |r|^2 by at most sqrt(b) * 3 (||x||_1 + ||k||_1) 2^-24 relative; the
remaining roundings (|r|^2, D, the 1.5-ulp reciprocal, the product and a's own
rounding) add below 16 * 2^-24.  For lookup factors coef * T: three roundings.
"""

from __future__ import annotations

import numpy as np

import oracle
from workloads import LeveledGraph, transpose
from workloads.graphs import level_offsets

LAMBDA = 8.0
# unit roundoff, smallest subnormal spacing
FORMATS = {"fp16r": (2.0 ** -11, 2.0 ** -24), "bf16r": (2.0 ** -8, 2.0 ** -133)}


def edge_factors(g: LeveledGraph, x: np.ndarray, sl: slice) -> np.ndarray:
    """w_e(x_s) in binary64 for the edges of slice sl: float64[edges, S]."""
    if g.slot is None:
        k = g.k[sl]
        r2 = sum((x[c][None, :] - k[:, c:c + 1]) ** 2 for c in range(3))
        return g.a[sl][:, None] / (1.0 + g.b[sl][:, None] * r2)
    return g.coef[sl][:, None] * x[g.slot[sl]]


def headroom16(g: LeveledGraph) -> np.ndarray:
    """h_l = max(0, ceil(log2 R_l) - 14), R_l the largest row sum of |a_e| into node level l."""
    off = level_offsets(g.widths)
    h = np.zeros(g.L, np.int64)
    for l, sl in enumerate(g.level_slices()[:-1], start=1):
        R = np.zeros(int(g.widths[l]))
        np.add.at(R, g.dst[sl] - off[l], np.abs(g.a[sl]))
        top = float(R.max()) if len(R) else 0.0
        if top > 0:
            m, e = np.frexp(top)
            h[l] = max(0, (e - 1 if m == 0.5 else e) - 14)
    return h


def factor_eps(g: LeveledGraph, x: np.ndarray) -> float:
    if g.slot is not None:
        return 4 * 2.0 ** -24
    xn = float(np.max(np.sum(np.abs(x), axis=0))) if x.size else 0.0
    kn = float(np.max(np.sum(np.abs(g.k), axis=1))) if len(g.k) else 0.0
    bm = float(np.max(g.b)) if len(g.b) else 0.0
    return (3.0 * np.sqrt(bm) * (xn + kn) + 16.0) * 2.0 ** -24


def _headroom(g, precision):
    return headroom16(g) if (precision == "fp16r" and g.slot is None) else np.zeros(g.L, np.int64)


def storage_bound(g: LeveledGraph, x: np.ndarray, precision: str, lam: float = LAMBDA):
    """(B, B_first, V): the probabilistic bound, the worst-case first-order bound
    and the oracle value, per sample (see the module docstring)."""
    u, sub = FORMATS[precision]
    L, S = g.L, x.shape[1]
    v = oracle.node_values(g, x)
    t = oracle.node_values(transpose(g), x)
    off, off_t = level_offsets(g.widths), level_offsets(g.widths[::-1])
    h = _headroom(g, precision)
    eps = factor_eps(g, x)
    rand2, lin, first = np.zeros(S), np.zeros(S), np.zeros(S)
    for l, sl in enumerate(g.level_slices()[:-1], start=1):
        W = int(g.widths[l])
        dl = g.dst[sl] - off[l]
        w = edge_factors(g, x, sl)
        R = np.zeros((W, S))
        np.add.at(R, dl, np.abs(w) * np.abs(v[g.src[sl]]))
        deg = np.bincount(dl, minlength=W)[:, None]
        vl = v[off[l]:off[l + 1]]
        Gl = np.abs(t[off_t[L - l]:off_t[L - l + 1]])  # (level l, i) <-> transposed (level L-l, i)
        Mprev = np.max(np.abs(v[off[l - 1]:off[l]]), axis=0)
        b = u * np.abs(vl) + 0.5 * sub * 2.0 ** float(h[l]) * Mprev * (1 + 2.0 ** -10)
        c = deg * 2.0 ** -24 * R
        f = eps * R
        rand2 += np.sum(((b + c) * Gl) ** 2, axis=0)
        lin += np.sum(f * Gl, axis=0)
        first += np.sum((b + c + f) * Gl, axis=0)
    V = v[-1]
    hi = 1 + 2 * (L - 1) * u
    final = 1e-13 * np.abs(V)  # binary64 final node
    return (lam * np.sqrt(rand2) + lin) * hi + final, first * hi + final, V


def _round_storage(z: np.ndarray, precision: str) -> np.ndarray:
    """Round binary64 values to the storage format, through binary32 (round to nearest even)."""
    if precision == "fp16r":
        return z.astype(np.float32).astype(np.float16).astype(np.float64)
    b = np.ascontiguousarray(z.astype(np.float32)).view(np.uint32)
    b = (b + np.uint32(0x7FFF) + ((b >> np.uint32(16)) & np.uint32(1))) & np.uint32(0xFFFF0000)
    return b.view(np.float32).astype(np.float64)


def emulate_storage(g: LeveledGraph, x: np.ndarray, precision: str) -> np.ndarray:
    """The 16-bit storage scheme in binary64 arithmetic (a test double for the
    bound, not a reference for the library): level l is scaled by
    2^-(h_l + ilogb(largest scaled |value| of level l-1)) and rounded."""
    L, S = g.L, x.shape[1]
    off = level_offsets(g.widths)
    h = _headroom(g, precision)
    prev = np.ones((1, S))
    E = np.zeros(S)
    top = np.ones(S)  # largest |scaled value| of the previous level
    for l, sl in enumerate(g.level_slices(), start=1):
        w = edge_factors(g, x, sl)
        cur = np.zeros((int(g.widths[l]), S))
        np.add.at(cur, g.dst[sl] - off[l], w * prev[g.src[sl] - off[l - 1]])
        if l == L:
            return cur[0] * np.exp2(E)
        with np.errstate(divide="ignore"):
            esh = np.where(top > 0, np.floor(np.log2(np.where(top > 0, top, 1.0))), 0.0) + h[l]
        z = cur * np.exp2(-esh)
        E += esh
        top = np.max(np.abs(z), axis=0)
        prev = _round_storage(z, precision)
    return prev[0]
