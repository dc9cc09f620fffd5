"""Monte Carlo over sample configurations -- TEST INFRASTRUCTURE ONLY.

The paper integrates the diagram sum over the vertex coordinates by Monte
Carlo sampling (Sec. II.B), runs the many Markov-chain walkers as the many
configurations evaluated at once (Sec. II.C, "Distributing the task on a grid
of blocks"), and does proposal and acceptance on the device (Sec. IV).  It
does not fix the chain; this module writes out the one the library runs, step
by step, with the level sweep from the C oracle:

  walker c, step t (global step index), key (seed, 0), counter (c, t, 0, 0):
    r0..r3 = Philox4x64-10(counter, key)       (Salmon et al., SC'11)
    u_i    = (r_i >> 11) * 2^-53               (exact binary64 in [0, 1))
    x'_i   = x_i + sigma * (2 u_i - 1), i < 3   (product rounded, then the sum)
    v'     = V(x')                             (the level sweep)
    accept iff u_3 * |v| < |v'|                (Metropolis for the density |V|)
    then, at the walker's current state (x, v):
      acc[0] += sign(v),  acc[1] += |x|^2,  accepted += (1 if accepted)

Only the test suite may import this module.
"""

from __future__ import annotations

import numpy as np

from . import sweep

# Philox4x64-10 (multipliers and Weyl key increments of the published definition)
PHILOX_M = (0xD2E7470EE14C6C93, 0xCA5A826395121157)
PHILOX_W = (0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B)
_M32 = np.uint64(0xFFFFFFFF)


def _mulhilo(a: int, b: np.ndarray):
    """(hi, lo) 64-bit halves of the 128-bit products a * b (b uint64 array)."""
    a_lo, a_hi = np.uint64(a & 0xFFFFFFFF), np.uint64(a >> 32)
    b_lo, b_hi = b & _M32, b >> np.uint64(32)
    ll, lh, hl, hh = a_lo * b_lo, a_lo * b_hi, a_hi * b_lo, a_hi * b_hi
    mid = (ll >> np.uint64(32)) + (lh & _M32) + (hl & _M32)
    lo = (ll & _M32) | ((mid & _M32) << np.uint64(32))
    hi = hh + (lh >> np.uint64(32)) + (hl >> np.uint64(32)) + (mid >> np.uint64(32))
    return hi, lo


def philox4x64(c0, c1, c2, c3, k0: int, k1: int, rounds: int = 10):
    """Philox4x64 on arrays of counters (uint64), one key: the four output words."""
    c = [np.asarray(v, dtype=np.uint64).copy() for v in (c0, c1, c2, c3)]
    k0, k1 = int(k0) & 0xFFFFFFFFFFFFFFFF, int(k1) & 0xFFFFFFFFFFFFFFFF
    with np.errstate(over="ignore"):
        for r in range(rounds):
            if r:
                k0 = (k0 + PHILOX_W[0]) & 0xFFFFFFFFFFFFFFFF
                k1 = (k1 + PHILOX_W[1]) & 0xFFFFFFFFFFFFFFFF
            hi0, lo0 = _mulhilo(PHILOX_M[0], c[0])
            hi1, lo1 = _mulhilo(PHILOX_M[1], c[2])
            c = [hi1 ^ c[1] ^ np.uint64(k0), lo1, hi0 ^ c[3] ^ np.uint64(k1), lo0]
    return c


def uniforms(seed: int, step: int, C: int):
    """The four uniforms in [0, 1) of every walker at one step: float64[4, C]."""
    r = philox4x64(np.arange(C, dtype=np.uint64), np.full(C, step, dtype=np.uint64), np.zeros(C, np.uint64),
                   np.zeros(C, np.uint64), seed, 0)
    return np.stack([(w >> np.uint64(11)).astype(np.float64) * 2.0 ** -53 for w in r])


def run(g, x, v, step0: int, n_steps: int, seed: int, sigma: float, accepted=None, acc=None):
    """n_steps Metropolis steps of every walker from global step step0.

    x float64[3, C] and v float64[C] (v = V(x)) are the walkers' states; returns
    (x, v, accepted int64[C], acc float64[2, C]) with the accumulators continued
    from the given ones (zeros when None).
    """
    x = np.array(x, dtype=np.float64)
    v = np.array(v, dtype=np.float64)
    C = x.shape[1]
    accepted = np.zeros(C, np.int64) if accepted is None else np.array(accepted, dtype=np.int64)
    acc = np.zeros((2, C)) if acc is None else np.array(acc, dtype=np.float64)
    for t in range(step0, step0 + n_steps):
        u = uniforms(seed, t, C)
        xp = x + sigma * (2.0 * u[:3] - 1.0)
        vp = sweep(g, xp)
        take = u[3] * np.abs(v) < np.abs(vp)
        x[:, take] = xp[:, take]
        v[take] = vp[take]
        accepted += take
        acc[0] += np.sign(v)
        acc[1] += x[0] * x[0] + x[1] * x[1] + x[2] * x[2]
    return x, v, accepted, acc

