"""The Monte Carlo oracle: its counter-based generator and its Metropolis chain (no GPU)."""

import numpy as np
import pytest

import oracle
from oracle import mc
from workloads import make_config


@pytest.mark.parametrize("ctr,key", [((0, 0, 0, 0), (0, 0)), ((5, 7, 11, 13), (123, 456)),
                                     ((2 ** 64 - 1,) * 4, (2 ** 64 - 1,) * 2),
                                     ((2 ** 63 + 1, 3, 2 ** 40, 9), (0x9E3779B97F4A7C15, 1))])
def test_philox_matches_numpy(ctr, key):
    # numpy's Philox is Philox4x64-10; it advances its 256-bit counter before each block
    v = (sum(c << (64 * i) for i, c in enumerate(ctr)) - 1) % (1 << 256)
    bg = np.random.Philox(counter=np.array([(v >> (64 * i)) & (2 ** 64 - 1) for i in range(4)], dtype=np.uint64),
                          key=np.array(key, dtype=np.uint64))
    ref = [int(bg.random_raw()) for _ in range(4)]
    out = mc.philox4x64(*[np.array([c], dtype=np.uint64) for c in ctr], *key)
    assert [int(w[0]) for w in out] == ref


def test_uniforms_are_53_bit_grid_values_in_unit_interval():
    u = mc.uniforms(seed=3, step=11, C=4096)
    assert u.shape == (4, 4096)
    assert np.all((u >= 0) & (u < 1))
    assert np.all(u * 2.0 ** 53 == np.floor(u * 2.0 ** 53))
    assert abs(u.mean() - 0.5) < 0.01


def test_zero_step_accepts_every_proposal():
    g, x = make_config("tiny", S=64)
    v = oracle.sweep(g, x)
    x2, v2, n, acc = mc.run(g, x, v, 0, 5, seed=1, sigma=0.0)
    assert np.array_equal(x2, x) and np.array_equal(v2, v)
    assert np.all(n == 5) and np.array_equal(acc[0], 5 * np.sign(v))


def test_resume_and_walker_independence():
    g, x = make_config("tiny", S=48)
    v = oracle.sweep(g, x)
    whole = mc.run(g, x, v, 0, 20, seed=9, sigma=0.7)
    a = mc.run(g, x, v, 0, 12, seed=9, sigma=0.7)
    b = mc.run(g, a[0], a[1], 12, 8, seed=9, sigma=0.7, accepted=a[2], acc=a[3])
    for p, q in zip(whole, b):
        assert np.array_equal(p, q)
    # walker c's chain depends only on (seed, c, step): the first 16 walkers alone agree
    part = mc.run(g, x[:, :16], v[:16], 0, 20, seed=9, sigma=0.7)
    assert np.array_equal(part[0], whole[0][:, :16]) and np.array_equal(part[2], whole[2][:16])


def quadrature(g, h=0.1, R=10.0):
    """(int V, int |V|, int |x|^2 |V|) over the cube [-R, R]^3 by the midpoint rule."""
    ax = np.arange(-R + h / 2, R, h)
    out = np.zeros(3)
    for i0 in range(0, len(ax), 20):
        X0, X1, X2 = np.meshgrid(ax[i0:i0 + 20], ax, ax, indexing="ij")
        xs = np.ascontiguousarray(np.stack([X0.ravel(), X1.ravel(), X2.ravel()]))
        V = oracle.sweep(g, xs)
        out += [V.sum(), np.abs(V).sum(), (np.sum(xs * xs, axis=0) * np.abs(V)).sum()]
    return out * h ** 3


def test_chain_samples_the_density_abs_v():
    # Metropolis for |V|: <sign V> = int V / int |V| and <|x|^2> = int |x|^2 |V| / int |V|.
    # The tiny graph's V changes sign (<sign> ~ -0.49), so a chain for another
    # density (V^2, uniform, 1/|V|) would miss both by far more than the bar.
    g, x = make_config("tiny", S=256)
    I = quadrature(g)
    v = oracle.sweep(g, x)
    xb, vb, _, _ = mc.run(g, x, v, 0, 500, seed=7, sigma=1.0)  # burn-in
    _, _, n, acc = mc.run(g, xb, vb, 500, 3000, seed=7, sigma=1.0)
    per_walker = acc / 3000  # walkers are independent: their spread gives the standard error
    se = per_walker.std(axis=1) / np.sqrt(x.shape[1])
    est = per_walker.mean(axis=1)
    assert abs(est[0] - I[0] / I[1]) <= 5 * se[0] + 5e-3
    assert abs(est[1] - I[2] / I[1]) <= 5 * se[1] + 1e-2
    assert 0.2 < n.mean() / 3000 < 0.8
