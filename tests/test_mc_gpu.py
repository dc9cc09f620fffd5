"""Monte Carlo walkers on the GPU (cos_mc_run) against the oracle's chain.

Given the same generator outputs, proposals are bit-identical on both sides
(the same IEEE operations, unfused), and an acceptance could only differ if
u_3 |v| fell within the sweeps' last-bit difference of |v'| (probability
~1e-15 per decision).  So the chains must agree exactly: positions, accepted
counts and both sums; the walkers' values agree with the oracle's to the
FP64 parity bar.
"""

import numpy as np
import pytest
import torch

import oracle
from gpu_util import TOL, say, to_dev
from oracle import mc
from test_mc_oracle import quadrature
from workloads import make_config

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2501_00675_amd as P

    assert torch.cuda.is_available()
    return P


def walk(P, g, x, steps, seed, sigma, precision="fp64", path="auto", split=None):
    G = P.Graph.from_leveled(g).set_path(path)
    W = P.Walkers(G, to_dev(x), precision, seed=seed, sigma=sigma)
    for n in (split or [steps]):
        W.run(n)
    torch.cuda.synchronize()
    return (W.x.cpu().numpy(), W.v.cpu().numpy(), W.accepted.cpu().numpy(), W.acc.cpu().numpy()), W


@pytest.mark.parametrize("name,C,steps,sigma", [("tiny", 300, 40, 0.8), ("mid", 1000, 8, 0.5)])
def test_chain_matches_oracle(P, name, C, steps, sigma):
    g, x = make_config(name, S=C)
    say(f"mc {name} C={C} steps={steps}")
    (xg, vg, ng, ag), _ = walk(P, g, x, steps, seed=5, sigma=sigma)
    xo, vo, no, ao = mc.run(g, x, oracle.sweep(g, x), 0, steps, seed=5, sigma=sigma)
    assert np.array_equal(ng, no), f"{np.sum(ng != no)} walkers' acceptance counts differ"
    assert np.array_equal(xg, xo)
    assert np.array_equal(ag, ao)
    err = oracle.scaled_error(vg, vo, oracle.sweep(g, xo, "square"))
    assert np.all(err <= TOL["fp64"])
    assert 0 < ng.sum() < C * steps


def test_split_runs_and_streamed_plan_are_bit_identical(P):
    g, x = make_config("mid", S=512)
    a, _ = walk(P, g, x, 12, seed=3, sigma=0.6)
    b, _ = walk(P, g, x, 12, seed=3, sigma=0.6, split=[5, 7])
    c, _ = walk(P, g, x, 12, seed=3, sigma=0.6, path="streamed")
    sub, _ = walk(P, g, np.ascontiguousarray(x[:, :100]), 12, seed=3, sigma=0.6)
    for p, q, r in zip(a, b, c):
        assert np.array_equal(p, q) and np.array_equal(p, r)
    assert np.array_equal(sub[0], a[0][:, :100]) and np.array_equal(sub[2], a[2][:100])


@pytest.mark.parametrize("precision", ["fp64", "fp32r", "fp32"])
def test_persistent_run_matches_step_by_step(P, precision):
    # graphs on the fused plan run a whole call in one launch; the streamed
    # plan takes three launches per step: the chains must be the same bits
    g, x = make_config("tiny", S=1000)
    a, _ = walk(P, g, x, 30, seed=2, sigma=0.9, precision=precision)
    b, _ = walk(P, g, x, 30, seed=2, sigma=0.9, precision=precision, path="streamed")
    c, _ = walk(P, g, x, 30, seed=2, sigma=0.9, precision=precision, split=[1, 13, 16])
    for p, q, r in zip(a, b, c):
        assert np.array_equal(p, q) and np.array_equal(p, r)


def test_zero_step_accepts_every_proposal(P):
    g, x = make_config("tiny", S=200)
    (xg, vg, ng, ag), _ = walk(P, g, x, 6, seed=1, sigma=0.0)
    assert np.array_equal(xg, x) and np.all(ng == 6)
    assert np.array_equal(ag[0], 6 * np.sign(vg))


@pytest.mark.parametrize("precision", ["fp64", "fp32r"])
def test_long_chains_sample_abs_v(P, precision):
    # <sign V> -> int V / int |V| and <|x|^2> -> int |x|^2 |V| / int |V| (midpoint
    # quadrature: sign converged to ~1e-6; |x|^2 carries the cube's cut tail, ~1e-3)
    g, x = make_config("tiny", S=65536)  # the tiny graph: V changes sign, <sign V> ~ -0.49
    I = quadrature(g, h=0.1, R=14.0)
    G = P.Graph.from_leveled(g)
    W = P.Walkers(G, to_dev(x), precision, seed=11, sigma=1.0)
    W.run(200).reset_sums().run(1000)
    e = W.estimates()
    say(f"mc tiny {precision}: sign {e['sign']:.5f} +- {e['sign_se']:.5f} (quadrature {I[0] / I[1]:.5f}), "
        f"|x|^2 {e['x2']:.4f} +- {e['x2_se']:.4f} ({I[2] / I[1]:.4f}), acceptance {e['acceptance']:.3f}")
    assert abs(e["sign"] - I[0] / I[1]) <= 5 * e["sign_se"] + 1e-4
    assert abs(e["x2"] - I[2] / I[1]) <= 5 * e["x2_se"] + 3e-3


def test_mc_argument_errors(P):
    g, x = make_config("tiny", S=8)
    G = P.Graph.from_leveled(g)
    with pytest.raises(ValueError):
        P.Walkers(G, to_dev(x[:2]))
    W = P.Walkers(G, to_dev(x))
    W.sigma = float("nan")
    with pytest.raises(P.CosError, match="sigma"):
        W.run(1)
    # the library refuses lookup graphs (the walkers move coordinates, not tables)
    gl, _ = make_config("tiny", S=8, factor="lookup")
    Gl = P.Graph.from_leveled(gl)
    xd, v = to_dev(x), torch.zeros(8, dtype=torch.float64, device="cuda:0")
    n, acc = torch.zeros(8, dtype=torch.int64, device="cuda:0"), torch.zeros(2, 8, dtype=torch.float64, device="cuda:0")
    st = P.LIB.cos_mc_run(Gl.handle, 0, 8, xd.data_ptr(), v.data_ptr(), 0, 1, 0, 1.0, n.data_ptr(), acc.data_ptr(),
                          None, 0, None)
    assert st == -1 and "rational" in P.LIB.cos_last_error().decode()
    st = P.LIB.cos_mc_run(G.handle, 0, 0, xd.data_ptr(), v.data_ptr(), 0, 1, 0, 1.0, n.data_ptr(), acc.data_ptr(),
                          None, 0, None)
    assert st == -1 and "C must be" in P.LIB.cos_last_error().decode()


def test_checkpoint_and_graph_file_resume_bit_identical(P, tmp_path):
    # a run interrupted after 7 steps, with the graph and the walkers written to files and
    # re-created, continues with the bits of the uninterrupted run
    g, x = make_config("mid", S=700)
    whole, _ = walk(P, g, x, 15, seed=4, sigma=0.6, split=[7, 8])
    G = P.Graph.from_leveled(g)
    W = P.Walkers(G, to_dev(x), "fp64", seed=4, sigma=0.6).run(7)
    G.save(tmp_path / "graph.npz")
    W.save(tmp_path / "walkers.npz")
    G2 = P.Graph.load(tmp_path / "graph.npz")
    for k, v in G.export().items():
        assert np.array_equal(v, G2.export()[k])
    W2 = P.Walkers.load(G2, tmp_path / "walkers.npz").run(8)
    torch.cuda.synchronize()
    got = (W2.x.cpu().numpy(), W2.v.cpu().numpy(), W2.accepted.cpu().numpy(), W2.acc.cpu().numpy())
    for p, q in zip(whole, got):
        assert np.array_equal(p, q)
    assert W2.step == 15
