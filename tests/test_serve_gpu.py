"""Serving runtime (cos_server_*) on the GPU.

Every request's result must be bit-identical to cos_evaluate on the same graph,
samples and precision -- alone and in a mix of graphs, plans and precisions
sharing steps -- and within the oracle tolerance of the FP64 oracle.
Admission, budget, cancellation and argument checks are exercised too.
"""

import numpy as np
import pytest
import torch

from gpu_util import PRECISIONS, assert_parity, gpu_eval, oracle_ref, sample_subset, say, to_dev
from workloads import make_config, serving_mix

pytestmark = pytest.mark.gpu

MiB = 1 << 20


@pytest.fixture(scope="module")
def P():
    import paper_2501_00675_amd as P

    assert torch.cuda.is_available()
    return P


def bits(y):
    return np.asarray(y, np.float64).view(np.uint64)


@pytest.mark.parametrize("precision", PRECISIONS)
@pytest.mark.parametrize("path", ["auto", "streamed"])
def test_single_request_matches_evaluate_and_oracle(P, precision, path):
    g, x = make_config("mid", S=1000, width=40, L=6)
    G = P.Graph.from_leveled(g).set_path(path)
    fused = path == "auto"
    say(f"serve single {precision} {path}")
    with P.Server(64 * MiB, 4) as srv:
        gid = srv.add_graph(G)
        t = srv.submit(gid, to_dev(x), precision)
        st = srv.wait(t)
        y = t.out.cpu().numpy()
    assert st["status"] == 0
    assert st["steps"] == (1 if fused else g.L + 1)
    assert (st["footprint"] == 0) == fused
    assert st["t_submit_ns"] <= st["t_admit_ns"] <= st["t_done_ns"]
    assert np.array_equal(bits(y), bits(gpu_eval(G, x, precision)))
    V, Q = oracle_ref(g, x)
    assert_parity(y, V, Q, precision, f"serve {path}")


def _mix(P, n_graphs=10, n_requests=40, seed=11):
    graphs, reqs = serving_mix(n_graphs=n_graphs, n_requests=n_requests, seed=seed, max_width=900, max_S=2500)
    Gs = [P.Graph.from_leveled(g) for g in graphs]
    # the first graphs once more under the streamed plan, so one graph is served both ways
    Gs += [P.Graph.from_leveled(g).set_path("streamed") for g in graphs[:3]]
    rng = np.random.default_rng(seed)
    jobs = []
    for i, r in enumerate(reqs):
        gi = r["graph"] if i % 4 else len(graphs) + r["graph"] % 3
        jobs.append(dict(G=gi, x=r["x"], precision=PRECISIONS[int(rng.integers(3))]))
    return graphs, Gs, jobs


def test_mix_bit_identical_to_evaluate_and_alone(P):
    graphs, Gs, jobs = _mix(P)
    code = {"fp64": 0, "fp32r": 1, "fp32": 2}
    n_fused = sum(j["G"] < len(graphs) and (Gs[j["G"]].info()["fused_mask"] >> code[j["precision"]]) & 1
                  for j in jobs)
    say(f"serve mix: {len(jobs)} requests, {n_fused} whole-graph, {len(Gs)} graphs")
    refs = [gpu_eval(Gs[j["G"]], j["x"], j["precision"]) for j in jobs]
    xs = [to_dev(j["x"]) for j in jobs]
    torch.cuda.synchronize()
    with P.Server(512 * MiB, 16) as srv:
        gids = [srv.add_graph(G) for G in Gs]
        tickets = [srv.submit(gids[j["G"]], x, j["precision"], sync_inputs=False) for j, x in zip(jobs, xs)]
        stats = [srv.wait(t) for t in tickets]
        outs = [t.out.cpu().numpy() for t in tickets]
        s = srv.stats()
        trace = srv.read_steps()
    assert all(st["status"] == 0 for st in stats)
    # the step trace accounts for every step, every request's stages and every item
    assert [r["step"] for r in trace] == list(range(s["steps"]))
    assert all(r["t_done_ns"] >= r["t_launch_ns"] > 0 for r in trace)
    assert sum(r["n_fused"] + r["n_streamed"] for r in trace) == sum(st["steps"] for st in stats)
    assert sum(r["items"] for r in trace) == s["items"]
    assert max(r["n_fused"] + r["n_streamed"] for r in trace) == s["max_step_requests"]
    assert all(0 <= st["first_step"] and st["first_step"] + st["steps"] <= len(trace) for st in stats)
    for i, (y, r) in enumerate(zip(outs, refs)):
        assert np.array_equal(bits(y), bits(r)), f"request {i} ({jobs[i]['precision']}) differs from cos_evaluate"
    assert s["completed"] == len(jobs) and s["failed"] == 0
    assert s["max_step_requests"] > 1, "requests never shared a step"
    assert s["peak_bytes"] <= s["budget_bytes"]
    # the same requests alone (one at a time) give the same bits
    with P.Server(512 * MiB, 16) as srv:
        gids = [srv.add_graph(G) for G in Gs]
        for i in range(0, len(jobs), 5):
            j = jobs[i]
            t = srv.submit(gids[j["G"]], xs[i], j["precision"], sync_inputs=False)
            srv.wait(t)
            assert np.array_equal(bits(t.out.cpu().numpy()), bits(outs[i]))
        assert srv.stats()["max_step_requests"] == 1
    # and against the oracle on a sample of each of a few requests
    for i in range(0, len(jobs), 7):
        j = jobs[i]
        idx = sample_subset(j["x"].shape[1], 64, seed=i)
        V, Q = oracle_ref(graphs[j["G"] if j["G"] < len(graphs) else j["G"] - len(graphs)], j["x"], idx)
        assert_parity(outs[i][idx], V, Q, j["precision"], f"mix request {i}")


def test_large_admission_batches_carry_their_set_up(P):
    # 512 slots: a long request keeps the steps busy while 600 small ones are submitted, so the
    # scheduler admits them in large batches whose set-up (slot entries; exponent rows of the
    # streamed rescaled ones) rides on one step each.  Every result must equal cos_evaluate's bits.
    gb, xb = make_config("mid", S=3000, width=20000, L=8, degree=8, seed=52)
    g1, _ = make_config("tiny", S=64)
    g2, _ = make_config("mid", S=64, width=300, L=5, degree=3, seed=51)
    Gb = P.Graph.from_leveled(gb)
    Gs = [P.Graph.from_leveled(g1), P.Graph.from_leveled(g2).set_path("streamed")]
    rng = np.random.default_rng(8)
    jobs = [(i % 2, ("fp64", "fp32r", "bf16r", "fp16r")[i % 4], int(rng.integers(1, 200))) for i in range(600)]
    xs = [rng.normal(size=(3, S)) for _, _, S in jobs]
    refs = [gpu_eval(Gs[gi], x, p) for (gi, p, _), x in zip(jobs, xs)]
    ref_b = gpu_eval(Gb, xb, "fp64")
    xd = [to_dev(x) for x in xs]
    xbd = to_dev(xb)
    torch.cuda.synchronize()
    say("serve 600 requests on 512 slots behind a long request")
    with P.Server(2 << 30, 512) as srv:
        gb_id = srv.add_graph(Gb)
        gids = [srv.add_graph(G) for G in Gs]
        tb = srv.submit(gb_id, xbd, "fp64", sync_inputs=False)
        tickets = [srv.submit(gids[gi], x, p, sync_inputs=False) for (gi, p, _), x in zip(jobs, xd)]
        stats = [srv.wait(t) for t in tickets]
        sb = srv.wait(tb)
    assert sb["status"] == 0 and all(st["status"] == 0 for st in stats)
    assert np.array_equal(bits(tb.out.cpu().numpy()), bits(ref_b))
    for i, (t, r) in enumerate(zip(tickets, refs)):
        assert np.array_equal(bits(t.out.cpu().numpy()), bits(r)), f"request {i} {jobs[i]}"
    batch = np.bincount([st["first_step"] for st in stats]).max()
    say(f"largest batch of requests starting in one step: {batch}")
    assert batch >= 32


def test_lookup_graphs_served_bit_identical_alone_and_mixed(P):
    # lookup-factor graphs (a narrow one on the fused plan, a wide one streamed) share steps
    # with a rational graph; every result must equal cos_evaluate's bits.  Streamed lookup
    # requests at the binary32 precisions take one more step, which copies their tables to
    # binary32
    graphs = [make_config("mid", S=1500, factor="lookup", width=200, L=6, degree=3, seed=31),
              make_config("mid", S=1300, factor="lookup", width=900, L=5, degree=3, seed=32),
              make_config("mid", S=1200, width=700, L=5, degree=3, seed=33)]
    Gs = [P.Graph.from_leveled(g) for g, _ in graphs]
    code = {"fp64": 0, "fp32r": 1, "fp32": 2}
    assert (Gs[0].info()["fused_mask"] >> code["fp64"]) & 1 and not Gs[1].info()["fused_mask"]
    jobs = [(gi, p) for p in ("fp64", "fp32r", "fp32", "bf16r") for gi in range(3)]
    xs = [to_dev(graphs[gi][1]) for gi, _ in jobs]
    refs = [gpu_eval(Gs[gi], graphs[gi][1], p) for gi, p in jobs]
    torch.cuda.synchronize()
    say(f"serve lookup mix: {len(jobs)} requests")
    with P.Server(512 * MiB, 16) as srv:
        gids = [srv.add_graph(G) for G in Gs]
        tickets = [srv.submit(gids[gi], x, p, sync_inputs=False) for (gi, p), x in zip(jobs, xs)]
        stats = [srv.wait(t) for t in tickets]
        s = srv.stats()
    assert all(st["status"] == 0 for st in stats) and s["max_step_requests"] > 1
    for i, (t, r) in enumerate(zip(tickets, refs)):
        assert np.array_equal(bits(t.out.cpu().numpy()), bits(r)), f"request {i} {jobs[i]}"
    for (gi, p), st in zip(jobs, stats):
        fused = p in code and (Gs[gi].info()["fused_mask"] >> code[p]) & 1
        lookup_b32 = gi < 2 and p != "fp64"
        want = 1 if fused else graphs[gi][0].L + 1 + int(lookup_b32)
        assert st["steps"] == want, (gi, p, st["steps"], want)
    # alone, and against the oracle on sampled outputs
    with P.Server(512 * MiB, 4) as srv:
        gid = srv.add_graph(Gs[1])
        t = srv.submit(gid, xs[1], "fp64")
        srv.wait(t)
        assert np.array_equal(bits(t.out.cpu().numpy()), bits(refs[1]))
        with pytest.raises(ValueError):
            srv.submit(gid, to_dev(graphs[2][1]), "fp64")  # coordinates where a table is due
    for i, (gi, p) in enumerate(jobs):
        if p == "bf16r":  # its bar is the storage bound, checked for cos_evaluate's identical bits elsewhere
            continue
        g, x = graphs[gi]
        idx = sample_subset(x.shape[1], 48, seed=i)
        V, Q = oracle_ref(g, x, idx)
        assert_parity(tickets[i].out.cpu().numpy()[idx], V, Q, p, f"lookup mix {i}")


def test_16bit_storage_served_bit_identical_alone_and_mixed(P):
    # binary16 and bfloat16 level storage in the serving runtime: 16-bit requests run on the
    # streamed plan (also for a graph that takes the whole-graph plan at 32 and 64 bits) and
    # share steps with FP64 and FP32-rescaled requests; every result must equal cos_evaluate's
    # bits at the same precision (whose error is checked against the oracle's bound elsewhere)
    graphs = [make_config("mid", S=1500, width=200, L=6, degree=3, seed=41),
              make_config("mid", S=1300, width=900, L=7, degree=3, seed=42),
              make_config("mid", S=1100, factor="lookup", width=600, L=5, degree=3, seed=43)]
    Gs = [P.Graph.from_leveled(g) for g, _ in graphs]
    assert Gs[0].info()["fused_mask"] & 1 and not Gs[1].info()["fused_mask"]
    jobs = [(0, "fp16r"), (0, "bf16r"), (1, "fp16r"), (1, "bf16r"), (2, "bf16r"), (0, "fp64"), (1, "fp32r"),
            (2, "fp32r"), (1, "fp16r")]
    xs = [to_dev(graphs[gi][1]) for gi, _ in jobs]
    refs = [gpu_eval(Gs[gi], graphs[gi][1], p) for gi, p in jobs]
    torch.cuda.synchronize()
    say(f"serve 16-bit mix: {len(jobs)} requests")
    with P.Server(512 * MiB, 16) as srv:
        gids = [srv.add_graph(G) for G in Gs]
        tickets = [srv.submit(gids[gi], x, p, sync_inputs=False) for (gi, p), x in zip(jobs, xs)]
        stats = [srv.wait(t) for t in tickets]
        s = srv.stats()
    assert all(st["status"] == 0 for st in stats) and s["max_step_requests"] > 1
    for i, (t, r) in enumerate(zip(tickets, refs)):
        assert np.array_equal(bits(t.out.cpu().numpy()), bits(r)), f"request {i} {jobs[i]}"
    with P.Server(256 * MiB, 2) as srv:
        gid = srv.add_graph(Gs[1])
        t = srv.submit(gid, xs[2], "fp16r")
        srv.wait(t)
        assert np.array_equal(bits(t.out.cpu().numpy()), bits(refs[2]))
        # refused as by cos_evaluate: binary16 with lookup factors, 16-bit with the whole-graph plan forced
        gl = srv.add_graph(Gs[2])
        with pytest.raises(P.CosError, match="binary16"):
            srv.submit(gl, xs[4], "fp16r")
        g0 = srv.add_graph(Gs[0])
        Gs[0].set_path("fused")
        with pytest.raises(P.CosError, match="streamed plan"):
            srv.submit(g0, xs[0], "bf16r")
        Gs[0].set_path("auto")


@pytest.mark.parametrize("precision", ["fp64", "fp32r"])
def test_admission_waits_for_budget(P, precision):
    g, x = make_config("mid", S=2000, width=700, L=5, degree=3)
    G = P.Graph.from_leveled(g)
    assert G.info()["fused_mask"] == 0
    W = G.workspace_bytes(2000, precision)
    budget = W + W // 2  # one request at a time
    xd = to_dev(x)
    torch.cuda.synchronize()
    say(f"serve admission {precision} W={W}")
    with P.Server(budget, 8) as srv:
        gid = srv.add_graph(G)
        tickets = [srv.submit(gid, xd, precision, sync_inputs=False) for _ in range(5)]
        stats = [srv.wait(t) for t in tickets]
        s = srv.stats()
    ref = gpu_eval(G, x, precision)
    for t, st in zip(tickets, stats):
        assert st["status"] == 0 and st["footprint"] >= W
        assert np.array_equal(bits(t.out.cpu().numpy()), bits(ref))
    assert s["peak_bytes"] <= budget and s["max_active"] == 1
    order = sorted(stats, key=lambda d: d["t_admit_ns"])
    for a, b in zip(order, order[1:]):
        assert b["t_admit_ns"] >= a["t_done_ns"], "a request was admitted before the budget was free"


@pytest.mark.parametrize("precision", ["fp64", "fp32r"])
def test_failed_setup_fails_only_that_request_and_frees_its_slot(P, precision):
    # the set-up of the third admission is made to fail from the host (no device fault);
    # with a budget for two requests at a time, a failed request that kept its workspace
    # or slot would stall everything submitted after it
    g, x = make_config("mid", S=2000, width=700, L=5, degree=3)
    G = P.Graph.from_leveled(g)
    W = G.workspace_bytes(2000, precision)
    xs = [to_dev(x * (1.0 + 0.01 * i)) for i in range(8)]
    torch.cuda.synchronize()
    say(f"serve injected failure {precision} W={W}")
    with P.Server(2 * W + W // 2, 2) as srv:
        srv.fail_admission(2)
        gid = srv.add_graph(G)
        tickets = [srv.submit(gid, xs[i], precision, sync_inputs=False) for i in range(6)]
        for i, t in enumerate(tickets):
            if i == 2:
                with pytest.raises(P.CosError) as e:
                    srv.wait(t)
                assert e.value.status == -3  # COS_EDEVICE
            else:
                assert srv.wait(t)["status"] == 0
        later = [srv.submit(gid, xs[6 + i], precision, sync_inputs=False) for i in range(2)]
        for t in later:
            assert srv.wait(t)["status"] == 0
        s = srv.stats()
    assert s["failed"] == 1 and s["completed"] == 7 and s["max_active"] <= 2
    for i, t in enumerate(tickets + later):
        if i != 2:
            ref = gpu_eval(G, xs[i].cpu().numpy(), precision)
            assert np.array_equal(bits(t.out.cpu().numpy()), bits(ref)), i


def test_request_that_never_fits_is_rejected(P):
    g, x = make_config("mid", S=2000, width=700, L=5, degree=3)
    G = P.Graph.from_leveled(g)
    W = G.workspace_bytes(2000, "fp64")
    with P.Server(W // 2, 4) as srv:
        gid = srv.add_graph(G)
        with pytest.raises(P.CosError) as e:
            srv.submit(gid, to_dev(x), "fp64")
        assert e.value.status == -2  # COS_ENOMEM
        assert srv.stats()["submitted"] == 0


def test_cancel_queued_request(P):
    g, x = make_config("mid", S=2000, width=700, L=5, degree=3)
    G = P.Graph.from_leveled(g)
    xd = to_dev(x)
    torch.cuda.synchronize()
    ref = gpu_eval(G, x, "fp64")
    with P.Server(G.workspace_bytes(2000, "fp64") * 3 // 2, 1) as srv:
        gid = srv.add_graph(G)
        tickets = [srv.submit(gid, xd, "fp64", sync_inputs=False) for _ in range(6)]
        cancelled = srv.cancel(tickets[-1])
        stats = [srv.wait(t) for t in tickets]
        s = srv.stats()
    for t, st in zip(tickets[:-1], stats[:-1]):
        assert st["status"] == 0
        assert np.array_equal(bits(t.out.cpu().numpy()), bits(ref))
    if cancelled:
        assert stats[-1]["status"] == -5 and stats[-1]["steps"] == 0  # COS_ECANCELED
        assert s["cancelled"] == 1 and s["completed"] == 5
    else:  # already admitted: it completes
        assert stats[-1]["status"] == 0


def test_bad_arguments(P):
    g, x = make_config("mid", S=100, width=700, L=4, degree=2)
    G = P.Graph.from_leveled(g)
    xd = to_dev(x)
    with P.Server(64 * MiB, 2) as srv:
        gid = srv.add_graph(G)
        for bad in (lambda: srv.submit(gid + 5, xd, "fp64"),               # unknown graph
                    lambda: srv.submit(gid, xd[:, :0].contiguous(), "fp64"),  # S = 0
                    lambda: srv.poll(12345),                                # unknown ticket
                    lambda: srv.cancel(12345)):
            with pytest.raises(P.CosError) as e:
                bad()
            assert e.value.status == -1
        G.set_path("fused")  # too wide for the whole-graph plan
        with pytest.raises(P.CosError):
            srv.submit(gid, xd, "fp64")
        G.set_path("auto")
        t = srv.submit(gid, xd, "fp64")
        assert srv.wait(t)["status"] == 0
        with pytest.raises(P.CosError):  # the ticket is forgotten once reported
            srv.poll(t)
    with pytest.raises(P.CosError):
        P.Server(64 * MiB, 0)


@pytest.mark.parametrize("path", ["auto", "streamed"])
def test_out_exp_form(P, path):
    g, x = make_config("mid", S=700, width=48, L=8)
    G = P.Graph.from_leveled(g).set_path(path)
    xd = to_dev(x)
    e_ref = torch.empty(700, dtype=torch.int32, device=xd.device)
    y_ref = G.evaluate(xd, "fp32r", out_exp=e_ref)
    torch.cuda.synchronize()
    with P.Server(64 * MiB, 2) as srv:
        gid = srv.add_graph(G)
        t = srv.submit(gid, xd, "fp32r", out_exp=torch.empty(700, dtype=torch.int32, device=xd.device))
        srv.wait(t)
    assert np.array_equal(bits(t.out.cpu().numpy()), bits(y_ref.cpu().numpy()))
    assert np.array_equal(t.out_exp.cpu().numpy(), e_ref.cpu().numpy())


def test_poll_until_done_and_destroy_with_queue(P):
    g, x = make_config("mid", S=1500, width=300, L=10, degree=4)
    G = P.Graph.from_leveled(g).set_path("streamed")
    xd = to_dev(x)
    torch.cuda.synchronize()
    srv = P.Server(256 * MiB, 2)
    gid = srv.add_graph(G)
    t = srv.submit(gid, xd, "fp32r", sync_inputs=False)
    st = None
    for _ in range(200000):
        st = srv.poll(t)
        if st is not None:
            break
    if st is None:
        st = srv.wait(t)
    assert st["status"] == 0 and st["steps"] == g.L + 1
    for _ in range(10):  # left queued / running: destroy cancels the queued ones and drains the rest
        srv.submit(gid, xd, "fp64", sync_inputs=False)
    srv.close()
    torch.cuda.synchronize()


def test_timing_probe_counts_serving_steps(P):
    g, x = make_config("mid", S=1000, width=300, L=6, degree=3)
    G = P.Graph.from_leveled(g).set_path("streamed")
    xd = to_dev(x)
    torch.cuda.synchronize()
    P.timing_enable(True)
    try:
        P.timing_read("serve")
        with P.Server(64 * MiB, 2) as srv:
            gid = srv.add_graph(G)
            srv.wait(srv.submit(gid, xd, "fp64", sync_inputs=False))
            steps = srv.stats()["steps"]
        ms, n = P.timing_read("serve")
    finally:
        P.timing_enable(False)
    assert steps == g.L + 1 and n == steps and ms > 0
