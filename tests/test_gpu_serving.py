"""The request server (vc_server_*): continuous batching of a stream of MVC / PVC requests.

Every served result must equal what the single-graph call gives for the same graph, alone:
the same MVC size and PVC decision, a cover checked edge by edge here, and for PVC-no the same
node count (that tree does not depend on the schedule). The stored trace's answers come from
the CPU oracle (tests/golden/make_serving_trace.py).
"""

import json
import os
import time

import numpy as np
import pytest

import graphs as G
import oracle

pytestmark = pytest.mark.gpu

TRACE = os.path.join(os.path.dirname(__file__), "golden", "serving_trace.json")


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


@pytest.fixture(scope="module")
def solver(torch_cuda):
    import paper_2204_10402_amd as vc
    s = vc.Solver(0)
    yield s
    s.close()


def check_cover(g, cover, size):
    cover = np.asarray(cover)
    assert cover.shape == (g.n,)
    assert oracle.is_cover(g, cover)
    assert int(cover.sum()) == size


def mixed_requests(seed, count):
    """Easy requests of both kernel families (every one needs at most a few thousand oracle
    nodes; pinned by test_mixed_requests_are_easy in the CPU suite)."""
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(count):
        fam = i % 3
        if fam == 0:
            n = int(rng.integers(20, 200))
            g = G.erdos_renyi(n, float(rng.uniform(1.5, 3.0)) / n, 100 * seed + i)
        elif fam == 1:
            n = int(rng.integers(20, 600))
            g = G.planted_cover(n, max(1, int(0.3 * n)), 2 * n, 0.75, 100 * seed + i)
        else:
            n = 2 * int(rng.integers(10, 25))
            g = G.random_regular(n, 3, 100 * seed + i)
        problem = "pvc" if i % 2 else "mvc"
        reqs.append((g, problem))
    return reqs


def drain(server, want, timeout_s=60.0):
    got = {}
    t0 = time.time()
    while len(got) < want:
        for r in server.poll(timeout_ms=50):
            got[r["ticket"]] = r
        assert time.time() - t0 < timeout_s, f"only {len(got)} of {want} results"
    return got


def solo(solver, g, problem, k):
    return solver.pvc(g, k) if problem == "pvc" else solver.mvc(g)


@pytest.mark.parametrize("workers,max_batch", [(1, 1), (3, 8), (4, 256)])
def test_served_results_equal_solo_results(solver, oracle_lib, workers, max_batch):
    import paper_2204_10402_amd as vc
    reqs = mixed_requests(5, 36)
    ks = {}
    with vc.Server(0, workers=workers, max_batch=max_batch) as srv:
        tickets = []
        for i, (g, problem) in enumerate(reqs):
            k = max(solver.mvc(g).size - (i % 2), 0) if problem == "pvc" else 0
            ks[i] = k
            tickets.append(srv.submit(g, problem, k))
        got = drain(srv, len(reqs))
    for i, ((g, problem), t) in enumerate(zip(reqs, tickets)):
        r = got[t]
        alone = solo(solver, g, problem, ks[i])
        assert r["status"] == 0
        assert r["size"] == alone.size and bool(r["yes"]) == alone.yes, i
        if problem == "mvc" or alone.yes:
            check_cover(g, r["cover"], r["size"])
        else:
            assert r["nodes"] == alone.stats["nodes"]
            assert int(r["cover"].sum()) == 0
        assert 1 <= r["batch_size"] <= max_batch
        assert r["submit_ms"] <= r["start_ms"] <= r["done_ms"]


def test_streamed_arrivals_overlap(solver, oracle_lib):
    """Requests submitted while others run are admitted by free workers: with a stream of
    arrivals several batches are in flight at once (a request of a search of ~2.4e5 nodes
    first keeps one worker busy while the rest arrive), and answers still equal solo answers."""
    import paper_2204_10402_amd as vc
    reqs = [(G.random_regular(100, 5, 7), "mvc")] + mixed_requests(9, 60)
    with vc.Server(0, workers=4, max_batch=16) as srv:
        tickets = []
        for g, problem in reqs:
            tickets.append(srv.submit(g, problem, g.n))  # k = n: always yes for PVC
            time.sleep(0.0002)
        got = drain(srv, len(reqs))
    spans = sorted((got[t]["start_ms"], got[t]["done_ms"]) for t in tickets)
    for (g, problem), t in zip(reqs, tickets):
        r = got[t]
        assert r["status"] == 0 and r["yes"] == 1
        if problem == "mvc":
            assert r["size"] == solver.mvc(g).size
        check_cover(g, r["cover"], r["size"])
    workers = {got[t]["worker"] for t in tickets}
    assert len(workers) >= 2
    assert len(spans) == len(reqs)
    # two batches of different workers were on the device at the same time
    rs = [got[t] for t in tickets]
    overlap = any(a["worker"] != b["worker"] and
                  max(a["start_ms"], b["start_ms"]) < min(a["done_ms"], b["done_ms"])
                  for i, a in enumerate(rs) for b in rs[i + 1:])
    assert overlap, sorted((r["worker"], r["start_ms"], r["done_ms"]) for r in rs)


def test_memory_budget_serializes_batches(solver, oracle_lib):
    import paper_2204_10402_amd as vc
    reqs = mixed_requests(13, 12)
    with vc.Server(0, workers=3, max_batch=64, memory_budget=1) as srv:
        tickets = [srv.submit(g, p, g.n) for g, p in reqs]
        got = drain(srv, len(reqs))
    rs = [got[t] for t in tickets]
    assert all(r["batch_size"] == 1 for r in rs)  # each request alone exceeds the budget
    iv = sorted((r["start_ms"], r["done_ms"]) for r in rs)
    for (s0, d0), (s1, d1) in zip(iv, iv[1:]):
        assert s1 >= d0 - 1e-6  # never two batches in flight
    for (g, p), r in zip(reqs, rs):
        if p == "mvc":
            assert r["size"] == solver.mvc(g).size


def test_rejected_request_does_not_disturb_others(solver, oracle_lib):
    import paper_2204_10402_amd as vc

    class Raw:
        pass
    bad = Raw()
    good = G.path(6)
    bad.n, bad.row_ptr, bad.col_idx = 6, good.row_ptr.copy(), good.col_idx.copy()
    bad.col_idx[0] = 0  # self-loop
    with vc.Server(0, workers=1, max_batch=8) as srv:
        ts = [srv.submit(G.cycle(7), "mvc"), srv.submit(bad, "mvc"), srv.submit(G.star(5), "mvc")]
        got = drain(srv, 3)
    assert [got[t]["status"] for t in ts] == [0, vc.ERR_INVALID_GRAPH, 0]
    assert got[ts[0]]["size"] == 4 and got[ts[2]]["size"] == 1


def test_server_arguments(torch_cuda):
    import paper_2204_10402_amd as vc
    with pytest.raises(vc.VCError):
        vc.Server(0, options=vc.Options(num_wg=4))
    with pytest.raises(vc.VCError):
        vc.Server(0, options=vc.Options(flags=vc.OPT_AUTOTUNE))
    with vc.Server(0, workers=1) as srv:
        with pytest.raises(vc.VCError):
            srv.submit(G.path(4), "pvc", -1)
        assert srv.pending() == (0, 0)


@pytest.mark.skipif(not os.path.exists(TRACE), reason="serving trace not generated")
def test_trace_requests_match_oracle(oracle_lib):
    """The first 300 requests of the stored trace, submitted at once: every answer equals the
    oracle's stored answer."""
    import paper_2204_10402_amd as vc
    with open(TRACE) as f:
        trace = json.load(f)
    reqs = trace["requests"][:300]
    graphs = [G.serving_draw(trace["master_seed"], r["draw"])[1] for r in reqs]
    with vc.Server(0, workers=4, max_batch=64) as srv:
        tickets = [srv.submit(g, r["problem"], r.get("k", 0)) for g, r in zip(graphs, reqs)]
        got = drain(srv, len(reqs), timeout_s=120)
    for g, r, t in zip(graphs, reqs, tickets):
        out = got[t]
        assert out["status"] == 0
        if r["problem"] == "mvc":
            assert out["size"] == r["tau"]
            check_cover(g, out["cover"], r["tau"])
        else:
            assert bool(out["yes"]) == r["yes"]
            if r["yes"]:
                assert out["size"] <= r["k"]
                check_cover(g, out["cover"], out["size"])
            else:
                assert out["nodes"] == r["pvc_nodes"]
