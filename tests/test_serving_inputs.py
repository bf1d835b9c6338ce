"""CPU checks of the serving inputs: the test request mix stays easy (so a GPU test that
compares served and solo answers cannot turn into an exponential search), and the stored
request trace is well formed and regenerates the graphs it names."""

import json
import os

import numpy as np
import pytest

import graphs as G
import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
TRACE = os.path.join(HERE, "golden", "serving_trace.json")


def test_mixed_requests_are_easy(oracle_lib):
    from test_gpu_serving import mixed_requests
    worst = 0
    for seed, count in ((5, 36), (9, 60), (13, 12)):
        for g, problem in mixed_requests(seed, count):
            r = oracle.mvc(g, node_cap=200_000)
            worst = max(worst, r.nodes)
            if problem == "pvc":
                for k in (max(r.size - 1, 0), r.size):
                    worst = max(worst, oracle.pvc(g, k, node_cap=200_000).nodes)
    assert worst <= 5000


@pytest.mark.skipif(not os.path.exists(TRACE), reason="serving trace not generated")
def test_trace_is_well_formed(oracle_lib):
    with open(TRACE) as f:
        trace = json.load(f)
    reqs = trace["requests"]
    t = np.array([r["t_ms"] for r in reqs])
    assert len(reqs) == 2000 and (np.diff(t) >= 0).all() and t[0] == 0.0
    # Poisson arrivals at 2,000 per second: mean gap 0.5 ms
    assert abs(np.diff(t).mean() - 0.5) < 0.05
    assert 0.0 <= trace["discard_rate"] < 1.0
    draws = [r["draw"] for r in reqs]
    assert draws == sorted(draws) and len(set(draws)) == len(draws)
    for r in reqs[:25]:  # the stored draw regenerates the graph and its answer
        desc, g = G.serving_draw(trace["master_seed"], r["draw"])
        assert desc["n"] == r["n"] and g.nnz == r["nnz"] and desc["problem"] == r["problem"]
        assert oracle.mvc(g, node_cap=trace["node_cap"]).size == r["tau"]
