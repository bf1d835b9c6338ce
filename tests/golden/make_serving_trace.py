"""Write tests/golden/serving_trace.json: a fixed stream of served requests.

    python tests/golden/make_serving_trace.py

Requests arrive as a Poisson process of 2,000 per second (exponential gaps, mean 0.5 ms).
Request slot r takes the next draw of ``graphs.serving_draw(0, i)`` (n log-uniform in
[50, 2000]; ER, planted-cover or 3-5-regular; MVC or PVC). PVC's k is |C| or |C| - 1 for
planted graphs and tau or tau - 1 otherwise (a fair coin per request). Every draw is screened
by the CPU oracle with a node cap: a draw whose MVC search (and, for PVC, whose PVC search)
needs more than NODE_CAP nodes is discarded and the slot takes the next draw; the discard
rate is recorded. Only the oracle computes the stored answers.
"""

import json
import os
import sys
from multiprocessing import Pool

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import graphs as G  # noqa: E402
import oracle  # noqa: E402

MASTER_SEED = 0
REQUESTS = 2000
RATE_PER_S = 2000.0
NODE_CAP = 50_000


def screen(i):
    desc, g = G.serving_draw(MASTER_SEED, i)
    try:
        r = oracle.mvc(g, node_cap=NODE_CAP)
    except oracle.BudgetExceeded:
        return i, None
    out = dict(desc, tau=r.size, mvc_nodes=r.nodes, nnz=int(g.nnz))
    if desc["problem"] == "pvc":
        coin = int(np.random.default_rng([MASTER_SEED, i, 1]).integers(0, 2))
        base = desc["cover"] if desc["family"] == "planted" else r.size
        k = max(base - coin, 0)
        try:
            p = oracle.pvc(g, k, node_cap=NODE_CAP)
        except oracle.BudgetExceeded:
            return i, None
        out.update(k=k, yes=bool(p.yes), pvc_nodes=p.nodes)
    return i, out


def main():
    oracle.build(force=False)
    accepted, draws, nxt = [], 0, 0
    with Pool(8) as pool:
        while len(accepted) < REQUESTS:
            batch = list(range(nxt, nxt + 256))
            nxt += 256
            for i, out in pool.map(screen, batch, chunksize=2):
                draws = i + 1
                if out is not None:
                    accepted.append(out)
                if len(accepted) == REQUESTS:
                    break
            print(f"{len(accepted)} accepted of {draws} draws", flush=True)
    gaps = np.random.default_rng([MASTER_SEED, 2**31 - 1]).exponential(1000.0 / RATE_PER_S, REQUESTS)
    t = np.cumsum(gaps) - gaps[0]
    for r, ti in zip(accepted, t):
        r["t_ms"] = round(float(ti), 4)
    doc = {
        "_about": "Served request stream (fixed). Arrival t_ms; the graph is "
                  "graphs.serving_draw(master_seed, draw). Answers from the CPU oracle.",
        "master_seed": MASTER_SEED, "rate_per_s": RATE_PER_S, "node_cap": NODE_CAP,
        "draws": draws, "discard_rate": 1.0 - REQUESTS / draws, "requests": accepted,
    }
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "serving_trace.json"), "w") as f:
        json.dump(doc, f, indent=0)
    print(f"discard rate {doc['discard_rate']:.3f}")


if __name__ == "__main__":
    main()
