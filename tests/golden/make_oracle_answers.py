"""Write tests/golden/oracle_answers.json: the CPU oracle's answers on the full-size workloads.

Calls only ``oracle`` (and the seeded generators in ``graphs``). The GPU parity tests read
the stored values instead of re-running the slow exhaustive searches on every test run.

Workloads (all seeded, see graphs.generators):
- mvc_er60:      MVC, G(60, 0.10), seed 0
- pvc_planted:   PVC, planted cover n=5000, |C|=400, 40,000 edges (75% C-rest), k in {400, 399},
                 seeds 0-3
- mvc_reg120:    MVC, random 5-regular n=120, seeds 0-7
- mvc_er150:     MVC, G(150, 0.08), seeds 0-7
- pvc_reg120, pvc_er150: PVC with k = tau - 1 on the same graphs (every answer "no"; the search
                 tree is then the same whatever the schedule, so node counts compare exactly)

Usage: python tests/golden/make_oracle_answers.py [--jobs 8]
"""

import argparse
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import graphs as G  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_answers.json")


def cases():
    yield ("mvc_er60", 0, None)
    for seed in range(4):
        for k in (400, 399):
            yield ("pvc_planted", seed, k)
    for seed in range(8):
        yield ("mvc_reg120", seed, None)
    for seed in range(8):
        yield ("mvc_er150", seed, None)


def make_graph(name, seed):
    if name == "mvc_er60":
        return G.erdos_renyi(60, 0.10, seed)
    if name == "pvc_planted":
        return G.planted_cover(5000, 400, 40000, 0.75, seed)
    if name in ("mvc_reg120", "pvc_reg120"):
        return G.random_regular(120, 5, seed)
    if name in ("mvc_er150", "pvc_er150"):
        return G.erdos_renyi(150, 0.08, seed)
    raise KeyError(name)


def solve(case):
    name, seed, k = case
    g = make_graph(name, seed)
    t0 = time.perf_counter()
    if k is None:
        r = oracle.mvc(g)
        out = {"size": r.size, "greedy": r.greedy}
    else:
        r = oracle.pvc(g, k)
        out = {"yes": r.yes, "size": r.size}
    dt = time.perf_counter() - t0
    out.update({"workload": name, "seed": seed, "k": k, "n": g.n, "m": g.m,
                "nodes": r.nodes, "oracle_seconds": round(dt, 3)})
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=8)
    a = ap.parse_args()
    oracle.build(force=False)
    todo = list(cases())
    with ProcessPoolExecutor(a.jobs) as ex:
        res = list(ex.map(solve, todo))
        # PVC at k = tau - 1 on the hard graphs, tau from the MVC answers just computed
        hard = [("pvc_" + r["workload"][4:], r["seed"], r["size"] - 1) for r in res
                if r["workload"] in ("mvc_reg120", "mvc_er150")]
        res += list(ex.map(solve, hard))
    doc = {"_about": "CPU oracle answers (oracle/vc_oracle.c) on the seeded full-size "
                     "workloads; written by tests/golden/make_oracle_answers.py.",
           "results": res}
    with open(OUT, "w") as f:
        json.dump(doc, f, indent=1)
    for r in res:
        print(r)


if __name__ == "__main__":
    main()
