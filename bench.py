"""Benchmark: search-tree nodes/s and time-to-solve of the hybrid vertex-cover traversal on
one MI355X, inputs resident in device memory.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-cpu-baseline]

A step solves every instance of the workload once, inputs resident in device memory:
  --mode batch   one batched call for all of them (vc_pvc_batch_device / vc_mvc_batch_device;
                 the default)
  --mode single  one device-form call per instance (vc_pvc_device / vc_mvc_device)
After the timed steps, one untimed pass of single calls gives each instance's time-to-solve
and the throughput of the plain form (one persistent launch per instance).
Workloads (seeded, synthetic):
  planted-pvc    PVC on planted-cover graphs n=5000, |C|=400, 40,000 edges (75% C-rest),
                 k in {400, 399}, seeds 0-3: 8 solves per step (default)
  er60-mvc       MVC on G(60, 0.10), seed 0
  hard-mvc       MVC on random 5-regular n=120 and G(150, 0.08), seeds 0-7: 16 solves
  planted-batch  4,096 planted-cover PVC instances, n uniform in [40, 400], average degree in
                 [3, 12], |C| = 0.3n, k = |C| (even i) or |C| - 1 (odd i), master seed 0
  serving        the stored request stream tests/golden/serving_trace.json (2,000 requests
                 arriving as a Poisson process of 2,000 per second; n log-uniform in
                 [50, 2000]; ER, planted-cover and 3-5-regular graphs; MVC or PVC) replayed in
                 real time into a vc_server (continuous batching); compared with the plain form
                 (one worker, one request per launch, in arrival order)
Prints one JSON line on stdout; progress goes to stderr.

Ablation (--ablation, hard instances): the hybrid traversal against StackOnly, the method the
paper compares with (static sub-trees at start depth 8, 12 or 16, no worklist), on 5-regular
n=120 and G(150, 0.08), seeds 0-1: time per solve, per-workgroup load distribution (load =
nodes visited by a workgroup / mean over workgroups) and the activity breakdown of the
instrumented kernels (each workgroup's cycles per activity / its total, mean over workgroups).

HBM traffic of the traversal kernel (roofline "traffic"): two rocprofv3 counter runs of
    python bench.py --workload W --traffic-probe
one with --pmc FETCH_SIZE and one with --pmc WRITE_SIZE, each writing CSV under a directory;
the probe also runs a plain elementwise kernel over 512 MiB (read once, written once) whose
counters calibrate the units.
    python bench.py --workload W --summarize-traffic FETCH_DIR WRITE_DIR
then writes profiles/traverse_kernel_W_traffic.md, which later runs read while the kernel
sources are unchanged.
"""

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "search-tree nodes/s & time-to-solve; batched instances/s, p50/p99 latency"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def instances(workload):
    import graphs as G
    if workload == "planted-pvc":
        out = []
        for seed in range(4):
            g = G.planted_cover(5000, 400, 40000, 0.75, seed)
            for k in (400, 399):
                out.append(("pvc", g, k, f"planted seed {seed} k={k}"))
        return out, {"n": 5000, "m": 40000, "cover": 400, "k": [400, 399], "seeds": [0, 1, 2, 3]}
    if workload == "er60-mvc":
        return [("mvc", G.erdos_renyi(60, 0.10, 0), None, "G(60,0.10) seed 0")], \
            {"n": 60, "p": 0.10, "seeds": [0]}
    if workload == "hard-mvc":
        out = [("mvc", G.random_regular(120, 5, s), None, f"5-regular n=120 seed {s}") for s in range(8)]
        out += [("mvc", G.erdos_renyi(150, 0.08, s), None, f"G(150,0.08) seed {s}") for s in range(8)]
        return out, {"families": ["5-regular n=120", "G(150, 0.08)"], "seeds": list(range(8))}
    if workload == "planted-batch":
        out = [("pvc", g, k, f"planted batch instance {i}")
               for i, (g, k) in enumerate(G.planted_batch(4096, 0))]
        return out, {"n": [40, 400], "avg_degree": [3, 12], "cover_frac": 0.3,
                     "k": "|C| for even i, |C|-1 for odd i", "master_seed": 0}
    raise SystemExit(f"unknown workload {workload}")


WORKLOADS = ["planted-pvc", "er60-mvc", "hard-mvc", "planted-batch", "serving"]
TRACE = os.path.join(ROOT, "tests", "golden", "serving_trace.json")


def _trace_graph(args):
    import graphs as G
    seed, draw = args
    return G.serving_draw(seed, draw)[1]


def replay(vc, graphs, reqs, server_kw, label):
    """Submit every request at its arrival time (relative to the start) from a second thread
    while this one polls; returns the per-request results and the wall time."""
    import threading
    srv = vc.Server(0, **server_kw)
    results = {}
    tickets = [None] * len(reqs)
    t_start = time.perf_counter()

    def submitter():
        for i, (g, r) in enumerate(zip(graphs, reqs)):
            due = t_start + r["t_ms"] / 1000.0
            while True:
                left = due - time.perf_counter()
                if left <= 0:
                    break
                time.sleep(min(left, 0.0005) if left > 0.0002 else 0)
            tickets[i] = srv.submit(g, r["problem"], r.get("k", 0), cover=False)

    th = threading.Thread(target=submitter)
    th.start()
    while len(results) < len(reqs):
        for out in srv.poll(timeout_ms=20):
            results[out["ticket"]] = out
        if not th.is_alive() and len(results) < len(reqs) and time.perf_counter() - t_start > 600:
            raise SystemExit(f"{label}: results missing")
    th.join()
    wall = time.perf_counter() - t_start
    srv.close()
    return [results[t] for t in tickets], wall


def serving_summary(res, wall, reqs):
    lat = sorted(r["done_ms"] - r["submit_ms"] for r in res)
    first = min(r["submit_ms"] for r in res)
    last = max(r["done_ms"] for r in res)
    pct = lambda q: lat[min(len(lat) - 1, int(q * len(lat)))]
    return {"instances_per_s": len(res) / ((last - first) / 1000.0),
            "latency_ms": {"p50": pct(0.50), "p90": pct(0.90), "p99": pct(0.99), "max": lat[-1]},
            "nodes": int(sum(r["nodes"] for r in res)), "wall_s": round(wall, 3),
            "mean_batch": statistics.mean(r["batch_size"] for r in res),
            "span_ms": last - first}


def load_distribution(loads):
    import numpy as np
    m = loads.mean() if loads.size and loads.mean() > 0 else 1.0
    q = lambda x: float(np.percentile(loads, x) / m)
    return {"min": float(loads.min() / m), "p25": q(25), "median": q(50), "p75": q(75),
            "max": float(loads.max() / m), "workgroups": int(loads.size)}


def activity_breakdown(cycles):
    """Mean over workgroups of each activity's share of the workgroup's own total."""
    import numpy as np
    import paper_2204_10402_amd as vc
    names = vc.ACTIVITIES
    tot = cycles[:, names.index("total")].astype(float)
    keep = tot > 0
    out = {}
    for i, name in enumerate(names):
        if name != "total":
            out[name] = float(np.mean(cycles[keep, i] / tot[keep])) if keep.any() else 0.0
    return out


def ablation_main(a):
    import graphs as G
    import paper_2204_10402_amd as vc
    insts = [("5-regular n=120 seed 0", G.random_regular(120, 5, 0)),
             ("5-regular n=120 seed 1", G.random_regular(120, 5, 1)),
             ("G(150,0.08) seed 0", G.erdos_renyi(150, 0.08, 0)),
             ("G(150,0.08) seed 1", G.erdos_renyi(150, 0.08, 1))]
    solver = vc.Solver(0)
    modes = [("hybrid", vc.Options())] + [
        (f"stack_only_d{d}", vc.Options(flags=vc.OPT_STACK_ONLY, start_depth=d)) for d in (8, 12, 16)]
    rows = []
    for name, g in insts:
        row = {"instance": name}
        for mode, o in modes:
            solver.mvc(g, o)  # warm
            t = time.perf_counter()
            r = solver.mvc(g, o)
            dt = time.perf_counter() - t
            row[mode] = {"ms": 1000 * dt, "kernel_ms": r.stats["kernel_ms"], "size": r.size,
                         "nodes": r.stats["nodes"], "load": load_distribution(solver.wg_loads())}
            log(f"{name} {mode}: {1000 * dt:.1f} ms")
        best = min((m for m, _ in modes[1:]), key=lambda m: row[m]["ms"])
        row["best_stack_only"] = best
        row["hybrid_speedup_over_best_stack_only"] = row[best]["ms"] / row["hybrid"]["ms"]
        prof = {}
        for mode, o in (("hybrid", modes[0][1]), (best, dict(modes)[best])):
            po = vc.Options(flags=o.flags | vc.OPT_PROFILE, start_depth=o.start_depth)
            solver.mvc(g, po)
            _, cyc = solver.wg_loads(cycles=True)
            prof[mode] = activity_breakdown(cyc)
        row["activity_breakdown"] = prof
        if len({row[m]["size"] for m, _ in modes}) != 1:
            raise SystemExit(f"{name}: answers differ between methods")
        rows.append(row)
    sp = [r["hybrid_speedup_over_best_stack_only"] for r in rows]
    out = {"metric": METRIC, "value": statistics.geometric_mean(sp),
           "unit": "x (hybrid over best StackOnly, geometric mean)", "n_gpus": 1,
           "steps": 1, "warmup": 1, "ms_per_step": sum(r["hybrid"]["ms"] for r in rows),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
           "data": "synthetic", "config": {"workload": "ablation: hybrid vs StackOnly",
                                           "instances": [r["instance"] for r in rows]},
           "ablation": rows}
    solver.close()
    print(json.dumps(out), flush=True)


def serving_main(a):
    import multiprocessing as mp
    import paper_2204_10402_amd as vc
    with open(TRACE) as f:
        trace = json.load(f)
    reqs = trace["requests"]
    log(f"regenerating {len(reqs)} graphs")
    with mp.get_context("fork").Pool(16) as pool:
        graphs = pool.map(_trace_graph, [(trace["master_seed"], r["draw"]) for r in reqs], chunksize=8)
    served = dict(workers=4, max_batch=32, wg_per_request=256)
    plain = dict(workers=1, max_batch=1, wg_per_request=1 << 16)  # one request, the whole GPU
    for i in range(a.warmup):
        replay(vc, graphs[:200], reqs[:200], served, "warm-up")
        log(f"warmup {i + 1}/{a.warmup} done")
    runs = []
    for i in range(a.steps):
        res, wall = replay(vc, graphs, reqs, served, "served")
        bad = [r for r, q in zip(res, reqs) if r["status"] != 0 or
               (q["problem"] == "mvc" and r["size"] != q["tau"]) or
               (q["problem"] == "pvc" and bool(r["yes"]) != q["yes"])]
        if bad:
            raise SystemExit(f"{len(bad)} served answers differ from the trace's oracle answers")
        runs.append(serving_summary(res, wall, reqs))
        log(f"step {i + 1}/{a.steps} done: {runs[-1]['instances_per_s']:.0f} requests/s")
    log("replaying the plain form (one worker, one request per launch)")
    pres, pwall = replay(vc, graphs, reqs, plain, "plain")
    base = serving_summary(pres, pwall, reqs)
    # capacity: the same requests all submitted at once
    burst = [dict(r, t_ms=0.0) for r in reqs]
    log("saturation: all requests at once, served and plain")
    sres, swall = replay(vc, graphs, burst, served, "served, saturated")
    pres2, pwall2 = replay(vc, graphs, burst, plain, "plain, saturated")
    sat = {"served": serving_summary(sres, swall, burst),
           "plain": serving_summary(pres2, pwall2, burst)}
    sat["served_over_plain"] = sat["served"]["instances_per_s"] / sat["plain"]["instances_per_s"]
    best = max(runs, key=lambda r: r["instances_per_s"])
    med = sorted(runs, key=lambda r: r["instances_per_s"])[len(runs) // 2]
    out = {
        "metric": METRIC,
        "value": med["instances_per_s"],
        "unit": "instances/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": 1000.0 * statistics.mean(r["wall_s"] for r in runs),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32", "data": "synthetic",
        "config": {"workload": "serving", "requests": len(reqs), "rate_per_s": trace["rate_per_s"],
                   "oracle_node_cap": trace["node_cap"], "discard_rate": trace["discard_rate"],
                   **served},
        "latency_ms": med["latency_ms"],
        "served": med, "best_step": best,
        "plain_sequential": base,
        "served_over_plain": med["instances_per_s"] / base["instances_per_s"],
        "saturated": sat,
        "nodes_per_s": med["nodes"] / (med["span_ms"] / 1000.0),
    }
    print(json.dumps(out), flush=True)


def algorithmic_bytes(gs, st):
    """HBM bytes the method itself must move in one call: every node copy between a
    workgroup and its stack or the worklist (st["node_bytes"]: the node's state -- degree
    array or live-vertex bitset, s, the pending vertex and the instance), plus one read of
    each graph's CSR."""
    copies = st["stack_pushes"] + st["stack_pops"] + st["wl_enqueues"] + st["wl_dequeues"]
    return st["node_bytes"] * copies + sum(4 * (g.n + 1 + g.nnz) for g in gs)


COPY_BYTES = 512 << 20


def traffic_path(workload):
    return os.path.join(ROOT, "profiles", f"traverse_kernel_{workload}_traffic.md")


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("vc_device.hip", "vc_bitset.hip", "vc_device_common.h", "vc_internal.h"):
        with open(os.path.join(ROOT, "paper_2204_10402_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload):
    """HBM bytes per traversal launch from rocprofv3 FETCH_SIZE/WRITE_SIZE, if a summary for
    the current kernel sources is on file under profiles/ (a JSON block in the .md)."""
    try:
        with open(traffic_path(workload)) as f:
            text = f.read()
        doc = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    except (OSError, ValueError, IndexError):
        return None
    if doc.get("kernel_source_hash") != kernel_source_hash():
        return None
    return doc.get("hbm_bytes_per_launch")


def read_counter_csv(directory, counter):
    """(kernel name, value) of every dispatch in a rocprofv3 --pmc CSV under `directory`."""
    import csv
    rows = []
    for dirpath, _, files in os.walk(directory):
        for f in files:
            if f.endswith("counter_collection.csv"):
                with open(os.path.join(dirpath, f)) as fh:
                    for r in csv.DictReader(fh):
                        if r.get("Counter_Name") == counter:
                            rows.append((r["Kernel_Name"], float(r["Counter_Value"])))
    if not rows:
        raise SystemExit(f"no {counter} rows under {directory}")
    return rows


def summarize_traffic(workload, fetch_dir, write_dir):
    """Per-launch HBM bytes of the traversal kernels from the two counter runs, each scaled by
    what the same counter reads for the calibration copy (COPY_BYTES read and written)."""
    out = {"workload": workload, "kernel_source_hash": kernel_source_hash()}
    for counter, directory in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = read_counter_csv(directory, counter)
        copy = [v for k, v in rows if "copy" in k.lower() or "elementwise" in k.lower()]
        trav = [v for k, v in rows if "traverse_kernel" in k]
        if not copy or not trav:
            raise SystemExit(f"{counter}: calibration copy or traversal dispatches missing")
        scale = COPY_BYTES / max(copy)  # bytes per counter unit
        out[counter] = {"dispatches": len(trav), "raw_mean": statistics.mean(trav),
                        "calibration_raw": max(copy), "bytes_per_unit": scale,
                        "bytes_per_launch": statistics.mean(trav) * scale}
    out["hbm_bytes_per_launch"] = out["FETCH_SIZE"]["bytes_per_launch"] + \
        out["WRITE_SIZE"]["bytes_per_launch"]
    with open(traffic_path(workload), "w") as f:
        f.write(f"# HBM traffic of the traversal kernel, workload {workload}\n\n"
                "Two rocprofv3 counter runs of the traffic probe, then the summary:\n\n"
                f"    rocprofv3 --pmc FETCH_SIZE --output-format csv -d FETCH_DIR -- "
                f"python3 bench.py --workload {workload} --traffic-probe\n"
                f"    rocprofv3 --pmc WRITE_SIZE --output-format csv -d WRITE_DIR -- "
                f"python3 bench.py --workload {workload} --traffic-probe\n"
                f"    python bench.py --workload {workload} --summarize-traffic FETCH_DIR WRITE_DIR\n\n"
                "Each counter is scaled by its reading for a plain elementwise kernel over "
                f"{COPY_BYTES >> 20} MiB (read once, written once) in the same run.\n\n"
                "```json\n" + json.dumps(out, indent=1) + "\n```\n")
    print(json.dumps(out))


CPU_SAMPLE_S = 10.0  # oracle work per CPU baseline: whole passes until at least this long


def cpu_baseline(workload, insts):
    """The oracle on one host core over a bounded sample of the workload: whole passes over its
    instances (hard-mvc: whole searches, one instance after another) until at least
    CPU_SAMPLE_S seconds have passed."""
    import oracle
    oracle.build(force=False)
    t0 = time.perf_counter()
    nodes = 0
    solved = 0
    passes = 0
    if workload == "hard-mvc":
        for kind, g, k, name in insts:
            nodes += oracle.mvc(g).nodes
            solved += 1
            if time.perf_counter() - t0 >= CPU_SAMPLE_S:
                break
        sample = (f"the first {solved} instances ({', '.join(n for _, _, _, n in insts[:solved])}), "
                  "whole searches")
    else:
        while True:
            for kind, g, k, name in insts:
                r = oracle.pvc(g, k) if kind == "pvc" else oracle.mvc(g)
                nodes += r.nodes
            solved += len(insts)
            passes += 1
            if time.perf_counter() - t0 >= CPU_SAMPLE_S:
                break
        sample = f"all {len(insts)} instances of the workload, {passes} passes"
    dt = time.perf_counter() - t0
    return {"value": nodes / dt, "unit": "nodes/s", "cores": 1, "kind": "oracle",
            "sample": sample, "seconds": round(dt, 3), "instances_per_s": solved / dt,
            "time_to_solve_ms": round(1000 * dt / solved, 4)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="planted-pvc", choices=WORKLOADS)
    ap.add_argument("--mode", default="batch", choices=["single", "batch"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="fixed launch knobs instead of VC_OPT_AUTOTUNE (the warm-up steps "
                         "absorb the trial launches of the first call)")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="run 2 steps and a calibration copy, for rocprofv3 --pmc")
    ap.add_argument("--summarize-traffic", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"))
    ap.add_argument("--no-single-pass", action="store_true",
                    help="skip the untimed pass of single calls (for profiles of the batched call)")
    ap.add_argument("--ablation", action="store_true",
                    help="hybrid against StackOnly on hard MVC instances (one JSON line)")
    a = ap.parse_args()
    if a.gpus != 1:
        log("bench.py measures one GPU: the traversal runs on a single MI355X and no multi-GPU "
            "path is built; run with --gpus 1")
        sys.exit(2)
    if a.summarize_traffic:
        summarize_traffic(a.workload, *a.summarize_traffic)
        return
    if a.workload == "serving":
        serving_main(a)
        return
    if a.ablation:
        ablation_main(a)
        return
    mode = a.mode

    import numpy as np
    import torch
    import paper_2204_10402_amd as vc

    insts, cfg = instances(a.workload)
    kinds = {kind for kind, _, _, _ in insts}
    assert len(kinds) == 1, "a workload is all MVC or all PVC"
    kind = kinds.pop()
    gs = [g for _, g, _, _ in insts]
    ks = [k for _, _, k, _ in insts]
    dev = torch.device("cuda:0")
    resident = []
    for _, g, k, name in insts if (mode == "single" or not a.no_single_pass) else []:
        rp = torch.from_numpy(g.row_ptr).to(dev)
        ci = torch.from_numpy(g.col_idx).to(dev)
        cover = torch.zeros(max(g.n, 1), dtype=torch.uint8, device=dev)
        resident.append((g, k, rp, ci, cover))
    n_arr, nnz_arr, rp_all, ci_all = vc.pack_batch(gs)
    rp_all_d = torch.from_numpy(rp_all).to(dev)
    ci_all_d = torch.from_numpy(ci_all).to(dev)
    cover_all_d = torch.zeros(max(int(n_arr.sum()), 1), dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    solver = vc.Solver(0, stream=torch.cuda.current_stream(dev))

    opts = vc.Options(flags=0 if a.no_autotune else vc.OPT_AUTOTUNE)

    def run_single(record):
        for g, k, rp, ci, cover in resident:
            t = time.perf_counter()
            if kind == "pvc":
                r = solver.pvc_device(rp, ci, k, cover, options=opts)
            else:
                r = solver.mvc_device(rp, ci, cover, options=opts)
            dt = time.perf_counter() - t
            if record is not None:
                record.append(([g], r.stats, dt, 1))

    def run_batch(record):
        t = time.perf_counter()
        if kind == "pvc":
            r = solver.pvc_batch_device(n_arr, nnz_arr, rp_all_d, ci_all_d, ks, cover_all_d,
                                        options=opts)
        else:
            r = solver.mvc_batch_device(n_arr, nnz_arr, rp_all_d, ci_all_d, cover_all_d,
                                        options=opts)
        dt = time.perf_counter() - t
        if not (r.status == 0).all():
            raise SystemExit("a batched instance failed: status " + str(np.unique(r.status)))
        if record is not None:
            record.append((gs, r.stats, dt, len(gs)))

    step = run_batch if mode == "batch" else run_single
    if a.traffic_probe:
        for _ in range(2):
            step(None)
        src = torch.ones(COPY_BYTES, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.add(src, 1, out=dst)  # an elementwise kernel: COPY_BYTES read, COPY_BYTES written
        torch.cuda.synchronize()
        log("traffic probe done")
        return
    for i in range(a.warmup):
        step(None)
        log(f"warmup {i + 1}/{a.warmup} done")
    torch.cuda.synchronize()
    rec = []
    t0 = time.perf_counter()
    for i in range(a.steps):
        step(rec)
        if (i + 1) % max(1, a.steps // 5) == 0:
            log(f"step {i + 1}/{a.steps} done")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    nodes = sum(st["nodes"] for _, st, _, _ in rec)
    kernel_s = sum(st["kernel_ms"] for _, st, _, _ in rec) / 1000.0
    alg_bytes = sum(algorithmic_bytes(g_list, st) for g_list, st, _, _ in rec)
    calls = len(rec)
    solved = sum(c for _, _, _, c in rec)
    avg_kernel_s = kernel_s / calls
    achieved = alg_bytes / calls / avg_kernel_s / 1e9
    traffic = measured_traffic(a.workload)
    last = rec[-1][1]
    out = {
        "metric": METRIC,
        "value": nodes / wall,
        "unit": "nodes/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1000.0 * wall / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": a.workload, "mode": mode, "instances": len(insts), **cfg,
                   "autotune": not a.no_autotune,
                   "wg_size": last["wg_size"], "num_wg": last["num_wg"],
                   "wl_capacity": last["wl_capacity"], "wl_threshold": last["wl_threshold"]},
        "nodes_per_step": nodes // a.steps,
        "instances_per_s": solved / wall,
        "call_ms": {"median": 1000 * statistics.median(dt for _, _, dt, _ in rec),
                    "max": 1000 * max(dt for _, _, dt, _ in rec),
                    "per": "batched call" if mode == "batch" else "single call"},
        "kernel_ms_avg": 1000 * avg_kernel_s,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": ("bitset_traverse_kernel" if last["bitset_words"]
                                else "traverse_kernel")
                     + (" (all launches of a call)" if mode == "batch" else ""),
                     "algorithmic_bytes_per_launch": alg_bytes / calls},
    }
    if a.no_single_pass:
        if not a.no_cpu_baseline:
            out["cpu_baseline"] = cpu_baseline(a.workload, insts)
        solver.close()
        print(json.dumps(out), flush=True)
        return
    # one untimed pass of single calls: per-instance time-to-solve, and the plain form's rate
    log("one pass of single calls (time-to-solve per instance)")
    if not a.no_autotune:
        run_single(None)  # single calls are their own size class: tune them untimed first
    torch.cuda.synchronize()
    single = []
    t = time.perf_counter()
    run_single(single)
    torch.cuda.synchronize()
    plain = time.perf_counter() - t
    tts = sorted(1000 * dt for _, _, dt, _ in single)
    out["single_calls"] = {
        "instances_per_s": len(insts) / plain, "seconds": round(plain, 4),
        "nodes_per_s": sum(st["nodes"] for _, st, _, _ in single) / plain,
        "time_to_solve_ms": {"median": statistics.median(tts),
                             "p99": tts[int(0.99 * (len(tts) - 1))], "max": tts[-1]}}
    out["batched_over_single_calls"] = out["instances_per_s"] / (len(insts) / plain)
    if not a.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(a.workload, insts)
    solver.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
