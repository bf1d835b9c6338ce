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
  hard-mvc       MVC on random 5-regular n=120 and G(150, 0.08), seeds 0-7: 16 solves per
                 step (default); the line also carries planted-pvc's time-to-solve
  planted-pvc    PVC on planted-cover graphs n=5000, |C|=400, 40,000 edges (75% C-rest),
                 k in {400, 399}, seeds 0-3: 8 solves per step
  er60-mvc       MVC on G(60, 0.10), seed 0
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

Roofline. The bitset traversal (hard-mvc) is bound by VALU instruction issue: "achieved" is
the VALU wave-instructions it issues per search-tree node (rocprofv3 SQ_INSTS_VALU over one
call's nodes) times the nodes per call and over the traversal time per call measured in this
run, against 256 CUs x 4 SIMDs x 2.4 GHz / 4 cycles = 614.4 G/s. The degree-array traversal
reports HBM: algorithmic bytes (node copies through device memory, graph data copied in, one
read of each CSR) over its time, against 8 TB/s. The counters come from the probe:
    python bench.py --workload W --probe DIR     (one warm-up call, one recorded call,
                                                  DIR/probe.json, a 512 MiB calibration kernel)
run under four rocprofv3 --pmc runs (FETCH_SIZE; WRITE_SIZE; two sets of SQ counters), then
    python bench.py --workload W --summarize-profile DIR/probe.json FETCH WRITE SQ1 SQ2
writes profiles/traverse_W_counters.md, which later runs read while the kernel sources are
unchanged. --summarize-trace summarizes a rocprofv3 --kernel-trace --stats run.
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
    """HBM bytes the method itself moves in one call: node copies that go through device memory
    (worklist enqueues and dequeues, and pushes and pops of stacks kept in device memory;
    st["hbm_node_bytes"]), the graph data workgroups copy in on taking an instance
    (st["graph_bytes"]), and one read of each graph's CSR. Stack copies of stacks held in LDS
    are not HBM traffic (st["lds_node_bytes"], reported beside)."""
    return st["hbm_node_bytes"] + st["graph_bytes"] + sum(4 * (g.n + 1 + g.nnz) for g in gs)


COPY_BYTES = 512 << 20
# MI355X: 256 CUs x 4 SIMDs at 2.4 GHz; a wavefront-64 VALU instruction occupies its SIMD for
# four cycles, so the chip issues at most 256 * 4 * 2.4e9 / 4 VALU wave-instructions per second.
VALU_PEAK_G = 256 * 4 * 2.4 / 4  # G wave-instructions / s
CUS, SIMDS, XCDS = 256, 1024, 8
SQ_SETS = (
    ("SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_INSTS_SMEM", "SQ_INSTS_FLAT",
     "SQ_WAVES", "GRBM_GUI_ACTIVE"),
    ("SQ_ACTIVE_INST_VALU", "SQ_INST_CYCLES_SALU", "SQ_ACTIVE_INST_LDS", "SQ_WAIT_INST_ANY",
     "SQ_WAVE_CYCLES", "SQ_BUSY_CYCLES", "GRBM_GUI_ACTIVE"),
)


def profile_path(workload):
    return os.path.join(ROOT, "profiles", f"traverse_{workload}_counters.md")


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("vc_device.hip", "vc_bitset.hip", "vc_device_common.h", "vc_internal.h"):
        with open(os.path.join(ROOT, "paper_2204_10402_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_profile(workload):
    """The counter summary of `workload` under profiles/ (a JSON block in the .md), if it was
    taken from the current kernel sources; else None."""
    try:
        with open(profile_path(workload)) as f:
            text = f.read()
        doc = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    except (OSError, ValueError, IndexError):
        return None
    if doc.get("kernel_source_hash") != kernel_source_hash():
        return None
    return doc


def read_counter_csv(directory, counters):
    """{dispatch id: {"kernel": name, counter: value}} of a rocprofv3 --pmc CSV under
    `directory`, for the named counters."""
    import csv
    out = {}
    for dirpath, _, files in os.walk(directory):
        for f in files:
            if f.endswith("counter_collection.csv"):
                with open(os.path.join(dirpath, f)) as fh:
                    for r in csv.DictReader(fh):
                        if r.get("Counter_Name") in counters:
                            d = out.setdefault(int(r.get("Dispatch_Id", len(out))),
                                               {"kernel": r["Kernel_Name"]})
                            d[r["Counter_Name"]] = d.get(r["Counter_Name"], 0.0) + \
                                float(r["Counter_Value"])
    if not out:
        raise SystemExit(f"no {counters} rows under {directory}")
    return out


def last_call(dispatches, launches):
    """The traversal dispatches of the probe's last call: the last `launches` dispatches whose
    kernel is a traversal kernel (trial launches of the autotuner and earlier calls excluded)."""
    trav = [d for _, d in sorted(dispatches.items()) if "traverse_kernel" in d["kernel"]]
    if len(trav) < launches:
        raise SystemExit("fewer traversal dispatches than launches per call")
    return trav[-launches:]


def summarize_profile(workload, probe_json, fetch_dir, write_dir, sq_dirs):
    """Counter summary of the traversal launches of one call (the probe's last): HBM bytes
    (FETCH_SIZE, WRITE_SIZE, each scaled by its reading for the calibration kernel that moves
    COPY_BYTES each way) and instruction counts and busy fractions (SQ_* sets), per call and per
    search-tree node. Writes profile_path(workload)."""
    with open(probe_json) as f:
        probe = json.load(f)
    launches = probe["launches_per_call"]
    out = {"workload": workload, "kernel_source_hash": kernel_source_hash(),
           "launches_per_call": launches, "nodes_per_call": probe["nodes"],
           "kernel_ms_per_call": probe["kernel_ms"], "probe_config": probe["config"]}
    for counter, directory in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = read_counter_csv(directory, (counter,))
        copy = [d[counter] for d in rows.values()
                if "copy" in d["kernel"].lower() or "elementwise" in d["kernel"].lower()]
        if not copy:
            raise SystemExit(f"{counter}: calibration kernel missing")
        scale = COPY_BYTES / max(copy)  # bytes per counter unit
        call = last_call(rows, launches)
        out[counter] = {"raw_per_call": sum(d[counter] for d in call),
                        "calibration_raw": max(copy), "bytes_per_unit": scale,
                        "bytes_per_call": sum(d[counter] for d in call) * scale,
                        "kernels": [d["kernel"][:80] for d in call]}
    out["hbm_bytes_per_call"] = out["FETCH_SIZE"]["bytes_per_call"] + \
        out["WRITE_SIZE"]["bytes_per_call"]
    sq = {}
    for names, directory in zip(SQ_SETS, sq_dirs):
        call = last_call(read_counter_csv(directory, names), launches)
        for name in names:
            if name == "GRBM_GUI_ACTIVE":
                sq.setdefault("GRBM_GUI_ACTIVE", []).append(sum(d[name] for d in call))
            else:
                sq[name] = sum(d[name] for d in call)
    # GRBM_GUI_ACTIVE is summed over the XCDs: cycles of the launches = its value / XCDS
    cycles = statistics.mean(sq.pop("GRBM_GUI_ACTIVE")) / XCDS
    nodes = probe["nodes"]
    out["instructions_per_call"] = {k: sq[k] for k in ("SQ_INSTS_VALU", "SQ_INSTS_SALU",
                                                       "SQ_INSTS_LDS", "SQ_INSTS_SMEM",
                                                       "SQ_INSTS_FLAT")}
    out["instructions_per_node"] = {k: v / nodes for k, v in out["instructions_per_call"].items()}
    out["cycles_per_call"] = cycles
    # busy fractions: VALU and LDS counters are in quad-cycles per wave, summed over the waves
    # of all SIMDs; the scalar unit is one per CU
    out["valu_busy"] = 4.0 * sq["SQ_ACTIVE_INST_VALU"] / (SIMDS * cycles)
    out["salu_busy"] = sq["SQ_INST_CYCLES_SALU"] / (CUS * cycles)
    out["lds_busy"] = 4.0 * sq["SQ_ACTIVE_INST_LDS"] / (SIMDS * cycles)
    out["wait_inst_any_per_wave_cycle"] = sq["SQ_WAIT_INST_ANY"] / max(sq["SQ_WAVE_CYCLES"], 1.0)
    out["valu_issue_frac"] = 4.0 * sq["SQ_INSTS_VALU"] / (SIMDS * cycles)
    out["raw_sq"] = sq
    cmd_pmc = ("rocprofv3 --pmc {c} --output-format csv -d {d} -- python3 bench.py --workload "
               f"{workload} --probe PROBE_DIR")
    with open(profile_path(workload), "w") as f:
        f.write(
            f"# Counters of the traversal kernels, workload {workload}\n\n"
            "One call of the workload (the probe's last; the autotuner's trial launches and the "
            "warm-up call are excluded), from four rocprofv3 counter runs of the probe, each of "
            "its own (from /tmp, TMPDIR=/tmp):\n\n"
            + "".join("    " + cmd_pmc.format(c=c, d=d) + "\n" for c, d in (
                ("FETCH_SIZE", "FETCH_DIR"), ("WRITE_SIZE", "WRITE_DIR"),
                (" ".join(SQ_SETS[0]), "SQ1_DIR"), (" ".join(SQ_SETS[1]), "SQ2_DIR")))
            + f"    python bench.py --workload {workload} --summarize-profile PROBE_DIR/probe.json "
            "FETCH_DIR WRITE_DIR SQ1_DIR SQ2_DIR\n\n"
            "FETCH_SIZE and WRITE_SIZE are scaled by what they read for a plain elementwise kernel "
            f"over {COPY_BYTES >> 20} MiB (read once, written once) in the same run. "
            "GRBM_GUI_ACTIVE is summed over the 8 XCDs. Busy fractions: VALU and LDS "
            "instruction cycles (quad-cycles per wave, summed over waves) over the 1,024 SIMDs' "
            "cycles; scalar ALU cycles over the 256 CUs' cycles.\n\n"
            f"| per call | value |\n|---|---|\n"
            f"| search-tree nodes | {nodes:,} |\n"
            f"| HBM bytes (FETCH + WRITE) | {out['hbm_bytes_per_call']:,.0f} |\n"
            + "".join(f"| {k} per node | {v:.1f} |\n" for k, v in out["instructions_per_node"].items())
            + f"| VALU busy | {out['valu_busy']:.3f} |\n| scalar ALU busy | {out['salu_busy']:.3f} |\n"
            f"| LDS busy | {out['lds_busy']:.3f} |\n\n"
            "```json\n" + json.dumps(out, indent=1) + "\n```\n")
    print(json.dumps(out))


def summarize_trace(workload, directory, steps):
    """profiles/kernel_trace_<workload>.md from a rocprofv3 --kernel-trace --stats run of
    `bench.py --workload W --steps K --warmup 1 --no-single-pass --no-cpu-baseline
    --no-time-to-solve`: the whole-run kernel summary and each traversal kernel's average over
    its last K dispatches (the timed steps)."""
    import csv
    stats = trace = None
    for dirpath, _, files in os.walk(directory):
        for f in files:
            if f.endswith("kernel_stats.csv"):
                stats = os.path.join(dirpath, f)
            if f.endswith("kernel_trace.csv"):
                trace = os.path.join(dirpath, f)
    if not stats or not trace:
        raise SystemExit("kernel_stats.csv / kernel_trace.csv missing")
    with open(stats) as fh:
        srows = list(csv.DictReader(fh))
    with open(trace) as fh:
        trows = list(csv.DictReader(fh))
    per = {}
    for r in trows:
        name = r["Kernel_Name"]
        if "traverse_kernel" in name:
            # one launch per kernel family and call: the degree-array kernel's instantiations
            # (its memory-mode argument differs between the autotuner's trials) are one family
            key = ("degree arrays: " + name.split("<")[0]) if "bitset" not in name else name
            per.setdefault(key, []).append(
                (int(r["Start_Timestamp"]), int(r["End_Timestamp"]) - int(r["Start_Timestamp"]), name))
    lines = [f"# Kernel trace: {workload}\n",
             "Command (from /tmp, with TMPDIR=/tmp):\n",
             "```",
             f"rocprofv3 --kernel-trace --stats --output-format csv -d TRACE_DIR -o run -- python3 "
             f"bench.py --workload {workload} --steps {steps} --warmup 1 --no-single-pass "
             "--no-cpu-baseline --no-time-to-solve",
             f"python bench.py --workload {workload} --summarize-trace TRACE_DIR --steps {steps}",
             "```\n",
             "Whole run (`run_kernel_stats.csv`; includes the warm-up call and the autotuner's "
             "trial launches):\n",
             "| kernel | calls | total (us) | average (us) | % of GPU time |", "|---|---|---|---|---|"]
    for r in srows:
        name = r["Name"] if len(r["Name"]) <= 80 else r["Name"][:77] + "..."
        lines.append(f"| `{name}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e3:.1f} | "
                     f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |")
    lines += ["", f"Timed steps only (the last {steps} dispatches of each traversal kernel family):",
              "", "| kernel | average over the timed steps (us) |", "|---|---|"]
    for k, v in sorted(per.items()):
        v = sorted(v)[-steps:]
        names = sorted({n for _, _, n in v})
        lines.append(f"| `{' / '.join(names)}` | {statistics.mean(d for _, d, _ in v) / 1e3:.1f} |")
    text = "\n".join(lines) + "\n"
    with open(os.path.join(ROOT, "profiles", f"kernel_trace_{workload}.md"), "w") as f:
        f.write(text)
    print(text)


CPU_SAMPLE_S = 10.0  # oracle work per CPU baseline: whole passes until at least this long


def hard_sample():
    """hard-mvc's CPU sample: one whole search per family, the instance of each family with the
    fewest oracle nodes: (family, seed, graph)."""
    import graphs as G
    return [("5-regular n=120", 3, G.random_regular(120, 5, 3)),
            ("G(150, 0.08)", 7, G.erdos_renyi(150, 0.08, 7))]


def cpu_baseline(workload, insts):
    """The oracle on one host core over a bounded sample of the workload. hard-mvc: one whole
    search per family (5-regular n=120 seed 3, G(150, 0.08) seed 7), nodes/s per family and
    over both; other workloads: whole passes over every instance until at least CPU_SAMPLE_S
    seconds have passed."""
    import oracle
    oracle.build(force=False)
    if workload == "hard-mvc":
        fam = {}
        nodes = 0
        t0 = time.perf_counter()
        for label, seed, g in hard_sample():
            t = time.perf_counter()
            r = oracle.mvc(g)
            dt = time.perf_counter() - t
            nodes += r.nodes
            fam[label] = {"seed": seed, "nodes": r.nodes, "seconds": round(dt, 6),
                          "nodes_per_s": r.nodes / dt, "size": r.size}
        dt = time.perf_counter() - t0
        return {"value": nodes / dt, "unit": "nodes/s", "cores": 1, "kind": "oracle",
                "sample": "whole searches of one instance per family: "
                          + ", ".join(f"{k} seed {v['seed']}" for k, v in fam.items()),
                "seconds": round(dt, 6), "families": fam,
                "instances_per_s": len(fam) / dt,
                "time_to_solve_ms": round(1000 * dt / len(fam), 3)}
    t0 = time.perf_counter()
    nodes = solved = passes = 0
    while True:
        for kind, g, k, name in insts:
            r = oracle.pvc(g, k) if kind == "pvc" else oracle.mvc(g)
            nodes += r.nodes
        solved += len(insts)
        passes += 1
        if time.perf_counter() - t0 >= CPU_SAMPLE_S:
            break
    dt = time.perf_counter() - t0
    return {"value": nodes / dt, "unit": "nodes/s", "cores": 1, "kind": "oracle",
            "sample": f"all {len(insts)} instances of the workload, {passes} passes",
            "seconds": round(dt, 6), "instances_per_s": solved / dt,
            "time_to_solve_ms": round(1000 * dt / solved, 4)}


class Runner:
    """The instances of one workload resident in device memory, and one solver context."""

    def __init__(self, workload, autotune=True, single=True):
        import torch
        import paper_2204_10402_amd as vc
        self.vc, self.torch = vc, torch
        self.workload = workload
        self.insts, self.cfg = instances(workload)
        kinds = {kind for kind, _, _, _ in self.insts}
        assert len(kinds) == 1, "a workload is all MVC or all PVC"
        self.kind = kinds.pop()
        self.gs = [g for _, g, _, _ in self.insts]
        self.ks = [k for _, _, k, _ in self.insts]
        dev = torch.device("cuda:0")
        self.resident = []
        for _, g, k, name in (self.insts if single else []):
            rp = torch.from_numpy(g.row_ptr).to(dev)
            ci = torch.from_numpy(g.col_idx).to(dev)
            cover = torch.zeros(max(g.n, 1), dtype=torch.uint8, device=dev)
            self.resident.append((g, k, rp, ci, cover))
        self.n_arr, self.nnz_arr, rp_all, ci_all = vc.pack_batch(self.gs)
        self.rp_all = torch.from_numpy(rp_all).to(dev)
        self.ci_all = torch.from_numpy(ci_all).to(dev)
        self.cover_all = torch.zeros(max(int(self.n_arr.sum()), 1), dtype=torch.uint8, device=dev)
        torch.cuda.synchronize()
        self.solver = vc.Solver(0, stream=torch.cuda.current_stream(dev))
        self.opts = vc.Options(flags=vc.OPT_AUTOTUNE if autotune else 0)

    def single(self, record):
        for g, k, rp, ci, cover in self.resident:
            t = time.perf_counter()
            if self.kind == "pvc":
                r = self.solver.pvc_device(rp, ci, k, cover, options=self.opts)
            else:
                r = self.solver.mvc_device(rp, ci, cover, options=self.opts)
            dt = time.perf_counter() - t
            if record is not None:
                record.append(([g], r.stats, dt, 1))

    def batch(self, record):
        t = time.perf_counter()
        if self.kind == "pvc":
            r = self.solver.pvc_batch_device(self.n_arr, self.nnz_arr, self.rp_all, self.ci_all,
                                             self.ks, self.cover_all, options=self.opts)
        else:
            r = self.solver.mvc_batch_device(self.n_arr, self.nnz_arr, self.rp_all, self.ci_all,
                                             self.cover_all, options=self.opts)
        dt = time.perf_counter() - t
        if not (r.status == 0).all():
            raise SystemExit("a batched instance failed: status " + str(set(r.status.tolist())))
        if record is not None:
            record.append((self.gs, r.stats, dt, len(self.gs)))

    def timed(self, step, steps, warmup, label):
        for i in range(warmup):
            step(None)
            log(f"{label}: warmup {i + 1}/{warmup} done")
        self.torch.cuda.synchronize()
        rec = []
        t0 = time.perf_counter()
        for i in range(steps):
            step(rec)
            if (i + 1) % max(1, steps // 5) == 0:
                log(f"{label}: step {i + 1}/{steps} done")
        self.torch.cuda.synchronize()
        return rec, time.perf_counter() - t0

    def close(self):
        self.solver.close()


def single_pass(runner, autotune):
    """One untimed pass of single calls after tuning them: per-instance time-to-solve and the
    plain form's throughput."""
    if autotune:
        runner.single(None)  # single calls are their own size class: tune them first
    runner.torch.cuda.synchronize()
    rec = []
    t = time.perf_counter()
    runner.single(rec)
    runner.torch.cuda.synchronize()
    plain = time.perf_counter() - t
    tts = sorted(1000 * dt for _, _, dt, _ in rec)
    return {"instances_per_s": len(rec) / plain, "seconds": round(plain, 4),
            "nodes_per_s": sum(st["nodes"] for _, st, _, _ in rec) / plain,
            "time_to_solve_ms": {"median": statistics.median(tts),
                                 "p99": tts[int(0.99 * (len(tts) - 1))], "max": tts[-1]}}


def roofline(workload, rec, kernel_s_per_call, nodes_per_call, alg_per_call):
    """Roofline object of the traversal kernels. Bitset launches (all of a hard-mvc call) are
    bound by VALU issue: achieved = VALU wave-instructions per node (rocprofv3 SQ_INSTS_VALU of
    one call over its nodes, from the counter summary under profiles/ when it matches the
    kernel sources) x nodes per call measured here / traversal time per call measured here,
    against 614.4 G/s. Degree-array launches report the HBM roofline of their algorithmic
    bytes."""
    last = rec[-1][1]
    prof = measured_profile(workload)
    traffic = prof["hbm_bytes_per_call"] if prof else None
    hbm = {"bound": "hbm", "achieved": alg_per_call / kernel_s_per_call / 1e9,
           "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": alg_per_call / kernel_s_per_call / 1e9 / HBM_PEAK_GBS, "traffic": traffic,
           "algorithmic_bytes_per_call": alg_per_call,
           "lds_node_bytes_per_call": statistics.mean(st["lds_node_bytes"] for _, st, _, _ in rec)}
    kernel = ("bitset_traverse_kernel" if last["bitset_words"] else "traverse_kernel") + \
        f" ({last['launches']} launch{'es' if last['launches'] > 1 else ''} per call)"
    if last["bitset_words"] and prof:
        per_node = prof["instructions_per_node"]["SQ_INSTS_VALU"]
        achieved = per_node * nodes_per_call / kernel_s_per_call / 1e9
        return {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_G,
                "unit": "G VALU wave-instructions/s", "frac": achieved / VALU_PEAK_G,
                "traffic": traffic, "kernel": kernel,
                "valu_instructions_per_node": per_node,
                "counters": {"valu_busy": prof["valu_busy"], "salu_busy": prof["salu_busy"],
                             "lds_busy": prof["lds_busy"],
                             "per_node": prof["instructions_per_node"]},
                "hbm": hbm}
    return dict(hbm, kernel=kernel)


def time_to_solve(autotune, steps=20, warmup=3):
    """planted-pvc time-to-solve beside the main line: 8 PVC instances of 5,000 vertices (k =
    400 and 399, seeds 0-3) that the rules settle at the root."""
    r = Runner("planted-pvc", autotune)
    rec, wall = r.timed(r.batch, steps, warmup, "planted-pvc")
    single = single_pass(r, autotune)
    r.close()
    calls = sorted(1000 * dt for _, _, dt, _ in rec)
    return {"workload": "planted-pvc", "instances": len(r.insts),
            "batched_call_ms": {"median": statistics.median(calls), "max": calls[-1]},
            "instances_per_s": len(r.insts) * len(rec) / wall,
            "traversal_ms_per_call": statistics.mean(st["kernel_ms"] for _, st, _, _ in rec),
            "single_calls": single}


def probe(workload, directory, autotune):
    """For rocprofv3 counter runs: one warm-up call (the autotuner's trials), one recorded call,
    its statistics in DIRECTORY/probe.json, then the calibration kernel."""
    os.makedirs(directory, exist_ok=True)
    r = Runner(workload, autotune, single=False)
    r.batch(None)
    rec = []
    r.batch(rec)
    r.torch.cuda.synchronize()
    st = rec[0][1]
    with open(os.path.join(directory, "probe.json"), "w") as f:
        json.dump({"workload": workload, "nodes": st["nodes"], "kernel_ms": st["kernel_ms"],
                   "launches_per_call": st["launches"],
                   "config": {"num_wg": st["num_wg"], "wg_size": st["wg_size"],
                              "wl_threshold": st["wl_threshold"]},
                   "stats": {k: v for k, v in st.items() if k != "cycles"}}, f)
    src = r.torch.ones(COPY_BYTES, dtype=r.torch.uint8, device="cuda:0")
    dst = r.torch.empty_like(src)
    r.torch.cuda.synchronize()
    r.torch.add(src, 1, out=dst)  # an elementwise kernel: COPY_BYTES read, COPY_BYTES written
    r.torch.cuda.synchronize()
    r.close()
    log("probe done")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="hard-mvc", choices=WORKLOADS)
    ap.add_argument("--mode", default="batch", choices=["single", "batch"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="fixed launch knobs instead of VC_OPT_AUTOTUNE (the warm-up steps "
                         "absorb the trial launches of the first call)")
    ap.add_argument("--probe", metavar="DIR",
                    help="one warm-up call, one recorded call (DIR/probe.json) and a calibration "
                         "kernel, for rocprofv3 counter runs")
    ap.add_argument("--summarize-profile", nargs=5,
                    metavar=("PROBE_JSON", "FETCH_DIR", "WRITE_DIR", "SQ1_DIR", "SQ2_DIR"))
    ap.add_argument("--summarize-trace", metavar="TRACE_DIR")
    ap.add_argument("--no-single-pass", action="store_true",
                    help="skip the untimed pass of single calls (for profiles of the batched call)")
    ap.add_argument("--no-time-to-solve", action="store_true",
                    help="skip the planted-pvc time-to-solve block of the hard-mvc line")
    ap.add_argument("--ablation", action="store_true",
                    help="hybrid against StackOnly on hard MVC instances (one JSON line)")
    a = ap.parse_args()
    if a.gpus != 1:
        log("bench.py measures one GPU: the traversal runs on a single MI355X and no multi-GPU "
            "path is built; run with --gpus 1")
        sys.exit(2)
    if a.summarize_profile:
        summarize_profile(a.workload, a.summarize_profile[0], a.summarize_profile[1],
                          a.summarize_profile[2], a.summarize_profile[3:])
        return
    if a.summarize_trace:
        summarize_trace(a.workload, a.summarize_trace, a.steps)
        return
    if a.workload == "serving":
        serving_main(a)
        return
    if a.ablation:
        ablation_main(a)
        return
    autotune = not a.no_autotune
    if a.probe:
        probe(a.workload, a.probe, autotune)
        return
    mode = a.mode
    run = Runner(a.workload, autotune, single=(mode == "single" or not a.no_single_pass))
    rec, wall = run.timed(run.batch if mode == "batch" else run.single, a.steps, a.warmup,
                          a.workload)
    nodes = sum(st["nodes"] for _, st, _, _ in rec)
    calls = len(rec)
    kernel_s_per_call = sum(st["kernel_ms"] for _, st, _, _ in rec) / 1000.0 / calls
    alg_per_call = sum(algorithmic_bytes(g_list, st) for g_list, st, _, _ in rec) / calls
    solved = sum(c for _, _, _, c in rec)
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
        "config": {"workload": a.workload, "mode": mode, "instances": len(run.insts), **run.cfg,
                   "autotune": autotune,
                   "wg_size": last["wg_size"], "num_wg": last["num_wg"],
                   "wl_capacity": last["wl_capacity"], "wl_threshold": last["wl_threshold"]},
        "nodes_per_step": nodes // a.steps,
        "instances_per_s": solved / wall,
        "call_ms": {"median": 1000 * statistics.median(dt for _, _, dt, _ in rec),
                    "max": 1000 * max(dt for _, _, dt, _ in rec),
                    "per": "batched call" if mode == "batch" else "single call"},
        "kernel_ms_avg": 1000 * kernel_s_per_call,
        "roofline": roofline(a.workload, rec, kernel_s_per_call, nodes / calls, alg_per_call),
    }
    if not a.no_single_pass:
        log("one pass of single calls (time-to-solve per instance)")
        out["single_calls"] = single_pass(run, autotune)
        out["batched_over_single_calls"] = out["instances_per_s"] / \
            out["single_calls"]["instances_per_s"]
    run.close()
    if a.workload == "hard-mvc" and not a.no_time_to_solve:
        log("time-to-solve of planted-pvc")
        out["time_to_solve"] = time_to_solve(autotune)
    if not a.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(a.workload, run.insts)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
