"""Parity of the HIP path (libvc.so, called through the C ABI) with the CPU oracle.

The bar (integer work, exact): MVC size and PVC decision identical to the oracle on every
instance; every returned cover verified edge by edge here as well as in the library; the
greedy cover and the reduction-rule fixpoint identical to the oracle's, vertex by vertex;
node counts identical where the tree does not depend on the schedule (one workgroup that
never donates; PVC instances whose answer is no).
"""

import json
import os

import numpy as np
import pytest

import graphs as G
import oracle

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


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


# kernel families: bitsets (n <= 512), degree arrays with the node in LDS, and degree arrays
# with the node in device memory (chosen automatically only when the node does not fit in LDS)
# degree_arrays stages small graphs' CSR in LDS; csr_global reads it from device memory
KERNELS = {"bitsets": 0x40, "degree_arrays": 0x20, "csr_global": 0x420, "global_nodes": 0x200}


def single_wg(flags=0):
    import paper_2204_10402_amd as vc
    return vc.Options(num_wg=1, wl_threshold=-1, flags=flags)


def opts(**kw):
    import paper_2204_10402_amd as vc
    return vc.Options(**kw)


def check_cover(g, cover, size):
    cover = np.asarray(cover)
    assert cover.shape == (g.n,)
    assert set(np.unique(cover).tolist()) <= {0, 1}
    assert oracle.is_cover(g, cover)
    assert int(cover.sum()) == size


def golden():
    with open(os.path.join(GOLDEN, "oracle_answers.json")) as f:
        return json.load(f)["results"]


# ---- small graphs: answers, covers and node counts ----------------------------------------

@pytest.mark.parametrize("kernel", sorted(KERNELS))
@pytest.mark.parametrize("seed", range(40))
def test_small_mvc_and_pvc(solver, oracle_lib, seed, kernel):
    n = 5 + seed % 14
    g = G.random_small(n, 20000 + seed) if seed % 2 else G.erdos_renyi(n, 0.3, 20000 + seed)
    tau, _ = oracle.tau_by_definition(g)
    o = opts(flags=KERNELS[kernel])
    r = solver.mvc(g, o)
    assert r.size == tau
    assert (r.stats["bitset_words"] > 0) == (kernel == "bitsets")
    check_cover(g, r.cover, tau)
    for k in (max(tau - 2, 0), tau - 1, tau, tau + 1):
        if k < 0:
            continue
        p = solver.pvc(g, k, o)
        assert p.yes == (k >= tau)
        if p.yes:
            check_cover(g, p.cover, p.size)
            assert p.size <= k
        else:
            assert p.size == -1 and int(p.cover.sum()) == 0


@pytest.mark.parametrize("kernel", sorted(KERNELS))
@pytest.mark.parametrize("seed", range(12))
def test_single_workgroup_node_parity(solver, oracle_lib, seed, kernel):
    """One workgroup that never donates visits the oracle's tree in the oracle's order."""
    g = G.erdos_renyi(30 + 7 * seed, 0.12 + 0.01 * (seed % 5), 300 + seed)
    o = oracle.mvc(g)
    r = solver.mvc(g, single_wg(KERNELS[kernel]))
    assert (r.size, r.stats["nodes"], r.stats["greedy_size"]) == (o.size, o.nodes, o.greedy)
    check_cover(g, r.cover, o.size)
    for k in (o.size - 1, o.size):
        op = oracle.pvc(g, k)
        gp = solver.pvc(g, k, single_wg(KERNELS[kernel]))
        assert (gp.yes, gp.stats["nodes"]) == (op.yes, op.nodes)


def test_c1_er60(solver, oracle_lib):
    """MVC on G(60, 0.10), seed 0, plain method (one persistent launch, all workgroups)."""
    g = G.erdos_renyi(60, 0.10, 0)
    o = oracle.mvc(g)
    r = solver.mvc(g)
    assert r.size == o.size == 37
    check_cover(g, r.cover, o.size)
    assert r.stats["greedy_size"] == o.greedy
    one = solver.mvc(g, single_wg())
    assert one.stats["nodes"] == o.nodes
    arr = solver.mvc(g, opts(flags=KERNELS["degree_arrays"]))
    assert arr.size == o.size


@pytest.mark.parametrize("kernel", sorted(KERNELS))
@pytest.mark.parametrize("rules", [0x1, 0x2, 0x4, 0x8, 0x3])
def test_ablation_flags(solver, oracle_lib, rules, kernel):
    """Switching rules off leaves tau unchanged; single-workgroup node counts follow the
    oracle with the same rules switched off."""
    import paper_2204_10402_amd as vc
    mask = oracle.ALL
    if rules & vc.OPT_NO_DEGREE_ONE:
        mask &= ~oracle.RULE_DEG1
    if rules & vc.OPT_NO_TRIANGLE:
        mask &= ~oracle.RULE_TRI
    if rules & vc.OPT_NO_HIGH_DEGREE:
        mask &= ~(oracle.RULE_HIGH | oracle.PRUNE_EDGES)
    if rules & vc.OPT_NO_EDGE_PRUNE:
        mask &= ~oracle.PRUNE_EDGES
    for seed in range(4):
        g = G.erdos_renyi(40, 0.12, 700 + seed)
        o = oracle.mvc(g, rules=mask)
        r = solver.mvc(g, vc.Options(num_wg=1, wl_threshold=-1, flags=rules | KERNELS[kernel]))
        assert (r.size, r.stats["nodes"]) == (o.size, o.nodes)
        assert solver.mvc(g, vc.Options(flags=rules | KERNELS[kernel])).size == o.size


# ---- reduction rules and greedy: vertex-by-vertex parity --------------------------------

def random_consistent_state(g, rng, frac):
    """A degree array of the graph with a random vertex set already in the cover."""
    removed = rng.random(g.n) < frac
    deg = np.zeros(g.n, np.int32)
    for v in range(g.n):
        if removed[v]:
            deg[v] = -1
        else:
            nb = g.neighbors(v)
            deg[v] = int(np.sum(~removed[nb]))
    return deg, int(removed.sum())


@pytest.mark.parametrize("kernel", sorted(KERNELS))
@pytest.mark.parametrize("seed", range(30))
def test_reduce_fixpoint_parity(solver, oracle_lib, torch_cuda, seed, kernel):
    torch = torch_cuda
    rng = np.random.default_rng(900 + seed)
    n = [12, 40, 63, 64, 65, 130, 200, 256, 700][seed % 9]
    if kernel == "bitsets" and n > 512:
        n = 193
    g = G.random_small(n, 900 + seed) if n <= 40 else G.erdos_renyi(n, float(rng.uniform(0.02, 0.1)), seed)
    deg, s = random_consistent_state(g, rng, float(rng.uniform(0.0, 0.4)))
    rp = torch.from_numpy(g.row_ptr).cuda()
    ci = torch.from_numpy(g.col_idx.copy() if g.nnz else np.zeros(1, np.int32)).cuda()[:g.nnz]
    for bound, flags in ((10**9, 0x4), (s + n // 3, 0), (s + 2, 0), (s, 0), (s - 1, 0),
                         (s + n // 4, 0x1), (s + n // 4, 0x2)):
        mask = oracle.ALL
        if flags & 0x1:
            mask &= ~oracle.RULE_DEG1
        if flags & 0x2:
            mask &= ~oracle.RULE_TRI
        if flags & 0x4:
            mask &= ~(oracle.RULE_HIGH | oracle.PRUNE_EDGES)
        od, os_ = oracle.reduce(g, deg, s, bound, mask)
        dd = torch.from_numpy(deg.copy()).cuda()
        gs = solver.reduce_device(rp, ci, dd, s, bound, flags | KERNELS[kernel])
        assert gs == os_, (bound, flags)
        assert np.array_equal(dd.cpu().numpy(), od), (bound, flags)


@pytest.mark.parametrize("kernel", ["degree_arrays", "csr_global", "global_nodes"])
@pytest.mark.parametrize("bound,flags", [(60, 0), (100, 0), (200, 0), (10**9, 0x4), (10**9, 0x5)])
def test_reduce_fixpoint_planted_full_size(solver, oracle_lib, torch_cuda, kernel, bound, flags):
    """The root reduction of a 5,000-vertex planted graph (rows of about 125 entries, walked in
    64-entry pieces by a 1,024-thread workgroup through its removal list), element by element
    against the oracle's fixpoint, on every degree-array memory placement. Bounds 60 and 200
    stop the cascade midway; at bound 100 the high-degree rule removes 1,488 vertices, more
    than the removal list holds; without the high-degree rule, and with the triangle rule
    alone, the fixpoints differ again."""
    torch = torch_cuda
    g = G.planted_cover(5000, 400, 40000, 0.75, 1)
    deg = np.diff(g.row_ptr).astype(np.int32)
    mask = oracle.ALL
    if flags & 0x1:
        mask &= ~oracle.RULE_DEG1
    if flags & 0x2:
        mask &= ~oracle.RULE_TRI
    if flags & 0x4:
        mask &= ~(oracle.RULE_HIGH | oracle.PRUNE_EDGES)
    od, os_ = oracle.reduce(g, deg, 0, bound, mask)
    rp = torch.from_numpy(g.row_ptr).cuda()
    ci = torch.from_numpy(g.col_idx).cuda()
    dd = torch.from_numpy(deg.copy()).cuda()
    assert solver.reduce_device(rp, ci, dd, 0, bound, flags | KERNELS[kernel]) == os_
    assert np.array_equal(dd.cpu().numpy(), od)


@pytest.mark.parametrize("kernel", ["degree_arrays", "csr_global", "global_nodes"])
@pytest.mark.parametrize("shape", ["matching", "triangles"])
def test_removal_step_beyond_the_list(solver, oracle_lib, torch_cuda, kernel, shape):
    """One removal step of more than 1,024 vertices, the capacity of a workgroup's removal list
    (the rest are taken in further rounds): 1,500 disjoint edges, where the degree-one rule
    removes one end of every edge in a single pass, or 1,100 disjoint triangles, where the
    triangle rule removes two vertices of each. The fixpoint equals the oracle's element by
    element; MVC gives tau and a valid cover; PVC at tau - 1 visits the oracle's node count."""
    import paper_2204_10402_amd as vc
    torch = torch_cuda
    if shape == "matching":
        g, tau = G.disjoint_union(*([G.path(2)] * 1500)), 1500
    else:
        g, tau = G.disjoint_union(*([G.complete(3)] * 1100)), 2200
    deg = np.diff(g.row_ptr).astype(np.int32)
    od, os_ = oracle.reduce(g, deg, 0, 10**9, oracle.ALL & ~(oracle.RULE_HIGH | oracle.PRUNE_EDGES))
    assert os_ == tau
    rp = torch.from_numpy(g.row_ptr).cuda()
    ci = torch.from_numpy(g.col_idx).cuda()
    dd = torch.from_numpy(deg.copy()).cuda()
    assert solver.reduce_device(rp, ci, dd, 0, 10**9, 0x4 | KERNELS[kernel]) == tau
    assert np.array_equal(dd.cpu().numpy(), od)
    r = solver.mvc(g, vc.Options(flags=KERNELS[kernel]))
    assert r.size == tau
    check_cover(g, r.cover, tau)
    p = solver.pvc(g, tau - 1, vc.Options(flags=KERNELS[kernel]))
    assert not p.yes and p.stats["nodes"] == oracle.pvc(g, tau - 1).nodes


@pytest.mark.parametrize("n,p,seed", [(60, 0.1, 0), (150, 0.08, 1), (500, 0.02, 2),
                                      (2000, 0.004, 3), (5000, 0.0016, 4)])
def test_greedy_parity(solver, oracle_lib, torch_cuda, n, p, seed):
    torch = torch_cuda
    g = G.erdos_renyi(n, p, seed)
    size, cover = oracle.greedy(g)
    rp = torch.from_numpy(g.row_ptr).cuda()
    ci = torch.from_numpy(g.col_idx).cuda()
    out = torch.zeros(n, dtype=torch.uint8, device="cuda")
    assert solver.greedy_device(rp, ci, out) == size
    assert np.array_equal(out.cpu().numpy(), cover)


def test_greedy_planted_full_size(solver, oracle_lib, torch_cuda):
    torch = torch_cuda
    g = G.planted_cover(5000, 400, 40000, 0.75, 0)
    size, cover = oracle.greedy(g)
    out = torch.zeros(g.n, dtype=torch.uint8, device="cuda")
    got = solver.greedy_device(torch.from_numpy(g.row_ptr).cuda(),
                               torch.from_numpy(g.col_idx).cuda(), out)
    assert got == size and np.array_equal(out.cpu().numpy(), cover)


# ---- full-size workloads -----------------------------------------------------------------

@pytest.mark.parametrize("seed", range(4))
def test_planted_pvc_full_size(solver, oracle_lib, torch_cuda, seed):
    """PVC on planted-cover graphs, n = 5000, |C| = 400, 40,000 edges, k = 400 and 399, through
    the device-resident entry point the benchmark times."""
    torch = torch_cuda
    ans = {(r["seed"], r["k"]): r for r in golden() if r["workload"] == "pvc_planted"}
    g = G.planted_cover(5000, 400, 40000, 0.75, seed)
    rp = torch.from_numpy(g.row_ptr).cuda()
    ci = torch.from_numpy(g.col_idx).cuda()
    for k in (400, 399):
        cover = torch.zeros(g.n, dtype=torch.uint8, device="cuda")
        r = solver.pvc_device(rp, ci, k, cover)
        want = ans[(seed, k)]
        assert r.yes == want["yes"]
        # the answer is "no" at 399: the tree cannot depend on the schedule
        if not want["yes"]:
            assert r.stats["nodes"] == want["nodes"]
            assert int(cover.sum().item()) == 0
        else:
            check_cover(g, cover.cpu().numpy(), r.size)
            assert r.size <= k
        h = solver.pvc(g, k)
        assert h.yes == want["yes"]


@pytest.mark.parametrize("workload,seed", [("mvc_reg120", s) for s in range(8)] +
                         [("mvc_er150", s) for s in range(8)])
def test_hard_mvc_full_size(solver, oracle_lib, workload, seed):
    """MVC on random 5-regular n=120 and G(150, 0.08), seeds 0-7: deep imbalanced trees that
    exercise donation and termination. tau must equal the oracle's (stored by
    tests/golden/make_oracle_answers.py)."""
    want = {(r["workload"], r["seed"]): r for r in golden()}[(workload, seed)]
    g = G.random_regular(120, 5, seed) if workload == "mvc_reg120" else G.erdos_renyi(150, 0.08, seed)
    r = solver.mvc(g)
    assert r.size == want["size"]
    assert r.stats["greedy_size"] == want["greedy"]
    check_cover(g, r.cover, want["size"])
    assert r.stats["nodes"] > 0


@pytest.mark.parametrize("workload,seed", [("mvc_reg120", 1), ("mvc_er150", 7)])
def test_hard_mvc_degree_arrays(solver, oracle_lib, workload, seed):
    """The degree-array kernels on two of the hard instances (the bitset kernels run them by
    default)."""
    want = {(r["workload"], r["seed"]): r for r in golden()}[(workload, seed)]
    g = G.random_regular(120, 5, seed) if workload == "mvc_reg120" else G.erdos_renyi(150, 0.08, seed)
    r = solver.mvc(g, opts(flags=KERNELS["degree_arrays"]))
    assert r.size == want["size"] and r.stats["bitset_words"] == 0
    check_cover(g, r.cover, want["size"])


def test_hard_pvc_no_node_parity(solver, oracle_lib):
    """PVC k = tau - 1 (no instance): every workgroup schedule visits the same tree."""
    want = {(r["workload"], r["seed"]): r for r in golden()}[("mvc_reg120", 3)]
    g = G.random_regular(120, 5, 3)
    o = oracle.pvc(g, want["size"] - 1)
    r = solver.pvc(g, want["size"] - 1)
    assert not o.yes and not r.yes
    assert r.stats["nodes"] == o.nodes
    r2 = solver.pvc(g, want["size"] - 1, opts(flags=KERNELS["degree_arrays"]))
    assert not r2.yes and r2.stats["nodes"] == o.nodes
    y = solver.pvc(g, want["size"])
    assert y.yes and y.size <= want["size"]
    check_cover(g, y.cover, y.size)


@pytest.mark.parametrize("kernel", ["bitsets", "degree_arrays"])
def test_hard_pvc_no_node_parity_all_instances(solver, kernel):
    """PVC k = tau - 1 on all 16 hard graphs (5-regular n=120 and G(150, 0.08), seeds 0-7) in
    one batched call per kernel family: every answer no, and every instance's node count equal
    to the oracle's stored count (the tree does not depend on the schedule)."""
    want = [r for r in golden() if r["workload"] in ("pvc_reg120", "pvc_er150")]
    assert len(want) == 16
    gs = [G.random_regular(120, 5, r["seed"]) if r["workload"] == "pvc_reg120"
          else G.erdos_renyi(150, 0.08, r["seed"]) for r in want]
    res = solver.pvc_batch(gs, [r["k"] for r in want], opts(flags=KERNELS[kernel]))
    for i, r in enumerate(want):
        assert res.status[i] == 0 and not res.yes[i], (r["workload"], r["seed"])
        assert res.nodes[i] == r["nodes"], (r["workload"], r["seed"])


# ---- edge cases -----------------------------------------------------------------------------

def test_edge_cases(solver, oracle_lib):
    import paper_2204_10402_amd as vc
    e = G.empty(7)
    assert solver.mvc(e).size == 0 and int(solver.mvc(e).cover.sum()) == 0
    p = solver.pvc(e, 0)
    assert p.yes and p.size == 0
    assert solver.mvc(G.empty(0)).size == 0
    one = G.path(2)
    assert solver.mvc(one).size == 1
    assert not solver.pvc(one, 0).yes and solver.pvc(one, 1).yes
    k5 = G.complete(5)
    r = solver.pvc(k5, 10**6)  # k far above n
    assert r.yes and r.size <= 5
    check_cover(k5, r.cover, r.size)
    with pytest.raises(vc.VCError) as ei:
        solver.pvc(k5, -1)
    assert ei.value.code == vc.ERR_INVALID_ARG


@pytest.mark.parametrize("n", [63, 64, 65, 127, 128, 129, 191, 1000, 1025])
def test_ragged_sizes(solver, oracle_lib, n):
    g = G.disjoint_union(G.cycle(n // 2 + 3), G.path(n - n // 2 - 3)) if n > 8 else G.path(n)
    want = (n // 2 + 3 + 1) // 2 + (n - n // 2 - 3) // 2
    r = solver.mvc(g)
    assert r.size == want
    check_cover(g, r.cover, want)


def test_large_n_near_lds_limit(solver, oracle_lib):
    """n = 29,034: the node takes ~113 KB of LDS (one workgroup per CU)."""
    g = G.disjoint_union(G.star(29000), G.petersen(), G.cycle(11), G.complete(12))
    want = 1 + 6 + 6 + 11
    r = solver.mvc(g)
    assert r.size == want
    check_cover(g, r.cover, want)
    p = solver.pvc(g, want - 1)
    assert not p.yes


def invalid_graphs():
    good = G.path(5)
    rp, ci = good.row_ptr.copy(), good.col_idx.copy()
    cases = []
    a = ci.copy(); a[0] = 9          # out of range
    cases.append(("out_of_range", rp.copy(), a, 0))
    a = ci.copy(); a[0] = 0          # self-loop in row 0
    cases.append(("self_loop", rp.copy(), a, 0))
    # asymmetric: drop the reverse entry of edge 3-4 by rewriting row 4 to point at 2
    a = ci.copy(); a[-1] = 2
    cases.append(("asymmetric", rp.copy(), a, 3))
    # unsorted row 1 (entries 0,2 -> 2,0)
    a = ci.copy(); a[1], a[2] = a[2], a[1]
    cases.append(("unsorted", rp.copy(), a, 0))  # row 0's reverse lookup fails first
    # duplicate neighbour: row 2 holds 1,3 -> 1,1
    a = ci.copy(); a[4] = a[3]
    cases.append(("duplicate", rp.copy(), a, 2))
    r = rp.copy(); r[2] = 7          # row_ptr not monotone
    cases.append(("row_ptr", r, ci.copy(), 1))
    return cases


@pytest.mark.parametrize("name,rp,ci,first_row", invalid_graphs(), ids=lambda x: x if isinstance(x, str) else "")
def test_invalid_graph_rejected(solver, name, rp, ci, first_row):
    import paper_2204_10402_amd as vc

    class Raw:
        pass
    g = Raw()
    g.n, g.row_ptr, g.col_idx = 5, rp, ci
    for call in (lambda: solver.mvc(g), lambda: solver.pvc(g, 3)):
        with pytest.raises(vc.VCError) as ei:
            call()
        assert ei.value.code == vc.ERR_INVALID_GRAPH
        assert f"row {first_row} " in str(ei.value)
    # the context still works afterwards
    assert solver.mvc(G.path(5)).size == 2


def first_bad_row(n, rp, ci):
    """The first offending row as include/vc.h defines it: its bounds, and each entry in range,
    not a self-loop, above the one before it, and found in reverse by a binary search of the
    neighbour's row (bisect here). The row pointers here are non-decreasing, so every entry
    belongs to exactly one row."""
    import bisect
    nnz = len(ci)
    for v in range(n):
        b, e = int(rp[v]), int(rp[v + 1])
        if (v == 0 and b != 0) or (v == n - 1 and e != nnz) or b < 0 or e < b or e > nnz:
            return v
        for j in range(b, e):
            u = int(ci[j])
            if u < 0 or u >= n or u == v or (j > b and int(ci[j - 1]) >= u):
                return v
            row = [int(x) for x in ci[rp[u]:rp[u + 1]]]
            at = bisect.bisect_left(row, v)
            if at >= len(row) or row[at] != v:
                return v
    return None


@pytest.mark.parametrize("kind", ["out_of_range", "self_loop", "asymmetric", "unsorted"])
def test_invalid_entry_deep_in_a_large_graph(solver, kind):
    """A defect in one entry of G(600, 0.05) (about 18,000 entries, many validation blocks):
    the reported row is the first offending row by the format's definition."""
    import paper_2204_10402_amd as vc
    g = G.erdos_renyi(600, 0.05, 77)
    rp, ci = g.row_ptr.copy(), g.col_idx.copy()
    v = 411
    j = int(rp[v]) + 1
    if kind == "out_of_range":
        ci[j] = 600
    elif kind == "self_loop":
        ci[j] = v
    elif kind == "asymmetric":
        ci[j] = int(ci[j]) + 1 if int(ci[j]) + 1 < int(ci[j + 1]) else int(ci[j]) - 1
    else:
        ci[j], ci[j + 1] = ci[j + 1], ci[j]
    want = first_bad_row(600, rp, ci)
    assert want is not None

    class Raw:
        pass
    bad = Raw()
    bad.n, bad.row_ptr, bad.col_idx = 600, rp, ci
    with pytest.raises(vc.VCError) as ei:
        solver.mvc(bad, vc.Options(flags=vc.OPT_DEGREE_ARRAYS))
    assert ei.value.code == vc.ERR_INVALID_GRAPH and f"row {want} " in str(ei.value)
    # inside a batch, between two valid graphs: only its own status changes (the valid graph
    # is sparse, G(300, 2/300): its oracle search takes a handful of nodes)
    good = G.erdos_renyi(300, 2.0 / 300, 78)
    r = solver.mvc_batch([good, bad, good])
    assert list(r.status) == [0, vc.ERR_INVALID_GRAPH, 0]
    assert r.size[0] == r.size[2] == solver.mvc(good).size


@pytest.mark.parametrize("n", [257, 320, 384, 448, 511, 512])
@pytest.mark.parametrize("family", ["planted", "er"])
def test_wide_bitsets_match_oracle(solver, oracle_lib, n, family):
    """Bitset nodes of 5 to 8 words (257 <= n <= 512, on request): the
    oracle's answers; one workgroup visits the oracle's tree node for node; PVC-no visits it
    with the full grid too; the default family gives the same answers."""
    if family == "planted":
        g = G.planted_cover(n, int(0.3 * n), 4 * n, 0.75, 900 + n)
    else:
        g = G.erdos_renyi(n, 3.0 / n, 900 + n)
    bits = KERNELS["bitsets"]
    o = oracle.mvc(g, node_cap=200000)
    r = solver.mvc(g, opts(flags=bits))
    assert r.stats["bitset_words"] == (n + 63) // 64
    assert r.size == o.size
    check_cover(g, r.cover, o.size)
    one = solver.mvc(g, single_wg(bits))
    assert one.size == o.size and one.stats["nodes"] == o.nodes
    k = o.size - 1
    want = oracle.pvc(g, k, node_cap=200000)
    p = solver.pvc(g, k, opts(flags=bits))
    assert not p.yes and p.stats["nodes"] == want.nodes
    yes = solver.pvc(g, o.size, opts(flags=bits))
    assert yes.yes and yes.size <= o.size
    check_cover(g, yes.cover, yes.size)
    auto = solver.mvc(g)
    assert auto.size == o.size and auto.stats["bitset_words"] == 0


@pytest.mark.parametrize("flags", [0, 0x40])
def test_batch_across_all_bitset_widths(solver, oracle_lib, flags):
    """One batch over 1 to 8 bitset words (by default: 1 to 4 words and degree arrays above
    256 vertices): PVC-no node counts per graph equal the oracle's."""
    import paper_2204_10402_amd as vc
    sizes = [40, 100, 150, 230, 300, 350, 430, 500] + ([600] if flags == 0 else [])
    gs = [G.erdos_renyi(n, 3.0 / n, 1700 + n) for n in sizes]
    taus = [oracle.mvc(g, node_cap=200000).size for g in gs]
    ks = [t - 1 for t in taus]
    r = solver.pvc_batch(gs, ks, vc.Options(flags=flags))
    assert list(r.status) == [0] * len(gs) and not r.yes.any()
    for g, k, nodes in zip(gs, ks, r.nodes):
        assert nodes == oracle.pvc(g, k, node_cap=200000).nodes
    m = solver.mvc_batch(gs, vc.Options(flags=flags))
    assert list(m.size) == taus


def test_node_budget(solver, oracle_lib):
    import paper_2204_10402_amd as vc
    g = G.random_regular(120, 5, 0)
    with pytest.raises(vc.VCError) as ei:
        solver.mvc(g, vc.Options(node_budget=20000))
    assert ei.value.code == vc.ERR_BUDGET
    assert solver.mvc(G.cycle(9)).size == 5


def test_bad_options(solver):
    import paper_2204_10402_amd as vc
    for o in (vc.Options(wg_size=100), vc.Options(num_wg=-1), vc.Options(flags=0x1000),
              vc.Options(wl_threshold=-2), vc.Options(flags=0x60), vc.Options(wg_size=128)):
        with pytest.raises(vc.VCError) as ei:
            solver.mvc(G.path(4), o)
        assert ei.value.code == vc.ERR_INVALID_ARG
    with pytest.raises(vc.VCError) as ei:
        solver.mvc(G.path(600), vc.Options(flags=vc.OPT_BITSETS))
    assert ei.value.code == vc.ERR_INVALID_ARG


@pytest.mark.parametrize("knobs", [dict(wl_capacity=1), dict(wl_capacity=1, wl_threshold=1),
                                   dict(num_wg=3), dict(num_wg=7, wl_threshold=1),
                                   dict(wg_size=128, flags=0x20), dict(wg_size=256, num_wg=64, flags=0x20),
                                   dict(wg_size=1024, flags=0x20), dict(num_wg=5, flags=0x20),
                                   dict(wl_capacity=1, flags=0x20)])
def test_launch_knobs_keep_answers(solver, oracle_lib, knobs):
    import paper_2204_10402_amd as vc
    g = G.erdos_renyi(90, 0.1, 5)
    o = oracle.mvc(g)
    r = solver.mvc(g, vc.Options(**knobs))
    assert r.size == o.size
    check_cover(g, r.cover, o.size)
    pn = solver.pvc(g, o.size - 1, vc.Options(**knobs))
    assert not pn.yes and pn.stats["nodes"] == oracle.pvc(g, o.size - 1).nodes


def test_device_entry_matches_host_entry(solver, oracle_lib, torch_cuda):
    torch = torch_cuda
    g = G.erdos_renyi(100, 0.08, 11)
    o = oracle.mvc(g)
    rp = torch.from_numpy(g.row_ptr).cuda()
    ci = torch.from_numpy(g.col_idx).cuda()
    cov = torch.zeros(g.n, dtype=torch.uint8, device="cuda")
    r = solver.mvc_device(rp, ci, cov)
    assert r.size == o.size
    check_cover(g, cov.cpu().numpy(), o.size)


def test_context_reuse_across_sizes(solver, oracle_lib):
    for g in (G.erdos_renyi(200, 0.02, 1), G.path(7), G.erdos_renyi(1500, 0.0015, 2),
              G.complete(12), G.erdos_renyi(70, 0.1, 3), G.planted_cover(3000, 300, 6000, 0.75, 5),
              G.erdos_renyi(120, 0.05, 4)):
        o = oracle.mvc(g)
        r = solver.mvc(g)
        assert r.size == o.size
        check_cover(g, r.cover, o.size)


def test_profiled_kernel_same_answers(solver, oracle_lib):
    import paper_2204_10402_amd as vc
    g = G.erdos_renyi(80, 0.1, 21)
    o = oracle.mvc(g)
    r = solver.mvc(g, vc.Options(flags=vc.OPT_PROFILE))
    assert r.size == o.size
    check_cover(g, r.cover, o.size)
    cyc = r.stats["cycles"]
    assert cyc["total"] > 0 and cyc["reduce"] > 0
    main = ("acquire", "reduce", "branch", "donate", "other")
    assert sum(cyc[k] for k in main) <= cyc["total"]
    one = solver.mvc(g, vc.Options(num_wg=1, wl_threshold=-1, flags=vc.OPT_PROFILE))
    assert one.stats["nodes"] == o.nodes
    arr = solver.mvc(g, vc.Options(num_wg=1, wl_threshold=-1, flags=vc.OPT_PROFILE | 0x20))
    assert arr.stats["nodes"] == o.nodes and arr.stats["cycles"]["reduce"] > 0
    plain = solver.mvc(g)
    assert all(v == 0 for v in plain.stats["cycles"].values())


# ---- StackOnly ablation (the comparison method of §V-A) ------------------------------------

@pytest.mark.parametrize("kernel", sorted(KERNELS))
@pytest.mark.parametrize("depth", [1, 4, 8, 12])
def test_stack_only_answers(solver, oracle_lib, kernel, depth):
    """Static sub-tree partition at a start depth: same answers as the oracle; a PVC-no tree is
    counted node for node (nodes above the start depth count once, on their owning path)."""
    import paper_2204_10402_amd as vc
    for seed in range(3):
        g = G.erdos_renyi(40 + 10 * seed, 0.12, 900 + seed)
        o = oracle.mvc(g)
        opt = vc.Options(flags=vc.OPT_STACK_ONLY | KERNELS[kernel], start_depth=depth)
        r = solver.mvc(g, opt)
        assert r.size == o.size
        check_cover(g, r.cover, o.size)
        loads = solver.wg_loads()
        assert loads.size == r.stats["num_wg"] and loads.sum() >= 1
        for k in (o.size - 1, o.size):
            want = oracle.pvc(g, k)
            p = solver.pvc(g, k, opt)
            assert p.yes == want.yes
            if not want.yes:
                assert p.stats["nodes"] == want.nodes
            else:
                check_cover(g, p.cover, p.size)


def test_stack_only_larger_tree_and_limits(solver, oracle_lib):
    """G(100, 0.1), seed 1: a 30,000-node tree (oracle); StackOnly at depths 8 and 16."""
    import paper_2204_10402_amd as vc
    g = G.erdos_renyi(100, 0.1, 1)
    o = oracle.mvc(g)
    for depth in (8, 16):
        r = solver.mvc(g, vc.Options(flags=vc.OPT_STACK_ONLY, start_depth=depth))
        assert r.size == o.size
        check_cover(g, r.cover, o.size)
        p = solver.pvc(g, o.size - 1, vc.Options(flags=vc.OPT_STACK_ONLY, start_depth=depth))
        assert not p.yes and p.stats["nodes"] == oracle.pvc(g, o.size - 1).nodes
    with pytest.raises(vc.VCError) as ei:
        solver.mvc_batch([G.path(5), G.path(6)], vc.Options(flags=vc.OPT_STACK_ONLY))
    assert ei.value.code == vc.ERR_INVALID_ARG
    for bad in (vc.Options(flags=vc.OPT_STACK_ONLY, start_depth=25), vc.Options(start_depth=4)):
        with pytest.raises(vc.VCError) as ei:
            solver.mvc(G.path(5), bad)
        assert ei.value.code == vc.ERR_INVALID_ARG


def test_graph_beyond_lds(solver, oracle_lib):
    """n = 50,040 (a degree array of 200 KB: more than a CU's LDS), so the node lives in device
    memory: 20 stars of 2,500 leaves and 2 Petersen graphs; tau = 20 + 2 * 6 = 32 (textbook
    values of the components); the PVC-no tree is the oracle's node for node."""
    import paper_2204_10402_amd as vc
    g = G.disjoint_union(*([G.star(2500)] * 20 + [G.petersen()] * 2))
    assert g.n == 50040
    r = solver.mvc(g)
    assert r.size == 32
    check_cover(g, r.cover, 32)
    assert r.stats["bitset_words"] == 0
    p = solver.pvc(g, 31)
    assert not p.yes and p.stats["nodes"] == oracle.pvc(g, 31, node_cap=100000).nodes
    q = solver.pvc(g, 32)
    assert q.yes and q.size <= 32
    check_cover(g, q.cover, q.size)
    with pytest.raises(vc.VCError) as ei:
        solver.mvc(g, vc.Options(flags=vc.OPT_GLOBAL_NODES | vc.OPT_BITSETS))
    assert ei.value.code == vc.ERR_INVALID_ARG
