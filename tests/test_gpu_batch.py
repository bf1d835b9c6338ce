"""Batched search (vc_mvc_batch / vc_pvc_batch and their device forms) against the CPU
oracle, one graph at a time.

The bar is the single-graph bar, per graph: MVC size and PVC decision identical to the
oracle's; every cover checked edge by edge here; node counts identical where the tree does not
depend on the schedule (one workgroup that never donates; PVC graphs whose answer is no, in any
launch configuration). A graph's answer must not depend on the graphs it is batched with.
"""

import numpy as np
import pytest

import graphs as G
import oracle

pytestmark = pytest.mark.gpu

KERNELS = {"auto": 0, "bitsets": 0x40, "degree_arrays": 0x20}


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
    assert set(np.unique(cover).tolist()) <= {0, 1}
    assert oracle.is_cover(g, cover)
    assert int(cover.sum()) == size


def mixed_graphs(seed, count=24, n_hi=300):
    """Small random graphs of 1..4 bitset words and degree arrays (the batch tests also run
    them all on the degree-array kernels by flag)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.integers(5, n_hi + 1))
        p = float(rng.uniform(1.5, 5.0)) / n
        out.append(G.erdos_renyi(n, p, 1000 * seed + i))
    return out


@pytest.mark.parametrize("kernel", ["auto", "degree_arrays"])
@pytest.mark.parametrize("seed", range(4))
def test_mvc_batch_matches_oracle(solver, oracle_lib, seed, kernel):
    import paper_2204_10402_amd as vc
    gs = mixed_graphs(seed)
    res = solver.mvc_batch(gs, vc.Options(flags=KERNELS[kernel]))
    for i, g in enumerate(gs):
        o = oracle.mvc(g)
        assert res.status[i] == 0
        assert res.size[i] == o.size, i
        check_cover(g, res.cover_of(i), o.size)
    assert res.stats["nodes"] == int(res.nodes.sum())


@pytest.mark.parametrize("kernel", ["bitsets", "degree_arrays"])
def test_mvc_batch_single_workgroup_node_parity(solver, oracle_lib, kernel):
    """One workgroup that never donates walks the graphs one after another, each in the
    oracle's order: per-graph node counts equal the oracle's."""
    import paper_2204_10402_amd as vc
    gs = [G.erdos_renyi(20 + 9 * i, 0.12, 500 + i) for i in range(10)]
    res = solver.mvc_batch(gs, vc.Options(num_wg=1, wl_threshold=-1, flags=KERNELS[kernel]))
    for i, g in enumerate(gs):
        o = oracle.mvc(g)
        assert (res.size[i], res.nodes[i]) == (o.size, o.nodes), i
        check_cover(g, res.cover_of(i), o.size)


@pytest.mark.parametrize("kernel", ["auto", "degree_arrays"])
@pytest.mark.parametrize("seed", range(3))
def test_pvc_batch_decisions_and_no_node_counts(solver, oracle_lib, seed, kernel):
    import paper_2204_10402_amd as vc
    gs = mixed_graphs(100 + seed, count=20, n_hi=200)
    taus = [oracle.mvc(g).size for g in gs]
    ks = [max(t - (i % 3), 0) for i, t in enumerate(taus)]  # tau, tau-1, tau-2 in turn
    res = solver.pvc_batch(gs, ks, vc.Options(flags=KERNELS[kernel]))
    for i, g in enumerate(gs):
        want = ks[i] >= taus[i]
        assert res.status[i] == 0
        assert bool(res.yes[i]) == want, i
        if want:
            assert 0 <= res.size[i] <= ks[i]
            check_cover(g, res.cover_of(i), int(res.size[i]))
        else:
            # a no-instance's tree is searched whole, whatever the schedule
            assert res.size[i] == -1 and int(res.cover_of(i).sum()) == 0
            assert res.nodes[i] == oracle.pvc(g, ks[i]).nodes, i


def test_planted_batch_full_size(solver, oracle_lib):
    """4,096 planted-cover PVC instances (n uniform in [40, 400], average degree in [3, 12],
    |C| = 0.3n, k = |C| for even i and |C| - 1 for odd i) in one call: every decision equals
    the oracle's; no-instances visit exactly the oracle's nodes."""
    import paper_2204_10402_amd as vc
    batch = G.planted_batch(4096, 0)
    gs = [g for g, _ in batch]
    ks = [k for _, k in batch]
    res = solver.pvc_batch(gs, ks)
    assert (res.status == 0).all()
    # the instances above 256 vertices on the degree-array kernels too
    wide = [i for i, g in enumerate(gs) if g.n > 256]
    arr = solver.pvc_batch([gs[i] for i in wide], [ks[i] for i in wide],
                           vc.Options(flags=vc.OPT_DEGREE_ARRAYS))
    assert (arr.status == 0).all()
    assert [bool(x) for x in arr.yes] == [bool(res.yes[i]) for i in wide]
    for i, (g, k) in enumerate(batch):
        o = oracle.pvc(g, k)
        assert bool(res.yes[i]) == o.yes, i
        if o.yes:
            assert res.size[i] <= k
            check_cover(g, res.cover_of(i), int(res.size[i]))
        else:
            assert res.nodes[i] == o.nodes, i
    assert res.yes[0::2].all()  # k = |C| always has the planted cover


def test_batch_answers_do_not_depend_on_the_mix(solver, oracle_lib):
    import paper_2204_10402_amd as vc
    gs = mixed_graphs(7, count=12)
    alone = [solver.mvc(g) for g in gs]
    mixed = solver.mvc_batch(gs)
    rev = solver.mvc_batch(gs[::-1])
    for i, g in enumerate(gs):
        assert mixed.size[i] == alone[i].size == rev.size[len(gs) - 1 - i]
    ks = [max(r.size - 1, 0) for r in alone]
    pv = solver.pvc_batch(gs, ks, vc.Options(num_wg=17))
    for i, g in enumerate(gs):
        assert bool(pv.yes[i]) == (alone[i].size == 0)
        if not pv.yes[i]:
            assert pv.nodes[i] == solver.pvc(g, ks[i]).stats["nodes"]


def test_batch_with_rejected_empty_and_edgeless_graphs(solver, oracle_lib):
    import paper_2204_10402_amd as vc

    class Raw:
        pass
    bad = Raw()
    good = G.path(5)
    bad.n, bad.row_ptr = 5, good.row_ptr.copy()
    bad.col_idx = good.col_idx.copy()
    bad.col_idx[0] = 9  # out of range
    empty = G.empty(0)
    edgeless = G.empty(7)
    gs = [G.cycle(9), bad, empty, edgeless, G.complete(6), bad, G.erdos_renyi(150, 0.03, 3)]
    res = solver.mvc_batch(gs)
    want_status = [0, vc.ERR_INVALID_GRAPH, 0, 0, 0, vc.ERR_INVALID_GRAPH, 0]
    assert res.status.tolist() == want_status
    assert res.size[0] == 5 and res.size[2] == 0 and res.size[3] == 0 and res.size[4] == 5
    assert res.size[6] == oracle.mvc(gs[6]).size
    assert res.size[1] == -1 and int(res.cover_of(1).sum()) == 0
    for i in (0, 3, 4, 6):
        check_cover(gs[i], res.cover_of(i), int(res.size[i]))
    p = solver.pvc_batch(gs, [5, 3, 0, 0, 4, 3, 0])
    assert p.status.tolist() == want_status
    assert p.yes.tolist() == [True, False, True, True, False, False, False]


def test_batch_budget_is_per_graph(solver, oracle_lib):
    import paper_2204_10402_amd as vc
    hard = G.random_regular(120, 5, 0)
    easy = [G.cycle(11), G.erdos_renyi(80, 0.05, 1), G.path(30)]
    res = solver.mvc_batch([easy[0], hard, easy[1], easy[2]], vc.Options(node_budget=20000))
    assert res.status.tolist() == [0, vc.ERR_BUDGET, 0, 0]
    assert res.size[0] == 6 and res.size[3] == 15
    assert res.size[2] == oracle.mvc(easy[1]).size
    assert int(res.cover_of(1).sum()) == 0


def test_batch_device_form(solver, oracle_lib, torch_cuda):
    import paper_2204_10402_amd as vc
    torch = torch_cuda
    gs = mixed_graphs(9, count=16)
    n, nnz, rp, ci = vc.pack_batch(gs)
    rp_d = torch.from_numpy(rp).cuda()
    ci_d = torch.from_numpy(ci).cuda()
    cov = torch.zeros(int(n.sum()), dtype=torch.uint8, device="cuda")
    res = solver.mvc_batch_device(n, nnz, rp_d, ci_d, cov)
    host = solver.mvc_batch(gs)
    assert res.size.tolist() == host.size.tolist()
    c = cov.cpu().numpy()
    for i, g in enumerate(gs):
        check_cover(g, c[res.offsets[i]:res.offsets[i + 1]], int(res.size[i]))
    ks = np.maximum(res.size - 1, 0).tolist()
    pres = solver.pvc_batch_device(n, nnz, rp_d, ci_d, ks, cov)
    assert pres.yes.tolist() == (res.size == 0).tolist()
    assert int(cov.sum().item()) == 0


def test_empty_batch_and_bad_arguments(solver):
    import paper_2204_10402_amd as vc
    res = solver.mvc_batch([])
    assert res.status.size == 0
    with pytest.raises(vc.VCError) as ei:
        solver.pvc_batch([G.path(4)], [-1])
    assert ei.value.code == vc.ERR_INVALID_ARG
    with pytest.raises(vc.VCError) as ei:
        solver.mvc_batch([G.path(600)], vc.Options(flags=vc.OPT_BITSETS))
    assert ei.value.code == vc.ERR_INVALID_ARG


def test_autotuned_batches_keep_answers(torch_cuda, oracle_lib):
    """With VC_OPT_AUTOTUNE the first call times trial launches and later calls reuse the
    choice; answers and PVC-no node counts stay the oracle's either way."""
    import paper_2204_10402_amd as vc
    s = vc.Solver(0)  # a fresh context: nothing tuned yet
    try:
        gs = mixed_graphs(11, count=20)
        o = vc.Options(flags=vc.OPT_AUTOTUNE)
        first = s.mvc_batch(gs, o)
        second = s.mvc_batch(gs, o)
        for i, g in enumerate(gs):
            want = oracle.mvc(g).size
            assert first.size[i] == second.size[i] == want, i
            check_cover(g, second.cover_of(i), want)
        ks = [max(int(x) - 1, 0) for x in first.size]
        p = s.pvc_batch(gs, ks, o)
        for i, g in enumerate(gs):
            if not p.yes[i]:
                assert p.nodes[i] == oracle.pvc(g, ks[i]).nodes
        # explicit knobs switch the tuner off
        fixed = s.mvc_batch(gs, vc.Options(flags=vc.OPT_AUTOTUNE, num_wg=5))
        assert fixed.stats["num_wg"] <= 5 and fixed.size.tolist() == first.size.tolist()
    finally:
        s.close()
