"""Caller-owned workspace forms (vc_*_device_ws), the host abort (vc_abort), the time limit
(vc_options.timeout_ms) and the stack-depth guard (vc_options.stack_depth), on the GPU.

The bar is the oracle's: MVC size and PVC decision exact, covers verified edge by edge, PVC-no
node counts equal; a stopped call returns ERR_BUDGET (abort, time limit) or ERR_INTERNAL (a
stack deeper than promised), every kernel of it has returned, and the context solves the next
graph correctly.
"""

import threading
import time

import numpy as np
import pytest

import graphs as G
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


@pytest.fixture(scope="module")
def solver(torch_cuda):
    import paper_2204_10402_amd as vc
    s = vc.Solver(0, stream=torch_cuda.cuda.current_stream(0))
    yield s
    s.close()


def dev(torch, g):
    return (torch.from_numpy(g.row_ptr).to("cuda:0"), torch.from_numpy(g.col_idx).to("cuda:0"),
            torch.zeros(max(g.n, 1), dtype=torch.uint8, device="cuda:0"))


def check_cover(g, cover, size):
    c = cover.cpu().numpy()[:g.n]
    assert oracle.is_cover(g, c) and int(c.sum()) == size


def workspace(torch, nbytes):
    return torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")


GRAPHS = [("er60", lambda: G.erdos_renyi(60, 0.10, 0)),
          ("reg120", lambda: G.random_regular(120, 5, 1)),
          ("er300", lambda: G.erdos_renyi(300, 3.5 / 300, 4)),
          ("star", lambda: G.star(40)),
          ("edgeless", lambda: G.empty(9))]


@pytest.mark.parametrize("name,make", GRAPHS)
def test_workspace_forms_match_oracle(solver, oracle_lib, torch_cuda, name, make):
    import paper_2204_10402_amd as vc
    g = make()
    rp, ci, cover = dev(torch_cuda, g)
    need = solver.workspace_bytes(g.n, g.nnz)
    assert need > 0
    ws = workspace(torch_cuda, need)
    want = oracle.mvc(g)
    r = solver.mvc_device_ws(rp, ci, ws, cover)
    assert r.size == want.size
    check_cover(g, cover, r.size)
    for k in (want.size, max(want.size - 1, 0)):
        o = oracle.pvc(g, k)
        cover.zero_()
        p = solver.pvc_device_ws(rp, ci, k, ws, cover)
        assert p.yes == o.yes, k
        if o.yes:
            check_cover(g, cover, p.size)
            assert p.size <= k
        else:
            assert p.stats["nodes"] == o.nodes and int(cover.sum()) == 0
    # the workspace holds nothing the context keeps: its own buffers serve the next call
    assert solver.wg_loads().size == 0
    assert solver.mvc(g).size == want.size


def test_workspace_degree_arrays_planted(solver, oracle_lib, torch_cuda):
    """A planted-cover graph of 5,000 vertices on the degree-array kernels, k = 400 and 399,
    with the stack depth and grid the workspace was sized for."""
    import paper_2204_10402_amd as vc
    g = G.planted_cover(5000, 400, 40000, 0.75, 1)
    rp, ci, cover = dev(torch_cuda, g)
    o = vc.Options(num_wg=64)
    ws = workspace(torch_cuda, solver.workspace_bytes(g.n, g.nnz, depth=401, options=o))
    for k, want_yes in ((400, True), (399, False)):
        cover.zero_()
        r = solver.pvc_device_ws(rp, ci, k, ws, cover, options=o)
        assert r.yes == want_yes
        if r.yes:
            check_cover(g, cover, r.size)


def test_batch_workspace_forms(solver, oracle_lib, torch_cuda):
    """A batch of both kernel families (bitset words 1-4 and degree arrays), run one launch
    after another in the workspace."""
    import paper_2204_10402_amd as vc
    rng = np.random.default_rng(5)
    gs = [G.erdos_renyi(int(n), float(rng.uniform(1.5, 4.0)) / int(n), 50 + i)
          for i, n in enumerate(rng.integers(5, 320, size=20))]
    n, nnz, rp, ci = vc.pack_batch(gs)
    rp_d = torch_cuda.from_numpy(rp).to("cuda:0")
    ci_d = torch_cuda.from_numpy(ci).to("cuda:0")
    cover = torch_cuda.zeros(int(n.sum()), dtype=torch_cuda.uint8, device="cuda:0")
    ws = workspace(torch_cuda, solver.batch_workspace_bytes(n, nnz))
    res = solver.mvc_batch_device_ws(n, nnz, rp_d, ci_d, ws, cover)
    taus = [oracle.mvc(g).size for g in gs]
    host = cover.cpu().numpy()
    for i, g in enumerate(gs):
        assert res.status[i] == 0 and res.size[i] == taus[i], i
        c = host[res.offsets[i]:res.offsets[i + 1]]
        assert oracle.is_cover(g, c) and int(c.sum()) == taus[i], i
    ks = [max(t - (i % 2), 0) for i, t in enumerate(taus)]
    res = solver.pvc_batch_device_ws(n, nnz, rp_d, ci_d, ks, ws, cover)
    for i, g in enumerate(gs):
        o = oracle.pvc(g, ks[i])
        assert res.status[i] == 0 and bool(res.yes[i]) == o.yes, i
        if not o.yes:
            assert res.nodes[i] == o.nodes, i


def test_workspace_too_small_and_smaller_grid(solver, oracle_lib, torch_cuda):
    import paper_2204_10402_amd as vc
    g = G.random_regular(120, 5, 2)
    rp, ci, cover = dev(torch_cuda, g)
    with pytest.raises(vc.VCError) as e:
        solver.mvc_device_ws(rp, ci, workspace(torch_cuda, 4096), cover)
    assert e.value.code == vc.ERR_NO_MEMORY
    # a quarter of the full need: the grid shrinks until the stacks fit; same answer
    need = solver.workspace_bytes(g.n, g.nnz)
    full = solver.mvc_device_ws(rp, ci, workspace(torch_cuda, need), cover)
    small = solver.mvc_device_ws(rp, ci, workspace(torch_cuda, need // 4 // 256 * 256), cover)
    assert small.size == full.size == oracle.mvc(g).size
    assert small.stats["num_wg"] < full.stats["num_wg"]


def hard_batch(torch, count):
    """`count` G(150, 0.08) graphs: MVC searches of millions of nodes each."""
    import paper_2204_10402_amd as vc
    gs = [G.erdos_renyi(150, 0.08, s) for s in range(count)]
    n, nnz, rp, ci = vc.pack_batch(gs)
    return gs, n, nnz, torch.from_numpy(rp).to("cuda:0"), torch.from_numpy(ci).to("cuda:0")


def test_time_limit_stops_the_call(solver, oracle_lib, torch_cuda):
    import paper_2204_10402_amd as vc
    gs, n, nnz, rp, ci = hard_batch(torch_cuda, 16)
    t = time.perf_counter()
    with pytest.raises(vc.VCError) as e:
        solver.mvc_batch_device(n, nnz, rp, ci, options=vc.Options(timeout_ms=5))
    assert e.value.code == vc.ERR_BUDGET and "time limit" in str(e.value)
    assert time.perf_counter() - t < 2.0
    small = G.erdos_renyi(60, 0.1, 0)
    assert solver.mvc(small).size == oracle.mvc(small).size


def test_host_abort_stops_the_call(solver, oracle_lib, torch_cuda):
    """vc_abort from another thread while a long batch runs: the call returns ERR_BUDGET long
    before the search could end. A 30 s time limit bounds the call if the abort were lost."""
    import paper_2204_10402_amd as vc
    gs, n, nnz, rp, ci = hard_batch(torch_cuda, 64)
    out = {}

    def run():
        t = time.perf_counter()
        try:
            solver.mvc_batch_device(n, nnz, rp, ci, options=vc.Options(timeout_ms=30000))
            out["rc"] = 0
        except vc.VCError as e:
            out["rc"], out["msg"] = e.code, str(e)
        out["s"] = time.perf_counter() - t

    th = threading.Thread(target=run)
    th.start()
    time.sleep(0.05)
    solver.abort()
    th.join(60)
    assert not th.is_alive()
    assert out["rc"] == vc.ERR_BUDGET and "vc_abort" in out["msg"], out
    assert out["s"] < 5.0, out
    small = G.erdos_renyi(60, 0.1, 0)
    assert solver.mvc(small).size == oracle.mvc(small).size


def test_abort_between_calls_is_ignored(solver, oracle_lib):
    g = G.erdos_renyi(60, 0.1, 0)
    solver.abort()
    assert solver.mvc(g).size == oracle.mvc(g).size


@pytest.mark.parametrize("flags", [0x40, 0x20], ids=["bitsets", "degree_arrays"])
def test_stack_deeper_than_promised_is_an_internal_error(solver, oracle_lib, flags):
    """stack_depth = 2 with one workgroup that never donates: the first push past two entries
    stops the launch (no entry is written past the ring) and the call reports the overflow."""
    import paper_2204_10402_amd as vc
    g = G.random_regular(120, 5, 0)
    o = vc.Options(num_wg=1, wl_threshold=-1, flags=flags, stack_depth=2)
    with pytest.raises(vc.VCError) as e:
        solver.mvc(g, o)
    assert e.value.code == vc.ERR_INTERNAL and "stack overflow" in str(e.value)
    assert solver.mvc(g, vc.Options(flags=flags)).size == oracle.mvc(g).size
