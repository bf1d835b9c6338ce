"""vc_pvc_device_noalloc (the entry point that allocates nothing) against vc_pvc_device, the
entry point it is a variant of: the same decision, a verified cover of size <= k on yes, the
same node count on no (the tree does not depend on the schedule), on two calls in a row, the
second on a smaller graph (the library's scratch keeps the first call's contents)."""

import json
import os

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


def same_as_pvc_device(solver, torch, g, k, want=None):
    """`want` = (decision, node count) from the stored oracle answers, else the oracle runs."""
    rp, ci, cover = dev(torch, g)
    cover_ref = torch.zeros_like(cover)
    a = solver.pvc_device_noalloc(rp, ci, k, cover)
    b = solver.pvc_device(rp, ci, k, cover_ref)
    if want is None:
        o = oracle.pvc(g, k)
        want = (o.yes, o.nodes)
    assert a.yes == b.yes == want[0], (g.n, k)
    if a.yes:
        c = cover.cpu().numpy()[:g.n]
        assert oracle.is_cover(g, c) and int(c.sum()) == a.size and a.size <= k
    else:
        assert a.stats["nodes"] == b.stats["nodes"] == want[1]
        assert int(cover.sum()) == 0
    return a


def stored_hard_answer(seed):
    """tau - 1 and the oracle's PVC node count for G(150, 0.08) of `seed`, from
    tests/golden/oracle_answers.json (the oracle's exhaustive search takes tens of seconds)."""
    with open(os.path.join(os.path.dirname(__file__), "golden", "oracle_answers.json")) as f:
        rows = json.load(f)["results"]
    r = next(r for r in rows if r["workload"] == "pvc_er150" and r["seed"] == seed)
    return r["k"], (r["yes"], r["nodes"])


@pytest.mark.parametrize("order", ["large_then_small", "small_twice"])
def test_two_calls_match_pvc_device(solver, oracle_lib, torch_cuda, order):
    big = G.erdos_renyi(150, 0.08, 3)          # bitset kernels, a search of millions of nodes
    small = G.planted_cover(90, 27, 250, 0.75, 4)
    tau_small = oracle.mvc(small).size
    if order == "large_then_small":
        k, want = stored_hard_answer(3)
        same_as_pvc_device(solver, torch_cuda, big, k, want)     # no: the whole tree
    else:
        same_as_pvc_device(solver, torch_cuda, small, tau_small - 1)
    same_as_pvc_device(solver, torch_cuda, small, tau_small)      # yes, smaller input
    same_as_pvc_device(solver, torch_cuda, small, tau_small - 1)


def test_degree_array_graph_fits_by_shrinking(solver, oracle_lib, torch_cuda):
    """A 1,000-vertex planted graph (degree-array kernels): the plan shrinks into the scratch
    and the answers match vc_pvc_device."""
    g = G.planted_cover(1000, 200, 4000, 0.75, 2)
    same_as_pvc_device(solver, torch_cuda, g, 200)
    same_as_pvc_device(solver, torch_cuda, g, 199)


def test_graph_beyond_the_scratch_is_rejected(solver, torch_cuda):
    """50,040 vertices and k = 300: one workgroup's stack of k + 1 degree arrays (200 KB each)
    and the smallest worklist ring do not fit in 64 MiB: a clear error before any launch, and
    the context keeps working."""
    import paper_2204_10402_amd as vc
    stars = [G.star(2500) for _ in range(20)]
    g = G.disjoint_union(*stars, G.petersen(), G.petersen())
    rp, ci, cover = dev(torch_cuda, g)
    with pytest.raises(vc.VCError) as e:
        solver.pvc_device_noalloc(rp, ci, 300, cover)
    assert e.value.code == vc.ERR_NO_MEMORY and "no-allocation" in str(e.value)
    small = G.erdos_renyi(60, 0.1, 0)
    rp, ci, cover = dev(torch_cuda, small)
    assert solver.pvc_device_noalloc(rp, ci, 40, cover).yes
