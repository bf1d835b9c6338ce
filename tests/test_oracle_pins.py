"""Pins of the CPU oracle to facts fixed by the paper and by mathematics, not by the oracle.

- brute force: the minimum cover by its definition (paper §II-A), every subset tried;
- closed forms of textbook graph families;
- König's theorem on bipartite graphs (tau = maximum matching, scipy's matcher);
- planted covers (a known cover bounds tau from above; a matching saturating it, from below);
- MVC/PVC consistency: PVC(tau) = yes and PVC(tau - 1) = no (paper §II-A);
- soundness of the reduction rules (paper §II-B): tau(G) = s + tau(reduced graph);
- ablation: switching off any rule or the edge-count prune leaves tau unchanged;
- hand-derived traces in tests/golden/hand_traces.json.
Each of these fails on a plausible slip in the oracle: a dropped rule condition, a wrong
tie-break, an off-by-one in r, a wrong prune, a wrong child.
"""

import json
import os

import numpy as np
import pytest
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import maximum_bipartite_matching

import graphs as G
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def residual(g, deg):
    """The graph left by a degree array: live vertices only, induced edges."""
    live = np.asarray(deg) >= 0
    u, v = G.edges_of(g)
    keep = live[u] & live[v]
    return G.from_edges(g.n, u[keep], v[keep])


def matching_size(a, b, u, v):
    """Maximum matching of a bipartite graph with parts [0,a) and [0,b), edges (u[i], v[i])."""
    if len(u) == 0:
        return 0
    m = csr_matrix((np.ones(len(u)), (u, v)), shape=(a, b))
    match = maximum_bipartite_matching(m, perm_type="column")
    return int(np.sum(match >= 0))


# ---- brute force --------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(240))
def test_mvc_equals_definition(oracle_lib, seed):
    n = 4 + seed % 13
    g = G.random_small(n, seed) if seed % 2 else G.erdos_renyi(n, 0.15 + 0.05 * (seed % 9), seed)
    tau, _ = oracle.tau_by_definition(g)
    r = oracle.mvc(g)
    assert r.size == tau
    assert oracle.is_cover(g, r.cover) and int(r.cover.sum()) == tau
    assert r.greedy >= tau
    gr, gc = oracle.greedy(g)
    assert gr == r.greedy and oracle.is_cover(g, gc) and int(gc.sum()) == gr


@pytest.mark.parametrize("seed", range(60))
def test_pvc_every_k_matches_definition(oracle_lib, seed):
    n = 5 + seed % 11
    g = G.random_small(n, 1000 + seed)
    tau, _ = oracle.tau_by_definition(g)
    for k in range(0, n + 2):
        r = oracle.pvc(g, k)
        assert r.yes == (k >= tau), (k, tau)
        if r.yes:
            assert oracle.is_cover(g, r.cover) and r.size == int(r.cover.sum()) <= k
        else:
            assert r.size == -1 and int(r.cover.sum()) == 0


# ---- closed forms -------------------------------------------------------------------

def closed_form_cases():
    # Textbook minimum vertex cover sizes.
    cases = []
    for n in range(1, 13):
        cases.append((f"K{n}", G.complete(n), n - 1))          # all but one vertex
    for n in range(3, 26):
        cases.append((f"C{n}", G.cycle(n), (n + 1) // 2))      # ceil(n/2)
    for n in range(1, 26):
        cases.append((f"P{n}", G.path(n), n // 2))             # floor(n/2)
    for a in range(1, 7):
        for b in range(1, 7):
            cases.append((f"K{a},{b}", G.complete_bipartite(a, b), min(a, b)))
    for leaves in range(0, 12):
        cases.append((f"star{leaves}", G.star(leaves), 1 if leaves else 0))
    for n in (0, 1, 7):
        cases.append((f"empty{n}", G.empty(n), 0))
    for parts in ([1, 1, 1], [2, 3], [2, 2, 2], [1, 2, 3, 4], [3, 3, 3]):
        cases.append((f"multi{parts}", G.complete_multipartite(parts), sum(parts) - max(parts)))
    for d in range(0, 5):
        cases.append((f"Q{d}", G.hypercube(d), (1 << d) // 2))  # bipartite, perfect matching
    for a, b in ((1, 5), (2, 3), (3, 3), (3, 4), (4, 4)):
        cases.append((f"grid{a}x{b}", G.grid(a, b), (a * b) // 2))
    cases.append(("petersen", G.petersen(), 6))
    return cases


@pytest.mark.parametrize("name,g,tau", closed_form_cases(), ids=lambda x: x if isinstance(x, str) else "")
def test_closed_forms(oracle_lib, name, g, tau):
    if g.n <= 20:
        assert oracle.tau_by_definition(g)[0] == tau
    r = oracle.mvc(g)
    assert r.size == tau
    assert oracle.is_cover(g, r.cover) and int(r.cover.sum()) == tau


@pytest.mark.parametrize("name,g,tau", [
    ("K40", G.complete(40), 39),
    ("C61", G.cycle(61), 31),
    ("P60", G.path(60), 30),
    ("K7,30", G.complete_bipartite(7, 30), 7),
    ("Q6", G.hypercube(6), 32),
    ("grid6x7", G.grid(6, 7), 21),
])
def test_closed_forms_larger(oracle_lib, name, g, tau):
    assert oracle.mvc(g).size == tau
    assert oracle.pvc(g, tau).yes and not oracle.pvc(g, tau - 1).yes


def test_disjoint_union_adds(oracle_lib):
    parts = [G.petersen(), G.cycle(7), G.complete(5), G.path(6), G.erdos_renyi(12, 0.3, 4)]
    g = G.disjoint_union(*parts)
    assert oracle.mvc(g).size == sum(oracle.mvc(p).size for p in parts)


# ---- König ----------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(40))
def test_koenig_bipartite(oracle_lib, seed):
    rng = np.random.default_rng(seed)
    a, b = int(rng.integers(3, 28)), int(rng.integers(3, 28))
    p = float(rng.uniform(0.05, 0.35))
    g = G.random_bipartite(a, b, p, seed)
    u, v = G.edges_of(g)
    nu = matching_size(a, b, u, v - a)
    r = oracle.mvc(g)
    assert r.size == nu
    assert oracle.is_cover(g, r.cover)


# ---- planted covers ---------------------------------------------------------------------

def saturating_matching(g):
    cover = g.meta["cover"]
    in_c = np.zeros(g.n, bool)
    in_c[cover] = True
    pos = -np.ones(g.n, np.int64)
    pos[cover] = np.arange(cover.size)
    rest = np.flatnonzero(~in_c)
    rpos = -np.ones(g.n, np.int64)
    rpos[rest] = np.arange(rest.size)
    u, v = G.edges_of(g)
    cu = np.where(in_c[u], u, v)
    rv = np.where(in_c[u], v, u)
    cross = ~(in_c[u] & in_c[v])
    return matching_size(cover.size, rest.size, pos[cu[cross]], rpos[rv[cross]])


@pytest.mark.parametrize("seed", range(6))
def test_planted_small(oracle_lib, seed):
    g = G.planted_cover(120, 24, 300, 0.75, seed)
    c = g.meta["cover"].size
    assert oracle.is_cover(g, np.isin(np.arange(g.n), g.meta["cover"]))
    assert oracle.pvc(g, c).yes
    nu = saturating_matching(g)
    r = oracle.mvc(g)
    assert nu <= r.size <= c
    if nu == c:
        assert r.size == c and not oracle.pvc(g, c - 1).yes


@pytest.mark.parametrize("seed", range(4))
def test_planted_full_size(oracle_lib, seed):
    """n = 5000, |C| = 400, 40,000 edges (75% C-rest): PVC(400) = yes; a matching of the
    C-rest edges saturating C proves tau = 400, hence PVC(399) = no."""
    g = G.planted_cover(5000, 400, 40000, 0.75, seed)
    assert g.m == 40000
    assert saturating_matching(g) == 400
    yes = oracle.pvc(g, 400)
    assert yes.yes and yes.size <= 400 and oracle.is_cover(g, yes.cover)
    assert not oracle.pvc(g, 399).yes


# ---- consistency and soundness ------------------------------------------------------

@pytest.mark.parametrize("seed", range(12))
def test_mvc_pvc_consistent(oracle_lib, seed):
    g = G.erdos_renyi(40 + seed, 0.12, seed)
    tau = oracle.mvc(g).size
    assert oracle.pvc(g, tau).yes
    assert not oracle.pvc(g, tau - 1).yes


@pytest.mark.parametrize("seed", range(150))
def test_reduction_rules_sound(oracle_lib, seed):
    """tau(G) = s + tau(G reduced) for the degree-one and degree-two-triangle rules; with the
    high-degree rule at bound b >= tau the same holds, and at b < tau the reduced node must
    still have no cover within the remaining budget."""
    n = 5 + seed % 10
    g = G.random_small(n, 5000 + seed)
    tau, _ = oracle.tau_by_definition(g)
    deg0 = g.degrees()
    d, s = oracle.reduce(g, deg0, 0, 10**9, oracle.RULE_DEG1 | oracle.RULE_TRI)
    assert s + oracle.tau_by_definition(residual(g, d))[0] == tau
    for b in range(max(tau - 2, 0), tau + 2):
        d, s = oracle.reduce(g, deg0, 0, b)
        if s > b:
            assert tau > b
            continue
        rest = oracle.tau_by_definition(residual(g, d))[0]
        if b >= tau:
            assert s + rest == tau
        else:
            assert s + rest > b
        # the reduced degree array is consistent with the residual graph
        live = d >= 0
        assert np.array_equal(d[live], residual(g, d).degrees()[live])


@pytest.mark.parametrize("mask", [
    oracle.ALL & ~oracle.RULE_DEG1,
    oracle.ALL & ~oracle.RULE_TRI,
    oracle.ALL & ~oracle.PRUNE_EDGES,
    oracle.RULE_DEG1 | oracle.RULE_TRI,
    0,
])
def test_ablation_keeps_tau(oracle_lib, mask):
    for seed in range(30):
        g = G.random_small(6 + seed % 9, 9000 + seed)
        assert oracle.mvc(g, rules=mask).size == oracle.mvc(g).size
    g = G.erdos_renyi(60, 0.10, 0)
    full = oracle.mvc(g)
    abl = oracle.mvc(g, rules=mask, node_cap=5_000_000)
    assert abl.size == full.size
    assert abl.nodes >= full.nodes or mask == oracle.ALL & ~oracle.PRUNE_EDGES


def test_greedy_complete_graph(oracle_lib):
    for n in range(2, 30):
        s, c = oracle.greedy(G.complete(n))
        assert s == n - 1 and oracle.is_cover(G.complete(n), c)


def test_hand_traces(oracle_lib):
    with open(os.path.join(GOLDEN, "hand_traces.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        u, v = zip(*c["edges"])
        g = G.from_edges(c["n"], u, v)
        d, s = oracle.reduce(g, g.degrees(), 0, 10**9, oracle.RULE_DEG1 | oracle.RULE_TRI)
        assert d.tolist() == c["reduce"]["deg"] and s == c["reduce"]["s"], c["name"]
        r = oracle.mvc(g)
        assert (r.size, r.nodes, r.greedy) == (c["mvc"]["size"], c["mvc"]["nodes"],
                                              c["mvc"]["greedy"]), c["name"]
        gs, gcov = oracle.greedy(g)
        assert np.flatnonzero(gcov).tolist() == c["greedy_cover"], c["name"]


def test_budget_is_reported(oracle_lib):
    g = G.random_regular(120, 5, 0)
    with pytest.raises(oracle.BudgetExceeded):
        oracle.mvc(g, node_cap=1000)


def test_edgeless_and_k_zero(oracle_lib):
    g = G.empty(5)
    assert oracle.mvc(g).size == 0 and oracle.mvc(g).nodes == 0
    r = oracle.pvc(g, 0)
    assert r.yes and r.size == 0
    g = G.path(2)
    assert not oracle.pvc(g, 0).yes and oracle.pvc(g, 1).yes
