"""Seeded graph generators.

The random families stand in for the paper's public graph collections (DIMACS p_hat
complements, KONECT, SNAP, PACE; paper §V-A and Table I), which are not reproduced here:
- ``erdos_renyi``: G(n, p), each pair i<j drawn once, row-major order of the upper triangle;
- ``planted_cover``: a hidden cover C; every edge has an endpoint in C;
- ``random_regular``: the configuration model, resampled whole on a loop or multi-edge.
The structured families (complete, cycle, path, ...) have textbook minimum-cover sizes.
"""

from __future__ import annotations

import numpy as np

from .csr import CSRGraph, from_edges


def erdos_renyi(n: int, p: float, seed: int) -> CSRGraph:
    """G(n, p): the upper-triangle Bernoulli(p) mask is drawn in row-major i<j order."""
    rng = np.random.default_rng(seed)
    iu, ju = np.triu_indices(n, 1)
    mask = rng.random(iu.shape[0]) < p
    return from_edges(n, iu[mask], ju[mask],
                      meta={"family": "er", "n": n, "p": p, "seed": seed})


def planted_cover(n: int, c: int, m: int, cross_frac: float, seed: int) -> CSRGraph:
    """Planted-cover graph: C = ``rng.choice(n, c)`` without replacement; ``round(m*cross_frac)``
    distinct C-rest edges (C endpoint uniform in C, other endpoint uniform in the rest) and the
    remaining edges distinct pairs inside C. Duplicates and loops are rejected and redrawn, so
    every edge has at least one endpoint in C and C is a vertex cover of size c.
    """
    return _planted(np.random.default_rng(seed), n, c, m, cross_frac,
                    {"family": "planted", "n": n, "c": c, "m": m, "cross_frac": cross_frac,
                     "seed": seed})


def _planted(rng, n, c, m, cross_frac, meta):
    if not (0 < c <= n):
        raise ValueError("need 0 < c <= n")
    cover = np.sort(rng.choice(n, size=c, replace=False))
    in_c = np.zeros(n, dtype=bool)
    in_c[cover] = True
    rest = np.flatnonzero(~in_c)
    m_cross = int(round(m * cross_frac))
    m_in = m - m_cross
    if m_cross > c * rest.size or m_in > c * (c - 1) // 2:
        raise ValueError("too many edges for the planted structure")
    seen: set[int] = set()
    us: list[int] = []
    vs: list[int] = []

    def draw(count, pick_a, pick_b):
        got = 0
        while got < count:
            batch = max(64, 2 * (count - got))
            a = pick_a(batch)
            b = pick_b(batch)
            for x, y in zip(a.tolist(), b.tolist()):
                if x == y:
                    continue
                lo, hi = (x, y) if x < y else (y, x)
                key = lo * n + hi
                if key in seen:
                    continue
                seen.add(key)
                us.append(lo)
                vs.append(hi)
                got += 1
                if got == count:
                    break

    if rest.size:
        draw(m_cross, lambda k: cover[rng.integers(0, c, k)],
             lambda k: rest[rng.integers(0, rest.size, k)])
    draw(m_in, lambda k: cover[rng.integers(0, c, k)], lambda k: cover[rng.integers(0, c, k)])
    return from_edges(n, us, vs, meta={**meta, "cover": cover.astype(np.int32)})


def planted_batch(count: int, seed: int, n_lo: int = 40, n_hi: int = 400,
                  deg_lo: float = 3.0, deg_hi: float = 12.0, cover_frac: float = 0.3,
                  cross_frac: float = 0.75) -> list[tuple[CSRGraph, int]]:
    """A batch of independent planted-cover PVC instances.

    Instance ``i`` draws everything from ``default_rng([seed, i])``: n uniform in
    [n_lo, n_hi], average degree d uniform in [deg_lo, deg_hi), |C| = floor(cover_frac*n),
    m = round(d*n/2) edges split ``cross_frac`` C-rest and the rest inside C, as in
    ``planted_cover``. Its parameter is k = |C| for even i (a yes-instance) and |C|-1 for
    odd i. Returns ``[(graph, k), ...]``; ``graph.meta["cover"]`` holds C.
    """
    out = []
    for i in range(count):
        rng = np.random.default_rng([seed, i])
        n = int(rng.integers(n_lo, n_hi + 1))
        d = float(rng.uniform(deg_lo, deg_hi))
        c = int(np.floor(cover_frac * n))
        m = int(round(d * n / 2))
        g = _planted(rng, n, c, m, cross_frac,
                     {"family": "planted_batch", "n": n, "c": c, "m": m, "avg_degree": d,
                      "cross_frac": cross_frac, "seed": seed, "index": i})
        out.append((g, c if i % 2 == 0 else c - 1))
    return out


def random_regular(n: int, d: int, seed: int, max_tries: int = 100000) -> CSRGraph:
    """d-regular simple graph by the configuration model: n*d stubs, a uniform random perfect
    pairing, the whole pairing redrawn whenever it has a loop or a multi-edge."""
    if (n * d) % 2 or d >= n:
        raise ValueError("no simple d-regular graph on n vertices")
    rng = np.random.default_rng(seed)
    stubs = np.repeat(np.arange(n, dtype=np.int64), d)
    for tries in range(1, max_tries + 1):
        pairs = rng.permutation(stubs).reshape(-1, 2)
        a, b = pairs[:, 0], pairs[:, 1]
        if np.any(a == b):
            continue
        lo, hi = np.minimum(a, b), np.maximum(a, b)
        if np.unique(lo * n + hi).size != lo.size:
            continue
        return from_edges(n, lo, hi, meta={"family": "regular", "n": n, "d": d,
                                           "seed": seed, "tries": tries})
    raise RuntimeError("configuration model did not produce a simple graph")


def random_bipartite(a: int, b: int, p: float, seed: int) -> CSRGraph:
    """Random bipartite graph: parts [0, a) and [a, a+b), each cross pair kept with prob. p."""
    rng = np.random.default_rng(seed)
    mask = rng.random((a, b)) < p
    i, j = np.nonzero(mask)
    return from_edges(a + b, i, j + a, meta={"family": "bipartite", "a": a, "b": b,
                                             "p": p, "seed": seed})


def random_small(n: int, seed: int) -> CSRGraph:
    """Small random graph for exhaustive checks: a G(n, p) with p drawn from [0.1, 0.6], plus
    seeded pendant vertices and triangles so the degree-one and degree-two rules fire."""
    rng = np.random.default_rng(seed)
    p = float(rng.uniform(0.1, 0.6))
    iu, ju = np.triu_indices(n, 1)
    keep = rng.random(iu.shape[0]) < p
    edges = set(zip(iu[keep].tolist(), ju[keep].tolist()))
    if n >= 4:
        for _ in range(int(rng.integers(0, 3))):
            x, y, z = rng.choice(n, size=3, replace=False).tolist()
            # make x a degree-two vertex of the triangle x-y-z
            edges = {e for e in edges if x not in e}
            for e in ((x, y), (x, z), (y, z)):
                edges.add((min(e), max(e)))
        for _ in range(int(rng.integers(0, 3))):
            x, y = rng.choice(n, size=2, replace=False).tolist()
            edges = {e for e in edges if x not in e}
            edges.add((min(x, y), max(x, y)))
    if not edges:
        return from_edges(n, [], [], meta={"family": "small", "seed": seed})
    u, v = zip(*sorted(edges))
    return from_edges(n, u, v, meta={"family": "small", "seed": seed})


# ---- structured families with known minimum cover sizes -------------------------------

def empty(n: int) -> CSRGraph:
    return from_edges(n, [], [], meta={"family": "empty"})


def complete(n: int) -> CSRGraph:
    iu, ju = np.triu_indices(n, 1)
    return from_edges(n, iu, ju, meta={"family": "K"})


def cycle(n: int) -> CSRGraph:
    if n < 3:
        raise ValueError("cycle needs n >= 3")
    u = np.arange(n)
    return from_edges(n, u, (u + 1) % n, meta={"family": "C"})


def path(n: int) -> CSRGraph:
    u = np.arange(max(n - 1, 0))
    return from_edges(n, u, u + 1, meta={"family": "P"})


def complete_bipartite(a: int, b: int) -> CSRGraph:
    i, j = np.meshgrid(np.arange(a), np.arange(a, a + b), indexing="ij")
    return from_edges(a + b, i.ravel(), j.ravel(), meta={"family": "Kab"})


def star(leaves: int) -> CSRGraph:
    return from_edges(leaves + 1, np.zeros(leaves, np.int64), np.arange(1, leaves + 1),
                      meta={"family": "star"})


def complete_multipartite(parts: list[int]) -> CSRGraph:
    """Every pair of vertices in different parts is adjacent."""
    label = np.repeat(np.arange(len(parts)), parts)
    n = label.size
    iu, ju = np.triu_indices(n, 1)
    keep = label[iu] != label[ju]
    return from_edges(n, iu[keep], ju[keep], meta={"family": "multipartite"})


def hypercube(d: int) -> CSRGraph:
    n = 1 << d
    us, vs = [], []
    for x in range(n):
        for bit in range(d):
            y = x ^ (1 << bit)
            if x < y:
                us.append(x)
                vs.append(y)
    return from_edges(n, us, vs, meta={"family": "Q"})


def grid(a: int, b: int) -> CSRGraph:
    idx = np.arange(a * b).reshape(a, b)
    us = np.concatenate([idx[:, :-1].ravel(), idx[:-1, :].ravel()])
    vs = np.concatenate([idx[:, 1:].ravel(), idx[1:, :].ravel()])
    return from_edges(a * b, us, vs, meta={"family": "grid"})


def petersen() -> CSRGraph:
    outer = [(i, (i + 1) % 5) for i in range(5)]
    spokes = [(i, i + 5) for i in range(5)]
    inner = [(5 + i, 5 + (i + 2) % 5) for i in range(5)]
    u, v = zip(*(outer + spokes + inner))
    return from_edges(10, u, v, meta={"family": "petersen"})



def serving_draw(master_seed: int, i: int) -> tuple[dict, CSRGraph]:
    """Draw number ``i`` of a served request stream, from ``default_rng([master_seed, i])``:
    n = round(exp(U[ln 50, ln 2000])); family uniform over
      - "er": G(n, d/(n-1)) with average degree d uniform in [4, 10),
      - "planted": planted cover |C| = floor(0.3 n), m = round(d n / 2) edges, d uniform in
        [3, 12), 75 % C-rest (capped at what the structure allows),
      - "regular": random d-regular, d uniform in {3, 4, 5} (n + 1 when n d is odd);
    problem "mvc" or "pvc" with probability 1/2 each. Returns (description, graph).
    """
    rng = np.random.default_rng([master_seed, i])
    n = int(round(np.exp(rng.uniform(np.log(50), np.log(2000)))))
    family = ("er", "planted", "regular")[int(rng.integers(0, 3))]
    problem = ("mvc", "pvc")[int(rng.integers(0, 2))]
    sub = int(rng.integers(0, 2**31))
    desc = {"draw": i, "family": family, "problem": problem, "sub_seed": sub}
    if family == "er":
        d = float(rng.uniform(4, 10))
        g = erdos_renyi(n, d / (n - 1), sub)
        desc.update(avg_degree=d)
    elif family == "planted":
        d = float(rng.uniform(3, 12))
        c = int(0.3 * n)
        m = int(round(d * n / 2))
        m = min(m, int(round((c * (n - c)) / 0.75)) - 1, c * (n - c) + c * (c - 1) // 2 - 1)
        g = planted_cover(n, c, m, 0.75, sub)
        desc.update(avg_degree=d, cover=c, m=m)
    else:
        d = int(rng.integers(3, 6))
        if (n * d) % 2:
            n += 1
        g = random_regular(n, d, sub)
        desc.update(degree=d)
    desc["n"] = n
    return desc, g
