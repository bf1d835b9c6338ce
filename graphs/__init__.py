"""Seeded synthetic graph inputs shared by the tests, the benchmark and the oracle checks.

This package only draws graphs and packs them into CSR form. It contains none of the
vertex-cover method's arithmetic (no reduction rules, no search, no bounds), so both the
HIP path and the CPU oracle can be fed from it without sharing any of the method's code.

Every generator takes an explicit ``seed`` and uses ``numpy.random.default_rng(seed)``
(PCG64); the same seed always gives the same graph.
"""

from .csr import CSRGraph, from_edges, edges_of, disjoint_union
from .generators import (
    erdos_renyi,
    planted_cover,
    planted_batch,
    serving_draw,
    random_regular,
    complete,
    cycle,
    path,
    complete_bipartite,
    star,
    empty,
    complete_multipartite,
    hypercube,
    grid,
    petersen,
    random_bipartite,
    random_small,
)

__all__ = [
    "CSRGraph", "from_edges", "edges_of", "disjoint_union",
    "erdos_renyi", "planted_cover",
    "planted_batch", "serving_draw", "random_regular", "complete", "cycle", "path",
    "complete_bipartite", "star", "empty", "complete_multipartite", "hypercube", "grid",
    "petersen", "random_bipartite", "random_small",
]
