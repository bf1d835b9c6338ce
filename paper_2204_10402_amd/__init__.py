"""MI355X-native vertex-cover search (hybrid parallel branch-and-reduce, arXiv 2204.10402).

The work runs in libvc.so (HIP kernels for gfx950, C ABI in include/vc.h); this package is
the thin Python binding. Importing it does not load the library; creating a ``Solver`` does,
and fails loudly if the library has not been built.
"""

from ._binding import (  # noqa: F401
    EXPORTS, LIB_PATH, OK, ERR_BUDGET, ERR_DEVICE, ERR_INTERNAL, ERR_INVALID_ARG,
    ERR_INVALID_GRAPH, ERR_NO_MEMORY, OPT_NO_DEGREE_ONE, OPT_NO_EDGE_PRUNE, OPT_NO_HIGH_DEGREE,
    OPT_NO_TRIANGLE, OPT_PROFILE, OPT_DEGREE_ARRAYS, OPT_BITSETS, OPT_AUTOTUNE, OPT_STACK_ONLY, OPT_GLOBAL_NODES, OPT_CSR_GLOBAL, ACTIVITIES, BatchResult, Options,
    Result, Server, Solver, VCError, load_library, pack_batch, version, PROBLEM_MVC, PROBLEM_PVC,
)
