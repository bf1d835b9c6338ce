/*
 * vc.h -- C ABI of the MI355X vertex-cover search library (libvc.so).
 *
 * The library solves the two problems of the paper's problem statement (paper §II-A):
 *   - Minimum Vertex Cover (MVC): the smallest set S of vertices such that every edge has an
 *     endpoint in S. vc_mvc returns |S| and one such S.
 *   - Parameterized Vertex Cover (PVC): given k, a vertex cover with at most k vertices if
 *     one exists. vc_pvc returns yes/no and, on yes, a cover of size <= k.
 * Both run the paper's hybrid branch-and-reduce traversal (§IV-A) on one GPU: a persistent
 * grid in which every workgroup walks a sub-tree with its own stack in device memory and
 * shares branches through a global worklist; intermediate graphs are degree arrays over one
 * read-only CSR copy of the input (§IV-B).
 *
 * Graph format (all entry points): simple undirected graph (§II-A) in int32 CSR.
 *   n          number of vertices, 0 <= n < 2^31
 *   nnz        number of stored entries = 2|E| (every edge appears in both rows)
 *   row_ptr    n+1 entries, row_ptr[0] = 0, non-decreasing, row_ptr[n] = nnz
 *   col_idx    nnz entries; row v holds the neighbours of v, strictly ascending, no v itself,
 *              and u in row v  <=>  v in row u.
 * An input that breaks any of these rules is rejected with VC_ERR_INVALID_GRAPH; nothing is
 * repaired. The message names the first offending row: the smallest v whose bounds are wrong
 * or which holds an entry u that is out of range, equal to v, not above the entry before it,
 * or not found in row u by a binary search (which assumes row u ascending, so an unsorted row
 * can also make a neighbour's row the first one named). Vertices of degree 0 never enter a
 * returned cover.
 *
 * Threading: one call at a time per context. Separate contexts may be used concurrently.
 * Ownership: every pointer argument stays owned by the caller; the library keeps no
 * reference after a call returns. The context owns its device workspace (kept and grown
 * across calls) and, if it created one, its HIP stream.
 * Errors: every entry point returns VC_OK (0) or a negative VC_ERR_* code. On error the
 * host output arguments are left untouched (device cover buffers may have been written) and
 * vc_last_error() describes the failure.
 *
 * Batches: vc_mvc_batch / vc_pvc_batch solve many independent graphs in one persistent
 * launch per kernel family (bitset kernels by words per row, degree-array kernels): every
 * graph's root is handed out to the workgroups in turn, and the sub-trees of all graphs share
 * one worklist. A single-graph call is a batch of one.
 */
#ifndef VC_H
#define VC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------------------- */
#define VC_OK 0
#define VC_ERR_INVALID_GRAPH (-1) /* CSR breaks the format above (first offending row named) */
#define VC_ERR_INVALID_ARG (-2)   /* NULL pointer, k < 0, bad option, graph too large for LDS */
#define VC_ERR_NO_MEMORY (-3)     /* stacks + worklist do not fit in free device memory */
#define VC_ERR_BUDGET (-4)        /* node budget exhausted, time limit reached or vc_abort
                                     called before the search ended */
#define VC_ERR_DEVICE (-5)        /* a HIP runtime call failed, or no usable device */
#define VC_ERR_INTERNAL (-6)      /* a device-side invariant failed (stack overflow, or a
                                     returned cover failed edge-by-edge verification) */

/* ---- option flags (vc_options.flags) -------------------------------------------------- */
#define VC_OPT_NO_DEGREE_ONE 0x1  /* ablation: switch off the degree-one rule */
#define VC_OPT_NO_TRIANGLE 0x2    /* ablation: switch off the degree-two-triangle rule */
#define VC_OPT_NO_HIGH_DEGREE 0x4 /* ablation: switch off the high-degree rule (this also
                                     switches off the |E| > r^2 prune, which relies on it) */
#define VC_OPT_NO_EDGE_PRUNE 0x8  /* ablation: switch off the |E| > r^2 prune */
#define VC_OPT_PROFILE 0x10       /* run the instrumented traversal kernel, which charges shader
                                     clock cycles to activities (vc_stats.cycles) */
#define VC_OPT_DEGREE_ARRAYS 0x20 /* use the degree-array kernels (the default above 256
                                     vertices): a node is an int32 degree array in LDS */
#define VC_OPT_BITSETS 0x40       /* use the bitset kernels (the default up to 256 vertices;
                                     available up to 512, VC_ERR_INVALID_ARG above): a node is
                                     the set of live vertices, held in registers */
#define VC_OPT_STACK_ONLY 0x100   /* ablation: the StackOnly method the paper compares with
                                     (§V-A): no worklist; workgroup w takes the sub-trees at
                                     depth start_depth numbered w, w + grid, ..., walks down
                                     to each from the root and walks it with its own stack.
                                     One graph per call (a batch of one). */
#define VC_OPT_GLOBAL_NODES 0x200 /* keep the degree-array node in device memory instead of LDS
                                     (implies the degree-array kernels). Chosen automatically
                                     when a node does not fit in LDS (n above about 39,000) */
#define VC_OPT_CSR_GLOBAL 0x400  /* degree-array kernels: read the graph's column indices from
                                     device memory on every row walk. Without it a launch copies
                                     each instance's CSR into LDS beside the node when that keeps
                                     at least half of its resident workgroups; answers and node
                                     counts are the same either way */
#define VC_OPT_AUTOTUNE 0x80      /* pick workgroup size, grid size and donation threshold of
                                     each launch by timing trial launches the first time this
                                     context sees its kernel family, problem, options and size
                                     class (n_max and number of graphs, by powers of two), and
                                     reuse the choice afterwards; ignored when any launch knob
                                     of vc_options is set */

typedef struct vc_ctx vc_ctx;
typedef struct vc_server vc_server;

typedef struct {
  int32_t n;
  int32_t nnz;
  const int32_t *row_ptr; /* n+1 entries */
  const int32_t *col_idx; /* nnz entries */
} vc_graph;

/* Launch and search knobs; a zeroed struct (or NULL) means "choose automatically". */
typedef struct {
  int32_t wg_size;      /* threads per workgroup, a multiple of 64 up to 1024; 0 = auto
                           (the occupancy rule of §IV-E) */
  int32_t num_wg;       /* workgroups in the persistent grid; 0 = as many as are co-resident;
                           larger values are clamped to the co-resident maximum */
  int32_t wl_capacity;  /* global worklist entries (rounded up to a power of two); 0 = auto */
  int32_t wl_threshold; /* a branch is donated to the worklist only while it holds fewer than
                           this many entries (§IV-A); 0 = auto; -1 = never donate (every
                           workgroup keeps its whole sub-tree on its own stack) */
  int64_t node_budget;  /* stop with VC_ERR_BUDGET after about this many nodes (per graph
                           of a batch); 0 = none */
  int32_t flags;        /* VC_OPT_* */
  int32_t grid_share;   /* > 0: use at most 1/grid_share of the co-resident grid (callers that
                           run several launches side by side); 0 = all of it */
  int32_t start_depth;  /* with VC_OPT_STACK_ONLY: depth of the sub-trees handed out, 1..24;
                           0 = 12 */
  int32_t stack_depth;  /* stack entries per workgroup; 0 = the depth bound of §IV-E (enough
                           for any search). A smaller value is the caller's promise: a
                           workgroup that would need more stops the call with
                           VC_ERR_INTERNAL ("stack overflow") */
  int32_t timeout_ms;   /* > 0: stop each traversal launch after about this many milliseconds
                           of the device clock (measured from the launch's start, checked every
                           few nodes and while idle); the call returns VC_ERR_BUDGET. 0: none */
  int32_t reserved;     /* must be zero */
} vc_options;

/* A batch of independent graphs, each in the format above, packed one after the other. */
typedef struct {
  int32_t count;           /* number of graphs, 0 <= count <= 2^22 */
  const int32_t *n;        /* HOST, count entries: vertices of graph i */
  const int32_t *nnz;      /* HOST, count entries: stored CSR entries of graph i */
  const int32_t *row_ptr;  /* sum(n[i] + 1) entries: graph i's row_ptr (starting at 0), then
                              graph i+1's */
  const int32_t *col_idx;  /* sum(nnz[i]) entries: graph i's neighbour ids (0..n[i]-1), then
                              graph i+1's */
} vc_batch;

/* Per-call statistics. A search-tree node is one visit: a node is taken from the stack or
 * the worklist (or continued in place) and the reduction rules run on it. */
typedef struct {
  int64_t nodes;          /* search-tree nodes visited, each counted once */
  int64_t wg_nodes_max;   /* most nodes visited by one workgroup (with VC_OPT_STACK_ONLY
                             including its walks down from the root) */
  int64_t wg_nodes_min;   /* fewest nodes visited by one workgroup */
  int64_t stack_pushes;   /* deferred children kept on a workgroup's own stack */
  int64_t stack_pops;
  int64_t wl_enqueues;    /* deferred children donated to the worklist */
  int64_t wl_dequeues;    /* worklist entries taken (roots are handed out separately) */
  int32_t max_stack_depth;
  int32_t greedy_size;    /* MVC: size of the greedy cover that seeds the bound; PVC: -1 */
  int32_t wg_size;
  int32_t num_wg;
  int32_t wl_capacity;
  int32_t wl_threshold;
  int32_t depth_cap;      /* stack entries provisioned per workgroup */
  int32_t n;              /* vertices (batches: of the largest graph) */
  int32_t bitset_words;   /* 64-bit words per node with the bitset kernels; 0 = degree arrays
                             (batches: the largest used) */
  int32_t node_bytes;     /* bytes of one search node's state (batches: the largest) */
  double kernel_ms;       /* traversal kernel time (HIP events; batches: summed over the
                             launches, or, when a batch's degree-array launch runs beside its
                             bitset launches, the span from its start to the last one's end) */
  double greedy_ms;       /* greedy kernel time (MVC) */
  double total_ms;        /* wall clock of the whole call */
  /* With VC_OPT_PROFILE, shader-clock cycles summed over the workgroups (paper §V-D):
   * [0] taking nodes (stack pops, worklist dequeues, waiting for work), [1] reduction rules,
   * [2] branching (max-degree pass, stopping test, removing v_max or N(v_max)),
   * [3] deferring children (stack pushes, worklist enqueues), [4] other (flags, bound,
   * recording covers), [5] the whole kernel; with the degree-array kernels [1] is split into
   * [6] degree-one decisions, [7] degree-two-triangle decisions, [8] high-degree decisions,
   * [9] removing the decided vertices. Zero without VC_OPT_PROFILE. */
  int64_t cycles[10];
  /* Where the search moved its nodes (paper §IV-A, §IV-E: stacks and worklist), in bytes of
   * node state (the degree array or live-vertex bitset, |S|, pending vertex, instance):
   * hbm_node_bytes counts worklist enqueues and dequeues and the pushes and pops of stacks in
   * device memory; lds_node_bytes the pushes and pops of stacks held in LDS. graph_bytes
   * estimates the graph data workgroups copied from device memory into LDS or registers on
   * taking an instance (bitset adjacency rows, or the staged CSR of the degree-array kernels),
   * from each launch's mean graph size. */
  int64_t hbm_node_bytes;
  int64_t lds_node_bytes;
  int64_t graph_bytes;
  int32_t stack_lds;      /* 1 if a traversal launch kept its stacks in LDS */
  int32_t launches;       /* traversal launches of the call (one per kernel family) */
} vc_stats;

/* Create a context on HIP device `device`. `hip_stream` is a hipStream_t to run on, or NULL
 * for a stream owned by the context. A batch holding graphs of both kernel families (unless
 * vc_options.grid_share is set) also runs on a second stream and workspace that the context
 * creates on first use and owns; the call still returns only when all of its work is done,
 * ordered after earlier work on `hip_stream` and before later work there. */
int vc_create(vc_ctx **ctx_out, int device, void *hip_stream);

/* Release the context, its workspace and its own stream. NULL is accepted. */
int vc_destroy(vc_ctx *ctx);

/* Text of a status code. */
const char *vc_strerror(int status);

/* Per-workgroup statistics of the context's last traversal launch (the last kernel family of
 * a batch launched), for up to `max` workgroups; *count_out = the grid size. `nodes_out` (may be NULL):
 * nodes visited by each workgroup (with VC_OPT_STACK_ONLY including its walks down from the
 * root). `cycles_out` (may be NULL; 10 per workgroup, in the order of vc_stats.cycles):
 * its activity clocks, zero unless the launch ran with VC_OPT_PROFILE. */
int vc_wg_loads(vc_ctx *ctx, int64_t *nodes_out, int64_t *cycles_out, int32_t max,
                int32_t *count_out);

/* Stop the call running on this context, from any thread (the one function that may run while
 * another call on the context is in progress). The traversal kernels see the request within
 * about 50 microseconds of the device clock (workgroup 0 reads a host-pinned word; every
 * workgroup then sees the launch-wide stop at its next look at the control words), every
 * workgroup exits normally, and the call returns VC_ERR_BUDGET. Calling it when no call runs
 * has no effect on later calls. */
int vc_abort(vc_ctx *ctx);

/* Description of the last failure on this context ("" if none). Valid until the next call. */
const char *vc_last_error(const vc_ctx *ctx);

/* Library version, "major.minor.patch". */
const char *vc_version(void);

/* MVC (paper §II-A, §II-B, §IV-A). `g` holds HOST pointers. On success *size_out = tau(G) and,
 * if cover_out is not NULL, cover_out[v] = 1 for the n vertices of one minimum cover
 * (any minimum cover may be returned), 0 elsewhere. `opts` and `stats` may be NULL. */
int vc_mvc(vc_ctx *ctx, const vc_graph *g, const vc_options *opts, int32_t *size_out,
           uint8_t *cover_out, vc_stats *stats);

/* PVC (paper §II-A; search differences in §II-B and §IV-A). `g` holds HOST pointers; k >= 0.
 * On success *yes_out = 1 and *size_out = |S| <= k with cover_out[v] = 1 on S, or
 * *yes_out = 0, *size_out = -1 and cover_out all zero. `opts` and `stats` may be NULL. */
int vc_pvc(vc_ctx *ctx, const vc_graph *g, int32_t k, const vc_options *opts,
           int32_t *yes_out, int32_t *size_out, uint8_t *cover_out, vc_stats *stats);

/* Device-resident forms of vc_mvc / vc_pvc: `g->row_ptr` and `g->col_idx` are DEVICE
 * pointers on the context's device and `cover_dev` (n bytes, may be NULL) is written in
 * device memory. The call runs on the context stream, after work already queued on it, and
 * returns when the search has finished. Size and yes/no are returned in host memory. */
int vc_mvc_device(vc_ctx *ctx, const vc_graph *g, const vc_options *opts, int32_t *size_out,
                  uint8_t *cover_dev, vc_stats *stats);
int vc_pvc_device(vc_ctx *ctx, const vc_graph *g, int32_t k, const vc_options *opts,
                  int32_t *yes_out, int32_t *size_out, uint8_t *cover_dev, vc_stats *stats);

/* Batched MVC / PVC (paper §II-A, §IV-A). Each graph of the batch is solved exactly as the
 * single-graph calls solve it; the graphs share the device. `batch->row_ptr` and
 * `batch->col_idx` are HOST pointers (vc_*_batch) or DEVICE pointers on the context's device
 * (vc_*_batch_device); `k` (PVC) has count entries, each >= 0. Per graph i (HOST arrays of
 * count entries):
 *   status_out[i]  VC_OK, VC_ERR_INVALID_GRAPH (graph i breaks the CSR format) or
 *                  VC_ERR_BUDGET (graph i used up opts->node_budget, which applies per graph);
 *   size_out[i]    MVC: tau(G_i); PVC: |S| <= k[i] on yes, -1 on no; -1 unless status is OK;
 *   yes_out[i]     PVC: 1 or 0 (0 unless status is OK);
 *   nodes_out[i]   search-tree nodes visited on graph i (may be NULL).
 * The cover output (may be NULL) has sum(n[i]) bytes, graph i's n[i] bytes after those of the
 * graphs before it: 1 on its cover, all 0 for PVC no or a status other than VC_OK; it is host
 * memory for vc_*_batch and device memory for vc_*_batch_device. The call itself returns VC_OK
 * when every graph has a status, else an error for the whole batch (bad arguments, device or
 * internal error). `stats` (may be NULL) sums over the batch. */
int vc_mvc_batch(vc_ctx *ctx, const vc_batch *batch, const vc_options *opts, int32_t *status_out,
                 int32_t *size_out, uint8_t *cover_out, int64_t *nodes_out, vc_stats *stats);
int vc_pvc_batch(vc_ctx *ctx, const vc_batch *batch, const int32_t *k, const vc_options *opts,
                 int32_t *status_out, int32_t *yes_out, int32_t *size_out, uint8_t *cover_out,
                 int64_t *nodes_out, vc_stats *stats);
int vc_mvc_batch_device(vc_ctx *ctx, const vc_batch *batch, const vc_options *opts,
                        int32_t *status_out, int32_t *size_out, uint8_t *cover_dev,
                        int64_t *nodes_out, vc_stats *stats);
int vc_pvc_batch_device(vc_ctx *ctx, const vc_batch *batch, const int32_t *k,
                        const vc_options *opts, int32_t *status_out, int32_t *yes_out,
                        int32_t *size_out, uint8_t *cover_dev, int64_t *nodes_out,
                        vc_stats *stats);

/* ---- caller-owned workspace (device memory from the caller, e.g. a torch tensor) ----------
 * The *_ws forms are the device forms above with every piece of device memory a call needs --
 * instance table and per-instance state, worklist ring and tickets (§IV-A), per-workgroup
 * stacks (§IV-E), control words, covers when cover_dev is NULL -- carved from one caller buffer
 * instead of the context's own allocations, on the context's stream (pass the caller's stream
 * to vc_create). They allocate no device memory and create no stream; host staging uses the
 * context's pinned buffer, or ordinary host memory for a batch larger than it. They do not
 * autotune (vc_options.flags' VC_OPT_AUTOTUNE is ignored: a trial grid need not fit the
 * workspace), and a batch mixing kernel families runs its launches one after another.
 * Ownership: the workspace stays the caller's; the library keeps no pointer into it after the
 * call returns (vc_wg_loads then reports no workgroups). Two calls must not share a workspace
 * at the same time.
 *
 * vc_workspace_bytes: bytes that a *_ws call on one graph of n vertices and nnz CSR entries
 * needs with the launch knobs of `opts` (the same options the call will take; NULL = automatic)
 * and `depth` stack entries per workgroup (0: n + 1, enough for MVC and every k). It takes the
 * larger of the MVC and PVC needs. A smaller workspace still works while the worklist and one
 * workgroup's stack fit: the grid then shrinks until the stacks fit (the memory bound on
 * parallelism of §IV-E); else the call fails with VC_ERR_NO_MEMORY.
 * vc_batch_workspace_bytes: the same for a batch (its count, n and nnz; pointers may be NULL). */
int vc_workspace_bytes(vc_ctx *ctx, int32_t n, int32_t nnz, int32_t depth,
                       const vc_options *opts, size_t *bytes_out);
int vc_batch_workspace_bytes(vc_ctx *ctx, const vc_batch *batch, int32_t depth,
                             const vc_options *opts, size_t *bytes_out);

/* MVC / PVC (paper §II-A) as vc_mvc_device / vc_pvc_device, in the caller's workspace
 * (`workspace`: device memory on the context's device, 256-byte aligned, `workspace_bytes`
 * long). */
int vc_mvc_device_ws(vc_ctx *ctx, const vc_graph *g, const vc_options *opts, void *workspace,
                     size_t workspace_bytes, int32_t *size_out, uint8_t *cover_dev,
                     vc_stats *stats);
int vc_pvc_device_ws(vc_ctx *ctx, const vc_graph *g, int32_t k, const vc_options *opts,
                     void *workspace, size_t workspace_bytes, int32_t *yes_out,
                     int32_t *size_out, uint8_t *cover_dev, vc_stats *stats);

/* Batched MVC / PVC (paper §II-A) as vc_mvc_batch_device / vc_pvc_batch_device, in the caller's
 * workspace. */
int vc_mvc_batch_device_ws(vc_ctx *ctx, const vc_batch *batch, const vc_options *opts,
                           void *workspace, size_t workspace_bytes, int32_t *status_out,
                           int32_t *size_out, uint8_t *cover_dev, int64_t *nodes_out,
                           vc_stats *stats);
int vc_pvc_batch_device_ws(vc_ctx *ctx, const vc_batch *batch, const int32_t *k,
                           const vc_options *opts, void *workspace, size_t workspace_bytes,
                           int32_t *status_out, int32_t *yes_out, int32_t *size_out,
                           uint8_t *cover_dev, int64_t *nodes_out, vc_stats *stats);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): vc_pvc_device (paper §II-A) whose worklist, stacks,
 * control words and instance state live in a fixed device array of the library, 64 MiB per
 * device, held by each GPU the library has run on until the process ends. The call allocates
 * no device or pinned memory and creates no stream (its host bookkeeping uses ordinary heap
 * memory); graph, k, outputs and errors are those of vc_pvc_device. The launch plan shrinks
 * (grid, worklist ring) until it fits the array; a graph that does not fit even one workgroup
 * returns VC_ERR_NO_MEMORY with a message naming the limit. Every call on a device shares
 * that device's array: calls that overlap on one device -- from different contexts or threads
 * -- race and must not be made. Each call resets what must start at zero. No autotuning; a
 * call runs on the context's stream and returns when the search has finished. */
int vc_pvc_device_noalloc(vc_ctx *ctx, const vc_graph *g, int32_t k, const vc_options *opts,
                          int32_t *yes_out, int32_t *size_out, uint8_t *cover_dev,
                          vc_stats *stats);

/* ---- serving: continuous batching of a request stream ----------------------------------
 * A server owns `workers` threads, each with its own context (device workspace and stream).
 * Submitted requests are queued with a copy of their graph. A free worker takes the oldest
 * waiting request's problem kind and, in arrival order, every waiting request of that kind
 * that fits the memory budget (at most max_batch), and solves them as one batch (as
 * vc_mvc_batch / vc_pvc_batch) with wg_per_request traversal workgroups per request; requests
 * arriving meanwhile are taken by other workers, so batches overlap on the device (each batch's
 * grid is at most 1/workers of the co-resident grid). Each result
 * is exactly the answer the single-graph call gives for that graph (size, decision, a verified
 * cover). The budget counts the node stacks a batch provisions (workgroups x depth bound x
 * node bytes); a request that alone exceeds it runs when nothing else is in flight. */
#define VC_PROBLEM_MVC 0
#define VC_PROBLEM_PVC 1

typedef struct {
  int32_t workers;         /* concurrent batches; 0 = 4 */
  int32_t max_batch;       /* requests per batch at most; 0 = 32 */
  int64_t memory_budget;   /* bytes of node stacks in flight at most; 0 = 1/4 of free memory */
  int32_t wg_per_request;  /* traversal workgroups per request of a batch, up to an equal share
                              of the device per worker; 0 = 256 */
  int32_t reserved[3];     /* must be zero */
} vc_server_options;

typedef struct {
  int64_t ticket;          /* from vc_server_submit */
  int32_t status;          /* VC_OK, VC_ERR_INVALID_GRAPH, VC_ERR_BUDGET, or the batch's error */
  int32_t size;            /* MVC: tau(G); PVC: |S| <= k on yes, -1 on no; -1 on error */
  int32_t yes;             /* PVC decision (1 for an MVC answer) */
  int32_t batch_size;      /* requests in the batch that solved it */
  int32_t worker;          /* the worker (stream) that ran the batch */
  int32_t pad;
  int64_t nodes;           /* search-tree nodes visited on this graph */
  double submit_ms;        /* times on the server's clock (ms since vc_server_create) */
  double start_ms;
  double done_ms;
} vc_served;

/* Create a server on `device`. `opts` (may be NULL) applies to every batch; its num_wg and
 * VC_OPT_AUTOTUNE are not accepted (the grid follows the batch size). */
int vc_server_create(vc_server **server_out, int device, const vc_server_options *sopts,
                     const vc_options *opts);
/* Queue one request: `g` holds HOST pointers and is copied before the call returns; k is
 * used for VC_PROBLEM_PVC. `cover_out` (may be NULL; n bytes of host memory that must stay
 * valid until the result is polled) receives the cover before the result is reported. */
int vc_server_submit(vc_server *server, const vc_graph *g, int32_t problem, int32_t k,
                     uint8_t *cover_out, int64_t *ticket_out);
/* Move up to `max` finished results to `out`, in completion order; if none is ready, wait up
 * to timeout_ms for one. *count_out is the number moved. */
int vc_server_poll(vc_server *server, vc_served *out, int32_t max, int32_t timeout_ms,
                   int32_t *count_out);
/* Requests waiting and requests in running batches (either may be NULL). */
int vc_server_pending(vc_server *server, int32_t *queued, int32_t *running);
/* Finish the running batches, drop the waiting requests, release everything. */
int vc_server_destroy(vc_server *server);

/* The greedy approximation that seeds MVC's bound (paper §II-B, §IV-E), on the GPU with one
 * workgroup: apply the degree-one and degree-two-triangle rules, put a vertex of maximum
 * degree (smallest id on ties) in the cover, repeat until no edge is left. DEVICE graph
 * pointers; `cover_dev` (n bytes, may be NULL) in device memory; size in host memory. */
int vc_greedy_device(vc_ctx *ctx, const vc_graph *g, int32_t *size_out, uint8_t *cover_dev);

/* The reduction rules of one search-tree node (paper §II-B, parallel rules §IV-D), applied
 * until the graph stops changing, exactly as the traversal applies them, by one workgroup.
 * DEVICE pointers: `deg_dev` (n int32, in/out) is a degree array (degree of each vertex, -1
 * for vertices already in the cover) consistent with the CSR; *s_inout (host) is the cover
 * size so far. `bound` is the largest cover size still of interest (MVC: best - 1, PVC: k);
 * the passes stop early once the cover size exceeds it. `flags` takes VC_OPT_NO_* bits. */
int vc_reduce_device(vc_ctx *ctx, const vc_graph *g, int32_t *deg_dev, int32_t *s_inout,
                     int64_t bound, int32_t flags);

#ifdef __cplusplus
}
#endif

#endif /* VC_H */
