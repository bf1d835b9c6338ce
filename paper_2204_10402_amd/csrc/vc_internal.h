// vc_internal.h -- shared between the device code (vc_device.hip, vc_bitset.hip) and the host
// runtime (vc_host.cpp). Not part of the public ABI.
//
// Every launch works on a batch of instances; a single call is a batch of one. The graphs of
// a batch are packed: instance i's n_i + 1 row pointers (its own numbering, starting at 0)
// sit at rp_off in one row_ptr array, its nnz_i neighbour ids (0..n_i-1) at ci_off in one
// col_idx array. A search-tree node carries the instance it belongs to; a workgroup takes the
// root of an unstarted instance or a node from the worklist, and loads that node's instance
// (its row pointers or adjacency rows) only when it differs from the one it had.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stddef.h>
#include <stdint.h>

#include "vc.h"

namespace vc {

// Reduction rules switched on for a node (bit set = rule on).
enum : int32_t {
  kRuleDeg1 = 1,
  kRuleTri = 2,
  kRuleHigh = 4,
  kPruneEdges = 8,
  kRulesAll = 15,
};

constexpr int32_t kNoRow = 0x7FFFFFFF;  // err_row of a graph that passed every check

// Control words of one launch, each on its own 128-byte line so unrelated atomics never share
// a line.
enum CounterSlot : int {
  kQCount = 0,     // int32: worklist entries reserved by producers and not yet by consumers
  kQHead = 1,      // uint64: next consumer ticket
  kQTail = 2,      // uint64: next producer ticket
  kWork = 3,       // int32: sub-trees not finished: unstarted roots, queued or held nodes
  kRootNext = 4,   // int32: next unstarted instance (root ticket)
  kOpen = 5,       // int32: PVC: instances still without a cover (0 stops every workgroup)
  kAbort = 6,      // int32: non-zero stops every workgroup (internal error)
  kError = 7,      // int32: internal error code (1 = stack overflow, 2 = node of no instance)
  kQMaxCount = 8,  // int32: largest worklist count seen by a producer
  kStopReason = 9, // int32: why the launch was stopped from outside the search (kStop*)
  kNumCounters = 10,
};

// Reasons a launch stops before its search ends, other than an internal error.
enum : int32_t {
  kStopHost = 1,     // the host asked the context to stop (vc_abort)
  kStopTimeout = 2,  // the call's time limit (vc_options.timeout_ms) ran out
};
constexpr int kCounterStride = 32;  // int32 words per control line (128 bytes)

// Activities of the instrumented traversal (paper §V-D, Fig. 6).
enum Activity : int {
  kActAcquire = 0,  // taking a node: stack pops, worklist dequeues and the wait for work
  kActReduce = 1,   // the reduction rules
  kActBranch = 2,   // max-degree pass and stopping test, removing v_max or N(v_max)
  kActDonate = 3,   // deferring a child: stack pushes and worklist enqueues
  kActOther = 4,    // flags, bound, budget, recording solutions, loading an instance
  kActTotal = 5,    // the whole kernel, per workgroup
  // parts of kActReduce (degree-array kernels only)
  kActDeg1 = 6,     // degree-one decisions
  kActTri = 7,      // degree-two-triangle decisions
  kActHigh = 8,     // high-degree decisions
  kActApply = 9,    // removing the decided vertices
  kNumActivities = 10,
};

struct WgStats {
  int64_t nodes;
  int64_t pushes;
  int64_t pops;
  int64_t enqueues;
  int64_t dequeues;
  int32_t max_depth;
  int32_t instances;  // instances this workgroup loaded (roots and switches)
  int64_t cycles[kNumActivities];
};

// One instance of a batch (device memory, read-only during a launch). The instances of one
// launch form a contiguous slice of the batch; vtx_first / ent_first number their vertices and
// CSR entries consecutively across that slice (the index spaces of the prepare and finalize
// kernels, and the bitset kernels' adjacency rows).
struct Instance {
  int32_t n;
  int32_t nnz;
  int32_t rp_off;     // first of its n + 1 row pointers in the packed row_ptr
  int32_t vtx_off;    // its cover is covers[vtx_off .. vtx_off + n) (the caller's packing)
  int64_t ci_off;     // first of its nnz neighbour ids in the packed col_idx
  int64_t ent_first;  // launch-local number of its first CSR entry
  int32_t vtx_first;  // launch-local number of its first vertex
  int32_t k;          // PVC parameter (>= 0)
};

// Per-instance search state and results (device memory). `best` and `state` share one
// aligned 64-bit word, read with a single load at every search-tree node.
enum : int32_t {
  kInstFound = 1,        // PVC: a cover of size <= k has been recorded
  kInstOutOfBudget = 2,  // the instance used up its node budget
};
struct InstState {
  int32_t best;         // MVC: best cover size recorded (the greedy's first); PVC: size found
  int32_t state;        // kInstFound | kInstOutOfBudget
  int32_t err_row;      // first CSR row found to break the format, kNoRow if none
  int32_t lock;         // MVC: held while a workgroup writes the instance's cover
  int32_t greedy;       // MVC: size of the greedy cover
  int32_t uncovered;    // CSR entries the recorded cover leaves uncovered (finalize)
  int32_t cover_count;  // vertices in the recorded cover (finalize)
  int32_t pad;
  int64_t nodes;        // search-tree nodes visited on this instance
};

// Largest batch a launch takes: a bitset node packs its instance with the pending vertex.
constexpr int32_t kMaxLaunchInstances = 1 << 22;

struct DevResult;

// Everything a kernel needs; passed by value.
struct Params {
  int32_t num_inst;     // instances of this launch (a contiguous slice of the batch)
  int32_t stride;       // int32 words per stored node
  int32_t n_max;        // largest n of this launch
  int32_t rules;
  const Instance* inst;
  InstState* ist;
  int32_t* work;        // per instance: sub-trees not finished (root, queued, held). Kept apart
                        // from InstState: its atomics would slow the per-node header loads
  const int32_t* __restrict__ rp_all;
  const int32_t* __restrict__ ci_all;
  int32_t* payload;     // worklist node storage: q_cap * stride
  uint32_t* seq;        // worklist slot tickets: q_cap
  int32_t* ctr;         // control lines: kNumCounters * kCounterStride
  int32_t* stacks;      // per-workgroup stacks: num_wg * depth_cap * stride
  uint8_t* covers;      // packed covers, one n_i-byte cover per instance
  WgStats* wg_stats;    // num_wg
  DevResult* res;       // launch result block: every workgroup adds its statistics at exit
  int64_t node_budget;  // per instance; 0 = none
  int64_t budget_chunk; // nodes a workgroup visits between two reports to its instance
  uint32_t q_cap;       // power of two, >= q_threshold + 2 * num_wg
  uint32_t q_threshold; // donate while count < threshold (0 = never)
  int32_t depth_cap;
  int32_t num_wg;
  uint64_t* bits;       // bitset kernels: adjacency rows, words per launch-local vertex
  int32_t words;        // bitset kernels: words per row of this launch; 0 = degree arrays
  int32_t rp_lds;       // degree-array kernels: 1 = copy the instance's row_ptr into LDS after
                        // the node, 2 = its col_idx too (after row_ptr); 0 = neither
  int32_t nnz_max;      // largest nnz of this launch (sizes the LDS copy of col_idx)
  int32_t* gnodes;      // degree-array kernels with the node in device memory: one stride-word
                        // slot per workgroup (nullptr: the node lives in LDS)
  int32_t stack_lds;    // bitset kernels: 1 = each workgroup's stack ring lives in LDS after the
                        // adjacency matrix (depth_cap nodes), 0 = in `stacks`
  int32_t pvc;          // 1: PVC (instances stop once answered), 0: MVC
  int32_t start_depth;  // > 0: StackOnly traversal of instance 0 from this depth; 0: hybrid
  // Watchdog: a host-pinned word that workgroup 0 reads every few tens of microseconds of the
  // device's constant-rate clock (non-zero stops the launch; nullptr: none), and a time limit
  // in ticks of that clock, measured by every workgroup from its own start (0: none).
  const int32_t* host_abort;
  int32_t abort_base;   // the host word's value when the call began; any other value stops
  uint64_t timeout_ticks;
};

// Degree-array node, stored and in LDS: deg[0..n_i), s at n_i, pending vertex at n_i + 1, the
// instance (launch-local index) in the last word. stride >= n_max + 3, a multiple of 64.
inline int32_t array_stride(int32_t n_max) {
  return static_cast<int32_t>((static_cast<int64_t>(n_max) + 3 + 63) / 64 * 64);
}

// LDS words that hold a staged row_ptr (n_max + 1 entries, padded to 16 bytes).
__host__ __device__ inline size_t rp_lds_words(int32_t n_max) { return (static_cast<size_t>(n_max) + 1 + 3) / 4 * 4; }

// Dynamic LDS of a degree-array kernel: the node (stride words), then row_ptr if staged
// (rp_lds >= 1), then col_idx if staged (rp_lds == 2).
inline size_t node_lds_bytes(int32_t stride, int32_t n_max, int32_t rp_lds, int64_t nnz_max) {
  size_t words = static_cast<size_t>(stride);
  if (rp_lds >= 1) words += rp_lds_words(n_max);
  if (rp_lds == 2) words += (static_cast<size_t>(nnz_max) + 3) / 4 * 4;
  return words * 4;
}

// Launch-wide result block written by the finalize kernel and copied to the host once.
struct DevResult {
  int32_t aborted;
  int32_t error;
  int32_t max_depth;
  int32_t q_max_count;
  int32_t active_wgs;   // workgroups that took any work (only they add their statistics)
  int32_t stop_reason;  // kStopHost / kStopTimeout, 0 if the launch was not stopped from outside
  int64_t nodes;
  int64_t wg_nodes_max;
  int64_t wg_nodes_min;
  int64_t pushes;
  int64_t pops;
  int64_t enqueues;
  int64_t dequeues;
  int64_t instances;
  int64_t cycles[kNumActivities];
};

// Kernel launchers. All run on `stream`; they return the HIP status of the launch itself.
// `vertices` / `entries` are totals over the launch's instances (sum of n, sum of nnz).

// vc_device.hip
// Reset the launch's control words, result block and worklist tickets, and validate every CSR.
hipError_t launch_prepare(const Params& p, DevResult* res, int64_t vertices, int64_t entries,
                          hipStream_t stream);
hipError_t launch_greedy(const Params& p, int32_t wg_size, hipStream_t stream);
int greedy_grid(const Params& p);
hipError_t launch_traverse(bool pvc, bool prof, const Params& p, int32_t wg_size,
                           hipStream_t stream);
hipError_t launch_finalize(const Params& p, int64_t vertices, int64_t entries, DevResult* res,
                           hipStream_t stream);
hipError_t launch_reduce(const Params& p, int32_t wg_size, int32_t* deg, int32_t* s,
                         int64_t bound, hipStream_t stream);
hipError_t traverse_occupancy(bool pvc, bool prof, bool global_node, int32_t rp_lds,
                              int32_t wg_size, size_t lds_bytes, int* blocks_per_cu);
hipError_t set_lds_limit(size_t lds_bytes);
hipError_t launch_max_greedy(const Params& p, int32_t* out, hipStream_t stream);

// vc_bitset.hip: graphs of at most kMaxBitsetN vertices
constexpr int kMaxBitsetN = 512;
constexpr int kMaxBitsetWords = 8;  // ceil(kMaxBitsetN / 64)
// Largest n that takes the bitset kernels by default. Wider bitsets (5 to 8 words) hold so many
// registers that fewer wavefronts stay resident: they were up to 2.3 times faster than the
// degree-array kernels on searches of ~20,000 nodes, slower on 10^5-10^6 nodes and on batches
// and request streams of graphs settled near the root, so they are used only on request.
constexpr int kAutoBitsetN = 256;
hipError_t launch_bitset_greedy(const Params& p, hipStream_t stream);
hipError_t launch_bitset_traverse(bool pvc, bool prof, const Params& p, hipStream_t stream);
hipError_t launch_bitset_reduce(const Params& p, int32_t* deg, int32_t* s, int64_t bound,
                                hipStream_t stream);
// Resident workgroups per CU of a bitset traversal launch with `lds` bytes of dynamic LDS.
hipError_t bitset_occupancy(int words, bool pvc, bool prof, size_t lds, int* blocks_per_cu);
// Dynamic LDS of the bitset kernels: the adjacency matrix (and, for a traversal launch with
// stack_lds, the stack ring after it).
size_t bitset_lds_bytes(int n_max, int words);
size_t bitset_traverse_lds_bytes(const Params& p);
int bitset_stride(int words);

// vc_host.cpp: the device a context runs on.
int context_device(const vc_ctx* ctx);
// vc_host.cpp: vc_pvc_device with every device buffer carved from `ws` (`bytes` long) and host
// staging limited to the context's pinned buffer: no device, pinned or stream allocation.
int pvc_device_in(vc_ctx* ctx, const vc_graph* g, int32_t k, const vc_options* opts, void* ws,
                  size_t bytes, int32_t* yes_out, int32_t* size_out, uint8_t* cover_dev,
                  vc_stats* stats);
// vc_noalloc.hip: resolve the device address of the no-allocation scratch on `device` (current),
// once per device.
int noalloc_setup(int device);

}  // namespace vc
