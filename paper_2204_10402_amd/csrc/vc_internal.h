// vc_internal.h -- shared between the device code (vc_device.hip) and the host runtime
// (vc_host.cpp). Not part of the public ABI.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stddef.h>
#include <stdint.h>

namespace vc {

// Reduction rules switched on for a node (bit set = rule on).
enum : int32_t {
  kRuleDeg1 = 1,
  kRuleTri = 2,
  kRuleHigh = 4,
  kPruneEdges = 8,
  kRulesAll = 15,
};

// Control words, each on its own 128-byte line so unrelated atomics never share a line.
enum CounterSlot : int {
  kQCount = 0,    // int32: worklist entries reserved by producers and not yet by consumers
  kQHead = 1,     // uint64: next consumer ticket
  kQTail = 2,     // uint64: next producer ticket
  kWork = 3,      // int32: sub-trees in the worklist or being walked by a workgroup
  kBestKey = 4,   // uint64: (best cover size << 32) | index of the cover buffer holding it
  kFound = 5,     // int32: PVC: 1 + index of the workgroup that found a cover, else 0
  kAbort = 6,     // int32: non-zero stops every workgroup (budget, internal error)
  kError = 7,     // int32: internal error code (1 = stack overflow)
  kNodes = 8,     // uint64: nodes counted against the budget
  kErrRow = 9,    // int32: first CSR row that breaks the format, INT32_MAX if none
  kEdges0 = 10,   // int32: |E| of the input graph (sum of degrees / 2)
  kQMaxCount = 11,// int32: largest worklist count seen by a producer
  kNumCounters = 12,
};
constexpr int kCounterStride = 32;  // int32 words per control line (128 bytes)

// Activities of the instrumented traversal (paper §V-D, Fig. 6).
enum Activity : int {
  kActAcquire = 0,  // taking a node: stack pops, worklist dequeues and the wait for work
  kActReduce = 1,   // the reduction rules
  kActBranch = 2,   // max-degree pass and stopping test, removing v_max or N(v_max)
  kActDonate = 3,   // deferring a child: stack pushes and worklist enqueues
  kActOther = 4,    // flags, bound, budget, recording solutions
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
  int32_t pad;
  int64_t cycles[kNumActivities];
};

// Everything a search kernel needs; passed by value.
struct Params {
  int32_t n;
  int32_t stride;       // int32 words per stored node: deg[n], s, pending, padding (mult. of 64)
  int32_t nnz;
  int32_t rules;
  const int32_t* __restrict__ rp;
  const int32_t* __restrict__ ci;
  int32_t* payload;     // worklist node storage: cap * stride
  uint32_t* seq;        // worklist slot tickets: cap
  int32_t* ctr;         // control lines: kNumCounters * kCounterStride
  int32_t* stacks;      // per-workgroup stacks: num_wg * depth_cap * stride
  uint8_t* covers;      // cover buffers: (num_wg + 1) * cover_stride; the last is the greedy's
  WgStats* wg_stats;    // num_wg
  int64_t k;            // PVC parameter
  int64_t node_budget;  // 0 = none
  int64_t budget_chunk; // nodes a workgroup visits between two reports to the budget counter
  uint32_t q_cap;       // power of two
  uint32_t q_threshold; // donate while count < threshold (0 = never)
  int32_t depth_cap;
  int32_t num_wg;
  int32_t cover_stride;
  int32_t greedy_slot;  // cover buffer index of the greedy's cover
  uint64_t* bits;       // bitset kernels: adjacency rows, n * words 64-bit words
  int32_t words;        // bitset kernels: 64-bit words per row; 0 selects the degree-array kernels
  int32_t rp_lds;       // degree-array kernels: copy row_ptr into LDS after the node
};

// Dynamic LDS of a degree-array kernel: the node (stride words), then row_ptr if staged.
inline size_t node_lds_bytes(int32_t stride, int32_t n, bool rp_lds) {
  const size_t node = static_cast<size_t>(stride) * 4;
  return rp_lds ? node + ((static_cast<size_t>(n) + 1) * 4 + 15) / 16 * 16 : node;
}

// Result block written by the finalize kernel and copied to the host once.
struct DevResult {
  int32_t err_row;
  int32_t edges0;
  int32_t size;
  int32_t yes;
  int32_t greedy;
  int32_t aborted;
  int32_t error;
  int32_t uncovered;    // edges with no endpoint in the returned cover
  int32_t cover_count;  // vertices in the returned cover
  int32_t max_depth;
  int32_t q_max_count;
  int32_t pad;
  int64_t nodes;
  int64_t wg_nodes_max;
  int64_t wg_nodes_min;
  int64_t pushes;
  int64_t pops;
  int64_t enqueues;
  int64_t dequeues;
  int64_t cycles[kNumActivities];
};

// Kernel launchers (vc_device.hip). All run on `stream`; they return the HIP status of the
// launch itself.
hipError_t launch_init(const Params& p, DevResult* res, hipStream_t stream);
hipError_t launch_prepare(const Params& p, hipStream_t stream);
hipError_t launch_greedy(const Params& p, int32_t wg_size, DevResult* res, hipStream_t stream);
hipError_t launch_traverse(bool pvc, bool prof, const Params& p, int32_t wg_size,
                           hipStream_t stream);
hipError_t launch_finalize(bool pvc, const Params& p, uint8_t* cover_out, DevResult* res,
                           hipStream_t stream);
hipError_t launch_reduce(const Params& p, int32_t wg_size, int32_t* deg, int32_t* s,
                         int64_t bound, DevResult* res, hipStream_t stream);

// Bitset kernels (vc_bitset.hip), graphs of at most kMaxBitsetN vertices.
constexpr int kMaxBitsetN = 256;
hipError_t launch_bitset_pack(const Params& p, hipStream_t stream);
hipError_t launch_bitset_greedy(const Params& p, DevResult* res, hipStream_t stream);
hipError_t launch_bitset_traverse(bool pvc, bool prof, const Params& p, hipStream_t stream);
hipError_t launch_bitset_reduce(const Params& p, int32_t* deg, int32_t* s, int64_t bound,
                                DevResult* res, hipStream_t stream);
hipError_t bitset_occupancy(int words, bool pvc, bool prof, int n, int* blocks_per_cu);
size_t bitset_lds_bytes(int n, int words);
int bitset_stride(int words);

// Resident workgroups per CU for the traversal kernel at this size (occupancy API).
hipError_t traverse_occupancy(bool pvc, bool prof, int32_t wg_size, size_t lds_bytes,
                              int* blocks_per_cu);
hipError_t set_lds_limit(size_t lds_bytes);

}  // namespace vc
