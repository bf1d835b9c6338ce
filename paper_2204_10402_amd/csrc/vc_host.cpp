// vc_host.cpp -- host runtime of libvc.so: contexts, workspace, launch sizing and the C ABI
// declared in include/vc.h. Every step of the search runs in the HIP kernels of vc_device.hip
// and vc_bitset.hip; this file only checks arguments, lays out a batch, sizes and allocates
// device memory, queues the kernels on the context stream and copies the small result blocks
// back. A single-graph call is a batch of one.

#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "vc.h"
#include "vc_internal.h"

namespace {

struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
};

}  // namespace

struct vc_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  hipDeviceProp_t prop{};
  size_t lds_limit_set = 0;
  // meta: the instance table, per-instance state, work counters and result blocks of a call,
  // mirrored in pinned host memory so that each call makes one copy in and one copy out
  DevBuf rp, ci, meta, payload, seq, ctr, stacks, covers, wg_stats, scratch, bits, gnodes;
  void* pinned = nullptr;
  size_t pinned_bytes = 0;
  std::vector<hipEvent_t> ev;  // two per launch group
  int32_t last_num_wg = 0;     // grid of the last traversal launch (its WgStats are kept)
  std::string last_error;
  // occupancy-API answers: (kernel family, pvc, profiled, workgroup size, words, LDS bytes)
  std::map<std::tuple<int, int, int, int, int, size_t>, int> occupancy;
  // autotuner choices: (bitset words, pvc, flags, log2 n_max, log2 instances) -> knobs
  std::map<std::tuple<int, int, int, int, int>, std::tuple<int, int, int>> tuned;
  // A second context (own stream, worklist, counters, stacks) on which a batch's degree-array
  // launch runs while its bitset launches run on this one; created on first use.
  vc_ctx* aux = nullptr;
  vc_ctx* stats_src = nullptr;  // the context holding the last traversal's per-workgroup stats
  // vc_abort: a host-pinned word, mapped for the device; vc_abort increments it and a launch
  // stops when it differs from its value at the start of the call
  int32_t* abort_host = nullptr;
  const int32_t* abort_dev = nullptr;
  int64_t clock_khz = 0;  // rate of the device's constant clock (s_memrealtime), for timeouts
  // During a call of a caller-workspace form: the workspace every device buffer is carved from
  // (no allocation), and whether host staging may use ordinary host memory beyond `pinned`.
  struct Workspace {
    char* base = nullptr;
    size_t bytes = 0;
    size_t used = 0;
    bool host_heap = true;
  };
  Workspace* ws = nullptr;
  std::vector<char> host_heap;
};

namespace {

// Launch groups of one call at most: bitset words 1 to 8, then degree arrays.
constexpr size_t kMaxGroups = vc::kMaxBitsetWords + 1;
// Pinned staging made with a context (grown by the allocating forms as batches need).
constexpr size_t kPinnedStart = size_t(1) << 20;

using vc::DevResult;
using vc::Instance;
using vc::InstState;
using vc::Params;

int fail(vc_ctx* ctx, int code, const std::string& msg) {
  if (ctx) ctx->last_error = msg;
  return code;
}

int hip_fail(vc_ctx* ctx, hipError_t e, const char* what) {
  return fail(ctx, VC_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define VC_HIP(ctx, call)                                   \
  do {                                                      \
    hipError_t e_ = (call);                                 \
    if (e_ != hipSuccess) return hip_fail((ctx), e_, #call); \
  } while (0)

// Take `bytes` for b from the caller's workspace (a caller-workspace call): keep b's region if
// it is large enough, else carve the next one (256-byte aligned).
int carve(vc_ctx* ctx, DevBuf& b, size_t bytes) {
  vc_ctx::Workspace& w = *ctx->ws;
  if (b.ptr && b.bytes >= bytes) return VC_OK;
  const size_t off = (w.used + 255) / 256 * 256;
  if (off > w.bytes || bytes > w.bytes - off)
    return fail(ctx, VC_ERR_NO_MEMORY,
                "the workspace of " + std::to_string(w.bytes) + " bytes is too small (" +
                    std::to_string(off + bytes) + " bytes needed so far; see vc_workspace_bytes)");
  b.ptr = w.base + off;
  b.bytes = bytes;
  w.used = off + bytes;
  return VC_OK;
}

// Grow-only device buffer (from the caller's workspace during a caller-workspace call).
int ensure(vc_ctx* ctx, DevBuf& b, size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (ctx->ws) return carve(ctx, b, bytes);
  if (b.bytes >= bytes) return VC_OK;
  if (b.ptr) {
    hipError_t e = hipFree(b.ptr);
    b.ptr = nullptr;
    b.bytes = 0;
    if (e != hipSuccess) return hip_fail(ctx, e, "hipFree");
  }
  hipError_t e = hipMalloc(&b.ptr, bytes);
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {
    (void)hipGetLastError();
    return fail(ctx, VC_ERR_NO_MEMORY,
                "device allocation of " + std::to_string(bytes) + " bytes failed");
  }
  if (e != hipSuccess) return hip_fail(ctx, e, "hipMalloc");
  b.bytes = bytes;
  return VC_OK;
}

// Grow-only pinned host buffer (the mirror of the meta buffer).
int ensure_pinned(vc_ctx* ctx, size_t bytes) {
  if (ctx->pinned_bytes >= bytes) return VC_OK;
  if (ctx->pinned) {
    hipError_t e = hipHostFree(ctx->pinned);
    ctx->pinned = nullptr;
    ctx->pinned_bytes = 0;
    if (e != hipSuccess) return hip_fail(ctx, e, "hipHostFree");
  }
  hipError_t e = hipHostMalloc(&ctx->pinned, bytes, hipHostMallocDefault);
  if (e != hipSuccess) {
    ctx->pinned = nullptr;
    return hip_fail(ctx, e, "hipHostMalloc");
  }
  ctx->pinned_bytes = bytes;
  return VC_OK;
}

// Host staging of `bytes` for a call: the pinned mirror, grown as needed; during a
// caller-workspace call it is not grown: ordinary host memory takes a larger batch, or (the
// no-allocation entry point) the call fails.
int host_staging(vc_ctx* ctx, size_t bytes, char** out) {
  if (!ctx->ws) {
    int rc = ensure_pinned(ctx, bytes);
    if (rc) return rc;
    *out = static_cast<char*>(ctx->pinned);
    return VC_OK;
  }
  if (ctx->pinned_bytes >= bytes) {
    *out = static_cast<char*>(ctx->pinned);
    return VC_OK;
  }
  if (!ctx->ws->host_heap)
    return fail(ctx, VC_ERR_NO_MEMORY,
                "the batch needs " + std::to_string(bytes) + " bytes of host staging, more than "
                "the context's " + std::to_string(ctx->pinned_bytes) + " pinned bytes");
  if (ctx->host_heap.size() < bytes) ctx->host_heap.resize(bytes);
  *out = ctx->host_heap.data();
  return VC_OK;
}

// Byte offsets of the meta regions: [Instance m | InstState m | work m | DevResult ng |
// greedy maxima ng] in device memory and its pinned mirror; the mirror also holds the host
// cover staging after them.
struct MetaLayout {
  size_t inst = 0, ist = 0, work = 0, res = 0, gmax = 0, dev_end = 0, cover = 0, host_end = 0;
};

MetaLayout meta_layout(int32_t m, int32_t ng, int64_t cover_bytes) {
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  MetaLayout L;
  L.ist = al(static_cast<size_t>(m) * sizeof(vc::Instance));
  L.work = L.ist + al(static_cast<size_t>(m) * sizeof(vc::InstState));
  L.res = L.work + al(static_cast<size_t>(m) * sizeof(int32_t));
  L.gmax = L.res + al(static_cast<size_t>(ng) * sizeof(vc::DevResult));
  L.dev_end = L.gmax + al(static_cast<size_t>(ng) * sizeof(int32_t));
  L.cover = L.dev_end;
  L.host_end = L.cover + al(static_cast<size_t>(cover_bytes));
  return L;
}

// Fresh per-instance state: nothing rejected yet, no cover, one outstanding sub-tree (the root).
void init_state(vc::InstState* is, int32_t* work, int32_t m) {
  for (int32_t j = 0; j < m; ++j) {
    vc::InstState s{};
    s.err_row = vc::kNoRow;
    s.best = 0x7FFFFFFF;
    s.greedy = -1;
    is[j] = s;
    work[j] = 1;
  }
}

int ensure_events(vc_ctx* ctx, size_t count) {
  while (ctx->ev.size() < count) {
    hipEvent_t e = nullptr;
    VC_HIP(ctx, hipEventCreate(&e));
    ctx->ev.push_back(e);
  }
  return VC_OK;
}

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

uint32_t next_pow2(uint64_t x) {
  uint64_t p = 1;
  while (p < x) p <<= 1;
  return static_cast<uint32_t>(p);
}

int rules_from_flags(int32_t flags) {
  int rules = vc::kRulesAll;
  if (flags & VC_OPT_NO_DEGREE_ONE) rules &= ~vc::kRuleDeg1;
  if (flags & VC_OPT_NO_TRIANGLE) rules &= ~vc::kRuleTri;
  if (flags & VC_OPT_NO_HIGH_DEGREE) rules &= ~(vc::kRuleHigh | vc::kPruneEdges);
  if (flags & VC_OPT_NO_EDGE_PRUNE) rules &= ~vc::kPruneEdges;
  return rules;
}

int check_options(vc_ctx* ctx, const vc_options* o) {
  if (!o) return VC_OK;
  if (o->reserved != 0) return fail(ctx, VC_ERR_INVALID_ARG, "vc_options.reserved must be zero");
  if (o->stack_depth < 0 || o->timeout_ms < 0)
    return fail(ctx, VC_ERR_INVALID_ARG, "stack_depth and timeout_ms must be >= 0");
  if (o->wg_size != 0 && (o->wg_size < 64 || o->wg_size > 1024 || o->wg_size % 64 != 0))
    return fail(ctx, VC_ERR_INVALID_ARG, "wg_size must be 0 or a multiple of 64 in [64, 1024]");
  if (o->num_wg < 0 || o->wl_capacity < 0 || o->wl_threshold < -1 || o->node_budget < 0 ||
      o->grid_share < 0)
    return fail(ctx, VC_ERR_INVALID_ARG, "negative option value");
  const int32_t known = VC_OPT_NO_DEGREE_ONE | VC_OPT_NO_TRIANGLE | VC_OPT_NO_HIGH_DEGREE |
                        VC_OPT_NO_EDGE_PRUNE | VC_OPT_PROFILE | VC_OPT_DEGREE_ARRAYS |
                        VC_OPT_BITSETS | VC_OPT_AUTOTUNE | VC_OPT_STACK_ONLY |
                        VC_OPT_GLOBAL_NODES | VC_OPT_CSR_GLOBAL;
  if ((o->flags & VC_OPT_GLOBAL_NODES) && (o->flags & VC_OPT_BITSETS))
    return fail(ctx, VC_ERR_INVALID_ARG, "VC_OPT_GLOBAL_NODES and VC_OPT_BITSETS exclude each other");
  if (o->start_depth < 0 || o->start_depth > 24)
    return fail(ctx, VC_ERR_INVALID_ARG, "start_depth must be in [0, 24]");
  if (o->start_depth && !(o->flags & VC_OPT_STACK_ONLY))
    return fail(ctx, VC_ERR_INVALID_ARG, "start_depth needs VC_OPT_STACK_ONLY");
  if (o->flags & ~known) return fail(ctx, VC_ERR_INVALID_ARG, "unknown option flag");
  if ((o->flags & VC_OPT_DEGREE_ARRAYS) && (o->flags & VC_OPT_BITSETS))
    return fail(ctx, VC_ERR_INVALID_ARG, "VC_OPT_DEGREE_ARRAYS and VC_OPT_BITSETS exclude each other");
  return VC_OK;
}

int check_graph_args(vc_ctx* ctx, const vc_graph* g) {
  if (!g) return fail(ctx, VC_ERR_INVALID_ARG, "graph is NULL");
  if (g->n < 0 || g->nnz < 0) return fail(ctx, VC_ERR_INVALID_ARG, "negative n or nnz");
  if (!g->row_ptr) return fail(ctx, VC_ERR_INVALID_ARG, "row_ptr is NULL");
  if (g->nnz > 0 && !g->col_idx) return fail(ctx, VC_ERR_INVALID_ARG, "col_idx is NULL");
  if (g->n == 0 && g->nnz != 0) return fail(ctx, VC_ERR_INVALID_GRAPH, "n = 0 but nnz > 0");
  return VC_OK;
}

struct Plan {
  int32_t wg_size = 0;
  int32_t num_wg = 0;
  int32_t stride = 0;
  uint32_t cap = 0;
  uint32_t threshold = 0;
  size_t lds = 0;
  int32_t rp_lds = 0;       // degree-array kernels: 1 = row_ptr staged in LDS, 2 = the CSR
  int32_t global_node = 0;  // degree-array kernels: the node lives in device memory
};

// Resident workgroups per CU, from the occupancy API, remembered per context.
int occupancy(vc_ctx* ctx, int words, bool pvc, bool prof, int ws, size_t lds, int n_max,
              int* out, bool global_node = false, int rp_lds = 0) {
  const int family = words ? 1 : (global_node ? 2 : 3 + rp_lds);
  const auto key = std::make_tuple(family, pvc ? 1 : 0, prof ? 1 : 0, ws, words, lds);
  const auto it = ctx->occupancy.find(key);
  if (it != ctx->occupancy.end()) {
    *out = it->second;
    return VC_OK;
  }
  if (words) VC_HIP(ctx, vc::bitset_occupancy(words, pvc, prof, lds, out));
  else VC_HIP(ctx, vc::traverse_occupancy(pvc, prof, global_node, rp_lds, ws, lds, out));
  ctx->occupancy[key] = *out;
  return VC_OK;
}

// Kernel family of a graph: bitset kernels with ceil(n/64) words up to kAutoBitsetN vertices
// (up to kMaxBitsetN when the caller asks for them), else degree arrays (0).
int choose_words(vc_ctx* ctx, int32_t n, int32_t flags, int32_t* words) {
  const bool force_bits = flags & VC_OPT_BITSETS;
  const bool force_arrays = flags & (VC_OPT_DEGREE_ARRAYS | VC_OPT_GLOBAL_NODES);
  if (force_bits && n > vc::kMaxBitsetN)
    return fail(ctx, VC_ERR_INVALID_ARG, "VC_OPT_BITSETS needs n <= 512");
  const bool bits = force_bits || (!force_arrays && n <= vc::kAutoBitsetN);
  *words = bits ? (std::max(n, 1) + 63) / 64 : 0;
  return VC_OK;
}

void size_worklist(Plan& pl, const vc_options* o, uint64_t min_cap);

// Workgroup size and count for one launch (paper §IV-E, adapted): a power-of-two workgroup of
// about n_max/4 threads; as many workgroups as can be resident at once, fewer if their stacks
// do not fit in device memory (size_stacks).
int plan_launch(vc_ctx* ctx, bool pvc, int32_t n_max, int64_t nnz_max, int32_t words,
                const vc_options* o, Plan& pl) {
  const bool prof = o && (o->flags & VC_OPT_PROFILE);
  const int cus = ctx->prop.multiProcessorCount;
  int best_ws = 0, best_occ = 0, rc;
  if (words) {
    // one wavefront per workgroup; the adjacency matrix (n_max * words * 8 bytes) in LDS
    pl.stride = vc::bitset_stride(words);
    pl.lds = vc::bitset_lds_bytes(n_max, words);
    best_ws = 64;
    if (o && o->wg_size && o->wg_size != 64)
      return fail(ctx, VC_ERR_INVALID_ARG, "the bitset kernels use 64-thread workgroups");
    if ((rc = occupancy(ctx, words, pvc, prof, 64, pl.lds, n_max, &best_occ))) return rc;
  } else {
    pl.stride = vc::array_stride(n_max);
    pl.lds = vc::node_lds_bytes(pl.stride, n_max, 0, 0);
    const size_t lds_cap = static_cast<size_t>(ctx->prop.maxSharedMemoryPerMultiProcessor);
    // Selection rule (§IV-E, adapted): the node stays in LDS while it fits there with room
    // to spare; larger graphs (or VC_OPT_GLOBAL_NODES) keep it in device memory.
    pl.global_node = ((o && (o->flags & VC_OPT_GLOBAL_NODES)) || pl.lds + 1024 > lds_cap) ? 1 : 0;
    if (pl.global_node) pl.lds = 0;
    const size_t lds_rp = vc::node_lds_bytes(pl.stride, n_max, 1, 0);
    const size_t lds_csr = vc::node_lds_bytes(pl.stride, n_max, 2, nnz_max);
    const bool csr_fits = !pl.global_node && !(o && (o->flags & VC_OPT_CSR_GLOBAL)) &&
                          lds_csr + 1024 <= lds_cap;
    const size_t lds_max = pl.global_node ? 0
                           : csr_fits     ? lds_csr
                                          : (lds_rp + 1024 <= lds_cap ? lds_rp : pl.lds);
    if (lds_max > 65536 && ctx->lds_limit_set < lds_max) {
      VC_HIP(ctx, vc::set_lds_limit(lds_max));
      ctx->lds_limit_set = lds_max;
    }
    if (o && o->wg_size) {
      best_ws = o->wg_size;
    } else {
      // The paper's rule (§IV-E) admits any power of two between the size that fills the CU
      // and min(1024, n). A node's passes are chains of dependent LDS and L2 accesses, so the
      // time per node falls with more wavefronts per node: take about n/4 threads (four
      // vertices per thread per pass), as a power of two in [64, 1024].
      int ws = 64;
      while (ws < 1024 && ws * 2 <= std::max(n_max, 1) / 4) ws *= 2;
      best_ws = ws;
    }
    if ((rc = occupancy(ctx, 0, pvc, prof, best_ws, pl.lds, n_max, &best_occ,
                        pl.global_node != 0)))
      return rc;
    // Keep row_ptr in LDS too when that costs no resident workgroup.
    if (!pl.global_node && lds_rp + 1024 <= lds_cap) {
      int occ_rp = 0;
      if ((rc = occupancy(ctx, 0, pvc, prof, best_ws, lds_rp, n_max, &occ_rp, false, 1))) return rc;
      if (occ_rp == best_occ) {
        pl.rp_lds = 1;
        pl.lds = lds_rp;
      }
    }
    // And the column indices when that keeps at least half of the resident workgroups: a
    // rule pass is a chain of dependent row walks, which then read LDS instead of L2 or HBM.
    if (csr_fits) {
      int occ_csr = 0;
      if ((rc = occupancy(ctx, 0, pvc, prof, best_ws, lds_csr, n_max, &occ_csr, false, 2)))
        return rc;
      if (occ_csr >= 1 && 2 * occ_csr >= best_occ) {
        pl.rp_lds = 2;
        pl.lds = lds_csr;
        best_occ = occ_csr;
      }
    }
  }
  if (best_occ < 1)
    return fail(ctx, VC_ERR_INVALID_ARG, "traversal kernel cannot be resident at this size");
  pl.wg_size = best_ws;
  pl.num_wg = best_occ * cus;
  // Untuned, at most eight one-wavefront workgroups per CU: idle workgroups beyond that only
  // add polling on the worklist counters in small searches. The autotuner also tries 12 and 16,
  // which large searches use well (the hard MVC batch: 400 -> 460 million nodes/s at 16).
  if (words && !(o && o->num_wg > 0)) pl.num_wg = std::min(pl.num_wg, 8 * cus);
  if (o && o->grid_share > 0) pl.num_wg = std::max(1, pl.num_wg / o->grid_share);
  if (o && o->num_wg > 0) pl.num_wg = std::min(pl.num_wg, o->num_wg);

  size_worklist(pl, o, 4096);
  return VC_OK;
}

// Worklist capacity and donation threshold (§IV-A) for pl.num_wg workgroups, at least
// `min_cap` entries unless the caller chose the capacity. A producer only reserves a slot after
// reading fewer than `threshold` reserved entries; at most num_wg producers can be past that
// check at once, and consumers giving back a lost reservation can hide at most num_wg more, so
// threshold + 2 * num_wg <= cap keeps every reservation inside the ring.
void size_worklist(Plan& pl, const vc_options* o, uint64_t min_cap) {
  uint64_t cap = o && o->wl_capacity ? static_cast<uint64_t>(o->wl_capacity)
                                     : std::max<uint64_t>(8ull * pl.num_wg, min_cap);
  cap = std::max<uint64_t>(cap, 4ull * pl.num_wg);
  pl.cap = next_pow2(cap);
  uint64_t thr;
  if (o && o->wl_threshold == -1) thr = 0;
  else if (o && o->wl_threshold > 0) thr = static_cast<uint64_t>(o->wl_threshold);
  else thr = std::max<uint64_t>(64, static_cast<uint64_t>(pl.num_wg) / 4);
  thr = std::min<uint64_t>(thr, pl.cap - 2ull * static_cast<uint64_t>(pl.num_wg));
  pl.threshold = static_cast<uint32_t>(thr);
}

// A caller-workspace call: halve the grid, and with it the worklist ring, until one launch's
// buffers -- worklist slots and tickets, workgroup statistics, adjacency rows, node slots and
// at least one workgroup's stack of `depth` entries -- fit in what is left of the workspace.
// (size_stacks then shrinks the grid further if all stacks do not fit.)
int fit_plan_to_workspace(vc_ctx* ctx, Plan& pl, const vc_options* o, int32_t words,
                          int64_t vertices, int64_t count, int32_t depth) {
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  const size_t stride_b = static_cast<size_t>(pl.stride) * sizeof(int32_t);
  auto need = [&](const Plan& q) {
    size_t b = al(q.cap * stride_b) + al(q.cap * sizeof(uint32_t)) +
               al(static_cast<size_t>(q.num_wg) * sizeof(vc::WgStats)) +
               al(static_cast<size_t>(depth) * stride_b);
    if (words) b += al(static_cast<size_t>(vertices) * words * sizeof(uint64_t));
    if (q.global_node)
      b += al(static_cast<size_t>(std::max<int64_t>(q.num_wg, std::min<int64_t>(count, 65535))) *
              stride_b);
    return b;
  };
  const size_t off = (ctx->ws->used + 255) / 256 * 256;
  const size_t left = off < ctx->ws->bytes ? ctx->ws->bytes - off : 0;
  while (need(pl) > left && pl.num_wg > 1) {
    pl.num_wg = (pl.num_wg + 1) / 2;
    size_worklist(pl, o, 64);
  }
  if (need(pl) > left)
    return fail(ctx, VC_ERR_NO_MEMORY,
                "the workspace of " + std::to_string(ctx->ws->bytes) +
                    " bytes cannot hold one workgroup's worklist share and stack (" +
                    std::to_string(off + need(pl)) + " bytes needed)");
  return VC_OK;
}

// Shrink the grid so that num_wg stacks of depth_cap nodes fit in free device memory
// (§IV-E: the stacks bound the number of workgroups), then make sure they are allocated.
int size_stacks(vc_ctx* ctx, Plan& pl, int32_t depth_cap) {
  const size_t per_wg = static_cast<size_t>(depth_cap) * pl.stride * sizeof(int32_t);
  if (per_wg * static_cast<size_t>(pl.num_wg) <= ctx->stacks.bytes) return VC_OK;
  size_t avail = 0;
  if (ctx->ws) {
    // what is left of the caller's workspace
    const size_t off = (ctx->ws->used + 255) / 256 * 256;
    avail = off < ctx->ws->bytes ? ctx->ws->bytes - off : 0;
  } else {
    size_t free_b = 0, total_b = 0;
    VC_HIP(ctx, hipMemGetInfo(&free_b, &total_b));
    avail = ctx->stacks.bytes + (free_b > (size_t(1) << 30) ? free_b - (size_t(1) << 30) : 0);
  }
  const size_t fit = per_wg ? avail / per_wg : static_cast<size_t>(pl.num_wg);
  if (fit < 1)
    return fail(ctx, VC_ERR_NO_MEMORY, "no room for a single workgroup stack of " +
                                           std::to_string(per_wg) + " bytes");
  if (fit < static_cast<size_t>(pl.num_wg)) pl.num_wg = static_cast<int32_t>(fit);
  return ensure(ctx, ctx->stacks, per_wg * static_cast<size_t>(pl.num_wg));
}

double ms_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// A batch whose packed CSR is already in device memory.
struct BatchIn {
  int32_t count = 0;
  const int32_t* n = nullptr;    // host
  const int32_t* nnz = nullptr;  // host
  const int32_t* k = nullptr;    // host, PVC
  const int32_t* rp = nullptr;   // device, packed
  const int32_t* ci = nullptr;   // device, packed
};

// Per-instance results in the caller's order (host arrays; any may be null).
struct BatchOut {
  int32_t* status = nullptr;
  int32_t* size = nullptr;
  int32_t* yes = nullptr;
  int64_t* nodes = nullptr;
  uint8_t* cover_host = nullptr;  // sum of n bytes
  uint8_t* cover_dev = nullptr;   // sum of n bytes (device)
  vc_stats* stats = nullptr;
  bool single = false;            // a batch of one: its status is the call's status
};

// Instances of one launch: a contiguous slice [begin, end) of the sorted instance table.
struct Group {
  int32_t words = 0;
  int32_t begin = 0, end = 0;
  int32_t n_max = 0;
  int32_t nnz_max = 0;
  int32_t k_max = 0;
  int64_t vertices = 0, entries = 0;
  Plan pl;
  int32_t depth_cap = 0;
};

// Check the host side of a batch: sizes, and that the packed offsets fit their types.
int check_batch(vc_ctx* ctx, const BatchIn& b, bool pvc, int64_t* total_rp, int64_t* total_n,
                int64_t* total_nnz) {
  if (b.count < 0) return fail(ctx, VC_ERR_INVALID_ARG, "negative batch count");
  if (b.count > 0 && (!b.n || !b.nnz)) return fail(ctx, VC_ERR_INVALID_ARG, "n or nnz is NULL");
  if (pvc && b.count > 0 && !b.k) return fail(ctx, VC_ERR_INVALID_ARG, "k is NULL");
  int64_t rp = 0, nv = 0, ne = 0;
  for (int32_t i = 0; i < b.count; ++i) {
    if (b.n[i] < 0 || b.nnz[i] < 0)
      return fail(ctx, VC_ERR_INVALID_ARG, "negative n or nnz (instance " + std::to_string(i) + ")");
    if (pvc && b.k[i] < 0)
      return fail(ctx, VC_ERR_INVALID_ARG, "k must be >= 0 (instance " + std::to_string(i) + ")");
    rp += static_cast<int64_t>(b.n[i]) + 1;
    nv += b.n[i];
    ne += b.nnz[i];
  }
  if (rp > 0x7FFFFFFF || nv > 0x7FFFFFFF)
    return fail(ctx, VC_ERR_INVALID_ARG, "batch has more than 2^31 row pointers");
  if (ne > 0x7FFFFFFF) return fail(ctx, VC_ERR_INVALID_ARG, "batch has more than 2^31 CSR entries");
  if (b.count > vc::kMaxLaunchInstances)
    return fail(ctx, VC_ERR_INVALID_ARG, "batch has more than 2^22 graphs");
  if (b.count > 0 && !b.rp) return fail(ctx, VC_ERR_INVALID_ARG, "row_ptr is NULL");
  if (ne > 0 && !b.ci) return fail(ctx, VC_ERR_INVALID_ARG, "col_idx is NULL");
  *total_rp = rp;
  *total_n = nv;
  *total_nnz = ne;
  return VC_OK;
}

std::string bad_row_message(int32_t row) {
  return "CSR row " + std::to_string(row) +
         " breaks the format (bounds, order, self-loop, duplicate or symmetry)";
}

// The whole search for every instance of a batch.
int run_batch(vc_ctx* ctx, const BatchIn& b, bool pvc, const vc_options* o, BatchOut& out,
              std::chrono::steady_clock::time_point t0, int32_t abort_base) {
  int64_t total_rp = 0, total_n = 0, total_nnz = 0;
  int rc = check_batch(ctx, b, pvc, &total_rp, &total_n, &total_nnz);
  if (rc) return rc;
  const int32_t flags = o ? o->flags : 0;
  const bool prof = flags & VC_OPT_PROFILE;
  const bool stack_only = flags & VC_OPT_STACK_ONLY;

  // instance table, sorted by kernel family; graphs without vertices are answered here
  std::vector<int32_t> words(b.count, 0), order;
  order.reserve(b.count);
  for (int32_t i = 0; i < b.count; ++i) {
    if (b.n[i] == 0) {
      if (b.nnz[i] != 0) {
        if (out.single) return fail(ctx, VC_ERR_INVALID_GRAPH, "n = 0 but nnz > 0");
      }
      continue;
    }
    if ((rc = choose_words(ctx, b.n[i], flags, &words[i]))) return rc;
    order.push_back(i);
  }
  std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
    const int32_t kx = words[x] ? words[x] : 99, ky = words[y] ? words[y] : 99;
    return kx < ky;
  });
  std::vector<int64_t> rp_off(b.count), ci_off(b.count), vtx_off(b.count);
  {
    int64_t r = 0, c = 0, v = 0;
    for (int32_t i = 0; i < b.count; ++i) {
      rp_off[i] = r;
      ci_off[i] = c;
      vtx_off[i] = v;
      r += static_cast<int64_t>(b.n[i]) + 1;
      c += b.nnz[i];
      v += b.n[i];
    }
  }
  const int32_t m = static_cast<int32_t>(order.size());
  // groups first (the layout needs their number), then the table straight into pinned memory
  std::vector<Group> groups;
  for (int32_t s = 0; s < m; ++s)
    if (groups.empty() || groups.back().words != words[order[s]]) {
      Group g;
      g.words = words[order[s]];
      g.begin = s;
      groups.push_back(g);
    }
  const int32_t ng = static_cast<int32_t>(groups.size());
  const MetaLayout L = meta_layout(m, ng, out.cover_host ? total_n : 0);
  if ((rc = ensure(ctx, ctx->meta, L.dev_end))) return rc;
  char* host = nullptr;
  if ((rc = host_staging(ctx, L.host_end, &host))) return rc;
  char* dev = static_cast<char*>(ctx->meta.ptr);
  Instance* h_inst = reinterpret_cast<Instance*>(host + L.inst);
  InstState* h_ist = reinterpret_cast<InstState*>(host + L.ist);
  DevResult* h_res = reinterpret_cast<DevResult*>(host + L.res);
  int32_t* h_gmax = reinterpret_cast<int32_t*>(host + L.gmax);
  init_state(h_ist, reinterpret_cast<int32_t*>(host + L.work), m);
  int32_t gcur = -1;
  for (int32_t s = 0; s < m; ++s) {
    const int32_t i = order[s];
    if (gcur < 0 || groups[gcur].words != words[i]) ++gcur;
    Group& g = groups[gcur];
    Instance& in = h_inst[s];
    in = Instance{};
    in.n = b.n[i];
    in.nnz = b.nnz[i];
    in.rp_off = static_cast<int32_t>(rp_off[i]);
    in.vtx_off = static_cast<int32_t>(vtx_off[i]);
    in.ci_off = ci_off[i];
    in.ent_first = g.entries;
    in.vtx_first = static_cast<int32_t>(g.vertices);
    in.k = pvc ? b.k[i] : 0;
    g.end = s + 1;
    g.n_max = std::max(g.n_max, in.n);
    g.nnz_max = std::max(g.nnz_max, in.nnz);
    g.k_max = std::max(g.k_max, std::min(in.k, in.n));
    g.vertices += in.n;
    g.entries += in.nnz;
  }
  hipStream_t st = ctx->stream;
  // A batch with both kernel families runs its degree-array launch on the auxiliary context
  // (first, as the longest) while the bitset launches follow on this one: the two persistent
  // launches share the device instead of queueing behind each other. Not when the caller
  // already runs launches side by side on shares of the grid (vc_options.grid_share).
  const bool use_aux = !stack_only && ng >= 2 && groups.back().words == 0 &&
                       !(o && o->grid_share > 0) && !ctx->ws;
  if (use_aux && !ctx->aux) {
    vc_ctx* a = nullptr;
    if ((rc = vc_create(&a, ctx->device, nullptr)) != VC_OK)
      return fail(ctx, rc, "could not create the auxiliary launch context");
    ctx->aux = a;
  }
  auto lane = [&](int32_t gi) -> vc_ctx* {
    return use_aux && groups[gi].words == 0 ? ctx->aux : ctx;
  };

  if (m > 0) {
    if ((rc = ensure(ctx, ctx->ctr, vc::kNumCounters * vc::kCounterStride * sizeof(int32_t)))) return rc;
    if ((rc = ensure_events(ctx, 4 * static_cast<size_t>(ng) + 4))) return rc;
    if (ctx->aux) {
      // whatever an earlier call left on the auxiliary stream (an error return does not wait
      // for it) finishes before this call's table overwrites the meta buffer
      VC_HIP(ctx, hipEventRecord(ctx->ev[2 * ng + 3], ctx->aux->stream));
      VC_HIP(ctx, hipStreamWaitEvent(st, ctx->ev[2 * ng + 3], 0));
    }
    if (use_aux &&
        (rc = ensure(ctx, ctx->aux->ctr, vc::kNumCounters * vc::kCounterStride * sizeof(int32_t))))
      return rc;
    // one copy in: instance table, fresh per-instance state and work counters
    VC_HIP(ctx, hipMemcpyAsync(dev, host, L.res, hipMemcpyHostToDevice, st));
    if (use_aux) {
      VC_HIP(ctx, hipEventRecord(ctx->ev[2 * ng + 2], st));
      VC_HIP(ctx, hipStreamWaitEvent(ctx->aux->stream, ctx->ev[2 * ng + 2], 0));
    }
  }
  uint8_t* covers = out.cover_dev;
  if (!covers && total_n > 0) {
    if ((rc = ensure(ctx, ctx->covers, static_cast<size_t>(total_n)))) return rc;
    covers = static_cast<uint8_t*>(ctx->covers.ptr);
  }

  // one launch per kernel family, in turn on the context stream
  const Instance* d_inst = reinterpret_cast<const Instance*>(dev + L.inst);
  InstState* d_ist = reinterpret_cast<InstState*>(dev + L.ist);
  int32_t* d_work = reinterpret_cast<int32_t*>(dev + L.work);
  DevResult* d_res = reinterpret_cast<DevResult*>(dev + L.res);
  int32_t* d_greedy = reinterpret_cast<int32_t*>(dev + L.gmax);
  std::vector<Params> params(ng);
  float greedy_ms = 0.f;
  const int cus = ctx->prop.multiProcessorCount;

  // Everything of one launch group up to (and, if `final`, including) the cover check, with
  // the knobs of `go` and, if thr_div > 0, a donation threshold of num_wg / thr_div.
  auto run_group = [&](int32_t gi, const vc_options* go, int thr_div, bool final) -> int {
    Group& g = groups[gi];
    vc_ctx* lc = lane(gi);
    const hipStream_t gst = lc->stream;
    int rc2;
    vc_options shared = go ? *go : vc_options{};
    if (use_aux) {
      // Two launches side by side, each on a share of the co-resident grid; the rest stays free
      // for the short validation and check kernels of the other stream. Full grids starved them
      // (the degree-array launch holds its CUs to the end); a third for the degree-array launch,
      // which waits for work much of the time, and half for the bitset launches measured best.
      shared.grid_share = std::max(shared.grid_share, 1) * (g.words ? 2 : 3);
      go = &shared;
    }
    if ((rc2 = plan_launch(ctx, pvc, g.n_max, g.nnz_max, g.words, go, g.pl))) return rc2;
    Plan& pl = g.pl;
    if (thr_div > 0)
      pl.threshold = static_cast<uint32_t>(std::min<int64_t>(
          std::max<int64_t>(16, pl.num_wg / thr_div), static_cast<int64_t>(pl.cap) - 2 * pl.num_wg));
    if (ctx->ws) {
      // the stack depth this launch will use (see below), then a plan that fits
      const int32_t d = (o && o->stack_depth > 0) ? o->stack_depth
                        : pvc                     ? g.k_max + 1
                                                  : std::max(g.n_max, 1);
      if ((rc2 = fit_plan_to_workspace(ctx, pl, go, g.words, g.vertices, g.end - g.begin, d)))
        return rc2;
    }
    const size_t stride_b = static_cast<size_t>(pl.stride) * sizeof(int32_t);
    if ((rc2 = ensure(ctx, lc->payload, static_cast<size_t>(pl.cap) * stride_b))) return rc2;
    if ((rc2 = ensure(ctx, lc->seq, static_cast<size_t>(pl.cap) * sizeof(uint32_t)))) return rc2;
    if ((rc2 = ensure(ctx, lc->wg_stats, static_cast<size_t>(pl.num_wg) * sizeof(vc::WgStats)))) return rc2;
    if (g.words &&
        (rc2 = ensure(ctx, lc->bits, static_cast<size_t>(g.vertices) * g.words * sizeof(uint64_t))))
      return rc2;
    Params& p = params[gi];
    p = Params{};
    p.num_inst = g.end - g.begin;
    p.stride = pl.stride;
    p.n_max = g.n_max;
    p.nnz_max = g.nnz_max;
    p.rules = rules_from_flags(flags);
    p.inst = d_inst + g.begin;
    p.ist = d_ist + g.begin;
    p.work = d_work + g.begin;
    p.rp_all = b.rp;
    p.ci_all = b.ci;
    p.payload = static_cast<int32_t*>(lc->payload.ptr);
    p.seq = static_cast<uint32_t*>(lc->seq.ptr);
    p.ctr = static_cast<int32_t*>(lc->ctr.ptr);
    p.covers = covers;
    p.wg_stats = static_cast<vc::WgStats*>(lc->wg_stats.ptr);
    p.node_budget = o ? o->node_budget : 0;
    // report often enough that the whole grid overshoots a budget by at most about half
    p.budget_chunk = std::max<int64_t>(1, std::min<int64_t>(1024, p.node_budget / (2 * pl.num_wg)));
    p.q_cap = pl.cap;
    p.q_threshold = pl.threshold;
    p.num_wg = pl.num_wg;
    p.bits = g.words ? static_cast<uint64_t*>(lc->bits.ptr) : nullptr;
    p.words = g.words;
    p.rp_lds = pl.rp_lds;
    p.pvc = pvc ? 1 : 0;
    if (pl.global_node) {
      // one node slot per traversal workgroup and per greedy workgroup
      const int64_t slots = std::max<int64_t>(pl.num_wg, std::min<int64_t>(g.end - g.begin, 65535));
      if ((rc2 = ensure(ctx, lc->gnodes, static_cast<size_t>(slots) * stride_b))) return rc2;
      p.gnodes = static_cast<int32_t*>(lc->gnodes.ptr);
    }
    if (stack_only) {
      p.start_depth = o->start_depth ? o->start_depth : 12;
      p.q_threshold = 0;  // no worklist
    }
    DevResult* dres = d_res + gi;
    p.res = dres;
    // watchdog: vc_abort's word, and what is left of the call's time limit
    p.host_abort = ctx->abort_dev;
    p.abort_base = abort_base;
    if (o && o->timeout_ms > 0) {
      const double left_ms = static_cast<double>(o->timeout_ms) - ms_since(t0);
      if (left_ms <= 0.0) return fail(ctx, VC_ERR_BUDGET, "time limit reached");
      p.timeout_ticks = std::max<uint64_t>(1, static_cast<uint64_t>(left_ms * ctx->clock_khz));
    }

    VC_HIP(ctx, vc::launch_prepare(p, dres, g.vertices, g.entries, gst));
    if (!pvc) {
      const int gws = g.words ? 64 : static_cast<int>(std::min<int64_t>(1024, round_up(g.n_max, 64)));
      hipEvent_t e0 = ctx->ev[2 * ng + 4 + 2 * gi], e1 = ctx->ev[2 * ng + 5 + 2 * gi];
      VC_HIP(ctx, hipEventRecord(e0, gst));
      if (g.words) VC_HIP(ctx, vc::launch_bitset_greedy(p, gst));
      else VC_HIP(ctx, vc::launch_greedy(p, gws, gst));
      VC_HIP(ctx, hipEventRecord(e1, gst));
      if (g.words || ctx->ws) {
        // A path branches at most best - 1 <= n - 1 times. Bitset nodes are a few dozen bytes,
        // so their stacks are provisioned for that bound straight away instead of waiting on
        // the host for the largest greedy size (the traversal reads each instance's greedy
        // size from its state as the first best); so are those of a caller-workspace call,
        // which was sized for it.
        g.depth_cap = std::max(g.n_max, 1);
      } else {
        VC_HIP(ctx, vc::launch_max_greedy(p, d_greedy + gi, gst));
        VC_HIP(ctx, hipMemcpyAsync(h_gmax + gi, d_greedy + gi, sizeof(int32_t), hipMemcpyDeviceToHost, gst));
        VC_HIP(ctx, hipStreamSynchronize(gst));
        // bound = best - 1: a path branches at most best - 1 times (each branching adds to s)
        g.depth_cap = std::max(h_gmax[gi], 1);
      }
    } else {
      g.depth_cap = g.k_max + 1;
    }
    if (o && o->stack_depth > 0) g.depth_cap = o->stack_depth;  // the caller's choice
    if ((rc2 = size_stacks(lc, pl, g.depth_cap))) {
      if (lc != ctx) ctx->last_error = lc->last_error;
      return rc2;
    }
    p.stacks = static_cast<int32_t*>(lc->stacks.ptr);
    p.depth_cap = g.depth_cap;
    p.num_wg = pl.num_wg;
    p.stack_lds = 0;
    if (g.words) {
      // A bitset node is a few dozen bytes: keep the stack ring in LDS when it fits there
      // (within the default 64 KB) without lowering the launch's residency, so a pop is an LDS
      // read instead of a dependent device-memory load.
      p.stack_lds = 1;
      const size_t lds = vc::bitset_traverse_lds_bytes(p);
      int occ = 0;
      if (lds <= 65536 && (rc2 = occupancy(ctx, g.words, pvc, prof, 64, lds, g.n_max, &occ)))
        return rc2;
      if (static_cast<int64_t>(occ) * ctx->prop.multiProcessorCount < pl.num_wg) p.stack_lds = 0;
    }
    lc->last_num_wg = pl.num_wg;
    ctx->stats_src = lc;
    VC_HIP(ctx, hipEventRecord(ctx->ev[2 * gi], gst));
    if (g.words) VC_HIP(ctx, vc::launch_bitset_traverse(pvc, prof, p, gst));
    else VC_HIP(ctx, vc::launch_traverse(pvc, prof, p, pl.wg_size, gst));
    VC_HIP(ctx, hipEventRecord(ctx->ev[2 * gi + 1], gst));
    if (final) VC_HIP(ctx, vc::launch_finalize(p, g.vertices, g.entries, dres, gst));
    return VC_OK;
  };

  // Fresh per-instance state of one group again (the pinned mirror still holds it).
  auto reset_group = [&](int32_t gi) -> int {
    const Group& g = groups[gi];
    const size_t cnt = static_cast<size_t>(g.end - g.begin);
    const hipStream_t gst = lane(gi)->stream;
    VC_HIP(ctx, hipMemcpyAsync(d_ist + g.begin, h_ist + g.begin, cnt * sizeof(InstState),
                               hipMemcpyHostToDevice, gst));
    VC_HIP(ctx, hipMemcpyAsync(d_work + g.begin, reinterpret_cast<int32_t*>(host + L.work) + g.begin,
                               cnt * sizeof(int32_t), hipMemcpyHostToDevice, gst));
    return VC_OK;
  };

  if (stack_only && m > 1)
    return fail(ctx, VC_ERR_INVALID_ARG, "VC_OPT_STACK_ONLY takes one graph per call");
  const bool explicit_knobs = o && (o->wg_size || o->num_wg || o->wl_capacity || o->wl_threshold);
  const bool autotune = (flags & VC_OPT_AUTOTUNE) && !explicit_knobs && !stack_only && !ctx->ws;
  for (int32_t step = 0; step < ng; ++step) {
    // with the auxiliary context, the degree-array group (the last) goes first
    const int32_t gi = use_aux ? (step == 0 ? ng - 1 : step - 1) : step;
    Group& g = groups[gi];
    vc_options go = o ? *o : vc_options{};
    int thr_div = 0;
    if (autotune) {
      auto lg = [](int64_t x) { int l = 0; while ((int64_t(1) << l) < x) ++l; return l; };
      const auto key = std::make_tuple(g.words, pvc ? 1 : 0, flags & ~VC_OPT_AUTOTUNE, lg(g.n_max),
                                       lg(g.end - g.begin));
      auto it = ctx->tuned.find(key);
      if (it == ctx->tuned.end()) {
        // trial launches over a small grid; the default knobs are one of the candidates
        std::vector<std::tuple<int, int, int>> cand;  // (wg_size, num_wg, threshold divisor)
        cand.emplace_back(0, 0, 0);
        if (g.words) {
          // up to 16 one-wavefront workgroups per CU (the default plan stops at 8; 20 to 28 per
          // CU measured slower on the hard MVC batch: more workgroups polling the worklist)
          for (int mult : {1, 2, 4, 8, 12, 16})
            for (int div : {8, 2}) cand.emplace_back(0, mult * cus, div);
        } else {
          Plan base;
          if ((rc = plan_launch(ctx, pvc, g.n_max, g.nnz_max, 0, &go, base))) return rc;
          // and, for fewer instances than the grid holds, one workgroup per instance (no idle
          // workgroups polling the worklist; donations then have no takers but for finished
          // instances' workgroups)
          const int64_t count = g.end - g.begin;
          for (int ws : {base.wg_size / 2, base.wg_size, base.wg_size * 2})
            if (ws >= 64 && ws <= 1024) {
              for (int div : {8, 1}) cand.emplace_back(ws, 0, div);
              if (count < base.num_wg) cand.emplace_back(ws, static_cast<int>(count), 8);
            }
        }
        float best_ms = 0.f;
        std::tuple<int, int, int> best = cand[0];
        for (const auto& c : cand) {
          vc_options t = go;
          t.wg_size = std::get<0>(c);
          t.num_wg = std::get<1>(c);
          // two trial launches per candidate, the faster one counts (one launch's noise is as
          // large as the differences that matter)
          float cand_ms = 0.f;
          bool fits = true;
          for (int trial = 0; trial < 2 && fits; ++trial) {
            if ((rc = reset_group(gi))) return rc;
            rc = run_group(gi, &t, std::get<2>(c), false);
            if (rc == VC_ERR_INVALID_ARG || rc == VC_ERR_NO_MEMORY) {  // does not fit
              fits = false;
              break;
            }
            if (rc) return rc;
            VC_HIP(ctx, hipStreamSynchronize(lane(gi)->stream));
            float ms = 0.f;
            VC_HIP(ctx, hipEventElapsedTime(&ms, ctx->ev[2 * gi], ctx->ev[2 * gi + 1]));
            if (trial == 0 || ms < cand_ms) cand_ms = ms;
          }
          if (!fits) continue;
          if (best_ms == 0.f || cand_ms < best_ms) {
            best_ms = cand_ms;
            best = c;
          }
        }
        ctx->last_error.clear();
        it = ctx->tuned.emplace(key, best).first;
        if ((rc = reset_group(gi))) return rc;
      }
      go.wg_size = std::get<0>(it->second);
      go.num_wg = std::get<1>(it->second);
      thr_div = std::get<2>(it->second);
    }
    if ((rc = run_group(gi, &go, thr_div, true))) return rc;
  }
  if (use_aux) {  // the degree-array launch and its cover check end before the copy out
    VC_HIP(ctx, hipEventRecord(ctx->ev[2 * ng + 3], ctx->aux->stream));
    VC_HIP(ctx, hipStreamWaitEvent(st, ctx->ev[2 * ng + 3], 0));
  }

  // one copy out: per-instance state, work counters and result blocks
  if (m > 0)
    VC_HIP(ctx, hipMemcpyAsync(host + L.ist, dev + L.ist, L.gmax - L.ist, hipMemcpyDeviceToHost, st));
  uint8_t* h_cover = reinterpret_cast<uint8_t*>(host + L.cover);
  if (out.cover_host && total_n > 0)
    VC_HIP(ctx, hipMemcpyAsync(h_cover, covers, static_cast<size_t>(total_n), hipMemcpyDeviceToHost, st));
  VC_HIP(ctx, hipStreamSynchronize(st));
  if (!pvc)
    for (int32_t gi = 0; gi < ng; ++gi) {
      float ms = 0.f;
      VC_HIP(ctx, hipEventElapsedTime(&ms, ctx->ev[2 * ng + 4 + 2 * gi], ctx->ev[2 * ng + 5 + 2 * gi]));
      greedy_ms += ms;
    }
  // traversal time: the launches' durations added up, or with the auxiliary context (whose
  // degree-array launch starts first) the span until the last traversal ends
  double kernel_ms = 0.0;
  for (int32_t gi = 0; gi < ng; ++gi) {
    float ms = 0.f;
    if (use_aux) {
      VC_HIP(ctx, hipEventElapsedTime(&ms, ctx->ev[2 * (ng - 1)], ctx->ev[2 * gi + 1]));
      kernel_ms = std::max(kernel_ms, static_cast<double>(ms));
    } else {
      VC_HIP(ctx, hipEventElapsedTime(&ms, ctx->ev[2 * gi], ctx->ev[2 * gi + 1]));
      kernel_ms += ms;
    }
  }

  // launch-wide failures end the whole call
  for (int32_t gi = 0; gi < ng; ++gi) {
    const DevResult& r = h_res[gi];
    if (r.stop_reason == vc::kStopHost && !r.error)
      return fail(ctx, VC_ERR_BUDGET, "stopped by vc_abort");
    if (r.stop_reason == vc::kStopTimeout && !r.error)
      return fail(ctx, VC_ERR_BUDGET,
                  "time limit of " + std::to_string(o ? o->timeout_ms : 0) + " ms reached");
    if (r.error)
      return fail(ctx, VC_ERR_INTERNAL,
                  "device invariant failed (code " + std::to_string(r.error) +
                      (r.error == 1 ? ": stack overflow)" : ": node of an unknown instance)"));
    if (r.aborted) return fail(ctx, VC_ERR_INTERNAL, "search aborted on the device");
  }
  // per-instance answers, checked against the verification done by finalize_kernel
  std::vector<int32_t> status(b.count, VC_OK), size(b.count, 0), yes(b.count, 1);
  std::vector<int64_t> nodes(b.count, 0);
  int32_t first_bad = -1;
  std::string bad_msg;
  for (int32_t s = 0; s < m; ++s) {
    const int32_t i = order[s];
    const InstState& is = h_ist[s];
    nodes[i] = is.nodes;
    if (is.err_row != vc::kNoRow) {
      status[i] = VC_ERR_INVALID_GRAPH;
      size[i] = -1;
      yes[i] = 0;
      if (first_bad < 0) first_bad = i, bad_msg = bad_row_message(is.err_row);
      continue;
    }
    if (is.state & vc::kInstOutOfBudget) {
      status[i] = VC_ERR_BUDGET;
      size[i] = -1;
      yes[i] = 0;
      if (first_bad < 0) first_bad = i, bad_msg = "node budget exhausted";
      continue;
    }
    const bool answered = !pvc || (is.state & vc::kInstFound);
    yes[i] = answered ? 1 : 0;
    size[i] = answered ? is.best : -1;
    const bool ok = !answered ? (is.cover_count == 0)
                              : (is.uncovered == 0 && is.cover_count == is.best &&
                                 (!pvc || is.best <= b.k[i]));
    if (!ok)
      return fail(ctx, VC_ERR_INTERNAL,
                  "recorded cover of instance " + std::to_string(i) + " failed verification: " +
                      std::to_string(is.uncovered) + " uncovered edge entries, " +
                      std::to_string(is.cover_count) + " vertices for size " +
                      std::to_string(is.best));
  }
  for (int32_t i = 0; i < b.count; ++i)
    if (b.n[i] == 0 && b.nnz[i] != 0) {
      status[i] = VC_ERR_INVALID_GRAPH;
      size[i] = -1;
      yes[i] = 0;
    }
  if (out.single && status[0] != VC_OK) return fail(ctx, status[0], bad_msg);

  for (int32_t i = 0; i < b.count; ++i) {
    if (out.status) out.status[i] = status[i];
    if (out.size) out.size[i] = size[i];
    if (out.yes) out.yes[i] = yes[i];
    if (out.nodes) out.nodes[i] = nodes[i];
  }
  if (out.cover_host && total_n > 0)
    std::memcpy(out.cover_host, h_cover, static_cast<size_t>(total_n));
  if (out.stats) {
    vc_stats* sp = out.stats;
    std::memset(sp, 0, sizeof *sp);
    sp->wg_nodes_min = ng ? INT64_MAX : 0;
    for (int32_t s = 0; s < m; ++s) sp->nodes += h_ist[s].nodes;  // each tree node once
    for (int32_t gi = 0; gi < ng; ++gi) {
      const DevResult& r = h_res[gi];
      const Group& g = groups[gi];
      sp->wg_nodes_max = std::max(sp->wg_nodes_max, r.wg_nodes_max);
      // idle workgroups do not report: any idle one makes the minimum zero
      sp->wg_nodes_min = std::min<int64_t>(
          sp->wg_nodes_min, r.active_wgs < g.pl.num_wg ? 0 : r.wg_nodes_min);
      sp->stack_pushes += r.pushes;
      sp->stack_pops += r.pops;
      sp->wl_enqueues += r.enqueues;
      sp->wl_dequeues += r.dequeues;
      sp->max_stack_depth = std::max(sp->max_stack_depth, r.max_depth);
      sp->wg_size = std::max(sp->wg_size, g.pl.wg_size);
      sp->num_wg = std::max(sp->num_wg, g.pl.num_wg);
      sp->wl_capacity = std::max(sp->wl_capacity, static_cast<int32_t>(g.pl.cap));
      sp->wl_threshold = std::max(sp->wl_threshold, static_cast<int32_t>(g.pl.threshold));
      sp->depth_cap = std::max(sp->depth_cap, g.depth_cap);
      sp->n = std::max(sp->n, g.n_max);
      sp->bitset_words = std::max(sp->bitset_words, g.words);
      const int32_t nb = g.words ? 8 * g.words + 8 : 4 * (g.n_max + 3);
      sp->node_bytes = std::max(sp->node_bytes, nb);
      for (int a = 0; a < vc::kNumActivities; ++a) sp->cycles[a] += r.cycles[a];
      // node copies by where they went: the worklist is in device memory; a stack is in LDS
      // only for a bitset launch with stack_lds
      const int64_t stack_copies = r.pushes + r.pops;
      sp->hbm_node_bytes += static_cast<int64_t>(nb) *
                            (r.enqueues + r.dequeues + (params[gi].stack_lds ? 0 : stack_copies));
      if (params[gi].stack_lds) sp->lds_node_bytes += static_cast<int64_t>(nb) * stack_copies;
      sp->stack_lds |= params[gi].stack_lds;
      sp->launches += 1;
      // graph data copied per instance taken, at the launch's mean graph size
      const double count = static_cast<double>(std::max(g.end - g.begin, 1));
      const double per_inst =
          g.words ? 8.0 * g.words * (static_cast<double>(g.vertices) / count)
                  : (g.pl.rp_lds >= 1 ? 4.0 * (static_cast<double>(g.vertices) / count + 1.0) : 0.0) +
                        (g.pl.rp_lds == 2 ? 4.0 * static_cast<double>(g.entries) / count : 0.0);
      sp->graph_bytes += static_cast<int64_t>(per_inst * static_cast<double>(r.instances));
    }
    sp->greedy_size = (!pvc && out.single && m == 1) ? h_ist[0].greedy : -1;
    sp->kernel_ms = kernel_ms;
    sp->greedy_ms = greedy_ms;
    sp->total_ms = ms_since(t0);
  }
  return VC_OK;
}

// Copy a host CSR (one graph, or a packed batch) into the context's device buffers.
int upload(vc_ctx* ctx, const int32_t* rp, int64_t rp_count, const int32_t* ci, int64_t ci_count,
           const int32_t** rp_dev, const int32_t** ci_dev) {
  int rc;
  if ((rc = ensure(ctx, ctx->rp, static_cast<size_t>(std::max<int64_t>(rp_count, 1)) * sizeof(int32_t)))) return rc;
  if ((rc = ensure(ctx, ctx->ci, static_cast<size_t>(std::max<int64_t>(ci_count, 1)) * sizeof(int32_t)))) return rc;
  if (rp_count > 0)
    VC_HIP(ctx, hipMemcpyAsync(ctx->rp.ptr, rp, static_cast<size_t>(rp_count) * sizeof(int32_t),
                               hipMemcpyHostToDevice, ctx->stream));
  if (ci_count > 0)
    VC_HIP(ctx, hipMemcpyAsync(ctx->ci.ptr, ci, static_cast<size_t>(ci_count) * sizeof(int32_t),
                               hipMemcpyHostToDevice, ctx->stream));
  *rp_dev = static_cast<const int32_t*>(ctx->rp.ptr);
  *ci_dev = static_cast<const int32_t*>(ctx->ci.ptr);
  return VC_OK;
}

int enter(vc_ctx* ctx) {
  if (!ctx) return VC_ERR_INVALID_ARG;
  ctx->last_error.clear();
  VC_HIP(ctx, hipSetDevice(ctx->device));
  return VC_OK;
}

// vc_abort's word as the call begins: a launch stops once the word differs from it.
int32_t abort_mark(const vc_ctx* ctx) {
  return ctx->abort_host ? __atomic_load_n(ctx->abort_host, __ATOMIC_ACQUIRE) : 0;
}

// A caller-workspace call: for its duration the context's device buffers are empty and every
// one it needs is carved from the caller's workspace; its own buffers come back afterwards and
// nothing of the workspace stays referenced (per-workgroup statistics included).
class WorkspaceScope {
 public:
  WorkspaceScope(vc_ctx* ctx, void* base, size_t bytes, bool host_heap) : ctx_(ctx) {
    if (!base) return;
    ws_.base = static_cast<char*>(base);
    ws_.bytes = bytes;
    ws_.host_heap = host_heap;
    for (size_t i = 0; i < kBufs; ++i) {
      saved_[i] = *buf(i);
      *buf(i) = DevBuf{};
    }
    ctx->ws = &ws_;
    active_ = true;
  }
  ~WorkspaceScope() {
    if (!active_) return;
    for (size_t i = 0; i < kBufs; ++i) *buf(i) = saved_[i];
    ctx_->ws = nullptr;
    // the last launch's workgroup statistics were in the workspace: none to report
    ctx_->last_num_wg = 0;
    ctx_->stats_src = nullptr;
  }
  WorkspaceScope(const WorkspaceScope&) = delete;
  WorkspaceScope& operator=(const WorkspaceScope&) = delete;

 private:
  static constexpr size_t kBufs = 12;
  DevBuf* buf(size_t i) {
    DevBuf* all[kBufs] = {&ctx_->rp,     &ctx_->ci,       &ctx_->meta,     &ctx_->payload,
                          &ctx_->seq,    &ctx_->ctr,      &ctx_->stacks,   &ctx_->covers,
                          &ctx_->wg_stats, &ctx_->scratch, &ctx_->bits,    &ctx_->gnodes};
    return all[i];
  }
  vc_ctx* ctx_;
  vc_ctx::Workspace ws_;
  DevBuf saved_[kBufs];
  bool active_ = false;
};

struct WsArgs {
  void* base = nullptr;    // nullptr: the context's own buffers
  size_t bytes = 0;
  bool host_heap = true;   // host staging may grow beyond the pinned buffer
};

// One graph: a batch of one.
int solve(vc_ctx* ctx, const vc_graph* g, bool device_graph, bool pvc, int32_t k,
          const vc_options* o, int32_t* yes_out, int32_t* size_out, uint8_t* cover_dev,
          uint8_t* cover_host, vc_stats* stats, const WsArgs& wsa = WsArgs{}) {
  const auto t0 = std::chrono::steady_clock::now();
  int rc = enter(ctx);
  if (rc) return rc;
  const int32_t abort_base = abort_mark(ctx);
  if (!size_out || (pvc && !yes_out)) return fail(ctx, VC_ERR_INVALID_ARG, "output pointer is NULL");
  if (pvc && k < 0) return fail(ctx, VC_ERR_INVALID_ARG, "k must be >= 0");
  if ((rc = check_graph_args(ctx, g))) return rc;
  if ((rc = check_options(ctx, o))) return rc;
  if (g->n == 0) {
    *size_out = 0;
    if (yes_out) *yes_out = 1;
    if (stats) std::memset(stats, 0, sizeof *stats), stats->total_ms = ms_since(t0);
    return VC_OK;
  }
  BatchIn b;
  b.count = 1;
  b.n = &g->n;
  b.nnz = &g->nnz;
  b.k = &k;
  if (device_graph) {
    b.rp = g->row_ptr;
    b.ci = g->col_idx;
  } else if ((rc = upload(ctx, g->row_ptr, static_cast<int64_t>(g->n) + 1, g->col_idx, g->nnz,
                          &b.rp, &b.ci))) {
    return rc;
  }
  BatchOut out;
  int32_t status = 0, size = 0, yes = 0;
  out.status = &status;
  out.size = &size;
  out.yes = &yes;
  out.cover_host = cover_host;
  out.cover_dev = cover_dev;
  out.stats = stats;
  out.single = true;
  {
    WorkspaceScope scope(ctx, wsa.base, wsa.bytes, wsa.host_heap);
    if ((rc = run_batch(ctx, b, pvc, o, out, t0, abort_base))) return rc;
  }
  *size_out = size;
  if (yes_out) *yes_out = yes;
  return VC_OK;
}

int solve_batch(vc_ctx* ctx, const vc_batch* batch, bool device_graph, bool pvc,
                const int32_t* k, const vc_options* o, int32_t* status_out, int32_t* yes_out,
                int32_t* size_out, uint8_t* cover_dev, uint8_t* cover_host, int64_t* nodes_out,
                vc_stats* stats, const WsArgs& wsa = WsArgs{}) {
  const auto t0 = std::chrono::steady_clock::now();
  int rc = enter(ctx);
  if (rc) return rc;
  const int32_t abort_base = abort_mark(ctx);
  if (!batch) return fail(ctx, VC_ERR_INVALID_ARG, "batch is NULL");
  if (!status_out || !size_out || (pvc && !yes_out))
    return fail(ctx, VC_ERR_INVALID_ARG, "output pointer is NULL");
  if ((rc = check_options(ctx, o))) return rc;
  BatchIn b;
  b.count = batch->count;
  b.n = batch->n;
  b.nnz = batch->nnz;
  b.k = k;
  int64_t total_rp = 0, total_n = 0, total_nnz = 0;
  if ((rc = check_batch(ctx, BatchIn{b.count, b.n, b.nnz, k, batch->row_ptr, batch->col_idx},
                        pvc, &total_rp, &total_n, &total_nnz)))
    return rc;
  if (device_graph) {
    b.rp = batch->row_ptr;
    b.ci = batch->col_idx;
  } else if ((rc = upload(ctx, batch->row_ptr, total_rp, batch->col_idx, total_nnz, &b.rp, &b.ci))) {
    return rc;
  }
  BatchOut out;
  out.status = status_out;
  out.size = size_out;
  out.yes = yes_out;
  out.nodes = nodes_out;
  out.cover_host = cover_host;
  out.cover_dev = cover_dev;
  out.stats = stats;
  WorkspaceScope scope(ctx, wsa.base, wsa.bytes, wsa.host_heap);
  return run_batch(ctx, b, pvc, o, out, t0, abort_base);
}

// Device bytes a caller-workspace call on these graphs needs (an upper bound): the buffers
// run_batch carves, summed over its launch groups (each group's own worklist, tickets,
// statistics, adjacency rows, node slots and stacks of `depth` entries, 0 = n + 1), with the
// larger of the MVC and PVC launch plans.
int workspace_need(vc_ctx* ctx, int32_t count, const int32_t* n, const int32_t* nnz,
                   int32_t depth, const vc_options* o, size_t* out) {
  const int32_t flags = o ? o->flags : 0;
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  struct Fam {
    int32_t n_max = 0, nnz_max = 0, count = 0;
    int64_t vertices = 0;
  };
  std::map<int32_t, Fam> fams;  // by bitset words (0: degree arrays)
  int64_t total_n = 0;
  int32_t m = 0;
  for (int32_t i = 0; i < count; ++i) {
    if (n[i] < 0 || nnz[i] < 0) return fail(ctx, VC_ERR_INVALID_ARG, "negative n or nnz");
    if (n[i] == 0) continue;
    int32_t words = 0;
    int rc = choose_words(ctx, n[i], flags, &words);
    if (rc) return rc;
    Fam& f = fams[words];
    f.n_max = std::max(f.n_max, n[i]);
    f.nnz_max = std::max(f.nnz_max, nnz[i]);
    f.count += 1;
    f.vertices += n[i];
    total_n += n[i];
    ++m;
  }
  size_t total = 256 + al(meta_layout(m, static_cast<int32_t>(fams.size()), 0).dev_end) +
                 al(static_cast<size_t>(total_n)) +
                 al(vc::kNumCounters * vc::kCounterStride * sizeof(int32_t));
  for (const auto& kv : fams) {
    const int32_t words = kv.first;
    const Fam& f = kv.second;
    size_t best = 0;
    for (bool pvc : {false, true}) {
      Plan pl;
      int rc = plan_launch(ctx, pvc, f.n_max, f.nnz_max, words, o, pl);
      if (rc) return rc;
      const size_t stride_b = static_cast<size_t>(pl.stride) * sizeof(int32_t);
      int64_t d = depth > 0 ? depth : static_cast<int64_t>(f.n_max) + 1;
      if (o && o->stack_depth > 0) d = o->stack_depth;
      size_t need = al(pl.cap * stride_b) + al(pl.cap * sizeof(uint32_t)) +
                    al(static_cast<size_t>(pl.num_wg) * sizeof(vc::WgStats)) +
                    al(static_cast<size_t>(pl.num_wg) * static_cast<size_t>(d) * stride_b);
      if (words) need += al(static_cast<size_t>(f.vertices) * words * sizeof(uint64_t));
      if (pl.global_node)
        need += al(static_cast<size_t>(std::max<int64_t>(pl.num_wg, std::min(f.count, 65535))) *
                   stride_b);
      best = std::max(best, need);
    }
    total += best;
  }
  *out = total;
  return VC_OK;
}

int check_workspace(vc_ctx* ctx, void* ws, size_t bytes) {
  if (!ws || bytes == 0) return fail(ctx, VC_ERR_INVALID_ARG, "workspace is NULL or empty");
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0)
    return fail(ctx, VC_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  return VC_OK;
}

// Validate a device CSR (a batch of one) for a one-workgroup kernel (greedy, reduce).
int setup_single(vc_ctx* ctx, const vc_graph* g, int rules, int32_t flags, uint8_t* covers,
                 Params& p, int32_t* wg_size) {
  int32_t words = 0;
  int rc = choose_words(ctx, g->n, flags, &words);
  if (rc) return rc;
  Plan pl;
  vc_options o{};
  o.flags = flags & (VC_OPT_GLOBAL_NODES | VC_OPT_CSR_GLOBAL);
  if ((rc = plan_launch(ctx, false, g->n, g->nnz, words, &o, pl))) return rc;
  const MetaLayout L = meta_layout(1, 1, 0);
  if ((rc = ensure(ctx, ctx->meta, L.dev_end))) return rc;
  if ((rc = ensure_pinned(ctx, L.host_end))) return rc;
  if ((rc = ensure(ctx, ctx->ctr, vc::kNumCounters * vc::kCounterStride * sizeof(int32_t)))) return rc;
  if ((rc = ensure(ctx, ctx->seq, sizeof(uint32_t)))) return rc;
  if (!covers) {
    if ((rc = ensure(ctx, ctx->covers, static_cast<size_t>(g->n)))) return rc;
    covers = static_cast<uint8_t*>(ctx->covers.ptr);
  }
  if (words && (rc = ensure(ctx, ctx->bits, static_cast<size_t>(g->n) * words * sizeof(uint64_t))))
    return rc;
  char* host = static_cast<char*>(ctx->pinned);
  char* dev = static_cast<char*>(ctx->meta.ptr);
  Instance& in = *reinterpret_cast<Instance*>(host + L.inst);
  in = Instance{};
  in.n = g->n;
  in.nnz = g->nnz;
  init_state(reinterpret_cast<InstState*>(host + L.ist), reinterpret_cast<int32_t*>(host + L.work), 1);
  VC_HIP(ctx, hipMemcpyAsync(dev, host, L.res, hipMemcpyHostToDevice, ctx->stream));
  p = Params{};
  p.num_inst = 1;
  p.stride = pl.stride;
  p.n_max = g->n;
  p.nnz_max = g->nnz;
  p.rules = rules;
  p.inst = reinterpret_cast<const Instance*>(dev + L.inst);
  p.ist = reinterpret_cast<InstState*>(dev + L.ist);
  p.work = reinterpret_cast<int32_t*>(dev + L.work);
  p.rp_all = g->row_ptr;
  p.ci_all = g->col_idx;
  p.seq = static_cast<uint32_t*>(ctx->seq.ptr);
  p.ctr = static_cast<int32_t*>(ctx->ctr.ptr);
  p.covers = covers;
  p.q_cap = 1;
  p.bits = words ? static_cast<uint64_t*>(ctx->bits.ptr) : nullptr;
  p.words = words;
  p.rp_lds = pl.rp_lds;
  if (pl.global_node) {
    if ((rc = ensure(ctx, ctx->gnodes, static_cast<size_t>(pl.stride) * sizeof(int32_t)))) return rc;
    p.gnodes = static_cast<int32_t*>(ctx->gnodes.ptr);
  }
  *wg_size = words ? 64 : static_cast<int32_t>(std::min<int64_t>(1024, round_up(g->n, 64)));
  DevResult* dres = reinterpret_cast<DevResult*>(dev + L.res);
  p.res = dres;
  VC_HIP(ctx, vc::launch_prepare(p, dres, g->n, g->nnz, ctx->stream));
  return VC_OK;
}

}  // namespace

namespace vc {

int context_device(const vc_ctx* ctx) { return ctx->device; }

int pvc_device_in(vc_ctx* ctx, const vc_graph* g, int32_t k, const vc_options* opts, void* ws,
                  size_t bytes, int32_t* yes_out, int32_t* size_out, uint8_t* cover_dev,
                  vc_stats* stats) {
  int rc = enter(ctx);
  if (rc) return rc;
  if ((rc = check_workspace(ctx, ws, bytes))) return rc;
  rc = solve(ctx, g, true, true, k, opts, yes_out, size_out, cover_dev, nullptr, stats,
             WsArgs{ws, bytes, false});
  if (rc == VC_ERR_NO_MEMORY)
    ctx->last_error = "the graph is too large for the no-allocation entry point, whose device "
                      "scratch holds " + std::to_string(bytes) + " bytes: " + ctx->last_error;
  return rc;
}

}  // namespace vc

extern "C" {

const char* vc_version(void) { return "0.3.0"; }

const char* vc_strerror(int status) {
  switch (status) {
    case VC_OK: return "ok";
    case VC_ERR_INVALID_GRAPH: return "invalid graph";
    case VC_ERR_INVALID_ARG: return "invalid argument";
    case VC_ERR_NO_MEMORY: return "out of device memory";
    case VC_ERR_BUDGET: return "node budget exhausted";
    case VC_ERR_DEVICE: return "HIP device error";
    case VC_ERR_INTERNAL: return "internal error";
    default: return "unknown status";
  }
}

const char* vc_last_error(const vc_ctx* ctx) { return ctx ? ctx->last_error.c_str() : ""; }

int vc_wg_loads(vc_ctx* ctx, int64_t* nodes_out, int64_t* cycles_out, int32_t max,
                int32_t* count_out) {
  int rc = enter(ctx);
  if (rc) return rc;
  if (!count_out || max < 0) return fail(ctx, VC_ERR_INVALID_ARG, "NULL argument");
  const vc_ctx* src = ctx->stats_src ? ctx->stats_src : ctx;
  const int32_t cnt = src->wg_stats.ptr ? src->last_num_wg : 0;
  *count_out = cnt;
  const int32_t take = std::min(cnt, max);
  if (take > 0) {
    std::vector<vc::WgStats> w(static_cast<size_t>(take));
    VC_HIP(ctx, hipMemcpyAsync(w.data(), src->wg_stats.ptr, w.size() * sizeof(vc::WgStats),
                               hipMemcpyDeviceToHost, src->stream));
    VC_HIP(ctx, hipStreamSynchronize(src->stream));
    for (int32_t i = 0; i < take; ++i) {
      const vc::WgStats& x = w[static_cast<size_t>(i)];
      if (nodes_out) nodes_out[i] = x.nodes;
      if (cycles_out)
        for (int a = 0; a < vc::kNumActivities; ++a) cycles_out[i * vc::kNumActivities + a] = x.cycles[a];
    }
  }
  return VC_OK;
}

int vc_create(vc_ctx** ctx_out, int device, void* hip_stream) {
  if (!ctx_out) return VC_ERR_INVALID_ARG;
  *ctx_out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count == 0) return VC_ERR_DEVICE;
  if (device < 0 || device >= count) return VC_ERR_INVALID_ARG;
  vc_ctx* ctx = new vc_ctx();
  ctx->device = device;
  hipError_t e = hipSetDevice(device);
  if (e == hipSuccess) e = hipGetDeviceProperties(&ctx->prop, device);
  if (e == hipSuccess) {
    if (hip_stream) {
      ctx->stream = static_cast<hipStream_t>(hip_stream);
    } else {
      e = hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking);
      ctx->own_stream = e == hipSuccess;
    }
  }
  // Everything a call may need besides its device buffers is made here, so that the
  // caller-workspace forms allocate nothing: the events of up to kMaxGroups launch groups, a
  // pinned staging buffer for the instance table of a batch of a few thousand graphs, the
  // mapped word of vc_abort and the device clock's rate.
  if (e == hipSuccess && ensure_events(ctx, 4 * kMaxGroups + 4) != VC_OK) e = hipErrorUnknown;
  if (e == hipSuccess && ensure_pinned(ctx, kPinnedStart) != VC_OK) e = hipErrorUnknown;
  if (e == hipSuccess) {
    void* word = nullptr;
    e = hipHostMalloc(&word, sizeof(int32_t), hipHostMallocMapped | hipHostMallocCoherent);
    if (e == hipSuccess) {
      ctx->abort_host = static_cast<int32_t*>(word);
      *ctx->abort_host = 0;
      void* dptr = nullptr;
      e = hipHostGetDevicePointer(&dptr, word, 0);
      ctx->abort_dev = static_cast<const int32_t*>(dptr);
    }
  }
  if (e == hipSuccess) {
    int khz = 0;
    e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device);
    ctx->clock_khz = khz > 0 ? khz : 100000;
  }
  if (e == hipSuccess && vc::noalloc_setup(device) != VC_OK) e = hipErrorUnknown;
  if (e != hipSuccess) {
    vc_destroy(ctx);
    return VC_ERR_DEVICE;
  }
  *ctx_out = ctx;
  return VC_OK;
}

int vc_abort(vc_ctx* ctx) {
  if (!ctx || !ctx->abort_host) return VC_ERR_INVALID_ARG;
  __atomic_fetch_add(ctx->abort_host, 1, __ATOMIC_RELEASE);
  return VC_OK;
}

int vc_destroy(vc_ctx* ctx) {
  if (!ctx) return VC_OK;
  (void)hipSetDevice(ctx->device);
  if (ctx->aux) vc_destroy(ctx->aux);  // first: its launches read this context's buffers
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  DevBuf* bufs[] = {&ctx->rp,     &ctx->ci,       &ctx->meta,     &ctx->payload, &ctx->seq,
                    &ctx->ctr,    &ctx->stacks,   &ctx->covers,   &ctx->wg_stats, &ctx->scratch,
                    &ctx->bits,   &ctx->gnodes};
  for (DevBuf* b : bufs)
    if (b->ptr) (void)hipFree(b->ptr);
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  if (ctx->abort_host) (void)hipHostFree(ctx->abort_host);
  for (hipEvent_t ev : ctx->ev)
    if (ev) (void)hipEventDestroy(ev);
  if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
  return VC_OK;
}

int vc_mvc(vc_ctx* ctx, const vc_graph* g, const vc_options* opts, int32_t* size_out,
           uint8_t* cover_out, vc_stats* stats) {
  return solve(ctx, g, false, false, 0, opts, nullptr, size_out, nullptr, cover_out, stats);
}

int vc_pvc(vc_ctx* ctx, const vc_graph* g, int32_t k, const vc_options* opts, int32_t* yes_out,
           int32_t* size_out, uint8_t* cover_out, vc_stats* stats) {
  return solve(ctx, g, false, true, k, opts, yes_out, size_out, nullptr, cover_out, stats);
}

int vc_mvc_device(vc_ctx* ctx, const vc_graph* g, const vc_options* opts, int32_t* size_out,
                  uint8_t* cover_dev, vc_stats* stats) {
  return solve(ctx, g, true, false, 0, opts, nullptr, size_out, cover_dev, nullptr, stats);
}

int vc_pvc_device(vc_ctx* ctx, const vc_graph* g, int32_t k, const vc_options* opts,
                  int32_t* yes_out, int32_t* size_out, uint8_t* cover_dev, vc_stats* stats) {
  return solve(ctx, g, true, true, k, opts, yes_out, size_out, cover_dev, nullptr, stats);
}

int vc_mvc_batch(vc_ctx* ctx, const vc_batch* batch, const vc_options* opts, int32_t* status_out,
                 int32_t* size_out, uint8_t* cover_out, int64_t* nodes_out, vc_stats* stats) {
  return solve_batch(ctx, batch, false, false, nullptr, opts, status_out, nullptr, size_out,
                     nullptr, cover_out, nodes_out, stats);
}

int vc_pvc_batch(vc_ctx* ctx, const vc_batch* batch, const int32_t* k, const vc_options* opts,
                 int32_t* status_out, int32_t* yes_out, int32_t* size_out, uint8_t* cover_out,
                 int64_t* nodes_out, vc_stats* stats) {
  return solve_batch(ctx, batch, false, true, k, opts, status_out, yes_out, size_out, nullptr,
                     cover_out, nodes_out, stats);
}

int vc_mvc_batch_device(vc_ctx* ctx, const vc_batch* batch, const vc_options* opts,
                        int32_t* status_out, int32_t* size_out, uint8_t* cover_dev,
                        int64_t* nodes_out, vc_stats* stats) {
  return solve_batch(ctx, batch, true, false, nullptr, opts, status_out, nullptr, size_out,
                     cover_dev, nullptr, nodes_out, stats);
}

int vc_pvc_batch_device(vc_ctx* ctx, const vc_batch* batch, const int32_t* k,
                        const vc_options* opts, int32_t* status_out, int32_t* yes_out,
                        int32_t* size_out, uint8_t* cover_dev, int64_t* nodes_out,
                        vc_stats* stats) {
  return solve_batch(ctx, batch, true, true, k, opts, status_out, yes_out, size_out, cover_dev,
                     nullptr, nodes_out, stats);
}

int vc_workspace_bytes(vc_ctx* ctx, int32_t n, int32_t nnz, int32_t depth,
                       const vc_options* opts, size_t* bytes_out) {
  int rc = enter(ctx);
  if (rc) return rc;
  if (!bytes_out) return fail(ctx, VC_ERR_INVALID_ARG, "bytes_out is NULL");
  if (depth < 0) return fail(ctx, VC_ERR_INVALID_ARG, "depth must be >= 0");
  if ((rc = check_options(ctx, opts))) return rc;
  return workspace_need(ctx, 1, &n, &nnz, depth, opts, bytes_out);
}

int vc_batch_workspace_bytes(vc_ctx* ctx, const vc_batch* batch, int32_t depth,
                             const vc_options* opts, size_t* bytes_out) {
  int rc = enter(ctx);
  if (rc) return rc;
  if (!batch || !bytes_out) return fail(ctx, VC_ERR_INVALID_ARG, "NULL argument");
  if (batch->count < 0 || (batch->count > 0 && (!batch->n || !batch->nnz)))
    return fail(ctx, VC_ERR_INVALID_ARG, "bad batch count, n or nnz");
  if (depth < 0) return fail(ctx, VC_ERR_INVALID_ARG, "depth must be >= 0");
  if ((rc = check_options(ctx, opts))) return rc;
  return workspace_need(ctx, batch->count, batch->n, batch->nnz, depth, opts, bytes_out);
}

int vc_mvc_device_ws(vc_ctx* ctx, const vc_graph* g, const vc_options* opts, void* workspace,
                     size_t workspace_bytes, int32_t* size_out, uint8_t* cover_dev,
                     vc_stats* stats) {
  int rc = enter(ctx);
  if (rc) return rc;
  if ((rc = check_workspace(ctx, workspace, workspace_bytes))) return rc;
  return solve(ctx, g, true, false, 0, opts, nullptr, size_out, cover_dev, nullptr, stats,
               WsArgs{workspace, workspace_bytes, true});
}

int vc_pvc_device_ws(vc_ctx* ctx, const vc_graph* g, int32_t k, const vc_options* opts,
                     void* workspace, size_t workspace_bytes, int32_t* yes_out,
                     int32_t* size_out, uint8_t* cover_dev, vc_stats* stats) {
  int rc = enter(ctx);
  if (rc) return rc;
  if ((rc = check_workspace(ctx, workspace, workspace_bytes))) return rc;
  return solve(ctx, g, true, true, k, opts, yes_out, size_out, cover_dev, nullptr, stats,
               WsArgs{workspace, workspace_bytes, true});
}

int vc_mvc_batch_device_ws(vc_ctx* ctx, const vc_batch* batch, const vc_options* opts,
                           void* workspace, size_t workspace_bytes, int32_t* status_out,
                           int32_t* size_out, uint8_t* cover_dev, int64_t* nodes_out,
                           vc_stats* stats) {
  int rc = enter(ctx);
  if (rc) return rc;
  if ((rc = check_workspace(ctx, workspace, workspace_bytes))) return rc;
  return solve_batch(ctx, batch, true, false, nullptr, opts, status_out, nullptr, size_out,
                     cover_dev, nullptr, nodes_out, stats, WsArgs{workspace, workspace_bytes, true});
}

int vc_pvc_batch_device_ws(vc_ctx* ctx, const vc_batch* batch, const int32_t* k,
                           const vc_options* opts, void* workspace, size_t workspace_bytes,
                           int32_t* status_out, int32_t* yes_out, int32_t* size_out,
                           uint8_t* cover_dev, int64_t* nodes_out, vc_stats* stats) {
  int rc = enter(ctx);
  if (rc) return rc;
  if ((rc = check_workspace(ctx, workspace, workspace_bytes))) return rc;
  return solve_batch(ctx, batch, true, true, k, opts, status_out, yes_out, size_out, cover_dev,
                     nullptr, nodes_out, stats, WsArgs{workspace, workspace_bytes, true});
}

int vc_greedy_device(vc_ctx* ctx, const vc_graph* g, int32_t* size_out, uint8_t* cover_dev) {
  int rc = enter(ctx);
  if (rc) return rc;
  if (!size_out) return fail(ctx, VC_ERR_INVALID_ARG, "size_out is NULL");
  if ((rc = check_graph_args(ctx, g))) return rc;
  if (g->n == 0) {
    *size_out = 0;
    return VC_OK;
  }
  Params p{};
  int32_t ws = 0;
  if ((rc = setup_single(ctx, g, vc::kRulesAll, 0, nullptr, p, &ws))) return rc;
  hipStream_t s = ctx->stream;
  if (p.words) VC_HIP(ctx, vc::launch_bitset_greedy(p, s));
  else VC_HIP(ctx, vc::launch_greedy(p, ws, s));
  InstState* h_is =
      reinterpret_cast<InstState*>(static_cast<char*>(ctx->pinned) + meta_layout(1, 1, 0).ist);
  VC_HIP(ctx, hipMemcpyAsync(h_is, p.ist, sizeof(InstState), hipMemcpyDeviceToHost, s));
  VC_HIP(ctx, hipStreamSynchronize(s));
  const InstState is = *h_is;
  if (is.err_row != vc::kNoRow) return fail(ctx, VC_ERR_INVALID_GRAPH, bad_row_message(is.err_row));
  if (cover_dev) {
    VC_HIP(ctx, hipMemcpyAsync(cover_dev, p.covers, static_cast<size_t>(g->n),
                               hipMemcpyDeviceToDevice, s));
    VC_HIP(ctx, hipStreamSynchronize(s));
  }
  *size_out = is.greedy;
  return VC_OK;
}

int vc_reduce_device(vc_ctx* ctx, const vc_graph* g, int32_t* deg_dev, int32_t* s_inout,
                     int64_t bound, int32_t flags) {
  int rc = enter(ctx);
  if (rc) return rc;
  if (!deg_dev || !s_inout) return fail(ctx, VC_ERR_INVALID_ARG, "NULL argument");
  if ((rc = check_graph_args(ctx, g))) return rc;
  vc_options o{};
  o.flags = flags;
  if ((rc = check_options(ctx, &o))) return rc;
  if (g->n == 0) return VC_OK;
  Params p{};
  int32_t ws = 0;
  if ((rc = setup_single(ctx, g, rules_from_flags(flags), flags, nullptr, p, &ws))) return rc;
  hipStream_t s = ctx->stream;
  if ((rc = ensure(ctx, ctx->scratch, sizeof(int32_t)))) return rc;
  int32_t* sdev = static_cast<int32_t*>(ctx->scratch.ptr);
  VC_HIP(ctx, hipMemcpyAsync(sdev, s_inout, sizeof(int32_t), hipMemcpyHostToDevice, s));
  if (p.words) VC_HIP(ctx, vc::launch_bitset_reduce(p, deg_dev, sdev, bound, s));
  else VC_HIP(ctx, vc::launch_reduce(p, ws, deg_dev, sdev, bound, s));
  InstState* h_is =
      reinterpret_cast<InstState*>(static_cast<char*>(ctx->pinned) + meta_layout(1, 1, 0).ist);
  int32_t s_new = 0;
  VC_HIP(ctx, hipMemcpyAsync(h_is, p.ist, sizeof(InstState), hipMemcpyDeviceToHost, s));
  VC_HIP(ctx, hipMemcpyAsync(&s_new, sdev, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  VC_HIP(ctx, hipStreamSynchronize(s));
  const InstState is = *h_is;
  if (is.err_row != vc::kNoRow) return fail(ctx, VC_ERR_INVALID_GRAPH, bad_row_message(is.err_row));
  *s_inout = s_new;
  return VC_OK;
}

}  // extern "C"
