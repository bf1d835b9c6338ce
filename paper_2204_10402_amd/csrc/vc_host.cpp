// vc_host.cpp -- host runtime of libvc.so: contexts, workspace, launch sizing and the C ABI
// declared in include/vc.h. Every step of the search runs in the HIP kernels of
// vc_device.hip; this file only checks arguments, sizes and allocates device memory, queues
// the kernels on the context stream and copies the small result block back.

#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <tuple>

#include "vc.h"
#include "vc_internal.h"

namespace {

struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
};

constexpr int32_t kNoRow = 0x7FFFFFFF;

}  // namespace

struct vc_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  hipDeviceProp_t prop{};
  size_t lds_limit_set = 0;
  DevBuf rp, ci, payload, seq, ctr, stacks, covers, wg_stats, result, cover_tmp, scratch_s, bits;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  std::string last_error;
  // occupancy-API answers: (kernel family, pvc, profiled, workgroup size, words, LDS bytes)
  std::map<std::tuple<int, int, int, int, int, size_t>, int> occupancy;
};

namespace {

using vc::DevResult;
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

// Grow-only device buffer.
int ensure(vc_ctx* ctx, DevBuf& b, size_t bytes) {
  if (bytes == 0) bytes = 256;
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
  for (int32_t r : o->reserved)
    if (r != 0) return fail(ctx, VC_ERR_INVALID_ARG, "vc_options.reserved must be zero");
  if (o->wg_size != 0 && (o->wg_size < 64 || o->wg_size > 1024 || o->wg_size % 64 != 0))
    return fail(ctx, VC_ERR_INVALID_ARG, "wg_size must be 0 or a multiple of 64 in [64, 1024]");
  if (o->num_wg < 0 || o->wl_capacity < 0 || o->wl_threshold < -1 || o->node_budget < 0)
    return fail(ctx, VC_ERR_INVALID_ARG, "negative option value");
  const int32_t known = VC_OPT_NO_DEGREE_ONE | VC_OPT_NO_TRIANGLE | VC_OPT_NO_HIGH_DEGREE |
                        VC_OPT_NO_EDGE_PRUNE | VC_OPT_PROFILE | VC_OPT_DEGREE_ARRAYS |
                        VC_OPT_BITSETS;
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
  int32_t max_wg = 0;  // workgroups the per-workgroup buffers are sized for
  int32_t stride = 0;
  int32_t cover_stride = 0;
  uint32_t cap = 0;
  uint32_t threshold = 0;
  size_t lds = 0;
  int32_t words = 0;  // > 0: bitset kernels with this many 64-bit words per node
  int32_t rp_lds = 0;  // degree-array kernels: row_ptr staged in LDS
};

// Resident workgroups per CU, from the occupancy API, remembered per context.
int occupancy(vc_ctx* ctx, int words, bool pvc, bool prof, int ws, size_t lds, int n, int* out) {
  const auto key = std::make_tuple(words ? 1 : 0, pvc ? 1 : 0, prof ? 1 : 0, ws, words, lds);
  const auto it = ctx->occupancy.find(key);
  if (it != ctx->occupancy.end()) {
    *out = it->second;
    return VC_OK;
  }
  if (words) VC_HIP(ctx, vc::bitset_occupancy(words, pvc, prof, n, out));
  else VC_HIP(ctx, vc::traverse_occupancy(pvc, prof, ws, lds, out));
  ctx->occupancy[key] = *out;
  return VC_OK;
}

// Bitset kernels up to 256 vertices unless the caller asks for degree arrays.
int choose_words(vc_ctx* ctx, int32_t n, int32_t flags, int32_t* words) {
  const bool force_bits = flags & VC_OPT_BITSETS;
  const bool force_arrays = flags & VC_OPT_DEGREE_ARRAYS;
  if (force_bits && n > vc::kMaxBitsetN)
    return fail(ctx, VC_ERR_INVALID_ARG, "VC_OPT_BITSETS needs n <= 256");
  *words = (!force_arrays && n <= vc::kMaxBitsetN) ? (std::max(n, 1) + 63) / 64 : 0;
  return VC_OK;
}

// Workgroup size and count (paper §IV-E, adapted): a power-of-two workgroup of about n/4
// threads; as many workgroups as can be resident at once (all must be, since they wait on
// each other), fewer if their stacks do not fit in device memory.
int plan_launch(vc_ctx* ctx, bool pvc, int32_t n, const vc_options* o, Plan& pl) {
  const bool prof = o && (o->flags & VC_OPT_PROFILE);
  int rc = choose_words(ctx, n, o ? o->flags : 0, &pl.words);
  if (rc) return rc;
  pl.cover_stride = static_cast<int32_t>(round_up(std::max<int64_t>(n, 1), 256));
  const int cus = ctx->prop.multiProcessorCount;
  int best_ws = 0, best_occ = 0;
  if (pl.words) {
    // one wavefront per workgroup; the adjacency matrix (n * words * 8 bytes) in LDS
    pl.stride = vc::bitset_stride(pl.words);
    pl.lds = vc::bitset_lds_bytes(n, pl.words);
    best_ws = 64;
    if (o && o->wg_size && o->wg_size != 64)
      return fail(ctx, VC_ERR_INVALID_ARG, "the bitset kernels use 64-thread workgroups");
    if ((rc = occupancy(ctx, pl.words, pvc, prof, 64, pl.lds, n, &best_occ))) return rc;
  } else {
    pl.stride = static_cast<int32_t>(round_up(static_cast<int64_t>(n) + 2, 64));
    pl.lds = vc::node_lds_bytes(pl.stride, n, false);
    const size_t lds_cap = static_cast<size_t>(ctx->prop.maxSharedMemoryPerMultiProcessor);
    if (pl.lds + 1024 > lds_cap)
      return fail(ctx, VC_ERR_INVALID_ARG,
                  "graph too large for the LDS-resident node (n = " + std::to_string(n) + ")");
    const size_t lds_rp = vc::node_lds_bytes(pl.stride, n, true);
    const size_t lds_max = lds_rp + 1024 <= lds_cap ? lds_rp : pl.lds;
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
      while (ws < 1024 && ws * 2 <= std::max(n, 1) / 4) ws *= 2;
      best_ws = ws;
    }
    if ((rc = occupancy(ctx, 0, pvc, prof, best_ws, pl.lds, n, &best_occ))) return rc;
    // Keep row_ptr in LDS too when that costs no resident workgroup.
    if (lds_rp + 1024 <= lds_cap) {
      int occ_rp = 0;
      if ((rc = occupancy(ctx, 0, pvc, prof, best_ws, lds_rp, n, &occ_rp))) return rc;
      if (occ_rp == best_occ) {
        pl.rp_lds = 1;
        pl.lds = lds_rp;
      }
    }
  }
  if (best_occ < 1)
    return fail(ctx, VC_ERR_INVALID_ARG, "traversal kernel cannot be resident at this size");
  pl.wg_size = best_ws;
  pl.num_wg = best_occ * cus;
  // Bitset nodes take a few microseconds each, so more than eight workgroups per CU only add
  // contention on the worklist counters (measured on the hard MVC instances).
  if (pl.words && !(o && o->num_wg > 0)) pl.num_wg = std::min(pl.num_wg, 8 * cus);
  if (o && o->num_wg > 0) pl.num_wg = std::min(pl.num_wg, o->num_wg);
  pl.max_wg = pl.num_wg;

  // Worklist: capacity and donation threshold (§IV-A). A producer only reserves a slot after
  // reading fewer than `threshold` reserved entries; at most num_wg producers can be past that
  // check at once, and consumers giving back a lost reservation can hide at most num_wg more,
  // so threshold + 2 * num_wg <= cap keeps every reservation inside the ring.
  uint64_t cap = o && o->wl_capacity ? static_cast<uint64_t>(o->wl_capacity)
                                     : std::max<uint64_t>(8ull * pl.num_wg, 4096);
  cap = std::max<uint64_t>(cap, 4ull * pl.num_wg);
  pl.cap = next_pow2(cap);
  uint64_t thr;
  if (o && o->wl_threshold == -1) thr = 0;
  else if (o && o->wl_threshold > 0) thr = static_cast<uint64_t>(o->wl_threshold);
  else thr = std::max<uint64_t>(64, static_cast<uint64_t>(pl.num_wg) / 4);
  thr = std::min<uint64_t>(thr, pl.cap - 2ull * static_cast<uint64_t>(pl.num_wg));
  pl.threshold = static_cast<uint32_t>(thr);
  return VC_OK;
}

// Shrink the grid so that num_wg stacks of depth_cap nodes fit in free device memory
// (§IV-E: the stacks bound the number of workgroups), then make sure they are allocated.
int size_stacks(vc_ctx* ctx, Plan& pl, int32_t depth_cap) {
  const size_t per_wg = static_cast<size_t>(depth_cap) * pl.stride * sizeof(int32_t);
  if (per_wg * static_cast<size_t>(pl.num_wg) <= ctx->stacks.bytes) return VC_OK;
  size_t free_b = 0, total_b = 0;
  VC_HIP(ctx, hipMemGetInfo(&free_b, &total_b));
  const size_t avail = ctx->stacks.bytes + (free_b > (size_t(1) << 30) ? free_b - (size_t(1) << 30) : 0);
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

// The whole search on a graph whose CSR already sits in device memory.
int run_search(vc_ctx* ctx, const vc_graph* g, bool pvc, int64_t k, const vc_options* o,
               int32_t* size_out, int32_t* yes_out, uint8_t* cover_dev, uint8_t* cover_host,
               vc_stats* stats, std::chrono::steady_clock::time_point t0) {
  const int32_t n = g->n;
  Plan pl;
  int rc = plan_launch(ctx, pvc, n, o, pl);
  if (rc) return rc;
  const size_t stride_b = static_cast<size_t>(pl.stride) * sizeof(int32_t);
  if ((rc = ensure(ctx, ctx->payload, static_cast<size_t>(pl.cap) * stride_b))) return rc;
  if ((rc = ensure(ctx, ctx->seq, static_cast<size_t>(pl.cap) * sizeof(uint32_t)))) return rc;
  if ((rc = ensure(ctx, ctx->ctr, vc::kNumCounters * vc::kCounterStride * sizeof(int32_t)))) return rc;
  if ((rc = ensure(ctx, ctx->covers, static_cast<size_t>(pl.max_wg + 1) * pl.cover_stride))) return rc;
  if ((rc = ensure(ctx, ctx->wg_stats, static_cast<size_t>(pl.max_wg) * sizeof(vc::WgStats)))) return rc;
  if ((rc = ensure(ctx, ctx->result, sizeof(DevResult)))) return rc;
  if ((rc = ensure(ctx, ctx->cover_tmp, static_cast<size_t>(std::max(n, 1))))) return rc;

  Params p{};
  p.n = n;
  p.stride = pl.stride;
  p.nnz = g->nnz;
  p.rules = rules_from_flags(o ? o->flags : 0);
  p.rp = g->row_ptr;
  p.ci = g->col_idx;
  p.payload = static_cast<int32_t*>(ctx->payload.ptr);
  p.seq = static_cast<uint32_t*>(ctx->seq.ptr);
  p.ctr = static_cast<int32_t*>(ctx->ctr.ptr);
  p.covers = static_cast<uint8_t*>(ctx->covers.ptr);
  p.wg_stats = static_cast<vc::WgStats*>(ctx->wg_stats.ptr);
  p.k = k;
  p.node_budget = o ? o->node_budget : 0;
  // report often enough that the whole grid overshoots the budget by at most about half
  p.budget_chunk = std::max<int64_t>(1, std::min<int64_t>(1024, p.node_budget / (2 * pl.num_wg)));
  p.q_cap = pl.cap;
  p.q_threshold = pl.threshold;
  p.num_wg = pl.num_wg;
  p.greedy_slot = pl.max_wg;
  p.cover_stride = pl.cover_stride;
  p.words = pl.words;
  p.rp_lds = pl.rp_lds;
  if (pl.words) {
    if ((rc = ensure(ctx, ctx->bits, static_cast<size_t>(n) * pl.words * sizeof(uint64_t)))) return rc;
    p.bits = static_cast<uint64_t*>(ctx->bits.ptr);
  }
  DevResult* dres = static_cast<DevResult*>(ctx->result.ptr);
  hipStream_t s = ctx->stream;

  VC_HIP(ctx, vc::launch_init(p, dres, s));
  VC_HIP(ctx, vc::launch_prepare(p, s));
  if (pl.words) VC_HIP(ctx, vc::launch_bitset_pack(p, s));

  DevResult res{};
  int32_t depth_cap;
  float greedy_ms = 0.f;
  if (!pvc) {
    const int gws = static_cast<int>(std::min<int64_t>(1024, round_up(std::max(n, 1), 64)));
    VC_HIP(ctx, hipEventRecord(ctx->ev[2], s));
    if (pl.words) VC_HIP(ctx, vc::launch_bitset_greedy(p, dres, s));
    else VC_HIP(ctx, vc::launch_greedy(p, gws, dres, s));
    VC_HIP(ctx, hipEventRecord(ctx->ev[3], s));
    VC_HIP(ctx, hipMemcpyAsync(&res, dres, sizeof res, hipMemcpyDeviceToHost, s));
    VC_HIP(ctx, hipStreamSynchronize(s));
    VC_HIP(ctx, hipEventElapsedTime(&greedy_ms, ctx->ev[2], ctx->ev[3]));
    if (res.err_row != kNoRow)
      return fail(ctx, VC_ERR_INVALID_GRAPH,
                  "CSR row " + std::to_string(res.err_row) +
                      " breaks the format (bounds, order, self-loop, duplicate or symmetry)");
    if (res.edges0 == 0) {  // edgeless: the empty set is the minimum cover
      if (cover_dev) VC_HIP(ctx, hipMemsetAsync(cover_dev, 0, static_cast<size_t>(n), s));
      VC_HIP(ctx, hipStreamSynchronize(s));
      if (cover_host) std::memset(cover_host, 0, static_cast<size_t>(n));
      *size_out = 0;
      if (stats) {
        std::memset(stats, 0, sizeof *stats);
        stats->greedy_size = 0;
        stats->n = n;
        stats->greedy_ms = greedy_ms;
        stats->total_ms = ms_since(t0);
      }
      return VC_OK;
    }
    // bound = best - 1: a path branches at most best - 1 times (each branching adds to s)
    depth_cap = std::max(res.greedy, 1);
  } else {
    depth_cap = static_cast<int32_t>(std::min<int64_t>(k, n)) + 1;
  }
  if ((rc = size_stacks(ctx, pl, depth_cap))) return rc;
  p.stacks = static_cast<int32_t*>(ctx->stacks.ptr);
  p.depth_cap = depth_cap;
  p.num_wg = pl.num_wg;

  VC_HIP(ctx, hipEventRecord(ctx->ev[0], s));
  const bool prof = o && (o->flags & VC_OPT_PROFILE);
  if (pl.words) VC_HIP(ctx, vc::launch_bitset_traverse(pvc, prof, p, s));
  else VC_HIP(ctx, vc::launch_traverse(pvc, prof, p, pl.wg_size, s));
  VC_HIP(ctx, hipEventRecord(ctx->ev[1], s));
  uint8_t* cover_dst = cover_dev ? cover_dev : static_cast<uint8_t*>(ctx->cover_tmp.ptr);
  VC_HIP(ctx, vc::launch_finalize(pvc, p, cover_dst, dres, s));
  VC_HIP(ctx, hipMemcpyAsync(&res, dres, sizeof res, hipMemcpyDeviceToHost, s));
  if (cover_host && n > 0)
    VC_HIP(ctx, hipMemcpyAsync(cover_host, cover_dst, static_cast<size_t>(n),
                               hipMemcpyDeviceToHost, s));
  VC_HIP(ctx, hipStreamSynchronize(s));
  float kernel_ms = 0.f;
  VC_HIP(ctx, hipEventElapsedTime(&kernel_ms, ctx->ev[0], ctx->ev[1]));

  if (res.err_row != kNoRow)
    return fail(ctx, VC_ERR_INVALID_GRAPH,
                "CSR row " + std::to_string(res.err_row) +
                    " breaks the format (bounds, order, self-loop, duplicate or symmetry)");
  if (res.error)
    return fail(ctx, VC_ERR_INTERNAL, "device invariant failed (code " +
                                          std::to_string(res.error) + ": stack overflow)");
  if (res.aborted) return fail(ctx, VC_ERR_BUDGET, "node budget exhausted");
  if (pvc && res.yes) res.size = res.cover_count;  // PVC reports the size of the cover found
  if (res.yes) {
    if (res.uncovered != 0 || res.cover_count != res.size)
      return fail(ctx, VC_ERR_INTERNAL,
                  "returned cover failed verification: " + std::to_string(res.uncovered) +
                      " uncovered edge entries, " + std::to_string(res.cover_count) +
                      " vertices for size " + std::to_string(res.size));
    if (pvc && res.size > k)
      return fail(ctx, VC_ERR_INTERNAL, "PVC cover larger than k");
  }
  *size_out = res.size;
  if (yes_out) *yes_out = res.yes;
  if (stats) {
    std::memset(stats, 0, sizeof *stats);
    stats->nodes = res.nodes;
    stats->wg_nodes_max = res.wg_nodes_max;
    stats->wg_nodes_min = res.wg_nodes_min;
    stats->stack_pushes = res.pushes;
    stats->stack_pops = res.pops;
    stats->wl_enqueues = res.enqueues;
    stats->wl_dequeues = res.dequeues;
    stats->max_stack_depth = res.max_depth;
    stats->greedy_size = pvc ? -1 : res.greedy;
    stats->wg_size = pl.wg_size;
    stats->num_wg = pl.num_wg;
    stats->wl_capacity = static_cast<int32_t>(pl.cap);
    stats->wl_threshold = static_cast<int32_t>(pl.threshold);
    stats->depth_cap = depth_cap;
    stats->n = n;
    stats->bitset_words = pl.words;
    stats->node_bytes = pl.words ? 8 * pl.words + 8 : 4 * (n + 2);
    stats->kernel_ms = kernel_ms;
    for (int a = 0; a < vc::kNumActivities; ++a) stats->cycles[a] = res.cycles[a];
    stats->greedy_ms = greedy_ms;
    stats->total_ms = ms_since(t0);
  }
  return VC_OK;
}

// Copy a host CSR into the context's device buffers.
int upload(vc_ctx* ctx, const vc_graph* g, vc_graph* dev) {
  int rc;
  if ((rc = ensure(ctx, ctx->rp, (static_cast<size_t>(g->n) + 1) * sizeof(int32_t)))) return rc;
  if ((rc = ensure(ctx, ctx->ci, static_cast<size_t>(std::max(g->nnz, 1)) * sizeof(int32_t)))) return rc;
  VC_HIP(ctx, hipMemcpyAsync(ctx->rp.ptr, g->row_ptr, (static_cast<size_t>(g->n) + 1) * sizeof(int32_t),
                             hipMemcpyHostToDevice, ctx->stream));
  if (g->nnz > 0)
    VC_HIP(ctx, hipMemcpyAsync(ctx->ci.ptr, g->col_idx, static_cast<size_t>(g->nnz) * sizeof(int32_t),
                               hipMemcpyHostToDevice, ctx->stream));
  dev->n = g->n;
  dev->nnz = g->nnz;
  dev->row_ptr = static_cast<const int32_t*>(ctx->rp.ptr);
  dev->col_idx = static_cast<const int32_t*>(ctx->ci.ptr);
  return VC_OK;
}

int enter(vc_ctx* ctx) {
  if (!ctx) return VC_ERR_INVALID_ARG;
  ctx->last_error.clear();
  VC_HIP(ctx, hipSetDevice(ctx->device));
  return VC_OK;
}

int solve(vc_ctx* ctx, const vc_graph* g, bool device_graph, bool pvc, int64_t k,
          const vc_options* o, int32_t* yes_out, int32_t* size_out, uint8_t* cover_dev,
          uint8_t* cover_host, vc_stats* stats) {
  const auto t0 = std::chrono::steady_clock::now();
  int rc = enter(ctx);
  if (rc) return rc;
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
  vc_graph dev = *g;
  if (!device_graph && (rc = upload(ctx, g, &dev))) return rc;
  return run_search(ctx, &dev, pvc, k, o, size_out, yes_out, cover_dev, cover_host, stats, t0);
}

// Validate a device CSR and stage its root node for a one-workgroup kernel (greedy, reduce).
int setup_single(vc_ctx* ctx, const vc_graph* g, int rules, int32_t flags, Params& p) {
  Plan pl;
  vc_options o{};
  o.flags = flags & (VC_OPT_DEGREE_ARRAYS | VC_OPT_BITSETS);
  int rc = plan_launch(ctx, false, g->n, &o, pl);
  if (rc) return rc;
  if ((rc = ensure(ctx, ctx->payload, static_cast<size_t>(pl.stride) * sizeof(int32_t)))) return rc;
  if ((rc = ensure(ctx, ctx->seq, sizeof(uint32_t)))) return rc;
  if ((rc = ensure(ctx, ctx->ctr, vc::kNumCounters * vc::kCounterStride * sizeof(int32_t)))) return rc;
  if ((rc = ensure(ctx, ctx->covers, static_cast<size_t>(pl.cover_stride)))) return rc;
  if ((rc = ensure(ctx, ctx->result, sizeof(DevResult)))) return rc;
  p = Params{};
  p.n = g->n;
  p.stride = pl.stride;
  p.nnz = g->nnz;
  p.rules = rules;
  p.rp = g->row_ptr;
  p.ci = g->col_idx;
  p.payload = static_cast<int32_t*>(ctx->payload.ptr);
  p.seq = static_cast<uint32_t*>(ctx->seq.ptr);
  p.ctr = static_cast<int32_t*>(ctx->ctr.ptr);
  p.covers = static_cast<uint8_t*>(ctx->covers.ptr);
  p.q_cap = 1;
  p.cover_stride = pl.cover_stride;
  p.words = pl.words;
  p.rp_lds = pl.rp_lds;
  if (pl.words) {
    if ((rc = ensure(ctx, ctx->bits, static_cast<size_t>(g->n) * pl.words * sizeof(uint64_t)))) return rc;
    p.bits = static_cast<uint64_t*>(ctx->bits.ptr);
  }
  DevResult* dres = static_cast<DevResult*>(ctx->result.ptr);
  VC_HIP(ctx, vc::launch_init(p, dres, ctx->stream));
  VC_HIP(ctx, vc::launch_prepare(p, ctx->stream));
  if (pl.words) VC_HIP(ctx, vc::launch_bitset_pack(p, ctx->stream));
  return VC_OK;
}

}  // namespace

extern "C" {

const char* vc_version(void) { return "0.1.0"; }

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
  for (int i = 0; i < 4 && e == hipSuccess; ++i) e = hipEventCreate(&ctx->ev[i]);
  if (e != hipSuccess) {
    vc_destroy(ctx);
    return VC_ERR_DEVICE;
  }
  *ctx_out = ctx;
  return VC_OK;
}

int vc_destroy(vc_ctx* ctx) {
  if (!ctx) return VC_OK;
  (void)hipSetDevice(ctx->device);
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  DevBuf* bufs[] = {&ctx->rp,     &ctx->ci,       &ctx->payload, &ctx->seq,
                    &ctx->ctr,    &ctx->stacks,   &ctx->covers,  &ctx->wg_stats,
                    &ctx->result, &ctx->cover_tmp, &ctx->scratch_s, &ctx->bits};
  for (DevBuf* b : bufs)
    if (b->ptr) (void)hipFree(b->ptr);
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

int vc_greedy_device(vc_ctx* ctx, const vc_graph* g, int32_t* size_out, uint8_t* cover_dev) {
  int rc = enter(ctx);
  if (rc) return rc;
  if (!size_out) return fail(ctx, VC_ERR_INVALID_ARG, "size_out is NULL");
  if ((rc = check_graph_args(ctx, g))) return rc;
  const int32_t n = g->n;
  if (n == 0) {
    *size_out = 0;
    return VC_OK;
  }
  Params p{};
  if ((rc = setup_single(ctx, g, vc::kRulesAll, 0, p))) return rc;
  DevResult* dres = static_cast<DevResult*>(ctx->result.ptr);
  hipStream_t s = ctx->stream;
  const int gws = static_cast<int>(std::min<int64_t>(1024, round_up(n, 64)));
  if (p.words) VC_HIP(ctx, vc::launch_bitset_greedy(p, dres, s));
  else VC_HIP(ctx, vc::launch_greedy(p, gws, dres, s));
  DevResult res{};
  VC_HIP(ctx, hipMemcpyAsync(&res, dres, sizeof res, hipMemcpyDeviceToHost, s));
  VC_HIP(ctx, hipStreamSynchronize(s));
  if (res.err_row != kNoRow)
    return fail(ctx, VC_ERR_INVALID_GRAPH, "CSR row " + std::to_string(res.err_row) +
                                               " breaks the format");
  if (cover_dev) {
    VC_HIP(ctx, hipMemcpyAsync(cover_dev, p.covers, static_cast<size_t>(n),
                               hipMemcpyDeviceToDevice, s));
    VC_HIP(ctx, hipStreamSynchronize(s));
  }
  *size_out = res.greedy;
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
  const int32_t n = g->n;
  if (n == 0) return VC_OK;
  Params p{};
  if ((rc = setup_single(ctx, g, rules_from_flags(flags), flags, p))) return rc;
  if ((rc = ensure(ctx, ctx->scratch_s, sizeof(int32_t)))) return rc;
  DevResult* dres = static_cast<DevResult*>(ctx->result.ptr);
  hipStream_t s = ctx->stream;
  int32_t* sdev = static_cast<int32_t*>(ctx->scratch_s.ptr);
  VC_HIP(ctx, hipMemcpyAsync(sdev, s_inout, sizeof(int32_t), hipMemcpyHostToDevice, s));
  const int ws = static_cast<int>(std::min<int64_t>(1024, round_up(n, 64)));
  if (p.words) VC_HIP(ctx, vc::launch_bitset_reduce(p, deg_dev, sdev, bound, dres, s));
  else VC_HIP(ctx, vc::launch_reduce(p, ws, deg_dev, sdev, bound, dres, s));
  DevResult res{};
  int32_t s_new = 0;
  VC_HIP(ctx, hipMemcpyAsync(&res, dres, sizeof res, hipMemcpyDeviceToHost, s));
  VC_HIP(ctx, hipMemcpyAsync(&s_new, sdev, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  VC_HIP(ctx, hipStreamSynchronize(s));
  if (res.err_row != kNoRow)
    return fail(ctx, VC_ERR_INVALID_GRAPH, "CSR row " + std::to_string(res.err_row) +
                                               " breaks the format");
  *s_inout = s_new;
  return VC_OK;
}

}  // extern "C"
