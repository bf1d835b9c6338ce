// vc_device.hip -- HIP kernels for gfx950 (MI355X) of the hybrid vertex-cover traversal.
//
// Method (paper §IV): a persistent grid; every workgroup walks a sub-tree of the
// branch-and-reduce search tree depth first with its own stack in device memory, and hands
// branches to a global worklist while the worklist holds fewer entries than a threshold
// (§IV-A). An intermediate graph is a degree array over one read-only CSR (§IV-B): one int32
// per vertex holding its degree, or -1 once the vertex is in the cover, followed by the cover
// size s (the |S| counter of §IV-B) and a pending branch vertex (see below).
//
// gfx950 mapping:
//  - the node being worked on lives in LDS; every rule pass, the max-degree search and the
//    vertex removals read and update it there (LDS atomics for degree decrements);
//  - vertices are processed in 64-vertex chunks, one chunk per wavefront at a time; a
//    ballot over the chunk yields the candidates, and each candidate's CSR row is then
//    scanned by the whole wavefront (coalesced 64-wide loads from the L2-resident CSR);
//  - the maximum-degree vertex and the degree sum come from one pass reduced with DPP row
//    operations inside each wavefront and one LDS step across wavefronts;
//  - a deferred child is stored as its parent's reduced degree array plus the vertex whose
//    neighbourhood it removes (the "pending" vertex); the removal is done in LDS by whoever
//    takes the child, so a branch costs one plain copy of the node out and one copy back in,
//    and no global-memory atomics touch node data;
//  - the worklist is a bounded ring of node slots with per-slot lap tickets; producers and
//    consumers synchronise through agent-scope atomics, so a node written on one XCD is seen
//    correctly by a workgroup on another;
//  - termination: a counter of outstanding sub-trees (queued, or held by a workgroup) is
//    raised before a node is published and lowered when a workgroup has finished the whole
//    sub-tree it took; the search is over when it reads zero (§IV-C).
//
// Rule semantics (paper §II-B, parallel tie-breaks §IV-D): each rule is one pass that decides
// from the degree array as it stood at the start of the pass (decisions are marked with a
// flag bit that leaves the degree bits untouched), then removes every marked vertex at once.
// The passes run degree-one, degree-two-triangle, high-degree, and repeat until a whole round
// changes nothing or s exceeds the bound.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vc_device_common.h"
#include "vc_internal.h"

namespace vc {

constexpr int32_t kFlag = 0x40000000;     // "decided this pass" mark on a live entry
constexpr int32_t kDegMask = 0x3FFFFFFF;  // degree bits of a live entry

// ---- node operations on the LDS degree array -------------------------------------------------
// st[0..n) degrees (kSent = in cover), st[n] = s, st[n+1] = pending vertex (-1 = none).

struct Node {
  int32_t* st;
  int n;
  const int32_t* __restrict__ rp;
  const int32_t* __restrict__ ci;
  int32_t* heads;  // 64 LDS words per wavefront for wave_expand_rows
};

// Inclusive max-scan over the 64 lanes (DPP, as wave_incl_scan), identity -1.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ int32_t dpp_or_minus1(int32_t x) {
  return __builtin_amdgcn_update_dpp(-1, x, CTRL, ROW_MASK, 0xF, false);
}
__device__ __forceinline__ int32_t wave_incl_max(int32_t x) {
  x = max(x, dpp_or_minus1<0x111, 0xF>(x));
  x = max(x, dpp_or_minus1<0x112, 0xF>(x));
  x = max(x, dpp_or_minus1<0x114, 0xF>(x));
  x = max(x, dpp_or_minus1<0x118, 0xF>(x));
  x = max(x, dpp_or_minus1<0x142, 0xA>(x));
  x = max(x, dpp_or_minus1<0x143, 0xC>(x));
  return x;
}

// Walk the CSR rows [beg, end) held by the lanes of a wavefront (empty where beg >= end) as one
// list, 64 consecutive entries per step, so rows of any length keep every lane busy and
// neighbouring lanes read neighbouring entries. fn(x, tag) runs for every entry x = ci[j], with
// `tag` the value the row's owner lane passed in. The owner of each entry of a step comes from
// head flags: every row writes its lane into `heads` (this wavefront's 64 LDS words) at its
// first position in the step, and a max-scan over the lanes carries it forward. Eight steps
// are issued together, with unconditional loads (an index past the list reads entry 0, whose
// value is discarded), so eight loads are in flight before the first is used.
template <typename Fn>
__device__ __forceinline__ void wave_expand_rows(const int32_t* __restrict__ ci, int32_t* heads,
                                                 int beg, int end, int tag, Fn fn) {
  const int lane = lane_id();
  const int len = end > beg ? end - beg : 0;
  const int incl = wave_incl_scan(len);
  const int excl = incl - len;
  const int total = __builtin_amdgcn_readlane(incl, 63);
  constexpr int kUnroll = 8;
  for (int t0 = 0; t0 < total; t0 += 64 * kUnroll) {
    int xs[kUnroll], tags[kUnroll];
    bool ok[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      ok[u] = false;
      const int s0 = t0 + u * 64;
      if (s0 < total) {  // uniform: only as many steps as the rows need
        heads[lane] = -1;
        __builtin_amdgcn_wave_barrier();
        if (len > 0 && excl < s0 + 64 && incl > s0) heads[excl > s0 ? excl - s0 : 0] = lane;
        __builtin_amdgcn_wave_barrier();
        const int i = wave_incl_max(heads[lane]);  // owner of entry s0 + lane
        __builtin_amdgcn_wave_barrier();
        const int t = s0 + lane;
        const int src = i < 0 ? 0 : i;  // i < 0 only past the end of the list
        const int ob = shfl(beg, src);
        const int oe = shfl(excl, src);
        tags[u] = shfl(tag, src);
        ok[u] = t < total;
        xs[u] = ci[ok[u] ? ob + (t - oe) : 0];  // not read until every step has issued
      }
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u)
      if (ok[u]) fn(xs[u], tags[u]);
  }
}

// Collect the vertices of this wavefront's 64-vertex chunks that satisfy pred(v, d) into
// batches of up to 64, one candidate per lane, and hand each batch to process(cand, count)
// (lanes < count hold a candidate). Whole wavefront, uniform control flow.
template <typename Pred, typename Proc>
__device__ __forceinline__ void for_each_batch(const int32_t* st, int n, Pred pred, Proc process) {
  const int lane = lane_id();
  int held = -1;
  int count = 0;
  for (int base = wave_id() * 64; base < n; base += blockDim.x) {
    const int v = base + lane;
    const int32_t d = v < n ? st[v] : kSent;
    const uint64_t mask = __builtin_amdgcn_ballot_w64(v < n && pred(v, d));
    if (!mask) continue;
    const int cnt = __popcll(mask);
    if (count + cnt > 64) {
      process(held, count);
      held = -1;
      count = 0;
    }
    const int k = lane - count;
    const bool take = k >= 0 && k < cnt;
    const int got = shfl(v, take ? kth_set_bit(mask, k) : lane);
    if (take) held = got;
    count += cnt;
  }
  if (count) process(held, count);
}

// Remove every marked vertex (paper §IV-B): each live unmarked neighbour of a marked vertex
// loses one degree per marked neighbour, then marked vertices become kSent and s grows by
// their number. Called right after a barrier that ends a decide step.
__device__ void apply_marks(const Node nd) {
  const int n = nd.n;
  int32_t* st = nd.st;
  for_each_batch(st, n, [](int, int32_t d) { return d >= 0 && (d & kFlag); },
                 [&](int f, int count) {
                   const bool mine = lane_id() < count;
                   wave_expand_rows(nd.ci, nd.heads + 64 * wave_id(), mine ? nd.rp[f] : 0,
                                    mine ? nd.rp[f + 1] : 0, f,
                                    [&](int x, int) {
                                      const int32_t dx = st[x];
                                      if (dx >= 0 && !(dx & kFlag)) atomicSub(&st[x], 1);
                                    });
                 });
  __syncthreads();
  int cnt = 0;
  for (int v = threadIdx.x; v < n; v += blockDim.x) {
    const int32_t d = st[v];
    if (d >= 0 && (d & kFlag)) {
      st[v] = kSent;
      ++cnt;
    }
  }
  cnt = wave_sum(cnt);
  if (lane_id() == 0 && cnt) atomicAdd(&st[n], cnt);
  __syncthreads();
}

// Degree-one rule (§II-B): v with one live neighbour u puts u in the cover; of two adjacent
// degree-one vertices only the smaller id is removed, and a shared neighbour once (§IV-D).
// The rows of all degree-one vertices are walked together; the one live entry of a row names
// u, and the lane that reads it makes the decision for that row's owner.
__device__ void decide_degree_one(const Node nd, Ctrl& c, int epoch) {
  int32_t* st = nd.st;
  for_each_batch(st, nd.n, [](int, int32_t d) { return d >= 0 && (d & kDegMask) == 1; },
                 [&](int cv, int count) {
                   const bool mine = lane_id() < count;
                   wave_expand_rows(nd.ci, nd.heads + 64 * wave_id(), mine ? nd.rp[cv] : 0,
                                    mine ? nd.rp[cv + 1] : 0, cv,
                                    [&](int u, int v) {
                                      const int32_t du = st[u];
                                      if (du < 0) return;  // not the live neighbour of v
                                      if ((du & kDegMask) != 1 || u < v) {
                                        atomicOr(&st[u], kFlag);
                                        c.flag_epoch = epoch;
                                      }
                                    });
                 });
}

// Is `key` in the sorted CSR segment ci[lo, hi)? An 8-ary search: each round reads seven
// evenly spaced entries at once and keeps the part that can hold the key, so a row of 125
// entries takes three rounds of independent loads instead of seven dependent ones.
__device__ __forceinline__ bool row_contains(const int32_t* __restrict__ ci, int lo, int hi,
                                             int key) {
  while (hi - lo > 8) {
    const int step = (hi - lo + 7) >> 3;
    int probe[7];
#pragma unroll
    for (int i = 0; i < 7; ++i) {
      const int at = lo + (i + 1) * step;
      probe[i] = at < hi ? ci[at] : 0x7FFFFFFF;
    }
    int below = 0;  // probes that are <= key
#pragma unroll
    for (int i = 0; i < 7; ++i) below += probe[i] <= key;
    const int nlo = lo + below * step;
    const int nhi = nlo + step < hi ? nlo + step : hi;
    lo = nlo;
    hi = nhi;
  }
  bool hit = false;
#pragma unroll
  for (int i = 0; i < 8; ++i) hit |= lo + i < hi && ci[lo + i] == key;
  return hit;
}

// Degree-two-triangle rule (§II-B): v with live neighbours u, w and uw an edge puts u and w in
// the cover; among degree-two vertices of one triangle only the smallest id fires (§IV-D).
// Each lane takes one degree-two vertex: it finds the two live neighbours in its own row (rows
// longer than kLaneRow are searched by the whole wavefront), then searches the shorter of the
// two neighbours' rows for the other.
__device__ void decide_triangle(const Node nd, Ctrl& c, int epoch) {
  constexpr int kLaneRow = 32;
  int32_t* st = nd.st;
  const int lane = lane_id();
  for_each_batch(st, nd.n, [](int, int32_t d) { return d >= 0 && (d & kDegMask) == 2; },
                 [&](int cv, int count) {
                   const bool mine = lane < count;
                   const int beg = mine ? nd.rp[cv] : 0, end = mine ? nd.rp[cv + 1] : 0;
                   int a = -1, b = -1;
                   if (mine && end - beg <= kLaneRow) {
                     for (int j = beg; j < end && b < 0; j += 8) {
                       int x[8];
#pragma unroll
                       for (int u = 0; u < 8; ++u) x[u] = j + u < end ? nd.ci[j + u] : -1;
#pragma unroll
                       for (int u = 0; u < 8; ++u) {
                         if (x[u] >= 0 && b < 0 && st[x[u]] >= 0) {
                           if (a < 0) a = x[u]; else b = x[u];
                         }
                       }
                     }
                   }
                   // long rows: the whole wavefront scans one row at a time
                   uint64_t longs = __builtin_amdgcn_ballot_w64(mine && end - beg > kLaneRow);
                   while (longs) {
                     const int owner = first_lane(longs);
                     longs &= longs - 1;
                     const int rb = __builtin_amdgcn_readlane(beg, owner);
                     const int re = __builtin_amdgcn_readlane(end, owner);
                     int fa = -1, fb = -1;
                     for (int j = rb; j < re && fb < 0; j += 64) {
                       const int x = j + lane < re ? nd.ci[j + lane] : -1;
                       uint64_t live = __builtin_amdgcn_ballot_w64(x >= 0 && st[x] >= 0);
                       while (live && fb < 0) {
                         const int y = bcast(x, first_lane(live));
                         live &= live - 1;
                         if (fa < 0) fa = y; else fb = y;
                       }
                     }
                     if (lane == owner) {
                       a = fa;
                       b = fb;
                     }
                   }
                   if (b < 0) return;  // no candidate in this lane
                   // is b in row a? search the shorter of the two sorted rows
                   const int ab = nd.rp[a], ae = nd.rp[a + 1];
                   const int bb = nd.rp[b], be = nd.rp[b + 1];
                   const bool in_a = ae - ab <= be - bb;
                   if (!row_contains(nd.ci, in_a ? ab : bb, in_a ? ae : be, in_a ? b : a)) return;
                   const int32_t da = st[a] & kDegMask, db = st[b] & kDegMask;
                   if ((da == 2 && a < cv) || (db == 2 && b < cv)) return;
                   atomicOr(&st[a], kFlag);
                   atomicOr(&st[b], kFlag);
                   c.flag_epoch = epoch;
                 });
}

// High-degree rule (§II-B): a vertex whose degree exceeds r = bound - s is in every cover of
// size <= bound (bound = best - 1 for MVC, k for PVC).
__device__ void decide_high_degree(const Node nd, Ctrl& c, int epoch, int64_t r) {
  int32_t* st = nd.st;
  for (int v = threadIdx.x; v < nd.n; v += blockDim.x) {
    const int32_t d = st[v];
    if (d >= 0 && static_cast<int64_t>(d & kDegMask) > r) {
      st[v] = d | kFlag;
      c.flag_epoch = epoch;
    }
  }
}

// No-op activity clock for the uninstrumented callers.
struct NoClock {
  __device__ void charge(int) {}
};

// The reduction rules until the graph stops changing (§II-B, §IV-D), or until s > bound.
// Precondition: the node in LDS is consistent and visible to the whole workgroup.
template <typename Clock>
__device__ void reduce_node(const Node nd, Ctrl& c, int64_t bound, int rules, int& epoch,
                            Clock& clk) {
  const int n = nd.n;
  int32_t* st = nd.st;
  for (;;) {
    const int32_t s0 = st[n];
    if (s0 > bound) return;
    if (rules & kRuleDeg1) {
      ++epoch;
      decide_degree_one(nd, c, epoch);
      __syncthreads();
      clk.charge(kActDeg1);
      if (c.flag_epoch == epoch) {
        apply_marks(nd);
        clk.charge(kActApply);
        if (st[n] > bound) return;
      }
    }
    if (rules & kRuleTri) {
      ++epoch;
      decide_triangle(nd, c, epoch);
      __syncthreads();
      clk.charge(kActTri);
      if (c.flag_epoch == epoch) {
        apply_marks(nd);
        clk.charge(kActApply);
        if (st[n] > bound) return;
      }
    }
    if (rules & kRuleHigh) {
      ++epoch;
      decide_high_degree(nd, c, epoch, bound - st[n]);
      __syncthreads();
      clk.charge(kActHigh);
      if (c.flag_epoch == epoch) {
        apply_marks(nd);
        clk.charge(kActApply);
      }
    }
    if (st[n] == s0) return;
  }
}

__device__ void reduce_node(const Node nd, Ctrl& c, int64_t bound, int rules, int& epoch) {
  NoClock none;
  reduce_node(nd, c, bound, rules, epoch, none);
}

// One pass over the degree array: the sum of live degrees (= 2|E|) and the live vertex of
// maximum degree, smallest id on ties (§IV-B). Results are the same in every thread.
__device__ void max_degree_and_sum(const Node nd, Ctrl& c, int& vmax, int& dmax,
                                   int32_t& degsum) {
  const int n = nd.n;
  const int32_t* st = nd.st;
  uint64_t key = 0;
  int32_t sum = 0;
  for (int v = threadIdx.x; v < n; v += blockDim.x) {
    const int32_t d = st[v];
    if (d >= 0) {
      sum += d;
      key = umax64(key, (static_cast<uint64_t>(static_cast<uint32_t>(d)) << 32) |
                            static_cast<uint32_t>(~static_cast<uint32_t>(v)));
    }
  }
  key = wave_max(key);
  sum = wave_sum(sum);
  if (lane_id() == 0) {
    c.red_key[wave_id()] = key;
    c.red_sum[wave_id()] = sum;
  }
  __syncthreads();
  key = 0;
  sum = 0;
  const int waves = blockDim.x >> 6;
  for (int w = 0; w < waves; ++w) {
    key = umax64(key, c.red_key[w]);
    sum += c.red_sum[w];
  }
  vmax = static_cast<int>(~static_cast<uint32_t>(key));
  dmax = static_cast<int>(key >> 32);
  degsum = sum;
}

// Mark every live neighbour of v (the "N(v) in the cover" child, §II-B) and remove them.
__device__ void remove_neighbourhood(const Node nd, int v) {
  int32_t* st = nd.st;
  const int lane = lane_id();
  if (wave_id() == 0) {
    const int beg = nd.rp[v], end = nd.rp[v + 1];
    for (int j = beg + lane; j < end; j += 64) {
      const int x = nd.ci[j];
      if (st[x] >= 0) st[x] |= kFlag;  // distinct x per lane: plain read-modify-write
    }
  }
  __syncthreads();
  apply_marks(nd);
}

// Mark v alone (the "v in the cover" child, §II-B) and remove it.
__device__ void remove_vertex(const Node nd, int v) {
  if (threadIdx.x == 0) nd.st[v] |= kFlag;
  __syncthreads();
  apply_marks(nd);
}

// Copy a node between LDS and device memory, 16 bytes per thread per step. The same thread
// always handles the same words, so a node written to the workgroup's own stack is read back
// by the threads that wrote it. `pending` replaces word n+1 on the way out.
__device__ void node_store(int32_t* __restrict__ dst, const int32_t* st, int stride, int n,
                           int pending) {
  const int4* s4 = reinterpret_cast<const int4*>(st);
  int4* d4 = reinterpret_cast<int4*>(dst);
  const int q = (n + 1) >> 2, r = (n + 1) & 3;
  for (int i = threadIdx.x; i < (stride >> 2); i += blockDim.x) {
    int4 x = s4[i];
    if (i == q) {
      if (r == 0) x.x = pending;
      else if (r == 1) x.y = pending;
      else if (r == 2) x.z = pending;
      else x.w = pending;
    }
    d4[i] = x;
  }
}

// The row pointers a kernel reads: a copy in LDS right after the node when the host found room
// for it (one LDS access instead of an L2 round trip at the head of every row walk), else the
// input array itself. Whole workgroup; ends with a barrier.
__device__ const int32_t* stage_row_ptr(const Params& p, int32_t* st) {
  if (!p.rp_lds) return p.rp;
  int32_t* dst = st + p.stride;
  for (int i = threadIdx.x; i <= p.n; i += blockDim.x) dst[i] = p.rp[i];
  __syncthreads();
  return dst;
}

// Copy a stored node between two device-memory slots with the same thread-to-word mapping as
// node_store / node_load, so each thread reads back words it wrote itself.
__device__ void node_copy(int32_t* __restrict__ dst, const int32_t* __restrict__ src, int stride) {
  const int4* s4 = reinterpret_cast<const int4*>(src);
  int4* d4 = reinterpret_cast<int4*>(dst);
  for (int i = threadIdx.x; i < (stride >> 2); i += blockDim.x) d4[i] = s4[i];
}

__device__ void node_load(int32_t* st, const int32_t* __restrict__ src, int stride) {
  const int4* s4 = reinterpret_cast<const int4*>(src);
  int4* d4 = reinterpret_cast<int4*>(st);
  for (int i = threadIdx.x; i < (stride >> 2); i += blockDim.x) d4[i] = s4[i];
}

// Whole workgroup: donate a deferred child to the worklist; true if the worklist took it. The
// child is the stored node at `oldest` (the bottom of this workgroup's stack) when that is not
// null, else the node in LDS with `pending` as its branch vertex.
__device__ bool try_enqueue(const Params& p, const Node nd, Ctrl& c, int pending,
                            const int32_t* oldest) {
  if (!enqueue_begin(p, c)) return false;
  int32_t* dst = p.payload + static_cast<size_t>(c.slot) * p.stride;
  if (oldest) node_copy(dst, oldest, p.stride);
  else node_store(dst, nd.st, p.stride, nd.n, pending);
  enqueue_publish(p, c);
  return true;
}

// Whole workgroup: take a node from the worklist into LDS. Returns 1 on success, 0 when the
// whole search is finished, -1 when it is being stopped.
__device__ int dequeue(const Params& p, const Node nd, Ctrl& c) {
  const int status = dequeue_begin(p, c);
  if (status != 1) return status;
  node_load(nd.st, p.payload + static_cast<size_t>(c.slot) * p.stride, p.stride);
  dequeue_finish(p, c);
  return 1;
}

// ---- kernels ---------------------------------------------------------------------------------

// Zero the control lines, mark every worklist slot free, publish slot 0 (the root, written by
// prepare_kernel) and the single outstanding sub-tree it stands for.
__global__ void init_kernel(Params p, DevResult* res) {
  for (int i = threadIdx.x; i < kNumCounters * kCounterStride; i += blockDim.x) p.ctr[i] = 0;
  for (uint32_t i = threadIdx.x; i < p.q_cap; i += blockDim.x) p.seq[i] = (i == 0) ? 1u : 0u;
  __syncthreads();
  if (threadIdx.x == 0) {
    *ctr_i32(p, kQCount) = 1;
    *ctr_u64(p, kQHead) = 0;
    *ctr_u64(p, kQTail) = 1;
    *ctr_i32(p, kWork) = 1;
    *ctr_u64(p, kBestKey) = ~0ull;
    *ctr_i32(p, kErrRow) = 0x7FFFFFFF;
    char* r = reinterpret_cast<char*>(res);
    for (size_t i = 0; i < sizeof(DevResult); ++i) r[i] = 0;
    res->wg_nodes_min = INT64_MAX;
  }
}

// Check the CSR (simple undirected graph, §II-A) and write the root node -- the input's
// degree array, s = 0, no pending vertex -- into worklist slot 0. Index i < stride checks row
// i's bounds and writes its degree; index i < nnz checks entry i: in range, not a self-loop,
// larger than the entry before it in its row, and present in reverse. Every read is
// bounds-checked before it is made, so a malformed input cannot send a thread out of its
// arrays. The smallest offending row is recorded.
__global__ void prepare_kernel(Params p) {
  const int n = p.n, nnz = p.nnz;
  int32_t* root = p.payload;
  int32_t local_sum = 0;
  // the bitset kernels build their own root node (bitset_pack_kernel)
  const int vertex_items = p.words ? n : p.stride;
  const int total = vertex_items > nnz ? vertex_items : nnz;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
    if (i < vertex_items) {
      if (i >= n) {
        root[i] = (i == n + 1) ? -1 : 0;
      } else {
        const int beg = p.rp[i], end = p.rp[i + 1];
        const bool bad = (i == 0 && beg != 0) || (i == n - 1 && end != nnz) || beg < 0 ||
                         end < beg || end > nnz;
        if (bad) atomicMin(ctr_i32(p, kErrRow), i);
        const int32_t d = bad ? 0 : end - beg;
        if (!p.words) root[i] = d;
        local_sum += d;
      }
    }
    if (i < nnz) {
      const int v = owner_row(p.rp, n, i);
      const int beg = p.rp[v], end = p.rp[v + 1];
      if (beg <= i && i < end && beg >= 0 && end <= nnz) {  // otherwise row bounds are bad
        const int u = p.ci[i];
        bool bad = u < 0 || u >= n || u == v || (i > beg && p.ci[i - 1] >= u);
        if (!bad) {
          const int ub = p.rp[u], ue = p.rp[u + 1];
          bad = ub < 0 || ue < ub || ue > nnz;
          if (!bad) {
            int lo = ub, hi = ue;
            while (lo < hi) {
              const int mid = lo + ((hi - lo) >> 1);
              if (p.ci[mid] < v) lo = mid + 1; else hi = mid;
            }
            bad = lo >= ue || p.ci[lo] != v;
          }
        }
        if (bad) atomicMin(ctr_i32(p, kErrRow), v);
      }
    }
  }
  local_sum = wave_sum(local_sum);
  if (lane_id() == 0 && local_sum) atomicAdd(ctr_i32(p, kEdges0), local_sum);
}

// Greedy approximation (§II-B, used as the initial best and the stack depth bound, §IV-E):
// degree-one and degree-two-triangle rules, then a maximum-degree vertex into the cover, until
// no edge is left. One workgroup. Its cover is the last cover buffer.
__global__ void __launch_bounds__(1024) greedy_kernel(Params p, DevResult* res) {
  extern __shared__ int4 lds4[];
  __shared__ Ctrl c;
  __shared__ int32_t heads[kMaxWaves * 64];
  int32_t* st = reinterpret_cast<int32_t*>(lds4);
  if (threadIdx.x == 0) {
    const int32_t err_row = load_relaxed(ctr_i32(p, kErrRow));
    res->err_row = err_row;
    res->edges0 = load_relaxed(ctr_i32(p, kEdges0)) / 2;
    res->greedy = 0;
    c.err = err_row != 0x7FFFFFFF;
    c.flag_epoch = -1;
  }
  __syncthreads();
  if (c.err) return;
  const Node nd{st, p.n, stage_row_ptr(p, st), p.ci, heads};
  node_load(st, p.payload, p.stride);  // the root written by prepare_kernel
  __syncthreads();
  int epoch = 0;
  const int64_t unbounded = 0x3FFFFFFFFFFFFFFFll;
  for (;;) {
    reduce_node(nd, c, unbounded, kRuleDeg1 | kRuleTri, epoch);
    int vmax, dmax;
    int32_t degsum;
    max_degree_and_sum(nd, c, vmax, dmax, degsum);
    if (degsum == 0) break;
    remove_vertex(nd, vmax);
  }
  const int s = st[p.n];
  uint8_t* cov = p.covers + static_cast<size_t>(p.greedy_slot) * p.cover_stride;
  for (int v = threadIdx.x; v < p.n; v += blockDim.x) cov[v] = st[v] == kSent;
  if (threadIdx.x == 0) {
    *ctr_u64(p, kBestKey) =
        (static_cast<unsigned long long>(s) << 32) | static_cast<uint32_t>(p.greedy_slot);
    res->greedy = s;
  }
}

// The hybrid traversal (§IV-A, Fig. 4; PVC differences in §IV-A, termination §IV-C).
template <bool PVC, bool PROF>
__global__ void __launch_bounds__(1024) traverse_kernel(Params p) {
  extern __shared__ int4 lds4[];
  __shared__ Ctrl c;
  __shared__ int32_t heads[kMaxWaves * 64];
  int32_t* st = reinterpret_cast<int32_t*>(lds4);
  const int n = p.n;
  const int wg = blockIdx.x;
  const int tid = threadIdx.x;
  if (tid == 0) {
    c.err = load_relaxed(ctr_i32(p, kErrRow)) != 0x7FFFFFFF ||
            load_relaxed(ctr_i32(p, kEdges0)) == 0;
    c.flag_epoch = -1;
  }
  __syncthreads();
  if (c.err) {
    if (tid == 0) p.wg_stats[wg] = WgStats{};
    return;
  }
  const Node nd{st, n, stage_row_ptr(p, st), p.ci, heads};
  ActivityClock<PROF> clk;
  clk.begin();

  int32_t* stack = p.stacks + static_cast<size_t>(wg) * p.depth_cap * p.stride;
  // The stack is a ring of depth_cap entries holding [bot, top): pops take the top, donations
  // take the bottom (the oldest deferred child, nearest its sub-tree root).
  int top = 0, bot = 0;
  bool have = false;      // a node is in LDS and still to be visited
  bool holding = false;   // this workgroup holds a sub-tree taken from the worklist
  int epoch = 0;
  int64_t nodes = 0, pushes = 0, pops = 0, enqueues = 0, dequeues = 0;
  int max_depth = 0;
  int64_t budget_mark = 0;

  for (;;) {
    // node header: global flags and the current best, read once and broadcast
    if (tid == 0) {
      c.stop = load_relaxed(ctr_i32(p, kAbort)) | (PVC ? load_relaxed(ctr_i32(p, kFound)) : 0);
      c.best = PVC ? 0 : static_cast<int32_t>(load_relaxed(ctr_u64(p, kBestKey)) >> 32);
    }
    __syncthreads();
    clk.charge(kActOther);
    if (c.stop) break;

    if (!have) {
      if (top > bot) {
        --top;
        node_load(st, stack + static_cast<size_t>(top % p.depth_cap) * p.stride, p.stride);
        ++pops;
        __syncthreads();
      } else {
        if (holding) {
          if (tid == 0) fetch_add(ctr_i32(p, kWork), -1);
          holding = false;
        }
        const int got = dequeue(p, nd, c);
        clk.charge(kActAcquire);
        if (got != 1) break;
        holding = true;
        ++dequeues;
      }
      clk.charge(kActAcquire);
      const int pending = st[n + 1];
      if (pending >= 0) {
        __syncthreads();  // every thread has read the pending vertex
        if (tid == 0) st[n + 1] = -1;
        remove_neighbourhood(nd, pending);
      }
      clk.charge(kActBranch);
      have = true;
    }

    ++nodes;
    if (p.node_budget > 0 && nodes - budget_mark >= p.budget_chunk) {
      if (tid == 0) {
        const unsigned long long total =
            fetch_add(ctr_u64(p, kNodes), static_cast<unsigned long long>(nodes - budget_mark));
        if (static_cast<int64_t>(total) + (nodes - budget_mark) >= p.node_budget)
          store_relaxed(ctr_i32(p, kAbort), 1);
      }
      budget_mark = nodes;
    }

    const int64_t bound = PVC ? p.k : static_cast<int64_t>(c.best) - 1;
    clk.charge(kActOther);
    reduce_node(nd, c, bound, p.rules, epoch, clk);
    clk.charge(kActReduce);

    // stopping condition (§II-B): no cover of size <= bound below this node if r < 0 or
    // |E| > r^2 (every remaining degree is <= r once the high-degree rule has run)
    const int32_t s = st[n];
    const int64_t r = bound - s;
    if (r < 0) {
      have = false;
      continue;
    }
    int vmax, dmax;
    int32_t degsum;
    max_degree_and_sum(nd, c, vmax, dmax, degsum);
    clk.charge(kActBranch);
    const int64_t edges = degsum / 2;
    if ((p.rules & kPruneEdges) && (p.rules & kRuleHigh) && edges > r * r) {
      have = false;
      continue;
    }
    if (edges == 0) {  // a vertex cover of size s
      if (tid == 0) {
        if (PVC) {
          c.status = atomicCAS(ctr_i32(p, kFound), 0, wg + 1) == 0;
        } else {
          const unsigned long long key =
              (static_cast<unsigned long long>(s) << 32) | static_cast<uint32_t>(wg);
          c.status = atomicMin(ctr_u64(p, kBestKey), key) > key;
        }
      }
      __syncthreads();
      if (c.status) {
        uint8_t* cov = p.covers + static_cast<size_t>(wg) * p.cover_stride;
        for (int v = tid; v < n; v += blockDim.x) cov[v] = st[v] == kSent;
      }
      clk.charge(kActOther);
      have = false;
      continue;
    }

    // branch on v_max (§II-B): defer the N(v_max) child, continue with the v_max child. While
    // the worklist is below its threshold a deferred child is donated (§IV-A): the oldest one on
    // this workgroup's stack if there is one (the largest sub-tree it holds), else this one.
    bool kept_local = true;
    if (p.q_threshold > 0) {
      const bool from_stack = top > bot;
      const int32_t* oldest =
          from_stack ? stack + static_cast<size_t>(bot % p.depth_cap) * p.stride : nullptr;
      if (try_enqueue(p, nd, c, vmax, oldest)) {
        ++enqueues;
        if (from_stack) ++bot;
        else kept_local = false;
      }
    }
    if (kept_local) {
      if (top - bot >= p.depth_cap) {  // cannot happen: the depth bound of §IV-E holds
        if (tid == 0) {
          atomicMax(ctr_i32(p, kError), 1);
          store_relaxed(ctr_i32(p, kAbort), 1);
        }
        break;
      }
      node_store(stack + static_cast<size_t>(top % p.depth_cap) * p.stride, st, p.stride, n, vmax);
      ++top;
      ++pushes;
      if (top - bot > max_depth) max_depth = top - bot;
      __syncthreads();  // the copy has read the node before it changes below
    }
    clk.charge(kActDonate);
    remove_vertex(nd, vmax);
    clk.charge(kActBranch);
  }
  clk.end();

  if (tid == 0) {
    if (p.node_budget > 0 && nodes > budget_mark)
      fetch_add(ctr_u64(p, kNodes), static_cast<unsigned long long>(nodes - budget_mark));
    WgStats w{};
    w.nodes = nodes;
    w.pushes = pushes;
    w.pops = pops;
    w.enqueues = enqueues;
    w.dequeues = dequeues;
    w.max_depth = max_depth;
    for (int a = 0; a < kNumActivities; ++a) w.cycles[a] = static_cast<int64_t>(clk.cycles[a]);
    p.wg_stats[wg] = w;
  }
}

// Index of the cover buffer holding the answer: >= 0, or -2 for "no cover" (rejected input,
// edgeless graph, PVC no).
__device__ __forceinline__ int32_t answer_buffer(const Params& p, int pvc) {
  if (*ctr_i32(p, kErrRow) != 0x7FFFFFFF || *ctr_i32(p, kEdges0) == 0) return -2;
  if (pvc) {
    const int32_t f = *ctr_i32(p, kFound);
    return f ? f - 1 : -2;
  }
  return static_cast<int32_t>(*ctr_u64(p, kBestKey) & 0xFFFFFFFFull);
}

// After the traversal (256-thread blocks, any grid): pick the answer, copy its cover out, check
// the cover edge by edge (one thread per CSR entry) and count its vertices, and gather the
// per-workgroup statistics.
__global__ void __launch_bounds__(256) finalize_kernel(Params p, int pvc, uint8_t* cover_out,
                                                       DevResult* res) {
  __shared__ int64_t buf[256];
  const int32_t src = answer_buffer(p, pvc);
  const bool valid = *ctr_i32(p, kErrRow) == 0x7FFFFFFF;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const int32_t edges0 = *ctr_i32(p, kEdges0) / 2;
    res->err_row = *ctr_i32(p, kErrRow);
    res->edges0 = edges0;
    res->aborted = *ctr_i32(p, kAbort);
    res->error = *ctr_i32(p, kError);
    res->q_max_count = *ctr_i32(p, kQMaxCount);
    if (valid && edges0 == 0) {
      res->size = 0;
      res->yes = 1;
    } else if (valid && pvc) {
      res->size = -1;
      res->yes = src >= 0;
    } else if (valid) {
      res->size = static_cast<int32_t>(*ctr_u64(p, kBestKey) >> 32);
      res->yes = 1;
    }
  }
  const uint8_t* from = src >= 0 ? p.covers + static_cast<size_t>(src) * p.cover_stride : nullptr;
  int32_t bad = 0, ones = 0;
  if (valid) {
    const int total = p.n > p.nnz ? p.n : p.nnz;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
      if (i < p.n) {
        const uint8_t c = from ? from[i] : 0;
        if (cover_out) cover_out[i] = c;
        ones += c != 0;
      }
      if (i < p.nnz && from) {
        const int v = owner_row(p.rp, p.n, i);
        bad += from[v] == 0 && from[p.ci[i]] == 0;
      }
    }
  }
  bad = wave_sum(bad);
  ones = wave_sum(ones);
  if (lane_id() == 0) {
    if (bad) atomicAdd(&res->uncovered, bad);
    if (ones) atomicAdd(&res->cover_count, ones);
  }
  // per-workgroup statistics: only the blocks that cover workgroup slots
  if (static_cast<int>(blockIdx.x) * static_cast<int>(blockDim.x) >= p.num_wg) return;
  int64_t nodes = 0, pushes = 0, pops = 0, enq = 0, deq = 0, mx = 0, mn = INT64_MAX, depth = 0;
  int64_t cyc[kNumActivities] = {};
  for (int w = blockIdx.x * blockDim.x + threadIdx.x; w < p.num_wg; w += gridDim.x * blockDim.x) {
    const WgStats s = p.wg_stats[w];
    nodes += s.nodes;
    pushes += s.pushes;
    pops += s.pops;
    enq += s.enqueues;
    deq += s.dequeues;
    mx = s.nodes > mx ? s.nodes : mx;
    mn = s.nodes < mn ? s.nodes : mn;
    depth = s.max_depth > depth ? s.max_depth : depth;
    for (int a = 0; a < kNumActivities; ++a) cyc[a] += s.cycles[a];
  }
  auto add = [](int64_t x, int64_t y) { return x + y; };
  auto hi = [](int64_t x, int64_t y) { return x > y ? x : y; };
  auto lo = [](int64_t x, int64_t y) { return x < y ? x : y; };
  nodes = block_reduce_256(nodes, buf, add);
  pushes = block_reduce_256(pushes, buf, add);
  pops = block_reduce_256(pops, buf, add);
  enq = block_reduce_256(enq, buf, add);
  deq = block_reduce_256(deq, buf, add);
  mx = block_reduce_256(mx, buf, hi);
  mn = block_reduce_256(mn, buf, lo);
  depth = block_reduce_256(depth, buf, hi);
  for (int a = 0; a < kNumActivities; ++a) cyc[a] = block_reduce_256(cyc[a], buf, add);
  if (threadIdx.x == 0) {
    using ull = unsigned long long;
    if (nodes) atomicAdd(reinterpret_cast<ull*>(&res->nodes), static_cast<ull>(nodes));
    if (pushes) atomicAdd(reinterpret_cast<ull*>(&res->pushes), static_cast<ull>(pushes));
    if (pops) atomicAdd(reinterpret_cast<ull*>(&res->pops), static_cast<ull>(pops));
    if (enq) atomicAdd(reinterpret_cast<ull*>(&res->enqueues), static_cast<ull>(enq));
    if (deq) atomicAdd(reinterpret_cast<ull*>(&res->dequeues), static_cast<ull>(deq));
    atomicMax(reinterpret_cast<ull*>(&res->wg_nodes_max), static_cast<ull>(mx));
    atomicMin(reinterpret_cast<ull*>(&res->wg_nodes_min), static_cast<ull>(mn));
    atomicMax(&res->max_depth, static_cast<int32_t>(depth));
    for (int a = 0; a < kNumActivities; ++a)
      if (cyc[a]) atomicAdd(reinterpret_cast<ull*>(&res->cycles[a]), static_cast<ull>(cyc[a]));
  }
}

// The reduction rules of one node, alone, on a degree array in device memory (one workgroup).
__global__ void __launch_bounds__(1024) reduce_kernel(Params p, int32_t* deg, int32_t* s,
                                                      int64_t bound, DevResult* res) {
  extern __shared__ int4 lds4[];
  __shared__ Ctrl c;
  __shared__ int32_t heads[kMaxWaves * 64];
  int32_t* st = reinterpret_cast<int32_t*>(lds4);
  if (threadIdx.x == 0) {
    const int32_t err_row = load_relaxed(ctr_i32(p, kErrRow));
    res->err_row = err_row;
    c.err = err_row != 0x7FFFFFFF;
  }
  __syncthreads();
  if (c.err) return;  // rejected input: leave the degree array alone
  for (int v = threadIdx.x; v < p.stride; v += blockDim.x)
    st[v] = v < p.n ? deg[v] : (v == p.n ? *s : (v == p.n + 1 ? -1 : 0));
  if (threadIdx.x == 0) c.flag_epoch = -1;
  __syncthreads();
  const Node nd{st, p.n, stage_row_ptr(p, st), p.ci, heads};
  int epoch = 0;
  reduce_node(nd, c, bound, p.rules, epoch);
  for (int v = threadIdx.x; v < p.n; v += blockDim.x) deg[v] = st[v];
  if (threadIdx.x == 0) *s = st[p.n];
}

// ---- launchers ---------------------------------------------------------------------------------

hipError_t launch_init(const Params& p, DevResult* res, hipStream_t stream) {
  hipLaunchKernelGGL(init_kernel, dim3(1), dim3(256), 0, stream, p, res);
  return hipGetLastError();
}

hipError_t launch_prepare(const Params& p, hipStream_t stream) {
  const int threads = 256;
  const int vertex_items = p.words ? p.n : p.stride;
  const int items = vertex_items > p.nnz ? vertex_items : p.nnz;
  int blocks = (items + threads - 1) / threads;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(prepare_kernel, dim3(blocks), dim3(threads), 0, stream, p);
  return hipGetLastError();
}

hipError_t launch_greedy(const Params& p, int32_t wg_size, DevResult* res, hipStream_t stream) {
  const size_t lds = node_lds_bytes(p.stride, p.n, p.rp_lds);
  hipLaunchKernelGGL(greedy_kernel, dim3(1), dim3(wg_size), lds, stream, p, res);
  return hipGetLastError();
}

static const void* traverse_fn(bool pvc, bool prof) {
  if (pvc) return prof ? reinterpret_cast<const void*>(&traverse_kernel<true, true>)
                       : reinterpret_cast<const void*>(&traverse_kernel<true, false>);
  return prof ? reinterpret_cast<const void*>(&traverse_kernel<false, true>)
              : reinterpret_cast<const void*>(&traverse_kernel<false, false>);
}

// A plain launch: the grid is sized by the occupancy API so that all workgroups are normally
// resident together, but the search does not depend on it. A workgroup only ever waits for
// workgroups that have already taken a worklist ticket (and are therefore running); one that
// starts late finds either work or a zero outstanding-work counter.
hipError_t launch_traverse(bool pvc, bool prof, const Params& p, int32_t wg_size,
                           hipStream_t stream) {
  const size_t lds = node_lds_bytes(p.stride, p.n, p.rp_lds);
  Params args = p;
  void* kargs[] = {&args};
  return hipLaunchKernel(traverse_fn(pvc, prof), dim3(p.num_wg), dim3(wg_size), kargs, lds, stream);
}

hipError_t launch_finalize(bool pvc, const Params& p, uint8_t* cover_out, DevResult* res,
                           hipStream_t stream) {
  const int threads = 256;
  int items = p.n > p.nnz ? p.n : p.nnz;
  if (p.num_wg > items) items = p.num_wg;
  int blocks = (items + threads - 1) / threads;
  if (blocks < 1) blocks = 1;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(finalize_kernel, dim3(blocks), dim3(threads), 0, stream, p, pvc ? 1 : 0,
                     cover_out, res);
  return hipGetLastError();
}

hipError_t launch_reduce(const Params& p, int32_t wg_size, int32_t* deg, int32_t* s,
                         int64_t bound, DevResult* res, hipStream_t stream) {
  const size_t lds = node_lds_bytes(p.stride, p.n, p.rp_lds);
  hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(wg_size), lds, stream, p, deg, s, bound, res);
  return hipGetLastError();
}

hipError_t traverse_occupancy(bool pvc, bool prof, int32_t wg_size, size_t lds_bytes,
                              int* blocks_per_cu) {
  const void* fn = traverse_fn(pvc, prof);
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, fn, wg_size, lds_bytes);
}

hipError_t set_lds_limit(size_t lds_bytes) {
  const void* fns[] = {traverse_fn(true, false), traverse_fn(false, false),
                       traverse_fn(true, true), traverse_fn(false, true),
                       reinterpret_cast<const void*>(&greedy_kernel),
                       reinterpret_cast<const void*>(&reduce_kernel)};
  for (const void* fn : fns) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(lds_bytes));
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace vc
