// vc_device.hip -- HIP kernels for gfx950 (MI355X) of the hybrid vertex-cover traversal.
//
// Method (paper §IV): a persistent grid; every workgroup walks a sub-tree of the
// branch-and-reduce search tree depth first with its own stack in device memory, and hands
// branches to a global worklist while the worklist holds fewer entries than a threshold
// (§IV-A). An intermediate graph is a degree array over one read-only CSR (§IV-B): one int32
// per vertex holding its degree, or a negative value once the vertex is in the cover, followed
// by the cover size s (the |S| counter of §IV-B) and a pending branch vertex (see below).
//
// gfx950 mapping:
//  - the node being worked on lives in LDS; every rule pass, the max-degree search and the
//    vertex removals read and update it there (LDS atomics for degree decrements); the row
//    pointers, and the column indices too when they fit, are staged in LDS after it. Where
//    each of them lives is a template parameter of the kernels, so every access compiles to
//    an LDS or a device-memory instruction, never a generic one;
//  - vertices are processed in 64-vertex chunks, one chunk per wavefront at a time; a
//    ballot over the chunk yields the candidates; a candidate's CSR row is walked by its own
//    lane when it is short, and in 64-entry pieces by the whole wavefront when it is long;
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
// "degree two, and its two live neighbours are not adjacent" on a live entry. Along a path of
// the search tree vertices are only removed, so a vertex that still has degree two has the same
// two neighbours: the mark stays true in every descendant node (stored nodes keep it) and the
// triangle rule checks each degree-two vertex once per path instead of once per pass.
constexpr int32_t kNoTri = 0x20000000;
constexpr int32_t kDegMask = 0x1FFFFFFF;  // degree bits of a live entry

// ---- node operations on the LDS degree array -------------------------------------------------
// st[0..n) degrees (negative = in the cover), st[n] = s, st[n+1] = pending vertex (-1 = none).

// Entries of the removal list: the vertices one removal step takes out, gathered from every
// wavefront's part of the node so that the wavefronts can share their rows evenly.
constexpr int kListCap = 1024;
// Workgroups of fewer wavefronts than this skip the removal list (one or two wavefronts have
// little to balance, and the list's append and read-back lengthen every removal step).
constexpr int kListWaves = 4;

struct Node {
  int32_t* st;
  int n;
  const int32_t* __restrict__ rp;
  const int32_t* __restrict__ ci;
  int32_t* list;   // kListCap LDS words: the removal list
  int32_t* heads;  // 64 LDS words per wavefront for walk_rows
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

// Rows longer than this are walked in 64-entry pieces; shorter ones are packed together.
constexpr int kLongRow = 64;

// Walk the CSR rows [beg, end) held by the lanes of a wavefront (empty where beg >= end).
// fn(x, tag, j) runs for every entry x = ci[j], with `tag` the value the row's owner lane
// passed in; it runs in divergent code. `heads` is this wavefront's 64 LDS words.
//  - Rows of at most kLongRow entries are walked as one list, 64 consecutive entries per step,
//    so many short rows fill one step and neighbouring lanes read neighbouring entries. The
//    owner of each entry of a step comes from head flags: every row writes its lane into
//    `heads` at its first position in the step, and a max-scan over the lanes carries it
//    forward. Eight steps are issued together, with unconditional loads (an index past the
//    list reads entry 0, whose value is discarded).
//  - Longer rows are cut into 64-entry pieces that the whole wavefront walks one after
//    another, eight pieces per round, with the cursor (row bounds, tag, position) in scalar
//    registers: a piece needs no owner lookup.
template <typename Fn>
__device__ __forceinline__ void walk_rows(const int32_t* __restrict__ ci, int32_t* heads, int beg,
                                          int end, int tag, Fn fn) {
  const int lane = lane_id();
  const int full = end > beg ? end - beg : 0;
  const bool longrow = full > kLongRow;
  const int len = longrow ? 0 : full;
  const int incl = wave_incl_scan(len);
  const int excl = incl - len;
  const int total = __builtin_amdgcn_readlane(incl, 63);
  constexpr int kUnroll = 8;
  for (int t0 = 0; t0 < total; t0 += 64 * kUnroll) {
    int xs[kUnroll], tags[kUnroll], js[kUnroll];
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
        js[u] = ok[u] ? ob + (t - oe) : 0;
        xs[u] = ci[js[u]];  // not read until every step has issued
      }
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u)
      if (ok[u]) fn(xs[u], tags[u], js[u]);
  }
  uint64_t longs = __builtin_amdgcn_ballot_w64(longrow);
  int rb = 0, re = 0, rt = 0;  // the piece cursor: next entry, end and tag of the current row
  while (longs || rb < re) {
    int xs[8], js[8], ts[8];
    bool ok[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (rb >= re && longs) {
        const int o = first_lane(longs);
        longs &= longs - 1;
        rb = __builtin_amdgcn_readlane(beg, o);
        re = __builtin_amdgcn_readlane(end, o);
        rt = __builtin_amdgcn_readlane(tag, o);
      }
      js[u] = rb + lane;
      ok[u] = js[u] < re;
      ts[u] = rt;
      xs[u] = ok[u] ? ci[js[u]] : 0;
      rb += 64;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (ok[u]) fn(xs[u], ts[u], js[u]);
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

// Remove every marked vertex (paper §IV-B): marked vertices become kSent and s grows by their
// number; each live unmarked neighbour of a marked vertex loses one degree per marked
// neighbour. The scan sets each marked vertex to kSent and appends it to the workgroup's
// removal list; after a barrier the wavefronts take the list's rows round-robin (list entry i
// goes to wavefront i mod waves), so a few marked vertices with long rows in one wavefront's
// part of the node do not leave the others idle. Marked vertices beyond the list's capacity
// stay marked and are taken by further rounds of scan and walk. Workgroups of fewer than
// kListWaves wavefronts skip the list: each wavefront walks the rows it finds. The walks only
// decrement entries that are live and unmarked (a marked vertex is set to kSent by the scan,
// whichever of the two happens first), which also keeps the LDS atomics off the entries of
// vertices already removed. Called right after a barrier that ends a decide step (or a mark
// step); ends with a barrier. Two calls are always separated by another barrier (a decide
// step), which orders the reset of the list count before the next call's appends.
__device__ __forceinline__ void apply_marks(const Node nd, Ctrl& c) {
  const int n = nd.n;
  int32_t* st = nd.st;
  const int lane = lane_id();
  const int waves = blockDim.x >> 6;
  const auto decrement = [&](int x, int, int) {
    const int32_t dx = st[x];
    if (dx >= 0 && !(dx & kFlag)) atomicSub(&st[x], 1);
  };
  if (waves < kListWaves) {
    // few wavefronts, little to balance: each walks the rows of the marked vertices it finds
    int cnt = 0;
    for_each_batch(st, n,
                   [&](int v, int32_t d) {
                     const bool marked = d >= 0 && (d & kFlag);
                     if (marked) {
                       st[v] = kSent;
                       ++cnt;
                     }
                     return marked;
                   },
                   [&](int f, int count) {
                     const bool mine = lane < count;
                     walk_rows(nd.ci, nd.heads + 64 * wave_id(), mine ? nd.rp[f] : 0,
                               mine ? nd.rp[f + 1] : 0, f, decrement);
                   });
    cnt = wave_sum(cnt);
    if (lane == 0 && cnt) atomicAdd(&st[n], cnt);
    __syncthreads();
    return;
  }
  for (;;) {
    for (int base = wave_id() * 64; base < n; base += blockDim.x) {
      const int v = base + lane;
      const int32_t d = v < n ? st[v] : kSent;
      const bool marked = v < n && d >= 0 && (d & kFlag);
      const uint64_t mask = __builtin_amdgcn_ballot_w64(marked);
      if (!mask) continue;
      int at = 0;
      if (lane == 0) at = atomicAdd(&c.list_n, __popcll(mask));
      at = __builtin_amdgcn_readfirstlane(at);
      const uint32_t below = __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mask), 0);
      const int rank = __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(mask >> 32), below);
      if (marked && at + rank < kListCap) {  // beyond the list: left marked for the next round
        st[v] = kSent;
        nd.list[at + rank] = v;
      }
    }
    __syncthreads();
    const int total = c.list_n;
    const int listed = total < kListCap ? total : kListCap;
    for (int i0 = wave_id(); i0 < listed; i0 += waves * 64) {
      const int i = i0 + waves * lane;
      const bool mine = i < listed;
      const int f = mine ? nd.list[i] : 0;
      walk_rows(nd.ci, nd.heads + 64 * wave_id(), mine ? nd.rp[f] : 0, mine ? nd.rp[f + 1] : 0, f,
                decrement);
    }
    if (threadIdx.x == 0) st[n] += listed;
    __syncthreads();
    if (total <= kListCap) break;
    // rare: more marked vertices than the list holds; the rest go in another round
    if (threadIdx.x == 0) c.list_n = 0;
    __syncthreads();
  }
  if (threadIdx.x == 0) c.list_n = 0;
}

// Degree-one rule (§II-B): v with one live neighbour u puts u in the cover; of two adjacent
// degree-one vertices only the smaller id is removed, and a shared neighbour once (§IV-D).
// The rows of all degree-one vertices are walked together; the one live entry of a row names
// u, and the lane that reads it makes the decision for that row's owner.
__device__ __forceinline__ void decide_degree_one(const Node nd, Ctrl& c, int epoch) {
  int32_t* st = nd.st;
  for_each_batch(st, nd.n, [](int, int32_t d) { return d >= 0 && (d & kDegMask) == 1; },
                 [&](int cv, int count) {
                   const bool mine = lane_id() < count;
                   walk_rows(nd.ci, nd.heads + 64 * wave_id(), mine ? nd.rp[cv] : 0,
                             mine ? nd.rp[cv + 1] : 0, cv,
                             [&](int u, int v, int) {
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
__device__ __forceinline__ void decide_triangle(const Node nd, Ctrl& c, int epoch) {
  constexpr int kLaneRow = 32;
  int32_t* st = nd.st;
  const int lane = lane_id();
  for_each_batch(st, nd.n,
                 [](int, int32_t d) { return d >= 0 && (d & kDegMask) == 2 && !(d & kNoTri); },
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
                   if (!row_contains(nd.ci, in_a ? ab : bb, in_a ? ae : be, in_a ? b : a)) {
                     // no triangle through cv: no other lane flags cv in this pass (a firing
                     // vertex flags only the two vertices of its own triangle)
                     atomicOr(&st[cv], kNoTri);
                     return;
                   }
                   const int32_t da = st[a] & kDegMask, db = st[b] & kDegMask;
                   if ((da == 2 && a < cv) || (db == 2 && b < cv)) return;
                   atomicOr(&st[a], kFlag);
                   atomicOr(&st[b], kFlag);
                   c.flag_epoch = epoch;
                 });
}

// High-degree rule (§II-B): a vertex whose degree exceeds r = bound - s is in every cover of
// size <= bound (bound = best - 1 for MVC, k for PVC).
__device__ __forceinline__ void decide_high_degree(const Node nd, Ctrl& c, int epoch, int64_t r) {
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
// Precondition: the node is visible to the whole workgroup. With `marked`, the vertices that
// mark_vertex / mark_neighbourhood flagged (a branch's removal) are removed first. The three
// rules take turns through one loop, so that the removal step, the longest code, is compiled
// once per kernel.
template <typename Clock>
__device__ __forceinline__ void reduce_node(const Node nd, Ctrl& c, int64_t bound, int rules,
                                            int& epoch, Clock& clk, bool marked) {
  const int n = nd.n;
  int32_t* st = nd.st;
  if (marked) {
    apply_marks(nd, c);
    clk.charge(kActBranch);
  }
  // A rule pass is skipped when nothing has been removed since it last found nothing: its
  // inputs (the graph, and |S| for the high-degree rule) are then unchanged, so it would find
  // nothing again. This drops the empty passes of the final round, not any decision.
  int changes = 0;                   // removal steps applied in this call
  int quiet[3] = {-1, -1, -1};       // `changes` when each rule last found nothing
  int32_t s0 = st[n];                // s at the start of the current round
  if (s0 > bound) return;
  for (int rule = 0;; rule = rule == 2 ? 0 : rule + 1) {
    if (rule == 0 && changes > 0) {  // a new round: stop if the last one removed nothing
      const int32_t s1 = st[n];
      if (s1 == s0) return;
      s0 = s1;
    }
    if (!(rules & (kRuleDeg1 << rule)) || quiet[rule] == changes) {
      if (rule == 2 && changes == 0) return;  // a first round that found nothing
      continue;
    }
    ++epoch;
    if (rule == 0) {
      decide_degree_one(nd, c, epoch);
      __syncthreads();
      clk.charge(kActDeg1);
    } else if (rule == 1) {
      decide_triangle(nd, c, epoch);
      __syncthreads();
      clk.charge(kActTri);
    } else {
      decide_high_degree(nd, c, epoch, bound - st[n]);
      __syncthreads();
      clk.charge(kActHigh);
    }
    if (c.flag_epoch != epoch) {
      quiet[rule] = changes;
      if (rule == 2 && changes == 0) return;
      continue;
    }
    apply_marks(nd, c);
    ++changes;
    clk.charge(kActApply);
    if (st[n] > bound) return;
  }
}

__device__ __forceinline__ void reduce_node(const Node nd, Ctrl& c, int64_t bound, int rules,
                                            int& epoch, bool marked = false) {
  NoClock none;
  reduce_node(nd, c, bound, rules, epoch, none, marked);
}

// One pass over the degree array: the sum of live degrees (= 2|E|) and the live vertex of
// maximum degree, smallest id on ties (§IV-B). Results are the same in every thread.
__device__ __forceinline__ void max_degree_and_sum(const Node nd, Ctrl& c, int& vmax, int& dmax,
                                   int32_t& degsum) {
  const int n = nd.n;
  const int32_t* st = nd.st;
  uint64_t key = 0;
  int32_t sum = 0;
  for (int v = threadIdx.x; v < n; v += blockDim.x) {
    const int32_t raw = st[v];
    if (raw >= 0) {
      const int32_t d = raw & kDegMask;
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

// Flag every live neighbour of v (the "N(v) in the cover" child, §II-B); the next reduce_node
// (marked = true) removes them. Ends with a barrier.
__device__ __forceinline__ void mark_neighbourhood(const Node nd, int v) {
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
}

// Flag v alone (the "v in the cover" child, §II-B); the next reduce_node (marked = true)
// removes it. Ends with a barrier.
__device__ __forceinline__ void mark_vertex(const Node nd, int v) {
  if (threadIdx.x == 0) nd.st[v] |= kFlag;
  __syncthreads();
}

// Copy a node between LDS and device memory, 16 bytes per thread per step. The same thread
// always handles the same words, so a node written to the workgroup's own stack is read back
// by the threads that wrote it. `pending` replaces word n+1 on the way out.
__device__ __forceinline__ void node_store(int32_t* __restrict__ dst, const int32_t* st, int stride,
                                           int n,
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


// Copy a stored node between two device-memory slots with the same thread-to-word mapping as
// node_store / node_load, so each thread reads back words it wrote itself.
__device__ __forceinline__ void node_copy(int32_t* __restrict__ dst, const int32_t* __restrict__ src,
                                          int stride) {
  const int4* s4 = reinterpret_cast<const int4*>(src);
  int4* d4 = reinterpret_cast<int4*>(dst);
  for (int i = threadIdx.x; i < (stride >> 2); i += blockDim.x) d4[i] = s4[i];
}

__device__ __forceinline__ void node_load(int32_t* st, const int32_t* __restrict__ src,
                                          int stride) {
  const int4* s4 = reinterpret_cast<const int4*>(src);
  int4* d4 = reinterpret_cast<int4*>(st);
  for (int i = threadIdx.x; i < (stride >> 2); i += blockDim.x) d4[i] = s4[i];
}

// The node a workgroup works on: in LDS (dynamic shared memory, followed by the staged row
// pointers), or, for graphs whose node does not fit there, in slot `slot` of the device-memory
// node array. The node operations take a plain pointer, so one body serves both; in device
// memory their reads, writes and atomics are global-memory accesses, ordered inside the
// workgroup by the same barriers.
// Where a launch keeps the node being worked on and the CSR it reads. Fixed per kernel
// instantiation, so that every access compiles to an LDS (ds_*) or a device-memory (global_*)
// instruction rather than a generic one that has to test its address.
enum MemMode : int {
  kMemGlobal = 0,  // node in device memory (graphs too large for LDS); CSR in device memory
  kMemLds = 1,     // node in LDS; CSR in device memory
  kMemLdsRp = 2,   // node and row pointers in LDS; column indices in device memory
  kMemLdsCsr = 3,  // node and the whole CSR in LDS
};

template <int MEM>
__device__ __forceinline__ int32_t* node_base(const Params& p, int slot) {
  if constexpr (MEM == kMemGlobal) {
    return p.gnodes + static_cast<size_t>(slot) * p.stride;
  } else {
    extern __shared__ int4 lds4[];
    return reinterpret_cast<int32_t*>(lds4);
  }
}

// ---- instances -------------------------------------------------------------------------------

// Whole workgroup: make instance j the one the node operations work on. Its row pointers are
// copied into LDS right after the node when the launch has room for them (one LDS access
// instead of an L2 round trip at the head of every row walk), and its column indices after
// them when the launch has room for those too (every row walk of a rule pass is then a chain
// of LDS accesses); the copy ends with a barrier. The copies read only the instance's own
// n + 1 row pointers and nnz entries, so they stay in bounds whatever the graph holds.
// Graphs whose column indices stay in device memory (up to 1 MB of them) are first touched
// once per 128-byte line, with independent loads, so that the dependent row walks of the rule
// passes find them in this XCD's L2.
constexpr int32_t kTouchMaxEntries = 1 << 18;

template <int MEM>
__device__ __forceinline__ Node load_instance(const Params& p, int j, int32_t* st,
                                              int32_t* list, int32_t* heads) {
  const Instance in = p.inst[j];
  const int32_t* rp = p.rp_all + in.rp_off;
  const int32_t* ci = p.ci_all + in.ci_off;
  if constexpr (MEM == kMemLds || MEM == kMemLdsRp) {
    if (in.nnz <= kTouchMaxEntries) {
      int32_t acc = 0;
      for (int i = threadIdx.x * 32; i < in.nnz; i += blockDim.x * 32) acc ^= ci[i];
      asm volatile("" ::"v"(acc));
    }
  }
  if constexpr (MEM >= kMemLdsRp) {
    int32_t* dst = st + p.stride;
    for (int i = threadIdx.x; i <= in.n; i += blockDim.x) dst[i] = rp[i];
    if constexpr (MEM == kMemLdsCsr) {
      int32_t* dci = dst + rp_lds_words(p.n_max);
      for (int i = threadIdx.x; i < in.nnz; i += blockDim.x) dci[i] = ci[i];
      ci = dci;
    }
    __syncthreads();
    rp = dst;
  }
  return Node{st, in.n, rp, ci, list, heads};
}

// A node with no instance yet, whose CSR pointers already point where this memory mode keeps
// them (so that the compiler sees one kind of memory behind each pointer).
template <int MEM>
__device__ __forceinline__ Node empty_node(const Params& p, int32_t* st, int32_t* list,
                                           int32_t* heads) {
  const int32_t* rp = p.rp_all;
  const int32_t* ci = p.ci_all;
  if constexpr (MEM >= kMemLdsRp) rp = st + p.stride;
  if constexpr (MEM == kMemLdsCsr) ci = st + p.stride + rp_lds_words(p.n_max);
  return Node{st, 0, rp, ci, list, heads};
}

// Whole workgroup: the root of instance j in LDS -- the input's degree array, s = 0, nothing
// pending, the instance in the last word. Ends with a barrier.
__device__ __forceinline__ void build_root(const Params& p, const Node nd, int j) {
  for (int v = threadIdx.x; v < p.stride; v += blockDim.x) {
    int32_t x = 0;
    if (v < nd.n) x = nd.rp[v + 1] - nd.rp[v];
    else if (v == nd.n + 1) x = -1;
    else if (v == p.stride - 1) x = j;
    nd.st[v] = x;
  }
  __syncthreads();
}

// Launch-local instance holding packed vertex i (or CSR entry i): the last instance whose
// first index is <= i. Instances with no vertices (entries) share their first index with the
// next one, so the search lands on the instance that owns i.
__device__ __forceinline__ int instance_of_vertex(const Params& p, int64_t i) {
  int lo = 0, hi = p.num_inst - 1;
  while (lo < hi) {
    const int mid = lo + ((hi - lo + 1) >> 1);
    if (p.inst[mid].vtx_first <= i) lo = mid; else hi = mid - 1;
  }
  return lo;
}
__device__ __forceinline__ int instance_of_entry(const Params& p, int64_t i) {
  int lo = 0, hi = p.num_inst - 1;
  while (lo < hi) {
    const int mid = lo + ((hi - lo + 1) >> 1);
    if (p.inst[mid].ent_first <= i) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// ---- worklist ---------------------------------------------------------------------------------

// Whole workgroup: donate a deferred child of instance `inst` to the worklist; true if the
// worklist took it. The child is the stored node at `oldest` (the bottom of this workgroup's
// stack) when that is not null, else the node in LDS with `pending` as its branch vertex.
__device__ __forceinline__ bool try_enqueue(const Params& p, const Node nd, Ctrl& c, int pending,
                            const int32_t* oldest, int inst) {
  if (!enqueue_begin(p, c, inst)) return false;
  int32_t* dst = p.payload + static_cast<size_t>(c.slot) * p.stride;
  if (oldest) node_copy(dst, oldest, p.stride);
  else node_store(dst, nd.st, p.stride, nd.n, pending);
  enqueue_publish(p, c);
  return true;
}

// ---- kernels ---------------------------------------------------------------------------------


// Check every graph of the launch (simple undirected, §II-A). Index i < vertices checks row
// i's bounds (and, for the bitset kernels, packs the row into adjacency words); index i <
// entries checks one CSR entry: in range, not a self-loop, larger than the entry before it in
// its row, and present in reverse. Every read is bounds-checked before it is made, so a
// malformed input cannot send a thread out of its instance's arrays. Each instance keeps the
// smallest offending row.
//
// The same launch first resets the launch's control lines and result block and marks every
// worklist slot free (the host uploads the fresh per-instance state with the instance table);
// every instance's root is handed out by the root ticket counter, so the worklist starts empty.
// Nothing in the validation reads what the reset writes.
__global__ void prepare_kernel(Params p, DevResult* res, int64_t vertices, int64_t entries) {
  const int64_t total = vertices > entries ? vertices : entries;
  const int64_t gsize = static_cast<int64_t>(gridDim.x) * blockDim.x;
  if (blockIdx.x == 0) {
    for (int i = threadIdx.x; i < kNumCounters * kCounterStride; i += blockDim.x) p.ctr[i] = 0;
    __syncthreads();
    if (threadIdx.x == 0) {
      *ctr_i32(p, kWork) = p.num_inst;
      *ctr_i32(p, kOpen) = p.num_inst;
      char* r = reinterpret_cast<char*>(res);
      for (size_t i = 0; i < sizeof(DevResult); ++i) r[i] = 0;
      res->wg_nodes_min = INT64_MAX;
    }
  }
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < p.q_cap;
       i += gsize)
    p.seq[i] = 0u;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < total;
       i += gsize) {
    if (i < vertices) {
      const int j = instance_of_vertex(p, i);
      const Instance in = p.inst[j];
      const int v = static_cast<int>(i - in.vtx_first);
      const int32_t* rp = p.rp_all + in.rp_off;
      const int32_t* ci = p.ci_all + in.ci_off;
      const int beg = rp[v], end = rp[v + 1];
      const bool bad = (v == 0 && beg != 0) || (v == in.n - 1 && end != in.nnz) || beg < 0 ||
                       end < beg || end > in.nnz;
      if (bad) atomicMin(&p.ist[j].err_row, v);
      if (p.words && !bad) {
        uint64_t row[kMaxBitsetWords] = {};
        for (int e = beg; e < end; ++e) {
          const int u = ci[e];
          if (u >= 0 && u < in.n) row[u >> 6] |= 1ull << (u & 63);
        }
        uint64_t* dst = p.bits + (static_cast<int64_t>(in.vtx_first) + v) * p.words;
        for (int w = 0; w < p.words; ++w) dst[w] = row[w];
      }
    }
    if (i < entries) {
      const int j = instance_of_entry(p, i);
      const Instance in = p.inst[j];
      const int e = static_cast<int>(i - in.ent_first);
      const int32_t* rp = p.rp_all + in.rp_off;
      const int32_t* ci = p.ci_all + in.ci_off;
      const int v = owner_row(rp, in.n, e);
      const int beg = rp[v], end = rp[v + 1];
      if (beg <= e && e < end && beg >= 0 && end <= in.nnz) {  // otherwise row bounds are bad
        const int u = ci[e];
        bool bad = u < 0 || u >= in.n || u == v || (e > beg && ci[e - 1] >= u);
        if (!bad) {
          const int ub = rp[u], ue = rp[u + 1];
          bad = ub < 0 || ue < ub || ue > in.nnz;
          if (!bad) {
            int lo = ub, hi = ue;
            while (lo < hi) {
              const int mid = lo + ((hi - lo) >> 1);
              if (ci[mid] < v) lo = mid + 1; else hi = mid;
            }
            bad = lo >= ue || ci[lo] != v;
          }
        }
        if (bad) atomicMin(&p.ist[j].err_row, v);
      }
    }
  }
}

// Greedy approximation (§II-B, used as an instance's first best and for the stack depth bound,
// §IV-E): degree-one and degree-two-triangle rules, then a maximum-degree vertex into the
// cover, until no edge is left. One workgroup per instance (a grid-stride loop over the
// launch's instances); the cover goes to the instance's cover output.
template <int MEM>
__global__ void __launch_bounds__(1024) greedy_kernel(Params p) {
  __shared__ Ctrl c;
  __shared__ int32_t rm_list[kListCap];
  __shared__ int32_t heads[kMaxWaves * 64];
  int32_t* st = node_base<MEM>(p, blockIdx.x);
  if (threadIdx.x == 0) {
    c.flag_epoch = -1;
    c.list_n = 0;
  }
  int epoch = 0;
  for (int j = blockIdx.x; j < p.num_inst; j += gridDim.x) {
    if (threadIdx.x == 0) c.err = load_relaxed(&p.ist[j].err_row) != kNoRow;
    __syncthreads();
    const bool skip = c.err;
    __syncthreads();  // every thread has read c.err before thread 0 writes it again
    if (skip) continue;
    const Node nd = load_instance<MEM>(p, j, st, rm_list, heads);
    build_root(p, nd, j);
    const int64_t unbounded = 0x3FFFFFFFFFFFFFFFll;
    for (bool marked = false;; marked = true) {
      reduce_node(nd, c, unbounded, kRuleDeg1 | kRuleTri, epoch, marked);
      int vmax, dmax;
      int32_t degsum;
      max_degree_and_sum(nd, c, vmax, dmax, degsum);
      if (degsum == 0) break;
      mark_vertex(nd, vmax);
    }
    const int s = st[nd.n];
    uint8_t* cov = p.covers + p.inst[j].vtx_off;
    for (int v = threadIdx.x; v < nd.n; v += blockDim.x) cov[v] = st[v] < 0;
    if (threadIdx.x == 0) {
      p.ist[j].best = s;
      p.ist[j].greedy = s;
    }
    __syncthreads();  // the node and row pointers in LDS are read before the next instance
  }
}

// Thread 0: claim the right to record a cover of size s for instance j (§IV-A: atomic best /
// found). PVC: the first cover found wins. MVC: a cover wins if it lowers the instance's best;
// the winner then takes the instance's lock, and keeps it only if no smaller cover has been
// claimed meanwhile, so the last cover written under the lock is one of the final best size.
template <bool PVC>
__device__ __forceinline__ int claim_solution(const Params& p, int j, int32_t s) {
  InstState* is = p.ist + j;
  if (PVC) return (atomicOr(&is->state, kInstFound) & kInstFound) == 0;
  if (atomicMin(&is->best, s) <= s) return 0;
  lock_acquire(&is->lock);
  if (load_relaxed(&is->best) == s) return 1;
  store_release(&is->lock, 0);
  return 0;
}

// Thread 0, after the whole workgroup has written the cover and fenced it: finish the claim.
template <bool PVC>
__device__ __forceinline__ void publish_solution(const Params& p, int j, int32_t s) {
  InstState* is = p.ist + j;
  if (PVC) {
    store_relaxed(&is->best, s);
    fetch_add(ctr_i32(p, kOpen), -1);
  } else {
    store_release(&is->lock, 0);
  }
}

// Thread 0: add this workgroup's nodes on instance j to the instance's counter, and mark the
// instance out of budget once the counter reaches the per-instance budget.
__device__ __forceinline__ void report_nodes(const Params& p, int j, int64_t count) {
  if (count <= 0) return;
  unsigned long long* total = reinterpret_cast<unsigned long long*>(&p.ist[j].nodes);
  const unsigned long long before = fetch_add(total, static_cast<unsigned long long>(count));
  if (p.node_budget > 0 && static_cast<int64_t>(before) + count >= p.node_budget)
    atomicOr(&p.ist[j].state, kInstOutOfBudget);
}

// The hybrid traversal (§IV-A, Fig. 4; PVC differences in §IV-A, termination §IV-C) over every
// instance of the launch. A workgroup takes the root of an unstarted instance or a node from
// the worklist, walks that node's sub-tree depth first with its stack, and loads an instance
// (row pointers) only when the node it takes belongs to another one than the last.
template <bool PVC, bool PROF, int MEM, bool SO>
__global__ void __launch_bounds__(1024) traverse_kernel(Params p) {
  __shared__ Ctrl c;
  __shared__ int32_t rm_list[kListCap];
  __shared__ int32_t heads[kMaxWaves * 64];
  int32_t* st = node_base<MEM>(p, blockIdx.x);
  const int wg = blockIdx.x;
  const int tid = threadIdx.x;
  if (tid == 0) {
    c.flag_epoch = -1;
    c.stop = 0;
    c.list_n = 0;
  }
  ActivityClock<PROF> clk;
  clk.begin();
  if (tid == 0) watch_begin(c);
  uint32_t headers = 0;  // thread 0: node headers read so far
  uint64_t root_header = 0;   // thread 0: a root's header, loaded when the root was taken
  bool header_ready = false;

  int32_t* stack = p.stacks + static_cast<size_t>(wg) * p.depth_cap * p.stride;
  // The stack is a ring of depth_cap entries holding [bot, top): pops take the top, donations
  // take the bottom (the oldest deferred child, nearest its sub-tree root). Every entry belongs
  // to the instance of the sub-tree being walked.
  int top = 0, bot = 0;
  bool have = false;      // a node is in LDS and still to be visited
  bool holding = false;   // this workgroup holds a sub-tree (a root or a worklist node)
  bool marked = false;    // the node in LDS has flagged vertices still to be removed
  int cur = -1;           // instance of the node in LDS
  int32_t cur_k = 0, cur_vtx = 0;
  Node nd = empty_node<MEM>(p, st, rm_list, heads);
  int epoch = 0;
  int64_t nodes = 0, pushes = 0, pops = 0, enqueues = 0, dequeues = 0, insts = 0;
  int64_t unreported = 0;  // nodes on `cur` not yet added to its counter
  int max_depth = 0;
  uint32_t so_path = 0;    // StackOnly: the current path index

  for (;;) {
    if (!have) {
      marked = false;   // whatever node comes next replaces the one in LDS
      __syncthreads();  // every thread has read the last broadcast before thread 0 writes
      if (top > bot) {
        --top;
        node_load(st, stack + static_cast<size_t>(top % p.depth_cap) * p.stride, p.stride);
        ++pops;
        __syncthreads();
        clk.charge(kActAcquire);
      } else if constexpr (SO) {
        // StackOnly (the comparison method of §V-A), as in bitset_traverse_kernel: walk this
        // workgroup's next path down from the root, then take the node at the start depth.
        if (cur < 0) {
          nd = load_instance<MEM>(p, 0, st, rm_list, heads);
          const Instance in = p.inst[0];
          cur = 0;
          cur_k = in.k;
          cur_vtx = in.vtx_off;
          ++insts;
          so_path = static_cast<uint32_t>(wg);
        } else {
          so_path += static_cast<uint32_t>(p.num_wg);
        }
        if (tid == 0) c.err = load_relaxed(&p.ist[0].err_row) != kNoRow;
        __syncthreads();
        if (so_path >= (1u << p.start_depth) || c.err) {
          clk.charge(kActAcquire);
          break;
        }
        build_root(p, nd, 0);
        bool reached = true;
        for (int d = 0; d < p.start_depth && reached; ++d) {
          const bool owner = (so_path >> d) == 0;
          if (tid == 0) {
            const uint64_t h = inst_header(p, cur);
            const int32_t state = static_cast<int32_t>(h >> 32);
            c.drop = (state & kInstOutOfBudget) | (PVC ? (state & kInstFound) : 0);
            c.best = static_cast<int32_t>(static_cast<uint32_t>(h));
          }
          __syncthreads();
          if (c.drop) {
            reached = false;
            break;
          }
          const int64_t bound = PVC ? static_cast<int64_t>(cur_k) : static_cast<int64_t>(c.best) - 1;
          ++nodes;
          if (owner) ++unreported;
          reduce_node(nd, c, bound, p.rules, epoch, clk, marked);
          marked = false;
          const int32_t s = st[nd.n];
          const int64_t r = bound - s;
          int vmax = 0, dmax = 0;
          int32_t degsum = 0;
          if (r >= 0) max_degree_and_sum(nd, c, vmax, dmax, degsum);
          const int64_t edges = degsum / 2;
          if (r < 0 || ((p.rules & kPruneEdges) && (p.rules & kRuleHigh) && edges > r * r)) {
            reached = false;
          } else if (edges == 0) {  // a cover: recorded once, on the owning path
            if (owner) {
              if (tid == 0) c.status = claim_solution<PVC>(p, cur, s);
              __syncthreads();
              if (c.status) {
                uint8_t* cov = p.covers + cur_vtx;
                for (int v = tid; v < nd.n; v += blockDim.x) cov[v] = st[v] < 0;
                __threadfence();
                __syncthreads();
                if (tid == 0) publish_solution<PVC>(p, cur, s);
              }
            }
            reached = false;
          } else {
            if ((so_path >> d) & 1u) mark_neighbourhood(nd, vmax);
            else mark_vertex(nd, vmax);
            marked = true;
          }
          __syncthreads();  // every thread has read c.* before thread 0 writes it again
        }
        clk.charge(kActAcquire);
        if (!reached) continue;
      } else {
        if (holding) {
          if (tid == 0) release_work(p, cur);
          holding = false;
        }
        const int got = dequeue_begin(p, c);
        if (got != 1 && got != 2) {
          clk.charge(kActAcquire);
          break;
        }
        int j;
        if (got == 1) {
          node_load(st, p.payload + static_cast<size_t>(c.slot) * p.stride, p.stride);
          dequeue_finish(p, c);  // ends with a barrier: the node is visible to every thread
          j = st[p.stride - 1];
          ++dequeues;
          if (j < 0 || j >= p.num_inst) {  // cannot happen: every stored node names its instance
            if (tid == 0) {
              atomicMax(ctr_i32(p, kError), 2);
              store_relaxed(ctr_i32(p, kAbort), 1);
            }
            break;
          }
        } else {
          j = static_cast<int>(c.slot);  // an unstarted instance: its root
        }
        holding = true;
        clk.charge(kActAcquire);
        // a root: its input check and its first header are loaded now, while the instance is
        // being staged, instead of one after the other once it is
        int32_t err_row = kNoRow;
        if (got == 2 && tid == 0) {
          err_row = load_relaxed(&p.ist[j].err_row);
          root_header = inst_header(p, j);
          header_ready = true;
        }
        if (j != cur) {
          if (tid == 0 && cur >= 0) report_nodes(p, cur, unreported);
          unreported = 0;
          nd = load_instance<MEM>(p, j, st, rm_list, heads);
          const Instance in = p.inst[j];
          cur = j;
          cur_k = in.k;
          cur_vtx = in.vtx_off;
          ++insts;
        }
        if (got == 2) {
          // c.err, not c.status: slow waves may still be reading the dequeue status
          if (tid == 0) c.err = err_row != kNoRow;
          __syncthreads();
          if (c.err) {  // rejected input: no search (PVC: the instance is settled)
            if (PVC && tid == 0) fetch_add(ctr_i32(p, kOpen), -1);
            header_ready = false;
            continue;
          }
          build_root(p, nd, j);
        }
        clk.charge(kActOther);
      }
      const int pending = st[nd.n + 1];
      if (pending >= 0) {
        __syncthreads();  // every thread has read the pending vertex
        if (tid == 0) st[nd.n + 1] = -1;
        mark_neighbourhood(nd, pending);
        marked = true;
      }
      clk.charge(kActBranch);
      have = true;
    }

    // node header: the instance's flags and current best (one load), and every 16 nodes
    // the launch-wide stop (idle workgroups also look at it while they wait for work)
    if (tid == 0) {
      const uint64_t h = header_ready ? root_header : inst_header(p, cur);
      header_ready = false;
      const int32_t state = static_cast<int32_t>(h >> 32);
      if ((headers++ & 15) == 0) c.stop = search_stopped(p, c);
      c.drop = (state & kInstOutOfBudget) | (PVC ? (state & kInstFound) : 0);
      c.best = static_cast<int32_t>(static_cast<uint32_t>(h));
    }
    __syncthreads();
    clk.charge(kActOther);
    if (c.stop) break;
    if (c.drop) {  // answered or out of budget: drop this node and the rest of the sub-tree
      have = false;
      top = bot;
      continue;
    }

    ++nodes;
    ++unreported;
    if (p.node_budget > 0 && unreported >= p.budget_chunk) {
      if (tid == 0) report_nodes(p, cur, unreported);
      unreported = 0;
    }

    const int64_t bound = PVC ? static_cast<int64_t>(cur_k) : static_cast<int64_t>(c.best) - 1;
    reduce_node(nd, c, bound, p.rules, epoch, clk, marked);
    marked = false;
    clk.charge(kActReduce);

    // stopping condition (§II-B): no cover of size <= bound below this node if r < 0 or
    // |E| > r^2 (every remaining degree is <= r once the high-degree rule has run)
    const int n = nd.n;
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
      if (tid == 0) c.status = claim_solution<PVC>(p, cur, s);
      __syncthreads();
      if (c.status) {
        uint8_t* cov = p.covers + cur_vtx;
        for (int v = tid; v < n; v += blockDim.x) cov[v] = st[v] < 0;
        __threadfence();
        __syncthreads();
        if (tid == 0) publish_solution<PVC>(p, cur, s);
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
      if (try_enqueue(p, nd, c, vmax, oldest, cur)) {
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
    mark_vertex(nd, vmax);
    marked = true;
    clk.charge(kActBranch);
  }
  clk.end();

  if (tid == 0) {
    if (cur >= 0) report_nodes(p, cur, unreported);
    WgStats w{};
    w.nodes = nodes;
    w.pushes = pushes;
    w.pops = pops;
    w.enqueues = enqueues;
    w.dequeues = dequeues;
    w.max_depth = max_depth;
    w.instances = static_cast<int32_t>(insts);
    for (int a = 0; a < kNumActivities; ++a) w.cycles[a] = static_cast<int64_t>(clk.cycles[a]);
    publish_wg_stats(p, wg, w);
  }
}

// Add each lane's x to *dst (dst may differ between lanes, or be null): one atomic per distinct
// destination in the wavefront. Whole wavefront, uniform control flow.
__device__ void add_grouped(int32_t* dst, int32_t x) {
  bool pending = dst != nullptr && x != 0;
  const uint64_t mine_addr = reinterpret_cast<uint64_t>(dst);
  for (;;) {
    const uint64_t m = __builtin_amdgcn_ballot_w64(pending);
    if (!m) break;
    const int leader = first_lane(m);
    const uint64_t target = readlane64(mine_addr, leader);
    const bool mine = pending && mine_addr == target;
    const int32_t sum = wave_sum(mine ? x : 0);
    if (lane_id() == leader) atomicAdd(reinterpret_cast<int32_t*>(target), sum);
    if (mine) pending = false;
  }
}

// After the traversal (256-thread blocks, any grid): check each recorded cover edge by edge
// and count its vertices. One wavefront per 64 consecutive vertices of the launch: a vertex in
// the cover covers its whole row, so only the rows of vertices outside it are walked (as one
// list, one lane per entry), and each entry of such a row must lead into the cover; an
// uncovered edge is counted from each end. Clear the cover output of instances without an
// answer (rejected, out of budget, PVC no). (The traversal's workgroups add their statistics
// to the result block themselves.) Packed entry offsets must fit in int32.
__global__ void __launch_bounds__(256) finalize_kernel(Params p, int64_t vertices,
                                                       int64_t entries, DevResult* res) {
  __shared__ int32_t heads[4 * 64];
  (void)entries;
  const int64_t waves = static_cast<int64_t>(gridDim.x) * (blockDim.x >> 6);
  for (int64_t w = static_cast<int64_t>(blockIdx.x) * (blockDim.x >> 6) + wave_id();
       w * 64 < vertices; w += waves) {
    const int64_t i = w * 64 + lane_id();
    int32_t* ones_dst = nullptr;
    int32_t one = 0;
    int beg = 0, end = 0, j = 0;
    if (i < vertices) {
      j = instance_of_vertex(p, i);
      const Instance in = p.inst[j];
      const InstState is = p.ist[j];
      const bool answer = is.err_row == kNoRow && !(is.state & kInstOutOfBudget) &&
                          (!p.pvc || (is.state & kInstFound));
      uint8_t* cov = p.covers + in.vtx_off;
      const int v = static_cast<int>(i - in.vtx_first);
      if (answer) {
        one = cov[v] != 0;
        if (!one) {
          const int32_t* rp = p.rp_all + in.rp_off;
          beg = static_cast<int>(in.ci_off) + rp[v];
          end = static_cast<int>(in.ci_off) + rp[v + 1];
        }
      } else {
        cov[v] = 0;
      }
      ones_dst = &p.ist[j].cover_count;
    }
    add_grouped(ones_dst, one);
    walk_rows(p.ci_all, heads + 64 * wave_id(), beg, end, j, [&](int u, int jj, int) {
      if (p.covers[p.inst[jj].vtx_off + u] == 0) atomicAdd(&p.ist[jj].uncovered, 1);
    });
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    res->aborted = *ctr_i32(p, kAbort);
    res->error = *ctr_i32(p, kError);
    res->stop_reason = *ctr_i32(p, kStopReason);
    res->q_max_count = *ctr_i32(p, kQMaxCount);
  }
}

// The reduction rules of one node, alone, on a degree array in device memory (instance 0 of
// the launch, one workgroup). A rejected input leaves the degree array alone.
template <int MEM>
__global__ void __launch_bounds__(1024) reduce_kernel(Params p, int32_t* deg, int32_t* s,
                                                      int64_t bound) {
  __shared__ Ctrl c;
  __shared__ int32_t rm_list[kListCap];
  __shared__ int32_t heads[kMaxWaves * 64];
  int32_t* st = node_base<MEM>(p, 0);
  if (threadIdx.x == 0) {
    c.err = load_relaxed(&p.ist[0].err_row) != kNoRow;
    c.flag_epoch = -1;
    c.list_n = 0;
  }
  __syncthreads();
  if (c.err) return;
  const Node nd = load_instance<MEM>(p, 0, st, rm_list, heads);
  const int n = nd.n;
  for (int v = threadIdx.x; v < p.stride; v += blockDim.x)
    st[v] = v < n ? deg[v] : (v == n ? *s : (v == n + 1 ? -1 : 0));
  __syncthreads();
  int epoch = 0;
  reduce_node(nd, c, bound, p.rules, epoch);
  for (int v = threadIdx.x; v < n; v += blockDim.x) deg[v] = st[v] < 0 ? kSent : (st[v] & kDegMask);
  if (threadIdx.x == 0) *s = st[n];
}

// Largest greedy cover size over the launch's instances (the stack depth bound of MVC).
__global__ void __launch_bounds__(256) max_greedy_kernel(Params p, int32_t* out) {
  int32_t m = 0;
  for (int j = threadIdx.x; j < p.num_inst; j += blockDim.x) {
    const int32_t g = p.ist[j].greedy;
    m = g > m ? g : m;
  }
  m = static_cast<int32_t>(wave_max(static_cast<uint64_t>(static_cast<uint32_t>(m))));
  __shared__ int32_t part[4];
  if (lane_id() == 0) part[wave_id()] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t r = part[0];
    for (int w = 1; w < static_cast<int>(blockDim.x >> 6); ++w) r = part[w] > r ? part[w] : r;
    *out = r;
  }
}

// ---- launchers ---------------------------------------------------------------------------------

static int grid_for(int64_t items, int threads, int cap) {
  int64_t blocks = (items + threads - 1) / threads;
  if (blocks < 1) blocks = 1;
  if (blocks > cap) blocks = cap;
  return static_cast<int>(blocks);
}

hipError_t launch_prepare(const Params& p, DevResult* res, int64_t vertices, int64_t entries,
                          hipStream_t stream) {
  const int64_t items = vertices > entries ? vertices : entries;
  const int blocks = std::max(grid_for(items, 256, 4096), grid_for(p.q_cap, 256, 1024));
  hipLaunchKernelGGL(prepare_kernel, dim3(blocks), dim3(256), 0, stream, p, res, vertices,
                     entries);
  return hipGetLastError();
}

// Grid of the greedy launch (one workgroup per instance, at most 65,535); the device-memory
// node array needs this many slots.
int greedy_grid(const Params& p) { return p.num_inst < 65535 ? p.num_inst : 65535; }

// Memory mode of a launch: node in device memory, else in LDS with the row pointers (rp_lds 1)
// or the whole CSR (rp_lds 2) staged after it.
static int mem_mode(bool global_node, int32_t rp_lds) {
  if (global_node) return kMemGlobal;
  return rp_lds >= 2 ? kMemLdsCsr : (rp_lds == 1 ? kMemLdsRp : kMemLds);
}

template <int MEM>
static size_t launch_lds(const Params& p) {
  return MEM == kMemGlobal ? 0 : node_lds_bytes(p.stride, p.n_max, p.rp_lds, p.nnz_max);
}

template <int MEM>
static void greedy_on(const Params& p, int32_t wg_size, hipStream_t stream) {
  hipLaunchKernelGGL(greedy_kernel<MEM>, dim3(greedy_grid(p)), dim3(wg_size), launch_lds<MEM>(p),
                     stream, p);
}

hipError_t launch_greedy(const Params& p, int32_t wg_size, hipStream_t stream) {
  switch (mem_mode(p.gnodes != nullptr, p.rp_lds)) {
    case kMemGlobal: greedy_on<kMemGlobal>(p, wg_size, stream); break;
    case kMemLds: greedy_on<kMemLds>(p, wg_size, stream); break;
    case kMemLdsRp: greedy_on<kMemLdsRp>(p, wg_size, stream); break;
    default: greedy_on<kMemLdsCsr>(p, wg_size, stream); break;
  }
  return hipGetLastError();
}

template <int MEM, bool SO>
static const void* traverse_fn_m(bool pvc, bool prof) {
  if (pvc) return prof ? reinterpret_cast<const void*>(&traverse_kernel<true, true, MEM, SO>)
                       : reinterpret_cast<const void*>(&traverse_kernel<true, false, MEM, SO>);
  return prof ? reinterpret_cast<const void*>(&traverse_kernel<false, true, MEM, SO>)
              : reinterpret_cast<const void*>(&traverse_kernel<false, false, MEM, SO>);
}

// The StackOnly walk-down is a separate instantiation, so the hybrid kernels carry none of its
// registers.
template <bool SO>
static const void* traverse_fn_s(bool pvc, bool prof, int mem) {
  switch (mem) {
    case kMemGlobal: return traverse_fn_m<kMemGlobal, SO>(pvc, prof);
    case kMemLds: return traverse_fn_m<kMemLds, SO>(pvc, prof);
    case kMemLdsRp: return traverse_fn_m<kMemLdsRp, SO>(pvc, prof);
    default: return traverse_fn_m<kMemLdsCsr, SO>(pvc, prof);
  }
}
static const void* traverse_fn(bool pvc, bool prof, int mem, bool stack_only = false) {
  return stack_only ? traverse_fn_s<true>(pvc, prof, mem) : traverse_fn_s<false>(pvc, prof, mem);
}

// A plain launch: the grid is sized by the occupancy API so that all workgroups are normally
// resident together, but the search does not depend on it. A workgroup only ever waits for
// workgroups that have already taken a worklist ticket or an instance's lock (and are
// therefore running); one that starts late finds either work or a zero outstanding-work
// counter.
hipError_t launch_traverse(bool pvc, bool prof, const Params& p, int32_t wg_size,
                           hipStream_t stream) {
  const bool global_node = p.gnodes != nullptr;
  const size_t lds = global_node ? 0 : node_lds_bytes(p.stride, p.n_max, p.rp_lds, p.nnz_max);
  Params args = p;
  void* kargs[] = {&args};
  return hipLaunchKernel(traverse_fn(pvc, prof, mem_mode(global_node, p.rp_lds), p.start_depth > 0),
                         dim3(p.num_wg), dim3(wg_size), kargs, lds, stream);
}

hipError_t launch_finalize(const Params& p, int64_t vertices, int64_t entries, DevResult* res,
                           hipStream_t stream) {
  const int64_t items = vertices;
  hipLaunchKernelGGL(finalize_kernel, dim3(grid_for(items, 256, 1024)), dim3(256), 0, stream, p,
                     vertices, entries, res);
  return hipGetLastError();
}

template <int MEM>
static void reduce_on(const Params& p, int32_t wg_size, int32_t* deg, int32_t* s, int64_t bound,
                      hipStream_t stream) {
  hipLaunchKernelGGL(reduce_kernel<MEM>, dim3(1), dim3(wg_size), launch_lds<MEM>(p), stream, p, deg,
                     s, bound);
}

hipError_t launch_reduce(const Params& p, int32_t wg_size, int32_t* deg, int32_t* s,
                         int64_t bound, hipStream_t stream) {
  switch (mem_mode(p.gnodes != nullptr, p.rp_lds)) {
    case kMemGlobal: reduce_on<kMemGlobal>(p, wg_size, deg, s, bound, stream); break;
    case kMemLds: reduce_on<kMemLds>(p, wg_size, deg, s, bound, stream); break;
    case kMemLdsRp: reduce_on<kMemLdsRp>(p, wg_size, deg, s, bound, stream); break;
    default: reduce_on<kMemLdsCsr>(p, wg_size, deg, s, bound, stream); break;
  }
  return hipGetLastError();
}

hipError_t launch_max_greedy(const Params& p, int32_t* out, hipStream_t stream) {
  hipLaunchKernelGGL(max_greedy_kernel, dim3(1), dim3(256), 0, stream, p, out);
  return hipGetLastError();
}

hipError_t traverse_occupancy(bool pvc, bool prof, bool global_node, int32_t rp_lds,
                              int32_t wg_size, size_t lds_bytes, int* blocks_per_cu) {
  const void* fn = traverse_fn(pvc, prof, mem_mode(global_node, rp_lds));
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, fn, wg_size, lds_bytes);
}

hipError_t set_lds_limit(size_t lds_bytes) {
  for (int mem = kMemLds; mem <= kMemLdsCsr; ++mem) {
    const void* fns[] = {traverse_fn(true, false, mem), traverse_fn(false, false, mem),
                         traverse_fn(true, true, mem), traverse_fn(false, true, mem),
                         traverse_fn(true, false, mem, true), traverse_fn(false, false, mem, true),
                         traverse_fn(true, true, mem, true), traverse_fn(false, true, mem, true)};
    for (const void* fn : fns) {
      hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                         static_cast<int>(lds_bytes));
      if (e != hipSuccess) return e;
    }
  }
  const void* others[] = {
      reinterpret_cast<const void*>(&greedy_kernel<kMemLds>),
      reinterpret_cast<const void*>(&greedy_kernel<kMemLdsRp>),
      reinterpret_cast<const void*>(&greedy_kernel<kMemLdsCsr>),
      reinterpret_cast<const void*>(&reduce_kernel<kMemLds>),
      reinterpret_cast<const void*>(&reduce_kernel<kMemLdsRp>),
      reinterpret_cast<const void*>(&reduce_kernel<kMemLdsCsr>)};
  for (const void* fn : others) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(lds_bytes));
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace vc
