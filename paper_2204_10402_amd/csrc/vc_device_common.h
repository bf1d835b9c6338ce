// vc_device_common.h -- device building blocks shared by the degree-array kernels
// (vc_device.hip) and the bitset kernels (vc_bitset.hip): scoped atomics on the control
// words, wavefront-64 DPP reductions and scans, the worklist protocol, the activity clock.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vc_internal.h"

namespace vc {

constexpr int32_t kSent = -1;
constexpr int kMaxWaves = 16;             // 1024 threads

// ---- scoped atomics ------------------------------------------------------------------------

__device__ __forceinline__ int32_t* ctr_i32(const Params& p, int slot) {
  return p.ctr + slot * kCounterStride;
}
__device__ __forceinline__ unsigned long long* ctr_u64(const Params& p, int slot) {
  return reinterpret_cast<unsigned long long*>(p.ctr + slot * kCounterStride);
}
__device__ __forceinline__ int32_t load_relaxed(int32_t* a) {
  return __hip_atomic_load(a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long load_relaxed(unsigned long long* a) {
  return __hip_atomic_load(a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t load_acquire(uint32_t* a) {
  return __hip_atomic_load(a, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_release(uint32_t* a, uint32_t v) {
  __hip_atomic_store(a, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_release(int32_t* a, int32_t v) {
  __hip_atomic_store(a, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_relaxed(int32_t* a, int32_t v) {
  __hip_atomic_store(a, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t fetch_add(int32_t* a, int32_t v) {
  return __hip_atomic_fetch_add(a, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long fetch_add(unsigned long long* a,
                                                        unsigned long long v) {
  return __hip_atomic_fetch_add(a, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---- wavefront-64 reductions (DPP row operations + lane reads) -----------------------------

template <int CTRL>
__device__ __forceinline__ uint32_t dpp(uint32_t x) {
  return static_cast<uint32_t>(
      __builtin_amdgcn_update_dpp(static_cast<int>(x), static_cast<int>(x), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ uint64_t dpp64(uint64_t x) {
  const uint32_t lo = dpp<CTRL>(static_cast<uint32_t>(x));
  const uint32_t hi = dpp<CTRL>(static_cast<uint32_t>(x >> 32));
  return (static_cast<uint64_t>(hi) << 32) | lo;
}
// DPP controls: quad_perm [1,0,3,2], quad_perm [2,3,0,1], row_half_mirror, row_mirror. After
// the four steps every lane of a 16-lane row holds the row's result.
constexpr int kDppQuadSwap1 = 0xB1;
constexpr int kDppQuadSwap2 = 0x4E;
constexpr int kDppHalfMirror = 0x141;
constexpr int kDppMirror = 0x140;

__device__ __forceinline__ int32_t wave_sum(int32_t x) {
  uint32_t u = static_cast<uint32_t>(x);
  u += dpp<kDppQuadSwap1>(u);
  u += dpp<kDppQuadSwap2>(u);
  u += dpp<kDppHalfMirror>(u);
  u += dpp<kDppMirror>(u);
  const uint32_t r = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(u), 0)) +
                     static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(u), 16)) +
                     static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(u), 32)) +
                     static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(u), 48));
  return static_cast<int32_t>(r);
}

__device__ __forceinline__ uint64_t umax64(uint64_t a, uint64_t b) { return a > b ? a : b; }

__device__ __forceinline__ uint64_t readlane64(uint64_t x, int lane) {
  const uint32_t lo = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(x), lane));
  const uint32_t hi =
      static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(x >> 32), lane));
  return (static_cast<uint64_t>(hi) << 32) | lo;
}

__device__ __forceinline__ uint64_t wave_max(uint64_t x) {
  x = umax64(x, dpp64<kDppQuadSwap1>(x));
  x = umax64(x, dpp64<kDppQuadSwap2>(x));
  x = umax64(x, dpp64<kDppHalfMirror>(x));
  x = umax64(x, dpp64<kDppMirror>(x));
  return umax64(umax64(readlane64(x, 0), readlane64(x, 16)),
                umax64(readlane64(x, 32), readlane64(x, 48)));
}

__device__ __forceinline__ uint32_t wave_max32(uint32_t x) {
  x = max(x, dpp<kDppQuadSwap1>(x));
  x = max(x, dpp<kDppQuadSwap2>(x));
  x = max(x, dpp<kDppHalfMirror>(x));
  x = max(x, dpp<kDppMirror>(x));
  const uint32_t a = max(static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(x), 0)),
                         static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(x), 16)));
  const uint32_t b = max(static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(x), 32)),
                         static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(x), 48)));
  return max(a, b);
}

__device__ __forceinline__ int lane_id() { return static_cast<int>(threadIdx.x) & 63; }
__device__ __forceinline__ int wave_id() { return static_cast<int>(threadIdx.x) >> 6; }
__device__ __forceinline__ int first_lane(uint64_t m) { return __ffsll(static_cast<long long>(m)) - 1; }
__device__ __forceinline__ int bcast(int x, int lane) { return __builtin_amdgcn_readlane(x, lane); }

// ---- per-workgroup LDS control block ------------------------------------------------------

struct Ctrl {
  uint64_t t_start;    // thread 0: the device clock when this workgroup started (watchdog)
  uint64_t t_host;     // thread 0 of workgroup 0: when it last read the host's stop word
  int32_t flag_epoch;  // epoch of the last decide step that marked a vertex
  int32_t status;      // broadcast of a result computed by thread 0
  uint32_t slot;
  uint32_t lap;
  int32_t best;        // broadcast of the current instance's best size (MVC)
  int32_t stop;        // broadcast: the launch is being stopped
  int32_t err;         // broadcast: the instance's input graph was rejected
  int32_t drop;        // broadcast: the current instance is answered or out of budget
  int32_t list_n;      // degree-array removal step: vertices appended to the removal list
  uint64_t red_key[kMaxWaves];
  int32_t red_sum[kMaxWaves];
};

// ---- wavefront building blocks ---------------------------------------------------------------

// Inclusive prefix sum over the 64 lanes: DPP row shifts inside each 16-lane row, then row
// broadcasts (row_bcast:15 to rows 1 and 3, row_bcast:31 to rows 2 and 3).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ int32_t dpp_or_zero(int32_t x) {
  return __builtin_amdgcn_update_dpp(0, x, CTRL, ROW_MASK, 0xF, false);
}
__device__ __forceinline__ int32_t wave_incl_scan(int32_t x) {
  x += dpp_or_zero<0x111, 0xF>(x);  // row_shr:1
  x += dpp_or_zero<0x112, 0xF>(x);  // row_shr:2
  x += dpp_or_zero<0x114, 0xF>(x);  // row_shr:4
  x += dpp_or_zero<0x118, 0xF>(x);  // row_shr:8
  x += dpp_or_zero<0x142, 0xA>(x);  // row_bcast:15
  x += dpp_or_zero<0x143, 0xC>(x);  // row_bcast:31
  return x;
}

__device__ __forceinline__ int shfl(int x, int src_lane) {
  return __builtin_amdgcn_ds_bpermute(src_lane << 2, x);
}

// Index of the k-th (from 0) set bit of m; m must have more than k set bits.
__device__ __forceinline__ int kth_set_bit(uint64_t m, int k) {
  int pos = 0;
  uint32_t w = static_cast<uint32_t>(m);
  int c = __popc(w);
  if (k >= c) {
    k -= c;
    pos = 32;
    w = static_cast<uint32_t>(m >> 32);
  }
#pragma unroll
  for (int half = 16; half > 0; half >>= 1) {
    c = __popc(w & ((1u << half) - 1u));
    if (k >= c) {
      k -= c;
      pos += half;
      w >>= half;
    }
  }
  return pos;
}

__device__ __forceinline__ void backoff(int& spins) {
  if (spins < 8) ++spins;
  for (int i = 0; i < spins; ++i) __builtin_amdgcn_s_sleep(8);
}


// An instance's best size (low half) and state flags (high half), read as one word.
__device__ __forceinline__ uint64_t inst_header(const Params& p, int j) {
  return load_relaxed(reinterpret_cast<unsigned long long*>(&p.ist[j].best));
}

// The device's constant-rate clock (s_memrealtime; its rate is the device's wall-clock rate).
__device__ __forceinline__ uint64_t realtime() { return __builtin_amdgcn_s_memrealtime(); }

// Ticks of that clock between two reads of the host's stop word by workgroup 0.
constexpr uint64_t kHostPollTicks = 5000;

// Thread 0, at the start of a traversal workgroup.
__device__ __forceinline__ void watch_begin(Ctrl& c) {
  c.t_start = realtime();
  c.t_host = c.t_start;
}

// Thread 0: has the launch's time limit run out, or (workgroup 0, every kHostPollTicks) has the
// host asked to stop? Either raises the launch-wide stop, which every workgroup sees at its next
// look at the control words; returns whether it did.
__device__ inline bool watchdog(const Params& p, Ctrl& c) {
  if (p.timeout_ticks == 0 && p.host_abort == nullptr) return false;
  const uint64_t now = realtime();
  int32_t reason = 0;
  if (p.timeout_ticks != 0 && now - c.t_start > p.timeout_ticks) {
    reason = kStopTimeout;
  } else if (p.host_abort != nullptr && blockIdx.x == 0 && now - c.t_host >= kHostPollTicks) {
    c.t_host = now;
    if (__hip_atomic_load(p.host_abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) !=
        p.abort_base)
      reason = kStopHost;
  }
  if (reason == 0) return false;
  atomicMax(ctr_i32(p, kStopReason), reason);
  store_relaxed(ctr_i32(p, kAbort), 1);
  return true;
}

// Thread 0: is the search being stopped: aborted (an internal error, the host, the time
// limit), or (PVC) every instance answered?
__device__ __forceinline__ bool search_stopped(const Params& p, Ctrl& c) {
  return watchdog(p, c) || load_relaxed(ctr_i32(p, kAbort)) != 0 ||
         (p.pvc && load_relaxed(ctr_i32(p, kOpen)) == 0);
}

// Spin lock taken by one thread for a short critical section with no waits inside (an
// instance's cover being written); acquire order on success.
__device__ inline void lock_acquire(int32_t* lock) {
  int spins = 0;
  for (;;) {
    int32_t expected = 0;
    if (__hip_atomic_compare_exchange_strong(lock, &expected, 1, __ATOMIC_ACQUIRE,
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      return;
    backoff(spins);
  }
}

// ---- global worklist -----------------------------------------------------------------------
// A bounded ring of q_cap node slots (a power of two). Ticket t uses slot t % cap in lap
// t / cap; seq[slot] = 2*lap means free for lap `lap`, 2*lap + 1 means filled in lap `lap`.
// `count` is the number of entries producers have reserved and consumers have not: a
// consumer only takes a ticket after lowering a positive count, so it never waits for a
// node that will not come. A producer raises the outstanding-work counter before it
// reserves, so that counter can read zero only when nothing is queued, held or unstarted
// (it starts at the number of instances: one root each).

// Thread 0 tries to reserve a slot for a donated node of instance `inst`; returns 1 with
// c.slot/c.lap set, 0 if the worklist is at its threshold, -1 if the search is being stopped.
// The instance's and the launch's outstanding-work counters are raised first.
__device__ inline int enqueue_reserve(const Params& p, Ctrl& c, int inst) {
  int32_t* count = ctr_i32(p, kQCount);
  const int32_t seen = load_relaxed(count);
  if (seen >= static_cast<int32_t>(p.q_threshold)) return 0;
  fetch_add(p.work + inst, 1);
  fetch_add(ctr_i32(p, kWork), 1);
  const int32_t before = fetch_add(count, 1);  // stays below cap: threshold + 2 num_wg <= cap
  if (before + 1 > load_relaxed(ctr_i32(p, kQMaxCount))) atomicMax(ctr_i32(p, kQMaxCount), before + 1);
  const unsigned long long t = fetch_add(ctr_u64(p, kQTail), 1ull);
  const uint32_t slot = static_cast<uint32_t>(t) & (p.q_cap - 1);
  const uint32_t lap = static_cast<uint32_t>(t / p.q_cap);
  int spins = 0;
  while (load_acquire(p.seq + slot) != 2u * lap) {
    if (search_stopped(p, c)) return -1;
    backoff(spins);
  }
  c.slot = slot;
  c.lap = lap;
  return 1;
}

// Whole workgroup: try to reserve a worklist slot for a donated node. Returns true with
// c.slot / c.lap set; the caller then writes the node and calls enqueue_publish.
__device__ inline bool enqueue_begin(const Params& p, Ctrl& c, int inst) {
  if (threadIdx.x == 0) c.status = enqueue_reserve(p, c, inst);
  __syncthreads();
  return c.status == 1;  // at threshold, or stopping: keep the node locally
}

// Whole workgroup, after every thread has written its part of the node: make the node visible
// at agent scope, then publish the slot.
__device__ inline void enqueue_publish(const Params& p, const Ctrl& c) {
  const uint32_t slot = c.slot, lap = c.lap;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) store_release(p.seq + slot, 2u * lap + 1u);
}

// Thread 0: one look for work. Returns 1 with *slot / *lap set when it has claimed a worklist
// ticket (the caller then waits for that slot to be filled), 2 with *root set to an instance
// whose search has not started, 0 when the launch is finished, -1 when it is being stopped
// (looked at only with check_stop), 3 when nothing is available yet. Queued nodes of started
// instances go first; roots are taken in instance order. The words are read one after
// another, each only when the ones before it offered nothing: loading them together shortened
// a look but made the thousands of idle workgroups of a small search poll the shared control
// lines harder, which slowed the workgroups doing the work more than it saved.
__device__ inline int worklist_take(const Params& p, Ctrl& c, bool check_stop, uint32_t* slot,
                                    uint32_t* lap, int32_t* root) {
  int32_t* count = ctr_i32(p, kQCount);
  if (check_stop && search_stopped(p, c)) return -1;
  if (load_relaxed(count) > 0) {
    if (fetch_add(count, -1) > 0) {
      const unsigned long long h = fetch_add(ctr_u64(p, kQHead), 1ull);
      *slot = static_cast<uint32_t>(h) & (p.q_cap - 1);
      *lap = static_cast<uint32_t>(h / p.q_cap);
      return 1;
    }
    fetch_add(count, 1);  // lost the race for the last entry: give the reservation back
    return 3;
  }
  if (load_relaxed(ctr_i32(p, kRootNext)) < p.num_inst) {
    const int32_t r = fetch_add(ctr_i32(p, kRootNext), 1);
    if (r < p.num_inst) {
      *root = r;
      return 2;
    }
    return 3;
  }
  // nothing queued, held or unstarted: the launch is over
  return load_relaxed(ctr_i32(p, kWork)) == 0 ? 0 : 3;
}

// Whole workgroup: wait for work. Returns 1 with c.slot / c.lap set for a worklist entry (the
// caller reads the node, then calls dequeue_finish), 2 with c.slot set to an instance whose
// search has not started (its root), 0 when the whole launch is finished, -1 when it is being
// stopped. An idle workgroup looks again with exponential back-off, and at the stop flags every
// fourth look.
__device__ inline int dequeue_begin(const Params& p, Ctrl& c) {
  int polls = 0;
  for (;;) {
    if (threadIdx.x == 0) {
      uint32_t slot = 0, lap = 0;
      int32_t root = 0;
      int status = worklist_take(p, c, (polls & 3) == 0, &slot, &lap, &root);
      if (status == 1) {
        int wait = 0;
        while (load_acquire(p.seq + slot) != 2u * lap + 1u) {
          if (search_stopped(p, c)) {
            status = -1;
            break;
          }
          backoff(wait);
        }
        c.slot = slot;
        c.lap = lap;
      } else if (status == 2) {
        c.slot = static_cast<uint32_t>(root);
      } else if (status == 3) {
        const int units = 1 << (polls < 5 ? polls : 5);
        for (int i = 0; i < units; ++i) __builtin_amdgcn_s_sleep(16);
        ++polls;
      }
      c.status = status;
    }
    __syncthreads();
    const int status = c.status;
    if (status != 3) return status;
    __syncthreads();  // every thread has read c.status before thread 0 writes it again
  }
}

// Thread 0: the workgroup has finished a sub-tree of instance `inst` that it took from the
// worklist or as a root.
__device__ inline void release_work(const Params& p, int inst) {
  fetch_add(p.work + inst, -1);
  fetch_add(ctr_i32(p, kWork), -1);
}

// Whole workgroup, after every thread has read its part of the node: free the slot.
__device__ inline void dequeue_finish(const Params& p, const Ctrl& c) {
  const uint32_t slot = c.slot, lap = c.lap;
  __syncthreads();
  if (threadIdx.x == 0) store_release(p.seq + slot, 2u * (lap + 1u));
}

// The CSR row holding entry i: the largest v in [0, n) with rp[v] <= i. Every probe stays in
// rp[0..n), whatever rp holds, so a malformed row_ptr cannot send the search out of bounds.
__device__ __forceinline__ int owner_row(const int32_t* __restrict__ rp, int n, int i) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = lo + ((hi - lo + 1) >> 1);
    if (rp[mid] <= i) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Per-workgroup activity clock of the instrumented kernel (paper §V-D, Fig. 6): shader-clock
// cycles are charged to the activity that just ended. Compiled out when PROF is false.
template <bool PROF>
struct ActivityClock {
  uint64_t cycles[kNumActivities] = {};
  uint64_t mark = 0, start = 0;
  __device__ void begin() {
    if (PROF) start = mark = clock64();
  }
  __device__ void charge(int activity) {
    if (PROF) {
      const uint64_t now = clock64();
      cycles[activity] += now - mark;
      mark = now;
    }
  }
  __device__ void end() {
    if (PROF) {
      cycles[kActTotal] = clock64() - start;
      // the reduction total includes its parts
      cycles[kActReduce] += cycles[kActDeg1] + cycles[kActTri] + cycles[kActHigh] + cycles[kActApply];
    }
  }
};

// Thread 0 of an exiting traversal workgroup: record its statistics and, if it took any work,
// add them into the launch's result block (sums, largest and smallest node count, deepest
// stack, one more active workgroup). Idle workgroups add nothing, so a short launch with many
// idle workgroups does not queue thousands of atomics on one line.
__device__ inline void publish_wg_stats(const Params& p, int wg, const WgStats& w) {
  using ull = unsigned long long;
  p.wg_stats[wg] = w;
  if (w.instances == 0 && w.nodes == 0) return;
  DevResult* r = p.res;
  atomicAdd(&r->active_wgs, 1);
  auto add = [](int64_t* dst, int64_t x) {
    if (x) atomicAdd(reinterpret_cast<ull*>(dst), static_cast<ull>(x));
  };
  add(&r->nodes, w.nodes);
  add(&r->pushes, w.pushes);
  add(&r->pops, w.pops);
  add(&r->enqueues, w.enqueues);
  add(&r->dequeues, w.dequeues);
  add(&r->instances, w.instances);
  for (int a = 0; a < kNumActivities; ++a) add(&r->cycles[a], w.cycles[a]);
  atomicMax(reinterpret_cast<ull*>(&r->wg_nodes_max), static_cast<ull>(w.nodes));
  atomicMin(reinterpret_cast<ull*>(&r->wg_nodes_min), static_cast<ull>(w.nodes));
  if (w.max_depth) atomicMax(&r->max_depth, w.max_depth);
}

}  // namespace vc
