// vc_bitset.hip -- the vertex-cover search for graphs of at most 512 vertices, with a search
// node held as a bitset of live vertices (gfx950).
//
// Same method and same rules as the degree-array kernels in vc_device.hip (paper §II-B, §IV):
// the same passes in the same order with the same tie-breaks, the same branching vertex, the
// same child order, the same stack / worklist protocol. Only the representation of an
// intermediate graph differs: instead of a degree array (§IV-B) a node is the set L of live
// vertices (W = ceil(n/64) 64-bit words, held in scalar registers) plus |S|. It is just as
// self-contained, given the read-only adjacency, and W*8 + 8 bytes instead of 4(n+2). A degree
// is recomputed as popcount(adj[v] & L).
//
// One wavefront per workgroup. Lane l holds vertices l, 64+l, ..., (W-1)*64+l and their W
// adjacency words each in vector registers; the whole adjacency matrix also sits in LDS for
// random access (the triangle test). A rule pass is a handful of ballots and bit operations;
// the main loop has no barriers except inside the worklist protocol.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vc_device_common.h"
#include "vc_internal.h"

namespace vc {

template <int W>
struct Rows {  // this lane's vertices (w*64 + lane) and their adjacency words
  uint64_t adj[W][W];
};

template <int W>
struct Live {  // a search node, uniform across the wavefront
  uint64_t bits[W];
  int32_t s;
};

__device__ __forceinline__ uint64_t ballot(bool b) { return __builtin_amdgcn_ballot_w64(b); }

__device__ __forceinline__ uint64_t uniform64(uint64_t x) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(x));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(x >> 32));
  return (static_cast<uint64_t>(hi) << 32) | lo;
}

// Lane mask test: bit `lane` of a wavefront-uniform 64-bit mask, used directly as the lane's
// condition (the mask becomes the lane mask of one v_cndmask; no shift per lane).
__device__ __forceinline__ bool lane_in(uint64_t m) { return __builtin_amdgcn_inverse_ballot_w64(m); }

// Is this lane's vertex of word wv live?
template <int W>
__device__ __forceinline__ bool held_live(const Live<W>& L, int wv) {
  return lane_in(L.bits[wv]);
}

// Bit x of a W-word mask (x < 64 W), without indexing the register array at run time.
template <int W>
__device__ __forceinline__ bool bit_of(const uint64_t (&M)[W], int x) {
  uint64_t word = 0;
#pragma unroll
  for (int w = 0; w < W; ++w) word = (x >> 6) == w ? M[w] : word;
  return (word >> (x & 63)) & 1ull;
}

// Per-lane cached degrees of the held vertices, and per-lane marks of held degree-two vertices
// already known to lie in no triangle (bit wv of no_tri: the lane's vertex of word wv; kept in
// a vector register rather than as W uniform masks, which would add to the scalar registers
// the traversal loop holds). Invariant at every rule pass: for each live held vertex v,
// deg = |N(v) ∩ L| (entries of removed vertices are stale; every use masks them with L). Along
// one root-to-leaf path vertices are only ever removed, so a vertex that still has degree two
// still has the same two neighbours, and if they were not adjacent they still are not: the
// marks stay valid down a path and are cleared whenever the node is replaced by one that is
// not its descendant (a pop, a dequeue, a root).
template <int W>
struct Degrees {
  int32_t deg[W];
  uint32_t no_tri;
};

// All degrees from scratch: deg(v) = popcount(adj(v) & L) over W words.
template <int W>
__device__ __forceinline__ void degrees_full(const Rows<W>& r, const Live<W>& L, Degrees<W>& D) {
#pragma unroll
  for (int wv = 0; wv < W; ++wv) {
    int d = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) d += __popcll(r.adj[wv][w] & L.bits[w]);
    D.deg[wv] = d;
  }
}

// The held vertices adjacent to vertex w*64 + b lose one degree. W is a compile-time word of
// the caller's unrolled loop; b is uniform, so the half select is a scalar condition.
template <int W>
__device__ __forceinline__ void drop_neighbour(const Rows<W>& r, int w, int b, Degrees<W>& D) {
#pragma unroll
  for (int wv = 0; wv < W; ++wv) {
    const uint64_t a = r.adj[wv][w];
    const uint32_t half = (b & 32) ? static_cast<uint32_t>(a >> 32) : static_cast<uint32_t>(a);
    D.deg[wv] -= static_cast<int32_t>(__builtin_amdgcn_ubfe(half, static_cast<uint32_t>(b & 31), 1u));
  }
}

// Remove the set F from the node: |S| grows by the number of live vertices in F (§IV-B, with
// the |S| counter) and the degrees follow, one removed vertex at a time for fewer than W of
// them, from scratch for more.
template <int W>
__device__ __forceinline__ int remove_set(const Rows<W>& r, Live<W>& L, const uint64_t (&F)[W],
                                          Degrees<W>& D) {
  uint64_t R[W];
  int removed = 0;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    R[w] = F[w] & L.bits[w];
    removed += __popcll(R[w]);
    L.bits[w] &= ~R[w];
  }
  L.s += removed;
  // one removed vertex costs 3W VALU and about 7 scalar instructions, a full count 4W^2 VALU
  if (removed >= W) {
    degrees_full(r, L, D);
  } else if (removed > 0) {
#pragma unroll
    for (int w = 0; w < W; ++w) {
      uint64_t m = R[w];
      while (m) {
        const int b = __ffsll(static_cast<long long>(m)) - 1;
        m &= m - 1;
        drop_neighbour(r, w, b, D);
      }
    }
  }
  return removed;
}

// Degree-one rule (§II-B, tie-breaks §IV-D). A live u is removed if it has a degree-one live
// neighbour c and either deg(u) != 1 or u < c (for deg(u) = 1, c is its only neighbour).
// With H the live vertices next to a degree-one vertex: every u in H of degree other than
// one goes; a u in H of degree one forms a mutual pair with its only neighbour, and only the
// smaller of the two goes.
template <int W>
__device__ __forceinline__ int pass_degree_one(const Rows<W>& r, Live<W>& L, Degrees<W>& D) {
  uint64_t D1[W];
  uint64_t any = 0;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    D1[w] = ballot(D.deg[w] == 1) & L.bits[w];
    any |= D1[w];
  }
  if (!any) return 0;
  uint64_t F[W], M[W];
  uint64_t mutual = 0;
#pragma unroll
  for (int wv = 0; wv < W; ++wv) {
    uint32_t near = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
      const uint64_t m = r.adj[wv][w] & D1[w];
      near |= static_cast<uint32_t>(m) | static_cast<uint32_t>(m >> 32);
    }
    const uint64_t H = ballot(near != 0) & L.bits[wv];
    F[wv] = H & ~D1[wv];
    M[wv] = H & D1[wv];
    mutual |= M[wv];
  }
  if (mutual) {
    const int lane = lane_id();
#pragma unroll
    for (int wv = 0; wv < W; ++wv) {
      bool bigger = false;
#pragma unroll
      for (int w = 0; w < W; ++w) {
        const uint64_t m = r.adj[wv][w] & D1[w];
        if (w > wv) bigger |= m != 0;
        if (w == wv) bigger |= ((m >> lane) >> 1) != 0;  // a neighbour with a larger id
      }
      F[wv] |= ballot(lane_in(M[wv]) && bigger);
    }
  }
  return remove_set(r, L, F, D);
}

// Lowest set bit of a W-word mask (the mask is not empty): the minimum over its 32-bit halves
// of (first set bit | 32 * half index), where an empty half gives 0xFFFFFFFF.
template <int W>
__device__ __forceinline__ int lowest_bit(const uint64_t (&N)[W]) {
  uint32_t best = 0xFFFFFFFFu;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    const uint32_t lo = static_cast<uint32_t>(N[w]), hi = static_cast<uint32_t>(N[w] >> 32);
    const uint32_t flo = lo ? (static_cast<uint32_t>(__builtin_ctz(lo)) | (64u * w)) : 0xFFFFFFFFu;
    const uint32_t fhi = hi ? (static_cast<uint32_t>(__builtin_ctz(hi)) | (64u * w + 32u)) : 0xFFFFFFFFu;
    best = min(best, min(flo, fhi));
  }
  return static_cast<int>(best);
}

// Degree-two-triangle rule (§II-B, tie-break §IV-D). A live v of degree two whose neighbours
// a < b are adjacent fires unless a or b is a degree-two vertex with a smaller id; the live
// neighbours of firing vertices (exactly their a and b) are removed. Degree-two vertices not
// yet marked in D.no_tri are checked (row a of the adjacency matrix against {a, b}); the pass ends
// there unless one of them lies in a triangle.
template <int W>
__device__ __forceinline__ int pass_triangle(const Rows<W>& r, Live<W>& L, Degrees<W>& D,
                                             const uint64_t* __restrict__ adj_lds) {
  uint64_t C[W], A[W];
  uint64_t any = 0;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    C[w] = ballot(D.deg[w] == 2 && !((D.no_tri >> w) & 1u)) & L.bits[w];
    any |= C[w];
  }
  if (!any) return 0;
  uint64_t anytri = 0;
#pragma unroll
  for (int wv = 0; wv < W; ++wv) {
    const uint64_t check = C[wv];
    A[wv] = 0;
    if (check) {
      bool adjacent = false;
      if (lane_in(check)) {
        uint64_t N[W];
#pragma unroll
        for (int w = 0; w < W; ++w) N[w] = r.adj[wv][w] & L.bits[w];
        const int a = min(lowest_bit<W>(N), 64 * W - 1);  // N holds exactly two bits
        uint32_t hit = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) {
          const uint64_t x = adj_lds[a * W + w] & N[w];
          hit |= static_cast<uint32_t>(x) | static_cast<uint32_t>(x >> 32);
        }
        adjacent = hit != 0;
      }
      A[wv] = ballot(adjacent) & check;
      if (lane_in(check & ~A[wv])) D.no_tri |= 1u << wv;
      anytri |= A[wv];
    }
  }
  if (!anytri) return 0;
  // A degree-two vertex lies in a triangle: the firing decisions with their tie-breaks.
  uint64_t D2[W];
#pragma unroll
  for (int w = 0; w < W; ++w) D2[w] = ballot(D.deg[w] == 2) & L.bits[w];
  const int lane = lane_id();
  uint64_t Fire[W];
#pragma unroll
  for (int wv = 0; wv < W; ++wv) {
    bool fires = false;
    if (lane_in(A[wv])) {
      const int v = wv * 64 + lane;
      int a = -1, b = -1;
#pragma unroll
      for (int w = 0; w < W; ++w) {
        uint64_t m = r.adj[wv][w] & L.bits[w];
        while (m && b < 0) {
          const int x = w * 64 + (__ffsll(static_cast<long long>(m)) - 1);
          m &= m - 1;
          if (a < 0) a = x; else b = x;
        }
      }
      const bool a2 = bit_of<W>(D2, a);
      const bool b2 = bit_of<W>(D2, b);
      fires = !((a2 && a < v) || (b2 && b < v));
    }
    Fire[wv] = ballot(fires);
  }
  uint64_t F[W];
#pragma unroll
  for (int wu = 0; wu < W; ++wu) {
    bool near = false;
#pragma unroll
    for (int w = 0; w < W; ++w) near |= (r.adj[wu][w] & L.bits[w] & Fire[w]) != 0;
    F[wu] = ballot(near) & L.bits[wu];
  }
  return remove_set(r, L, F, D);
}

// High-degree rule (§II-B): degree above r = bound - |S| (r >= 0 here).
template <int W>
__device__ __forceinline__ int pass_high_degree(const Rows<W>& r, Live<W>& L, Degrees<W>& D,
                                                int32_t rr) {
  uint64_t F[W];
#pragma unroll
  for (int w = 0; w < W; ++w) F[w] = ballot(D.deg[w] > rr) & L.bits[w];
  return remove_set(r, L, F, D);
}

// The rules until the graph stops changing or |S| exceeds bound (same order as the
// degree-array kernels). Callers clamp bound to [-1, n]: a larger bound (PVC with k >= n)
// removes and prunes exactly as n does, since no live degree reaches n - |S|.
template <int W>
__device__ __forceinline__ void reduce_bits(const Rows<W>& r, Live<W>& L, Degrees<W>& D,
                                            const uint64_t* adj_lds, int32_t bound, int rules) {
  // A pass is skipped when nothing has been removed since it last found nothing (its inputs
  // are unchanged), as in the degree-array kernels.
  int changes = 0, quiet1 = -1, quiet2 = -1, quiet3 = -1;
  for (;;) {
    const int32_t s0 = L.s;
    if (s0 > bound) return;
    if ((rules & kRuleDeg1) && quiet1 != changes) {
      if (pass_degree_one(r, L, D)) {
        ++changes;
        if (L.s > bound) return;
      } else {
        quiet1 = changes;
      }
    }
    if ((rules & kRuleTri) && quiet2 != changes) {
      if (pass_triangle(r, L, D, adj_lds)) {
        ++changes;
        if (L.s > bound) return;
      } else {
        quiet2 = changes;
      }
    }
    if ((rules & kRuleHigh) && quiet3 != changes) {
      if (pass_high_degree(r, L, D, bound - L.s)) ++changes;
      else quiet3 = changes;
    }
    if (L.s == s0) return;
  }
}

// Live vertex of maximum degree (smallest id on ties) and the sum of live degrees, from the
// cached degrees: one 32-bit key (degree << 16 | 0xFFFF - id) per vertex, reduced with DPP.
template <int W>
__device__ __forceinline__ void bits_max_degree(const Live<W>& L, const Degrees<W>& D, int& vmax,
                                                int32_t& degsum) {
  uint32_t key = 0;
  int32_t sum = 0;
  const int lane = lane_id();
#pragma unroll
  for (int wv = 0; wv < W; ++wv) {
    const bool live = held_live(L, wv);
    const uint32_t k = (static_cast<uint32_t>(D.deg[wv]) << 16) |
                       (0xFFFFu - static_cast<uint32_t>(wv * 64 + lane));
    key = max(key, live ? k : 0u);
    sum += live ? D.deg[wv] : 0;
  }
  key = wave_max32(key);
  degsum = wave_sum(sum);
  vmax = static_cast<int>(0xFFFFu - (key & 0xFFFFu));
}

// The v_max child: v joins the cover.
template <int W>
__device__ __forceinline__ void remove_vertex_bits(const Rows<W>& r, Live<W>& L, Degrees<W>& D,
                                                   int v) {
  const int wv = v >> 6, b = v & 63;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    if (w == wv) {
      L.bits[w] &= ~(1ull << b);
      drop_neighbour(r, w, b, D);
    }
  }
  L.s += 1;
}

// The N(v) child: every live neighbour of v joins the cover.
template <int W>
__device__ __forceinline__ void remove_neighbourhood_bits(const Rows<W>& r, Live<W>& L,
                                                          Degrees<W>& D, int v,
                                                          const uint64_t* adj_lds) {
  uint64_t F[W];
#pragma unroll
  for (int w = 0; w < W; ++w) F[w] = uniform64(adj_lds[v * W + w]);
  remove_set(r, L, F, D);
}

// A node taken from a stack or the worklist (or a root): its removal of N(pending) goes to
// the live set first, then the degrees are computed once.
template <int W>
__device__ __forceinline__ void enter_node(const Rows<W>& r, Live<W>& L, Degrees<W>& D,
                                           int pending, const uint64_t* adj_lds) {
  if (pending >= 0) {
    int removed = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
      const uint64_t f = uniform64(adj_lds[pending * W + w]) & L.bits[w];
      removed += __popcll(f);
      L.bits[w] &= ~f;
    }
    L.s += removed;
  }
  degrees_full(r, L, D);
  D.no_tri = 0;
}


// A stored node: W words of live bits (lo/hi 32-bit halves), |S|, then one word packing the
// pending vertex plus one (10 bits, n <= 512) with the instance (launch-local index below
// 2^22, shifted left 10), padding to a multiple of four words. Lane 0 writes and reads every
// stored node, so a node pushed on the workgroup's stack is read back in program order, and
// the worklist publishes it with one release store.
template <int W>
constexpr int bits_stride() {
  return ((2 * W + 2) + 3) & ~3;
}
constexpr int kPendingBits = 10;

template <int W>
__device__ __forceinline__ void bits_store(int32_t* dst, const Live<W>& L, int pending, int inst) {
  if (lane_id() == 0) {
#pragma unroll
    for (int w = 0; w < W; ++w) {
      dst[2 * w] = static_cast<int32_t>(static_cast<uint32_t>(L.bits[w]));
      dst[2 * w + 1] = static_cast<int32_t>(static_cast<uint32_t>(L.bits[w] >> 32));
    }
    dst[2 * W] = L.s;
    dst[2 * W + 1] = static_cast<int32_t>(static_cast<uint32_t>(pending + 1) |
                                          (static_cast<uint32_t>(inst) << kPendingBits));
  }
}

// Node words read by lane 0 into (uniform) L, pending vertex and instance.
template <int W>
__device__ __forceinline__ void bits_unpack(const uint32_t (&x)[2 * W + 2], Live<W>& L,
                                            int& pending, int& inst) {
#pragma unroll
  for (int w = 0; w < W; ++w) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane(x[2 * w]);
    const uint32_t hi = __builtin_amdgcn_readfirstlane(x[2 * w + 1]);
    L.bits[w] = (static_cast<uint64_t>(hi) << 32) | lo;
  }
  L.s = __builtin_amdgcn_readfirstlane(x[2 * W]);
  const uint32_t tag = __builtin_amdgcn_readfirstlane(x[2 * W + 1]);
  pending = static_cast<int>(tag & ((1u << kPendingBits) - 1u)) - 1;
  inst = static_cast<int>(tag >> kPendingBits);
}

template <int W>
__device__ __forceinline__ void bits_load(const int32_t* src, Live<W>& L, int& pending, int& inst) {
  uint32_t x[2 * W + 2];
  if (lane_id() == 0) {
#pragma unroll
    for (int i = 0; i < 2 * W + 2; ++i) x[i] = static_cast<uint32_t>(src[i]);
  }
  bits_unpack<W>(x, L, pending, inst);
}

// The same from an LDS stack entry: every lane reads the same words (an LDS broadcast, no
// exec mask to set up), and the reads are LDS instructions that wait only for LDS.
template <int W>
__device__ __forceinline__ void bits_load_lds(const int32_t* src, Live<W>& L, int& pending,
                                              int& inst) {
  uint32_t x[2 * W + 2];
#pragma unroll
  for (int i = 0; i < 2 * W + 2; ++i) x[i] = static_cast<uint32_t>(src[i]);
  bits_unpack<W>(x, L, pending, inst);
}

// Instance j: its adjacency rows into LDS (all rows) and this lane's rows into registers.
template <int W>
__device__ __forceinline__ int load_adjacency(const Params& p, int j, uint64_t* adj_lds,
                                              Rows<W>& r) {
  const Instance in = p.inst[j];
  const uint64_t* rows = p.bits + static_cast<int64_t>(in.vtx_first) * W;
  __syncthreads();  // the previous instance's rows are no longer read
  for (int i = threadIdx.x; i < in.n * W; i += blockDim.x) adj_lds[i] = rows[i];
#pragma unroll
  for (int wv = 0; wv < W; ++wv) {
    const int v = wv * 64 + lane_id();
#pragma unroll
    for (int w = 0; w < W; ++w) r.adj[wv][w] = v < in.n ? rows[v * W + w] : 0ull;
  }
  __syncthreads();
  return in.n;
}

// The root of an instance with n vertices: every vertex live, |S| = 0.
template <int W>
__device__ __forceinline__ void root_bits(Live<W>& L, int n) {
#pragma unroll
  for (int w = 0; w < W; ++w) {
    const int lo = w * 64, cnt = n - lo;
    L.bits[w] = cnt <= 0 ? 0ull : (cnt >= 64 ? ~0ull : ((1ull << cnt) - 1ull));
  }
  L.s = 0;
}

template <int W>
__device__ __forceinline__ void write_cover(uint8_t* cov, const Live<W>& L, int n) {
#pragma unroll
  for (int wv = 0; wv < W; ++wv) {
    const int v = wv * 64 + lane_id();
    if (v < n) cov[v] = !held_live(L, wv);
  }
}

// ---- worklist protocol for a one-wavefront workgroup ----------------------------------------
// Lane 0 runs the whole protocol (reservation, the node copy, the release / acquire of the slot
// ticket), so one agent-scope release store orders the node's words before the ticket and one
// acquire load orders them after it; the result reaches the other lanes by readfirstlane.

// Donate a deferred child of instance `inst` to the worklist; true if the worklist took it.
// The child is the stored node at `oldest` (the bottom of this workgroup's stack) when that is
// not null, else node L with `pending` as its branch vertex.
template <int W>
__device__ __forceinline__ bool bits_enqueue(const Params& p, Ctrl& c, const Live<W>& L,
                                             int pending, const int32_t* oldest, int inst) {
  int ok = 0;
  if (lane_id() == 0) {
    ok = enqueue_reserve(p, c, inst) == 1;
    if (ok) {
      int32_t* dst = p.payload + static_cast<size_t>(c.slot) * p.stride;
      if (oldest) {
#pragma unroll
        for (int i = 0; i < 2 * W + 2; ++i) dst[i] = oldest[i];
      } else {
        bits_store<W>(dst, L, pending, inst);
      }
      store_release(p.seq + c.slot, 2u * c.lap + 1u);
    }
  }
  return __builtin_amdgcn_readfirstlane(ok);
}

// Take work. Returns 1 with L / pending / inst set from a worklist node, 2 with inst set to an
// unstarted instance (its root), 0 when the launch is over, -1 when it is being stopped. Queued
// nodes go first, then roots in instance order; idle polling as in dequeue_begin.
template <int W>
__device__ __forceinline__ int bits_dequeue(const Params& p, Ctrl& c, Live<W>& L, int& pending,
                                            int& inst) {
  int status = 3;
  uint32_t words[2 * W + 2];
  int root = 0;
  if (lane_id() == 0) {
    int polls = 0;
    while (status == 3) {
      uint32_t slot = 0, lap = 0;
      status = worklist_take(p, c, (polls & 3) == 0, &slot, &lap, &root);
      if (status == 1) {
        int wait = 0;
        while (load_acquire(p.seq + slot) != 2u * lap + 1u) {
          if (search_stopped(p, c)) {
            status = -1;
            break;
          }
          backoff(wait);
        }
        if (status == 1) {
          const int32_t* src = p.payload + static_cast<size_t>(slot) * p.stride;
#pragma unroll
          for (int i = 0; i < 2 * W + 2; ++i) words[i] = static_cast<uint32_t>(src[i]);
          store_release(p.seq + slot, 2u * (lap + 1u));
        }
      } else if (status == 3) {
        const int units = 1 << (polls < 5 ? polls : 5);
        for (int i = 0; i < units; ++i) __builtin_amdgcn_s_sleep(16);
        ++polls;
      }
    }
  }
  status = __builtin_amdgcn_readfirstlane(status);
  if (status == 1) bits_unpack<W>(words, L, pending, inst);
  else if (status == 2) inst = __builtin_amdgcn_readfirstlane(root);
  return status;
}

// ---- kernels -----------------------------------------------------------------------------------

// Greedy approximation (§II-B), as greedy_kernel, on bitset nodes: one workgroup per instance
// (grid-stride loop over the launch's instances).
template <int W>
__global__ void __launch_bounds__(64) bitset_greedy_kernel(Params p) {
  extern __shared__ uint64_t adj_lds[];
  for (int j = blockIdx.x; j < p.num_inst; j += gridDim.x) {
    if (__builtin_amdgcn_readfirstlane(load_relaxed(&p.ist[j].err_row)) != kNoRow) continue;
    Rows<W> r;
    const int n = load_adjacency<W>(p, j, adj_lds, r);
    Live<W> L;
    Degrees<W> D;
    root_bits<W>(L, n);
    enter_node<W>(r, L, D, -1, adj_lds);
    const int32_t unbounded = 0x3FFFFFFF;
    for (;;) {
      reduce_bits<W>(r, L, D, adj_lds, unbounded, kRuleDeg1 | kRuleTri);
      int vmax;
      int32_t degsum;
      bits_max_degree<W>(L, D, vmax, degsum);
      if (degsum == 0) break;
      remove_vertex_bits<W>(r, L, D, vmax);
    }
    write_cover<W>(p.covers + p.inst[j].vtx_off, L, n);
    if (threadIdx.x == 0) {
      p.ist[j].best = L.s;
      p.ist[j].greedy = L.s;
    }
  }
}

// Lane 0: claim / publish a cover of size s for instance j (see claim_solution in the
// degree-array kernels; the same protocol).
template <bool PVC>
__device__ __forceinline__ int bits_claim(const Params& p, int j, int32_t s) {
  InstState* is = p.ist + j;
  if (PVC) return (atomicOr(&is->state, kInstFound) & kInstFound) == 0;
  if (atomicMin(&is->best, s) <= s) return 0;
  lock_acquire(&is->lock);
  if (load_relaxed(&is->best) == s) return 1;
  store_release(&is->lock, 0);
  return 0;
}

template <bool PVC>
__device__ __forceinline__ void bits_publish(const Params& p, int j, int32_t s) {
  InstState* is = p.ist + j;
  if (PVC) {
    store_relaxed(&is->best, s);
    fetch_add(ctr_i32(p, kOpen), -1);
  } else {
    store_release(&is->lock, 0);
  }
}

// Lane 0: add `count` nodes to instance j; returns 1 if that used up the instance's budget.
__device__ __forceinline__ int bits_report_nodes(const Params& p, int j, uint32_t count) {
  if (count == 0) return 0;
  unsigned long long* total = reinterpret_cast<unsigned long long*>(&p.ist[j].nodes);
  const unsigned long long before = fetch_add(total, static_cast<unsigned long long>(count));
  if (p.node_budget > 0 && static_cast<int64_t>(before + count) >= p.node_budget) {
    atomicOr(&p.ist[j].state, kInstOutOfBudget);
    return 1;
  }
  return 0;
}

// Nodes between two reads of the node header (a power of two).
constexpr uint32_t kPollNodes = 16;

// The hybrid traversal (§IV-A, Fig. 4; termination §IV-C) on bitset nodes, over every instance
// of the launch (as traverse_kernel).
template <int W, bool PVC, bool PROF, bool SO>
__global__ void __launch_bounds__(64) bitset_traverse_kernel(Params p) {
  extern __shared__ uint64_t adj_lds[];
  __shared__ Ctrl c;
  // 64-bit statistics, kept by lane 0 in LDS: the loop's scalar registers hold only the 32-bit
  // counts since the last flush
  __shared__ WgStats tally;
  const int wg = blockIdx.x;
  const int tid = threadIdx.x;
  Rows<W> r;
  ActivityClock<PROF> clk;
  clk.begin();
  if (tid == 0) {
    watch_begin(c);
    tally = WgStats{};
  }

  constexpr int kStride = bits_stride<W>();
  // Lane 0 alone writes and reads stack entries, in program order, so the ring needs no
  // barrier in LDS either.
  // The ring lives in LDS after the adjacency matrix (stack_lds) or in device memory. The two
  // are addressed through separate pointers, each access under a uniform branch, so that LDS
  // entries are read and written with LDS instructions rather than flat ones (a flat access
  // waits for every outstanding memory operation, the node header's load included).
  const bool stack_lds = p.stack_lds != 0;
  int32_t* const lstack = reinterpret_cast<int32_t*>(adj_lds + static_cast<size_t>(p.n_max) * W);
  int32_t* const gstack = p.stacks + static_cast<size_t>(wg) * p.depth_cap * kStride;
  // The stack is a ring of depth_cap entries holding [bot, top): pops take the top, donations
  // take the bottom (the oldest deferred child, nearest its sub-tree root). Every entry belongs
  // to the instance of the sub-tree being walked.
  int top = 0, bot = 0;
  // ring slots of top and bot, kept reduced modulo depth_cap (no division per push or pop)
  int top_slot = 0, bot_slot = 0;
  const int cap = p.depth_cap;
  bool have = false, holding = false;
  int cur = -1, cur_n = 0;
  int32_t cur_k = 0, cur_vtx = 0;
  // Statistics: nodes and stack traffic are counted in 32 bits since the last flush (instance
  // switch, budget report, or every 2^30 nodes) and folded into `tally` there.
  uint32_t unreported = 0, pushes32 = 0, pops32 = 0;  // since the last flush
  const uint32_t flush_at = p.node_budget > 0 ? static_cast<uint32_t>(p.budget_chunk) : (1u << 30);
  int max_depth = 0;
  uint32_t headers = 0;  // node headers read so far
  uint32_t so_path = 0;  // StackOnly: the current path index
  int seen_inst = -1;    // the instance whose header was last read, and what it showed:
  int32_t seen_best = 0; // MVC: its best (lowered by this workgroup's own covers)
  bool inst_done = false;  // it is answered (PVC) or out of budget
  int32_t seen_count = 0;  // worklist count at the last header
  int stop = 0;            // the launch is being stopped
  Live<W> L;
  Degrees<W> D;

  for (;;) {
    if (!have) {
      int pending, inst;
      if (top > bot) {
        --top;
        top_slot = top_slot == 0 ? cap - 1 : top_slot - 1;
        if (stack_lds) bits_load_lds<W>(lstack + top_slot * kStride, L, pending, inst);
        else bits_load<W>(gstack + static_cast<size_t>(top_slot) * kStride, L, pending, inst);
        ++pops32;
        clk.charge(kActAcquire);
      } else if constexpr (SO) {
        // StackOnly (the comparison method of §V-A): no worklist. This workgroup's sub-trees
        // are the paths wg, wg + num_wg, ... < 2^start_depth (bit d: which child at depth d);
        // it walks each path down from the root, then walks the sub-tree with its stack. A node
        // above the start depth counts for the instance only on the path whose remaining bits
        // are zero, so the instance's node count is the tree's.
        if (cur < 0) {
          cur_n = load_adjacency<W>(p, 0, adj_lds, r);
          const Instance in = p.inst[0];
          cur = 0;
          cur_k = min(in.k, cur_n);  // a k beyond n acts as n (see reduce_bits)
          cur_vtx = in.vtx_off;
          if (tid == 0) ++tally.instances;
          so_path = static_cast<uint32_t>(wg);
        } else {
          so_path += static_cast<uint32_t>(p.num_wg);
        }
        const int rejected =
            __builtin_amdgcn_readfirstlane(load_relaxed(&p.ist[0].err_row) != kNoRow);
        if (so_path >= (1u << p.start_depth) || rejected) {
          clk.charge(kActAcquire);
          break;
        }
        root_bits<W>(L, cur_n);
        enter_node<W>(r, L, D, -1, adj_lds);
        pending = -1;
        bool reached = true;
        for (int d = 0; d < p.start_depth && reached; ++d) {
          const bool owner = (so_path >> d) == 0;
          const uint64_t h = uniform64(inst_header(p, cur));
          const int32_t state = static_cast<int32_t>(h >> 32);
          if ((state & kInstOutOfBudget) || (PVC && (state & kInstFound))) {
            reached = false;
            break;
          }
          const int32_t bound = PVC ? cur_k : static_cast<int32_t>(h) - 1;
          if (owner) ++unreported;  // counted for the instance (and the workgroup) at the flush
          else if (tid == 0) ++tally.nodes;  // a walk through a node another path owns
          reduce_bits<W>(r, L, D, adj_lds, bound, p.rules);
          const int32_t rr = bound - L.s;
          int vmax = 0;
          int32_t degsum = 0;
          if (rr >= 0) bits_max_degree<W>(L, D, vmax, degsum);
          const int32_t edges = degsum / 2;
          if (rr < 0 || ((p.rules & kPruneEdges) && (p.rules & kRuleHigh) && rr < cur_n &&
                         edges > rr * rr)) {
            reached = false;
          } else if (edges == 0) {  // a cover: recorded once, on the owning path
            if (owner) {
              int won = 0;
              if (tid == 0) won = bits_claim<PVC>(p, cur, L.s);
              if (__builtin_amdgcn_readfirstlane(won)) {
                write_cover<W>(p.covers + cur_vtx, L, cur_n);
                __threadfence();
                if (tid == 0) bits_publish<PVC>(p, cur, L.s);
              }
            }
            reached = false;
          } else if ((so_path >> d) & 1u) {
            remove_neighbourhood_bits<W>(r, L, D, vmax, adj_lds);
          } else {
            remove_vertex_bits<W>(r, L, D, vmax);
          }
        }
        clk.charge(kActAcquire);
        if (!reached) continue;
      } else {
        if (holding) {
          if (tid == 0) release_work(p, cur);
          holding = false;
        }
        const int got = bits_dequeue<W>(p, c, L, pending, inst);
        if (got != 1 && got != 2) {
          clk.charge(kActAcquire);
          break;
        }
        holding = true;
        if (got == 1 && tid == 0) ++tally.dequeues;
        clk.charge(kActAcquire);
        if (inst < 0 || inst >= p.num_inst) {  // cannot happen: every stored node names its instance
          if (tid == 0) {
            atomicMax(ctr_i32(p, kError), 2);
            store_relaxed(ctr_i32(p, kAbort), 1);
          }
          break;
        }
        // a root's input check is loaded now, while the instance is being staged
        const int32_t err_row = got == 2 ? load_relaxed(&p.ist[inst].err_row) : kNoRow;
        if (inst != cur) {
          if (tid == 0) {
            if (cur >= 0) bits_report_nodes(p, cur, unreported);
            tally.nodes += unreported;
            tally.pushes += pushes32;
            tally.pops += pops32;
            ++tally.instances;
          }
          unreported = pushes32 = pops32 = 0;
          cur_n = load_adjacency<W>(p, inst, adj_lds, r);
          const Instance in = p.inst[inst];
          cur = inst;
          cur_k = min(in.k, cur_n);  // a k beyond n acts as n (see reduce_bits)
          cur_vtx = in.vtx_off;
        }
        if (got == 2) {
          const int rejected = __builtin_amdgcn_readfirstlane(err_row != kNoRow);
          if (rejected) {  // rejected input: no search (PVC: the instance is settled)
            if (PVC && tid == 0) fetch_add(ctr_i32(p, kOpen), -1);
            continue;
          }
          root_bits<W>(L, cur_n);
          pending = -1;
        }
        clk.charge(kActOther);
      }
      enter_node<W>(r, L, D, pending, adj_lds);
      clk.charge(kActBranch);
      have = true;
    }

    // Node header, read every kPollNodes nodes (and at the first node after a switch of
    // instance): the instance's flags and current best (one load), the worklist count for the
    // donation test, and the launch-wide stop. These are agent-scope loads of lines every
    // workgroup reads, so they are kept off most nodes: a stale best is only a weaker bound
    // (MVC), a stale count only a stale filter (the reservation re-reads it), and a workgroup
    // that answers its instance or exhausts its budget knows it at once (inst_done). The loads
    // are issued here and waited for after the reduction, which runs meanwhile with the bound
    // known before them: k (PVC), or the best this workgroup saw last, lowered by the covers it
    // found since (MVC); it then continues under the fresh best. With one workgroup the two
    // bounds always agree.
    const bool poll = (headers++ & (kPollNodes - 1)) == 0 || seen_inst != cur;
    uint64_t hraw = 0;
    int32_t qraw = 0, abort_raw = 0, open_raw = 1;
    if (poll) {
      hraw = inst_header(p, cur);
      if (p.q_threshold > 0) qraw = load_relaxed(ctr_i32(p, kQCount));
      abort_raw = load_relaxed(ctr_i32(p, kAbort));
      if (PVC) open_raw = load_relaxed(ctr_i32(p, kOpen));
      if (tid == 0 && watchdog(p, c)) abort_raw = 1;
    }
    if (seen_inst != cur) {
      // a new instance: wait for its header before the reduction
      seen_best = static_cast<int32_t>(static_cast<uint32_t>(uniform64(hraw)));
      seen_inst = cur;
      inst_done = false;
    }
    const int32_t early = PVC ? cur_k : seen_best - 1;
    reduce_bits<W>(r, L, D, adj_lds, early, p.rules);

    if (poll) {
      const uint64_t h = uniform64(hraw);
      const int32_t state = static_cast<int32_t>(h >> 32);
      if ((state & kInstOutOfBudget) || (PVC && (state & kInstFound))) inst_done = true;
      if (!PVC) seen_best = min(seen_best, static_cast<int32_t>(static_cast<uint32_t>(h)));
      seen_count = __builtin_amdgcn_readfirstlane(qraw);
      stop = __builtin_amdgcn_readfirstlane((abort_raw != 0 || open_raw == 0) ? 1 : 0);
    }
    clk.charge(kActReduce);
    if (stop) break;
    if (inst_done) {  // answered or out of budget: drop this node and the rest of the sub-tree
      have = false;
      top = bot;
      top_slot = bot_slot;
      continue;
    }

    if (++unreported >= flush_at) {
      int spent = 0;
      if (tid == 0) {
        if (p.node_budget > 0) spent = bits_report_nodes(p, cur, unreported);
        tally.nodes += unreported;
        tally.pushes += pushes32;
        tally.pops += pops32;
      }
      unreported = pushes32 = pops32 = 0;
      if (__builtin_amdgcn_readfirstlane(spent)) inst_done = true;
    }

    const int32_t bound = PVC ? cur_k : seen_best - 1;
    if (!PVC && bound < early) {
      reduce_bits<W>(r, L, D, adj_lds, bound, p.rules);
      clk.charge(kActReduce);
    }

    const int32_t rr = bound - L.s;
    if (rr < 0) {
      have = false;
      continue;
    }
    int vmax;
    int32_t degsum;
    bits_max_degree<W>(L, D, vmax, degsum);
    clk.charge(kActBranch);
    // (rr >= n - |S| leaves no room for the prune: |E| < (n - |S|)^2 / 2)
    const int32_t edges = degsum / 2;
    if ((p.rules & kPruneEdges) && (p.rules & kRuleHigh) && rr < cur_n && edges > rr * rr) {
      have = false;
      continue;
    }
    if (edges == 0) {  // a vertex cover of size |S|
      if (!PVC && L.s < seen_best) seen_best = L.s;
      int won = 0;
      if (tid == 0) won = bits_claim<PVC>(p, cur, L.s);
      if (__builtin_amdgcn_readfirstlane(won)) {
        write_cover<W>(p.covers + cur_vtx, L, cur_n);
        __threadfence();
        if (tid == 0) bits_publish<PVC>(p, cur, L.s);
      }
      // PVC: a cover of size <= k is recorded now, by this workgroup or another one
      if (PVC) inst_done = true;
      clk.charge(kActOther);
      have = false;
      continue;
    }

    // branch on v_max: defer the N(v_max) child, continue with the v_max child. While the
    // worklist is below its threshold a deferred child is donated: the oldest one on this
    // workgroup's stack if there is one (the largest sub-tree it holds), else this one.
    bool kept_local = true;
    if (p.q_threshold > 0 && seen_count < static_cast<int32_t>(p.q_threshold)) {
      const bool from_stack = top > bot;
      const int32_t* oldest =
          !from_stack ? nullptr
          : stack_lds ? lstack + bot_slot * kStride
                      : gstack + static_cast<size_t>(bot_slot) * kStride;
      if (bits_enqueue<W>(p, c, L, vmax, oldest, cur)) {
        if (tid == 0) ++tally.enqueues;
        if (from_stack) {
          ++bot;
          bot_slot = bot_slot + 1 == cap ? 0 : bot_slot + 1;
        }
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
      if (stack_lds) bits_store<W>(lstack + top_slot * kStride, L, vmax, cur);
      else bits_store<W>(gstack + static_cast<size_t>(top_slot) * kStride, L, vmax, cur);
      ++top;
      top_slot = top_slot + 1 == cap ? 0 : top_slot + 1;
      ++pushes32;
      if (top - bot > max_depth) max_depth = top - bot;
    }
    clk.charge(kActDonate);
    remove_vertex_bits<W>(r, L, D, vmax);
    clk.charge(kActBranch);
  }
  clk.end();

  if (tid == 0) {
    if (cur >= 0) bits_report_nodes(p, cur, unreported);
    WgStats w = tally;
    w.nodes += unreported;
    w.pushes += pushes32;
    w.pops += pops32;
    w.max_depth = max_depth;
    for (int a = 0; a < kNumActivities; ++a) w.cycles[a] = static_cast<int64_t>(clk.cycles[a]);
    publish_wg_stats(p, wg, w);
  }
}

// The reduction rules of one node on a degree array in device memory (-1 = in the cover),
// instance 0 of the launch.
template <int W>
__global__ void __launch_bounds__(64) bitset_reduce_kernel(Params p, int32_t* deg, int32_t* s,
                                                           int64_t bound) {
  extern __shared__ uint64_t adj_lds[];
  if (__builtin_amdgcn_readfirstlane(load_relaxed(&p.ist[0].err_row)) != kNoRow) return;
  Rows<W> r;
  const int n = load_adjacency<W>(p, 0, adj_lds, r);
  Live<W> L;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    const int v = w * 64 + lane_id();
    L.bits[w] = ballot(v < n && deg[v] >= 0);
  }
  L.s = __builtin_amdgcn_readfirstlane(*s);
  Degrees<W> D;
  enter_node<W>(r, L, D, -1, adj_lds);
  // a bound beyond n removes and prunes exactly as n does (see reduce_bits)
  const int32_t b32 = bound < -1 ? -1 : (bound > n ? n : static_cast<int32_t>(bound));
  reduce_bits<W>(r, L, D, adj_lds, b32, p.rules);
#pragma unroll
  for (int w = 0; w < W; ++w) {
    const int v = w * 64 + lane_id();
    if (v < n) deg[v] = held_live(L, w) ? D.deg[w] : -1;
  }
  if (threadIdx.x == 0) *s = L.s;
}

// ---- launchers ---------------------------------------------------------------------------------

template <int W, bool SO>
static const void* bitset_traverse_fn(bool pvc, bool prof) {
  if (pvc) return prof ? reinterpret_cast<const void*>(&bitset_traverse_kernel<W, true, true, SO>)
                       : reinterpret_cast<const void*>(&bitset_traverse_kernel<W, true, false, SO>);
  return prof ? reinterpret_cast<const void*>(&bitset_traverse_kernel<W, false, true, SO>)
              : reinterpret_cast<const void*>(&bitset_traverse_kernel<W, false, false, SO>);
}

// The StackOnly walk-down is a separate instantiation, so the hybrid kernels carry none of its
// registers.
static const void* bitset_fn(int words, bool pvc, bool prof, bool stack_only = false) {
#define VC_BITSET_CASE(WW) \
  case WW: return stack_only ? bitset_traverse_fn<WW, true>(pvc, prof) : bitset_traverse_fn<WW, false>(pvc, prof);
  switch (words) {
    VC_BITSET_CASE(1)
    VC_BITSET_CASE(2)
    VC_BITSET_CASE(3)
    VC_BITSET_CASE(4)
    VC_BITSET_CASE(5)
    VC_BITSET_CASE(6)
    VC_BITSET_CASE(7)
    default: return stack_only ? bitset_traverse_fn<8, true>(pvc, prof) : bitset_traverse_fn<8, false>(pvc, prof);
  }
#undef VC_BITSET_CASE
}

size_t bitset_lds_bytes(int n_max, int words) { return static_cast<size_t>(n_max) * words * 8; }

int bitset_stride(int words) { return ((2 * words + 2) + 3) & ~3; }

size_t bitset_traverse_lds_bytes(const Params& p) {
  const size_t stack = p.stack_lds ? static_cast<size_t>(p.depth_cap) * bitset_stride(p.words) * 4 : 0;
  return bitset_lds_bytes(p.n_max, p.words) + stack;
}

hipError_t launch_bitset_greedy(const Params& p, hipStream_t stream) {
  const size_t lds = bitset_lds_bytes(p.n_max, p.words);
  const dim3 grid(p.num_inst < 65535 ? p.num_inst : 65535);
  switch (p.words) {
    case 1: hipLaunchKernelGGL(bitset_greedy_kernel<1>, grid, dim3(64), lds, stream, p); break;
    case 2: hipLaunchKernelGGL(bitset_greedy_kernel<2>, grid, dim3(64), lds, stream, p); break;
    case 3: hipLaunchKernelGGL(bitset_greedy_kernel<3>, grid, dim3(64), lds, stream, p); break;
    case 4: hipLaunchKernelGGL(bitset_greedy_kernel<4>, grid, dim3(64), lds, stream, p); break;
    case 5: hipLaunchKernelGGL(bitset_greedy_kernel<5>, grid, dim3(64), lds, stream, p); break;
    case 6: hipLaunchKernelGGL(bitset_greedy_kernel<6>, grid, dim3(64), lds, stream, p); break;
    case 7: hipLaunchKernelGGL(bitset_greedy_kernel<7>, grid, dim3(64), lds, stream, p); break;
    default: hipLaunchKernelGGL(bitset_greedy_kernel<8>, grid, dim3(64), lds, stream, p); break;
  }
  return hipGetLastError();
}

hipError_t launch_bitset_traverse(bool pvc, bool prof, const Params& p, hipStream_t stream) {
  Params args = p;
  void* kargs[] = {&args};
  // plain launch; see launch_traverse for why co-residency is not required
  return hipLaunchKernel(bitset_fn(p.words, pvc, prof, p.start_depth > 0), dim3(p.num_wg),
                         dim3(64), kargs, bitset_traverse_lds_bytes(p), stream);
}

hipError_t launch_bitset_reduce(const Params& p, int32_t* deg, int32_t* s, int64_t bound,
                                hipStream_t stream) {
  const size_t lds = bitset_lds_bytes(p.n_max, p.words);
  switch (p.words) {
    case 1: hipLaunchKernelGGL(bitset_reduce_kernel<1>, dim3(1), dim3(64), lds, stream, p, deg, s, bound); break;
    case 2: hipLaunchKernelGGL(bitset_reduce_kernel<2>, dim3(1), dim3(64), lds, stream, p, deg, s, bound); break;
    case 3: hipLaunchKernelGGL(bitset_reduce_kernel<3>, dim3(1), dim3(64), lds, stream, p, deg, s, bound); break;
    case 4: hipLaunchKernelGGL(bitset_reduce_kernel<4>, dim3(1), dim3(64), lds, stream, p, deg, s, bound); break;
    case 5: hipLaunchKernelGGL(bitset_reduce_kernel<5>, dim3(1), dim3(64), lds, stream, p, deg, s, bound); break;
    case 6: hipLaunchKernelGGL(bitset_reduce_kernel<6>, dim3(1), dim3(64), lds, stream, p, deg, s, bound); break;
    case 7: hipLaunchKernelGGL(bitset_reduce_kernel<7>, dim3(1), dim3(64), lds, stream, p, deg, s, bound); break;
    default: hipLaunchKernelGGL(bitset_reduce_kernel<8>, dim3(1), dim3(64), lds, stream, p, deg, s, bound); break;
  }
  return hipGetLastError();
}

hipError_t bitset_occupancy(int words, bool pvc, bool prof, size_t lds, int* blocks_per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, bitset_fn(words, pvc, prof),
                                                      64, lds);
}

}  // namespace vc
