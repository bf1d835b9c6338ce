// worklist_model.cpp -- a CPU model of the traversal's worklist and termination protocol
// (paper §IV-A, §IV-C), for ThreadSanitizer and random interleavings. Test infrastructure: the
// library does not use it.
//
// Each std::thread plays one workgroup of the persistent launch. The shared state mirrors the
// device's control words and ring, with the same atomic operations and memory orders:
//   count      reservations made by producers and not yet by consumers (relaxed)
//   head/tail  consumer and producer tickets (64-bit, relaxed)
//   seq[slot]  lap ticket of each ring slot: 2*lap free for lap `lap`, 2*lap+1 filled
//              (acquire loads, release stores; the node words themselves are plain)
//   work       sub-trees not finished: unstarted roots, queued nodes, held sub-trees (relaxed)
//   inst_work  the same per instance; root_next hands out unstarted instances.
// A thread walks a sub-tree with its own bounded stack ring; at every branching it donates a
// deferred child while `count` is below the threshold -- the oldest entry of its stack if it has
// one, else the new child -- and otherwise keeps it. It releases the sub-tree it took (root or
// queued node) only when its stack is empty, and ends when nothing is queued, unstarted or held.
//
// The trees are seeded and imbalanced (a node has two children, one or none with depth-dependent
// odds). Checked after every thread has ended: every node of every tree visited exactly once (no
// node lost, none taken twice), every counter back at zero, every slot free for its next lap.
// A thread that would overflow its stack ring aborts the run (the depth bound is sized so that
// it never happens). Random pauses between protocol steps widen the interleavings.
//
//   worklist_model THREADS CAP THRESHOLD INSTANCES MAX_DEPTH SEED
// exits 0 when every check holds, 1 with a message otherwise.
//
// Built with -DVC_MODEL_MUTATION=1 a producer does not raise the outstanding-work counters for a
// donated node, and with -DVC_MODEL_MUTATION=2 it publishes a slot with a relaxed store: the
// tests check that the counter checks, and ThreadSanitizer, notice.

#include <atomic>
#include <chrono>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <thread>
#include <vector>

#ifndef VC_MODEL_MUTATION
#define VC_MODEL_MUTATION 0
#endif

namespace {

struct Tree {
  std::vector<int32_t> left, right;  // child indices, -1 if none
  int32_t size() const { return static_cast<int32_t>(left.size()); }
};

// Node 0 is the root; depth-first construction with a seeded generator.
Tree make_tree(uint64_t seed, int max_depth) {
  Tree t;
  std::mt19937_64 rng(seed);
  struct Item { int32_t node; int depth; };
  std::vector<Item> todo{{0, 0}};
  t.left.push_back(-1);
  t.right.push_back(-1);
  while (!todo.empty()) {
    const Item it = todo.back();
    todo.pop_back();
    if (it.depth >= max_depth) continue;
    const double u = std::uniform_real_distribution<double>(0.0, 1.0)(rng);
    const int kids = u < 0.62 ? 2 : (u < 0.85 ? 1 : 0);
    for (int c = 0; c < kids; ++c) {
      const int32_t id = t.size();
      t.left.push_back(-1);
      t.right.push_back(-1);
      (c == 0 ? t.left : t.right)[it.node] = id;
      todo.push_back({id, it.depth + 1});
    }
  }
  return t;
}

struct Shared {
  uint32_t cap = 0, threshold = 0;
  int32_t num_inst = 0;
  std::vector<Tree> trees;
  std::vector<std::vector<std::atomic<uint8_t>>*> visited;
  std::atomic<int32_t> count{0};
  std::atomic<uint64_t> head{0}, tail{0};
  std::atomic<int32_t> work{0}, root_next{0};
  std::vector<std::atomic<int32_t>> inst_work;
  std::vector<std::atomic<uint32_t>> seq;
  std::vector<int32_t> payload;  // two words per slot: instance, node (plain memory)
  std::atomic<int64_t> visits{0};
  std::atomic<int> failed{0};
  explicit Shared(size_t n_inst, size_t cap_) : inst_work(n_inst), seq(cap_), payload(2 * cap_) {}
};

void fail(Shared& s, const char* what) {
  if (s.failed.exchange(1) == 0) std::fprintf(stderr, "worklist model: %s\n", what);
}

// A random pause between protocol steps: nothing, a yield, or a few microseconds.
struct Jitter {
  std::mt19937 rng;
  explicit Jitter(uint32_t seed) : rng(seed) {}
  void operator()() {
    const uint32_t r = rng() % 64;
    if (r == 0) std::this_thread::sleep_for(std::chrono::microseconds(1 + rng() % 20));
    else if (r < 8) std::this_thread::yield();
  }
};

struct Node { int32_t inst, node; };

// Producer: reserve a slot (the device's enqueue_reserve), write the node, publish it.
bool try_enqueue(Shared& s, Jitter& j, Node n) {
  if (s.count.load(std::memory_order_relaxed) >= static_cast<int32_t>(s.threshold)) return false;
#if VC_MODEL_MUTATION != 1
  s.inst_work[n.inst].fetch_add(1, std::memory_order_relaxed);
  s.work.fetch_add(1, std::memory_order_relaxed);
#endif
  j();
  s.count.fetch_add(1, std::memory_order_relaxed);
  const uint64_t t = s.tail.fetch_add(1, std::memory_order_relaxed);
  const uint32_t slot = static_cast<uint32_t>(t) & (s.cap - 1);
  const uint32_t lap = static_cast<uint32_t>(t / s.cap);
  while (s.seq[slot].load(std::memory_order_acquire) != 2u * lap) std::this_thread::yield();
  j();
  s.payload[2 * slot] = n.inst;
  s.payload[2 * slot + 1] = n.node;
#if VC_MODEL_MUTATION == 2
  s.seq[slot].store(2u * lap + 1u, std::memory_order_relaxed);
#else
  s.seq[slot].store(2u * lap + 1u, std::memory_order_release);
#endif
  return true;
}

// Consumer (the device's worklist_take / dequeue_begin / dequeue_finish): 1 with a queued node,
// 2 with a root, 0 when the launch is over. As on the device, the entry count, the root
// counter and the outstanding-work counter are read in that order, each only when the ones
// before it offered nothing, and only an atomic claims anything.
int dequeue(Shared& s, Jitter& j, Node* out) {
  for (;;) {
    if (s.failed.load(std::memory_order_relaxed)) return 0;
    if (s.count.load(std::memory_order_relaxed) > 0) {
      if (s.count.fetch_add(-1, std::memory_order_relaxed) > 0) {
        const uint64_t h = s.head.fetch_add(1, std::memory_order_relaxed);
        const uint32_t slot = static_cast<uint32_t>(h) & (s.cap - 1);
        const uint32_t lap = static_cast<uint32_t>(h / s.cap);
        while (s.seq[slot].load(std::memory_order_acquire) != 2u * lap + 1u)
          std::this_thread::yield();
        out->inst = s.payload[2 * slot];
        out->node = s.payload[2 * slot + 1];
        j();
        s.seq[slot].store(2u * (lap + 1u), std::memory_order_release);
        return 1;
      }
      s.count.fetch_add(1, std::memory_order_relaxed);  // lost the race: give it back
    } else if (s.root_next.load(std::memory_order_relaxed) < s.num_inst) {
      const int32_t r = s.root_next.fetch_add(1, std::memory_order_relaxed);
      if (r < s.num_inst) {
        out->inst = r;
        out->node = 0;
        return 2;
      }
    } else if (s.work.load(std::memory_order_relaxed) == 0) {
      return 0;
    }
    j();
    std::this_thread::yield();
  }
}

// The sub-tree taken as a root or from the worklist is finished. Every release matches an
// earlier raise, so neither counter may drop below zero (checked here, not on the device).
void release(Shared& s, int32_t inst) {
  if (s.inst_work[inst].fetch_add(-1, std::memory_order_relaxed) <= 0)
    fail(s, "an instance's outstanding-work counter went below zero");
  if (s.work.fetch_add(-1, std::memory_order_relaxed) <= 0)
    fail(s, "the outstanding-work counter went below zero");
}

void workgroup(Shared& s, uint32_t seed, int depth_cap) {
  Jitter j(seed);
  std::vector<Node> ring(static_cast<size_t>(depth_cap));
  int top = 0, bot = 0;  // the stack ring holds [bot, top); pops at top, donations from bot
  bool have = false, holding = false;
  Node cur{};
  for (;;) {
    if (!have) {
      if (top > bot) {
        --top;
        cur = ring[top % depth_cap];
      } else {
        if (holding) {
          release(s, cur.inst);
          holding = false;
        }
        const int got = dequeue(s, j, &cur);
        if (got == 0) return;
        holding = true;
      }
      have = true;
    }
    // visit
    std::atomic<uint8_t>& v = (*s.visited[cur.inst])[cur.node];
    if (v.exchange(1, std::memory_order_relaxed) != 0) fail(s, "a node was visited twice");
    s.visits.fetch_add(1, std::memory_order_relaxed);
    const Tree& t = s.trees[cur.inst];
    const int32_t a = t.left[cur.node], b = t.right[cur.node];
    if (a < 0 && b < 0) {
      have = false;
      continue;
    }
    if (a >= 0 && b >= 0) {
      // defer b: donate the oldest stack entry if any, else b, while the worklist is short
      bool kept = true;
      const bool from_stack = top > bot;
      const Node donate = from_stack ? ring[bot % depth_cap] : Node{cur.inst, b};
      if (try_enqueue(s, j, donate)) {
        if (from_stack) ++bot;
        else kept = false;
      }
      if (kept) {
        if (top - bot >= depth_cap) {
          fail(s, "stack ring overflow");
          return;
        }
        ring[top % depth_cap] = Node{cur.inst, b};
        ++top;
      }
      cur.node = a;
    } else {
      cur.node = a >= 0 ? a : b;
    }
    j();
  }
}

}  // namespace

int main(int argc, char** argv) {
  if (argc != 7) {
    std::fprintf(stderr, "usage: %s THREADS CAP THRESHOLD INSTANCES MAX_DEPTH SEED\n", argv[0]);
    return 2;
  }
  const int threads = std::atoi(argv[1]);
  const uint32_t cap = static_cast<uint32_t>(std::atoi(argv[2]));
  const uint32_t threshold = static_cast<uint32_t>(std::atoi(argv[3]));
  const int insts = std::atoi(argv[4]);
  const int max_depth = std::atoi(argv[5]);
  const uint64_t seed = std::strtoull(argv[6], nullptr, 10);
  // the ring must hold every reservation: threshold + 2 * threads <= cap (as on the device)
  if (threads < 1 || cap == 0 || (cap & (cap - 1)) || threshold + 2u * threads > cap) {
    std::fprintf(stderr, "bad sizes: cap must be a power of two >= threshold + 2 * threads\n");
    return 2;
  }
  Shared s(static_cast<size_t>(insts), cap);
  s.cap = cap;
  s.threshold = threshold;
  s.num_inst = insts;
  int64_t total = 0;
  for (int i = 0; i < insts; ++i) {
    s.trees.push_back(make_tree(seed * 1000 + static_cast<uint64_t>(i), max_depth));
    total += s.trees.back().size();
  }
  std::vector<std::vector<std::atomic<uint8_t>>> visited(static_cast<size_t>(insts));
  for (int i = 0; i < insts; ++i) {
    visited[static_cast<size_t>(i)] =
        std::vector<std::atomic<uint8_t>>(static_cast<size_t>(s.trees[static_cast<size_t>(i)].size()));
    s.visited.push_back(&visited[static_cast<size_t>(i)]);
  }
  for (auto& w : s.inst_work) w.store(1);  // one root each
  s.work.store(insts);
  for (auto& q : s.seq) q.store(0);
  std::vector<std::thread> pool;
  for (int w = 0; w < threads; ++w)
    pool.emplace_back(workgroup, std::ref(s), static_cast<uint32_t>(seed * 7919 + w),
                      max_depth + 2);
  for (auto& th : pool) th.join();
  if (s.failed.load()) return 1;
  int64_t seen = 0;
  for (auto& vv : visited)
    for (auto& x : vv) seen += x.load();
  if (seen != total || s.visits.load() != total) {
    std::fprintf(stderr, "worklist model: %lld of %lld nodes visited (%lld visits)\n",
                 static_cast<long long>(seen), static_cast<long long>(total),
                 static_cast<long long>(s.visits.load()));
    return 1;
  }
  if (s.work.load() != 0 || s.count.load() != 0 || s.head.load() != s.tail.load()) {
    std::fprintf(stderr, "worklist model: counters not back at zero\n");
    return 1;
  }
  for (int i = 0; i < insts; ++i)
    if (s.inst_work[static_cast<size_t>(i)].load() != 0) {
      std::fprintf(stderr, "worklist model: instance %d not finished\n", i);
      return 1;
    }
  const uint64_t laps_done = s.tail.load();
  for (uint32_t slot = 0; slot < cap; ++slot) {
    const uint64_t used = laps_done / cap + (slot < laps_done % cap ? 1 : 0);
    if (s.seq[slot].load() != 2u * static_cast<uint32_t>(used)) {
      std::fprintf(stderr, "worklist model: slot %u not free for its next lap\n", slot);
      return 1;
    }
  }
  std::printf("ok %lld nodes, %llu enqueued, %d threads\n", static_cast<long long>(total),
              static_cast<unsigned long long>(laps_done), threads);
  return 0;
}
