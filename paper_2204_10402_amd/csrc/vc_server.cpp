// vc_server.cpp -- continuous batching of a request stream (the vc_server_* calls of
// include/vc.h).
//
// A server owns W worker threads, each with its own library context (device workspace and HIP
// stream). Requests are queued on submission with a copy of their graph. A free worker takes
// the oldest waiting request's problem kind (MVC or PVC) and, in arrival order, every waiting
// request of that kind that fits the memory budget (up to max_batch), and solves them as one
// batch (vc_mvc_batch / vc_pvc_batch: one persistent launch per kernel family) with a grid of
// wg_per_request workgroups per request, at most 1/W of the co-resident grid. While it runs,
// other workers admit the requests that arrive meanwhile, so batches overlap on the device. The budget counts the node stacks a batch
// provisions (workgroups x depth bound x node bytes); a request that alone exceeds it runs
// when nothing else is in flight. Each result carries the submission, start and completion
// times on the server's clock.

#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "vc.h"
#include "vc_internal.h"

namespace {

struct Request {
  int64_t ticket = 0;
  int32_t problem = 0;  // VC_PROBLEM_MVC or VC_PROBLEM_PVC
  int32_t k = 0;
  int32_t n = 0;
  std::vector<int32_t> rp, ci;
  uint8_t* cover_out = nullptr;
  double submit_ms = 0.0;
  int64_t footprint = 0;
};

// Bytes of node stacks a request adds to a batch: its workgroups (at most one per CU's worth,
// 256, since a batch's grid is capped by its share of the device) times the depth bound times
// the stored node size of its kernel family.
int64_t footprint(int32_t n, int32_t problem, int32_t k, int32_t wg_per_request) {
  const int64_t depth = problem == VC_PROBLEM_PVC ? std::min<int64_t>(k, n) + 1 : n;
  const int64_t node = n <= vc::kAutoBitsetN ? vc::bitset_stride((std::max(n, 1) + 63) / 64) * 4
                                            : static_cast<int64_t>(vc::array_stride(n)) * 4;
  return std::min<int64_t>(wg_per_request, 256) * depth * node;
}

}  // namespace

struct vc_server {
  int device = 0;
  vc_server_options so{};
  vc_options opts{};
  std::chrono::steady_clock::time_point t0;
  std::mutex mu;
  std::condition_variable work_cv;  // workers: a request arrived or memory was freed
  std::condition_variable done_cv;  // pollers: a result is ready
  std::deque<Request*> pending;
  std::deque<vc_served> done;
  int64_t in_flight_bytes = 0;
  int32_t running = 0;
  int64_t next_ticket = 1;
  bool stop = false;
  std::vector<vc_ctx*> ctxs;
  std::vector<std::thread> workers;

  double now_ms() const {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }

  // Under `mu`: can a worker start a batch now?
  bool admissible() const {
    if (pending.empty()) return false;
    return in_flight_bytes == 0 || in_flight_bytes + pending.front()->footprint <= so.memory_budget;
  }

  void worker_main(int w);
};

void vc_server::worker_main(int w) {
  (void)hipSetDevice(device);
  vc_ctx* ctx = ctxs[w];
  std::vector<Request*> take;
  std::vector<int32_t> n, nnz, k, status, size, yes, rp, ci;
  std::vector<int64_t> nodes;
  std::vector<uint8_t> cover;
  for (;;) {
    int32_t problem = 0;
    int64_t bytes = 0;
    {
      std::unique_lock<std::mutex> lk(mu);
      work_cv.wait(lk, [&] { return stop || admissible(); });
      if (stop) return;
      problem = pending.front()->problem;
      for (auto it = pending.begin(); it != pending.end() &&
                                      static_cast<int32_t>(take.size()) < so.max_batch;) {
        Request* r = *it;
        if (r->problem != problem) {
          ++it;
          continue;
        }
        if (!take.empty() && in_flight_bytes + bytes + r->footprint > so.memory_budget) break;
        bytes += r->footprint;
        take.push_back(r);
        it = pending.erase(it);
      }
      in_flight_bytes += bytes;
      running += static_cast<int32_t>(take.size());
    }
    const double start_ms = now_ms();
    const int32_t count = static_cast<int32_t>(take.size());
    n.resize(count);
    nnz.resize(count);
    k.resize(count);
    rp.clear();
    ci.clear();
    int64_t total_n = 0;
    for (int32_t i = 0; i < count; ++i) {
      const Request* r = take[i];
      n[i] = r->n;
      nnz[i] = static_cast<int32_t>(r->ci.size());
      k[i] = r->k;
      rp.insert(rp.end(), r->rp.begin(), r->rp.end());
      ci.insert(ci.end(), r->ci.begin(), r->ci.end());
      total_n += r->n;
    }
    status.assign(count, VC_ERR_INTERNAL);
    size.assign(count, -1);
    yes.assign(count, 0);
    nodes.assign(count, 0);
    cover.assign(static_cast<size_t>(std::max<int64_t>(total_n, 1)), 0);
    vc_batch b{count, n.data(), nnz.data(), rp.data(), ci.empty() ? nullptr : ci.data()};
    vc_options o = opts;
    o.num_wg = static_cast<int32_t>(
        std::max<int64_t>(1, std::min<int64_t>(1 << 20, int64_t{so.wg_per_request} * count)));
    o.grid_share = so.workers;  // side by side with the other workers' batches
    int rc = problem == VC_PROBLEM_PVC
                 ? vc_pvc_batch(ctx, &b, k.data(), &o, status.data(), yes.data(), size.data(),
                                cover.data(), nodes.data(), nullptr)
                 : vc_mvc_batch(ctx, &b, &o, status.data(), size.data(), cover.data(),
                                nodes.data(), nullptr);
    const double done_ms = now_ms();
    {
      std::lock_guard<std::mutex> lk(mu);
      int64_t off = 0;
      for (int32_t i = 0; i < count; ++i) {
        Request* r = take[i];
        vc_served s{};
        s.ticket = r->ticket;
        s.status = rc == VC_OK ? status[i] : rc;
        s.size = rc == VC_OK ? size[i] : -1;
        s.yes = rc == VC_OK ? (problem == VC_PROBLEM_PVC ? yes[i] : (status[i] == VC_OK)) : 0;
        s.batch_size = count;
        s.worker = w;
        s.nodes = rc == VC_OK ? nodes[i] : 0;
        s.submit_ms = r->submit_ms;
        s.start_ms = start_ms;
        s.done_ms = done_ms;
        if (r->cover_out && r->n > 0 && rc == VC_OK)
          std::memcpy(r->cover_out, cover.data() + off, static_cast<size_t>(r->n));
        off += r->n;
        done.push_back(s);
        delete r;
      }
      in_flight_bytes -= bytes;
      running -= count;
    }
    take.clear();
    done_cv.notify_all();
    work_cv.notify_all();
  }
}

extern "C" {

int vc_server_create(vc_server** out, int device, const vc_server_options* sopts,
                     const vc_options* opts) {
  if (!out) return VC_ERR_INVALID_ARG;
  *out = nullptr;
  vc_server_options so = sopts ? *sopts : vc_server_options{};
  for (int32_t r : so.reserved)
    if (r != 0) return VC_ERR_INVALID_ARG;
  if (so.workers < 0 || so.max_batch < 0 || so.memory_budget < 0 || so.wg_per_request < 0)
    return VC_ERR_INVALID_ARG;
  if (so.workers == 0) so.workers = 4;
  if (so.max_batch == 0) so.max_batch = 32;
  if (so.wg_per_request == 0) so.wg_per_request = 256;
  if (so.workers > 64) return VC_ERR_INVALID_ARG;
  if (opts && (opts->num_wg || opts->grid_share || (opts->flags & VC_OPT_AUTOTUNE)))
    return VC_ERR_INVALID_ARG;
  if (so.memory_budget == 0) {
    size_t free_b = 0, total_b = 0;
    if (hipSetDevice(device) != hipSuccess || hipMemGetInfo(&free_b, &total_b) != hipSuccess)
      return VC_ERR_DEVICE;
    so.memory_budget = static_cast<int64_t>(free_b / 4);
  }
  vc_server* s = new vc_server();
  s->device = device;
  s->so = so;
  if (opts) s->opts = *opts;
  s->t0 = std::chrono::steady_clock::now();
  for (int32_t w = 0; w < so.workers; ++w) {
    vc_ctx* c = nullptr;
    const int rc = vc_create(&c, device, nullptr);
    if (rc != VC_OK) {
      for (vc_ctx* x : s->ctxs) vc_destroy(x);
      delete s;
      return rc;
    }
    s->ctxs.push_back(c);
  }
  for (int32_t w = 0; w < so.workers; ++w) s->workers.emplace_back(&vc_server::worker_main, s, w);
  *out = s;
  return VC_OK;
}

int vc_server_submit(vc_server* s, const vc_graph* g, int32_t problem, int32_t k,
                     uint8_t* cover_out, int64_t* ticket_out) {
  if (!s || !g || !ticket_out) return VC_ERR_INVALID_ARG;
  if (problem != VC_PROBLEM_MVC && problem != VC_PROBLEM_PVC) return VC_ERR_INVALID_ARG;
  if (problem == VC_PROBLEM_PVC && k < 0) return VC_ERR_INVALID_ARG;
  if (g->n < 0 || g->nnz < 0 || !g->row_ptr || (g->nnz > 0 && !g->col_idx))
    return VC_ERR_INVALID_ARG;
  Request* r = new Request();
  r->problem = problem;
  r->k = problem == VC_PROBLEM_PVC ? k : 0;
  r->n = g->n;
  r->rp.assign(g->row_ptr, g->row_ptr + g->n + 1);
  if (g->nnz > 0) r->ci.assign(g->col_idx, g->col_idx + g->nnz);
  r->cover_out = cover_out;
  r->footprint = footprint(g->n, problem, r->k, s->so.wg_per_request);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) {
      delete r;
      return VC_ERR_INVALID_ARG;
    }
    r->ticket = s->next_ticket++;
    r->submit_ms = s->now_ms();
    *ticket_out = r->ticket;
    s->pending.push_back(r);
  }
  s->work_cv.notify_one();
  return VC_OK;
}

int vc_server_poll(vc_server* s, vc_served* out, int32_t max, int32_t timeout_ms,
                   int32_t* count_out) {
  if (!s || !count_out || (max > 0 && !out) || max < 0) return VC_ERR_INVALID_ARG;
  std::unique_lock<std::mutex> lk(s->mu);
  if (timeout_ms > 0 && s->done.empty())
    s->done_cv.wait_for(lk, std::chrono::milliseconds(timeout_ms),
                        [&] { return !s->done.empty(); });
  int32_t c = 0;
  while (c < max && !s->done.empty()) {
    out[c++] = s->done.front();
    s->done.pop_front();
  }
  *count_out = c;
  return VC_OK;
}

int vc_server_pending(vc_server* s, int32_t* queued, int32_t* running) {
  if (!s) return VC_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  if (queued) *queued = static_cast<int32_t>(s->pending.size());
  if (running) *running = s->running;
  return VC_OK;
}

int vc_server_destroy(vc_server* s) {
  if (!s) return VC_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->work_cv.notify_all();
  for (std::thread& t : s->workers) t.join();
  for (Request* r : s->pending) delete r;
  for (vc_ctx* c : s->ctxs) vc_destroy(c);
  delete s;
  return VC_OK;
}

}  // extern "C"
