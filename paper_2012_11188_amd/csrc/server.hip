// Query server with continuous batching over one resident index.
//
// Device memory is split into batch buffers, each with a fixed set of query
// slots (union-find parents, border flags, a device result array and a pinned
// host result array per slot), its own stream and event. A launcher thread
// takes queued requests whenever a batch buffer is free and submits up to
// max_batch of them as one batch: the four query kernels run once for all of
// them (unused entries are inactive descriptors) and every result is copied to
// its slot's pinned array. With use_graph the whole batch (descriptor upload,
// kernels, result copies) is a HIP graph captured once per buffer and
// replayed. A completer thread waits for batches in submission order, copies
// each result to the caller's destination (results for pinned host memory
// are copied there by the device directly; device destinations are written
// by the kernels) and frees the buffer. Requests that
// arrive while batches run are queued and admitted as buffers free up, so
// several batches overlap on the device.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "index.h"

using namespace scan;

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
  uint64_t ticket;
  int32_t mu;
  double eps;
  int32_t *dst;
  bool dst_on_device;
  bool dst_pinned;  // host memory the device can write directly
  double *latency_ms;
  Clock::time_point t_submit;
};

struct BatchBuf {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  std::vector<QuerySlot> slots;     // max_batch workspaces
  std::vector<int32_t *> d_memb;    // device results
  std::vector<int32_t *> h_memb;    // pinned host results
  QueryDesc *h_desc = nullptr;      // pinned, max_batch entries
  QueryDesc *d_desc = nullptr;      // device, max_batch entries
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<Request> reqs;        // requests of the batch in flight
};

}  // namespace

struct scan_server {
  const scan_index *ix = nullptr;
  scan_server_opts opts{};
  int32_t nbuf = 0;
  std::vector<BatchBuf> bufs;
  std::deque<int32_t> free_bufs;
  std::deque<Request> pending;
  size_t pending_cap = 0;
  std::deque<int32_t> inflight;  // buffers in submission order
  std::unordered_map<uint64_t, int> state;  // 0 queued, 1 running, 2 done
  uint64_t next_ticket = 1;
  std::mutex mu;
  std::condition_variable cv_launch, cv_complete, cv_done;
  bool stop = false;
  bool launcher_done = false;
  std::thread launcher, completer;
  scan_status error = SCAN_OK;
};

namespace {

void free_server_resources(scan_server *s) {
  for (auto &b : s->bufs) {
    if (b.exec) (void)hipGraphExecDestroy(b.exec);
    if (b.graph) (void)hipGraphDestroy(b.graph);
    for (auto &sl : b.slots) free_query_slot(&sl, b.stream);
    for (auto *p : b.d_memb)
      if (p) dev_free(p, (size_t)std::max<int64_t>(s->ix->n, 1) * 4, b.stream);
    for (auto *p : b.h_memb)
      if (p) (void)hipHostFree(p);
    if (b.d_desc) dev_free(b.d_desc, sizeof(QueryDesc) * s->opts.max_batch, b.stream);
    if (b.h_desc) (void)hipHostFree(b.h_desc);
    if (b.stream) (void)hipStreamSynchronize(b.stream);
    if (b.done) (void)hipEventDestroy(b.done);
    if (b.stream) (void)hipStreamDestroy(b.stream);
  }
  s->bufs.clear();
}

// The fixed part of a batch: descriptor upload (from b.h_desc) and the query
// kernels over all max_batch entries. Captured once as a graph with use_graph.
hipError_t enqueue_batch_kernels(scan_server *s, BatchBuf &b) {
  hipError_t e = hipMemcpyAsync(b.d_desc, b.h_desc, sizeof(QueryDesc) * s->opts.max_batch,
                                hipMemcpyHostToDevice, b.stream);
  if (e != hipSuccess) return e;
  launch_query_kernels(s->ix, b.d_desc, s->opts.max_batch, b.stream);
  return hipGetLastError();
}

void launcher_loop(scan_server *s) {
  (void)hipSetDevice(s->ix->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    // On shutdown the queue is drained first: requests still pending wait for
    // a buffer like any other.
    s->cv_launch.wait(lk, [&] {
      return (s->stop && s->pending.empty()) || (!s->pending.empty() && !s->free_bufs.empty());
    });
    if (s->pending.empty()) break;
    const int32_t bi = s->free_bufs.front();
    s->free_bufs.pop_front();
    BatchBuf &b = s->bufs[bi];
    b.reqs.clear();
    while (!s->pending.empty() && (int32_t)b.reqs.size() < s->opts.max_batch) {
      b.reqs.push_back(s->pending.front());
      s->pending.pop_front();
      s->state[b.reqs.back().ticket] = 1;
    }
    const int32_t count = (int32_t)b.reqs.size();
    lk.unlock();
    // Device destinations are written by the kernels directly; host ones go
    // through the slot's device and pinned arrays.
    for (int32_t i = 0; i < s->opts.max_batch; ++i) {
      if (i < count) {
        const Request &r = b.reqs[i];
        b.h_desc[i] = make_query_desc(r.mu, r.eps, b.slots[i], r.dst_on_device ? r.dst : b.d_memb[i], nullptr);
      } else {
        b.h_desc[i] = make_query_desc(2, 0.0, b.slots[i], nullptr, nullptr);  // inactive
      }
    }
    hipError_t e = b.exec ? hipGraphLaunch(b.exec, b.stream) : enqueue_batch_kernels(s, b);
    const int64_t n = s->ix->n;
    for (int32_t i = 0; i < count && n > 0 && e == hipSuccess; ++i)
      if (!b.reqs[i].dst_on_device)
        e = hipMemcpyAsync(b.reqs[i].dst_pinned ? b.reqs[i].dst : b.h_memb[i], b.d_memb[i], (size_t)n * 4,
                           hipMemcpyDeviceToHost, b.stream);
    if (e == hipSuccess) e = hipEventRecord(b.done, b.stream);
    lk.lock();
    if (e != hipSuccess) s->error = fail(SCAN_EDEVICE, "server batch launch: %s", hipGetErrorString(e));
    s->inflight.push_back(bi);
    s->cv_complete.notify_one();
  }
  s->launcher_done = true;
  s->cv_complete.notify_one();
}

void completer_loop(scan_server *s) {
  (void)hipSetDevice(s->ix->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    s->cv_complete.wait(lk, [&] { return s->launcher_done || !s->inflight.empty(); });
    if (s->inflight.empty()) break;  // launcher finished and every batch completed
    const int32_t bi = s->inflight.front();
    BatchBuf &b = s->bufs[bi];
    lk.unlock();
    (void)hipEventSynchronize(b.done);
    const int64_t n = s->ix->n;
    for (size_t i = 0; i < b.reqs.size(); ++i) {
      const Request &r = b.reqs[i];
      if (n > 0 && !r.dst_on_device && !r.dst_pinned) std::memcpy(r.dst, b.h_memb[i], (size_t)n * 4);
      if (r.latency_ms)
        *r.latency_ms = std::chrono::duration<double, std::milli>(Clock::now() - r.t_submit).count();
    }
    lk.lock();
    s->inflight.pop_front();
    for (auto &r : b.reqs) s->state[r.ticket] = 2;
    b.reqs.clear();
    s->free_bufs.push_back(bi);
    s->cv_launch.notify_one();
    s->cv_done.notify_all();
  }
}

}  // namespace

extern "C" {

scan_status scan_server_create(const scan_index *ix, const scan_server_opts *opts, scan_server **out) {
  if (!ix || !opts || !out) return fail(SCAN_EINVAL, "null argument");
  *out = nullptr;
  if (opts->max_slots < 1 || opts->max_batch < 1 || opts->max_batch > 1024 || opts->memory_budget < 0)
    return fail(SCAN_EINVAL, "bad server options (max_slots >= 1, 1 <= max_batch <= 1024, budget >= 0)");
  const int64_t n = std::max<int64_t>(ix->n, 1);
  const int64_t per_slot = n * (4 + 1 + 4) + 64;  // parents, flags, device result
  const int64_t by_budget = opts->memory_budget / per_slot;
  const int64_t slots = std::min<int64_t>(opts->max_slots, by_budget);
  if (slots < 1) return fail(SCAN_ENOMEM, "memory budget %lld holds no query slot (%lld bytes each)",
                             (long long)opts->memory_budget, (long long)per_slot);
  if (hipSetDevice(ix->device) != hipSuccess || hipStreamSynchronize(ix->stream) != hipSuccess)
    return fail(SCAN_EDEVICE, "index stream failed");
  scan_server *s = new scan_server();
  s->ix = ix;
  s->opts = *opts;
  s->opts.max_batch = (int32_t)std::min<int64_t>(opts->max_batch, slots);
  s->nbuf = (int32_t)std::max<int64_t>(1, slots / s->opts.max_batch);
  s->pending_cap = (size_t)std::max<int64_t>(4 * slots, 64);
  s->bufs.resize(s->nbuf);
  auto bail = [&](scan_status st) {
    free_server_resources(s);
    delete s;
    return st;
  };
  for (int32_t bi = 0; bi < s->nbuf; ++bi) {
    BatchBuf &b = s->bufs[bi];
    if (hipStreamCreateWithFlags(&b.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b.done, hipEventDisableTiming) != hipSuccess)
      return bail(fail(SCAN_EDEVICE, "server stream/event creation failed"));
    b.slots.resize(s->opts.max_batch);
    b.d_memb.assign(s->opts.max_batch, nullptr);
    b.h_memb.assign(s->opts.max_batch, nullptr);
    for (int32_t i = 0; i < s->opts.max_batch; ++i) {
      scan_status st = alloc_query_slot(ix, &b.slots[i], b.stream);
      if (st != SCAN_OK) return bail(st);
      b.d_memb[i] = (int32_t *)dev_alloc((size_t)n * 4, b.stream);
      if (!b.d_memb[i]) return bail(fail(SCAN_ENOMEM, "server result allocation failed"));
      if (hipHostMalloc((void **)&b.h_memb[i], (size_t)n * 4, hipHostMallocDefault) != hipSuccess)
        return bail(fail(SCAN_ENOMEM, "pinned host allocation failed"));
    }
    b.d_desc = (QueryDesc *)dev_alloc(sizeof(QueryDesc) * s->opts.max_batch, b.stream);
    if (!b.d_desc ||
        hipHostMalloc((void **)&b.h_desc, sizeof(QueryDesc) * s->opts.max_batch, hipHostMallocDefault) != hipSuccess)
      return bail(fail(SCAN_ENOMEM, "descriptor allocation failed"));
    for (int32_t i = 0; i < s->opts.max_batch; ++i) b.h_desc[i] = make_query_desc(2, 0.0, b.slots[i], nullptr, nullptr);
    if (hipStreamSynchronize(b.stream) != hipSuccess) return bail(fail(SCAN_EDEVICE, "server set-up failed"));
    if (opts->use_graph) {
      // The graph holds no memset node; flags are cleared by the kernels.
      if (hipStreamBeginCapture(b.stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return bail(fail(SCAN_EDEVICE, "graph capture failed to start"));
      hipError_t e = enqueue_batch_kernels(s, b);
      hipError_t e2 = hipStreamEndCapture(b.stream, &b.graph);
      if (e != hipSuccess || e2 != hipSuccess ||
          hipGraphInstantiate(&b.exec, b.graph, nullptr, nullptr, 0) != hipSuccess)
        return bail(fail(SCAN_EDEVICE, "graph capture failed"));
    }
    s->free_bufs.push_back(bi);
  }
  s->launcher = std::thread(launcher_loop, s);
  s->completer = std::thread(completer_loop, s);
  *out = s;
  return SCAN_OK;
}

scan_status scan_server_submit_ex(scan_server *s, int32_t mu, double eps, int32_t *dst, int32_t dst_on_device,
                                  double *latency_ms, uint64_t *ticket) {
  const Clock::time_point now = Clock::now();
  if (!s || !ticket || (!dst && s->ix->n > 0)) return fail(SCAN_EINVAL, "null argument");
  if (mu < 2 || std::isnan(eps)) return fail(SCAN_EINVAL, "invalid (mu, eps)");
  bool pinned = false;
  if (!dst_on_device && dst) {
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, dst) == hipSuccess)
      pinned = attr.type == hipMemoryTypeHost;
    else
      (void)hipGetLastError();  // pageable memory: not an error here
  }
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->error != SCAN_OK) return fail(s->error, "server failed earlier");
  if (s->pending.size() >= s->pending_cap) return fail(SCAN_EBUSY, "server queue full");
  const uint64_t t = s->next_ticket++;
  s->pending.push_back(Request{t, mu, eps, dst, dst_on_device != 0, pinned, latency_ms, now});
  s->state[t] = 0;
  *ticket = t;
  s->cv_launch.notify_one();
  return SCAN_OK;
}

scan_status scan_server_submit(scan_server *s, int32_t mu, double eps, int32_t *dst, uint64_t *ticket) {
  return scan_server_submit_ex(s, mu, eps, dst, 0, nullptr, ticket);
}

scan_status scan_server_poll(scan_server *s, uint64_t ticket, int32_t *done) {
  if (!s || !done) return fail(SCAN_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(s->mu);
  if (ticket == 0 || ticket >= s->next_ticket) return fail(SCAN_EINVAL, "unknown ticket");
  auto it = s->state.find(ticket);
  *done = (it == s->state.end() || it->second == 2) ? 1 : 0;
  if (it != s->state.end() && it->second == 2) s->state.erase(it);
  return SCAN_OK;
}

scan_status scan_server_wait(scan_server *s, uint64_t ticket) {
  if (!s) return fail(SCAN_EINVAL, "null argument");
  std::unique_lock<std::mutex> lk(s->mu);
  if (ticket == 0 || ticket >= s->next_ticket) return fail(SCAN_EINVAL, "unknown ticket");
  s->cv_done.wait(lk, [&] {
    auto it = s->state.find(ticket);
    return it == s->state.end() || it->second == 2;
  });
  s->state.erase(ticket);
  return s->error;
}

void scan_server_destroy(scan_server *s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_launch.notify_all();
  if (s->launcher.joinable()) s->launcher.join();
  if (s->completer.joinable()) s->completer.join();
  free_server_resources(s);
  delete s;
}

}  // extern "C"
