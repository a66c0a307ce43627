// Request server: continuous admission of independent resolves by slots
// and by an estimated device-footprint budget.  Host code only; every
// request runs the single-pair entry point on a worker's own context and
// stream.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/hfcr.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
  hfcr_pair *pair = nullptr;
  hfcr_opts opts;
  int64_t footprint = 0;
  Clock::time_point submitted, finished;
  bool done = false;
  hfcr_status status = HFCR_OK;
};

int64_t footprint_of(const hfcr_pair &p) {
  const int64_t nv = (int64_t)p.a.nv + p.b.nv, nt = (int64_t)p.a.nt + p.b.nt;
  return 512 * nv + 1024 * nt + (1 << 20);
}

}  // namespace

struct hfcr_server {
  int device = 0;
  hfcr_server_cfg cfg{8, 0, 0};
  std::mutex mu;
  std::condition_variable cv_work;  // workers: a request may be admissible
  std::condition_variable cv_done;  // waiters: a request finished
  std::deque<uint64_t> queue;       // tickets in arrival order
  std::unordered_map<uint64_t, Request> reqs;
  uint64_t next_ticket = 1;
  int64_t running = 0, completed = 0, admitted = 0;
  bool stopping = false;
  std::vector<std::thread> workers;
  std::vector<hfcr_ctx *> ctxs;
  std::vector<hipStream_t> streams;

  // Head of the queue if it fits the free budget (arrival order is kept:
  // a large request at the head waits for memory rather than being passed).
  bool admissible() const {
    if (queue.empty()) return false;
    const Request &r = reqs.at(queue.front());
    return cfg.pool_bytes <= 0 || admitted + r.footprint <= cfg.pool_bytes;
  }

  void work(int wi) {
    (void)hipSetDevice(device);
    for (;;) {
      uint64_t t = 0;
      Request *r = nullptr;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv_work.wait(lk, [&] { return admissible() || (stopping && queue.empty()); });
        if (queue.empty()) return;  // stopping and drained
        t = queue.front();
        queue.pop_front();
        r = &reqs.at(t);
        admitted += r->footprint;
        ++running;
      }
      hfcr_pair &q = *r->pair;
      hfcr_opts o = r->opts;
      o.inv_mass_a = q.inv_mass_a;
      o.inv_mass_b = q.inv_mass_b;
      const hfcr_status st = hfcr_resolve(ctxs[wi], &q.a, &q.b, q.orientation, q.d, &o, &q.res, streams[wi]);
      {
        std::lock_guard<std::mutex> lk(mu);
        q.status = st;
        r->status = st;
        r->finished = Clock::now();
        r->done = true;
        admitted -= r->footprint;
        --running;
        ++completed;
      }
      cv_done.notify_all();
      cv_work.notify_all();
    }
  }
};

extern "C" {

hfcr_status hfcr_server_create(hfcr_server **out, int device, const hfcr_server_cfg *cfg) {
  if (!out) return HFCR_E_INVALID;
  *out = nullptr;
  hfcr_server_cfg c{8, 0, 0};
  if (cfg) c = *cfg;
  if (c.slots < 1 || c.slots > 64 || c.pool_bytes < 0) return HFCR_E_INVALID;
  hfcr_server *s = new hfcr_server();
  s->device = device;
  s->cfg = c;
  int prev = 0;
  (void)hipGetDevice(&prev);
  hfcr_status st = HFCR_OK;
  for (int i = 0; i < c.slots && st == HFCR_OK; ++i) {
    hfcr_ctx *ctx = nullptr;
    st = hfcr_create(&ctx, device);
    if (st != HFCR_OK) break;
    s->ctxs.push_back(ctx);
    hipStream_t hs = nullptr;
    if (hipSetDevice(device) != hipSuccess || hipStreamCreateWithFlags(&hs, hipStreamNonBlocking) != hipSuccess) {
      st = HFCR_E_DEVICE;
      break;
    }
    s->streams.push_back(hs);
  }
  (void)hipSetDevice(prev);
  if (st != HFCR_OK) {
    hfcr_server_destroy(s);
    return st;
  }
  for (int i = 0; i < c.slots; ++i) s->workers.emplace_back([s, i] { s->work(i); });
  *out = s;
  return HFCR_OK;
}

void hfcr_server_destroy(hfcr_server *s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stopping = true;
  }
  s->cv_work.notify_all();
  for (auto &t : s->workers) t.join();
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(s->device);
  for (hipStream_t hs : s->streams) (void)hipStreamDestroy(hs);
  (void)hipSetDevice(prev);
  for (hfcr_ctx *c : s->ctxs) hfcr_destroy(c);
  delete s;
}

hfcr_status hfcr_server_submit(hfcr_server *s, hfcr_pair *pair, const hfcr_opts *opts, uint64_t *ticket) {
  if (!s || !pair || !ticket) return HFCR_E_INVALID;
  Request r;
  r.pair = pair;
  hfcr_default_opts(&r.opts);
  if (opts) r.opts = *opts;
  r.footprint = footprint_of(*pair);
  r.submitted = Clock::now();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stopping) return HFCR_E_REJECTED;
    if (s->cfg.pool_bytes > 0 && r.footprint > s->cfg.pool_bytes) return HFCR_E_REJECTED;
    *ticket = s->next_ticket++;
    s->reqs.emplace(*ticket, r);
    s->queue.push_back(*ticket);
  }
  s->cv_work.notify_one();
  return HFCR_OK;
}

hfcr_status hfcr_server_wait(hfcr_server *s, uint64_t ticket, int64_t timeout_us, double *latency_ms) {
  if (!s) return HFCR_E_INVALID;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return HFCR_E_INVALID;
  auto ready = [&] { return s->reqs.at(ticket).done; };
  if (timeout_us < 0)
    s->cv_done.wait(lk, ready);
  else if (!s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready))
    return HFCR_PENDING;
  Request r = s->reqs.at(ticket);
  s->reqs.erase(ticket);
  if (latency_ms) latency_ms[0] = std::chrono::duration<double, std::milli>(r.finished - r.submitted).count();
  return r.status;
}

void hfcr_server_counts(const hfcr_server *s, int64_t *queued, int64_t *running, int64_t *completed,
                        int64_t *admitted_bytes) {
  if (!s) return;
  std::lock_guard<std::mutex> lk(const_cast<hfcr_server *>(s)->mu);
  if (queued) *queued = (int64_t)s->queue.size();
  if (running) *running = s->running;
  if (completed) *completed = s->completed;
  if (admitted_bytes) *admitted_bytes = s->admitted;
}

}  // extern "C"
