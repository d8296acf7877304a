// Serving loop of libsfmgm: single-pair requests arriving one by one are
// batched on the fly and matched with the batched form.
//
// Pairs are independent (Section 6.1 matches them in parallel), so a request
// stream can be served by concatenating whatever requests are waiting into
// one batched launch.  A worker thread admits up to max_batch_pairs waiting
// requests whenever one of max_inflight slots is free and enqueues the batch
// on that slot's own stream and workspace (a share of the context's budget),
// so the launches of different slots overlap on the device; while they run,
// new arrivals queue up and form the next batch.  A completion thread waits for each batch in
// launch order, copies exactly the accepted matches into pinned host memory,
// and hands every request its rows.  A request's latency runs from its
// arrival time to the moment its rows are in host memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <system_error>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "sfm_gm.h"
#include "sfm_internal.h"

namespace sfm {
namespace {

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct Request {
  uint64_t ticket;
  sfm_pair pair;
  double F[9];
  int64_t arrival_ns;
};

struct Result {
  int32_t status = SFM_OK;
  int64_t n = 0;                   // accepted rows
  std::vector<int32_t> rows;       // query[n] | match[n] | d1[n] | d2[n]
  int64_t n_comparisons = 0;
  int64_t arrival_ns = 0, done_ns = 0;
};

// Launches with at least this many accepted rows copy them into the
// requests' results on several threads.
constexpr int64_t kParallelCopyRows = int64_t(1) << 18;
constexpr int kCopyThreads = 4;

// Device outputs of one launch and their pinned host mirrors.
struct Slot {
  int32_t *q = nullptr, *m = nullptr, *d1 = nullptr, *d2 = nullptr;
  int64_t *offset = nullptr, *ncmp = nullptr;
  int32_t *hq = nullptr, *hm = nullptr, *hd1 = nullptr, *hd2 = nullptr;
  int64_t *hoffset = nullptr, *hncmp = nullptr;
  hipEvent_t meta = nullptr, rows = nullptr;
  hipStream_t stream = nullptr;   // this slot's matching and metadata copies
  ServeSpace* space = nullptr;    // this slot's workspace
  std::vector<Request> reqs;
  int32_t status = SFM_OK;
};

struct Server {
  sfm_ctx* ctx = nullptr;
  int32_t device = 0;
  sfm_server_cfg cfg{};
  hipStream_t copy = nullptr;     // row copies
  std::vector<Slot> slots;

  std::mutex mu;
  std::condition_variable cv_work;   // worker: requests or a free slot
  std::condition_variable cv_done;   // completion thread and pollers
  std::deque<Request> queue;
  std::deque<int> free_slots;
  std::deque<int> inflight;          // launch order
  std::unordered_map<uint64_t, Result> results;
  std::unordered_set<uint64_t> outstanding;   // submitted, not yet collected
  uint64_t next_ticket = 1;
  bool stopping = false;
  bool worker_done = false;          // the worker has launched everything and exited
  bool closed = false;               // stopped: threads joined, slots freed
  int64_t launches = 0, launched_pairs = 0;
  size_t slot_budget = 0;            // device workspace per slot

  std::thread worker, completer;
};

// Servers are shared: a caller that found one keeps it alive until its call
// returns, even if another thread stops it meanwhile.
std::mutex g_servers_mu;
std::unordered_map<sfm_ctx*, std::shared_ptr<Server>> g_servers;

std::shared_ptr<Server> find_server(sfm_ctx* ctx) {
  std::lock_guard<std::mutex> lk(g_servers_mu);
  auto it = g_servers.find(ctx);
  return it == g_servers.end() ? nullptr : it->second;
}

void free_slot(Slot& s) {
  if (s.q) (void)hipFree(s.q);
  if (s.m) (void)hipFree(s.m);
  if (s.d1) (void)hipFree(s.d1);
  if (s.d2) (void)hipFree(s.d2);
  if (s.offset) (void)hipFree(s.offset);
  if (s.ncmp) (void)hipFree(s.ncmp);
  if (s.hq) (void)hipHostFree(s.hq);
  if (s.hm) (void)hipHostFree(s.hm);
  if (s.hd1) (void)hipHostFree(s.hd1);
  if (s.hd2) (void)hipHostFree(s.hd2);
  if (s.hoffset) (void)hipHostFree(s.hoffset);
  if (s.hncmp) (void)hipHostFree(s.hncmp);
  if (s.meta) (void)hipEventDestroy(s.meta);
  if (s.rows) (void)hipEventDestroy(s.rows);
  serve_space_destroy(s.space);
  if (s.stream) (void)hipStreamDestroy(s.stream);
  s = Slot();
}

bool alloc_slot(Slot& s, sfm_ctx* ctx, size_t budget, int64_t rows, int32_t pairs) {
  const size_t r4 = size_t(std::max<int64_t>(rows, 1)) * sizeof(int32_t);
  const size_t p8 = size_t(pairs + 1) * sizeof(int64_t);
  s.space = serve_space_create(ctx, budget);
  return s.space && hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) == hipSuccess &&
         hipMalloc(&s.q, r4) == hipSuccess && hipMalloc(&s.m, r4) == hipSuccess &&
         hipMalloc(&s.d1, r4) == hipSuccess && hipMalloc(&s.d2, r4) == hipSuccess &&
         hipMalloc(&s.offset, p8) == hipSuccess && hipMalloc(&s.ncmp, p8) == hipSuccess &&
         hipHostMalloc(reinterpret_cast<void**>(&s.hq), r4, hipHostMallocDefault) == hipSuccess &&
         hipHostMalloc(reinterpret_cast<void**>(&s.hm), r4, hipHostMallocDefault) == hipSuccess &&
         hipHostMalloc(reinterpret_cast<void**>(&s.hd1), r4, hipHostMallocDefault) == hipSuccess &&
         hipHostMalloc(reinterpret_cast<void**>(&s.hd2), r4, hipHostMallocDefault) == hipSuccess &&
         hipHostMalloc(reinterpret_cast<void**>(&s.hoffset), p8, hipHostMallocDefault) ==
             hipSuccess &&
         hipHostMalloc(reinterpret_cast<void**>(&s.hncmp), p8, hipHostMallocDefault) ==
             hipSuccess &&
         hipEventCreateWithFlags(&s.meta, hipEventDisableTiming) == hipSuccess &&
         hipEventCreateWithFlags(&s.rows, hipEventDisableTiming) == hipSuccess;
}

// Fails every request of a batch with `status`.
void fail_batch(Server& S, std::vector<Request>& reqs, int32_t status) {
  const int64_t t = now_ns();
  for (const Request& r : reqs) {
    Result& res = S.results[r.ticket];
    res.status = status;
    res.arrival_ns = r.arrival_ns;
    res.done_ns = t;
  }
  reqs.clear();
}

// Admits waiting requests into free slots and launches them.
void worker_main(Server* Sp) {
  Server& S = *Sp;
  (void)hipSetDevice(S.device);
  std::vector<sfm_pair> pairs;
  std::vector<double> F;
  for (;;) {
    int slot_id;
    std::vector<Request> batch;
    {
      std::unique_lock<std::mutex> lk(S.mu);
      S.cv_work.wait(lk, [&] { return (!S.queue.empty() && !S.free_slots.empty()) ||
                                      (S.stopping && S.queue.empty()); });
      if (S.queue.empty()) return;   // stopping, everything launched
      slot_id = S.free_slots.front();
      S.free_slots.pop_front();
      // Admission in arrival order while the launch stays within the pair
      // and query caps and its workspace within the context's budget.
      int64_t queries = 0;
      size_t bytes = ctx_call_bytes(S.ctx);
      const size_t budget = S.slot_budget;
      while (!S.queue.empty() && int32_t(batch.size()) < S.cfg.max_batch_pairs) {
        const Request& r = S.queue.front();
        const int64_t na = ctx_image_size(S.ctx, r.pair.a);
        const size_t rb = ctx_request_bytes(S.ctx, r.pair.a, r.pair.b);
        if (!batch.empty() && (queries + na > S.cfg.max_batch_queries || bytes + rb > budget))
          break;
        queries += na;
        bytes += rb;
        batch.push_back(r);
        S.queue.pop_front();
      }
    }
    Slot& s = S.slots[size_t(slot_id)];
    pairs.clear();
    F.clear();
    for (const Request& r : batch) {
      pairs.push_back(r.pair);
      F.insert(F.end(), r.F, r.F + 9);
    }
    sfm_matches out;
    memset(&out, 0, sizeof out);
    out.query = s.q;
    out.match = s.m;
    out.d1 = s.d1;
    out.d2 = s.d2;
    out.offset = s.offset;
    out.n_comparisons = s.ncmp;
    out.capacity = std::max<int64_t>(S.cfg.max_batch_queries, 0);
    int64_t need = 0;
    for (const Request& r : batch) need += ctx_image_size(S.ctx, r.pair.a);
    out.capacity = std::max(out.capacity, need);
    int rc = SFM_OK;
    if (need > S.cfg.max_batch_queries) {
      rc = SFM_ECAPACITY;   // a single request larger than the slot
    } else {
      rc = serve_match(S.ctx, s.space, pairs.data(), int32_t(pairs.size()), F.data(),
                       &S.cfg.opt, &out, s.stream);
    }
    const int32_t n = int32_t(batch.size());
    if (rc == SFM_OK) {
      if (hipMemcpyAsync(s.hoffset, s.offset, size_t(n + 1) * sizeof(int64_t),
                         hipMemcpyDeviceToHost, s.stream) != hipSuccess ||
          hipMemcpyAsync(s.hncmp, s.ncmp, size_t(n) * sizeof(int64_t), hipMemcpyDeviceToHost,
                         s.stream) != hipSuccess ||
          hipEventRecord(s.meta, s.stream) != hipSuccess)
        rc = SFM_EHIP;
    }
    std::lock_guard<std::mutex> lk(S.mu);
    s.reqs = std::move(batch);
    s.status = rc;
    S.inflight.push_back(slot_id);
    ++S.launches;
    S.launched_pairs += n;
    S.cv_done.notify_all();
  }
}

// Results [k0, k1) of one launch from the host mirrors of its rows.
void fill_results(const Slot& s, const std::vector<Request>& reqs, const std::vector<int64_t>& off,
                  const std::vector<int64_t>& ncmp, int64_t t, size_t k0, size_t k1,
                  std::vector<Result>& out) {
  for (size_t k = k0; k < k1; ++k) {
    Result& res = out[k];
    const int64_t b = off[k], n = off[k + 1] - off[k];
    res.status = SFM_OK;
    res.n = n;
    res.rows.resize(size_t(4 * n));
    int32_t* dst = res.rows.data();
    memcpy(dst, s.hq + b, size_t(n) * sizeof(int32_t));
    memcpy(dst + n, s.hm + b, size_t(n) * sizeof(int32_t));
    memcpy(dst + 2 * n, s.hd1 + b, size_t(n) * sizeof(int32_t));
    memcpy(dst + 3 * n, s.hd2 + b, size_t(n) * sizeof(int32_t));
    res.n_comparisons = ncmp[k];
    res.arrival_ns = reqs[k].arrival_ns;
    res.done_ns = t;
  }
}

// Waits for launches in order and hands out their results.  Once a launch's
// rows are in the slot's host mirrors, the slot's device buffers go back to
// the worker (its offsets and counts were copied out first), so the next
// launch runs while this thread copies the rows into the requests' results,
// outside the lock and on several threads for large launches.  The mirrors
// are rewritten only by this thread's own copy of a later launch.
void completer_main(Server* Sp) {
  Server& S = *Sp;
  (void)hipSetDevice(S.device);
  std::vector<int64_t> off, ncmp;
  for (;;) {
    int slot_id;
    {
      std::unique_lock<std::mutex> lk(S.mu);
      S.cv_done.wait(lk, [&] { return !S.inflight.empty() || S.worker_done; });
      if (S.inflight.empty()) return;
      slot_id = S.inflight.front();
    }
    Slot& s = S.slots[size_t(slot_id)];
    int32_t rc = s.status;
    const size_t n = s.reqs.size();
    if (rc == SFM_OK && hipEventSynchronize(s.meta) != hipSuccess) rc = SFM_EHIP;
    if (rc == SFM_OK) {
      off.assign(s.hoffset, s.hoffset + n + 1);
      ncmp.assign(s.hncmp, s.hncmp + n);
      const int64_t total = off[n];
      if (total > 0) {
        const size_t b = size_t(total) * sizeof(int32_t);
        if (hipMemcpyAsync(s.hq, s.q, b, hipMemcpyDeviceToHost, S.copy) != hipSuccess ||
            hipMemcpyAsync(s.hm, s.m, b, hipMemcpyDeviceToHost, S.copy) != hipSuccess ||
            hipMemcpyAsync(s.hd1, s.d1, b, hipMemcpyDeviceToHost, S.copy) != hipSuccess ||
            hipMemcpyAsync(s.hd2, s.d2, b, hipMemcpyDeviceToHost, S.copy) != hipSuccess ||
            hipEventRecord(s.rows, S.copy) != hipSuccess ||
            hipEventSynchronize(s.rows) != hipSuccess)
          rc = SFM_EHIP;
      }
    }
    const int64_t t = now_ns();
    std::vector<Request> reqs = std::move(s.reqs);
    s.reqs.clear();
    {
      std::lock_guard<std::mutex> lk(S.mu);
      S.inflight.pop_front();
      S.free_slots.push_back(slot_id);
      if (rc != SFM_OK) fail_batch(S, reqs, rc);
      S.cv_work.notify_all();
      S.cv_done.notify_all();
    }
    if (rc != SFM_OK) continue;
    std::vector<Result> out(n);
    if (off[n] < kParallelCopyRows || n < 2) {
      fill_results(s, reqs, off, ncmp, t, 0, n, out);
    } else {
      // Contiguous runs of requests with about equal rows per thread.
      std::vector<size_t> cut(kCopyThreads + 1, n);
      cut[0] = 0;
      for (int i = 1; i < kCopyThreads; ++i)
        cut[i] = size_t(std::lower_bound(off.begin(), off.end(), off[n] * i / kCopyThreads) -
                        off.begin());
      for (int i = 1; i <= kCopyThreads; ++i) cut[i] = std::max(std::min(cut[i], n), cut[i - 1]);
      std::vector<std::thread> helpers;
      int i = 1;
      for (; i < kCopyThreads; ++i) {
        try {
          helpers.emplace_back(fill_results, std::cref(s), std::cref(reqs), std::cref(off),
                               std::cref(ncmp), t, cut[size_t(i)], cut[size_t(i) + 1],
                               std::ref(out));
        } catch (const std::system_error&) {
          break;   // no thread to spare: this thread copies the rest
        }
      }
      fill_results(s, reqs, off, ncmp, t, cut[0], cut[1], out);
      for (; i < kCopyThreads; ++i)
        fill_results(s, reqs, off, ncmp, t, cut[size_t(i)], cut[size_t(i) + 1], out);
      for (std::thread& h : helpers) h.join();
    }
    std::lock_guard<std::mutex> lk(S.mu);
    for (size_t k = 0; k < n; ++k) S.results[reqs[k].ticket] = std::move(out[k]);
    S.cv_done.notify_all();
  }
}

void shutdown(Server* S) {
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stopping = true;
    S->cv_work.notify_all();
    S->cv_done.notify_all();
  }
  if (S->worker.joinable()) S->worker.join();
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->worker_done = true;
    S->cv_done.notify_all();
  }
  if (S->completer.joinable()) S->completer.join();
  (void)hipSetDevice(S->device);
  for (Slot& s : S->slots)
    if (s.stream) (void)hipStreamSynchronize(s.stream);
  if (S->copy) (void)hipStreamSynchronize(S->copy);
  for (Slot& s : S->slots) free_slot(s);
  if (S->copy) (void)hipStreamDestroy(S->copy);
  S->copy = nullptr;
  std::lock_guard<std::mutex> lk(S->mu);
  S->closed = true;
  S->cv_done.notify_all();   // pollers still waiting return SFM_EBUSY
}

}  // namespace

void server_release(sfm_ctx* ctx) {
  std::shared_ptr<Server> S;
  {
    std::lock_guard<std::mutex> lk(g_servers_mu);
    auto it = g_servers.find(ctx);
    if (it == g_servers.end()) return;
    S = it->second;
    g_servers.erase(it);
  }
  shutdown(S.get());
}

}  // namespace sfm

using namespace sfm;

extern "C" {

int64_t sfm_server_now_ns(void) { return now_ns(); }

int sfm_server_start(sfm_ctx* ctx, const sfm_server_cfg* cfg_in) {
  if (!ctx) return SFM_EINVAL;
  if (find_server(ctx)) return SFM_EBUSY;
  sfm_server_cfg cfg;
  memset(&cfg, 0, sizeof cfg);
  cfg.max_batch_pairs = 256;
  cfg.max_inflight = 2;
  cfg.max_batch_queries = int64_t(1) << 22;
  cfg.opt.ratio_num = 64;
  cfg.opt.ratio_den = 100;
  cfg.opt.recheck_margin_px = 1e-3;
  if (cfg_in) cfg = *cfg_in;
  if (cfg.max_batch_pairs < 1 || cfg.max_inflight < 1 || cfg.max_inflight > 8 ||
      cfg.max_batch_queries < 1 || cfg.opt.ratio_den <= 0 || cfg.opt.ratio_num < 0 ||
      cfg.opt.emit_all || !(cfg.opt.recheck_margin_px >= 0.0) ||
      !std::isfinite(cfg.opt.recheck_margin_px))
    return SFM_EINVAL;
  std::shared_ptr<Server> S = std::make_shared<Server>();
  S->ctx = ctx;
  S->device = ctx_device(ctx);
  S->cfg = cfg;
  // Each slot matches on its own stream and workspace, its share of the
  // context's budget.
  S->slot_budget = ctx_budget(ctx) / size_t(cfg.max_inflight);
  if (hipSetDevice(S->device) != hipSuccess ||
      hipStreamCreateWithFlags(&S->copy, hipStreamNonBlocking) != hipSuccess) {
    shutdown(S.get());
    return SFM_EHIP;
  }
  S->slots.resize(size_t(cfg.max_inflight));
  for (int k = 0; k < cfg.max_inflight; ++k) {
    if (!alloc_slot(S->slots[size_t(k)], ctx, S->slot_budget, cfg.max_batch_queries,
                    cfg.max_batch_pairs)) {
      shutdown(S.get());
      return SFM_ENOMEM;
    }
    S->free_slots.push_back(k);
  }
  {
    std::lock_guard<std::mutex> lk(g_servers_mu);
    g_servers[ctx] = S;
  }
  S->worker = std::thread(worker_main, S.get());
  S->completer = std::thread(completer_main, S.get());
  return SFM_OK;
}

int sfm_server_submit(sfm_ctx* ctx, const sfm_pair* pair, const double* F, int64_t arrival_ns,
                      uint64_t* ticket) {
  return sfm_server_submit_batch(ctx, pair, 1, F, arrival_ns, ticket);
}

int sfm_server_submit_batch(sfm_ctx* ctx, const sfm_pair* pairs, int32_t n, const double* F,
                            int64_t arrival_ns, uint64_t* tickets) {
  if (!ctx || n < 0 || (n > 0 && (!pairs || !F || !tickets))) return SFM_EINVAL;
  std::shared_ptr<Server> S = find_server(ctx);
  if (!S) return SFM_EBUSY;
  const int32_t n_images = ctx_n_images(ctx);
  for (int32_t i = 0; i < n; ++i) {
    const sfm_pair& p = pairs[i];
    if (p.a < 0 || p.a >= n_images || p.b < 0 || p.b >= n_images || !(p.band_px >= 0.0))
      return SFM_EINVAL;
    bool nonzero = false;
    for (int k = 0; k < 9; ++k) {
      const double f = F[int64_t(i) * 9 + k];
      if (!std::isfinite(f)) return SFM_EINVAL;
      nonzero |= f != 0.0;
    }
    if (!nonzero) return SFM_EINVAL;
  }
  const int64_t t = arrival_ns > 0 ? arrival_ns : now_ns();
  std::lock_guard<std::mutex> lk(S->mu);
  if (S->stopping) return SFM_EBUSY;
  for (int32_t i = 0; i < n; ++i) {
    Request r;
    r.pair = pairs[i];
    memcpy(r.F, F + int64_t(i) * 9, sizeof r.F);
    r.arrival_ns = t;
    r.ticket = S->next_ticket++;
    tickets[i] = r.ticket;
    S->outstanding.insert(r.ticket);
    S->queue.push_back(r);
  }
  if (n > 0) S->cv_work.notify_one();
  return SFM_OK;
}

int sfm_server_poll(sfm_ctx* ctx, uint64_t ticket, sfm_result_view* out, int32_t timeout_ms) {
  if (!ctx || !out) return SFM_EINVAL;
  std::shared_ptr<Server> S = find_server(ctx);
  if (!S) return SFM_EBUSY;
  std::unique_lock<std::mutex> lk(S->mu);
  if (!S->outstanding.count(ticket)) return SFM_ENOTFOUND;
  auto ready = [&] { return S->results.count(ticket) != 0; };
  auto done = [&] { return ready() || S->closed; };
  if (!ready()) {
    if (timeout_ms == 0) return S->closed ? SFM_EBUSY : SFM_ETIMEOUT;
    if (timeout_ms < 0) {
      S->cv_done.wait(lk, done);
    } else if (!S->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), done)) {
      return SFM_ETIMEOUT;
    }
    if (!ready()) return SFM_EBUSY;   // the server was stopped meanwhile
  }
  Result& res = S->results[ticket];
  const int64_t n = res.n;
  out->status = res.status;
  out->n_matches = n;
  out->n_comparisons = res.n_comparisons;
  out->arrival_ns = res.arrival_ns;
  out->done_ns = res.done_ns;
  if (res.status == SFM_OK && n > 0) {
    if (out->capacity < n || !out->query || !out->match || !out->d1 || !out->d2)
      return SFM_ECAPACITY;   // the result stays collectable with a larger buffer
    const int32_t* r = res.rows.data();
    memcpy(out->query, r, size_t(n) * sizeof(int32_t));
    memcpy(out->match, r + n, size_t(n) * sizeof(int32_t));
    memcpy(out->d1, r + 2 * n, size_t(n) * sizeof(int32_t));
    memcpy(out->d2, r + 3 * n, size_t(n) * sizeof(int32_t));
  }
  S->results.erase(ticket);
  S->outstanding.erase(ticket);
  return SFM_OK;
}

int sfm_server_stats(sfm_ctx* ctx, int64_t out[3]) {
  if (!ctx || !out) return SFM_EINVAL;
  std::shared_ptr<Server> S = find_server(ctx);
  if (!S) return SFM_EBUSY;
  std::lock_guard<std::mutex> lk(S->mu);
  out[0] = S->launches;
  out[1] = S->launched_pairs;
  out[2] = int64_t(S->queue.size());
  return SFM_OK;
}

int sfm_server_stop(sfm_ctx* ctx) {
  if (!ctx) return SFM_EINVAL;
  if (!find_server(ctx)) return SFM_EBUSY;
  server_release(ctx);
  return SFM_OK;
}

}  // extern "C"
