// Continuous batching of trace requests (ctr_server_* in include/ctrace.h).
//
// One worker thread per context (impurity), each on its context's stream:
// requests queue per impurity; when a worker's device pass ends it admits the
// requests that arrived meanwhile, in arrival order, up to the batch limit,
// the scratch budget and an optional cap on the pass's estimated work, and
// evaluates them as one batch.  Different
// impurities' passes run concurrently on their own streams.  An optional grid
// share per impurity launches only that fraction of each persistent grid, so
// the workgroups of one impurity's long pass leave slots on the device where
// another impurity's kernels start without waiting for that pass to end.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "ctrace_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
  uint64_t tag;
  std::vector<double> tau;
  std::vector<int32_t> op;
  double log_thr;
  Clock::time_point t0;
};

struct Lane {
  ctr_ctx* ctx = nullptr;
  int index = 0;
  double beta = 0.0;
  int nops = 0;
  size_t budget = 0;
  std::deque<Request> pending;
  std::mutex m;
  std::condition_variable cv;
  std::thread worker;
};

}  // namespace

struct ctr_server {
  std::vector<std::unique_ptr<Lane>> lanes;
  int max_batch = 1;
  int max_pending = 1;
  double max_pass_flop = 0.0;  // 0: no cap on a pass's estimated block-product flops
  std::mutex rm;
  std::condition_variable rcv;
  std::deque<ctr_result> done;
  std::atomic<long long> outstanding{0};
  std::atomic<long long> passes{0};
  std::atomic<long long> evaluated{0};
  std::atomic<bool> stop{false};
};

namespace {

void run_lane(ctr_server* srv, Lane* L) {
  std::vector<Request> batch;
  std::vector<int64_t> offs;
  std::vector<double> tau, thr;
  std::vector<int32_t> op;
  std::vector<ctr_value> out;
  for (;;) {
    batch.clear();
    {
      std::unique_lock<std::mutex> lk(L->m);
      L->cv.wait(lk, [&] { return srv->stop.load() || !L->pending.empty(); });
      if (srv->stop.load()) return;
      size_t bytes = 0;
      double flop = 0.0;
      while (!L->pending.empty() && (int)batch.size() < srv->max_batch) {
        const Request& f = L->pending.front();
        const size_t need = ctr::request_scratch_bytes(L->ctx, (long long)f.op.size(), f.op.data());
        if (!batch.empty() && bytes + need > L->budget) break;  // admission by scratch footprint
        if (srv->max_pass_flop > 0.0) {
          // a cap on the pass's work keeps passes short, so requests arriving meanwhile wait less
          const double w = ctr::request_flops(L->ctx, (long long)f.op.size(), f.op.data());
          if (!batch.empty() && flop + w > srv->max_pass_flop) break;
          flop += w;
        }
        bytes += need;
        batch.push_back(std::move(L->pending.front()));
        L->pending.pop_front();
      }
    }
    const int n = (int)batch.size();
    offs.assign(1, 0);
    tau.clear();
    op.clear();
    thr.clear();
    bool lazy = false;
    for (const Request& q : batch) {
      tau.insert(tau.end(), q.tau.begin(), q.tau.end());
      op.insert(op.end(), q.op.begin(), q.op.end());
      offs.push_back((int64_t)op.size());
      thr.push_back(q.log_thr);
      lazy = lazy || !(q.log_thr == -INFINITY);
    }
    out.assign(n, ctr_value{});
    ctr_opts o{};
    const ctr_status st = lazy ? ctr_trace_lazy_batch(L->ctx, n, offs.data(), tau.data(), op.data(), thr.data(),
                                                      &o, out.data())
                               : ctr_trace_batch(L->ctx, n, offs.data(), tau.data(), op.data(), &o, out.data());
    const Clock::time_point t1 = Clock::now();
    {
      std::lock_guard<std::mutex> lk(srv->rm);
      for (int i = 0; i < n; ++i) {
        ctr_result r{};
        r.tag = batch[i].tag;
        r.impurity = L->index;
        r.status = st;
        r.value = out[i];
        r.latency_ms = std::chrono::duration<double, std::milli>(t1 - batch[i].t0).count();
        r.batch = n;
        srv->done.push_back(r);
      }
      srv->passes += 1;
      srv->evaluated += n;
      srv->outstanding -= n;
    }
    srv->rcv.notify_all();
  }
}

}  // namespace

extern "C" {

ctr_status ctr_server_create(ctr_ctx* const* ctxs, int32_t n_ctx, const ctr_server_opts* opts, ctr_server** out) {
  if (!out) return CTR_ERR_ARG;
  *out = nullptr;
  if (!ctxs || n_ctx < 1 || !opts || opts->max_batch < 1 || opts->max_pending < 1) return CTR_ERR_ARG;
  for (int i = 0; i < n_ctx; ++i) {
    if (!ctxs[i]) return CTR_ERR_ARG;
    if (!ctr::context_loaded(ctxs[i])) return CTR_ERR_STATE;
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == ctxs[i]) return CTR_ERR_ARG;  // one worker per context
  }
  if (opts->grid_share)
    for (int i = 0; i < n_ctx; ++i)
      if (!(opts->grid_share[i] > 0.0 && opts->grid_share[i] <= 1.0)) return CTR_ERR_ARG;
  ctr_server* srv = new ctr_server();
  srv->max_batch = opts->max_batch;
  srv->max_pending = opts->max_pending;
  srv->max_pass_flop = opts->max_pass_flop > 0.0 ? opts->max_pass_flop : 0.0;
  for (int i = 0; i < n_ctx; ++i) {
    std::unique_ptr<Lane> L(new Lane());
    L->ctx = ctxs[i];
    L->index = i;
    L->beta = ctr::context_beta(ctxs[i]);
    L->nops = ctr::context_nops(ctxs[i]);
    const size_t free_bytes = ctr::context_free_scratch(ctxs[i]);
    L->budget = opts->hbm_budget ? std::min(opts->hbm_budget, free_bytes) : free_bytes;
    ctr::context_set_grid_share(ctxs[i], opts->grid_share ? opts->grid_share[i] : 1.0);
    srv->lanes.push_back(std::move(L));
  }
  for (auto& L : srv->lanes) L->worker = std::thread(run_lane, srv, L.get());
  *out = srv;
  return CTR_OK;
}

ctr_status ctr_server_submit(ctr_server* srv, int32_t impurity, uint64_t tag, int32_t n_ops, const double* tau,
                             const int32_t* op, double log_threshold) {
  if (!srv) return CTR_ERR_ARG;
  if (srv->stop.load()) return CTR_ERR_STATE;
  if (impurity < 0 || impurity >= (int)srv->lanes.size()) return CTR_ERR_ARG;
  if (n_ops < 0 || n_ops > ctr::kMaxOps || (n_ops > 0 && (!tau || !op))) return CTR_ERR_ARG;
  Lane* L = srv->lanes[impurity].get();
  for (int i = 0; i < n_ops; ++i) {
    if (!(tau[i] >= 0.0 && tau[i] < L->beta)) return CTR_ERR_RANGE;
    if (op[i] < 0 || op[i] >= L->nops) return CTR_ERR_RANGE;
    if (i > 0 && !(tau[i] >= tau[i - 1])) return CTR_ERR_UNSORTED;
  }
  Request q;
  q.tag = tag;
  q.tau.assign(tau, tau + n_ops);
  q.op.assign(op, op + n_ops);
  q.log_thr = log_threshold;
  q.t0 = Clock::now();
  {
    std::lock_guard<std::mutex> lk(L->m);
    if ((int)L->pending.size() >= srv->max_pending) return CTR_ERR_BUSY;
    srv->outstanding += 1;
    L->pending.push_back(std::move(q));
  }
  L->cv.notify_one();
  return CTR_OK;
}

ctr_status ctr_server_poll(ctr_server* srv, ctr_result* out, int32_t max, int32_t* n_out, int32_t wait) {
  if (!srv || !n_out || max < 0 || (max > 0 && !out)) return CTR_ERR_ARG;
  std::unique_lock<std::mutex> lk(srv->rm);
  if (wait) srv->rcv.wait(lk, [&] { return !srv->done.empty() || srv->outstanding.load() == 0; });
  int k = 0;
  while (k < max && !srv->done.empty()) {
    out[k++] = srv->done.front();
    srv->done.pop_front();
  }
  *n_out = k;
  return CTR_OK;
}

ctr_status ctr_server_drain(ctr_server* srv) {
  if (!srv) return CTR_ERR_ARG;
  std::unique_lock<std::mutex> lk(srv->rm);
  srv->rcv.wait(lk, [&] { return srv->outstanding.load() == 0; });
  return CTR_OK;
}

ctr_status ctr_server_stats(const ctr_server* srv, int64_t* n_passes, int64_t* n_requests) {
  if (!srv || !n_passes || !n_requests) return CTR_ERR_ARG;
  *n_passes = srv->passes.load();
  *n_requests = srv->evaluated.load();
  return CTR_OK;
}

void ctr_server_destroy(ctr_server* srv) {
  if (!srv) return;
  srv->stop.store(true);
  for (auto& L : srv->lanes) {
    { std::lock_guard<std::mutex> lk(L->m); }
    L->cv.notify_all();
  }
  for (auto& L : srv->lanes)
    if (L->worker.joinable()) L->worker.join();
  for (auto& L : srv->lanes) ctr::context_set_grid_share(L->ctx, 1.0);
  delete srv;
}

}  // extern "C"
