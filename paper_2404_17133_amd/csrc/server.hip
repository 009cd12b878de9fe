// Batched solves and the continuous-batching request server.
//
// Both run several solves at once, each on a host thread and HIP stream of
// its own, and share one Batcher: whenever solves wait for operator products,
// the Batcher runs all of them as one grouped product (one persistent grouped
// GEMM launch per contraction stage and tile shape), so that small molecules
// share the chip with large ones and the latency-bound steps of one solve
// (Rayleigh-Ritz, Gram-Schmidt, reads of a few scalars) overlap with the
// products of the others.  A solve's result does not depend on which other
// solves run beside it: every grouped launch computes each member's tiles
// with the same code and plan as a launch of that member alone.
//
// The server admits queued requests in arrival order when a slot is free and
// the request's estimated device footprint fits the remaining budget; a
// request admitted while others run joins their grouped products at the next
// round.  Every admitted solve keeps its subspace in device memory until it
// ends.  Result timestamps (arrival, admission, completion) are in
// milliseconds on the server's steady clock.
#include <algorithm>
#include <cstdlib>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <numeric>
#include <thread>

#include "engine.hpp"
#include "server.hpp"

namespace rid {
namespace {

typedef std::chrono::steady_clock Clock;

enum ReqState { RQ_QUEUED = 0, RQ_RUNNING = 1, RQ_DONE = 2 };

std::mutex g_err_mu;  // last_error is written from several threads

struct Req {
  uint64_t ticket = 0;
  rid_problem* P = nullptr;
  rid_request r{};
  rid_result* res = nullptr;
  int state = RQ_QUEUED;
  bool cancel = false;
  uint64_t bytes = 0;
};

void fill(rid_result* out, const SolveStats& s) { fill_stats(&out->stats, s); }

rid_status run_one(rid_problem* P, const rid_request& r, rid_result* res, const ExecCfg& ex) {
  SolveStats st;
  rid_status s;
  try {
    if (r.kind == 0) {
      s = eigen_solve(P, r.opts, r.k, r.mode, res->omega_host, r.x_dev, r.mode == RID_RPA ? r.y_dev : nullptr,
                      res->resid_host, st, ex);
    } else {
      s = response_solve(P, r.opts, r.nrhs, r.p_dev, r.nfreq, r.omega_host, res->alpha_host, nullptr,
                         res->resid_host, st, ex);
    }
  } catch (const Error& e) {
    std::lock_guard<std::mutex> g(g_err_mu);
    P->ctx->last_error = e.what();
    s = e.code;
  } catch (const std::exception& e) {
    std::lock_guard<std::mutex> g(g_err_mu);
    P->ctx->last_error = e.what();
    s = RID_ERR_INTERNAL;
  }
  fill(res, st);
  res->status = s;
  return s;
}

// A HIP stream owned by one worker thread.
struct WorkerStream {
  hipStream_t s = nullptr;
  explicit WorkerStream(int device) {
    RID_HIP(hipSetDevice(device));
    RID_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  }
  ~WorkerStream() {
    if (s) {
      (void)hipStreamSynchronize(s);
      (void)hipStreamDestroy(s);
    }
  }
};

// Order of a batch (largest first): the operator work per vector of the
// request's molecule.  The number of roots is left out on purpose: a solve's
// wall time inside a batch follows its outer iterations (14 to 41 in the
// 64-molecule workload, not predictable from k) times the latency of one
// iteration, which grows with the molecule and hardly with k, since the
// products of all running solves share grouped launches.
double request_weight(const rid_problem* P, const rid_request& r) {
  (void)r;
  const double n = (double)P->n();
  return n * (double)P->naux * (double)(P->no + P->nv);
}

}  // namespace

}  // namespace rid

struct rid_server {
  rid_context* ctx = nullptr;
  rid_server_opts opts{};
  std::vector<std::thread> workers;
  rid::Batcher* batcher = nullptr;
  rid::DeferFree* defer = nullptr;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<rid::Req*> queue;
  std::map<uint64_t, rid::Req*> all;
  bool stop = false;
  uint64_t next_ticket = 1;
  uint64_t used_bytes = 0;
  int running = 0;
  rid::Clock::time_point epoch;
  double now_ms() const {
    return std::chrono::duration<double, std::milli>(rid::Clock::now() - epoch).count();
  }
};

namespace rid {

uint64_t request_footprint(const rid_problem* P, const rid_request& r) {
  const uint64_t N = (uint64_t)P->n();
  const int k = r.kind == 0 ? r.k : r.nrhs * r.nfreq;
  const int mm = r.opts.m_max > 0 ? r.opts.m_max : std::max(200, 40 * k);
  const uint64_t basis = (uint64_t)(mm + 4 * k + 8) * N * 8 * 3;  // V and two product blocks
  const uint64_t inner = (uint64_t)(2 * k * (r.opts.inner_max_iter + 1)) * N * 8 * 3;
  // vector blocks of the solve, plus the operator scratch: exchange
  // intermediates (chunked to 256 MB each) and split partial sums (up to 8
  // splits of a (no * 2k) x nv block, two of them)
  const uint64_t part = (uint64_t)8 * P->no * (2 * k) * P->nv * 4 * 2;
  const uint64_t work = (uint64_t)(3 * k) * N * 8 * 6 + (768ull << 20) + part;
  // the problem's tensor copies are made before admission and charged to
  // the problem (rid_problem_footprint), not to its requests
  return basis + inner + work;
}

rid_status batch_run(rid_context* ctx, int n, rid_problem* const* probs, const rid_request* reqs,
                     rid_result* results) {
  if (n <= 0) return RID_OK;
  for (int i = 0; i < n; ++i) {
    RID_CHECK(probs[i] && probs[i]->ctx == ctx, RID_ERR_INVALID_ARG, "problem of another context");
    RID_CHECK(reqs[i].kind == 0 || reqs[i].kind == 1, RID_ERR_INVALID_ARG, "bad request kind");
    results[i].status = RID_ERR_PENDING;
  }
  for (int i = 0; i < n; ++i) prepare_problem(probs[i], reqs[i].opts);
  RID_HIP(hipStreamSynchronize(ctx->stream));
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return request_weight(probs[a], reqs[a]) > request_weight(probs[b], reqs[b]);
  });
  // concurrent solves: 16, or RID_BATCH_WORKERS (1..64; a tuning knob)
  static const int max_workers = [] {
    const char* e = std::getenv("RID_BATCH_WORKERS");
    const int v = e ? std::atoi(e) : 0;
    return v >= 1 && v <= 64 ? v : 16;
  }();
  const int nworkers = std::min(n, max_workers);
  // Two ends of the weight order: even workers take the heaviest request
  // left, odd workers the lightest.  The heavy solves keep the matrix cores
  // busy while the light ones, latency-bound, run in their gaps, instead of
  // all light solves queueing behind the heavy ones and then running on a
  // device they cannot fill.
  std::mutex omu;
  int heavy = 0, light = n - 1;
  auto take = [&](int w) {
    std::lock_guard<std::mutex> g(omu);
    if (heavy > light) return -1;
    return w % 2 == 0 ? order[heavy++] : order[light--];
  };
  // admission by estimated footprint against the device memory free at the
  // start (a request too large for the budget runs when it is alone)
  size_t free_b = 0, total_b = 0;
  RID_HIP(hipMemGetInfo(&free_b, &total_b));
  const uint64_t budget = (uint64_t)(0.8 * (double)free_b);
  std::mutex amu;
  std::condition_variable acv;
  uint64_t used = 0;
  int running = 0;
  const Clock::time_point t0 = Clock::now();
  auto ms = [&] { return std::chrono::duration<double, std::milli>(Clock::now() - t0).count(); };
  {
    DeferFree defer(ctx);
    Batcher batcher(ctx);
    std::vector<std::thread> th;
    for (int w = 0; w < nworkers; ++w)
      th.emplace_back([&, w] {
        try {
          WorkerStream ws(ctx->device);
          const ExecCfg ex{ws.s, &batcher};
          for (int i = take(w); i >= 0; i = take(w)) {
            const uint64_t need = request_footprint(probs[i], reqs[i]);
            {
              std::unique_lock<std::mutex> lk(amu);
              acv.wait(lk, [&] { return running == 0 || used + need <= budget; });
              used += need;
              running += 1;
            }
            results[i].t_arrival_ms = 0.0;
            results[i].t_admit_ms = ms();
            run_one(probs[i], reqs[i], &results[i], ex);
            results[i].t_done_ms = ms();
            // hand back what this solve freed before admitting more work
            reap_graveyard(ctx, false);
            {
              std::lock_guard<std::mutex> lk(amu);
              used -= need;
              running -= 1;
            }
            acv.notify_all();
          }
        } catch (const Error& e) {
          std::lock_guard<std::mutex> g(g_err_mu);
          ctx->last_error = e.what();
          for (int i = take(w); i >= 0; i = take(w)) results[i].status = e.code;
        }
      });
    for (std::thread& t : th) t.join();
  }
  rid_status worst = RID_OK;
  for (int i = 0; i < n; ++i) {
    const rid_status s = results[i].status;
    if (s < 0 && worst >= 0) worst = s;
    if (s == RID_WARN_NOT_CONVERGED && worst == RID_OK) worst = s;
  }
  return worst;
}

namespace {

void finish(rid_server* s, Req* q, rid_status st) {
  q->state = RQ_DONE;
  q->res->status = st;
  q->res->t_done_ms = s->now_ms();
  s->cv_done.notify_all();
}

void worker_body(rid_server* s, const ExecCfg& ex);

void worker_loop(rid_server* s) {
  try {
    WorkerStream ws(s->ctx->device);
    worker_body(s, ExecCfg{ws.s, s->batcher});
  } catch (const std::exception& e) {
    // no stream for this slot: the other slots serve the queue
    std::lock_guard<std::mutex> g(g_err_mu);
    s->ctx->last_error = e.what();
  }
}

void worker_body(rid_server* s, const ExecCfg& ex) {
  std::unique_lock<std::mutex> lk(s->mu);
  while (true) {
    // admission: the oldest request, once it fits the remaining budget
    s->cv_work.wait(lk, [&] {
      if (s->queue.empty()) return s->stop;
      Req* h = s->queue.front();
      return h->cancel || h->bytes > s->opts.hbm_budget_bytes ||
             s->used_bytes + h->bytes <= s->opts.hbm_budget_bytes;
    });
    if (s->queue.empty()) return;  // stop
    Req* q = s->queue.front();
    s->queue.pop_front();
    if (q->cancel) {
      finish(s, q, RID_ERR_CANCELLED);
      s->cv_work.notify_all();
      continue;
    }
    if (q->bytes > s->opts.hbm_budget_bytes) {
      finish(s, q, RID_ERR_NO_MEMORY);
      s->cv_work.notify_all();
      continue;
    }
    q->state = RQ_RUNNING;
    q->res->t_admit_ms = s->now_ms();
    s->used_bytes += q->bytes;
    s->running += 1;
    s->cv_work.notify_all();  // the next request may fit too
    lk.unlock();
    const rid_status st = run_one(q->P, q->r, q->res, ex);
    reap_graveyard(s->ctx, false);
    lk.lock();
    s->used_bytes -= q->bytes;
    s->running -= 1;
    finish(s, q, st);
    s->cv_work.notify_all();
  }
}

}  // namespace

rid_server* server_create(rid_context* ctx, const rid_server_opts& o) {
  RID_CHECK(o.max_slots >= 1 && o.max_slots <= 64, RID_ERR_INVALID_ARG, "max_slots must be in [1, 64]");
  RID_HIP(hipStreamSynchronize(ctx->stream));
  rid_server* s = new rid_server();
  s->ctx = ctx;
  s->opts = o;
  s->epoch = Clock::now();
  s->defer = new DeferFree(ctx);
  s->batcher = new Batcher(ctx);
  for (int w = 0; w < o.max_slots; ++w) s->workers.emplace_back(worker_loop, s);
  return s;
}

rid_status server_submit(rid_server* s, rid_problem* P, const rid_request* r, rid_result* res, uint64_t* ticket) {
  if (!P || !r || !res || !ticket) return RID_ERR_INVALID_ARG;
  if (P->ctx != s->ctx) return RID_ERR_INVALID_ARG;
  if (r->kind != 0 && r->kind != 1) return RID_ERR_INVALID_ARG;
  try {
    prepare_problem(P, r->opts);
  } catch (const Error& e) {
    std::lock_guard<std::mutex> g(g_err_mu);
    s->ctx->last_error = e.what();
    return e.code;
  }
  Req* q = new Req();
  q->P = P;
  q->r = *r;
  q->res = res;
  q->bytes = request_footprint(P, *r);
  std::lock_guard<std::mutex> g(s->mu);
  q->ticket = s->next_ticket++;
  res->status = RID_ERR_PENDING;
  res->t_arrival_ms = s->now_ms();
  res->t_admit_ms = res->t_done_ms = -1.0;
  s->all[q->ticket] = q;
  s->queue.push_back(q);
  *ticket = q->ticket;
  s->cv_work.notify_all();
  return RID_OK;
}

rid_status server_poll(rid_server* s, uint64_t ticket) {
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->all.find(ticket);
  if (it == s->all.end()) return RID_ERR_INVALID_ARG;
  return it->second->state == RQ_DONE ? RID_OK : RID_ERR_PENDING;
}

rid_status server_wait(rid_server* s, uint64_t ticket, int timeout_ms) {
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->all.find(ticket);
  if (it == s->all.end()) return RID_ERR_INVALID_ARG;
  Req* q = it->second;
  auto pred = [&] { return q->state == RQ_DONE; };
  if (timeout_ms < 0) {
    s->cv_done.wait(lk, pred);
  } else if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), pred)) {
    return RID_ERR_TIMEOUT;
  }
  return RID_OK;
}

rid_status server_cancel(rid_server* s, uint64_t ticket) {
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->all.find(ticket);
  if (it == s->all.end()) return RID_ERR_INVALID_ARG;
  it->second->cancel = true;
  s->cv_work.notify_all();
  return RID_OK;
}

void server_destroy(rid_server* s) {
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
    for (Req* q : s->queue) q->cancel = true;
  }
  s->cv_work.notify_all();
  for (std::thread& t : s->workers)
    if (t.joinable()) t.join();
  delete s->batcher;
  delete s->defer;
  for (auto& kv : s->all) delete kv.second;
  delete s;
}

}  // namespace rid
