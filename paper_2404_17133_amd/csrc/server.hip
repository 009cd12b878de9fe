// Batched solves and the request server.
//
// The server owns one worker thread.  Submitted requests wait in a FIFO
// queue; the worker admits a request when a slot is free and its estimated
// device footprint fits the remaining budget, then runs the admitted requests.
// Result timestamps (arrival, admission, completion) are in milliseconds on
// the server's steady clock.
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <thread>

#include "engine.hpp"
#include "server.hpp"

namespace rid {
namespace {

typedef std::chrono::steady_clock Clock;

enum ReqState { RQ_QUEUED = 0, RQ_RUNNING = 1, RQ_DONE = 2 };

struct Req {
  uint64_t ticket = 0;
  rid_problem* P = nullptr;
  rid_request r{};
  rid_result* res = nullptr;
  int state = RQ_QUEUED;
  bool cancel = false;
  uint64_t bytes = 0;
};

void fill(rid_result* out, const SolveStats& s) {
  rid_stats& o = out->stats;
  std::memset(&o, 0, sizeof(o));
  o.n_iter = s.n_iter;
  o.n_mv = s.n_mv;
  o.n_inner_mv = s.n_inner_mv;
  o.n_inner_iter = s.n_inner_iter;
  o.n_history = (int)std::min<size_t>(s.history.size(), RID_MAX_HISTORY);
  for (int i = 0; i < o.n_history; ++i) o.history[i] = s.history[i];
  o.t_matvec_ms = s.t_matvec;
  o.t_precond_ms = s.t_precond;
  o.t_total_ms = s.t_total;
  o.t_other_ms = std::max(0.0, s.t_total - s.t_matvec - s.t_precond);
  o.bytes_resident = s.peak_bytes;
}

rid_status run_one(rid_problem* P, const rid_request& r, rid_result* res) {
  SolveStats st;
  rid_status s;
  try {
    RID_HIP(hipSetDevice(P->ctx->device));
    if (r.kind == 0) {
      s = eigen_solve(P, r.opts, r.k, r.mode, res->omega_host, nullptr, nullptr, res->resid_host, st);
    } else {
      s = response_solve(P, r.opts, r.nrhs, r.p_dev, r.nfreq, r.omega_host, res->alpha_host, nullptr,
                         res->resid_host, st);
    }
  } catch (const Error& e) {
    P->ctx->last_error = e.what();
    s = e.code;
  } catch (const std::exception& e) {
    P->ctx->last_error = e.what();
    s = RID_ERR_INTERNAL;
  }
  fill(res, st);
  res->status = s;
  return s;
}

}  // namespace

}  // namespace rid

struct rid_server {
  rid_context* ctx = nullptr;
  rid_server_opts opts{};
  std::thread worker;
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
  const uint64_t tens = (uint64_t)P->naux * (N + (uint64_t)P->no * P->no + (uint64_t)P->nv * P->nv) *
                        (r.opts.precision == RID_PRECISION_MIXED ? 4 : 0);
  const uint64_t work = (uint64_t)(3 * k) * N * 8 * 6 + (256ull << 20);
  return basis + inner + tens + work;
}

rid_status batch_run(rid_context* ctx, int n, rid_problem* const* probs, const rid_request* reqs,
                     rid_result* results) {
  (void)ctx;
  rid_status worst = RID_OK;
  for (int i = 0; i < n; ++i) {
    const rid_status s = run_one(probs[i], reqs[i], &results[i]);
    if (s < 0 && worst >= 0) worst = s;
    if (s == RID_WARN_NOT_CONVERGED && worst == RID_OK) worst = s;
  }
  return worst;
}

namespace {

void worker_loop(rid_server* s) {
  std::unique_lock<std::mutex> lk(s->mu);
  while (true) {
    s->cv_work.wait(lk, [&] { return s->stop || !s->queue.empty(); });
    if (s->stop && s->queue.empty()) return;
    // admission: FIFO, by slot and footprint
    Req* q = s->queue.front();
    if (q->cancel) {
      s->queue.pop_front();
      q->state = RQ_DONE;
      q->res->status = RID_ERR_CANCELLED;
      q->res->t_done_ms = s->now_ms();
      s->cv_done.notify_all();
      continue;
    }
    if (q->bytes > s->opts.hbm_budget_bytes) {
      s->queue.pop_front();
      q->state = RQ_DONE;
      q->res->status = RID_ERR_NO_MEMORY;
      q->res->t_done_ms = s->now_ms();
      s->cv_done.notify_all();
      continue;
    }
    s->queue.pop_front();
    q->state = RQ_RUNNING;
    q->res->t_admit_ms = s->now_ms();
    s->used_bytes += q->bytes;
    s->running += 1;
    lk.unlock();
    run_one(q->P, q->r, q->res);
    lk.lock();
    s->used_bytes -= q->bytes;
    s->running -= 1;
    q->res->t_done_ms = s->now_ms();
    q->state = RQ_DONE;
    s->cv_done.notify_all();
  }
}

}  // namespace

rid_server* server_create(rid_context* ctx, const rid_server_opts& o) {
  rid_server* s = new rid_server();
  s->ctx = ctx;
  s->opts = o;
  s->epoch = Clock::now();
  s->worker = std::thread(worker_loop, s);
  return s;
}

rid_status server_submit(rid_server* s, rid_problem* P, const rid_request* r, rid_result* res, uint64_t* ticket) {
  if (!P || !r || !res || !ticket) return RID_ERR_INVALID_ARG;
  if (P->ctx != s->ctx) return RID_ERR_INVALID_ARG;
  if (r->kind != 0 && r->kind != 1) return RID_ERR_INVALID_ARG;
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
  return RID_OK;
}

void server_destroy(rid_server* s) {
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
    for (Req* q : s->queue) q->cancel = true;
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  for (auto& kv : s->all) delete kv.second;
  delete s;
}

}  // namespace rid
