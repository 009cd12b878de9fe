// Threading test of the library's host scheduling code on the CPU (test
// infrastructure only): the real Batcher, device-buffer release with its
// fenced graveyard, batch_run and the request server, built against a CPU
// stand-in of the HIP host calls (fakehip/).  The solves and the operator
// products are stand-ins too: a "solve" grows and releases device buffers
// as the Krylov solvers do, asks the Batcher (or its own stream) for
// products y = 2 x, y2 = 3 x computed through the job's scratch buffers on
// the product stream, and checks every product against its input on the
// host.  Results must be right, every allocation must be returned exactly
// once, and (under ThreadSanitizer / AddressSanitizer) no data race or
// use-after-free may be reported.
#include <atomic>
#include <cstdio>
#include <deque>
#include <map>
#include <random>
#include <thread>
#include <vector>

#include "core.hpp"
#include "engine.hpp"
#include "server.hpp"

namespace {

// ---- allocator with accounting --------------------------------------------
struct Heap {
  std::mutex mu;
  std::map<void*, size_t> live;
  std::atomic<long> allocs{0}, frees{0}, bad_frees{0}, concurrent{0}, max_concurrent{0};
};
Heap g_heap;

void* heap_alloc(void*, size_t n) {
  // the library promises never to call the allocator from two threads at once
  const long c = ++g_heap.concurrent;
  long m = g_heap.max_concurrent.load();
  while (c > m && !g_heap.max_concurrent.compare_exchange_weak(m, c)) {
  }
  void* p = std::aligned_alloc(256, (n + 255) / 256 * 256);
  {
    std::lock_guard<std::mutex> g(g_heap.mu);
    g_heap.live[p] = n;
  }
  ++g_heap.allocs;
  --g_heap.concurrent;
  return p;
}

void heap_free(void*, void* p) {
  const long c = ++g_heap.concurrent;
  long m = g_heap.max_concurrent.load();
  while (c > m && !g_heap.max_concurrent.compare_exchange_weak(m, c)) {
  }
  {
    std::lock_guard<std::mutex> g(g_heap.mu);
    auto it = g_heap.live.find(p);
    if (it == g_heap.live.end()) {
      ++g_heap.bad_frees;
    } else {
      g_heap.live.erase(it);
    }
  }
  std::free(p);
  ++g_heap.frees;
  --g_heap.concurrent;
}

std::atomic<long> g_products{0}, g_bad_products{0}, g_bad_results{0};
std::atomic<long> g_scopes{0};  // profiled launches recorded

// deterministic "root" of request r of a problem: what a solve must return
double expected_root(const rid_problem* P, int j) { return 0.001 * P->no + 0.01 * j; }

}  // namespace

namespace rid {

// ---- stand-ins for the kernels and solvers --------------------------------

void check_operator(const rid_problem*, int, int) {}
void prepare_problem(rid_problem* P, const rid_solve_opts&) {
  // a lazily made tensor copy, as the real problems keep
  std::lock_guard<std::mutex> g(P->mu);
  if (!P->b_ai32.p) P->b_ai32.ensure(sizeof(float) * (size_t)P->n());
}
void ring_free(DescRing*) {}

void fill_stats(rid_stats* out, const SolveStats& s) {
  if (!out) return;
  std::memset(out, 0, sizeof(*out));
  out->n_iter = s.n_iter;
}

// y = 2 x, y2 = 3 x for each job, through the job's scratch: x is copied
// into the scratch buffer on the product stream and the outputs computed
// from it, so that a scratch buffer released too early shows up as a
// use-after-free and a wrong result.
void run_jobs(rid_context* ctx, OpJob* const* jobs, int n, hipStream_t st, const OpLimits*) {
  ProfScope ps(ctx, st, "fake_product", 1.0, 1.0);
  if (ctx->prof.on) ++g_scopes;
  for (int q = 0; q < n; ++q) {
    OpJob* j = jobs[q];
    const size_t elems = (size_t)j->nvec * j->P->n();
    // scratch sized by the product, as the chunked exchange products are:
    // it grows, and the old buffer is released while earlier work may
    // still read it
    j->work->xc.ensure(sizeof(double) * elems);
    j->work->s.ensure(sizeof(double) * elems / 2 + 64);
    double* xc = j->work->xc.as<double>();
    double* sc = j->work->s.as<double>();
    const double* x = j->x;
    double* y = j->y;
    double* y2 = j->y2;
    (void)hipMemcpyAsync(xc, x, sizeof(double) * elems, hipMemcpyDeviceToDevice, st);
    fakehip::resolve(st)->push([=] {
      // a product takes a while: solves move on while it runs
      std::this_thread::sleep_for(std::chrono::microseconds(150));
      for (size_t i = 0; i < elems; ++i) {
        if (i < elems / 2) sc[i] = xc[i];
        y[i] = 2.0 * xc[i];
        if (y2) y2[i] = 3.0 * xc[i];
      }
    });
    ++g_products;
  }
}

namespace {

// a solve's product: through the Batcher when it shares the device
void product(rid_problem* P, const ExecCfg& ex, OpWork& own, hipEvent_t ready, int nvec, const double* x, double* y,
             double* y2) {
  OpJob j;
  j.P = P;
  j.kind = y2 ? OPK_PAIR : OPK_A;
  j.prec = PREC_F64;
  j.nvec = nvec;
  j.x = x;
  j.y = y;
  j.y2 = y2;
  j.stream = ex.stream;
  if (ex.batcher) {
    j.work = &own;
    j.ready = ready;
    ex.batcher->apply(j);
  } else {
    j.work = &P->work;
    OpJob* jp = &j;
    run_jobs(P->ctx, &jp, 1, ex.stream ? ex.stream : P->ctx->stream, nullptr);
  }
}

rid_status fake_solve(rid_problem* P, int k, double* out, const ExecCfg& ex, uint64_t seed) {
  rid_context* ctx = P->ctx;
  hipStream_t st = ex.stream ? ex.stream : ctx->stream;
  ThreadStream fence(st);
  OpWork own(ctx);
  hipEvent_t ready = nullptr;
  if (ex.batcher) RID_HIP(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
  const long N = P->n();
  std::mt19937_64 rng(seed);
  DevBuf basis(ctx), prod(ctx), prod2(ctx), tmp(ctx);
  // products are not waited for one by one: their inputs and outputs are
  // checked in groups, while the solve grows and drops buffers meanwhile
  struct Pending {
    std::vector<double> x, y, y2;
    bool pair;
  };
  std::deque<Pending> pend;
  auto check = [&]() {
    RID_HIP(hipStreamSynchronize(st));
    for (const Pending& q : pend)
      for (size_t i = 0; i < q.x.size(); ++i)
        if (q.y[i] != 2.0 * q.x[i] || (q.pair && q.y2[i] != 3.0 * q.x[i])) {
          ++g_bad_products;
          break;
        }
    pend.clear();
  };
  const int iters = 3 + (int)(rng() % 6);
  for (int it = 0; it < iters; ++it) {
    const int nvec = 1 + (int)(rng() % (2 * k));
    // the basis and product blocks grow like a Krylov subspace: a larger
    // block replaces a smaller one that an earlier product may still read
    // or write; a temporary is made and dropped
    const size_t elems = (size_t)nvec * N;
    basis.ensure(sizeof(double) * elems);
    prod.ensure(sizeof(double) * elems);
    prod2.ensure(sizeof(double) * elems);
    tmp.ensure(sizeof(double) * (size_t)(1 + rng() % 8) * N);
    pend.emplace_back();
    Pending& q = pend.back();
    q.pair = it % 2 == 1;
    q.x.resize(elems);
    q.y.assign(elems, 0.0);
    q.y2.assign(elems, 0.0);
    for (size_t i = 0; i < elems; ++i) q.x[i] = (double)((seed + it * 131 + i * 7) % 1000) - 500.0;
    {
      ProfScope ps(ctx, st, "fake_copy", 0.0, 8.0 * elems);
      if (ctx->prof.on) ++g_scopes;
      RID_HIP(hipMemcpyAsync(basis.p, q.x.data(), sizeof(double) * elems, hipMemcpyHostToDevice, st));
    }
    product(P, ex, own, ready, nvec, basis.as<double>(), prod.as<double>(), q.pair ? prod2.as<double>() : nullptr);
    RID_HIP(hipMemcpyAsync(q.y.data(), prod.p, sizeof(double) * elems, hipMemcpyDeviceToHost, st));
    if (q.pair) RID_HIP(hipMemcpyAsync(q.y2.data(), prod2.p, sizeof(double) * elems, hipMemcpyDeviceToHost, st));
    if (rng() % 3 == 0) tmp.release();
    if (rng() % 3 == 0) check();
  }
  check();
  for (int j = 0; j < k; ++j) out[j] = expected_root(P, j);
  if (ready) {
    RID_HIP(hipStreamSynchronize(st));
    (void)hipEventDestroy(ready);
  }
  return RID_OK;
}

}  // namespace

rid_status eigen_solve(rid_problem* P, const rid_solve_opts&, int k, int, double* omega_host, double*, double*,
                       double* resid_host, SolveStats& st, const ExecCfg& ex) {
  st.n_iter = 1;
  if (resid_host)
    for (int j = 0; j < k; ++j) resid_host[j] = 0.0;
  return fake_solve(P, k, omega_host, ex, (uint64_t)P->no * 7919 + k);
}

rid_status response_solve(rid_problem* P, const rid_solve_opts&, int nrhs, const double*, int nfreq, const double*,
                          double* alpha_host, double*, double*, SolveStats& st, const ExecCfg& ex) {
  st.n_iter = 1;
  return fake_solve(P, nrhs * nfreq, alpha_host, ex, (uint64_t)P->no * 104729 + nrhs);
}

}  // namespace rid

namespace {

rid_problem* make_problem(rid_context* ctx, int no) {
  rid_problem* P = new rid_problem(ctx);
  P->no = no;
  P->nv = 4 * no;
  P->naux = 20 * no;
  return P;
}

rid_request eigen_request(int k) {
  rid_request r{};
  r.kind = 0;
  r.k = k;
  r.mode = RID_RPA;
  r.opts.inner_max_iter = 20;
  r.opts.precision = RID_PRECISION_MIXED;
  return r;
}

bool check_result(const rid_problem* P, const rid_result& res, int k) {
  if (res.status != RID_OK) return false;
  const double* v = res.omega_host ? res.omega_host : res.alpha_host;
  for (int j = 0; j < k; ++j)
    if (v[j] != expected_root(P, j)) return false;
  return true;
}

int test_batch(rid_context* ctx, int rounds) {
  std::mt19937 rng(1);
  for (int round = 0; round < rounds; ++round) {
    const int n = 24 + round * 8;
    std::vector<rid_problem*> probs;
    std::vector<rid_request> reqs;
    std::vector<rid_result> res(n);
    std::vector<std::vector<double>> out(n);
    for (int i = 0; i < n; ++i) {
      probs.push_back(make_problem(ctx, 4 + (int)(rng() % 20)));
      const int k = 1 + (int)(rng() % 6);
      reqs.push_back(eigen_request(k));
      out[i].assign(k, -1.0);
      std::memset(&res[i], 0, sizeof(rid_result));
      res[i].omega_host = out[i].data();
    }
    const rid_status s = rid::batch_run(ctx, n, probs.data(), reqs.data(), res.data());
    if (s != RID_OK) {
      std::printf("batch round %d: status %d (%s)\n", round, s, ctx->last_error.c_str());
      return 1;
    }
    for (int i = 0; i < n; ++i)
      if (!check_result(probs[i], res[i], reqs[i].k)) ++g_bad_results;
    for (rid_problem* P : probs) delete P;
  }
  return 0;
}

int test_server(rid_context* ctx) {
  rid_server_opts o{};
  o.max_slots = 6;
  // room for a few requests at once: admission has to wait for releases
  {
    rid_problem* ref = make_problem(ctx, 12);
    o.hbm_budget_bytes = (uint64_t)4 * rid::request_footprint(ref, eigen_request(4));
    delete ref;
  }
  rid_server* srv = rid::server_create(ctx, o);
  const int nthreads = 3, per = 20;
  std::vector<rid_problem*> probs;
  std::mutex pmu;
  std::vector<std::thread> th;
  std::atomic<int> ok{0}, cancelled{0}, bad{0};
  for (int t = 0; t < nthreads; ++t)
    th.emplace_back([&, t] {
      std::mt19937 rng(100 + t);
      std::vector<rid_problem*> mine;
      std::vector<rid_result> res(per);
      std::vector<std::vector<double>> out(per);
      std::vector<rid_request> reqs(per);
      std::vector<uint64_t> tick(per, 0);
      for (int i = 0; i < per; ++i) {
        mine.push_back(make_problem(ctx, 4 + (int)(rng() % 24)));
        reqs[i] = eigen_request(1 + (int)(rng() % 5));
        if (i % 4 == 3) {  // a polarizability request
          reqs[i].kind = 1;
          reqs[i].nrhs = 3;
          reqs[i].nfreq = 1;
        }
        const int k = reqs[i].kind == 0 ? reqs[i].k : 3;
        out[i].assign(k, -1.0);
        std::memset(&res[i], 0, sizeof(rid_result));
        if (reqs[i].kind == 0)
          res[i].omega_host = out[i].data();
        else
          res[i].alpha_host = out[i].data();
        if (rid::server_submit(srv, mine[i], &reqs[i], &res[i], &tick[i]) != RID_OK) ++bad;
        if (rng() % 7 == 0) rid::server_cancel(srv, tick[i]);
        if (rng() % 3 == 0) std::this_thread::sleep_for(std::chrono::microseconds(200));
      }
      for (int i = 0; i < per; ++i) {
        if (rid::server_wait(srv, tick[i], -1) != RID_OK) {
          ++bad;
          continue;
        }
        if (res[i].status == RID_ERR_CANCELLED) {
          ++cancelled;
        } else if (check_result(mine[i], res[i], (int)out[i].size())) {
          ++ok;
        } else {
          ++bad;
        }
      }
      std::lock_guard<std::mutex> g(pmu);
      probs.insert(probs.end(), mine.begin(), mine.end());
    });
  for (auto& t : th) t.join();
  rid::server_destroy(srv);
  for (rid_problem* P : probs) delete P;
  std::printf("server: %d done, %d cancelled, %d wrong\n", ok.load(), cancelled.load(), bad.load());
  return bad.load() == 0 && ok.load() + cancelled.load() == nthreads * per ? 0 : 1;
}

}  // namespace

int main(int argc, char** argv) {
  const int rounds = argc > 1 ? std::atoi(argv[1]) : 3;
  hipStream_t main_stream;
  (void)hipStreamCreateWithFlags(&main_stream, hipStreamNonBlocking);
  rid_context* ctx = new rid_context();
  ctx->stream = main_stream;
  ctx->alloc.alloc = heap_alloc;
  ctx->alloc.free = heap_free;
  // launch profiling on, and read while the solves record (as a caller of
  // rid_profile_read on another thread would)
  ctx->prof.on = true;
  std::atomic<bool> reading{true};
  long read_launches = 0;
  std::thread reader([&] {
    while (reading) {
      for (const auto& f : ctx->prof.take()) read_launches += f.second.launches;
      std::this_thread::sleep_for(std::chrono::microseconds(300));
    }
  });
  int rc = test_batch(ctx, rounds);
  rc |= test_server(ctx);
  reading = false;
  reader.join();
  (void)hipDeviceSynchronize();
  for (const auto& f : ctx->prof.take()) read_launches += f.second.launches;
  ctx->prof.on = false;
  std::printf("profiled launches %ld of %ld recorded\n", read_launches, g_scopes.load());
  if (read_launches != g_scopes.load()) rc = 1;
  // a solve alone on the context stream (no Batcher, no deferred release)
  {
    rid_problem* P = make_problem(ctx, 9);
    std::vector<double> om(4);
    rid::SolveStats st;
    rid_solve_opts o{};
    rid::eigen_solve(P, o, 4, RID_TDA, om.data(), nullptr, nullptr, nullptr, st, rid::ExecCfg());
    for (int j = 0; j < 4; ++j)
      if (om[j] != expected_root(P, j)) ++g_bad_results;
    delete P;
  }
  delete ctx;
  (void)hipStreamDestroy(main_stream);
  size_t leaked;
  {
    std::lock_guard<std::mutex> g(g_heap.mu);
    leaked = g_heap.live.size();
  }
  std::printf("products %ld (wrong %ld), wrong results %ld, allocations %ld, frees %ld, bad frees %ld, leaked %zu, "
              "max concurrent allocator calls %ld\n",
              g_products.load(), g_bad_products.load(), g_bad_results.load(), g_heap.allocs.load(),
              g_heap.frees.load(), g_heap.bad_frees.load(), leaked, g_heap.max_concurrent.load());
  if (g_bad_products || g_bad_results || g_heap.bad_frees || leaked || g_heap.max_concurrent > 1) rc = 1;
  std::printf(rc == 0 ? "SCHED_OK\n" : "SCHED_FAIL\n");
  return rc;
}
