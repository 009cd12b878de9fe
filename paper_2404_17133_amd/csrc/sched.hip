// Host-side scheduling of the library: device buffers and their deferred
// release, the per-thread fence stream, launch profiling and the Batcher that
// groups the operator products of concurrent solves.  Only HIP host calls
// (streams, events, copies) -- no kernels -- so that the same source also
// builds against a CPU stand-in of those calls for the threading tests.
#include <algorithm>
#include <string>

#include "core.hpp"

namespace rid {

int Profiler::family(const char* name) {
  auto it = ids.find(name);
  if (it != ids.end()) return it->second;
  const int id = (int)names.size();
  names.push_back(name);
  ids[name] = id;
  acc.emplace_back();
  return id;
}

hipEvent_t Profiler::get_event() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e;
  RID_HIP(hipEventCreate(&e));
  return e;
}

void Profiler::resolve() {
  std::lock_guard<std::mutex> g(mu);
  std::vector<Rec> pending;
  for (const Rec& r : recs) {
    const hipError_t q = hipEventQuery(r.b);
    if (q == hipErrorNotReady) {
      pending.push_back(r);
      continue;
    }
    float ms = 0.0f;
    if (q == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      Acc& a = acc[r.fam];
      a.launches += 1;
      a.ms += ms;
      a.flops += r.flops;
      a.bytes += r.bytes;
    } else {
      (void)hipGetLastError();
    }
    pool.push_back(r.a);
    pool.push_back(r.b);
  }
  recs.swap(pending);
}

std::vector<std::pair<std::string, Profiler::Acc>> Profiler::take() {
  resolve();
  std::lock_guard<std::mutex> g(mu);
  std::vector<std::pair<std::string, Acc>> out;
  for (size_t f = 0; f < names.size(); ++f) {
    if (acc[f].launches == 0) continue;
    out.emplace_back(names[f], acc[f]);
    acc[f] = Acc();
  }
  return out;
}

Profiler::~Profiler() {
  for (const Rec& r : recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (hipEvent_t e : pool) (void)hipEventDestroy(e);
}

ProfScope::ProfScope(rid_context* c, hipStream_t s, const char* name, double fl, double by)
    : ctx(c), st(s), flops(fl), bytes(by) {
  if (!ctx || !ctx->prof.on) return;
  std::lock_guard<std::mutex> g(ctx->prof.mu);
  if (!ctx->prof.only.empty() && ctx->prof.only != name) return;
  fam = ctx->prof.family(name);
  a = ctx->prof.get_event();
  RID_HIP(hipEventRecord(a, st));
}

ProfScope::~ProfScope() {
  if (fam < 0) return;
  std::lock_guard<std::mutex> g(ctx->prof.mu);
  hipEvent_t b = nullptr;
  try {
    b = ctx->prof.get_event();
  } catch (...) {
    return;
  }
  (void)hipEventRecord(b, st);
  ctx->prof.recs.push_back(Profiler::Rec{fam, a, b, flops, bytes});
}

void* dev_alloc(rid_context* ctx, size_t bytes) {
  if (bytes == 0) bytes = 256;
  std::lock_guard<std::mutex> g(ctx->mu);
  void* p = ctx->alloc.alloc(ctx->alloc.user, bytes);
  RID_CHECK(p != nullptr, RID_ERR_NO_MEMORY, "allocator returned NULL for " + std::to_string(bytes) + " bytes");
  return p;
}

void dev_free(rid_context* ctx, void* p) {
  if (!p) return;
  std::lock_guard<std::mutex> g(ctx->mu);
  ctx->alloc.free(ctx->alloc.user, p);
}

namespace {
thread_local hipStream_t tl_stream = nullptr;
}  // namespace

hipStream_t thread_stream() { return tl_stream; }
ThreadStream::ThreadStream(hipStream_t s) : prev(tl_stream) { tl_stream = s; }
ThreadStream::~ThreadStream() { tl_stream = prev; }

void* Arena::take(size_t n) {
  const size_t want = (std::max<size_t>(n, 256) + 255) & ~(size_t)255;
  RID_CHECK(want <= cap - used, RID_ERR_SHAPE,
            "product needs more scratch than the fixed region holds (" + std::to_string(cap >> 20) + " MiB)");
  void* q = base + used;
  used += want;
  return q;
}

void DevBuf::release() {
  if (arena) {  // slices of a fixed region are never returned
    p = nullptr;
    bytes = 0;
    return;
  }
  if (p && ctx) {
    bool park = false;
    {
      std::lock_guard<std::mutex> g(ctx->grave_mu);
      park = ctx->defer_free > 0;
    }
    if (park) {
      hipEvent_t ev = nullptr;
      {
        std::lock_guard<std::mutex> g(ctx->grave_mu);
        if (!ctx->grave_events.empty()) {
          ev = ctx->grave_events.back();
          ctx->grave_events.pop_back();
        }
      }
      if (!ev && hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) ev = nullptr;
      hipStream_t s = tl_stream ? tl_stream : ctx->stream;
      if (ev && hipEventRecord(ev, s) != hipSuccess) {
        (void)hipEventDestroy(ev);
        ev = nullptr;
      }
      if (!ev) (void)hipDeviceSynchronize();  // no fence available: wait for everything
      {
        std::lock_guard<std::mutex> g(ctx->grave_mu);
        ctx->graveyard.push_back(rid_context::Parked{p, bytes, ev});
        ctx->grave_bytes += bytes;
      }
      reap_graveyard(ctx, false);
    } else {
      // memory may still be in use by queued work on the context stream
      (void)hipStreamSynchronize(ctx->stream);
      dev_free(ctx, p);
    }
  }
  p = nullptr;
  bytes = 0;
}

void reap_graveyard(rid_context* ctx, bool wait) {
  std::vector<rid_context::Parked> done;
  {
    std::lock_guard<std::mutex> g(ctx->grave_mu);
    std::vector<rid_context::Parked> keep;
    for (const rid_context::Parked& q : ctx->graveyard) {
      bool ready = !q.ev;
      if (!ready) {
        if (wait) {
          (void)hipEventSynchronize(q.ev);
          ready = true;
        } else {
          const hipError_t e = hipEventQuery(q.ev);
          ready = e == hipSuccess;
          if (e != hipSuccess && e != hipErrorNotReady) {
            (void)hipGetLastError();
            (void)hipEventSynchronize(q.ev);
            ready = true;
          }
        }
      }
      if (ready) {
        done.push_back(q);
        ctx->grave_bytes -= q.bytes;
        if (q.ev) ctx->grave_events.push_back(q.ev);
      } else {
        keep.push_back(q);
      }
    }
    ctx->graveyard.swap(keep);
  }
  for (const rid_context::Parked& q : done) dev_free(ctx, q.p);
}

DeferFree::DeferFree(rid_context* c) : ctx(c) {
  std::lock_guard<std::mutex> g(ctx->grave_mu);
  ctx->defer_free += 1;
}

DeferFree::~DeferFree() {
  bool last;
  {
    std::lock_guard<std::mutex> g(ctx->grave_mu);
    last = --ctx->defer_free == 0;
  }
  if (last) flush_graveyard(ctx);
}

void DevBuf::ensure(size_t n) {
  if (n <= bytes && p) return;
  if (arena) {
    p = arena->take(n);
    bytes = std::max<size_t>(n, 256);
    return;
  }
  release();
  size_t want = std::max<size_t>(n, 256);
  p = dev_alloc(ctx, want);
  bytes = want;
}

Batcher::Batcher(rid_context* ctx) : ctx_(ctx) {
  RID_HIP(hipSetDevice(ctx->device));
  for (Lane& L : lanes_) {
    RID_HIP(hipStreamCreateWithFlags(&L.st, hipStreamNonBlocking));
    L.events.resize(64, nullptr);
    for (hipEvent_t& e : L.events) RID_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }
  for (Lane& L : lanes_) L.thread = std::thread([this, &L] { loop(L); });
}

Batcher::~Batcher() {
  {
    std::lock_guard<std::mutex> g(mu_);
    stop_ = true;
  }
  for (Lane& L : lanes_) L.cv.notify_all();
  for (Lane& L : lanes_) {
    if (L.thread.joinable()) L.thread.join();
    (void)hipStreamSynchronize(L.st);
    for (hipEvent_t e : L.events)
      if (e) (void)hipEventDestroy(e);
    (void)hipStreamDestroy(L.st);
  }
}

void Batcher::apply(OpJob& j) {
  j.finished = false;
  j.code = 0;
  j.msg.clear();
  RID_HIP(hipEventRecord(j.ready, j.stream));
  Lane& L = lanes_[(j.kind == OPK_T || j.kind == OPK_TPAIR) ? 1 : 0];
  std::unique_lock<std::mutex> lk(mu_);
  L.pending.push_back(&j);
  L.cv.notify_all();
  cv_done_.wait(lk, [&] { return j.finished; });
  if (j.code != 0) throw Error((rid_status)j.code, j.msg);
}

void Batcher::loop(Lane& L) {
  (void)hipSetDevice(ctx_->device);
  ThreadStream ts(L.st);
  std::unique_lock<std::mutex> lk(mu_);
  while (true) {
    L.cv.wait(lk, [&] { return stop_ || !L.pending.empty(); });
    if (L.pending.empty()) {
      if (stop_) return;
      continue;
    }
    std::vector<OpJob*> batch;
    batch.swap(L.pending);
    lk.unlock();
    int code = 0;
    std::string msg;
    try {
      for (OpJob* j : batch) RID_HIP(hipStreamWaitEvent(L.st, j->ready, 0));
      run_jobs(ctx_, batch.data(), (int)batch.size(), L.st);
      hipEvent_t done = L.events[L.next_event];
      L.next_event = (L.next_event + 1) % (int)L.events.size();
      RID_HIP(hipEventRecord(done, L.st));
      for (OpJob* j : batch) RID_HIP(hipStreamWaitEvent(j->stream, done, 0));
    } catch (const Error& e) {
      code = e.code;
      msg = e.what();
    } catch (const std::exception& e) {
      code = RID_ERR_INTERNAL;
      msg = e.what();
    }
    lk.lock();
    L.rounds += 1;
    L.jobs += (int64_t)batch.size();
    for (OpJob* j : batch) {
      j->code = code;
      j->msg = msg;
      j->finished = true;
    }
    cv_done_.notify_all();
  }
}

OpGraph::~OpGraph() {
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
}

void GraphCache::clear() {
  for (OpGraph* g : graphs) delete g;
  graphs.clear();
  seen.clear();
  refused.clear();
}

GraphCache::~GraphCache() {
  clear();
  if (cap) {
    (void)hipStreamSynchronize(cap);
    (void)hipStreamDestroy(cap);
  }
}

}  // namespace rid

rid_context::~rid_context() {
  rid::ring_free(ring);
  ring = nullptr;
  rid::flush_graveyard(this);
  for (hipEvent_t e : grave_events) (void)hipEventDestroy(e);
}
