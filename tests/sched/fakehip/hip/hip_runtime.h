// CPU stand-in for the HIP host calls the library's scheduling code makes
// (test infrastructure only).  Streams are worker threads running their
// work in order; events complete when the stream reaches them; device
// memory is host memory.  It lets the real Batcher, buffer-release and
// server code run under ThreadSanitizer and AddressSanitizer on the CPU.
// Semantics kept from HIP: an event completes at its most recent record; a
// stream waiting on an event waits for the record made before the wait was
// enqueued; destroying an event or stream with work pending is allowed (the
// work still completes; a destroyed stream first drains).
#pragma once

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <functional>
#include <memory>
#include <mutex>
#include <set>
#include <thread>

#define __host__
#define __device__
#define __global__
#define __shared__
#define __forceinline__ inline

typedef int hipError_t;
enum { hipSuccess = 0, hipErrorInvalidValue = 1, hipErrorNotReady = 600 };
enum hipMemcpyKind { hipMemcpyHostToHost = 0, hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice,
                     hipMemcpyDefault };
#define hipEventDisableTiming 2u
#define hipStreamNonBlocking 1u
#define hipHostMallocDefault 0u

namespace fakehip {

typedef std::chrono::steady_clock Clock;

struct EventState {
  std::mutex mu;
  std::condition_variable cv;
  uint64_t recorded = 0, done = 0;
  Clock::time_point t{};
};

struct EventHandle {
  std::shared_ptr<EventState> s = std::make_shared<EventState>();
};

struct StreamImpl {
  std::mutex mu;
  std::condition_variable cv;
  std::deque<std::function<void()>> q;
  bool stop = false;
  std::thread th;
  StreamImpl() {
    th = std::thread([this] {
      std::unique_lock<std::mutex> lk(mu);
      while (true) {
        cv.wait(lk, [&] { return stop || !q.empty(); });
        if (q.empty()) return;
        std::function<void()> f = std::move(q.front());
        q.pop_front();
        lk.unlock();
        f();
        lk.lock();
      }
    });
  }
  void push(std::function<void()> f) {
    std::lock_guard<std::mutex> g(mu);
    q.push_back(std::move(f));
    cv.notify_all();
  }
  void drain() {
    std::mutex m;
    std::condition_variable c;
    bool hit = false;
    push([&] {
      std::lock_guard<std::mutex> g(m);
      hit = true;
      c.notify_all();
    });
    std::unique_lock<std::mutex> lk(m);
    c.wait(lk, [&] { return hit; });
  }
  ~StreamImpl() {
    {
      std::lock_guard<std::mutex> g(mu);
      stop = true;
      cv.notify_all();
    }
    th.join();
  }
};

inline StreamImpl* default_stream() {
  static StreamImpl* s = new StreamImpl();  // lives until the process ends
  return s;
}
inline std::mutex& reg_mu() {
  static std::mutex m;
  return m;
}
inline std::set<StreamImpl*>& registry() {
  static std::set<StreamImpl*> r;
  return r;
}
inline StreamImpl* resolve(StreamImpl* s) { return s ? s : default_stream(); }

}  // namespace fakehip

typedef fakehip::StreamImpl* hipStream_t;
typedef fakehip::EventHandle* hipEvent_t;

inline const char* hipGetErrorString(hipError_t) { return "fake HIP error"; }
inline hipError_t hipGetLastError() { return hipSuccess; }
inline hipError_t hipSetDevice(int) { return hipSuccess; }
inline hipError_t hipGetDevice(int* d) {
  *d = 0;
  return hipSuccess;
}
inline hipError_t hipMemGetInfo(size_t* free_b, size_t* total_b) {
  *free_b = (size_t)64 << 30;
  *total_b = (size_t)64 << 30;
  return hipSuccess;
}

inline hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) {
  *s = new fakehip::StreamImpl();
  std::lock_guard<std::mutex> g(fakehip::reg_mu());
  fakehip::registry().insert(*s);
  return hipSuccess;
}
inline hipError_t hipStreamDestroy(hipStream_t s) {
  if (!s) return hipErrorInvalidValue;
  {
    std::lock_guard<std::mutex> g(fakehip::reg_mu());
    fakehip::registry().erase(s);
  }
  s->drain();
  delete s;
  return hipSuccess;
}
inline hipError_t hipStreamSynchronize(hipStream_t s) {
  fakehip::resolve(s)->drain();
  return hipSuccess;
}
inline hipError_t hipDeviceSynchronize() {
  std::set<fakehip::StreamImpl*> all;
  {
    std::lock_guard<std::mutex> g(fakehip::reg_mu());
    all = fakehip::registry();
  }
  for (auto* s : all) s->drain();
  fakehip::default_stream()->drain();
  return hipSuccess;
}

inline hipError_t hipEventCreate(hipEvent_t* e) {
  *e = new fakehip::EventHandle();
  return hipSuccess;
}
inline hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { return hipEventCreate(e); }
inline hipError_t hipEventDestroy(hipEvent_t e) {
  delete e;  // pending work keeps the state alive through its shared pointer
  return hipSuccess;
}
inline hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
  std::shared_ptr<fakehip::EventState> st = e->s;
  uint64_t gen;
  {
    std::lock_guard<std::mutex> g(st->mu);
    gen = ++st->recorded;
  }
  fakehip::resolve(s)->push([st, gen] {
    std::lock_guard<std::mutex> g(st->mu);
    if (st->done < gen) st->done = gen;
    st->t = fakehip::Clock::now();
    st->cv.notify_all();
  });
  return hipSuccess;
}
inline hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned) {
  std::shared_ptr<fakehip::EventState> st = e->s;
  uint64_t gen;
  {
    std::lock_guard<std::mutex> g(st->mu);
    gen = st->recorded;
  }
  fakehip::resolve(s)->push([st, gen] {
    std::unique_lock<std::mutex> lk(st->mu);
    st->cv.wait(lk, [&] { return st->done >= gen; });
  });
  return hipSuccess;
}
inline hipError_t hipEventSynchronize(hipEvent_t e) {
  std::shared_ptr<fakehip::EventState> st = e->s;
  std::unique_lock<std::mutex> lk(st->mu);
  const uint64_t gen = st->recorded;
  st->cv.wait(lk, [&] { return st->done >= gen; });
  return hipSuccess;
}
inline hipError_t hipEventQuery(hipEvent_t e) {
  std::lock_guard<std::mutex> g(e->s->mu);
  return e->s->done >= e->s->recorded ? hipSuccess : hipErrorNotReady;
}
inline hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) {
  fakehip::Clock::time_point ta, tb;
  {
    std::lock_guard<std::mutex> g(a->s->mu);
    ta = a->s->t;
  }
  {
    std::lock_guard<std::mutex> g(b->s->mu);
    tb = b->s->t;
  }
  *ms = std::chrono::duration<float, std::milli>(tb - ta).count();
  return hipSuccess;
}

inline hipError_t hipMemcpyAsync(void* dst, const void* src, size_t n, hipMemcpyKind, hipStream_t s) {
  fakehip::resolve(s)->push([dst, src, n] { std::memcpy(dst, src, n); });
  return hipSuccess;
}
inline hipError_t hipHostMalloc(void** p, size_t n, unsigned) {
  *p = std::malloc(n);
  return *p ? hipSuccess : hipErrorInvalidValue;
}
inline hipError_t hipHostFree(void* p) {
  std::free(p);
  return hipSuccess;
}

// graphs: only created and destroyed by the code built here
typedef struct FakeGraph* hipGraph_t;
typedef struct FakeGraphExec* hipGraphExec_t;
inline hipError_t hipGraphDestroy(hipGraph_t) { return hipSuccess; }
inline hipError_t hipGraphExecDestroy(hipGraphExec_t) { return hipSuccess; }

// device intrinsics named in shared headers (never run on the CPU)
template <typename T>
inline T __shfl_xor(T v, int, int = 64) {
  return v;
}
