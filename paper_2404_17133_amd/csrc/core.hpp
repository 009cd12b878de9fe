// Host-side objects of the library: context, device buffers, problem and the
// operator driver.  Internal C++ (no exceptions cross the C ABI).
#pragma once

#include <atomic>
#include <condition_variable>
#include <map>
#include <thread>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"

namespace rid {

// Event-bracketed launch timing per kernel family (enabled on demand).
struct Profiler {
  struct Rec {
    int fam;
    hipEvent_t a, b;
    double flops, bytes;
  };
  struct Acc {
    int64_t launches = 0;
    double ms = 0.0, flops = 0.0, bytes = 0.0;
  };
  std::atomic<bool> on{false};
  std::mutex mu;  // solves on several host threads share the profiler
  std::string only;  // when set, the one family recorded (guarded by mu)
  std::vector<std::string> names;
  std::map<std::string, int> ids;
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  std::vector<Acc> acc;
  int family(const char* name);   // caller holds mu
  hipEvent_t get_event();         // caller holds mu
  // Fold the records whose launches have completed into the totals (those
  // still running stay for a later call); safe while solves record.
  void resolve();
  // resolve(), then the totals of every family with launches, which are
  // reset; safe while solves record.
  std::vector<std::pair<std::string, Acc>> take();
  ~Profiler();
};

// Autotuner cache: launch shape -> chosen tile configuration and split plan.
struct TuneKey {
  int family, esz;
  long M, N;
  int nz, np, K;
  bool operator<(const TuneKey& o) const {
    if (family != o.family) return family < o.family;
    if (esz != o.esz) return esz < o.esz;
    if (M != o.M) return M < o.M;
    if (N != o.N) return N < o.N;
    if (nz != o.nz) return nz < o.nz;
    if (np != o.np) return np < o.np;
    return K < o.K;
  }
};
struct TuneVal {
  int cfg, nsub, pps;
};

struct DescRing;
class Batcher;
void ring_free(DescRing* r);  // deletes a descriptor ring (null allowed)
// Tuning decisions of a context to / from a text file (returns the count);
// a file of another build or device is refused with RID_ERR_INVALID_ARG.
int tune_save(rid_context* ctx, const char* path);
int tune_load(rid_context* ctx, const char* path);

}  // namespace rid

struct rid_context {
  int device = 0;
  hipStream_t stream = nullptr;
  rid_allocator alloc{};  // every device buffer of the library comes from here
  std::string last_error;
  std::mutex mu;  // guards allocator use from several host threads
  rid::Profiler prof;
  std::mutex tune_mu;
  std::map<rid::TuneKey, rid::TuneVal> tune;
  // While solves run on several streams (batched solves, the server), a
  // freed device buffer is parked with an event recorded on the releasing
  // thread's stream, and handed back to the allocator once that event has
  // completed (every earlier use of the buffer is ordered before it).
  struct Parked {
    void* p;
    size_t bytes;
    hipEvent_t ev;
  };
  int defer_free = 0;  // nesting count, guarded by grave_mu
  std::mutex grave_mu;
  std::vector<Parked> graveyard;
  std::vector<hipEvent_t> grave_events;  // recycled
  uint64_t grave_bytes = 0;
  rid::DescRing* ring = nullptr;  // grouped-GEMM descriptor staging
  void* scratch = nullptr;  // device address of this device's fixed scratch (rid_apply_operator_noalloc)
  ~rid_context();
};

namespace rid {

// RAII bracket of one launch (no-op unless profiling is enabled).
struct ProfScope {
  rid_context* ctx;
  hipStream_t st;
  int fam = -1;
  hipEvent_t a = nullptr;
  double flops, bytes;
  ProfScope(rid_context* c, hipStream_t s, const char* name, double fl, double by);
  ~ProfScope();
};

}  // namespace rid

namespace rid {

void* dev_alloc(rid_context* ctx, size_t bytes);
void dev_free(rid_context* ctx, void* p);
// Release parked buffers whose fence events have completed; with wait, wait
// for all of them first.
void reap_graveyard(rid_context* ctx, bool wait);
inline void flush_graveyard(rid_context* ctx) { reap_graveyard(ctx, true); }
// The stream whose position fences this host thread's buffer releases: a
// solve's thread sets its stream, a batcher lane thread its lane stream.
hipStream_t thread_stream();
struct ThreadStream {
  hipStream_t prev;
  explicit ThreadStream(hipStream_t s);
  ~ThreadStream();
};
// Scope in which buffer releases are deferred (see rid_context::graveyard).
struct DeferFree {
  rid_context* ctx;
  explicit DeferFree(rid_context* c);
  ~DeferFree();
};

// A fixed device region handed out front to back (never freed piecewise):
// the scratch of an operator product that may not allocate.
struct Arena {
  char* base = nullptr;
  size_t cap = 0, used = 0;
  void* take(size_t n);  // throws RID_ERR_SHAPE when the region is exhausted
};

// Owning device buffer from the context's allocator, or (with an arena) a
// slice of a fixed region that is never returned.
struct DevBuf {
  rid_context* ctx = nullptr;
  Arena* arena = nullptr;
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  explicit DevBuf(rid_context* c) : ctx(c) {}
  explicit DevBuf(Arena* a) : arena(a) {}
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : ctx(o.ctx), arena(o.arena), p(o.p), bytes(o.bytes) {
    o.p = nullptr;
    o.bytes = 0;
  }
  ~DevBuf() { release(); }
  void release();
  // Grow to at least n bytes (contents are not preserved).
  void ensure(size_t n);
  template <typename T>
  T* as() const { return reinterpret_cast<T*>(p); }
};

// Reusable scratch for operator products (grown on demand, never shrunk).
struct OpWork {
  DevBuf xc, xa, xt, tpart, t64, jbuf, jpart, s, q, wpart, wppart;
  explicit OpWork(rid_context* c)
      : xc(c), xa(c), xt(c), tpart(c), t64(c), jbuf(c), jpart(c), s(c), q(c), wpart(c), wppart(c) {}
  explicit OpWork(Arena* a)
      : xc(a), xa(a), xt(a), tpart(a), t64(a), jbuf(a), jpart(a), s(a), q(a), wpart(a), wppart(a) {}
  size_t bytes() const {
    return xc.bytes + xa.bytes + xt.bytes + tpart.bytes + t64.bytes + jbuf.bytes + jpart.bytes + s.bytes + q.bytes +
           wpart.bytes + wppart.bytes;
  }
  std::vector<void*> addresses() const {
    return {xc.p, xa.p, xt.p, tpart.p, t64.p, jbuf.p, jpart.p, s.p, q.p, wpart.p, wppart.p};
  }
};

// An operator product of a single solve captured as a HIP graph: it reads
// its input from and writes its outputs to staging buffers of its own, and
// is replayed whenever the problem's solves ask for the same product shape
// (kind, precision, block width) again.  The scratch it was captured with
// is recorded: when the problem's scratch has been reallocated since, the
// graph is captured anew.
struct OpGraph {
  int kind = 0, prec = 0, nvec = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  DevBuf x, y, y2;
  std::vector<void*> work;  // addresses of the scratch buffers at capture
  explicit OpGraph(rid_context* c) : x(c), y(c), y2(c) {}
  OpGraph(const OpGraph&) = delete;
  OpGraph& operator=(const OpGraph&) = delete;
  ~OpGraph();
};

struct GraphCache {
  std::vector<OpGraph*> graphs;
  std::vector<long> seen;      // shapes run once without a graph (their GEMM shapes tuned)
  std::vector<long> refused;   // shapes whose capture failed: always run directly
  hipStream_t cap = nullptr;   // capture stream
  GraphCache() = default;
  GraphCache(const GraphCache&) = delete;
  GraphCache& operator=(const GraphCache&) = delete;
  void clear();
  ~GraphCache();
};

// A view of one three-index tensor in element type E, as one operator uses it.
template <typename E>
struct OpView {
  const E* b_ia = nullptr;  // (naux_j, no, nv)
  const E* b_ij = nullptr;  // (>= naux_k, no, no)
  const E* b_ab = nullptr;  // (>= naux_k, nv, nv)
  const E* b_ai = nullptr;  // (>= naux_k, nv, no): b_ia transposed per slice
  int naux_j = 0;           // rows in the Coulomb part
  int naux_k = 0;           // leading rows in the exchange part
  // long-range exchange tensor of a range-separated hybrid (naux_lr rows)
  const E *lr_ia = nullptr, *lr_ij = nullptr, *lr_ab = nullptr, *lr_ai = nullptr;
  int naux_lr = 0;
  double ax = 0.0, bx = 0.0;        // weights of the two exchange parts
  int i0 = 0, no_a = 0, nv_a = 0;  // exchange window
  bool ris = false;                 // profiling family prefix
};

// Long-range exchange tensor C of a range-separated hybrid, borrowed in FP64
// or FP32, with the copies the products read (transposes, casts).
struct LrSet {
  int rows = 0;
  int dt = RID_F64;
  const double *ia = nullptr, *ij = nullptr, *ab = nullptr;
  const float *ia_f = nullptr, *ij_f = nullptr, *ab_f = nullptr;
  DevBuf ai64, ia32, ij32, ab32, ai32, ia16, ij16, ab16, ai16;
  explicit LrSet(rid_context* c)
      : ai64(c), ia32(c), ij32(c), ab32(c), ai32(c), ia16(c), ij16(c), ab16(c), ai16(c) {}
  size_t bytes() const {
    return ai64.bytes + ia32.bytes + ij32.bytes + ab32.bytes + ai32.bytes + ia16.bytes + ij16.bytes + ab16.bytes +
           ai16.bytes;
  }
  const float* ia32v() const { return dt == RID_F32 ? ia_f : ia32.as<float>(); }
  const float* ij32v() const { return dt == RID_F32 ? ij_f : ij32.as<float>(); }
  const float* ab32v() const { return dt == RID_F32 ? ab_f : ab32.as<float>(); }
};

}  // namespace rid

struct rid_problem {
  rid_context* ctx = nullptr;
  int no = 0, nv = 0, naux = 0, naux_ris = 0, naux_ris_k = 0;
  double a_x = 0.0, t_cut = 0.0;
  int i0 = 0, nv_act = 0;  // exchange window of the ris model
  std::vector<double> eps_occ, eps_vir;
  double de_min = 0.0;
  // borrowed f64 tensors
  const double *b_ia = nullptr, *b_ij = nullptr, *b_ab = nullptr;
  const double *bris_ia = nullptr, *bris_ij = nullptr, *bris_ab = nullptr;
  // borrowed f32 tensors (b_dtype / bris_dtype RID_F32 instead of the f64 ones)
  int b_dt = RID_F64, bris_dt = RID_F64;
  const float *b_ia_f = nullptr, *b_ij_f = nullptr, *b_ab_f = nullptr;
  const float *bris_ia_f = nullptr, *bris_ij_f = nullptr, *bris_ab_f = nullptr;
  bool has_ris() const { return naux_ris > 0 && (bris_ia || bris_ia_f); }
  std::mutex mu;  // guards the lazily built copies
  // owned
  rid::DevBuf de, b_ai64, bris_ai64;
  rid::DevBuf b_ia32, b_ij32, b_ab32, b_ai32;
  rid::DevBuf bris_ia16, bris_ij16, bris_ab16, bris_ai16;
  rid::OpWork work;
  rid::GraphCache graphs;  // captured operator products of single solves (declared after work: freed first)
  // range-separated hybrid: exchange a_x (pq|rs) + b_x (pq|rs)^LR
  double b_x = 0.0;
  rid::LrSet lr, rislr;
  explicit rid_problem(rid_context* c)
      : ctx(c), de(c), b_ai64(c), bris_ai64(c), b_ia32(c), b_ij32(c), b_ab32(c), b_ai32(c), bris_ia16(c),
        bris_ij16(c), bris_ab16(c), bris_ai16(c), work(c), lr(c), rislr(c) {}
  long n() const { return (long)no * nv; }
  uint64_t footprint() const;
  // lazily built copies
  void ensure_f64_aux();
  void ensure_f32();
  void ensure_bf16();
  // f32 views of the full tensors (borrowed or cast copies; ensure_f32 first)
  const float* ia32() const { return b_dt == RID_F32 ? b_ia_f : b_ia32.as<float>(); }
  const float* ij32() const { return b_dt == RID_F32 ? b_ij_f : b_ij32.as<float>(); }
  const float* ab32() const { return b_dt == RID_F32 ? b_ab_f : b_ab32.as<float>(); }
};

namespace rid {

// Operator kinds for apply().
enum OpKind { OPK_A = 0, OPK_PAIR = 1, OPK_T = 2, OPK_TPAIR = 3 };
enum Prec { PREC_F64 = 0, PREC_F32 = 1, PREC_BF16 = 2 };

// y (and y2 for the pair kinds) = op(x) for nvec vectors; x, y, y2 f64 device.
// Runs on the context stream with the problem's own scratch.
void apply_operator(rid_problem* P, int kind, int prec, int nvec, const double* x, double* y, double* y2);

// Limits of a product whose scratch is a fixed region: exchange chunks of
// at most chunk_bytes of intermediate, at most max_splits partial sums per
// reduction, no autotuning (the default tile rule; results differ from a
// tuned product only by the rounding of the split sums), no profiling
// events, no host synchronisation.
struct OpLimits {
  long chunk_bytes;
  int max_splits;
};

// apply_operator with every scratch buffer carved from `arena` (nothing is
// allocated) under `lim`.  The problem's tensor copies for this operator and
// precision must exist already (RID_ERR_INVALID_ARG otherwise); a region too
// small gives RID_ERR_SHAPE before any kernel is launched.  Enqueued on the
// context stream; returns without waiting.
void apply_operator_fixed(rid_problem* P, int kind, int prec, int nvec, const double* x, double* y, double* y2,
                          Arena& arena, const OpLimits& lim);

// Whether the tensor copies that products of (kind, prec) read already exist.
bool operator_copies_ready(const rid_problem* P, int kind, int prec);

// One operator product request.
struct OpJob {
  rid_problem* P = nullptr;
  int kind = 0, prec = 0, nvec = 0;
  const double* x = nullptr;
  double* y = nullptr;
  double* y2 = nullptr;
  OpWork* work = nullptr;       // scratch of the requesting solve
  hipStream_t stream = nullptr; // stream of the requesting solve
  // set by the Batcher
  hipEvent_t ready = nullptr;
  bool finished = false;
  int code = 0;
  std::string msg;
};

// Run the products of several jobs on stream st.  Every GEMM stage of all
// jobs goes out as one grouped launch per tile configuration; each job's
// result is what it would be alone.  Jobs must have been checked.
void run_jobs(rid_context* ctx, OpJob* const* jobs, int n, hipStream_t st, const OpLimits* lim = nullptr);

// Collects operator products from solves running on several host threads
// and streams, and runs whatever is waiting as one grouped product on a
// stream of its own, from a thread of its own.  Two lanes, each with its own
// thread and stream: the outer products, and the small ris-model products of
// the inner solves, so that an inner iteration does not wait behind a round
// of large outer products.  apply() returns once the product is enqueued: the
// caller's stream waits for it with an event.
class Batcher {
 public:
  explicit Batcher(rid_context* ctx);
  ~Batcher();
  void apply(OpJob& j);  // throws rid::Error when the product failed
  int64_t rounds() const { return lanes_[0].rounds + lanes_[1].rounds; }
  int64_t jobs() const { return lanes_[0].jobs + lanes_[1].jobs; }

 private:
  struct Lane {
    hipStream_t st = nullptr;
    std::condition_variable cv;
    std::vector<OpJob*> pending;
    int64_t rounds = 0, jobs = 0;
    std::vector<hipEvent_t> events;
    int next_event = 0;
    std::thread thread;
  };
  void loop(Lane& L);
  rid_context* ctx_;
  std::mutex mu_;
  std::condition_variable cv_done_;
  bool stop_ = false;
  Lane lanes_[2];
};

// Validate (kind, prec) combinations; throws rid::Error.
void check_operator(const rid_problem* P, int kind, int prec);

// Build the problem's lazily made tensor copies that solves with options o
// read (FP32 casts and transposes for the mixed path, BF16 ris copies, FP64
// transposes), so that their memory is in place before solves are admitted.
void prepare_problem(rid_problem* P, const rid_solve_opts& o);

}  // namespace rid
