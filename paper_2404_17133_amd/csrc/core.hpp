// Host-side objects of the library: context, device buffers, problem and the
// operator driver.  Internal C++ (no exceptions cross the C ABI).
#pragma once

#include <map>
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
  bool on = false;
  std::vector<std::string> names;
  std::map<std::string, int> ids;
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  std::vector<Acc> acc;
  int family(const char* name);
  hipEvent_t get_event();
  void resolve();  // stream must be idle
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

}  // namespace rid

struct rid_context {
  int device = 0;
  hipStream_t stream = nullptr;
  rid_allocator alloc{};
  bool user_alloc = false;
  std::string last_error;
  std::mutex mu;  // guards allocator use from the server thread
  rid::Profiler prof;
  std::map<rid::TuneKey, rid::TuneVal> tune;
};

namespace rid {

// RAII bracket of one launch (no-op unless profiling is enabled).
struct ProfScope {
  rid_context* ctx;
  int fam = -1;
  hipEvent_t a = nullptr;
  double flops, bytes;
  ProfScope(rid_context* c, const char* name, double fl, double by);
  ~ProfScope();
};

}  // namespace rid

namespace rid {

void* dev_alloc(rid_context* ctx, size_t bytes);
void dev_free(rid_context* ctx, void* p);

// Owning device buffer from the context's allocator.
struct DevBuf {
  rid_context* ctx = nullptr;
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  explicit DevBuf(rid_context* c) : ctx(c) {}
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : ctx(o.ctx), p(o.p), bytes(o.bytes) { o.p = nullptr; o.bytes = 0; }
  ~DevBuf() { release(); }
  void release();
  // Grow to at least n bytes (contents are not preserved).
  void ensure(size_t n);
  template <typename T>
  T* as() const { return reinterpret_cast<T*>(p); }
};

// Reusable scratch for operator products (grown on demand, never shrunk).
struct OpWork {
  DevBuf xc, xa, xt, tpart, t64, jbuf, s, q, wpart, wppart;
  explicit OpWork(rid_context* c) : xc(c), xa(c), xt(c), tpart(c), t64(c), jbuf(c), s(c), q(c), wpart(c), wppart(c) {}
  size_t bytes() const {
    return xc.bytes + xa.bytes + xt.bytes + tpart.bytes + t64.bytes + jbuf.bytes + s.bytes + q.bytes + wpart.bytes +
           wppart.bytes;
  }
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
  int i0 = 0, no_a = 0, nv_a = 0;  // exchange window
  bool ris = false;                 // profiling family prefix
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
  // owned
  rid::DevBuf de, b_ai64, bris_ai64;
  rid::DevBuf b_ia32, b_ij32, b_ab32, b_ai32;
  rid::DevBuf bris_ia16, bris_ij16, bris_ab16, bris_ai16;
  rid::OpWork work;
  explicit rid_problem(rid_context* c)
      : ctx(c), de(c), b_ai64(c), bris_ai64(c), b_ia32(c), b_ij32(c), b_ab32(c), b_ai32(c), bris_ia16(c),
        bris_ij16(c), bris_ab16(c), bris_ai16(c), work(c) {}
  long n() const { return (long)no * nv; }
  uint64_t footprint() const;
  // lazily built copies
  void ensure_f64_aux();
  void ensure_f32();
  void ensure_bf16();
};

namespace rid {

// Operator kinds for apply().
enum OpKind { OPK_A = 0, OPK_PAIR = 1, OPK_T = 2, OPK_TPAIR = 3 };
enum Prec { PREC_F64 = 0, PREC_F32 = 1, PREC_BF16 = 2 };

// y (and y2 for the pair kinds) = op(x) for nvec vectors; x, y, y2 f64 device.
void apply_operator(rid_problem* P, int kind, int prec, int nvec, const double* x, double* y, double* y2);

// Validate (kind, prec) combinations; throws rid::Error.
void check_operator(const rid_problem* P, int kind, int prec);

}  // namespace rid
