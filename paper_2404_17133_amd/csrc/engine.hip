// Krylov solvers: Davidson for TDA (Eq. TDA) and full TDDFT (Eq. Casida), the
// inner Krylov solve of the preconditioning step (Eq. precondition) with the
// ris model, the ris initial guesses, and the polarizability linear solve
// (Eq. TDDFT_polar).
//
// The host drives one HIP stream.  Each outer iteration reads back only a few
// scalars (Ritz values, residual norms, Gram-Schmidt norms); every vector
// operation, the operator products, the projections and the small dense
// problems run on the device.
//
// Readings of the paper taken here (shared with the CPU reference the tests
// compare against):
//  * Gram-Schmidt: unit-normalise, project out the basis twice, then the
//    already accepted new directions twice, drop below 1e-8 (a block whose
//    directions stay well apart after the first step is orthonormalised
//    within itself by two Cholesky-QR passes instead, which spans the same
//    space and drops nothing);
//  * diagonal preconditioner: de = eps_a - eps_i, denominators guarded at
//    +-1e-8;
//  * inner solve: block Galerkin over a shared subspace, unit-normalised
//    right-hand sides, expansion by diagonally preconditioned inner
//    residuals, stop at ||rho|| < inner_tol or inner_max_iter products;
//  * full TDDFT: one subspace for Z = X+Y and Z' = X-Y, Cholesky of the
//    projected A-B, eigenpairs of L^T a_+ L, z^T z' = 1;
//  * N_init = k + min(k, 3) (ris) or k + 8 (diagonal), Sec. 3.2.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <memory>
#include <numeric>

#include "engine.hpp"
#include "engkern.hpp"

namespace rid {
namespace {

typedef std::chrono::steady_clock Clock;

double ms_since(Clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
}

// Per-solve device context: stream, scratch, transfers and operator products.
struct Eng {
  ThreadStream fence;  // first member: fences buffer releases until the last member is gone
  rid_problem* P;
  hipStream_t st;
  long N;
  DevBuf part, tmp1, tmp2, ints, dscal;
  SolveStats* stats;
  uint64_t live = 0;
  Batcher* batcher;
  OpWork own;     // operator scratch of a solve that shares the device
  hipEvent_t ready = nullptr;
  // timing of the outer products: event pairs read once the solve has
  // synchronised anyway, so that no product waits for the host
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> mv_ev;
  Eng(rid_problem* p, SolveStats* s, const ExecCfg& ex)
      : fence(ex.stream ? ex.stream : p->ctx->stream), P(p), st(ex.stream ? ex.stream : p->ctx->stream), N(p->n()), part(p->ctx), tmp1(p->ctx), tmp2(p->ctx),
        ints(p->ctx), dscal(p->ctx), stats(s), batcher(ex.batcher), own(p->ctx) {
    if (batcher) RID_HIP(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
  }
  ~Eng() {
    if (ready || !ev_pool.empty() || !mv_ev.empty()) (void)hipStreamSynchronize(st);
    if (ready) (void)hipEventDestroy(ready);
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    for (auto& pr : mv_ev) {
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
  }
  hipEvent_t get_event() {
    if (!ev_pool.empty()) {
      hipEvent_t e = ev_pool.back();
      ev_pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    RID_HIP(hipEventCreate(&e));
    return e;
  }
  // Device time of the outer products recorded so far (ms); waits for them.
  double take_product_ms() {
    double t = 0.0;
    for (auto& pr : mv_ev) {
      RID_HIP(hipEventSynchronize(pr.second));
      float ms = 0.0f;
      RID_HIP(hipEventElapsedTime(&ms, pr.first, pr.second));
      t += ms;
      ev_pool.push_back(pr.first);
      ev_pool.push_back(pr.second);
    }
    mv_ev.clear();
    return t;
  }
  Eng(const Eng&) = delete;
  Eng& operator=(const Eng&) = delete;
  // y (, y2) = op(x) for nvec vectors, ordered on the solve's stream
  void apply(int kind, int prec, int nvec, const double* x, double* y, double* y2) {
    check_operator(P, kind, prec);
    if (nvec <= 0) return;
    OpJob j;
    j.P = P;
    j.kind = kind;
    j.prec = prec;
    j.nvec = nvec;
    j.x = x;
    j.y = y;
    j.y2 = y2;
    j.stream = st;
    if (batcher) {
      j.work = &own;
      j.ready = ready;
      batcher->apply(j);
    } else if (!(use_graphs && graph_apply(kind, prec, nvec, x, y, y2))) {
      j.work = &P->work;
      OpJob* jp = &j;
      run_jobs(P->ctx, &jp, 1, st);
    }
  }
  // Replay (or capture, then replay) the product as a graph; false when
  // the product has to run directly: the shape's first product (which sizes
  // the scratch and tunes its GEMM shapes, so that the capture neither
  // allocates nor times anything), profiling on, or a capture that failed.
  bool use_graphs = false;
  bool graph_apply(int kind, int prec, int nvec, const double* x, double* y, double* y2) {
    rid_context* ctx = P->ctx;
    if (ctx->prof.on) return false;
    GraphCache& G = P->graphs;
    const long key = ((long)kind * 4 + prec) * (1L << 24) + nvec;
    if (std::find(G.refused.begin(), G.refused.end(), key) != G.refused.end()) return false;
    OpGraph* g = nullptr;
    for (OpGraph* h : G.graphs)
      if (h->kind == kind && h->prec == prec && h->nvec == nvec) g = h;
    if (g && g->work != P->work.addresses()) {
      // the scratch was reallocated since the capture: capture again
      G.graphs.erase(std::find(G.graphs.begin(), G.graphs.end(), g));
      RID_HIP(hipStreamSynchronize(st));
      delete g;
      g = nullptr;
    }
    if (!g) {
      if (std::find(G.seen.begin(), G.seen.end(), key) == G.seen.end()) {
        G.seen.push_back(key);
        return false;
      }
      if (!G.cap) RID_HIP(hipStreamCreateWithFlags(&G.cap, hipStreamNonBlocking));
      const bool pair = kind == OPK_PAIR || kind == OPK_TPAIR;
      std::unique_ptr<OpGraph> ng(new OpGraph(ctx));
      ng->kind = kind;
      ng->prec = prec;
      ng->nvec = nvec;
      ng->x.ensure(sizeof(double) * (size_t)nvec * N);
      ng->y.ensure(sizeof(double) * (size_t)nvec * N);
      if (pair) ng->y2.ensure(sizeof(double) * (size_t)nvec * N);
      const std::vector<void*> before = P->work.addresses();
      OpJob j;
      j.P = P;
      j.kind = kind;
      j.prec = prec;
      j.nvec = nvec;
      j.x = ng->x.as<double>();
      j.y = ng->y.as<double>();
      j.y2 = pair ? ng->y2.as<double>() : nullptr;
      j.stream = G.cap;
      j.work = &P->work;
      OpJob* jp = &j;
      bool ok = hipStreamBeginCapture(G.cap, hipStreamCaptureModeThreadLocal) == hipSuccess;
      if (ok) {
        try {
          run_jobs(ctx, &jp, 1, G.cap);
        } catch (const Error&) {
          ok = false;
        }
        hipGraph_t graph = nullptr;
        const hipError_t e = hipStreamEndCapture(G.cap, &graph);
        ng->graph = graph;
        ok = ok && e == hipSuccess && graph != nullptr && P->work.addresses() == before;
        if (ok) ok = hipGraphInstantiate(&ng->exec, ng->graph, nullptr, nullptr, 0) == hipSuccess;
      }
      if (!ok) {
        (void)hipGetLastError();
        G.refused.push_back(key);
        return false;
      }
      ng->work = P->work.addresses();
      g = ng.release();
      G.graphs.push_back(g);
    }
    const size_t bytes = sizeof(double) * (size_t)nvec * N;
    RID_HIP(hipMemcpyAsync(g->x.p, x, bytes, hipMemcpyDeviceToDevice, st));
    RID_HIP(hipGraphLaunch(g->exec, st));
    RID_HIP(hipMemcpyAsync(y, g->y.p, bytes, hipMemcpyDeviceToDevice, st));
    if (y2) RID_HIP(hipMemcpyAsync(y2, g->y2.p, bytes, hipMemcpyDeviceToDevice, st));
    return true;
  }
  RedScratch rs(int m, int n) {
    size_t need = std::max(gram_part_elems(m, n, N), (size_t)256 * std::max(n, 1));
    need = std::max(need, (size_t)256 * std::max(m, 1));
    part.ensure(need * sizeof(double));
    return RedScratch{part.as<double>(), part.bytes / sizeof(double)};
  }
  void sync() { RID_HIP(hipStreamSynchronize(st)); }
  void d2h(void* h, const void* d, size_t bytes) {
    RID_HIP(hipMemcpyAsync(h, d, bytes, hipMemcpyDeviceToHost, st));
    sync();
  }
  void h2d(void* d, const void* h, size_t bytes) {
    RID_HIP(hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, st));
    sync();  // h may be a stack temporary
  }
  // device copy of a small host double array (kept in dscal at offset slot)
  const double* put_doubles(DevBuf& buf, const std::vector<double>& v) {
    buf.ensure(std::max<size_t>(1, v.size()) * sizeof(double));
    if (!v.empty()) h2d(buf.p, v.data(), v.size() * sizeof(double));
    return buf.as<double>();
  }
  const int* put_ints(DevBuf& buf, const std::vector<int>& v) {
    buf.ensure(std::max<size_t>(1, v.size()) * sizeof(int));
    if (!v.empty()) h2d(buf.p, v.data(), v.size() * sizeof(int));
    return buf.as<int>();
  }
  void track(uint64_t b) {
    live = b;
    if (stats && b > stats->peak_bytes) stats->peak_bytes = b;
  }
};

// A Krylov subspace with up to two operator products per vector and the
// matching projected matrices.
struct Basis {
  int cap = 0, m = 0, nprod = 1;
  long N = 0;
  DevBuf v, p1, p2, a1, a2;
  Basis(rid_context* c) : v(c), p1(c), p2(c), a1(c), a2(c) {}
  void init(int capacity, long n, int np) {
    cap = capacity;
    N = n;
    nprod = np;
    m = 0;
    v.ensure(sizeof(double) * (size_t)cap * N);
    p1.ensure(sizeof(double) * (size_t)cap * N);
    a1.ensure(sizeof(double) * (size_t)cap * cap);
    if (np == 2) {
      p2.ensure(sizeof(double) * (size_t)cap * N);
      a2.ensure(sizeof(double) * (size_t)cap * cap);
    }
  }
  double* V(int j) { return v.as<double>() + (long)j * N; }
  double* P1(int j) { return p1.as<double>() + (long)j * N; }
  double* P2(int j) { return p2.as<double>() + (long)j * N; }
  uint64_t bytes() const { return v.bytes + p1.bytes + p2.bytes + a1.bytes + a2.bytes; }
};

// Copies columns n (length N, stride N) of src to dst for every n with
// done[n] == 0, one copy per run of consecutive such columns.
void copy_open_columns(const std::vector<char>& done, const double* src, double* dst, long N, hipStream_t st) {
  const int nr = (int)done.size();
  for (int n = 0; n < nr;) {
    if (done[n]) {
      ++n;
      continue;
    }
    int e = n + 1;
    while (e < nr && !done[e]) ++e;
    RID_HIP(hipMemcpyAsync(dst + (long)n * N, src + (long)n * N, sizeof(double) * (size_t)(e - n) * N,
                           hipMemcpyDeviceToDevice, st));
    n = e;
  }
}

// Orthonormalise nnew directions W (row-major, ld N; overwritten) against the
// basis and each other, append the accepted ones.  Returns the number added.
// Every step runs on the device.  After the projection against the basis,
// the block is orthonormalised within itself by one of two routes:
//  * Cholesky QR, twice: G = W^T W = L L^T, W <- W L^{-T}, repeated on the
//    result.  Taken when every Cholesky pivot of the first pass is at least
//    kCholQrMinPivot (each direction keeps at least that fraction of its
//    length against the ones before it): then the first pass is accurate
//    to about (n / kCholQrMinPivot)^2 * eps and the second restores full
//    orthonormality.  No direction is dropped.  A handful of launches for
//    the whole block.
//  * otherwise modified Gram-Schmidt, twice per direction, with the drop
//    test: direction j is written to basis slot m0 + j (zero when dropped),
//    the host reads the norms once, at the end, and then closes the gaps
//    left by dropped directions.
// Both give the Q of the QR factorisation of the projected block (the same
// in exact arithmetic); only the second can drop.
constexpr double kCholQrMinPivot = 1e-3;

bool block_cholqr2(Eng& E, Basis& B, double* W, int n, const double* nrm_d) {
  const long N = E.N;
  const int m0 = B.m;
  E.tmp2.ensure(sizeof(double) * (size_t)(2 * n * n + 2 * n + 8));
  E.ints.ensure(sizeof(int) * 2);
  double* G = E.tmp2.as<double>();
  double* Li = G + (size_t)n * n;
  double* chk = Li + (size_t)n * n;  // diag(L), initial norms, info
  int* info = E.ints.as<int>();
  {
    RedScratch rs = E.rs(n, n);
    gram(W, N, n, W, N, n, N, G, n, rs, E.st);
  }
  small_chol(G, n, n, info, E.st);
  chol_check_pack(G, n, n, nrm_d, info, chk, E.st);
  std::vector<double> hc(2 * (size_t)n + 1);
  E.d2h(hc.data(), chk, sizeof(double) * hc.size());
  if (hc[2 * n] != 0.0) return false;
  for (int j = 0; j < n; ++j) {
    const double d = hc[j], nj = hc[n + j];
    if (!std::isfinite(nj) || nj == 0.0 || !std::isfinite(d) || !(d >= kCholQrMinPivot)) return false;
  }
  // first pass into the basis slots, second pass back into W, then copy
  small_trinv_lower(G, n, n, Li, n, E.st);
  combo(W, N, n, Li, 1, n, n, N, 1.0, 0.0, B.V(m0), N, E.st);  // T_j = sum_i L^{-1}[j][i] W_i
  {
    RedScratch rs = E.rs(n, n);
    gram(B.V(m0), N, n, B.V(m0), N, n, N, G, n, rs, E.st);
  }
  small_chol(G, n, n, info, E.st);
  small_trinv_lower(G, n, n, Li, n, E.st);
  combo(B.V(m0), N, n, Li, 1, n, n, N, 1.0, 0.0, W, N, E.st);
  RID_HIP(hipMemcpyAsync(B.V(m0), W, sizeof(double) * (size_t)n * N, hipMemcpyDeviceToDevice, E.st));
  B.m = m0 + n;
  return true;
}

int append_orthonormal(Eng& E, Basis& B, double* W, int nnew, double drop_tol = 1e-8) {
  if (nnew <= 0) return 0;
  ProfScope ps(E.P->ctx, E.st, "orthonormalize", 0.0, 0.0);
  const long N = E.N;
  RID_CHECK(B.m + nnew <= B.cap, RID_ERR_INTERNAL, "basis capacity exceeded");
  E.tmp1.ensure(sizeof(double) * (size_t)(2 * nnew + 64));
  double* nrm_d = E.tmp1.as<double>();       // initial norms
  double* fin_d = nrm_d + nnew;               // norms after orthogonalisation
  {
    RedScratch rs = E.rs(1, nnew);
    col_norms(W, N, nnew, N, nrm_d, rs, E.st);
  }
  scale_cols(W, N, nnew, N, nrm_d, 1, E.st);  // unit vectors (zero stays zero)
  if (B.m > 0) {
    E.tmp2.ensure(sizeof(double) * (size_t)B.m * nnew);
    double* c = E.tmp2.as<double>();
    for (int pass = 0; pass < 2; ++pass) {
      RedScratch rs = E.rs(B.m, nnew);
      gram(B.V(0), N, B.m, W, N, nnew, N, c, nnew, rs, E.st);
      combo(B.V(0), N, B.m, c, nnew, 1, nnew, N, -1.0, 1.0, W, N, E.st);
    }
  }
  const int m0 = B.m;
  if (nnew >= 2 && block_cholqr2(E, B, W, nnew, nrm_d)) {
    if (E.stats) ++E.stats->n_blocks_cholqr;
    return nnew;
  }
  if (nnew >= 2 && E.stats) ++E.stats->n_blocks_mgs;
  E.tmp2.ensure(sizeof(double) * (size_t)(nnew + 8));
  double* c = E.tmp2.as<double>();
  for (int j = 0; j < nnew; ++j) {
    double* wj = W + (long)j * N;
    if (j > 0) {
      for (int pass = 0; pass < 2; ++pass) {
        RedScratch rs = E.rs(j, 1);
        gram(B.V(m0), N, j, wj, N, 1, N, c, 1, rs, E.st);
        combo(B.V(m0), N, j, c, 1, 1, 1, N, -1.0, 1.0, wj, N, E.st);
      }
    }
    {
      RedScratch rs = E.rs(1, 1);
      col_norms(wj, N, 1, N, fin_d + j, rs, E.st);
    }
    accept_scale(wj, N, fin_d + j, drop_tol, B.V(m0 + j), E.st);
  }
  std::vector<double> nrm(2 * nnew);
  E.d2h(nrm.data(), nrm_d, sizeof(double) * 2 * nnew);
  int pos = m0;
  for (int j = 0; j < nnew; ++j) {
    const bool ok = std::isfinite(nrm[j]) && nrm[j] != 0.0 && nrm[nnew + j] >= drop_tol;
    if (!ok) continue;
    if (pos != m0 + j)
      RID_HIP(hipMemcpyAsync(B.V(pos), B.V(m0 + j), sizeof(double) * N, hipMemcpyDeviceToDevice, E.st));
    ++pos;
  }
  B.m = pos;
  return B.m - m0;
}

// Products of the new basis vectors [m0, m) with the operator.
// t_acc: null for products that are not timed (the inner ones).  A solve
// alone on its stream brackets the product with events (read later by
// take_product_ms, no wait here); one that shares the device counts the
// submission time.
void multiply(Eng& E, Basis& B, int m0, int kind, int prec, double* t_acc) {
  const int nn = B.m - m0;
  if (nn <= 0) return;
  if (!t_acc) {
    E.apply(kind, prec, nn, B.V(m0), B.P1(m0), B.nprod == 2 ? B.P2(m0) : nullptr);
    return;
  }
  if (E.batcher) {
    auto t0 = Clock::now();
    E.apply(kind, prec, nn, B.V(m0), B.P1(m0), B.nprod == 2 ? B.P2(m0) : nullptr);
    *t_acc += ms_since(t0);
    return;
  }
  // the pair goes back to the pool if the product throws
  struct Pair {
    Eng& E;
    hipEvent_t a, b;
    bool used = false;
    ~Pair() {
      if (!used) {
        E.ev_pool.push_back(a);
        E.ev_pool.push_back(b);
      }
    }
  } pr{E, E.get_event(), E.get_event()};
  RID_HIP(hipEventRecord(pr.a, E.st));
  E.apply(kind, prec, nn, B.V(m0), B.P1(m0), B.nprod == 2 ? B.P2(m0) : nullptr);
  RID_HIP(hipEventRecord(pr.b, E.st));
  E.mv_ev.emplace_back(pr.a, pr.b);
  pr.used = true;
}

// Update the projected matrices with the columns [m0, m).
void project(Eng& E, Basis& B, int m0) {
  const int m = B.m, nn = m - m0;
  if (nn <= 0) return;
  const long N = E.N;
  ProfScope ps(E.P->ctx, E.st, "project", 4.0 * m * nn * (double)N * B.nprod, 8.0 * 2 * (m + nn) * (double)N * B.nprod);
  DevBuf c1(E.P->ctx), c2(E.P->ctx);
  c1.ensure(sizeof(double) * (size_t)m * nn);
  c2.ensure(sizeof(double) * (size_t)m * nn);
  for (int q = 0; q < B.nprod; ++q) {
    double* prod = q == 0 ? B.P1(0) : B.P2(0);
    double* a = q == 0 ? B.a1.as<double>() : B.a2.as<double>();
    RedScratch rs = E.rs(m, nn);
    gram(B.V(0), N, m, prod + (long)m0 * N, N, nn, N, c1.as<double>(), nn, rs, E.st);
    gram(prod, N, m, B.V(m0), N, nn, N, c2.as<double>(), nn, rs, E.st);
    proj_update(a, B.cap, m, m0, c1.as<double>(), c2.as<double>(), E.st);
  }
}

// Stable argsort of de (host copy) -> positions of the `count` smallest.
std::vector<int> smallest_positions(const rid_problem* P, int count) {
  const long N = P->n();
  std::vector<double> de(N);
  for (int i = 0; i < P->no; ++i)
    for (int a = 0; a < P->nv; ++a) de[(long)i * P->nv + a] = P->eps_vir[a] - P->eps_occ[i];
  std::vector<int> idx(N);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return de[x] < de[y]; });
  idx.resize(std::min<long>(count, N));
  return idx;
}

int default_m_max(int k, int m_max) { return m_max > 0 ? m_max : std::max(200, 40 * k); }

// ---------------------------------------------------------------------------
// Small dense steps of one Rayleigh-Ritz iteration.
// ---------------------------------------------------------------------------
struct Ritz {
  DevBuf acopy, w, q, work, lmat, t1, mmat, zc, zpc, om, info;
  int ldq = 0;  // leading dimension of q (the number of eigenpairs computed)
  Ritz(rid_context* c) : acopy(c), w(c), q(c), work(c), lmat(c), t1(c), mmat(c), zc(c), zpc(c), om(c), info(c) {}
};

// TDA: the nq lowest eigenpairs of a (m x m) -> w (device, nq), q (device,
// m x nq, ld R.ldq = nq).
void ritz_sym(Eng& E, Ritz& R, Basis& B, int nq) {
  const int m = B.m;
  nq = std::max(1, std::min(nq, m));
  R.acopy.ensure(sizeof(double) * (size_t)m * m);
  R.w.ensure(sizeof(double) * nq);
  R.q.ensure(sizeof(double) * (size_t)m * nq);
  R.work.ensure(sizeof(double) * small_syevx_work(m, nq));
  R.ldq = nq;
  ProfScope ps(E.P->ctx, E.st, "small_dense", 0.0, 0.0);
  copy_block(B.a1.as<double>(), B.cap, m, m, R.acopy.as<double>(), m, E.st);
  small_syevx(R.acopy.as<double>(), m, m, nq, R.w.as<double>(), R.q.as<double>(), nq, R.work.as<double>(), E.st);
}

__global__ void rpa_scale_kernel(const double* __restrict__ w2, int k, double* __restrict__ om,
                                 double* __restrict__ f1, double* __restrict__ f2) {
  const int j = threadIdx.x + blockIdx.x * blockDim.x;
  if (j >= k) return;
  const double x = w2[j];
  const double o = x > 0.0 ? sqrt(x) : 0.0;
  om[j] = o;
  f1[j] = o > 0.0 ? 1.0 / sqrt(o) : 0.0;  // z = L w / sqrt(Omega)
  f2[j] = o > 0.0 ? 1.0 / o : 0.0;        // z' = a_+ z / Omega
}

__global__ void scale_small_cols_kernel(double* c, int m, int k, int ld, const double* __restrict__ f) {
  const int t = threadIdx.x + blockIdx.x * blockDim.x;
  if (t >= m * k) return;
  const int i = t / k, j = t - i * k;
  c[(long)i * ld + j] *= f[j];
}

// Full TDDFT: from a_+ (a1) and a_- (a2) compute Omega (R.om, device, k),
// z (R.zc, m x k) and z' (R.zpc, m x k).  Returns the host Omega^2 of the k
// lowest and the Cholesky info.
void ritz_rpa(Eng& E, Ritz& R, Basis& B, int k, std::vector<double>& w2_host, int& chol_info) {
  const int m = B.m;
  const int kk = std::min(k, m);
  R.lmat.ensure(sizeof(double) * (size_t)m * m);
  R.t1.ensure(sizeof(double) * (size_t)m * m);
  R.mmat.ensure(sizeof(double) * (size_t)m * m);
  R.w.ensure(sizeof(double) * kk);
  R.q.ensure(sizeof(double) * (size_t)m * kk);
  R.work.ensure(sizeof(double) * small_syevx_work(m, kk));
  R.ldq = kk;
  R.zc.ensure(sizeof(double) * (size_t)m * kk);
  R.zpc.ensure(sizeof(double) * (size_t)m * kk);
  R.om.ensure(sizeof(double) * 3 * kk);
  R.info.ensure(sizeof(int) * 4);
  {
  ProfScope ps(E.P->ctx, E.st, "small_dense", 0.0, 0.0);
  copy_block(B.a2.as<double>(), B.cap, m, m, R.lmat.as<double>(), m, E.st);
  small_chol(R.lmat.as<double>(), m, m, R.info.as<int>(), E.st);
  // M = L^T a_+ L
  small_gemm(0, 0, m, m, m, 1.0, B.a1.as<double>(), B.cap, R.lmat.as<double>(), m, 0.0, R.t1.as<double>(), m, E.st);
  small_gemm(1, 0, m, m, m, 1.0, R.lmat.as<double>(), m, R.t1.as<double>(), m, 0.0, R.mmat.as<double>(), m, E.st);
  small_symmetrize(R.mmat.as<double>(), m, m, E.st);
  small_syevx(R.mmat.as<double>(), m, m, kk, R.w.as<double>(), R.q.as<double>(), kk, R.work.as<double>(), E.st);
  double* om = R.om.as<double>();
  double* f1 = om + kk;
  double* f2 = om + 2 * kk;
  hipLaunchKernelGGL(rpa_scale_kernel, dim3(ceil_div(kk, 256)), dim3(256), 0, E.st, R.w.as<double>(), kk, om, f1,
                     f2);
  // z = L q[:, :k] / sqrt(Omega), z' = a_+ z / Omega
  small_gemm(0, 0, m, kk, m, 1.0, R.lmat.as<double>(), m, R.q.as<double>(), kk, 0.0, R.zc.as<double>(), kk, E.st);
  hipLaunchKernelGGL(scale_small_cols_kernel, dim3(ceil_div(m * kk, 256)), dim3(256), 0, E.st, R.zc.as<double>(), m,
                     kk, kk, f1);
  small_gemm(0, 0, m, kk, m, 1.0, B.a1.as<double>(), B.cap, R.zc.as<double>(), kk, 0.0, R.zpc.as<double>(), kk, E.st);
  hipLaunchKernelGGL(scale_small_cols_kernel, dim3(ceil_div(m * kk, 256)), dim3(256), 0, E.st, R.zpc.as<double>(), m,
                     kk, kk, f2);
  RID_HIP(hipGetLastError());
  }
  w2_host.resize(kk);
  E.d2h(w2_host.data(), R.w.as<double>(), sizeof(double) * kk);
  int info = 0;
  E.d2h(&info, R.info.as<int>(), sizeof(int));
  chol_info = info;
}

// ---------------------------------------------------------------------------
// Inner Krylov solves with the ris model (Eq. precondition).
// ---------------------------------------------------------------------------
struct InnerResult {
  int n_mv = 0, n_iter = 0;
};

// Solve (T - s_n) v_n = r_n approximately for n < nr.  r: nr x N (row-major),
// sh_host: shifts; out: nr x N.
InnerResult inner_single(Eng& E, int prec, const double* r, int nr, const std::vector<double>& sh_host, double tol,
                         int max_iter, double* out) {
  InnerResult res;
  if (nr <= 0) return res;
  rid_context* ctx = E.P->ctx;
  const long N = E.N;
  DevBuf rh(ctx), nrm(ctx), shd(ctx), idxd(ctx), wn(ctx), gbuf(ctx), mats(ctx), sol(ctx), tuy(ctx), rho(ctx),
      rnd(ctx);
  rh.ensure(sizeof(double) * nr * N);
  nrm.ensure(sizeof(double) * nr);
  {
    RedScratch rs = E.rs(1, nr);
    col_norms(r, N, nr, N, nrm.as<double>(), rs, E.st);
  }
  std::vector<double> rn(nr);
  E.d2h(rn.data(), nrm.as<double>(), sizeof(double) * nr);
  for (auto& x : rn)
    if (x == 0.0) x = 1.0;
  E.h2d(nrm.p, rn.data(), sizeof(double) * nr);
  RID_HIP(hipMemcpyAsync(rh.p, r, sizeof(double) * nr * N, hipMemcpyDeviceToDevice, E.st));
  scale_cols(rh.as<double>(), N, nr, N, nrm.as<double>(), 1, E.st);
  const double* sh = E.put_doubles(shd, sh_host);

  Basis U(ctx);
  const int cap = nr * std::max(1, max_iter) + nr;
  U.init(cap, N, 1);
  wn.ensure(sizeof(double) * nr * N);
  diag_tda(E.P->de.as<double>(), rh.as<double>(), N, nr, N, sh, nullptr, wn.as<double>(), N, E.st);
  append_orthonormal(E, U, wn.as<double>(), nr);
  const int kind = OPK_T;
  multiply(E, U, 0, kind, prec, nullptr);
  project(E, U, 0);
  res.n_mv = U.m;
  res.n_iter = 1;
  sol.ensure(sizeof(double) * nr * N);
  tuy.ensure(sizeof(double) * nr * N);
  rho.ensure(sizeof(double) * nr * N);
  rnd.ensure(sizeof(double) * nr);
  std::vector<char> done(nr, 0);
  std::vector<double> rhon(nr);
  while (true) {
    const int m = U.m;
    gbuf.ensure(sizeof(double) * (size_t)nr * m);
    mats.ensure(sizeof(double) * (size_t)nr * m * m);
    {
      RedScratch rs = E.rs(nr, m);
      gram(rh.as<double>(), N, nr, U.V(0), N, m, N, gbuf.as<double>(), m, rs, E.st);  // g[n][i]
    }
    {
      ProfScope ps(E.P->ctx, E.st, "inner_solve", 0.0, 0.0);
      build_shifted(U.a1.as<double>(), nullptr, m, U.cap, sh, nr, 0, mats.as<double>(), E.st);
      small_lu_solve_cm(mats.as<double>(), gbuf.as<double>(), m, nr, E.st);  // y[n][i] (symmetric systems)
    }
    combo(U.V(0), N, m, gbuf.as<double>(), 1, m, nr, N, 1.0, 0.0, sol.as<double>(), N, E.st);
    combo(U.P1(0), N, m, gbuf.as<double>(), 1, m, nr, N, 1.0, 0.0, tuy.as<double>(), N, E.st);
    resid3(tuy.as<double>(), sol.as<double>(), rh.as<double>(), N, nr, N, sh, rho.as<double>(), N, E.st);
    {
      RedScratch rs = E.rs(1, nr);
      col_norms(rho.as<double>(), N, nr, N, rnd.as<double>(), rs, E.st);
    }
    E.d2h(rhon.data(), rnd.as<double>(), sizeof(double) * nr);
    // freeze the solution of every right-hand side still open at its latest iterate
    copy_open_columns(done, sol.as<double>(), out, N, E.st);
    std::vector<int> act;
    for (int n = 0; n < nr; ++n) {
      if (done[n]) continue;
      if (rhon[n] < tol)
        done[n] = 1;
      else
        act.push_back(n);
    }
    if (act.empty() || res.n_iter >= max_iter) break;
    const int* idx = E.put_ints(idxd, act);
    diag_tda(E.P->de.as<double>(), rho.as<double>(), N, (int)act.size(), N, sh, idx, wn.as<double>(), N, E.st);
    const int m0 = U.m;
    const int added = append_orthonormal(E, U, wn.as<double>(), (int)act.size());
    if (added == 0) break;
    multiply(E, U, m0, kind, prec, nullptr);
    project(E, U, m0);
    res.n_mv += added;
    res.n_iter += 1;
  }
  // undo the unit scaling of the right-hand sides
  scale_cols(out, N, nr, N, nrm.as<double>(), 0, E.st);
  E.sync();
  return res;
}

// Projected pair systems [[t+, -s_b I], [-s_b I, t-]] (y_b; y'_b) = (g1_b; g2_b)
// for b < nb; g (rows of length 2m: g1 then g2) is overwritten by (y; y').
// For s_b != 0 the second block is eliminated by multiplying the first
// equation with t-:
//   (t- t+ - s^2 I) y = t- g1 + s g2,   y' = (t+ y - g1) / s,
// one m x m system per right-hand side and no factorisation of t- at all;
// for s_b = 0 the two blocks decouple (t+ y = g1, t- y' = g2).  The systems
// are solved by Gaussian elimination with partial pivoting.
void solve_pair_systems(Eng& E, Basis& U, int m, const std::vector<double>& sh_host, int nb, double* g,
                        DevBuf& mats, DevBuf& work) {
  ProfScope ps(E.P->ctx, E.st, "inner_solve", 0.0, 0.0);
  std::vector<int> sb, st;
  std::vector<double> ss;
  for (int b = 0; b < nb; ++b) {
    if (sh_host[b] != 0.0) {
      sb.push_back(b);
      st.push_back(0);
      ss.push_back(sh_host[b]);
    } else {
      sb.push_back(b);
      st.push_back(1);
      ss.push_back(0.0);
      sb.push_back(b);
      st.push_back(2);
      ss.push_back(0.0);
    }
  }
  const int nsys = (int)sb.size();
  // system table on the device: b, type (ints) then shifts (doubles)
  std::vector<double> table((size_t)3 * nsys);
  for (int q = 0; q < nsys; ++q) {
    table[q] = ss[q];
    reinterpret_cast<int*>(table.data() + nsys)[q] = sb[q];
    reinterpret_cast<int*>(table.data() + nsys)[nsys + q] = st[q];
  }
  work.ensure(sizeof(double) * ((size_t)m * m + (size_t)3 * nsys * m + (size_t)nb * m + table.size() + 8));
  double* P = work.as<double>();                // t- t+ (row-major, m x m)
  double* rhs = P + (size_t)m * m;               // nsys x m
  double* yt = rhs + (size_t)nsys * m;           // nsys x m
  double* tg = yt + (size_t)nsys * m;            // nb x m: rows g1_b t-
  double* tab = tg + (size_t)nb * m;
  E.h2d(tab, table.data(), sizeof(double) * table.size());
  const double* sys_shift = tab;
  const int* sys_b = reinterpret_cast<const int*>(tab + nsys);
  const int* sys_type = sys_b + nsys;
  const double* tp = U.a1.as<double>();
  const double* tm = U.a2.as<double>();
  small_gemm(0, 0, m, m, m, 1.0, tm, U.cap, tp, U.cap, 0.0, P, m, E.st);
  small_gemm(0, 0, nb, m, m, 1.0, g, 2 * m, tm, U.cap, 0.0, tg, m, E.st);  // g1_b^T t- (t- symmetric)
  mats.ensure(sizeof(double) * (size_t)nsys * m * m);
  pair_systems_build(P, tp, tm, U.cap, m, sys_b, sys_type, sys_shift, nsys, g, 2 * m, tg, mats.as<double>(), rhs,
                     E.st);
  small_lu_solve_cm(mats.as<double>(), rhs, m, nsys, E.st);  // rhs <- solutions
  small_gemm(0, 0, nsys, m, m, 1.0, rhs, m, tp, U.cap, 0.0, yt, m, E.st);  // y^T t+ (t+ symmetric)
  pair_systems_unpack(g, 2 * m, rhs, yt, sys_b, sys_type, sys_shift, nsys, m, E.st);
}

// Solve [[T+, -s_n], [-s_n, T-]] (d1; d2) = (r1; r2) approximately.
InnerResult inner_pair(Eng& E, int prec, const double* r1, const double* r2, int nr, const std::vector<double>& sh_host,
                       double tol, int max_iter, double* out1, double* out2) {
  InnerResult res;
  if (nr <= 0) return res;
  rid_context* ctx = E.P->ctx;
  const long N = E.N;
  DevBuf h1(ctx), h2(ctx), nrm(ctx), n1(ctx), shd(ctx), idxd(ctx), wn(ctx), gbuf(ctx), mats(ctx), s1(ctx), s2(ctx),
      ty(ctx), rho1(ctx), rho2(ctx), rnd(ctx), schur(ctx);
  h1.ensure(sizeof(double) * nr * N);
  h2.ensure(sizeof(double) * nr * N);
  nrm.ensure(sizeof(double) * nr);
  n1.ensure(sizeof(double) * 2 * nr);
  {
    RedScratch rs = E.rs(1, nr);
    col_norms(r1, N, nr, N, n1.as<double>(), rs, E.st);
    col_norms(r2, N, nr, N, n1.as<double>() + nr, rs, E.st);
  }
  std::vector<double> nn(2 * nr), rn(nr);
  E.d2h(nn.data(), n1.as<double>(), sizeof(double) * 2 * nr);
  for (int n = 0; n < nr; ++n) {
    rn[n] = std::sqrt(nn[n] * nn[n] + nn[nr + n] * nn[nr + n]);
    if (rn[n] == 0.0) rn[n] = 1.0;
  }
  E.h2d(nrm.p, rn.data(), sizeof(double) * nr);
  RID_HIP(hipMemcpyAsync(h1.p, r1, sizeof(double) * nr * N, hipMemcpyDeviceToDevice, E.st));
  RID_HIP(hipMemcpyAsync(h2.p, r2, sizeof(double) * nr * N, hipMemcpyDeviceToDevice, E.st));
  scale_cols(h1.as<double>(), N, nr, N, nrm.as<double>(), 1, E.st);
  scale_cols(h2.as<double>(), N, nr, N, nrm.as<double>(), 1, E.st);
  const double* sh = E.put_doubles(shd, sh_host);

  Basis U(ctx);
  const int cap = 2 * nr * std::max(1, max_iter) + 2 * nr;
  U.init(cap, N, 2);
  wn.ensure(sizeof(double) * 2 * nr * N);
  double* de = E.P->de.as<double>();
  diag_pair(de, h1.as<double>(), h2.as<double>(), N, nr, N, sh, nullptr, wn.as<double>(),
            wn.as<double>() + (long)nr * N, N, E.st);
  append_orthonormal(E, U, wn.as<double>(), 2 * nr);
  const int kind = OPK_TPAIR;
  multiply(E, U, 0, kind, prec, nullptr);
  project(E, U, 0);
  res.n_mv = U.m;
  res.n_iter = 1;
  s1.ensure(sizeof(double) * nr * N);
  s2.ensure(sizeof(double) * nr * N);
  ty.ensure(sizeof(double) * nr * N);
  rho1.ensure(sizeof(double) * nr * N);
  rho2.ensure(sizeof(double) * nr * N);
  rnd.ensure(sizeof(double) * 2 * nr);
  std::vector<char> done(nr, 0);
  std::vector<double> rr(2 * nr);
  while (true) {
    const int m = U.m;
    const int d = 2 * m;
    gbuf.ensure(sizeof(double) * (size_t)nr * d);
    {
      RedScratch rs = E.rs(nr, m);
      gram(h1.as<double>(), N, nr, U.V(0), N, m, N, gbuf.as<double>(), d, rs, E.st);
      gram(h2.as<double>(), N, nr, U.V(0), N, m, N, gbuf.as<double>() + m, d, rs, E.st);
    }
    solve_pair_systems(E, U, m, sh_host, nr, gbuf.as<double>(), mats, schur);
    const double* y1 = gbuf.as<double>();
    const double* y2 = gbuf.as<double>() + m;
    combo(U.V(0), N, m, y1, 1, d, nr, N, 1.0, 0.0, s1.as<double>(), N, E.st);
    combo(U.V(0), N, m, y2, 1, d, nr, N, 1.0, 0.0, s2.as<double>(), N, E.st);
    // rho1 = T+ U y1 - s * s2 - h1 ; rho2 = T- U y2 - s * s1 - h2
    combo(U.P1(0), N, m, y1, 1, d, nr, N, 1.0, 0.0, ty.as<double>(), N, E.st);
    resid3(ty.as<double>(), s2.as<double>(), h1.as<double>(), N, nr, N, sh, rho1.as<double>(), N, E.st);
    combo(U.P2(0), N, m, y2, 1, d, nr, N, 1.0, 0.0, ty.as<double>(), N, E.st);
    resid3(ty.as<double>(), s1.as<double>(), h2.as<double>(), N, nr, N, sh, rho2.as<double>(), N, E.st);
    {
      RedScratch rs = E.rs(1, nr);
      col_norms(rho1.as<double>(), N, nr, N, rnd.as<double>(), rs, E.st);
      col_norms(rho2.as<double>(), N, nr, N, rnd.as<double>() + nr, rs, E.st);
    }
    E.d2h(rr.data(), rnd.as<double>(), sizeof(double) * 2 * nr);
    copy_open_columns(done, s1.as<double>(), out1, N, E.st);
    copy_open_columns(done, s2.as<double>(), out2, N, E.st);
    std::vector<int> act;
    for (int n = 0; n < nr; ++n) {
      if (done[n]) continue;
      if (std::sqrt(rr[n] * rr[n] + rr[nr + n] * rr[nr + n]) < tol)
        done[n] = 1;
      else
        act.push_back(n);
    }
    if (act.empty() || res.n_iter >= max_iter) break;
    const int na = (int)act.size();
    const int* idx = E.put_ints(idxd, act);
    diag_pair(de, rho1.as<double>(), rho2.as<double>(), N, na, N, sh, idx, wn.as<double>(),
              wn.as<double>() + (long)na * N, N, E.st);
    const int m0 = U.m;
    const int added = append_orthonormal(E, U, wn.as<double>(), 2 * na);
    if (added == 0) break;
    multiply(E, U, m0, kind, prec, nullptr);
    project(E, U, m0);
    res.n_mv += added;
    res.n_iter += 1;
  }
  scale_cols(out1, N, nr, N, nrm.as<double>(), 0, E.st);
  scale_cols(out2, N, nr, N, nrm.as<double>(), 0, E.st);
  E.sync();
  return res;
}

// ---------------------------------------------------------------------------
// Davidson cores.
// ---------------------------------------------------------------------------
struct EigCore {
  std::vector<double> omega, resid;
  int n_iter = 0, n_mv = 0, n_inner = 0, n_inner_iter = 0;
  std::vector<double> history;
  rid_status status = RID_OK;
};

// Preconditioner callback: given the residual block (row-major), active
// indices (host) and their shifts, write the new directions to out and return
// how many were written.  For the pair form the block holds R and R'.
typedef std::function<int(const double* r1, const double* r2, const std::vector<int>& act,
                          const std::vector<double>& sh, double* out, EigCore& core)>
    PrecondFn;

// TDA Davidson on operator `kind` (OPK_A or OPK_T).  v0: n0 vectors.  On
// return xout (k x N) holds the Ritz vectors.
void davidson_sym(Eng& E, int kind, int prec, int k, const double* v0, int n0, const PrecondFn& pc, double tol,
                  int max_iter, int m_max, int keep, double* xout, EigCore& core, bool timed) {
  rid_context* ctx = E.P->ctx;
  const long N = E.N;
  SolveStats& st = *E.stats;
  double tmv = 0.0;
  const int kk0 = std::min<long>(k, N);
  Basis B(ctx);
  const int cap = std::max(m_max, n0) + 2 * kk0 + 8;
  B.init(cap, N, 1);
  DevBuf wn(ctx), ax(ctx), r(ctx), rnd(ctx), idxd(ctx), vtmp(ctx), ptmp(ctx);
  wn.ensure(sizeof(double) * std::max(n0, 2 * kk0) * N);
  RID_HIP(hipMemcpyAsync(wn.p, v0, sizeof(double) * n0 * N, hipMemcpyDeviceToDevice, E.st));
  append_orthonormal(E, B, wn.as<double>(), n0);
  RID_CHECK(B.m > 0, RID_ERR_BREAKDOWN, "initial subspace is empty");
  multiply(E, B, 0, kind, prec, &tmv);
  project(E, B, 0);
  core.n_iter = 1;
  core.n_mv = B.m;
  Ritz R(ctx);
  ax.ensure(sizeof(double) * kk0 * N);
  r.ensure(sizeof(double) * kk0 * N);
  rnd.ensure(sizeof(double) * kk0);
  auto t_start = Clock::now();
  while (true) {
    const int m = B.m;
    const int kk = std::min(kk0, m);
    auto t0 = Clock::now();
    ritz_sym(E, R, B, std::max(kk, keep));
    // X = V q[:, :k], AX = AV q[:, :k], R = AX - w X
    combo(B.V(0), N, m, R.q.as<double>(), R.ldq, 1, kk, N, 1.0, 0.0, xout, N, E.st);
    combo(B.P1(0), N, m, R.q.as<double>(), R.ldq, 1, kk, N, 1.0, 0.0, ax.as<double>(), N, E.st);
    residual(ax.as<double>(), xout, N, kk, N, R.w.as<double>(), r.as<double>(), E.st);
    {
      RedScratch rs = E.rs(1, kk);
      col_norms(r.as<double>(), N, kk, N, rnd.as<double>(), rs, E.st);
    }
    core.omega.resize(kk);
    core.resid.resize(kk);
    E.d2h(core.omega.data(), R.w.as<double>(), sizeof(double) * kk);
    E.d2h(core.resid.data(), rnd.as<double>(), sizeof(double) * kk);
    if (timed) st.t_other += ms_since(t0);
    core.history.push_back(*std::max_element(core.resid.begin(), core.resid.end()));
    std::vector<int> act;
    for (int n = 0; n < kk; ++n)
      if (!(core.resid[n] < tol)) act.push_back(n);
    if (act.empty()) {
      core.status = RID_OK;
      break;
    }
    if (core.n_iter >= max_iter) {
      core.status = RID_WARN_NOT_CONVERGED;
      break;
    }
    std::vector<double> sh(act.size());
    for (size_t q = 0; q < act.size(); ++q) sh[q] = core.omega[act[q]];
    auto tp = Clock::now();
    const int nnew = pc(r.as<double>(), nullptr, act, sh, wn.as<double>(), core);
    if (timed) st.t_precond += ms_since(tp);
    t0 = Clock::now();
    if (B.m + nnew > m_max) {
      // restart on the leading Ritz vectors: exact by linearity, and the
      // projected matrix of the collapsed basis is diag(w)
      const int kp = std::min(keep, R.ldq);
      vtmp.ensure(sizeof(double) * kp * N);
      ptmp.ensure(sizeof(double) * kp * N);
      combo(B.V(0), N, m, R.q.as<double>(), R.ldq, 1, kp, N, 1.0, 0.0, vtmp.as<double>(), N, E.st);
      combo(B.P1(0), N, m, R.q.as<double>(), R.ldq, 1, kp, N, 1.0, 0.0, ptmp.as<double>(), N, E.st);
      RID_HIP(hipMemcpyAsync(B.V(0), vtmp.p, sizeof(double) * kp * N, hipMemcpyDeviceToDevice, E.st));
      RID_HIP(hipMemcpyAsync(B.P1(0), ptmp.p, sizeof(double) * kp * N, hipMemcpyDeviceToDevice, E.st));
      std::vector<double> wk(kp);
      E.d2h(wk.data(), R.w.as<double>(), sizeof(double) * kp);
      std::vector<double> a((size_t)B.cap * B.cap, 0.0);
      for (int i = 0; i < kp; ++i) a[(size_t)i * B.cap + i] = wk[i];
      E.h2d(B.a1.p, a.data(), sizeof(double) * a.size());
      B.m = kp;
    }
    const int m0 = B.m;
    const int added = append_orthonormal(E, B, wn.as<double>(), nnew);
    if (timed) st.t_other += ms_since(t0);
    if (added == 0) {
      core.status = RID_ERR_BREAKDOWN;
      break;
    }
    multiply(E, B, m0, kind, prec, &tmv);
    t0 = Clock::now();
    project(E, B, m0);
    if (timed) st.t_other += ms_since(t0);
    core.n_iter += 1;
    core.n_mv += added;
    E.track(B.bytes() + E.P->footprint());
  }
  tmv += E.take_product_ms();
  if (timed) st.t_matvec += tmv;
  (void)t_start;
}

// Restart of the shared (Z, Z') subspace: collapse the basis onto the span of
// the Z and Z' of the ncol lowest Ritz pairs (coefficient vectors: the
// columns of zc, zpc of the Ritz step, row stride ld), orthonormalised in the
// coefficient space.  Exact by linearity:
// V' = V Q, (A+-B) V' = P Q and a' = Q^T a Q.  The coefficient work is small
// (m x 2kk) and runs on the host.
void restart_pair(Eng& E, Basis& B, const Ritz& R, int ld, int ncol) {
  const int m = B.m;
  const long N = E.N;
  std::vector<double> zc((size_t)m * ld), zpc((size_t)m * ld);
  E.d2h(zc.data(), R.zc.p, sizeof(double) * zc.size());
  E.d2h(zpc.data(), R.zpc.p, sizeof(double) * zpc.size());
  std::vector<std::vector<double>> acc;
  for (int src = 0; src < 2; ++src)
    for (int j = 0; j < ncol; ++j) {
      const std::vector<double>& c = src == 0 ? zc : zpc;
      std::vector<double> v(m);
      for (int i = 0; i < m; ++i) v[i] = c[(size_t)i * ld + j];
      double nrm = 0.0;
      for (double x : v) nrm += x * x;
      nrm = std::sqrt(nrm);
      if (!(nrm > 0.0)) continue;
      for (double& x : v) x /= nrm;
      for (int pass = 0; pass < 2; ++pass)
        for (const std::vector<double>& q : acc) {
          double d = 0.0;
          for (int i = 0; i < m; ++i) d += q[i] * v[i];
          for (int i = 0; i < m; ++i) v[i] -= d * q[i];
        }
      nrm = 0.0;
      for (double x : v) nrm += x * x;
      nrm = std::sqrt(nrm);
      if (!(nrm >= 1e-8)) continue;
      for (double& x : v) x /= nrm;
      acc.push_back(std::move(v));
    }
  const int r = (int)acc.size();
  RID_CHECK(r > 0, RID_ERR_BREAKDOWN, "restart subspace is empty");
  std::vector<double> q((size_t)m * r);
  for (int c = 0; c < r; ++c)
    for (int i = 0; i < m; ++i) q[(size_t)i * r + c] = acc[c][i];
  // a' = Q^T a Q for both projected matrices
  for (int t = 0; t < 2; ++t) {
    DevBuf& ad = t == 0 ? B.a1 : B.a2;
    std::vector<double> a((size_t)B.cap * B.cap);
    E.d2h(a.data(), ad.p, sizeof(double) * a.size());
    std::vector<double> aq((size_t)m * r, 0.0), an((size_t)B.cap * B.cap, 0.0);
    for (int i = 0; i < m; ++i)
      for (int l = 0; l < m; ++l) {
        const double ail = a[(size_t)i * B.cap + l];
        for (int c = 0; c < r; ++c) aq[(size_t)i * r + c] += ail * q[(size_t)l * r + c];
      }
    for (int c = 0; c < r; ++c)
      for (int d = 0; d < r; ++d) {
        double v = 0.0;
        for (int i = 0; i < m; ++i) v += q[(size_t)i * r + c] * aq[(size_t)i * r + d];
        an[(size_t)c * B.cap + d] = v;
      }
    for (int c = 0; c < r; ++c)
      for (int d = 0; d < c; ++d) {
        const double v = 0.5 * (an[(size_t)c * B.cap + d] + an[(size_t)d * B.cap + c]);
        an[(size_t)c * B.cap + d] = an[(size_t)d * B.cap + c] = v;
      }
    E.h2d(ad.p, an.data(), sizeof(double) * an.size());
  }
  DevBuf qd(E.P->ctx), tmp(E.P->ctx);
  qd.ensure(sizeof(double) * q.size());
  E.h2d(qd.p, q.data(), sizeof(double) * q.size());
  tmp.ensure(sizeof(double) * (size_t)r * N);
  for (int t = 0; t < 3; ++t) {
    double* base = t == 0 ? B.V(0) : (t == 1 ? B.P1(0) : B.P2(0));
    combo(base, N, m, qd.as<double>(), r, 1, r, N, 1.0, 0.0, tmp.as<double>(), N, E.st);
    RID_HIP(hipMemcpyAsync(base, tmp.p, sizeof(double) * (size_t)r * N, hipMemcpyDeviceToDevice, E.st));
  }
  E.sync();
  B.m = r;
}

// Full-TDDFT Davidson on the pair operator `kind` (OPK_PAIR or OPK_TPAIR).
// On return zout / zpout (k x N) hold Z = X+Y and Z' = X-Y.
void davidson_rpa(Eng& E, int kind, int prec, int k, const double* v0, int n0, const PrecondFn& pc, double tol,
                  int max_iter, int m_max, int keep, double* zout, double* zpout, EigCore& core, bool timed) {
  rid_context* ctx = E.P->ctx;
  const long N = E.N;
  SolveStats& st = *E.stats;
  double tmv = 0.0;
  const int kk0 = std::min<long>(k, N);
  Basis B(ctx);
  const int cap = std::max(m_max, n0) + 4 * kk0 + 8;
  B.init(cap, N, 2);
  DevBuf wn(ctx), pz(ctx), mz(ctx), r1(ctx), r2(ctx), rnd(ctx);
  wn.ensure(sizeof(double) * std::max(n0, 2 * kk0) * N);
  RID_HIP(hipMemcpyAsync(wn.p, v0, sizeof(double) * n0 * N, hipMemcpyDeviceToDevice, E.st));
  append_orthonormal(E, B, wn.as<double>(), n0);
  RID_CHECK(B.m > 0, RID_ERR_BREAKDOWN, "initial subspace is empty");
  multiply(E, B, 0, kind, prec, &tmv);
  project(E, B, 0);
  core.n_iter = 1;
  core.n_mv = B.m;
  Ritz R(ctx);
  pz.ensure(sizeof(double) * kk0 * N);
  mz.ensure(sizeof(double) * kk0 * N);
  r1.ensure(sizeof(double) * kk0 * N);
  r2.ensure(sizeof(double) * kk0 * N);
  rnd.ensure(sizeof(double) * 2 * kk0);
  while (true) {
    const int m = B.m;
    const int kk = std::min(kk0, m);
    auto t0 = Clock::now();
    // the lowest kk pairs are the answer; up to `keep` pairs seed a restart
    const int nq = std::min(m, std::max(kk, keep));
    std::vector<double> w2;
    int info = 0;
    ritz_rpa(E, R, B, nq, w2, info);
    if (info != 0) throw Error(RID_ERR_INDEFINITE, "projected A-B is not positive definite");
    for (int j = 0; j < kk; ++j)
      if (!(w2[j] > 0.0)) throw Error(RID_ERR_INDEFINITE, "non-positive Omega^2 in the projected problem");
    int nkeep = kk;
    while (nkeep < nq && w2[nkeep] > 0.0) ++nkeep;
    core.omega.resize(kk);
    for (int j = 0; j < kk; ++j) core.omega[j] = std::sqrt(w2[j]);
    const double* om = R.om.as<double>();
    combo(B.V(0), N, m, R.zc.as<double>(), nq, 1, kk, N, 1.0, 0.0, zout, N, E.st);
    combo(B.V(0), N, m, R.zpc.as<double>(), nq, 1, kk, N, 1.0, 0.0, zpout, N, E.st);
    combo(B.P1(0), N, m, R.zc.as<double>(), nq, 1, kk, N, 1.0, 0.0, pz.as<double>(), N, E.st);
    combo(B.P2(0), N, m, R.zpc.as<double>(), nq, 1, kk, N, 1.0, 0.0, mz.as<double>(), N, E.st);
    residual_pair(pz.as<double>(), zpout, mz.as<double>(), zout, N, kk, N, om, r1.as<double>(), r2.as<double>(),
                  E.st);
    {
      RedScratch rs = E.rs(1, kk);
      col_norms(r1.as<double>(), N, kk, N, rnd.as<double>(), rs, E.st);
      col_norms(r2.as<double>(), N, kk, N, rnd.as<double>() + kk, rs, E.st);
    }
    std::vector<double> rr(2 * kk);
    E.d2h(rr.data(), rnd.as<double>(), sizeof(double) * 2 * kk);
    core.resid.resize(kk);
    for (int j = 0; j < kk; ++j) core.resid[j] = std::sqrt(rr[j] * rr[j] + rr[kk + j] * rr[kk + j]);
    if (timed) st.t_other += ms_since(t0);
    core.history.push_back(*std::max_element(core.resid.begin(), core.resid.end()));
    std::vector<int> act;
    for (int n = 0; n < kk; ++n)
      if (!(core.resid[n] < tol)) act.push_back(n);
    if (act.empty()) {
      core.status = RID_OK;
      break;
    }
    if (core.n_iter >= max_iter) {
      core.status = RID_WARN_NOT_CONVERGED;
      break;
    }
    std::vector<double> sh(act.size());
    for (size_t q = 0; q < act.size(); ++q) sh[q] = core.omega[act[q]];
    auto tp = Clock::now();
    const int nnew = pc(r1.as<double>(), r2.as<double>(), act, sh, wn.as<double>(), core);
    if (timed) st.t_precond += ms_since(tp);
    t0 = Clock::now();
    if (B.m + nnew > m_max) restart_pair(E, B, R, nq, nkeep);
    RID_CHECK(B.m + nnew <= B.cap, RID_ERR_INTERNAL, "basis capacity exceeded after restart");
    const int m0 = B.m;
    const int added = append_orthonormal(E, B, wn.as<double>(), nnew);
    if (timed) st.t_other += ms_since(t0);
    if (added == 0) {
      core.status = RID_ERR_BREAKDOWN;
      break;
    }
    multiply(E, B, m0, kind, prec, &tmv);
    t0 = Clock::now();
    project(E, B, m0);
    if (timed) st.t_other += ms_since(t0);
    core.n_iter += 1;
    core.n_mv += added;
    E.track(B.bytes() + E.P->footprint());
  }
  tmv += E.take_product_ms();
  if (timed) st.t_matvec += tmv;
}

int outer_prec(const rid_solve_opts& o) { return o.precision == RID_PRECISION_MIXED ? PREC_F32 : PREC_F64; }
int ris_prec(const rid_solve_opts& o) { return o.precision == RID_PRECISION_MIXED ? PREC_BF16 : PREC_F64; }

}  // namespace

void validate_opts(const rid_solve_opts& o, const rid_problem* P) {
  RID_CHECK(o.precond == RID_PRECOND_DIAG || o.precond == RID_PRECOND_RIS, RID_ERR_INVALID_ARG, "bad precond");
  RID_CHECK(o.precision == RID_PRECISION_FP64 || o.precision == RID_PRECISION_MIXED, RID_ERR_INVALID_ARG,
            "bad precision");
  RID_CHECK(o.tol > 0.0 && o.inner_tol > 0.0 && o.init_tol > 0.0, RID_ERR_INVALID_ARG, "tolerances must be > 0");
  RID_CHECK(o.max_iter >= 1 && o.inner_max_iter >= 1 && o.init_max_iter >= 1, RID_ERR_INVALID_ARG,
            "iteration limits must be >= 1");
  RID_CHECK(o.m_max >= 0 && o.m_max <= 1000, RID_ERR_INVALID_ARG, "m_max must be in [0, 1000]");
  RID_CHECK(o.graphs == 0 || o.graphs == 1, RID_ERR_INVALID_ARG, "graphs must be 0 or 1");
  if (o.precond == RID_PRECOND_RIS)
    RID_CHECK(P->has_ris(), RID_ERR_INVALID_ARG, "ris preconditioner needs a ris tensor");
  RID_CHECK(o.n_guess >= 0 && (o.n_guess == 0 || o.guess_dev != nullptr), RID_ERR_INVALID_ARG,
            "n_guess must be >= 0, with guess_dev when > 0");
  RID_CHECK((long)o.n_guess <= 4 * P->n(), RID_ERR_SHAPE, "too many guess vectors");
  if (o.precision == RID_PRECISION_FP64) {
    RID_CHECK(P->b_dt == RID_F64, RID_ERR_DTYPE, "an FP64 solve needs FP64 tensors");
    if (o.precond == RID_PRECOND_RIS)
      RID_CHECK(P->bris_dt == RID_F64, RID_ERR_DTYPE, "an FP64 solve with the ris model needs FP64 ris tensors");
  }
}

rid_status eigen_solve(rid_problem* P, const rid_solve_opts& o, int k, int mode, double* omega_host, double* x_dev,
                       double* y_dev, double* resid_host, SolveStats& st, const ExecCfg& ex) {
  validate_opts(o, P);
  const long N = P->n();
  RID_CHECK(k >= 1 && k <= N, RID_ERR_SHAPE, "k must be in [1, N]");
  RID_CHECK(mode == RID_TDA || mode == RID_RPA, RID_ERR_INVALID_ARG, "bad mode");
  auto t_all = Clock::now();
  Eng E(P, &st, ex);
  E.use_graphs = o.graphs != 0;
  rid_context* ctx = P->ctx;
  const bool ris = o.precond == RID_PRECOND_RIS;
  const int extra = o.n_extra_init >= 0 ? o.n_extra_init : (ris ? std::min(k, 3) : 8);
  const int n_init = (int)std::min<long>(N, k + extra);
  // the subspace must hold a restart (N_init vectors) plus two blocks of new
  // directions, and stay within the projected-problem limit of the dense
  // eigensolver: both checked before any work
  const int m_floor = 2 * n_init + 4 * k + 8;
  RID_CHECK(m_floor <= kMaxProjected, RID_ERR_SHAPE,
            "k = " + std::to_string(k) + " needs a subspace of at least " + std::to_string(m_floor) +
                " vectors, above the projected-problem limit of " + std::to_string(kMaxProjected));
  const int m_max = std::min(kMaxProjected, std::max(default_m_max(k, o.m_max), m_floor));
  RID_CHECK(o.n_guess + n_init <= kMaxProjected, RID_ERR_SHAPE,
            "warm-start vectors plus N_init exceed the projected-problem limit of " + std::to_string(kMaxProjected));
  const int pin = ris_prec(o), pout = outer_prec(o);
  const double* de = P->de.as<double>();
  DevBuf v0(ctx), zbuf(ctx), zpbuf(ctx), posd(ctx);
  EigCore core;
  auto tp = Clock::now();
  int n0 = n_init;
  if (o.n_guess > 0) {
    // warm start: the caller's vectors, then the unit vectors of the
    // smallest de; dependent directions are dropped when the basis is built
    n0 = o.n_guess + n_init;
    v0.ensure(sizeof(double) * (size_t)n0 * N);
    RID_HIP(hipMemcpyAsync(v0.p, o.guess_dev, sizeof(double) * (size_t)o.n_guess * N, hipMemcpyDeviceToDevice,
                           E.st));
    const int* pos = E.put_ints(posd, smallest_positions(P, n_init));
    unit_vectors(pos, n_init, N, v0.as<double>() + (long)o.n_guess * N, N, E.st);
  } else if (mode == RID_TDA) {
    if (!ris) {
      v0.ensure(sizeof(double) * n_init * N);
      const int* pos = E.put_ints(posd, smallest_positions(P, n_init));
      unit_vectors(pos, n_init, N, v0.as<double>(), N, E.st);
    } else {
      // initial guess: N_init lowest Ritz vectors of a Davidson run on T
      const int nt = (int)std::min<long>(N, n_init + 8);
      DevBuf u(ctx);
      u.ensure(sizeof(double) * nt * N);
      const int* pos = E.put_ints(posd, smallest_positions(P, nt));
      unit_vectors(pos, nt, N, u.as<double>(), N, E.st);
      v0.ensure(sizeof(double) * n_init * N);
      EigCore g;
      PrecondFn dpc = [&](const double* r1, const double*, const std::vector<int>& act, const std::vector<double>& sh,
                          double* out, EigCore&) {
        DevBuf idxd(ctx), shd(ctx);
        const int* idx = E.put_ints(idxd, act);
        std::vector<double> shf(n_init, 0.0);
        for (size_t q = 0; q < act.size(); ++q) shf[act[q]] = sh[q];
        const double* sd = E.put_doubles(shd, shf);
        diag_tda(de, r1, N, (int)act.size(), N, sd, idx, out, N, E.st);
        return (int)act.size();
      };
      davidson_sym(E, OPK_T, pin, n_init, u.as<double>(), nt, dpc, o.init_tol, o.init_max_iter,
                   std::min(kMaxProjected, std::max(200, 40 * n_init)), n_init, v0.as<double>(), g, false);
      st.n_inner_mv += g.n_mv;
      st.n_inner_iter += g.n_iter;
    }
  } else {
    if (!ris) {
      v0.ensure(sizeof(double) * n_init * N);
      const int* pos = E.put_ints(posd, smallest_positions(P, n_init));
      unit_vectors(pos, n_init, N, v0.as<double>(), N, E.st);
    } else {
      const int nt = (int)std::min<long>(N, n_init + 8);
      DevBuf u(ctx);
      u.ensure(sizeof(double) * nt * N);
      const int* pos = E.put_ints(posd, smallest_positions(P, nt));
      unit_vectors(pos, nt, N, u.as<double>(), N, E.st);
      v0.ensure(sizeof(double) * 2 * n_init * N);
      EigCore g;
      PrecondFn dpc = [&](const double* r1, const double* r2, const std::vector<int>& act,
                          const std::vector<double>& sh, double* out, EigCore&) {
        DevBuf idxd(ctx), shd(ctx);
        const int* idx = E.put_ints(idxd, act);
        std::vector<double> shf(n_init, 0.0);
        for (size_t q = 0; q < act.size(); ++q) shf[act[q]] = sh[q];
        const double* sd = E.put_doubles(shd, shf);
        const int na = (int)act.size();
        diag_pair(de, r1, r2, N, na, N, sd, idx, out, out + (long)na * N, N, E.st);
        return 2 * na;
      };
      davidson_rpa(E, OPK_TPAIR, pin, n_init, u.as<double>(), nt, dpc, o.init_tol, o.init_max_iter,
                   std::min(kMaxProjected, std::max(200, 40 * n_init)), n_init, v0.as<double>(), v0.as<double>() + (long)n_init * N, g,
                   false);
      st.n_inner_mv += g.n_mv;
      st.n_inner_iter += g.n_iter;
      n0 = 2 * n_init;
    }
  }
  st.t_precond += ms_since(tp);

  // outer preconditioner
  PrecondFn pc;
  if (mode == RID_TDA) {
    pc = [&](const double* r1, const double*, const std::vector<int>& act, const std::vector<double>& sh, double* out,
             EigCore& c) {
      const int na = (int)act.size();
      if (!ris) {
        DevBuf idxd(ctx), shd(ctx);
        const int* idx = E.put_ints(idxd, act);
        std::vector<double> shf(k, 0.0);
        for (int q = 0; q < na; ++q) shf[act[q]] = sh[q];
        const double* sd = E.put_doubles(shd, shf);
        diag_tda(de, r1, N, na, N, sd, idx, out, N, E.st);
        return na;
      }
      DevBuf rsel(ctx), idxd(ctx);
      rsel.ensure(sizeof(double) * na * N);
      const int* idx = E.put_ints(idxd, act);
      gather_cols(r1, N, idx, na, N, rsel.as<double>(), N, E.st);
      InnerResult ir = inner_single(E, pin, rsel.as<double>(), na, sh, o.inner_tol, o.inner_max_iter, out);
      c.n_inner += ir.n_mv;
      c.n_inner_iter += ir.n_iter;
      return na;
    };
  } else {
    pc = [&](const double* r1, const double* r2, const std::vector<int>& act, const std::vector<double>& sh,
             double* out, EigCore& c) {
      const int na = (int)act.size();
      if (!ris) {
        DevBuf idxd(ctx), shd(ctx);
        const int* idx = E.put_ints(idxd, act);
        std::vector<double> shf(k, 0.0);
        for (int q = 0; q < na; ++q) shf[act[q]] = sh[q];
        const double* sd = E.put_doubles(shd, shf);
        diag_pair(de, r1, r2, N, na, N, sd, idx, out, out + (long)na * N, N, E.st);
        return 2 * na;
      }
      DevBuf s1(ctx), s2(ctx), idxd(ctx);
      s1.ensure(sizeof(double) * na * N);
      s2.ensure(sizeof(double) * na * N);
      const int* idx = E.put_ints(idxd, act);
      gather_cols(r1, N, idx, na, N, s1.as<double>(), N, E.st);
      gather_cols(r2, N, idx, na, N, s2.as<double>(), N, E.st);
      InnerResult ir = inner_pair(E, pin, s1.as<double>(), s2.as<double>(), na, sh, o.inner_tol, o.inner_max_iter,
                                  out, out + (long)na * N);
      c.n_inner += ir.n_mv;
      c.n_inner_iter += ir.n_iter;
      return 2 * na;
    };
  }

  zbuf.ensure(sizeof(double) * k * N);
  if (mode == RID_TDA) {
    davidson_sym(E, OPK_A, pout, k, v0.as<double>(), n0, pc, o.tol, o.max_iter, m_max, n_init, zbuf.as<double>(),
                 core, true);
  } else {
    zpbuf.ensure(sizeof(double) * k * N);
    davidson_rpa(E, OPK_PAIR, pout, k, v0.as<double>(), n0, pc, o.tol, o.max_iter, m_max, n_init,
                 zbuf.as<double>(), zpbuf.as<double>(), core, true);
  }
  if (core.status == RID_ERR_BREAKDOWN) throw Error(RID_ERR_BREAKDOWN, "every new direction was dropped");
  st.n_iter = core.n_iter;
  st.n_mv = core.n_mv;
  st.n_inner_mv += core.n_inner;
  st.n_inner_iter += core.n_inner_iter;
  st.history = core.history;
  const int kk = (int)core.omega.size();
  for (int j = 0; j < k; ++j) omega_host[j] = j < kk ? core.omega[j] : NAN;
  if (resid_host)
    for (int j = 0; j < k; ++j) resid_host[j] = j < kk ? core.resid[j] : NAN;
  if (mode == RID_TDA) {
    if (x_dev) RID_HIP(hipMemcpyAsync(x_dev, zbuf.p, sizeof(double) * kk * N, hipMemcpyDeviceToDevice, E.st));
  } else if (x_dev || y_dev) {
    DevBuf half(ctx), mhalf(ctx);
    std::vector<double> hv(kk, 0.5), mv(kk, -0.5);
    const double* h = E.put_doubles(half, hv);
    const double* mh = E.put_doubles(mhalf, mv);
    if (x_dev) axpby_cols(zbuf.as<double>(), zpbuf.as<double>(), N, kk, N, h, h, x_dev, N, E.st);
    if (y_dev) axpby_cols(zbuf.as<double>(), zpbuf.as<double>(), N, kk, N, h, mh, y_dev, N, E.st);
  }
  E.sync();
  st.t_total = ms_since(t_all);
  return core.status;
}

rid_status response_solve(rid_problem* P, const rid_solve_opts& o, int nrhs, const double* p_dev, int nfreq,
                          const double* omega_host, double* alpha_host, double* u_dev, double* resid_host,
                          SolveStats& st, const ExecCfg& ex) {
  validate_opts(o, P);
  RID_CHECK(nrhs >= 1 && nfreq >= 1, RID_ERR_SHAPE, "nrhs and nfreq must be >= 1");
  RID_CHECK(p_dev && omega_host && alpha_host, RID_ERR_INVALID_ARG, "null argument");
  for (int f = 0; f < nfreq; ++f) {
    RID_CHECK(std::isfinite(omega_host[f]) && omega_host[f] >= 0.0, RID_ERR_INVALID_ARG,
              "frequencies must be finite and >= 0");
    RID_CHECK(omega_host[f] < 0.999 * P->de_min, RID_ERR_NEAR_SINGULAR,
              "frequency within the guard of the lowest orbital energy difference");
  }
  auto t_all = Clock::now();
  Eng E(P, &st, ex);
  E.use_graphs = o.graphs != 0;
  rid_context* ctx = P->ctx;
  const long N = P->n();
  const bool ris = o.precond == RID_PRECOND_RIS;
  const int pin = ris_prec(o), pout = outer_prec(o);
  const int npair = nrhs * nfreq;
  const double* de = P->de.as<double>();
  // right-hand side per (frequency, rhs) pair, rhs fastest
  DevBuf rhs(ctx), shd(ctx), zero(ctx), u0(ctx), pn(ctx);
  rhs.ensure(sizeof(double) * npair * N);
  for (int f = 0; f < nfreq; ++f)
    RID_HIP(hipMemcpyAsync(rhs.as<double>() + (long)f * nrhs * N, p_dev, sizeof(double) * nrhs * N,
                           hipMemcpyDeviceToDevice, E.st));
  std::vector<double> sh(npair);
  for (int c = 0; c < npair; ++c) sh[c] = omega_host[c / nrhs];
  const double* shdev = E.put_doubles(shd, sh);
  pn.ensure(sizeof(double) * npair);
  {
    RedScratch rs = E.rs(1, npair);
    col_norms(rhs.as<double>(), N, npair, N, pn.as<double>(), rs, E.st);
  }
  std::vector<double> pnh(npair);
  E.d2h(pnh.data(), pn.as<double>(), sizeof(double) * npair);
  for (double x : pnh) RID_CHECK(x > 0.0 && std::isfinite(x), RID_ERR_INVALID_ARG, "right-hand side is zero");
  // initial subspace: solution of the 2x2 system with right-hand side (-P, 0)
  zero.ensure(sizeof(double) * npair * N);
  RID_HIP(hipMemsetAsync(zero.p, 0, sizeof(double) * npair * N, E.st));
  DevBuf mp(ctx);
  mp.ensure(sizeof(double) * npair * N);
  scale_copy(rhs.as<double>(), (long)npair * N, -1.0, mp.as<double>(), E.st);
  u0.ensure(sizeof(double) * 2 * npair * N);
  auto tp = Clock::now();
  if (!ris) {
    diag_pair(de, mp.as<double>(), zero.as<double>(), N, npair, N, shdev, nullptr, u0.as<double>(),
              u0.as<double>() + (long)npair * N, N, E.st);
  } else {
    InnerResult ir = inner_pair(E, pin, mp.as<double>(), zero.as<double>(), npair, sh, o.init_tol, o.init_max_iter,
                                u0.as<double>(), u0.as<double>() + (long)npair * N);
    st.n_inner_mv += ir.n_mv;
    st.n_inner_iter += ir.n_iter;
  }
  st.t_precond += ms_since(tp);

  Basis B(ctx);
  const int m_max = std::max(default_m_max(npair, o.m_max), 4 * npair + 8);
  B.init(m_max + 4 * npair + 8, N, 2);
  append_orthonormal(E, B, u0.as<double>(), 2 * npair);
  RID_CHECK(B.m > 0, RID_ERR_BREAKDOWN, "initial subspace is empty");
  double tmv = 0.0;
  multiply(E, B, 0, OPK_PAIR, pout, &tmv);
  project(E, B, 0);
  st.n_iter = 1;
  st.n_mv = B.m;
  DevBuf g(ctx), mats(ctx), uu(ctx), uup(ctx), ty(ctx), r1(ctx), r2(ctx), rnd(ctx), wn(ctx), idxd(ctx), sha(ctx);
  uu.ensure(sizeof(double) * npair * N);
  uup.ensure(sizeof(double) * npair * N);
  ty.ensure(sizeof(double) * npair * N);
  r1.ensure(sizeof(double) * npair * N);
  r2.ensure(sizeof(double) * npair * N);
  rnd.ensure(sizeof(double) * 2 * npair);
  wn.ensure(sizeof(double) * 2 * npair * N);
  std::vector<double> rel(npair);
  rid_status status = RID_OK;
  while (true) {
    const int m = B.m, d = 2 * m;
    auto t0 = Clock::now();
    g.ensure(sizeof(double) * (size_t)npair * d);
    mats.ensure(sizeof(double) * (size_t)npair * d * d);
    {
      RedScratch rs = E.rs(npair, m);
      gram(mp.as<double>(), N, npair, B.V(0), N, m, N, g.as<double>(), d, rs, E.st);  // -V^T P
    }
    // lower halves of the right-hand sides are zero
    for (int c = 0; c < npair; ++c)
      RID_HIP(hipMemsetAsync(g.as<double>() + (long)c * d + m, 0, sizeof(double) * m, E.st));
    build_shifted(B.a1.as<double>(), B.a2.as<double>(), m, B.cap, shdev, npair, 1, mats.as<double>(), E.st);
    small_lu_solve_cm(mats.as<double>(), g.as<double>(), d, npair, E.st);  // symmetric systems
    const double* y = g.as<double>();
    const double* yp = g.as<double>() + m;
    combo(B.V(0), N, m, y, 1, d, npair, N, 1.0, 0.0, uu.as<double>(), N, E.st);
    combo(B.V(0), N, m, yp, 1, d, npair, N, 1.0, 0.0, uup.as<double>(), N, E.st);
    // R1 = (A+B) V y - w V y' + P ; R2 = (A-B) V y' - w V y
    combo(B.P1(0), N, m, y, 1, d, npair, N, 1.0, 0.0, ty.as<double>(), N, E.st);
    resid3(ty.as<double>(), uup.as<double>(), mp.as<double>(), N, npair, N, shdev, r1.as<double>(), N, E.st);
    combo(B.P2(0), N, m, yp, 1, d, npair, N, 1.0, 0.0, ty.as<double>(), N, E.st);
    resid3(ty.as<double>(), uu.as<double>(), nullptr, N, npair, N, shdev, r2.as<double>(), N, E.st);
    {
      RedScratch rs = E.rs(1, npair);
      col_norms(r1.as<double>(), N, npair, N, rnd.as<double>(), rs, E.st);
      col_norms(r2.as<double>(), N, npair, N, rnd.as<double>() + npair, rs, E.st);
    }
    std::vector<double> rr(2 * npair);
    E.d2h(rr.data(), rnd.as<double>(), sizeof(double) * 2 * npair);
    st.t_other += ms_since(t0);
    std::vector<int> act;
    double mx = 0.0;
    for (int c = 0; c < npair; ++c) {
      rel[c] = std::sqrt(rr[c] * rr[c] + rr[npair + c] * rr[npair + c]) / pnh[c];
      mx = std::max(mx, rel[c]);
      if (!(rel[c] < o.tol)) act.push_back(c);
    }
    st.history.push_back(mx);
    if (act.empty()) break;
    if (st.n_iter >= o.max_iter) {
      status = RID_WARN_NOT_CONVERGED;
      break;
    }
    const int na = (int)act.size();
    tp = Clock::now();
    std::vector<double> sa(na);
    for (int q = 0; q < na; ++q) sa[q] = sh[act[q]];
    const int* idx = E.put_ints(idxd, act);
    if (!ris) {
      diag_pair(de, r1.as<double>(), r2.as<double>(), N, na, N, shdev, idx, wn.as<double>(),
                wn.as<double>() + (long)na * N, N, E.st);
    } else {
      DevBuf s1(ctx), s2(ctx);
      s1.ensure(sizeof(double) * na * N);
      s2.ensure(sizeof(double) * na * N);
      gather_cols(r1.as<double>(), N, idx, na, N, s1.as<double>(), N, E.st);
      gather_cols(r2.as<double>(), N, idx, na, N, s2.as<double>(), N, E.st);
      InnerResult ir = inner_pair(E, pin, s1.as<double>(), s2.as<double>(), na, sa, o.inner_tol, o.inner_max_iter,
                                  wn.as<double>(), wn.as<double>() + (long)na * N);
      st.n_inner_mv += ir.n_mv;
      st.n_inner_iter += ir.n_iter;
    }
    st.t_precond += ms_since(tp);
    if (B.m + 2 * na > B.cap) {
      status = RID_WARN_NOT_CONVERGED;
      break;
    }
    t0 = Clock::now();
    const int m0 = B.m;
    const int added = append_orthonormal(E, B, wn.as<double>(), 2 * na);
    st.t_other += ms_since(t0);
    if (added == 0) throw Error(RID_ERR_BREAKDOWN, "every new direction was dropped");
    multiply(E, B, m0, OPK_PAIR, pout, &tmv);
    t0 = Clock::now();
    project(E, B, m0);
    st.t_other += ms_since(t0);
    st.n_iter += 1;
    st.n_mv += added;
    E.track(B.bytes() + P->footprint());
  }
  tmv += E.take_product_ms();
  st.t_matvec += tmv;
  // alpha[f][u][v] = -2 P_u^T U_{v,f} = 2 (-P_u)^T U_{v,f}
  DevBuf al(ctx);
  al.ensure(sizeof(double) * nrhs * npair);
  {
    RedScratch rs = E.rs(nrhs, npair);
    gram(mp.as<double>(), N, nrhs, uu.as<double>(), N, npair, N, al.as<double>(), npair, rs, E.st);
  }
  std::vector<double> a((size_t)nrhs * npair);
  E.d2h(a.data(), al.as<double>(), sizeof(double) * a.size());
  for (int f = 0; f < nfreq; ++f)
    for (int u = 0; u < nrhs; ++u)
      for (int v = 0; v < nrhs; ++v)
        alpha_host[((size_t)f * nrhs + u) * nrhs + v] = 2.0 * a[(size_t)u * npair + f * nrhs + v];
  if (resid_host)
    for (int c = 0; c < npair; ++c) resid_host[c] = rel[c];
  if (u_dev) RID_HIP(hipMemcpyAsync(u_dev, uu.p, sizeof(double) * npair * N, hipMemcpyDeviceToDevice, E.st));
  E.sync();
  st.t_total = ms_since(t_all);
  return status;
}

void fill_stats(rid_stats* out, const SolveStats& s) {
  if (!out) return;
  std::memset(out, 0, sizeof(*out));
  out->n_iter = s.n_iter;
  out->n_mv = s.n_mv;
  out->n_inner_mv = s.n_inner_mv;
  out->n_inner_iter = s.n_inner_iter;
  out->n_history = (int32_t)std::min<size_t>(s.history.size(), RID_MAX_HISTORY);
  for (int i = 0; i < out->n_history; ++i) out->history[i] = s.history[i];
  out->t_matvec_ms = s.t_matvec;
  out->t_precond_ms = s.t_precond;
  out->t_total_ms = s.t_total;
  out->t_other_ms = std::max(0.0, s.t_total - s.t_matvec - s.t_precond);
  out->bytes_resident = s.peak_bytes;
  out->n_blocks_cholqr = s.n_blocks_cholqr;
  out->n_blocks_mgs = s.n_blocks_mgs;
}

}  // namespace rid
