// Context memory, problem set-up and the operator driver.
//
// The operator driver evaluates, for a block of vectors X (nvec x N, f64),
//   Coulomb:  t^P_v = sum_ia B^P_ia X_v,ia          (GEMM over i-slices, split)
//             J_v,ia = sum_P B^P_ia t^P_v           (memory-bound kernel)
//   exchange: S^P_(i,v,b) = sum_j B^P_ij Xt_v,b,j    (batched GEMM per P)
//             W_(i,v),a = sum_P sum_b S^P_(i,v),b B^P_ab   (reduction GEMM)
//   pair:     Q^P_(i,v,j) = sum_b B^P_ib Xa_v,j,b    (batched GEMM per P)
//             W'_(i,v),a = sum_P sum_j Q^P_(i,v),j B^P_ja (reduction GEMM)
// and combines de X + c_J J - a_x (W +- W') in f64.  The exchange products are
// taken over the window [i0, i0+no_a) x [0, nv_a) and the leading naux_k
// rows (the full ranges for the outer operator).  The auxiliary index is
// processed in chunks so that the S / Q intermediates stay bounded; every
// chunk adds its split partial sums into the same partial buffers, which the
// combine kernel reduces in f64.
#include <algorithm>
#include <cmath>
#include <cstdlib>

#include "core.hpp"
#include "gemm.hpp"
#include "opkern.hpp"

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
  for (const Rec& r : recs) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
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
  recs.clear();
}

Profiler::~Profiler() {
  for (const Rec& r : recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (hipEvent_t e : pool) (void)hipEventDestroy(e);
}

ProfScope::ProfScope(rid_context* c, const char* name, double fl, double by) : ctx(c), flops(fl), bytes(by) {
  if (!ctx || !ctx->prof.on) return;
  fam = ctx->prof.family(name);
  a = ctx->prof.get_event();
  RID_HIP(hipEventRecord(a, ctx->stream));
}

ProfScope::~ProfScope() {
  if (fam < 0) return;
  hipEvent_t b = nullptr;
  try {
    b = ctx->prof.get_event();
  } catch (...) {
    return;
  }
  (void)hipEventRecord(b, ctx->stream);
  ctx->prof.recs.push_back(Profiler::Rec{fam, a, b, flops, bytes});
}

void* dev_alloc(rid_context* ctx, size_t bytes) {
  if (bytes == 0) bytes = 256;
  void* p = nullptr;
  if (ctx->user_alloc) {
    std::lock_guard<std::mutex> g(ctx->mu);
    p = ctx->alloc.alloc(ctx->alloc.user, bytes);
    RID_CHECK(p != nullptr, RID_ERR_NO_MEMORY, "allocator returned NULL for " + std::to_string(bytes) + " bytes");
  } else {
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      throw Error(RID_ERR_NO_MEMORY, "hipMalloc(" + std::to_string(bytes) + "): " + hipGetErrorString(e));
    }
  }
  return p;
}

void dev_free(rid_context* ctx, void* p) {
  if (!p) return;
  if (ctx->user_alloc) {
    std::lock_guard<std::mutex> g(ctx->mu);
    ctx->alloc.free(ctx->alloc.user, p);
  } else {
    (void)hipFree(p);
  }
}

void DevBuf::release() {
  if (p && ctx) {
    // memory may still be in use by queued work on the context stream
    (void)hipStreamSynchronize(ctx->stream);
    dev_free(ctx, p);
  }
  p = nullptr;
  bytes = 0;
}

void DevBuf::ensure(size_t n) {
  if (n <= bytes && p) return;
  release();
  size_t want = std::max<size_t>(n, 256);
  p = dev_alloc(ctx, want);
  bytes = want;
}

void check_operator(const rid_problem* P, int kind, int prec) {
  RID_CHECK(kind >= OPK_A && kind <= OPK_TPAIR, RID_ERR_INVALID_ARG, "unknown operator");
  RID_CHECK(prec >= PREC_F64 && prec <= PREC_BF16, RID_ERR_INVALID_ARG, "unknown precision");
  const bool ris = kind == OPK_T || kind == OPK_TPAIR;
  if (ris) RID_CHECK(P->naux_ris > 0 && P->bris_ia, RID_ERR_INVALID_ARG, "problem has no ris tensor");
  if (!ris) RID_CHECK(prec != PREC_BF16, RID_ERR_DTYPE, "BF16 is only offered for the ris operators");
}

namespace {

template <typename E>
struct GemmTag {
  typedef E type;
};
template <>
struct GemmTag<uint16_t> {
  typedef bf16_t type;
};

template <typename E>
struct AccOf {
  typedef float type;
};
template <>
struct AccOf<double> {
  typedef double type;
};

// Workgroup slots of the chip per GEMM tile configuration: 256 CUs times the
// workgroups one CU holds at the kernel's register and LDS use
// (cfg 0 = 128x128, 1 = 64x64, 2 = 128x64).
template <typename E>
int gemm_slots(int cfg = 0) {
  static const int f64[3] = {256, 512, 256};
  static const int f32[3] = {512, 1024, 512};
  return sizeof(E) == 8 ? f64[cfg] : f32[cfg];
}

// Split a reduction over np batches (each K deep) into nsub launches of pps
// batches so that the last round of workgroups is as full as possible, while
// keeping each workgroup's reduction deep enough to amortise its epilogue.
struct SplitPlan {
  int nsub, pps;
};

SplitPlan choose_splits(long tiles, int np, int K, int slots, int max_splits = 64) {
  SplitPlan best{1, np};
  double best_score = -1.0;
  for (int ns = 1; ns <= std::min(np, max_splits); ++ns) {
    const int pps = ceil_div(np, ns);
    const int ns2 = ceil_div(np, pps);
    const long total = tiles * ns2;
    const long rounds = (total + slots - 1) / slots;
    const double eff = (double)total / (double)(rounds * slots);
    const double depth = (double)pps * K;
    const double score = eff * depth / (depth + 512.0);
    if (score > best_score + 1e-9) {
      best_score = score;
      best = SplitPlan{ns2, pps};
    }
  }
  return best;
}

struct GemmChoice {
  int cfg, nsub, pps;
};

// Tile configuration and split plan of one launch shape.  reduction: the
// launch sums np batches (split over nsub workgroups per tile); otherwise np
// is 1 and nz independent batches run.
template <typename E>
GemmChoice plan_for(int cfg, long M, long N, int nz, int np, int K, bool reduction) {
  static const int bm[3] = {128, 64, 128}, bn[3] = {128, 64, 64};
  const long tiles = ceil_div_l(M, bm[cfg]) * ceil_div_l(N, bn[cfg]) * nz;
  if (!reduction) return GemmChoice{cfg, 1, np};
  const SplitPlan sp = choose_splits(tiles, np, K, gemm_slots<E>(cfg));
  return GemmChoice{cfg, sp.nsub, sp.pps};
}

bool autotune_enabled() {
  static const bool on = [] {
    const char* e = std::getenv("RID_AUTOTUNE");
    return !(e && e[0] == '0');
  }();
  return on;
}

// Autotuner: the first launch of a shape times every tile configuration
// (each with its own split plan) and keeps the fastest for the context.
// `launch` must be idempotent (GEMM_STORE or GEMM_PARTIAL_SET), so the
// candidate runs leave the same result as a single run of the winner.
template <typename E, typename F>
GemmChoice tuned(rid_context* ctx, int family, long M, long N, int nz, int np, int K, bool reduction, F&& launch) {
  const TuneKey key{family, (int)sizeof(E), M, N, nz, np, K};
  auto it = ctx->tune.find(key);
  if (it != ctx->tune.end()) {
    const GemmChoice ch{it->second.cfg, it->second.nsub, it->second.pps};
    launch(ch);
    return ch;
  }
  GemmChoice best = plan_for<E>(0, M, N, nz, np, K, reduction);
  if (!autotune_enabled()) {
    // without tuning: the 128x128 tile when it fills the chip, else 64x64
    static const int bm = 128;
    const long t128 = ceil_div_l(M, bm) * ceil_div_l(N, bm) * nz * best.nsub;
    if (t128 < gemm_slots<E>(0) / 2) best = plan_for<E>(1, M, N, nz, np, K, reduction);
    launch(best);
  } else {
    hipEvent_t a, b;
    RID_HIP(hipEventCreate(&a));
    RID_HIP(hipEventCreate(&b));
    float best_ms = 1e30f;
    GemmChoice last{};
    for (int cfg = 0; cfg < 3; ++cfg) {
      const GemmChoice ch = plan_for<E>(cfg, M, N, nz, np, K, reduction);
      launch(ch);  // warm
      RID_HIP(hipEventRecord(a, ctx->stream));
      launch(ch);
      RID_HIP(hipEventRecord(b, ctx->stream));
      RID_HIP(hipEventSynchronize(b));
      float ms = 0.0f;
      RID_HIP(hipEventElapsedTime(&ms, a, b));
      if (ms < best_ms) {
        best_ms = ms;
        best = ch;
      }
      last = ch;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (last.cfg != best.cfg) launch(best);
  }
  ctx->tune[key] = TuneVal{best.cfg, best.nsub, best.pps};
  return best;
}

template <typename E>
void run_operator(rid_problem* P, const OpView<E>& ov, bool pair, int nvec, const double* x, double* y,
                  double* y2) {
  typedef typename GemmTag<E>::type G;
  typedef typename AccOf<E>::type Acc;
  hipStream_t st = P->ctx->stream;
  rid_context* ctx = P->ctx;
  const std::string pre = ov.ris ? "ris_" : "";
  const double esz = (double)sizeof(E), asz = (double)sizeof(Acc);
  OpWork& w = P->work;
  const int no = P->no, nv = P->nv;
  const long n = P->n();
  const int no_a = ov.no_a, nv_a = ov.nv_a, i0 = ov.i0;
  const bool exch = P->a_x != 0.0 && ov.naux_k > 0 && no_a > 0 && nv_a > 0;

  // 1. vector layouts in the compute type
  w.xc.ensure(sizeof(E) * nvec * n);
  if (exch) {
    w.xa.ensure(sizeof(E) * (size_t)nvec * no_a * nv_a);
    w.xt.ensure(sizeof(E) * (size_t)nvec * no_a * nv_a);
  }
  prep_x<E>(x, nvec, no, nv, i0, no_a, nv_a, w.xc.as<E>(), exch ? w.xa.as<E>() : nullptr,
            exch ? w.xt.as<E>() : nullptr, st);

  // 2. Coulomb forward: t[v][P] = sum_i sum_a Xc[v][i nv + a] B[P][i nv + a]
  const int naux_j = ov.naux_j;
  double* t64 = nullptr;
  if (naux_j > 0) {
    // partial buffer sized for the largest split count any plan can pick
    w.tpart.ensure(sizeof(Acc) * (size_t)std::min(no, 64) * nvec * naux_j);
    w.t64.ensure(sizeof(double) * (size_t)nvec * naux_j);
    GemmParams g{};
    g.A = w.xc.p;
    g.B = ov.b_ia;
    g.C = w.tpart.p;
    g.M = nvec;
    g.N = naux_j;
    g.K = nv;
    g.np = no;
    g.nz2 = 1;
    g.lda = n;
    g.ldb = n;
    g.ldc = naux_j;
    g.sAp = nv;
    g.sBp = nv;
    g.sCs = (long)nvec * naux_j;
    g.alpha = 1.0;
    g.mode = GEMM_PARTIAL_SET;
    GemmChoice ch;
    {
      ProfScope ps(ctx, (pre + "coul_fwd").c_str(), 2.0 * nvec * naux_j * (double)n,
                   esz * ((double)naux_j * n + (double)nvec * n));
      ch = tuned<E>(ctx, GF_COUL, nvec, naux_j, 1, no, nv, true, [&](const GemmChoice& c) {
        g.pps = c.pps;
        gemm_nt<G>(g, 1, c.nsub, st, c.cfg, GF_COUL);
      });
    }
    const int nsplit = ch.nsub;
    reduce_splits<Acc>(w.tpart.as<Acc>(), nsplit, (long)nvec * naux_j, (long)nvec * naux_j, w.t64.as<double>(), st);
    t64 = w.t64.as<double>();
    w.jbuf.ensure(sizeof(double) * nvec * n);
    {
      ProfScope ps(ctx, (pre + "coul_bwd").c_str(), 2.0 * nvec * naux_j * (double)n,
                   esz * (double)naux_j * n * ceil_div(nvec, 8) + 8.0 * nvec * n);
      coul_bwd<E>(t64, ov.b_ia, naux_j, n, nvec, w.jbuf.as<double>(), st);
    }
  }

  // 3. exchange products, chunked over the auxiliary index
  int ns_w = 0, ns_wp = 0;
  const long rows = (long)no_a * nvec;  // output rows (i, v)
  const long part_elems = rows * nv_a;
  if (exch) {
    const int nk = ov.naux_k;
    const long s_per_p = (long)no_a * nvec * nv_a;
    const long q_per_p = (long)no_a * nvec * no_a;
    const long per_p = std::max(s_per_p, pair ? q_per_p : 0L);
    const long target = 256L << 20;  // bytes of intermediate per chunk
    const int pc = (int)std::max<long>(1, std::min<long>(nk, target / std::max<long>(1, per_p * (long)sizeof(E))));
    int max_splits = 1;
    for (int cfg = 0; cfg < 3; ++cfg) {
      max_splits = std::max(max_splits, plan_for<E>(cfg, rows, nv_a, 1, pc, nv_a, true).nsub);
      max_splits = std::max(max_splits, plan_for<E>(cfg, rows, nv_a, 1, pc, no_a, true).nsub);
    }
    w.s.ensure(sizeof(E) * (size_t)pc * s_per_p);
    w.wpart.ensure(sizeof(Acc) * (size_t)max_splits * part_elems);
    if (pair) {
      w.q.ensure(sizeof(E) * (size_t)pc * q_per_p);
      w.wppart.ensure(sizeof(Acc) * (size_t)max_splits * part_elems);
    }
    GemmChoice cw{}, cwp{};
    for (int c0 = 0; c0 < nk; c0 += pc) {
      const int pcc = std::min(pc, nk - c0);
      const bool first = c0 == 0;
      {  // S^P = B^P_ij (window) x Xt
        GemmParams g{};
        g.A = ov.b_ij + (long)c0 * no * no + (long)i0 * no + i0;
        g.B = w.xt.p;
        g.C = w.s.p;
        g.M = no_a;
        g.N = nvec * nv_a;
        g.K = no_a;
        g.np = 1;
        g.pps = 1;
        g.nz2 = 1;
        g.lda = no;
        g.ldb = no_a;
        g.ldc = (long)nvec * nv_a;
        g.sA1 = (long)no * no;
        g.sC1 = s_per_p;
        g.alpha = 1.0;
        g.mode = GEMM_STORE;
        ProfScope ps(ctx, (pre + "exch_s").c_str(), 2.0 * no_a * (double)nvec * nv_a * no_a * pcc,
                     esz * ((double)pcc * no_a * no_a + (double)nvec * nv_a * no_a + (double)pcc * s_per_p));
        tuned<E>(ctx, GF_EXCH_S, no_a, (long)nvec * nv_a, pcc, 1, no_a, false, [&](const GemmChoice& ch) {
          gemm_nt<G>(g, pcc, 1, st, ch.cfg, GF_EXCH_S);
        });
      }
      {  // W += sum_P S^P B^P_ab (window)
        GemmParams g{};
        g.A = w.s.p;
        g.B = ov.b_ab + (long)c0 * nv * nv;
        g.C = w.wpart.p;
        g.M = (int)rows;
        g.N = nv_a;
        g.K = nv_a;
        g.np = pcc;
        g.nz2 = 1;
        g.lda = nv_a;
        g.ldb = nv;
        g.ldc = nv_a;
        g.sAp = s_per_p;
        g.sBp = (long)nv * nv;
        g.sCs = part_elems;
        g.alpha = 1.0;
        g.mode = first ? GEMM_PARTIAL_SET : GEMM_PARTIAL_ADD;
        ProfScope ps(ctx, (pre + "exch_w").c_str(), 2.0 * rows * (double)nv_a * nv_a * pcc,
                     esz * ((double)pcc * s_per_p + (double)pcc * nv_a * nv_a) +
                         asz * part_elems * (first ? 1.0 : 2.0));
        auto launch = [&](const GemmChoice& ch) {
          g.pps = ch.pps;
          gemm_nt<G>(g, 1, ch.nsub, st, ch.cfg, GF_EXCH_W);
        };
        if (first)
          cw = tuned<E>(ctx, GF_EXCH_W, rows, nv_a, 1, pcc, nv_a, true, launch);
        else
          launch(cw);
      }
      if (pair) {
        {  // Q^P = B^P_ia (window) x Xa^T
          GemmParams g{};
          g.A = ov.b_ia + (long)c0 * n + (long)i0 * nv;
          g.B = w.xa.p;
          g.C = w.q.p;
          g.M = no_a;
          g.N = nvec * no_a;
          g.K = nv_a;
          g.np = 1;
          g.pps = 1;
          g.nz2 = 1;
          g.lda = nv;
          g.ldb = nv_a;
          g.ldc = (long)nvec * no_a;
          g.sA1 = n;
          g.sC1 = q_per_p;
          g.alpha = 1.0;
          g.mode = GEMM_STORE;
          ProfScope ps(ctx, (pre + "exch_q").c_str(), 2.0 * no_a * (double)nvec * no_a * nv_a * pcc,
                       esz * ((double)pcc * no_a * nv_a + (double)nvec * no_a * nv_a + (double)pcc * q_per_p));
          tuned<E>(ctx, GF_EXCH_Q, no_a, (long)nvec * no_a, pcc, 1, nv_a, false, [&](const GemmChoice& ch) {
            gemm_nt<G>(g, pcc, 1, st, ch.cfg, GF_EXCH_Q);
          });
        }
        {  // W' += sum_P Q^P B^P_ja (window), B_ja read from the transposed copy
          GemmParams g{};
          g.A = w.q.p;
          g.B = ov.b_ai + (long)c0 * nv * no + i0;
          g.C = w.wppart.p;
          g.M = (int)rows;
          g.N = nv_a;
          g.K = no_a;
          g.np = pcc;
          g.nz2 = 1;
          g.lda = no_a;
          g.ldb = no;
          g.ldc = nv_a;
          g.sAp = q_per_p;
          g.sBp = (long)nv * no;
          g.sCs = part_elems;
          g.alpha = 1.0;
          g.mode = first ? GEMM_PARTIAL_SET : GEMM_PARTIAL_ADD;
          ProfScope ps(ctx, (pre + "exch_wp").c_str(), 2.0 * rows * (double)nv_a * no_a * pcc,
                       esz * ((double)pcc * q_per_p + (double)pcc * nv_a * no_a) +
                           asz * part_elems * (first ? 1.0 : 2.0));
          auto launch = [&](const GemmChoice& ch) {
            g.pps = ch.pps;
            gemm_nt<G>(g, 1, ch.nsub, st, ch.cfg, GF_EXCH_WP);
          };
          if (first)
            cwp = tuned<E>(ctx, GF_EXCH_WP, rows, nv_a, 1, pcc, no_a, true, launch);
          else
            launch(cwp);
        }
      }
    }
    ns_w = cw.nsub;
    ns_wp = pair ? cwp.nsub : 0;
  }

  // 4. combine in f64
  CombineArgs c{};
  c.x = x;
  c.de = P->de.as<double>();
  c.j = naux_j > 0 ? w.jbuf.as<double>() : nullptr;
  c.y = y;
  c.y2 = y2;
  c.nvec = nvec;
  c.no = no;
  c.nv = nv;
  c.i0 = i0;
  c.no_a = no_a;
  c.nv_a = nv_a;
  c.ns_w = ns_w;
  c.ns_wp = ns_wp;
  c.sstride = part_elems;
  c.cj = pair ? 4.0 : 2.0;
  c.a_x = P->a_x;
  c.pair = pair ? 1 : 0;
  ProfScope ps(ctx, (pre + "combine").c_str(), 0.0,
               8.0 * nvec * n * (pair ? 5.0 : 3.0) + asz * (ns_w + ns_wp) * part_elems);
  combine<Acc>(c, exch ? w.wpart.as<Acc>() : nullptr, (exch && pair) ? w.wppart.as<Acc>() : nullptr, st);
}

}  // namespace

void apply_operator(rid_problem* P, int kind, int prec, int nvec, const double* x, double* y, double* y2) {
  check_operator(P, kind, prec);
  if (nvec <= 0) return;
  const bool ris = kind == OPK_T || kind == OPK_TPAIR;
  const bool pair = kind == OPK_PAIR || kind == OPK_TPAIR;
  // the outer operator uses every row and the full orbital ranges
  const int naux_j = ris ? P->naux_ris : P->naux;
  const int naux_k = ris ? P->naux_ris_k : P->naux;
  const int i0 = ris ? P->i0 : 0;
  const int no_a = ris ? P->no - P->i0 : P->no;
  const int nv_a = ris ? P->nv_act : P->nv;
  if (prec == PREC_F64) {
    P->ensure_f64_aux();
    OpView<double> ov;
    ov.b_ia = ris ? P->bris_ia : P->b_ia;
    ov.b_ij = ris ? P->bris_ij : P->b_ij;
    ov.b_ab = ris ? P->bris_ab : P->b_ab;
    ov.b_ai = ris ? P->bris_ai64.as<double>() : P->b_ai64.as<double>();
    ov.naux_j = naux_j;
    ov.naux_k = naux_k;
    ov.i0 = i0;
    ov.no_a = no_a;
    ov.nv_a = nv_a;
    ov.ris = ris;
    run_operator<double>(P, ov, pair, nvec, x, y, y2);
  } else if (prec == PREC_F32) {
    RID_CHECK(!ris, RID_ERR_DTYPE, "the ris operators run in FP64 or BF16");
    P->ensure_f32();
    OpView<float> ov;
    ov.b_ia = P->b_ia32.as<float>();
    ov.b_ij = P->b_ij32.as<float>();
    ov.b_ab = P->b_ab32.as<float>();
    ov.b_ai = P->b_ai32.as<float>();
    ov.naux_j = naux_j;
    ov.naux_k = naux_k;
    ov.i0 = i0;
    ov.no_a = no_a;
    ov.nv_a = nv_a;
    ov.ris = ris;
    run_operator<float>(P, ov, pair, nvec, x, y, y2);
  } else {
    P->ensure_bf16();
    OpView<uint16_t> ov;
    ov.b_ia = P->bris_ia16.as<uint16_t>();
    ov.b_ij = P->bris_ij16.as<uint16_t>();
    ov.b_ab = P->bris_ab16.as<uint16_t>();
    ov.b_ai = P->bris_ai16.as<uint16_t>();
    ov.naux_j = naux_j;
    ov.naux_k = naux_k;
    ov.i0 = i0;
    ov.no_a = no_a;
    ov.nv_a = nv_a;
    ov.ris = ris;
    run_operator<uint16_t>(P, ov, pair, nvec, x, y, y2);
  }
}

}  // namespace rid

uint64_t rid_problem::footprint() const {
  return de.bytes + b_ai64.bytes + bris_ai64.bytes + b_ia32.bytes + b_ij32.bytes + b_ab32.bytes + b_ai32.bytes +
         bris_ia16.bytes + bris_ij16.bytes + bris_ab16.bytes + bris_ai16.bytes + work.bytes();
}

void rid_problem::ensure_f64_aux() {
  hipStream_t st = ctx->stream;
  if (!b_ai64.p) {
    b_ai64.ensure(sizeof(double) * (size_t)naux * no * nv);
    rid::transpose_slices<double>(b_ia, naux, no, nv, b_ai64.as<double>(), st);
  }
  if (bris_ia && naux_ris_k > 0 && !bris_ai64.p) {
    bris_ai64.ensure(sizeof(double) * (size_t)naux_ris_k * no * nv);
    rid::transpose_slices<double>(bris_ia, naux_ris_k, no, nv, bris_ai64.as<double>(), st);
  }
}

void rid_problem::ensure_f32() {
  hipStream_t st = ctx->stream;
  if (b_ia32.p) return;
  const long n = (long)no * nv;
  b_ia32.ensure(sizeof(float) * naux * n);
  rid::cast_copy<float>(b_ia, naux * n, b_ia32.as<float>(), st);
  b_ij32.ensure(sizeof(float) * (size_t)naux * no * no);
  rid::cast_copy<float>(b_ij, (long)naux * no * no, b_ij32.as<float>(), st);
  b_ab32.ensure(sizeof(float) * (size_t)naux * nv * nv);
  rid::cast_copy<float>(b_ab, (long)naux * nv * nv, b_ab32.as<float>(), st);
  b_ai32.ensure(sizeof(float) * naux * n);
  rid::transpose_slices<float>(b_ia, naux, no, nv, b_ai32.as<float>(), st);
}

void rid_problem::ensure_bf16() {
  hipStream_t st = ctx->stream;
  if (bris_ia16.p) return;
  const long n = (long)no * nv;
  bris_ia16.ensure(2 * naux_ris * n);
  rid::cast_copy<uint16_t>(bris_ia, naux_ris * n, bris_ia16.as<uint16_t>(), st);
  const int nk = std::max(naux_ris_k, 1);
  bris_ij16.ensure(2 * (size_t)nk * no * no);
  bris_ab16.ensure(2 * (size_t)nk * nv * nv);
  bris_ai16.ensure(2 * (size_t)nk * n);
  if (naux_ris_k > 0) {
    rid::cast_copy<uint16_t>(bris_ij, (long)naux_ris_k * no * no, bris_ij16.as<uint16_t>(), st);
    rid::cast_copy<uint16_t>(bris_ab, (long)naux_ris_k * nv * nv, bris_ab16.as<uint16_t>(), st);
    rid::transpose_slices<uint16_t>(bris_ia, naux_ris_k, no, nv, bris_ai16.as<uint16_t>(), st);
  }
}
