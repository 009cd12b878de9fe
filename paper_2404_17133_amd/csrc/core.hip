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
#include <cstdio>
#include <cstdlib>

#include "core.hpp"
#include "gemm.hpp"
#include "opkern.hpp"

namespace rid {

void check_operator(const rid_problem* P, int kind, int prec) {
  RID_CHECK(kind >= OPK_A && kind <= OPK_TPAIR, RID_ERR_INVALID_ARG, "unknown operator");
  RID_CHECK(prec >= PREC_F64 && prec <= PREC_BF16, RID_ERR_INVALID_ARG, "unknown precision");
  const bool ris = kind == OPK_T || kind == OPK_TPAIR;
  if (ris) RID_CHECK(P->has_ris(), RID_ERR_INVALID_ARG, "problem has no ris tensor");
  if (!ris) RID_CHECK(prec != PREC_BF16, RID_ERR_DTYPE, "BF16 is only offered for the ris operators");
  if (prec == PREC_F64)
    RID_CHECK((ris ? P->bris_dt : P->b_dt) == RID_F64, RID_ERR_DTYPE,
              "an FP64 product needs FP64 tensors (the problem was created with FP32 ones)");
  if (ris && P->b_x != 0.0 && P->lr.rows > 0)
    RID_CHECK(P->rislr.rows > 0, RID_ERR_INVALID_ARG,
              "a range-separated problem with a ris tensor needs a long-range ris tensor");
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
  RID_CHECK(cfg >= 0 && cfg < 3, RID_ERR_INTERNAL, "gemm: bad tile configuration");
  return sizeof(E) == 8 ? f64[cfg] : f32[cfg];
}

// Split a reduction over np batches (each K deep) into nsub launches of pps
// batches so that the workgroup slots of the chip are evenly loaded, while
// keeping each workgroup's reduction deep enough to amortise its fixed cost
// (pipeline fill and epilogue).  That cost was measured on the exchange
// shapes of the no=200 workload as about 2 to 5 K stages (65 to 170 FP32
// elements: exch_wp runs at 87 TFLOP/s in 819 tiles of 125 stages and at
// 103 TFLOP/s in 4095 tiles of 25 stages); it is modelled as 4 stages.
struct SplitPlan {
  int nsub, pps;
};

SplitPlan choose_splits(long tiles, int np, int K, int slots, int stage_elems, int max_splits = 64) {
  SplitPlan best{1, np};
  double best_score = -1.0;
  for (int ns = 1; ns <= std::min(np, max_splits); ++ns) {
    const int pps = ceil_div(np, ns);
    const int ns2 = ceil_div(np, pps);
    const long total = tiles * ns2;
    const long rounds = (total + slots - 1) / slots;
    const double eff = (double)total / (double)(rounds * slots);
    const double stages = (double)pps * ceil_div(K, stage_elems);
    const double score = eff * stages / (stages + 4.0);
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
//
// The split plan is the same for every tile configuration (the one that
// suits the 64x64 tile): a tile's sum over its batches runs in the same
// order whatever the tile shape, so with a shared plan the tuner's choice of
// tile, which rests on timings, does not change a single bit of the result,
// and two runs of the same solve agree exactly.
template <typename E>
GemmChoice plan_for(int cfg, long M, long N, int nz, int np, int K, bool reduction, int max_splits = 64) {
  if (!reduction) return GemmChoice{cfg, 1, np};
  constexpr int ref = 1;  // 64x64
  int bm = 0, bn = 0;
  gemm_config_tile<typename GemmTag<E>::type>(ref, &bm, &bn);
  const long tiles = ceil_div_l(M, bm) * ceil_div_l(N, bn) * nz;
  const SplitPlan sp = choose_splits(tiles, np, K, gemm_slots<E>(ref), 128 / (int)sizeof(E), max_splits);
  return GemmChoice{cfg, sp.nsub, sp.pps};
}

// The tile configuration without tuning: 128x128 when it fills the chip,
// 64x64 otherwise.
template <typename E>
GemmChoice default_choice(long M, long N, int nz, int np, int K, bool reduction, int max_splits) {
  GemmChoice best = plan_for<E>(0, M, N, nz, np, K, reduction, max_splits);
  const long t128 = ceil_div_l(M, 128) * ceil_div_l(N, 128) * nz * best.nsub;
  if (t128 < gemm_slots<E>(0) / 2) best = plan_for<E>(1, M, N, nz, np, K, reduction, max_splits);
  return best;
}

// Bytes of exchange intermediate (S^P or Q^P) per chunk of the auxiliary
// index: 256 MB by default (the size of the Infinity Cache), RID_CHUNK_MB
// overrides it (a tuning knob; results do not depend on it beyond rounding
// of the split sums).
long chunk_target_bytes() {
  static const long b = [] {
    const char* e = std::getenv("RID_CHUNK_MB");
    const long mb = e ? std::atol(e) : 0;
    return (mb > 0 && mb <= 65536 ? mb : 256L) << 20;
  }();
  return b;
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
GemmChoice tuned(rid_context* ctx, int family, long M, long N, int nz, int np, int K, bool reduction, hipStream_t st,
                 F&& launch) {
  const TuneKey key{family, (int)sizeof(E), M, N, nz, np, K};
  {
    std::lock_guard<std::mutex> g(ctx->tune_mu);
    auto it = ctx->tune.find(key);
    if (it != ctx->tune.end()) {
      const GemmChoice ch{it->second.cfg, it->second.nsub, it->second.pps};
      launch(ch);
      return ch;
    }
  }
  GemmChoice best = plan_for<E>(0, M, N, nz, np, K, reduction);
  if (!autotune_enabled()) {
    best = default_choice<E>(M, N, nz, np, K, reduction, 64);
    launch(best);
  } else {
    hipEvent_t a, b;
    RID_HIP(hipEventCreate(&a));
    RID_HIP(hipEventCreate(&b));
    float best_ms = 1e30f;
    GemmChoice last{};
    for (int cfg = 0; cfg < gemm_num_configs<typename GemmTag<E>::type>(); ++cfg) {
      const GemmChoice ch = plan_for<E>(cfg, M, N, nz, np, K, reduction);
      launch(ch);  // warm
      // the faster of two timed runs: one run alone is at the mercy of
      // clock ramps and of whatever else shares the device
      float ms = 1e30f;
      for (int rep = 0; rep < 2; ++rep) {
        RID_HIP(hipEventRecord(a, st));
        launch(ch);
        RID_HIP(hipEventRecord(b, st));
        RID_HIP(hipEventSynchronize(b));
        float t = 0.0f;
        RID_HIP(hipEventElapsedTime(&t, a, b));
        ms = std::min(ms, t);
      }
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
  {
    std::lock_guard<std::mutex> g(ctx->tune_mu);
    ctx->tune[key] = TuneVal{best.cfg, best.nsub, best.pps};
  }
  return best;
}

// Lookup of a tuned launch shape (false when it has not been seen).
bool tuned_lookup(rid_context* ctx, const TuneKey& key, GemmChoice* ch) {
  std::lock_guard<std::mutex> g(ctx->tune_mu);
  auto it = ctx->tune.find(key);
  if (it == ctx->tune.end()) return false;
  *ch = GemmChoice{it->second.cfg, it->second.nsub, it->second.pps};
  return true;
}

}  // namespace

// Staging of grouped-GEMM descriptors: slots of pinned host memory and of
// device memory.  A slot is reused once the copy that read it has run.
struct DescRing {
  static constexpr int kSlots = 32, kMembers = 128;
  std::mutex mu;
  DevBuf dev;
  void* host = nullptr;
  size_t slot_bytes = 0;
  hipEvent_t ev[kSlots] = {};
  int next = 0;
  explicit DescRing(rid_context* c) : dev(c) {
    slot_bytes = (gemm_group_desc_bytes(kMembers) + 255) & ~(size_t)255;
    dev.ensure(slot_bytes * kSlots);
    RID_HIP(hipHostMalloc(&host, slot_bytes * kSlots, hipHostMallocDefault));
    for (hipEvent_t& e : ev) RID_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }
  ~DescRing() {
    for (hipEvent_t e : ev)
      if (e) (void)hipEventSynchronize(e);
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
    if (host) (void)hipHostFree(host);
  }
};

namespace {

std::mutex g_ring_mu;

// Launch the members of one stage that share a tile configuration: a plain
// launch for one member, grouped persistent launches otherwise.
template <typename G>
void launch_members(rid_context* ctx, const std::vector<GemmGroup>& mem, int cfg, int family, hipStream_t st,
                    int grid_cap) {
  if (mem.empty()) return;
  if (mem.size() == 1) {
    gemm_nt<G>(mem[0].p, mem[0].nz, mem[0].nsplit, st, cfg, family);
    return;
  }
  // the descriptors go through reused pinned host slots, which a captured
  // graph would read again at every replay: refuse the capture instead
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  RID_HIP(hipStreamIsCapturing(st, &cs));
  RID_CHECK(cs == hipStreamCaptureStatusNone, RID_ERR_INTERNAL, "grouped GEMM launch under graph capture");
  {
    std::lock_guard<std::mutex> g(g_ring_mu);
    if (!ctx->ring) ctx->ring = new DescRing(ctx);
  }
  DescRing& R = *ctx->ring;
  std::lock_guard<std::mutex> g(R.mu);
  for (size_t b = 0; b < mem.size(); b += DescRing::kMembers) {
    const int n = (int)std::min<size_t>(DescRing::kMembers, mem.size() - b);
    const int slot = R.next;
    R.next = (R.next + 1) % DescRing::kSlots;
    RID_HIP(hipEventSynchronize(R.ev[slot]));
    void* h = static_cast<char*>(R.host) + slot * R.slot_bytes;
    void* d = static_cast<char*>(R.dev.p) + slot * R.slot_bytes;
    gemm_grouped<G>(&mem[b], n, cfg, family, d, h, st, grid_cap);
    RID_HIP(hipEventRecord(R.ev[slot], st));
  }
}

// Members of one GEMM stage, by tile configuration.
template <typename E>
struct Stage {
  typedef typename GemmTag<E>::type G;
  static constexpr int kMaxCfgs = 3;  // the most tile configurations of any element type
  std::vector<GemmGroup> mem[kMaxCfgs];
  void add(const GemmParams& p, int nz, const GemmChoice& ch) {
    RID_CHECK(ch.cfg >= 0 && ch.cfg < gemm_num_configs<G>() && ch.cfg < kMaxCfgs, RID_ERR_INTERNAL,
              "gemm: bad tile configuration");
    GemmParams q = p;
    q.pps = ch.pps;
    mem[ch.cfg].push_back(GemmGroup{q, nz, ch.nsub});
  }
  void launch(rid_context* ctx, int family, hipStream_t st) {
    for (int c = 0; c < gemm_num_configs<G>() && c < kMaxCfgs; ++c)
      launch_members<G>(ctx, mem[c], c, family, st, gemm_slots<E>(c));
  }
};

// Either queue p into the stage (shape already tuned) or tune it now, which
// launches it alone.  Returns the choice.
template <typename E>
GemmChoice plan_or_tune(rid_context* ctx, Stage<E>& stage, int family, GemmParams p, long M, long N, int nz, int np,
                        int K, bool reduction, hipStream_t st, const OpLimits* lim) {
  typedef typename GemmTag<E>::type G;
  GemmChoice ch;
  if (lim) {  // fixed scratch: no tuning runs, no shared cache
    ch = default_choice<E>(M, N, nz, np, K, reduction, lim->max_splits);
    stage.add(p, nz, ch);
    return ch;
  }
  const TuneKey key{family, (int)sizeof(E), M, N, nz, np, K};
  if (tuned_lookup(ctx, key, &ch)) {
    stage.add(p, nz, ch);
    return ch;
  }
  return tuned<E>(ctx, family, M, N, nz, np, K, reduction, st, [&](const GemmChoice& c) {
    p.pps = reduction ? c.pps : 1;
    gemm_nt<G>(p, nz, c.nsub, st, c.cfg, family);
  });
}

template <typename E>
OpView<E> make_view(rid_problem* P, bool ris);

void fill_window(rid_problem* P, bool ris, int& naux_j, int& naux_k, int& i0, int& no_a, int& nv_a) {
  // the outer operator uses every row and the full orbital ranges
  naux_j = ris ? P->naux_ris : P->naux;
  naux_k = ris ? P->naux_ris_k : P->naux;
  i0 = ris ? P->i0 : 0;
  no_a = ris ? P->no - P->i0 : P->no;
  nv_a = ris ? P->nv_act : P->nv;
}

template <>
OpView<double> make_view<double>(rid_problem* P, bool ris) {
  P->ensure_f64_aux();
  OpView<double> ov;
  ov.b_ia = ris ? P->bris_ia : P->b_ia;
  ov.b_ij = ris ? P->bris_ij : P->b_ij;
  ov.b_ab = ris ? P->bris_ab : P->b_ab;
  ov.b_ai = ris ? P->bris_ai64.as<double>() : P->b_ai64.as<double>();
  const LrSet& L = ris ? P->rislr : P->lr;
  if (L.rows > 0 && P->b_x != 0.0) {
    ov.lr_ia = L.ia;
    ov.lr_ij = L.ij;
    ov.lr_ab = L.ab;
    ov.lr_ai = L.ai64.as<double>();
    ov.naux_lr = L.rows;
  }
  fill_window(P, ris, ov.naux_j, ov.naux_k, ov.i0, ov.no_a, ov.nv_a);
  ov.ax = P->a_x;
  ov.bx = P->b_x;
  ov.ris = ris;
  return ov;
}

template <>
OpView<float> make_view<float>(rid_problem* P, bool ris) {
  RID_CHECK(!ris, RID_ERR_DTYPE, "the ris operators run in FP64 or BF16");
  P->ensure_f32();
  OpView<float> ov;
  ov.b_ia = P->ia32();
  ov.b_ij = P->ij32();
  ov.b_ab = P->ab32();
  ov.b_ai = P->b_ai32.as<float>();
  if (P->lr.rows > 0 && P->b_x != 0.0) {
    ov.lr_ia = P->lr.ia32v();
    ov.lr_ij = P->lr.ij32v();
    ov.lr_ab = P->lr.ab32v();
    ov.lr_ai = P->lr.ai32.as<float>();
    ov.naux_lr = P->lr.rows;
  }
  fill_window(P, ris, ov.naux_j, ov.naux_k, ov.i0, ov.no_a, ov.nv_a);
  ov.ax = P->a_x;
  ov.bx = P->b_x;
  ov.ris = ris;
  return ov;
}

template <>
OpView<uint16_t> make_view<uint16_t>(rid_problem* P, bool ris) {
  P->ensure_bf16();
  OpView<uint16_t> ov;
  ov.b_ia = P->bris_ia16.as<uint16_t>();
  ov.b_ij = P->bris_ij16.as<uint16_t>();
  ov.b_ab = P->bris_ab16.as<uint16_t>();
  ov.b_ai = P->bris_ai16.as<uint16_t>();
  if (P->rislr.rows > 0 && P->b_x != 0.0) {
    ov.lr_ia = P->rislr.ia16.as<uint16_t>();
    ov.lr_ij = P->rislr.ij16.as<uint16_t>();
    ov.lr_ab = P->rislr.ab16.as<uint16_t>();
    ov.lr_ai = P->rislr.ai16.as<uint16_t>();
    ov.naux_lr = P->rislr.rows;
  }
  fill_window(P, ris, ov.naux_j, ov.naux_k, ov.i0, ov.no_a, ov.nv_a);
  ov.ax = P->a_x;
  ov.bx = P->b_x;
  ov.ris = ris;
  return ov;
}

// Per-job quantities of one product.
template <typename E>
struct JobPlan {
  OpJob* j = nullptr;
  OpView<E> ov;
  bool pair = false, exch = false;
  int no = 0, nv = 0, no_a = 0, nv_a = 0, i0 = 0, naux_j = 0, nk = 0, pc = 1, nchunks = 0, nvec = 0;
  int nk_lr = 0, nch_sr = 0;  // long-range rows; chunks of the first (a_x) part
  // K extent of the contractions over the active virtuals: nv_a rounded up
  // to a whole 16-byte chunk when that stays inside a row of B (the extra
  // columns meet zeros in the padded vector layouts), so that they can use
  // 16-byte loads; nv_a otherwise.
  int kv = 0;

  // Chunk c of the exchange: rows [c0, c0 + pcc) of the a_x-weighted tensor
  // (chunks [0, nch_sr)) or of the long-range b_x-weighted one (after).
  struct Chunk {
    const E *ia, *ij, *ab, *ai;
    int c0, pcc;
    double w;
  };
  Chunk chunk(int c) const {
    if (c < nch_sr) {
      const int c0 = c * pc;
      return Chunk{ov.b_ia, ov.b_ij, ov.b_ab, ov.b_ai, c0, std::min(pc, nk - c0), ov.ax};
    }
    const int c0 = (c - nch_sr) * pc;
    return Chunk{ov.lr_ia, ov.lr_ij, ov.lr_ab, ov.lr_ai, c0, std::min(pc, nk_lr - c0), ov.bx};
  }
  long n = 0, rows = 0, part_elems = 0, s_per_p = 0, q_per_p = 0;
  GemmChoice cw{}, cwp{};
  // S^P and Q^P of a chunk as one product over the stacked rows (P, i):
  // possible when the window spans all occupieds, so that those rows of
  // B_ij and B_ia are evenly spaced.
  bool stacked() const { return i0 == 0 && no_a == no; }
  int ns_coul = 1;
};

// Products of jobs that share element type E and operator (outer or ris).
template <typename E>
void run_group(rid_context* ctx, const std::vector<OpJob*>& jobs, bool ris, hipStream_t st, const OpLimits* lim) {
  typedef typename AccOf<E>::type Acc;
  const std::string pre = ris ? "ris_" : "";
  const double esz = (double)sizeof(E), asz = (double)sizeof(Acc);
  std::vector<JobPlan<E>> pl(jobs.size());
  // a product under fixed limits records no profiling events
  rid_context* pctx = lim ? nullptr : ctx;
  const int split_cap = lim ? lim->max_splits : 64;

  // 1. plans and every scratch buffer of every job (all sized before the
  // first launch, so that a fixed region too small fails before any work),
  // then the vector layouts in the compute type
  {
    ProfScope ps(pctx, st, (pre + "prep").c_str(), 0.0, 0.0);
    for (size_t q = 0; q < jobs.size(); ++q) {
      JobPlan<E>& J = pl[q];
      OpJob* j = jobs[q];
      rid_problem* P = j->P;
      J.j = j;
      J.ov = make_view<E>(P, ris);
      J.pair = j->kind == OPK_PAIR || j->kind == OPK_TPAIR;
      J.no = P->no;
      J.nv = P->nv;
      J.n = P->n();
      J.nvec = j->nvec;
      J.no_a = J.ov.no_a;
      J.nv_a = J.ov.nv_a;
      J.i0 = J.ov.i0;
      J.naux_j = J.ov.naux_j;
      const int nk_sr = P->a_x != 0.0 ? J.ov.naux_k : 0;
      const int nk_lr = J.ov.bx != 0.0 ? J.ov.naux_lr : 0;
      J.exch = nk_sr + nk_lr > 0 && J.no_a > 0 && J.nv_a > 0;
      {
        const int vw = 16 / (int)sizeof(E);
        const int up = ceil_div(J.nv_a, vw) * vw;
        J.kv = up <= J.nv ? up : J.nv_a;
      }
      OpWork& w = *j->work;
      w.xc.ensure(sizeof(E) * J.nvec * J.n);
      if (J.exch) {
        w.xa.ensure(sizeof(E) * (size_t)J.nvec * J.no_a * J.kv);
        w.xt.ensure(sizeof(E) * (size_t)J.nvec * J.no_a * J.kv);
      }
      if (J.naux_j > 0) {
        // Coulomb: partial sums for the largest split count any plan can
        // pick, the reduced t, J and the partials of its P ranges
        w.tpart.ensure(sizeof(Acc) * (size_t)std::min(J.no, split_cap) * J.nvec * J.naux_j);
        w.t64.ensure(sizeof(double) * (size_t)J.nvec * J.naux_j);
        w.jbuf.ensure(sizeof(double) * J.nvec * J.n);
        const int ns = coul_bwd_splits(J.n, J.nvec, J.naux_j);
        if (ns > 1) w.jpart.ensure(sizeof(double) * (size_t)ns * J.nvec * J.n);
      }
      J.rows = (long)J.no_a * J.nvec;  // exchange output rows (i, v)
      J.part_elems = J.rows * J.nv_a;
      if (J.exch) {
        J.nk = nk_sr;
        J.nk_lr = nk_lr;
        J.s_per_p = (long)J.no_a * J.nvec * J.kv;
        J.q_per_p = (long)J.no_a * J.nvec * J.no_a;
        const long per_p = std::max(J.s_per_p, J.pair ? J.q_per_p : 0L);
        // bytes of intermediate per chunk of the auxiliary index
        const long target = lim ? lim->chunk_bytes : chunk_target_bytes();
        J.pc = (int)std::max<long>(1, std::min<long>(std::max(J.nk, J.nk_lr),
                                                      target / std::max<long>(1, per_p * (long)sizeof(E))));
        J.nch_sr = ceil_div(J.nk, J.pc);
        J.nchunks = J.nch_sr + ceil_div(J.nk_lr, J.pc);
        int max_splits = 1;
        for (int cfg = 0; cfg < gemm_num_configs<typename GemmTag<E>::type>(); ++cfg) {
          max_splits = std::max(max_splits, plan_for<E>(cfg, J.rows, J.nv_a, 1, J.pc, J.kv, true, split_cap).nsub);
          max_splits = std::max(max_splits, plan_for<E>(cfg, J.rows, J.nv_a, 1, J.pc, J.no_a, true, split_cap).nsub);
        }
        w.s.ensure(sizeof(E) * (size_t)J.pc * J.s_per_p);
        w.wpart.ensure(sizeof(Acc) * (size_t)max_splits * J.part_elems);
        if (J.pair) {
          w.q.ensure(sizeof(E) * (size_t)J.pc * J.q_per_p);
          w.wppart.ensure(sizeof(Acc) * (size_t)max_splits * J.part_elems);
        }
      }
    }
  }

  {
    ProfScope ps(pctx, st, (pre + "prep").c_str(), 0.0, 0.0);
    for (JobPlan<E>& J : pl) {
      OpWork& w = *J.j->work;
      prep_x<E>(J.j->x, J.nvec, J.no, J.nv, J.i0, J.no_a, J.nv_a, J.kv, w.xc.as<E>(), J.exch ? w.xa.as<E>() : nullptr,
                J.exch ? w.xt.as<E>() : nullptr, st);
    }
  }

  // 2. Coulomb forward: t[v][P] = sum_i sum_a Xc[v][i nv + a] B[P][i nv + a]
  {
    Stage<E> stage;
    ProfScope ps(pctx, st, (pre + "coul_fwd").c_str(), 0.0, 0.0);
    for (JobPlan<E>& J : pl) {
      if (J.naux_j <= 0) continue;
      OpWork& w = *J.j->work;
      GemmParams g{};
      g.A = w.xc.p;
      g.B = J.ov.b_ia;
      g.C = w.tpart.p;
      g.M = J.nvec;
      g.N = J.naux_j;
      g.K = J.nv;
      g.np = J.no;
      g.pps = 1;
      g.nz2 = 1;
      g.lda = J.n;
      g.ldb = J.n;
      g.ldc = J.naux_j;
      g.sAp = J.nv;
      g.sBp = J.nv;
      g.sCs = (long)J.nvec * J.naux_j;
      g.alpha = 1.0;
      g.mode = GEMM_PARTIAL_SET;
      ps.flops += 2.0 * J.nvec * J.naux_j * (double)J.n;
      ps.bytes += esz * ((double)J.naux_j * J.n + (double)J.nvec * J.n);
      J.ns_coul = plan_or_tune<E>(ctx, stage, GF_COUL, g, J.nvec, J.naux_j, 1, J.no, J.nv, true, st, lim).nsub;
    }
    stage.launch(ctx, GF_COUL, st);
  }
  {
    ProfScope ps(pctx, st, (pre + "coul_bwd").c_str(), 0.0, 0.0);
    for (JobPlan<E>& J : pl) {
      if (J.naux_j <= 0) continue;
      OpWork& w = *J.j->work;
      reduce_splits<Acc>(w.tpart.as<Acc>(), J.ns_coul, (long)J.nvec * J.naux_j, (long)J.nvec * J.naux_j,
                         w.t64.as<double>(), st);
      const int ns = coul_bwd_splits(J.n, J.nvec, J.naux_j);
      coul_bwd<E>(w.t64.as<double>(), J.ov.b_ia, J.naux_j, J.n, J.nvec, w.jbuf.as<double>(),
                  ns > 1 ? w.jpart.as<double>() : nullptr, ns > 1 ? w.jpart.bytes / sizeof(double) : 0, st);
      ps.flops += 2.0 * J.nvec * J.naux_j * (double)J.n;
      ps.bytes += esz * (double)J.naux_j * J.n * (J.nvec <= 16 ? 1 : ceil_div(J.nvec, 24)) + 8.0 * J.nvec * J.n;
    }
  }

  // 3. exchange products, chunked over the auxiliary index; chunk c of every
  // job goes out in the same grouped launches
  int max_chunks = 0;
  bool any_pair = false;
  for (const JobPlan<E>& J : pl) {
    if (!J.exch) continue;
    max_chunks = std::max(max_chunks, J.nchunks);
    any_pair = any_pair || J.pair;
  }
  for (int c = 0; c < max_chunks; ++c) {
    {  // S^P = B^P_ij (window) x Xt
      Stage<E> stage;
      ProfScope ps(pctx, st, (pre + "exch_s").c_str(), 0.0, 0.0);
      for (JobPlan<E>& J : pl) {
        if (!J.exch || c >= J.nchunks) continue;
        const typename JobPlan<E>::Chunk ck = J.chunk(c);
        const int c0 = ck.c0, pcc = ck.pcc;
        OpWork& w = *J.j->work;
        GemmParams g{};
        g.B = w.xt.p;
        g.C = w.s.p;
        g.N = J.nvec * J.kv;
        g.K = J.no_a;
        g.pps = 1;
        g.nz2 = 1;
        g.lda = J.no;
        g.ldb = J.no_a;
        g.ldc = (long)J.nvec * J.kv;
        g.sBp = 0;
        g.alpha = 1.0;
        ps.flops += 2.0 * J.no_a * (double)J.nvec * J.nv_a * J.no_a * pcc;
        ps.bytes += esz * ((double)pcc * J.no_a * J.no_a + (double)J.nvec * J.nv_a * J.no_a + (double)pcc * J.s_per_p);
        if (J.stacked()) {
          // all occupieds active: the rows (P, i) of the chunk's B^P_ij are
          // contiguous, so the chunk is one product with pcc * no rows, and
          // S^P lands in its per-P layout (no tile padding per P)
          g.A = ck.ij + (long)c0 * J.no * J.no;
          g.M = pcc * J.no;
          g.np = 1;
          g.mode = GEMM_STORE;
          g.order = ORDER_MN;
          plan_or_tune<E>(ctx, stage, GF_EXCH_S, g, g.M, g.N, 1, 1, J.no_a, true, st, lim);
        } else {
          // one product per P, run back to back per workgroup (Xt shared)
          g.A = ck.ij + (long)c0 * J.no * J.no + (long)J.i0 * J.no + J.i0;
          g.M = J.no_a;
          g.np = pcc;
          g.sAp = (long)J.no * J.no;
          g.sCs = J.s_per_p;
          g.mode = GEMM_STORE_EACH;
          g.order = ORDER_ZIN;  // each XCD keeps its share of Xt in L2 across all P
          plan_or_tune<E>(ctx, stage, GF_EXCH_S, g, J.no_a, (long)J.nvec * J.kv, 1, pcc, J.no_a, true, st, lim);
        }
      }
      stage.launch(ctx, GF_EXCH_S, st);
    }
    {  // W += sum_P S^P B^P_ab (window)
      Stage<E> stage;
      ProfScope ps(pctx, st, (pre + "exch_w").c_str(), 0.0, 0.0);
      for (JobPlan<E>& J : pl) {
        if (!J.exch || c >= J.nchunks) continue;
        const typename JobPlan<E>::Chunk ck = J.chunk(c);
        const int c0 = ck.c0, pcc = ck.pcc;
        const bool first = c == 0;
        OpWork& w = *J.j->work;
        GemmParams g{};
        g.A = w.s.p;
        g.B = ck.ab + (long)c0 * J.nv * J.nv;
        g.C = w.wpart.p;
        g.M = (int)J.rows;
        g.N = J.nv_a;
        g.K = J.kv;
        g.np = pcc;
        g.pps = 1;
        g.nz2 = 1;
        g.lda = J.kv;
        g.ldb = J.nv;
        g.ldc = J.nv_a;
        g.sAp = J.s_per_p;
        g.sBp = (long)J.nv * J.nv;
        g.sCs = J.part_elems;
        g.alpha = ck.w;  // the exchange weight (a_x or b_x) is applied here
        g.mode = first ? GEMM_PARTIAL_SET : GEMM_PARTIAL_ADD;
        g.order = ORDER_NM;  // a row block of S^P meets every column block of B^P_ab in L2
        ps.flops += 2.0 * J.rows * (double)J.nv_a * J.nv_a * pcc;
        ps.bytes += esz * ((double)pcc * J.s_per_p + (double)pcc * J.nv_a * J.nv_a) +
                    asz * J.part_elems * (first ? 1.0 : 2.0);
        if (first)
          J.cw = plan_or_tune<E>(ctx, stage, GF_EXCH_W, g, J.rows, J.nv_a, 1, pcc, J.kv, true, st, lim);
        else
          stage.add(g, 1, J.cw);
      }
      stage.launch(ctx, GF_EXCH_W, st);
    }
    if (!any_pair) continue;
    {  // Q^P = B^P_ia (window) x Xa^T
      Stage<E> stage;
      ProfScope ps(pctx, st, (pre + "exch_q").c_str(), 0.0, 0.0);
      for (JobPlan<E>& J : pl) {
        if (!J.exch || !J.pair || c >= J.nchunks) continue;
        const typename JobPlan<E>::Chunk ck = J.chunk(c);
        const int c0 = ck.c0, pcc = ck.pcc;
        OpWork& w = *J.j->work;
        GemmParams g{};
        g.B = w.xa.p;
        g.C = w.q.p;
        g.N = J.nvec * J.no_a;
        g.K = J.kv;
        g.pps = 1;
        g.nz2 = 1;
        g.lda = J.nv;
        g.ldb = J.kv;
        g.ldc = (long)J.nvec * J.no_a;
        g.sBp = 0;
        g.alpha = 1.0;
        ps.flops += 2.0 * J.no_a * (double)J.nvec * J.no_a * J.nv_a * pcc;
        ps.bytes += esz * ((double)pcc * J.no_a * J.nv_a + (double)J.nvec * J.no_a * J.nv_a + (double)pcc * J.q_per_p);
        if (J.stacked()) {
          // rows (P, i) of the chunk's B^P_ia are contiguous: one product
          g.A = ck.ia + (long)c0 * J.n;
          g.M = pcc * J.no;
          g.np = 1;
          g.mode = GEMM_STORE;
          g.order = ORDER_MN;
          plan_or_tune<E>(ctx, stage, GF_EXCH_Q, g, g.M, g.N, 1, 1, J.kv, true, st, lim);
        } else {
          g.A = ck.ia + (long)c0 * J.n + (long)J.i0 * J.nv;
          g.M = J.no_a;
          g.np = pcc;
          g.sAp = J.n;
          g.sCs = J.q_per_p;
          g.mode = GEMM_STORE_EACH;
          g.order = ORDER_ZIN;
          plan_or_tune<E>(ctx, stage, GF_EXCH_Q, g, J.no_a, (long)J.nvec * J.no_a, 1, pcc, J.kv, true, st, lim);
        }
      }
      stage.launch(ctx, GF_EXCH_Q, st);
    }
    {  // W' += sum_P Q^P B^P_ja (window), B_ja read from the transposed copy
      Stage<E> stage;
      ProfScope ps(pctx, st, (pre + "exch_wp").c_str(), 0.0, 0.0);
      for (JobPlan<E>& J : pl) {
        if (!J.exch || !J.pair || c >= J.nchunks) continue;
        const typename JobPlan<E>::Chunk ck = J.chunk(c);
        const int c0 = ck.c0, pcc = ck.pcc;
        const bool first = c == 0;
        OpWork& w = *J.j->work;
        GemmParams g{};
        g.A = w.q.p;
        g.B = ck.ai + (long)c0 * J.nv * J.no + J.i0;
        g.C = w.wppart.p;
        g.M = (int)J.rows;
        g.N = J.nv_a;
        g.K = J.no_a;
        g.np = pcc;
        g.pps = 1;
        g.nz2 = 1;
        g.lda = J.no_a;
        g.ldb = J.no;
        g.ldc = J.nv_a;
        g.sAp = J.q_per_p;
        g.sBp = (long)J.nv * J.no;
        g.sCs = J.part_elems;
        g.alpha = ck.w;
        g.mode = first ? GEMM_PARTIAL_SET : GEMM_PARTIAL_ADD;
        g.order = ORDER_NM;
        ps.flops += 2.0 * J.rows * (double)J.nv_a * J.no_a * pcc;
        ps.bytes += esz * ((double)pcc * J.q_per_p + (double)pcc * J.nv_a * J.no_a) +
                    asz * J.part_elems * (first ? 1.0 : 2.0);
        if (first)
          J.cwp = plan_or_tune<E>(ctx, stage, GF_EXCH_WP, g, J.rows, J.nv_a, 1, pcc, J.no_a, true, st, lim);
        else
          stage.add(g, 1, J.cwp);
      }
      stage.launch(ctx, GF_EXCH_WP, st);
    }
  }

  // 4. combine in f64
  ProfScope ps(pctx, st, (pre + "combine").c_str(), 0.0, 0.0);
  for (JobPlan<E>& J : pl) {
    OpJob* j = J.j;
    OpWork& w = *j->work;
    const int ns_w = J.exch ? J.cw.nsub : 0;
    const int ns_wp = (J.exch && J.pair) ? J.cwp.nsub : 0;
    CombineArgs cb{};
    cb.x = j->x;
    cb.de = j->P->de.as<double>();
    cb.j = J.naux_j > 0 ? w.jbuf.as<double>() : nullptr;
    cb.y = j->y;
    cb.y2 = j->y2;
    cb.nvec = J.nvec;
    cb.no = J.no;
    cb.nv = J.nv;
    cb.i0 = J.i0;
    cb.no_a = J.no_a;
    cb.nv_a = J.nv_a;
    cb.ns_w = ns_w;
    cb.ns_wp = ns_wp;
    cb.sstride = J.part_elems;
    cb.cj = J.pair ? 4.0 : 2.0;
    cb.a_x = 1.0;  // the exchange partial sums carry their weights
    cb.pair = J.pair ? 1 : 0;
    ps.bytes += 8.0 * J.nvec * J.n * (J.pair ? 5.0 : 3.0) + asz * (ns_w + ns_wp) * J.part_elems;
    combine<Acc>(cb, J.exch ? w.wpart.as<Acc>() : nullptr, (J.exch && J.pair) ? w.wppart.as<Acc>() : nullptr, st);
  }
}

}  // namespace

void prepare_problem(rid_problem* P, const rid_solve_opts& o) {
  const bool mixed = o.precision == RID_PRECISION_MIXED;
  const bool ris = o.precond == RID_PRECOND_RIS && P->has_ris();
  if (mixed) {
    P->ensure_f32();
    if (ris) P->ensure_bf16();
  } else {
    if (P->b_dt == RID_F64) P->ensure_f64_aux();
  }
}

void run_jobs(rid_context* ctx, OpJob* const* jobs, int n, hipStream_t st, const OpLimits* lim) {
  for (int prec = PREC_F64; prec <= PREC_BF16; ++prec)
    for (int r = 0; r < 2; ++r) {
      const bool ris = r == 1;
      std::vector<OpJob*> sel;
      for (int i = 0; i < n; ++i) {
        OpJob* j = jobs[i];
        const bool jr = j->kind == OPK_T || j->kind == OPK_TPAIR;
        if (j->prec == prec && jr == ris && j->nvec > 0) sel.push_back(j);
      }
      if (sel.empty()) continue;
      if (prec == PREC_F64)
        run_group<double>(ctx, sel, ris, st, lim);
      else if (prec == PREC_F32)
        run_group<float>(ctx, sel, ris, st, lim);
      else
        run_group<uint16_t>(ctx, sel, ris, st, lim);
    }
}

void apply_operator(rid_problem* P, int kind, int prec, int nvec, const double* x, double* y, double* y2) {
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
  j.work = &P->work;
  j.stream = P->ctx->stream;
  OpJob* jp = &j;
  run_jobs(P->ctx, &jp, 1, P->ctx->stream);
}

bool operator_copies_ready(const rid_problem* P, int kind, int prec) {
  const bool ris = kind == OPK_T || kind == OPK_TPAIR;
  if (prec == PREC_BF16) return P->bris_ia16.p != nullptr;
  if (prec == PREC_F32) return P->b_ai32.p != nullptr;
  // FP64: the transposed copies ensure_f64_aux makes
  if (!ris) {
    if (P->b_dt == RID_F64 && !P->b_ai64.p) return false;
    if (P->lr.rows > 0 && P->lr.dt == RID_F64 && !P->lr.ai64.p) return false;
    return true;
  }
  if (P->bris_dt == RID_F64 && P->bris_ia && P->naux_ris_k > 0 && !P->bris_ai64.p) return false;
  if (P->rislr.rows > 0 && P->rislr.dt == RID_F64 && !P->rislr.ai64.p) return false;
  return true;
}

void apply_operator_fixed(rid_problem* P, int kind, int prec, int nvec, const double* x, double* y, double* y2,
                          Arena& arena, const OpLimits& lim) {
  check_operator(P, kind, prec);
  RID_CHECK(operator_copies_ready(P, kind, prec), RID_ERR_INVALID_ARG,
            "the problem's tensor copies for this operator and precision are not made yet (a first "
            "rid_apply_operator or solve in this precision makes them)");
  if (nvec <= 0) return;
  OpWork work(&arena);
  OpJob j;
  j.P = P;
  j.kind = kind;
  j.prec = prec;
  j.nvec = nvec;
  j.x = x;
  j.y = y;
  j.y2 = y2;
  j.work = &work;
  j.stream = P->ctx->stream;
  OpJob* jp = &j;
  run_jobs(P->ctx, &jp, 1, P->ctx->stream, &lim);
}

}  // namespace rid

uint64_t rid_problem::footprint() const {
  return de.bytes + b_ai64.bytes + bris_ai64.bytes + b_ia32.bytes + b_ij32.bytes + b_ab32.bytes + b_ai32.bytes +
         bris_ia16.bytes + bris_ij16.bytes + bris_ab16.bytes + bris_ai16.bytes + work.bytes() + lr.bytes() +
         rislr.bytes();
}

void rid_problem::ensure_f64_aux() {
  std::lock_guard<std::mutex> g(mu);
  hipStream_t st = ctx->stream;
  bool work = false;
  if (b_dt == RID_F64 && !b_ai64.p) {
    b_ai64.ensure(sizeof(double) * (size_t)naux * no * nv);
    rid::transpose_slices<double, double>(b_ia, naux, no, nv, b_ai64.as<double>(), st);
    work = true;
  }
  if (bris_dt == RID_F64 && bris_ia && naux_ris_k > 0 && !bris_ai64.p) {
    bris_ai64.ensure(sizeof(double) * (size_t)naux_ris_k * no * nv);
    rid::transpose_slices<double, double>(bris_ia, naux_ris_k, no, nv, bris_ai64.as<double>(), st);
    work = true;
  }
  for (rid::LrSet* L : {&lr, &rislr}) {
    if (L->rows > 0 && L->dt == RID_F64 && !L->ai64.p) {
      L->ai64.ensure(sizeof(double) * (size_t)L->rows * no * nv);
      rid::transpose_slices<double, double>(L->ia, L->rows, no, nv, L->ai64.as<double>(), st);
      work = true;
    }
  }
  // the copies are read from other streams too
  if (work) RID_HIP(hipStreamSynchronize(st));
}

void rid_problem::ensure_f32() {
  std::lock_guard<std::mutex> g(mu);
  hipStream_t st = ctx->stream;
  if (b_ai32.p) return;
  const long n = (long)no * nv;
  if (b_dt == RID_F64) {
    b_ia32.ensure(sizeof(float) * naux * n);
    rid::cast_copy<double, float>(b_ia, naux * n, b_ia32.as<float>(), st);
    b_ij32.ensure(sizeof(float) * (size_t)naux * no * no);
    rid::cast_copy<double, float>(b_ij, (long)naux * no * no, b_ij32.as<float>(), st);
    b_ab32.ensure(sizeof(float) * (size_t)naux * nv * nv);
    rid::cast_copy<double, float>(b_ab, (long)naux * nv * nv, b_ab32.as<float>(), st);
    b_ai32.ensure(sizeof(float) * naux * n);
    rid::transpose_slices<double, float>(b_ia, naux, no, nv, b_ai32.as<float>(), st);
  } else {
    b_ai32.ensure(sizeof(float) * naux * n);
    rid::transpose_slices<float, float>(b_ia_f, naux, no, nv, b_ai32.as<float>(), st);
  }
  if (lr.rows > 0) {
    const long r = lr.rows;
    if (lr.dt == RID_F64) {
      lr.ia32.ensure(sizeof(float) * r * n);
      rid::cast_copy<double, float>(lr.ia, r * n, lr.ia32.as<float>(), st);
      lr.ij32.ensure(sizeof(float) * (size_t)r * no * no);
      rid::cast_copy<double, float>(lr.ij, r * no * no, lr.ij32.as<float>(), st);
      lr.ab32.ensure(sizeof(float) * (size_t)r * nv * nv);
      rid::cast_copy<double, float>(lr.ab, r * nv * nv, lr.ab32.as<float>(), st);
      lr.ai32.ensure(sizeof(float) * r * n);
      rid::transpose_slices<double, float>(lr.ia, lr.rows, no, nv, lr.ai32.as<float>(), st);
    } else {
      lr.ai32.ensure(sizeof(float) * r * n);
      rid::transpose_slices<float, float>(lr.ia_f, lr.rows, no, nv, lr.ai32.as<float>(), st);
    }
  }
  RID_HIP(hipStreamSynchronize(st));
}

void rid_problem::ensure_bf16() {
  std::lock_guard<std::mutex> g(mu);
  hipStream_t st = ctx->stream;
  if (bris_ia16.p) return;
  const long n = (long)no * nv;
  const int nk = std::max(naux_ris_k, 1);
  bris_ia16.ensure(2 * naux_ris * n);
  bris_ij16.ensure(2 * (size_t)nk * no * no);
  bris_ab16.ensure(2 * (size_t)nk * nv * nv);
  bris_ai16.ensure(2 * (size_t)nk * n);
  if (bris_dt == RID_F64) {
    rid::cast_copy<double, uint16_t>(bris_ia, naux_ris * n, bris_ia16.as<uint16_t>(), st);
    if (naux_ris_k > 0) {
      rid::cast_copy<double, uint16_t>(bris_ij, (long)naux_ris_k * no * no, bris_ij16.as<uint16_t>(), st);
      rid::cast_copy<double, uint16_t>(bris_ab, (long)naux_ris_k * nv * nv, bris_ab16.as<uint16_t>(), st);
      rid::transpose_slices<double, uint16_t>(bris_ia, naux_ris_k, no, nv, bris_ai16.as<uint16_t>(), st);
    }
  } else {
    rid::cast_copy<float, uint16_t>(bris_ia_f, naux_ris * n, bris_ia16.as<uint16_t>(), st);
    if (naux_ris_k > 0) {
      rid::cast_copy<float, uint16_t>(bris_ij_f, (long)naux_ris_k * no * no, bris_ij16.as<uint16_t>(), st);
      rid::cast_copy<float, uint16_t>(bris_ab_f, (long)naux_ris_k * nv * nv, bris_ab16.as<uint16_t>(), st);
      rid::transpose_slices<float, uint16_t>(bris_ia_f, naux_ris_k, no, nv, bris_ai16.as<uint16_t>(), st);
    }
  }
  if (rislr.rows > 0) {
    rid::LrSet& L = rislr;
    const long r = L.rows;
    L.ia16.ensure(2 * (size_t)r * n);
    L.ij16.ensure(2 * (size_t)r * no * no);
    L.ab16.ensure(2 * (size_t)r * nv * nv);
    L.ai16.ensure(2 * (size_t)r * n);
    if (L.dt == RID_F64) {
      rid::cast_copy<double, uint16_t>(L.ia, r * n, L.ia16.as<uint16_t>(), st);
      rid::cast_copy<double, uint16_t>(L.ij, r * no * no, L.ij16.as<uint16_t>(), st);
      rid::cast_copy<double, uint16_t>(L.ab, r * nv * nv, L.ab16.as<uint16_t>(), st);
      rid::transpose_slices<double, uint16_t>(L.ia, L.rows, no, nv, L.ai16.as<uint16_t>(), st);
    } else {
      rid::cast_copy<float, uint16_t>(L.ia_f, r * n, L.ia16.as<uint16_t>(), st);
      rid::cast_copy<float, uint16_t>(L.ij_f, r * no * no, L.ij16.as<uint16_t>(), st);
      rid::cast_copy<float, uint16_t>(L.ab_f, r * nv * nv, L.ab16.as<uint16_t>(), st);
      rid::transpose_slices<float, uint16_t>(L.ia_f, L.rows, no, nv, L.ai16.as<uint16_t>(), st);
    }
  }
  RID_HIP(hipStreamSynchronize(st));
}

namespace rid {

void ring_free(DescRing* r) { delete r; }

namespace {

#ifndef RID_BUILD_ID
#define RID_BUILD_ID "unknown"
#endif

std::string tune_header(int device) {
  hipDeviceProp_t prop;
  RID_HIP(hipGetDeviceProperties(&prop, device));
  std::string arch = prop.gcnArchName;
  for (char& c : arch)
    if (c == ' ') c = '_';
  return std::string("rid-tune 1 ") + RID_BUILD_ID + " " + arch;
}

}  // namespace

int tune_save(rid_context* ctx, const char* path) {
  const std::string head = tune_header(ctx->device);
  std::lock_guard<std::mutex> g(ctx->tune_mu);
  FILE* f = std::fopen(path, "w");
  RID_CHECK(f != nullptr, RID_ERR_INVALID_ARG, std::string("cannot write ") + path);
  std::fprintf(f, "%s\n", head.c_str());
  for (const auto& kv : ctx->tune) {
    const TuneKey& k = kv.first;
    const TuneVal& v = kv.second;
    std::fprintf(f, "%d %d %ld %ld %d %d %d %d %d %d\n", k.family, k.esz, k.M, k.N, k.nz, k.np, k.K, v.cfg, v.nsub,
                 v.pps);
  }
  const bool ok = std::fclose(f) == 0;
  RID_CHECK(ok, RID_ERR_INVALID_ARG, std::string("cannot write ") + path);
  return (int)ctx->tune.size();
}

int tune_load(rid_context* ctx, const char* path) {
  const std::string head = tune_header(ctx->device);
  FILE* f = std::fopen(path, "r");
  RID_CHECK(f != nullptr, RID_ERR_INVALID_ARG, std::string("cannot read ") + path);
  char line[512];
  std::vector<std::pair<TuneKey, TuneVal>> got;
  std::string err;
  if (!std::fgets(line, sizeof(line), f)) {
    err = "empty tuning file";
  } else {
    std::string h(line);
    while (!h.empty() && (h.back() == '\n' || h.back() == '\r')) h.pop_back();
    if (h != head) err = "tuning file made by another build or device (" + h + "; this is " + head + ")";
  }
  while (err.empty() && std::fgets(line, sizeof(line), f)) {
    TuneKey k{};
    TuneVal v{};
    if (std::sscanf(line, "%d %d %ld %ld %d %d %d %d %d %d", &k.family, &k.esz, &k.M, &k.N, &k.nz, &k.np, &k.K, &v.cfg,
                    &v.nsub, &v.pps) != 10) {
      err = "malformed tuning line";
      break;
    }
    // a known family and element type, a tile configuration of that type,
    // and a split plan that covers its batches
    const int ncfg = k.esz == 8   ? gemm_num_configs<double>()
                     : k.esz == 4 ? gemm_num_configs<float>()
                     : k.esz == 2 ? gemm_num_configs<bf16_t>()
                                  : 0;
    if (k.family < GF_GENERIC || k.family > GF_EXCH_WP || v.cfg < 0 || v.cfg >= ncfg || k.M < 1 || k.N < 1 ||
        k.nz < 1 || k.K < 1 || k.np < 1 || v.nsub < 1 || v.pps < 1 || (long)v.nsub * v.pps < k.np) {
      err = "tuning line with an invalid plan";
      break;
    }
    got.emplace_back(k, v);
  }
  std::fclose(f);
  RID_CHECK(err.empty(), RID_ERR_INVALID_ARG, err);
  std::lock_guard<std::mutex> g(ctx->tune_mu);
  for (const auto& kv : got) ctx->tune[kv.first] = kv.second;
  return (int)got.size();
}

}  // namespace rid
