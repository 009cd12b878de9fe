// Batched, reduction-batched MFMA GEMM for gfx950:
//
//   C[z](m, n) (=|+=) alpha * sum_{p in split} sum_k A[z, p](m, k) * B[z, p](n, k)
//
// Both operands are K-contiguous ("NT"): A(m, k) at A + off_A(z, p) + m*lda + k,
// B(n, k) at B + off_B(z, p) + n*ldb + k.  z = blockIdx.y is split into
// (z1, z2) = (z / nz2, z % nz2) with independent strides, p runs over the
// reduction batches assigned to split s = blockIdx.z.  Element types:
// double (v_mfma_f64_16x16x4), float (v_mfma_f32_32x32x2), bf16 stored as
// uint16_t (v_mfma_f32_32x32x16_bf16, FP32 accumulation).
#pragma once

#include "common.hpp"

namespace rid {

// GEMM_STORE: C[z] = alpha * (sum over all batches), in the element type.
// GEMM_PARTIAL_SET / _ADD: each split writes (adds) its partial sum, in the
// accumulator type, at C + split * sCs.
// GEMM_STORE_EACH: no reduction; every batch p is its own product, stored in
// the element type at C + p * sCs.  A workgroup runs the pps batches of its
// split back to back through one pipeline (the operand that does not change
// with p has batch stride 0).
enum GemmMode { GEMM_STORE = 0, GEMM_PARTIAL_SET = 1, GEMM_PARTIAL_ADD = 2, GEMM_STORE_EACH = 3 };

// Contraction family of a launch.  Each family gets its own kernel symbol
// (same code) so that profilers report the families separately.
enum GemmFamily { GF_GENERIC = 0, GF_COUL = 1, GF_EXCH_S = 2, GF_EXCH_W = 3, GF_EXCH_Q = 4, GF_EXCH_WP = 5 };

struct GemmParams {
  const void* A;
  const void* B;
  void* C;
  int M, N, K;
  int np;    // reduction batches in total
  int pps;   // reduction batches per split
  int nz2;   // inner z extent
  long lda, ldb, ldc;
  long sAp, sBp;
  long sA1, sA2, sB1, sB2, sC1, sC2;
  long sCs;  // stride between split outputs (partial modes)
  double alpha;
  int mode;   // GemmMode
  int order;  // GemmOrder: the order in which workgroups walk the tiles
};

// Tile walk of a launch.  Workgroups are dealt to the chip's 8 XCDs in turn;
// every launch re-maps them so that each XCD takes one contiguous range of
// the walk below, whose fastest index keeps the operand that most tiles
// share in that XCD's L2.
//   ORDER_MN: tm fastest, then tn, batch, split (B row block reused);
//   ORDER_NM: tn fastest, then tm, batch, split (A row block reused);
//   ORDER_ZIN: tm fastest, then batch, then split, then tn (B row block
//              reused across all batches and splits).
enum GemmOrder { ORDER_MN = 0, ORDER_NM = 1, ORDER_ZIN = 2 };

// Element-type tag for bf16 operands stored as raw uint16_t.
struct bf16_t {};

// Launch one GEMM.  T = double, float or bf16_t.  For the partial modes the
// output is written in the accumulator type (double for T = double, float
// otherwise); for GEMM_STORE it is written in T.
template <typename T>
void gemm_nt(const GemmParams& p, int nz, int nsplit, hipStream_t stream, int tile_cfg = -1, int family = GF_GENERIC);

// One member of a grouped launch: a GEMM as gemm_nt(p, nz, nsplit, ...)
// would run it.
struct GemmGroup {
  GemmParams p;
  int nz, nsplit;
};

// Bytes of device (and pinned host staging) descriptor memory that a grouped
// launch of n members needs.
size_t gemm_group_desc_bytes(int n);

// Run n GEMMs of one element type and tile configuration in one persistent
// launch (two when some members cannot use 16-byte loads) of at most
// grid_cap workgroups.  Every member's output is bit for bit what gemm_nt
// with the same arguments writes: both kernels run the same tile code.  The
// descriptors are staged in desc_host (pinned) and copied to desc_dev on
// `stream`; the caller keeps both untouched until that copy has run.
template <typename T>
void gemm_grouped(const GemmGroup* members, int n, int tile_cfg, int family, void* desc_dev, void* desc_host,
                  hipStream_t stream, int grid_cap);

// Number of tile configurations available for T (for the autotuner).
template <typename T>
int gemm_num_configs();
template <typename T>
void gemm_config_tile(int cfg, int* bm, int* bn);

}  // namespace rid
