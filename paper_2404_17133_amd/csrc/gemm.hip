// MFMA GEMM kernels for gfx950 (see gemm.hpp for the operation).
//
// Tiling: a workgroup of 4 waves owns a BM x BN output tile; each wave owns a
// WM x WN sub-tile made of MFMA atoms (32x32 for f32/bf16, 16x16 for f64).
// Every K stage moves 128 bytes of K per operand row (32 f32, 16 f64, 64
// bf16) from global memory to LDS, double-buffered with one barrier per
// stage.  (Measured on gfx950: a second stage of register prefetch did not
// help at these shapes.)  With 16-byte vector loads the tiles load straight
// into unpadded, XOR-swizzled LDS rows (gemm_tile_dma); the scalar-load form
// (unaligned or odd operands) stages the loads through registers into LDS
// rows padded by 16 bytes (stride 144 B), so that the 16-byte fragment reads
// of 16 consecutive rows hit distinct banks.  The K order inside a stage is
// permuted so that each lane reads one contiguous slice per operand row: lane
// group g (lanes sharing a row) takes the g-th slice of the stage, and MFMA
// step s consumes the s-th element(s) of every group's slice.  Since A and B
// use the same permutation the sum over K is unchanged.
//
// When K is not a multiple of the stage width (K = no = 200 in the exchange
// S and W' products), a second form deals the chunks of a stage to the lane
// groups in turn (group g takes chunks g, g + G, ...), so that the valid
// chunks of a batch's last stage are the first chunk(s) of every group's
// slice, and that stage runs only the MFMA steps of those chunks (K = 200:
// 4 of the 16 steps of its last stage).  The form is chosen by K alone, so
// every tile shape of a product sums in the same order.
#include "gemm.hpp"
#include "gemm_limits.hpp"

#include <algorithm>
#include <type_traits>

namespace rid {
namespace {

typedef float v16f __attribute__((ext_vector_type(16)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));
typedef double v2d __attribute__((ext_vector_type(2)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

template <typename T>
struct Atom;

// v_mfma_f64_16x16x4_f64: A lane l holds A[l%16][k-group l/16]; D lane l,
// register r holds D[l/16 + 4*r][l%16] (rows interleaved across the four
// lane groups, unlike the FP32 16x16 layout; measured on gfx950).
template <>
struct Atom<double> {
  typedef double elem_t;
  typedef double acc_t;
  typedef v4d accv_t;
  typedef v2d vec_t;
  static constexpr int AM = 16, G = 4, E = 1, NACC = 4;
  __device__ static inline double op(const vec_t* f, int s) { return f[s >> 1][s & 1]; }
  __device__ static inline accv_t mma(double a, double b, accv_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lane, int r) { return (lane >> 4) + 4 * r; }
  __device__ static inline double out(acc_t v) { return v; }
};

// v_mfma_f32_32x32x2_f32: A lane l holds A[l%32][k-group l/32]; D lane l,
// register r holds D[(r/4)*8 + (l/32)*4 + r%4][l%32].
template <>
struct Atom<float> {
  typedef float elem_t;
  typedef float acc_t;
  typedef v16f accv_t;
  typedef v4f vec_t;
  static constexpr int AM = 32, G = 2, E = 1, NACC = 16;
  __device__ static inline float op(const vec_t* f, int s) { return f[s >> 2][s & 3]; }
  __device__ static inline accv_t mma(float a, float b, accv_t c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lane, int r) { return (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3); }
  __device__ static inline float out(acc_t v) { return v; }
};

// v_mfma_f32_32x32x16_bf16: A lane l holds 8 consecutive K of row l%32 in
// k-group l/32; D layout as for the f32 32x32 atom.
template <>
struct Atom<bf16_t> {
  typedef uint16_t elem_t;
  typedef float acc_t;
  typedef v16f accv_t;
  typedef v8bf vec_t;
  static constexpr int AM = 32, G = 2, E = 8, NACC = 16;
  __device__ static inline v8bf op(const vec_t* f, int s) { return f[s]; }
  __device__ static inline accv_t mma(v8bf a, v8bf b, accv_t c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lane, int r) { return (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3); }
  __device__ static inline uint16_t out(acc_t v) { return f32_to_bf16_bits(v); }
};

// Two workgroups per CU (two waves per SIMD) for the 4-byte and 2-byte
// element types; the FP64 128x128 tile needs the whole register file.
template <typename T>
struct MinBlocks {
  static constexpr int value = 2;
};
template <>
struct MinBlocks<double> {
  static constexpr int value = 1;
};

// One BM x BN output tile (tm, tn) of batch z and split `split`.  Shared by
// the single-GEMM and the grouped kernels, so that a tile's arithmetic does
// not depend on which kernel runs it.  Ends with every wave past the last
// read of its LDS buffers, so that the next tile may refill them.
template <typename T, int BM, int BN, int WM, int WN, bool VEC, bool IL>
__device__ __forceinline__ void gemm_tile(const GemmParams p, int tm, int tn, int z, int split) {
  using At = Atom<T>;
  using E_t = typename At::elem_t;
  using V_t = typename At::vec_t;
  using acc_t = typename At::acc_t;
  using accv_t = typename At::accv_t;
  constexpr int VW = 16 / (int)sizeof(E_t);  // elements per 16-byte chunk
  constexpr int BK = 8 * VW;                 // 128 bytes of K per stage
  constexpr int RS = 9;                      // LDS row stride in 16-byte chunks
  constexpr int ROWS = BM + BN;
  constexpr int CPT = ROWS * 8 / 256;        // chunks per thread per stage
  static_assert((ROWS * 8) % 256 == 0, "tile rows must be a multiple of 32");
  constexpr int NWM = BM / WM;
  constexpr int NWN = BN / WN;
  static_assert(NWM * NWN == 4, "four waves per workgroup");
  constexpr int AMN = WM / At::AM;
  constexpr int ANN = WN / At::AM;
  constexpr int SL = 8 / At::G;              // chunks per lane slice
  constexpr int KSTEPS = BK / At::G / At::E; // MFMA steps per stage
  constexpr int SPC = KSTEPS / SL;           // MFMA steps per chunk of a slice
  static_assert(SPC * SL == KSTEPS, "steps per chunk");

  __shared__ uint4 lds[2][ROWS * RS];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int m0 = tm * BM;
  const int n0 = tn * BN;
  const int z1 = z / p.nz2, z2 = z % p.nz2;
  const int pbeg = split * p.pps;
  const int pend = min(p.np, pbeg + p.pps);
  const E_t* Ab = reinterpret_cast<const E_t*>(p.A) + z1 * p.sA1 + z2 * p.sA2;
  const E_t* Bb = reinterpret_cast<const E_t*>(p.B) + z1 * p.sB1 + z2 * p.sB2;
  const int nkt = (p.K + BK - 1) / BK;
  const int nstage = pend > pbeg ? (pend - pbeg) * nkt : 0;

  const int kc = tid & 7;
  const int rbase = tid >> 3;
  // operand strides as plain values (selecting between fields of a local
  // copy of p would put that copy in scratch memory)
  const long lda = p.lda, ldb = p.ldb, sAp = p.sAp, sBp = p.sBp;
  const int M = p.M, N = p.N, K = p.K;

  // Chunk i of a thread holds row rbase + 32 i of the stacked (A; B) tile:
  // A rows for i < NA, B rows after.
  constexpr int NA = BM / 32;
  // 16-byte loads go through buffer resources based at the tile's first row
  // of the current batch: the per-thread byte offsets are fixed for the
  // tile, the K position of the stage is a uniform offset, and rows past M
  // (N) or chunks past K take an offset beyond the resource's range, which
  // the hardware returns as zeros - no branches, no 64-bit address math per
  // stage.
  constexpr int kOob = (int)0x80000000;
  int voff[CPT];
  if constexpr (VEC) {
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
      const bool a_row = i < NA;
      const int r = rbase + 32 * (a_row ? i : i - NA);
      const bool ok = a_row ? (m0 + r < M) : (n0 + r < N);
      const long ld = a_row ? lda : ldb;
      voff[i] = ok ? (int)(((long)r * ld + kc * VW) * (long)sizeof(E_t)) : kOob;
    }
  }
  int pcur = pbeg, kcur = 0;  // batch and K position of the next stage to load

  auto gload = [&](int t, uint4 (&pre)[CPT]) {
    if constexpr (VEC) {
      (void)t;
      const E_t* abase = Ab + (long)pcur * sAp + (long)m0 * lda;
      const E_t* bbase = Bb + (long)pcur * sBp + (long)n0 * ldb;
      const __amdgpu_buffer_rsrc_t ra =
          __builtin_amdgcn_make_buffer_rsrc(const_cast<E_t*>(abase), (short)0, 0x7fffffff, 0x00020000);
      const __amdgpu_buffer_rsrc_t rb =
          __builtin_amdgcn_make_buffer_rsrc(const_cast<E_t*>(bbase), (short)0, 0x7fffffff, 0x00020000);
      const bool kin = kcur + kc * VW < K;
      const int soff = kcur * (int)sizeof(E_t);
#pragma unroll
      for (int i = 0; i < CPT; ++i) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b128(i < NA ? ra : rb, kin ? voff[i] : kOob, soff, 0);
        pre[i] = make_uint4(v[0], v[1], v[2], v[3]);
      }
      kcur += BK;
      if (kcur >= nkt * BK) {
        kcur = 0;
        ++pcur;
      }
    } else {
      const int pp = pbeg + t / nkt;
      const int k = (t % nkt) * BK + kc * VW;
#pragma unroll
      for (int i = 0; i < CPT; ++i) {
        const int r = rbase + 32 * i;
        const E_t* src;
        bool ok;
        if (i < NA) {
          const int m = m0 + r;
          ok = m < M;
          src = Ab + pp * sAp + (long)m * lda + k;
        } else {
          const int n = n0 + (r - BM);
          ok = n < N;
          src = Bb + pp * sBp + (long)n * ldb + k;
        }
        union { uint4 v; E_t e[VW]; } u;
#pragma unroll
        for (int e = 0; e < VW; ++e) u.e[e] = (ok && k + e < K) ? src[e] : E_t(0);
        pre[i] = u.v;
      }
    }
  };
  auto lstore = [&](int buf, const uint4 (&pre)[CPT]) {
#pragma unroll
    for (int i = 0; i < CPT; ++i) lds[buf][(rbase + 32 * i) * RS + kc] = pre[i];
  };

  const int wm = (wave % NWM) * WM;
  const int wn = (wave / NWM) * WN;
  const int lr = lane % At::AM;
  const int g = lane / At::AM;

  accv_t acc[AMN][ANN];
#pragma unroll
  for (int i = 0; i < AMN; ++i)
#pragma unroll
    for (int j = 0; j < ANN; ++j)
#pragma unroll
      for (int r = 0; r < At::NACC; ++r) acc[i][j][r] = acc_t(0);

  // chunk c of lane group g's slice: chunk g*SL + c of the stage, or
  // chunk c*G + g in the interleaved form
  constexpr int CSTEP = IL ? At::G : 1;
  const int cbase = IL ? g : g * SL;
  // nc: chunks of every slice that hold valid K (all SL but in the last
  // stage of a batch in the interleaved form)
  auto compute = [&](int buf, int nc) {
    V_t fa[AMN][SL];
    V_t fb[ANN][SL];
#pragma unroll
    for (int i = 0; i < AMN; ++i) {
      const uint4* src = &lds[buf][(wm + i * At::AM + lr) * RS + cbase];
#pragma unroll
      for (int c = 0; c < SL; ++c) fa[i][c] = *reinterpret_cast<const V_t*>(src + c * CSTEP);
    }
#pragma unroll
    for (int j = 0; j < ANN; ++j) {
      const uint4* src = &lds[buf][(BM + wn + j * At::AM + lr) * RS + cbase];
#pragma unroll
      for (int c = 0; c < SL; ++c) fb[j][c] = *reinterpret_cast<const V_t*>(src + c * CSTEP);
    }
#pragma unroll
    for (int s = 0; s < KSTEPS; ++s) {
      if (IL && s % SPC == 0 && s / SPC >= nc) break;
#pragma unroll
      for (int i = 0; i < AMN; ++i)
#pragma unroll
        for (int j = 0; j < ANN; ++j) acc[i][j] = At::mma(At::op(fa[i], s), At::op(fb[j], s), acc[i][j]);
    }
  };

  const acc_t alpha = (acc_t)p.alpha;
  // store the tile in the element type at C (used per batch by
  // GEMM_STORE_EACH and once by GEMM_STORE)
  auto store_tile = [&](E_t* C) {
#pragma unroll
    for (int i = 0; i < AMN; ++i)
#pragma unroll
      for (int j = 0; j < ANN; ++j)
#pragma unroll
        for (int r = 0; r < At::NACC; ++r) {
          const int m = m0 + wm + i * At::AM + At::row(lane, r);
          const int n = n0 + wn + j * At::AM + lr;
          if (m < p.M && n < p.N) C[(long)m * p.ldc + n] = At::out(alpha * acc[i][j][r]);
        }
  };
  const bool each = p.mode == GEMM_STORE_EACH;
  E_t* Ce = reinterpret_cast<E_t*>(p.C) + z1 * p.sC1 + z2 * p.sC2;

  // One stage in flight: the next stage's global loads are issued before the
  // MFMAs of the current stage and written to the other LDS buffer after them.
  // In GEMM_STORE_EACH mode the batches of the split run back to back through
  // the same pipeline, the tile of each batch being stored when its last
  // stage is done, so that the next batch's first stage is already loaded.
  uint4 pa[CPT];
  if (nstage > 0) {
    gload(0, pa);
    lstore(0, pa);
  }
  __syncthreads();
  int kt_c = 0, p_c = pbeg;  // stage within its batch, and batch, of the stage being computed
  for (int t = 0; t < nstage; ++t) {
    if (t + 1 < nstage) gload(t + 1, pa);
    int nc = SL;
    if constexpr (IL) {
      const int valid = K - kt_c * BK;  // K elements of this stage
      if (valid < BK) nc = ((valid + VW - 1) / VW + At::G - 1) / At::G;
    }
    compute(t & 1, nc);
    if (++kt_c == nkt) {
      kt_c = 0;
      if (each) {
        store_tile(Ce + (long)p_c * p.sCs);
#pragma unroll
        for (int i = 0; i < AMN; ++i)
#pragma unroll
          for (int j = 0; j < ANN; ++j)
#pragma unroll
            for (int r = 0; r < At::NACC; ++r) acc[i][j][r] = acc_t(0);
        ++p_c;
      }
    }
    if (t + 1 < nstage) lstore((t + 1) & 1, pa);
    __syncthreads();
  }

  // epilogue
  if (each) {
    return;
  } else if (p.mode == GEMM_STORE) {
    store_tile(Ce);
  } else {
    acc_t* C = reinterpret_cast<acc_t*>(p.C) + split * p.sCs + z1 * p.sC1 + z2 * p.sC2;
    const bool add = p.mode == GEMM_PARTIAL_ADD;
#pragma unroll
    for (int i = 0; i < AMN; ++i)
#pragma unroll
      for (int j = 0; j < ANN; ++j)
#pragma unroll
        for (int r = 0; r < At::NACC; ++r) {
          const int m = m0 + wm + i * At::AM + At::row(lane, r);
          const int n = n0 + wn + j * At::AM + lr;
          if (m < p.M && n < p.N) {
            acc_t* dst = C + (long)m * p.ldc + n;
            const acc_t v = alpha * acc[i][j][r];
            *dst = add ? *dst + v : v;
          }
        }
  }
}

// The same tile with the operands moved from global memory straight into
// LDS (buffer loads with an LDS destination: no staging registers and no LDS
// stores by the waves), NSTG stage buffers.  Used for every vector-load
// tile: on the FP32 exchange shapes it matches the staged tile on 64x64
// tiles and is 4-16 % faster on 128x64 and 128x128 tiles, and the FP64
// step is 7 % faster; three or four buffers were slower (fewer workgroups
// per CU).  LDS rows are not padded: chunk lc of row r sits
// at chunk lc ^ sw(r), so that the 16-byte fragment reads of 16 consecutive
// rows fall on distinct banks.  The MFMA steps consume the same K elements
// in the same order as gemm_tile, so the two give identical results.
__device__ __forceinline__ int lds_swz(int r) { return (r & 7) ^ ((r >> 3) & 1); }

template <int N>
__device__ __forceinline__ void wait_vm() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt(0x0F70 | (N & 15) | ((N >> 4) << 14));
}

template <typename T, int BM, int BN, int WM, int WN, bool IL, int NSTG>
__device__ __forceinline__ void gemm_tile_dma(const GemmParams p, int tm, int tn, int z, int split) {
  using At = Atom<T>;
  using E_t = typename At::elem_t;
  using V_t = typename At::vec_t;
  using acc_t = typename At::acc_t;
  using accv_t = typename At::accv_t;
  constexpr int VW = 16 / (int)sizeof(E_t);
  constexpr int BK = 8 * VW;
  constexpr int ROWS = BM + BN;
  constexpr int NI = ROWS / 32;              // load instructions per wave per stage
  static_assert(ROWS % 32 == 0, "tile rows must be a multiple of 32");
  constexpr int STG_BYTES = ROWS * 128;
  constexpr int NWM = BM / WM;
  constexpr int NWN = BN / WN;
  static_assert(NWM * NWN == 4, "four waves per workgroup");
  constexpr int AMN = WM / At::AM;
  constexpr int ANN = WN / At::AM;
  constexpr int SL = 8 / At::G;
  constexpr int KSTEPS = BK / At::G / At::E;
  constexpr int SPC = KSTEPS / SL;
  static_assert(SPC * SL == KSTEPS, "steps per chunk");
  static_assert(NSTG >= 2 && NSTG <= 4, "stage buffers");

  __shared__ __attribute__((aligned(1024))) char lds[NSTG * STG_BYTES];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform: LDS destinations go through M0
  const int m0 = tm * BM;
  const int n0 = tn * BN;
  const int z1 = z / p.nz2, z2 = z % p.nz2;
  const int pbeg = split * p.pps;
  const int pend = min(p.np, pbeg + p.pps);
  const E_t* Ab = reinterpret_cast<const E_t*>(p.A) + z1 * p.sA1 + z2 * p.sA2;
  const E_t* Bb = reinterpret_cast<const E_t*>(p.B) + z1 * p.sB1 + z2 * p.sB2;
  const int nkt = (p.K + BK - 1) / BK;
  const int nstage = pend > pbeg ? (pend - pbeg) * nkt : 0;
  const long lda = p.lda, ldb = p.ldb, sAp = p.sAp, sBp = p.sBp;
  const int M = p.M, N = p.N, K = p.K;

  // load instruction q of this wave covers stacked rows r0 .. r0 + 7 with
  // r0 = (q * 4 + wave) * 8; lane i takes row r0 + i / 8, LDS chunk i % 8,
  // which holds logical chunk (i % 8) ^ sw(row)
  constexpr int kOob = (int)0x80000000;
  int voff[NI], vlc[NI];
#pragma unroll
  for (int q = 0; q < NI; ++q) {
    const int r = (q * 4 + wave) * 8 + (lane >> 3);
    const int lc = (lane & 7) ^ lds_swz(r);
    vlc[q] = lc;
    const bool a_row = r < BM;
    const int rr = a_row ? r : r - BM;
    const bool ok = a_row ? (m0 + rr < M) : (n0 + rr < N);
    const long ld = a_row ? lda : ldb;
    voff[q] = ok ? (int)(((long)rr * ld + lc * VW) * (long)sizeof(E_t)) : kOob;
  }
  int pcur = pbeg, kcur = 0;  // batch and K position of the next stage to load
  auto issue = [&](int buf) {
    const E_t* abase = Ab + (long)pcur * sAp + (long)m0 * lda;
    const E_t* bbase = Bb + (long)pcur * sBp + (long)n0 * ldb;
    const __amdgpu_buffer_rsrc_t ra =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<E_t*>(abase), (short)0, 0x7fffffff, 0x00020000);
    const __amdgpu_buffer_rsrc_t rb =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<E_t*>(bbase), (short)0, 0x7fffffff, 0x00020000);
    const int soff = kcur * (int)sizeof(E_t);
#pragma unroll
    for (int q = 0; q < NI; ++q) {
      const int r0 = (q * 4 + wave) * 8;  // wave-uniform
      const bool kin = kcur + vlc[q] * VW < K;
      char* dst = lds + buf * STG_BYTES + r0 * 128;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(r0 < BM ? ra : rb, (__attribute__((address_space(3))) void*)dst, 16,
                                               kin ? voff[q] : kOob, soff, 0, 0);
    }
    kcur += BK;
    if (kcur >= nkt * BK) {
      kcur = 0;
      ++pcur;
    }
  };

  const int wm = (wave % NWM) * WM;
  const int wn = (wave / NWM) * WN;
  const int lr = lane % At::AM;
  const int g = lane / At::AM;
  constexpr int CSTEP = IL ? At::G : 1;
  const int cbase = IL ? g : g * SL;
  // byte offsets (within a stage buffer) of the fragment chunks
  int offa[AMN][SL], offb[ANN][SL];
#pragma unroll
  for (int i = 0; i < AMN; ++i) {
    const int r = wm + i * At::AM + lr;
#pragma unroll
    for (int c = 0; c < SL; ++c) offa[i][c] = r * 128 + ((cbase + c * CSTEP) ^ lds_swz(r)) * 16;
  }
#pragma unroll
  for (int j = 0; j < ANN; ++j) {
    const int r = BM + wn + j * At::AM + lr;
#pragma unroll
    for (int c = 0; c < SL; ++c) offb[j][c] = r * 128 + ((cbase + c * CSTEP) ^ lds_swz(r)) * 16;
  }

  accv_t acc[AMN][ANN];
#pragma unroll
  for (int i = 0; i < AMN; ++i)
#pragma unroll
    for (int j = 0; j < ANN; ++j)
#pragma unroll
      for (int r = 0; r < At::NACC; ++r) acc[i][j][r] = acc_t(0);

  auto compute = [&](int buf, int nc) {
    const char* base = lds + buf * STG_BYTES;
    V_t fa[AMN][SL];
    V_t fb[ANN][SL];
#pragma unroll
    for (int i = 0; i < AMN; ++i)
#pragma unroll
      for (int c = 0; c < SL; ++c) fa[i][c] = *reinterpret_cast<const V_t*>(base + offa[i][c]);
#pragma unroll
    for (int j = 0; j < ANN; ++j)
#pragma unroll
      for (int c = 0; c < SL; ++c) fb[j][c] = *reinterpret_cast<const V_t*>(base + offb[j][c]);
#pragma unroll
    for (int s = 0; s < KSTEPS; ++s) {
      if (IL && s % SPC == 0 && s / SPC >= nc) break;
#pragma unroll
      for (int i = 0; i < AMN; ++i)
#pragma unroll
        for (int j = 0; j < ANN; ++j) acc[i][j] = At::mma(At::op(fa[i], s), At::op(fb[j], s), acc[i][j]);
    }
  };

  const acc_t alpha = (acc_t)p.alpha;
  auto store_tile = [&](E_t* C) {
#pragma unroll
    for (int i = 0; i < AMN; ++i)
#pragma unroll
      for (int j = 0; j < ANN; ++j)
#pragma unroll
        for (int r = 0; r < At::NACC; ++r) {
          const int m = m0 + wm + i * At::AM + At::row(lane, r);
          const int n = n0 + wn + j * At::AM + lr;
          if (m < p.M && n < p.N) C[(long)m * p.ldc + n] = At::out(alpha * acc[i][j][r]);
        }
  };
  const bool each = p.mode == GEMM_STORE_EACH;
  E_t* Ce = reinterpret_cast<E_t*>(p.C) + z1 * p.sC1 + z2 * p.sC2;

  // NSTG - 1 stages in flight ahead of the one being computed.  At step t:
  // wait for this wave's loads of stage t, barrier (every wave's loads of
  // stage t are in LDS, and every wave is done reading the buffer of stage
  // t - 1), refill that buffer with stage t + NSTG - 1, compute stage t.
#pragma unroll
  for (int q = 0; q < NSTG - 1; ++q)
    if (q < nstage) issue(q);
  int kt_c = 0, p_c = pbeg;
  for (int t = 0; t < nstage; ++t) {
    if (t + NSTG - 2 < nstage)
      wait_vm<NI * (NSTG - 2)>();
    else
      wait_vm<0>();
    __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0): this wave's reads of the previous buffer are done
    __builtin_amdgcn_s_barrier();
    if (t + NSTG - 1 < nstage) issue((t + NSTG - 1) % NSTG);
    int nc = SL;
    if constexpr (IL) {
      const int valid = K - kt_c * BK;
      if (valid < BK) nc = ((valid + VW - 1) / VW + At::G - 1) / At::G;
    }
    compute(t % NSTG, nc);
    if (++kt_c == nkt) {
      kt_c = 0;
      if (each) {
        store_tile(Ce + (long)p_c * p.sCs);
#pragma unroll
        for (int i = 0; i < AMN; ++i)
#pragma unroll
          for (int j = 0; j < ANN; ++j)
#pragma unroll
            for (int r = 0; r < At::NACC; ++r) acc[i][j][r] = acc_t(0);
        ++p_c;
      }
    }
  }
  // every wave is past its last LDS read before the next tile refills them
  __builtin_amdgcn_s_waitcnt(0xC07F);
  __builtin_amdgcn_s_barrier();

  if (each) {
    return;
  } else if (p.mode == GEMM_STORE) {
    store_tile(Ce);
  } else {
    acc_t* C = reinterpret_cast<acc_t*>(p.C) + split * p.sCs + z1 * p.sC1 + z2 * p.sC2;
    const bool add = p.mode == GEMM_PARTIAL_ADD;
#pragma unroll
    for (int i = 0; i < AMN; ++i)
#pragma unroll
      for (int j = 0; j < ANN; ++j)
#pragma unroll
        for (int r = 0; r < At::NACC; ++r) {
          const int m = m0 + wm + i * At::AM + At::row(lane, r);
          const int n = n0 + wn + j * At::AM + lr;
          if (m < p.M && n < p.N) {
            acc_t* dst = C + (long)m * p.ldc + n;
            const acc_t v = alpha * acc[i][j][r];
            *dst = add ? *dst + v : v;
          }
        }
  }
}

template <typename T, int BM, int BN, int WM, int WN, bool VEC, bool IL>
__device__ __forceinline__ void gemm_tile_any(const GemmParams p, int tm, int tn, int z, int split) {
  if constexpr (VEC)
    gemm_tile_dma<T, BM, BN, WM, WN, IL, 2>(p, tm, tn, z, split);
  else
    gemm_tile<T, BM, BN, WM, WN, VEC, IL>(p, tm, tn, z, split);
}

constexpr int kXcds = 8;

// Position in the tile walk of workgroup w of a launch of `total`: the
// workgroups that land on one XCD (w = x mod 8, dealt in turn) take one
// contiguous range of the walk, in dispatch order.
__device__ inline long xcd_walk(long w, long total) {
  const long q = total / kXcds, r = total % kXcds;
  const long x = w % kXcds;
  return x * q + (x < r ? x : r) + w / kXcds;
}

struct TileCoord {
  int tm, tn, z, split;
};

// Tile coordinates of walk position t (see GemmOrder).
__device__ inline TileCoord walk_decode(int order, long t, int tiles_m, int tiles_n, int nz, int nsplit) {
  TileCoord c;
  if (order == ORDER_ZIN) {
    c.tm = (int)(t % tiles_m);
    long r = t / tiles_m;
    c.z = (int)(r % nz);
    r /= nz;
    c.split = (int)(r % nsplit);
    c.tn = (int)(r / nsplit);
    return c;
  }
  const long tiles = (long)tiles_m * tiles_n;
  const long tile = t % tiles;
  const long r = t / tiles;
  c.z = (int)(r % nz);
  c.split = (int)(r / nz);
  const bool nm = order == ORDER_NM;
  c.tn = (int)(nm ? tile % tiles_n : tile / tiles_m);
  c.tm = (int)(nm ? tile / tiles_n : tile % tiles_m);
  return c;
}

template <typename T, int BM, int BN, int WM, int WN, bool VEC, bool IL, int FAM>
__global__ __launch_bounds__(256, MinBlocks<T>::value) void gemm_nt_kernel(GemmParams p, int nz, long total) {
  const int tiles_m = (p.M + BM - 1) / BM;
  const int tiles_n = (p.N + BN - 1) / BN;
  const int nsplit = (int)(total / ((long)tiles_m * tiles_n * nz));
  const TileCoord c = walk_decode(p.order, xcd_walk(blockIdx.x, total), tiles_m, tiles_n, nz, nsplit);
  gemm_tile_any<T, BM, BN, WM, WN, VEC, IL>(p, c.tm, c.tn, c.z, c.split);
}

// Device descriptor of one member of a grouped launch.
struct GroupDesc {
  GemmParams p;
  int tiles_m, tiles_n, nz, nsplit;
  long begin;  // index of the member's first tile in the launch
};

// Persistent grouped GEMM: the workgroups walk the concatenated tile walks
// of all members, each taking every gridDim.x-th position.  With a grid that
// is a multiple of the XCD count, a workgroup stays on one XCD, and the
// positions are re-mapped as in the single-GEMM kernel so that each XCD
// covers one contiguous range of the concatenated walk.
template <typename T, int BM, int BN, int WM, int WN, bool VEC, bool IL, int FAM>
__global__ __launch_bounds__(256, MinBlocks<T>::value) void gemm_grouped_kernel(const GroupDesc* __restrict__ gd,
                                                                               int ngroups, long total) {
  for (long b = blockIdx.x; b < total; b += gridDim.x) {
    const long t = xcd_walk(b, total);
    int lo = 0, hi = ngroups - 1;  // member holding position t
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (gd[mid].begin <= t)
        lo = mid;
      else
        hi = mid - 1;
    }
    const GemmParams p = gd[lo].p;
    const TileCoord c =
        walk_decode(p.order, t - gd[lo].begin, gd[lo].tiles_m, gd[lo].tiles_n, gd[lo].nz, gd[lo].nsplit);
    gemm_tile_any<T, BM, BN, WM, WN, VEC, IL>(p, c.tm, c.tn, c.z, c.split);
  }
}

struct TileCfg {
  int bm, bn;
};

template <typename T>
struct Cfgs;
template <>
struct Cfgs<double> {
  static constexpr TileCfg c[3] = {{128, 128}, {64, 64}, {128, 64}};
};
template <>
struct Cfgs<float> {
  static constexpr TileCfg c[3] = {{128, 128}, {64, 64}, {128, 64}};
};
template <>
struct Cfgs<bf16_t> {
  static constexpr TileCfg c[3] = {{128, 128}, {64, 64}, {128, 64}};
};

// Load form of a launch: 0 vector loads, 1 vector loads with interleaved
// chunks (K not a multiple of the stage width), 2 scalar loads.
template <typename T, int BM, int BN, int WM, int WN, int FAM>
void launch_fam(const GemmParams& p, int nz, long total, int form, hipStream_t stream) {
  if (form == 0)
    hipLaunchKernelGGL((gemm_nt_kernel<T, BM, BN, WM, WN, true, false, FAM>), dim3((unsigned)total), dim3(256), 0,
                       stream, p, nz, total);
  else if (form == 1)
    hipLaunchKernelGGL((gemm_nt_kernel<T, BM, BN, WM, WN, true, true, FAM>), dim3((unsigned)total), dim3(256), 0,
                       stream, p, nz, total);
  else
    hipLaunchKernelGGL((gemm_nt_kernel<T, BM, BN, WM, WN, false, false, FAM>), dim3((unsigned)total), dim3(256), 0,
                       stream, p, nz, total);
}

template <typename T, int BM, int BN, int WM, int WN>
void launch_cfg(const GemmParams& p, int nz, int nsplit, int form, hipStream_t stream, int family) {
  const long total = (long)ceil_div(p.M, BM) * ceil_div(p.N, BN) * nz * nsplit;
  RID_CHECK(total < (1L << 31), RID_ERR_SHAPE, "gemm: grid too large");
  switch (family) {
    case GF_COUL: launch_fam<T, BM, BN, WM, WN, GF_COUL>(p, nz, total, form, stream); break;
    case GF_EXCH_S: launch_fam<T, BM, BN, WM, WN, GF_EXCH_S>(p, nz, total, form, stream); break;
    case GF_EXCH_W: launch_fam<T, BM, BN, WM, WN, GF_EXCH_W>(p, nz, total, form, stream); break;
    case GF_EXCH_Q: launch_fam<T, BM, BN, WM, WN, GF_EXCH_Q>(p, nz, total, form, stream); break;
    case GF_EXCH_WP: launch_fam<T, BM, BN, WM, WN, GF_EXCH_WP>(p, nz, total, form, stream); break;
    default: launch_fam<T, BM, BN, WM, WN, GF_GENERIC>(p, nz, total, form, stream); break;
  }
}

template <typename T, int BM, int BN, int WM, int WN, bool VEC, bool IL>
void launch_grouped_fam(const GroupDesc* gd, int n, long total, int grid, int family, hipStream_t stream) {
#define RID_GROUPED(F)                                                                                             \
  hipLaunchKernelGGL((gemm_grouped_kernel<T, BM, BN, WM, WN, VEC, IL, F>), dim3(grid), dim3(256), 0, stream, gd, n, \
                     total)
  switch (family) {
    case GF_COUL: RID_GROUPED(GF_COUL); break;
    case GF_EXCH_S: RID_GROUPED(GF_EXCH_S); break;
    case GF_EXCH_W: RID_GROUPED(GF_EXCH_W); break;
    case GF_EXCH_Q: RID_GROUPED(GF_EXCH_Q); break;
    case GF_EXCH_WP: RID_GROUPED(GF_EXCH_WP); break;
    default: RID_GROUPED(GF_GENERIC); break;
  }
#undef RID_GROUPED
}

template <typename T, int BM, int BN, int WM, int WN>
void launch_grouped_cfg(const GroupDesc* gd, int n, long total, int grid, int form, int family, hipStream_t stream) {
  if (form == 0)
    launch_grouped_fam<T, BM, BN, WM, WN, true, false>(gd, n, total, grid, family, stream);
  else if (form == 1)
    launch_grouped_fam<T, BM, BN, WM, WN, true, true>(gd, n, total, grid, family, stream);
  else
    launch_grouped_fam<T, BM, BN, WM, WN, false, false>(gd, n, total, grid, family, stream);
}

template <typename T>
int elem_size() {
  return std::is_same<T, bf16_t>::value ? 2 : (int)sizeof(T);
}

template <typename T>
bool vec_ok(const GemmParams& p) {
  const int vw = 16 / elem_size<T>();
  return (p.K % vw == 0) && (p.lda % vw == 0) && (p.ldb % vw == 0) && (p.sAp % vw == 0) && (p.sBp % vw == 0) &&
         (p.sA1 % vw == 0) && (p.sA2 % vw == 0) && (p.sB1 % vw == 0) && (p.sB2 % vw == 0) &&
         ((uintptr_t)p.A % 16 == 0) && ((uintptr_t)p.B % 16 == 0) &&
         gemm_offsets_fit(p.lda, p.ldb, p.K, elem_size<T>());
}

// Load form (see launch_fam) of a GEMM.
template <typename T>
int load_form(const GemmParams& p) {
  if (!vec_ok<T>(p)) return 2;
  return p.K % (128 / elem_size<T>()) != 0 ? 1 : 0;
}

void check_params(const GemmParams& p, int nz, int nsplit) {
  RID_CHECK(p.np >= 1 && p.pps >= 1 && p.nz2 >= 1, RID_ERR_INTERNAL, "gemm: bad batch counts");
  RID_CHECK(p.order >= ORDER_MN && p.order <= ORDER_ZIN, RID_ERR_INTERNAL, "gemm: bad tile order");
  RID_CHECK(p.mode >= GEMM_STORE && p.mode <= GEMM_STORE_EACH, RID_ERR_INTERNAL, "gemm: bad mode");
  RID_CHECK((long)nsplit * p.pps >= p.np, RID_ERR_INTERNAL, "gemm: splits do not cover batches");
  RID_CHECK(ceil_div_l(p.M, 64) * ceil_div_l(p.N, 64) < (1L << 31), RID_ERR_SHAPE, "gemm: grid too large");
  RID_CHECK(nz < 65536 && nsplit < 65536, RID_ERR_SHAPE, "gemm: batch grid too large");
}

}  // namespace

size_t gemm_group_desc_bytes(int n) { return sizeof(GroupDesc) * (size_t)std::max(n, 1); }

template <typename T>
void gemm_grouped(const GemmGroup* mem, int n, int cfg, int family, void* desc_dev, void* desc_host,
                  hipStream_t stream, int grid_cap) {
  RID_CHECK(cfg >= 0 && cfg < 3, RID_ERR_INTERNAL, "gemm: bad tile configuration");
  const int bm = Cfgs<T>::c[cfg].bm, bn = Cfgs<T>::c[cfg].bn;
  GroupDesc* hd = reinterpret_cast<GroupDesc*>(desc_host);
  // members by load form: one launch per form
  int cnt[3] = {0, 0, 0};
  long total[3] = {0, 0, 0};
  for (int pass = 0; pass < 3; ++pass) {
    for (int i = 0; i < n; ++i) {
      const GemmParams& p = mem[i].p;
      if (p.M <= 0 || p.N <= 0 || mem[i].nz <= 0 || mem[i].nsplit <= 0) continue;
      if (load_form<T>(p) != pass) continue;
      check_params(p, mem[i].nz, mem[i].nsplit);
      GroupDesc& d = hd[cnt[0] + cnt[1] + cnt[2]];
      d.p = p;
      d.tiles_m = ceil_div(p.M, bm);
      d.tiles_n = ceil_div(p.N, bn);
      d.nz = mem[i].nz;
      d.nsplit = mem[i].nsplit;
      d.begin = total[pass];
      total[pass] += (long)d.tiles_m * d.tiles_n * mem[i].nz * mem[i].nsplit;
      ++cnt[pass];
    }
  }
  const int used = cnt[0] + cnt[1] + cnt[2];
  if (used == 0) return;
  RID_HIP(hipMemcpyAsync(desc_dev, desc_host, sizeof(GroupDesc) * used, hipMemcpyHostToDevice, stream));
  const GroupDesc* dd = reinterpret_cast<const GroupDesc*>(desc_dev);
  for (int pass = 0, first = 0; pass < 3; first += cnt[pass], ++pass) {
    if (cnt[pass] == 0) continue;
    const GroupDesc* base = dd + first;
    // a multiple of the XCD count keeps every workgroup on one XCD
    const int cap = std::max(kXcds, grid_cap / kXcds * kXcds);
    const int grid = (int)std::min<long>(total[pass], cap);
    switch (cfg) {
      case 0: launch_grouped_cfg<T, 128, 128, 64, 64>(base, cnt[pass], total[pass], grid, pass, family, stream); break;
      case 1: launch_grouped_cfg<T, 64, 64, 32, 32>(base, cnt[pass], total[pass], grid, pass, family, stream); break;
      default: launch_grouped_cfg<T, 128, 64, 64, 32>(base, cnt[pass], total[pass], grid, pass, family, stream); break;
    }
    RID_HIP(hipGetLastError());
  }
}

template <typename T>
int gemm_num_configs() {
  return 3;
}
template <typename T>
void gemm_config_tile(int cfg, int* bm, int* bn) {
  *bm = Cfgs<T>::c[cfg].bm;
  *bn = Cfgs<T>::c[cfg].bn;
}

template <typename T>
void gemm_nt(const GemmParams& p, int nz, int nsplit, hipStream_t stream, int cfg, int family) {
  if (p.M <= 0 || p.N <= 0 || nz <= 0 || nsplit <= 0) return;
  check_params(p, nz, nsplit);
  const int vec = load_form<T>(p);
  if (cfg < 0) {
    // default: big tiles when the output is large enough to fill the chip
    const long t128 = ceil_div_l(p.M, 128) * ceil_div_l(p.N, 128) * (long)nz * nsplit;
    cfg = (t128 >= 512) ? 0 : 1;
  }
  switch (cfg) {
    case 0: launch_cfg<T, 128, 128, 64, 64>(p, nz, nsplit, vec, stream, family); break;
    case 1: launch_cfg<T, 64, 64, 32, 32>(p, nz, nsplit, vec, stream, family); break;
    default: launch_cfg<T, 128, 64, 64, 32>(p, nz, nsplit, vec, stream, family); break;
  }
  RID_HIP(hipGetLastError());
}

template void gemm_grouped<double>(const GemmGroup*, int, int, int, void*, void*, hipStream_t, int);
template void gemm_grouped<float>(const GemmGroup*, int, int, int, void*, void*, hipStream_t, int);
template void gemm_grouped<bf16_t>(const GemmGroup*, int, int, int, void*, void*, hipStream_t, int);
template void gemm_nt<double>(const GemmParams&, int, int, hipStream_t, int, int);
template void gemm_nt<float>(const GemmParams&, int, int, hipStream_t, int, int);
template void gemm_nt<bf16_t>(const GemmParams&, int, int, hipStream_t, int, int);
template int gemm_num_configs<double>();
template int gemm_num_configs<float>();
template int gemm_num_configs<bf16_t>();
template void gemm_config_tile<double>(int, int*, int*);
template void gemm_config_tile<float>(int, int*, int*);
template void gemm_config_tile<bf16_t>(int, int*, int*);

}  // namespace rid
