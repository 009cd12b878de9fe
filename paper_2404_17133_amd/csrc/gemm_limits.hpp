// Address limits of the GEMM tile loads (host-only arithmetic, no HIP).
//
// The 16-byte loads of a tile go through buffer resources based at the
// tile's first row of the current batch, with a 32-bit byte offset per
// lane: row r * ld + the lane's K chunk, plus the stage's K position as a
// uniform offset.  Offsets at or beyond 2^31 - 1 are what the kernel uses to
// mean "out of range, read zeros", so every in-range offset must stay below
// it; otherwise the load path with 64-bit addresses has to be taken.
#pragma once

#include <cstdint>

namespace rid {

// Largest tile extent along M or N of any tile configuration.
constexpr int64_t kGemmMaxTileRows = 128;

// True when every byte offset a buffer-resource tile load forms stays below
// 2^31 - 1 for operand row strides lda and ldb (elements), reduction depth K
// (elements) and element size esize (bytes).  The last row of a tile is at
// (kGemmMaxTileRows - 1) * ld; the K stages walk 128 bytes at a time up to K
// rounded up to a whole stage, and a lane's chunk adds at most one more
// stage.
inline bool gemm_offsets_fit(int64_t lda, int64_t ldb, int64_t K, int64_t esize) {
  if (lda < 0 || ldb < 0 || K < 0 || esize <= 0) return false;
  const int64_t ld = lda > ldb ? lda : ldb;
  const int64_t kbytes = (K * esize + 127) / 128 * 128;
  const int64_t worst = (kGemmMaxTileRows - 1) * ld * esize + kbytes + 128;
  return worst < (int64_t)0x7fffffff;
}

}  // namespace rid
