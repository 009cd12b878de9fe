// Shared host/device helpers of the rid library (gfx950 / CDNA4 only).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>

#include "rid.h"

namespace rid {

// Status-carrying exception used inside the library; never crosses the C ABI.
struct Error : std::runtime_error {
  rid_status code;
  Error(rid_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define RID_HIP(call)                                                              \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess)                                                          \
      throw ::rid::Error(RID_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define RID_CHECK(cond, code, msg)                     \
  do {                                                 \
    if (!(cond)) throw ::rid::Error((code), (msg));    \
  } while (0)

typedef __hip_bfloat16 bf16;

__host__ __device__ inline int ceil_div(int a, int b) { return (a + b - 1) / b; }
__host__ __device__ inline long ceil_div_l(long a, long b) { return (a + b - 1) / b; }

// Round-to-nearest-even float -> bf16 and back, written out so that host and
// device agree bit for bit.
__host__ __device__ inline uint16_t f32_to_bf16_bits(float f) {
  union { float f; uint32_t u; } v;
  v.f = f;
  uint32_t u = v.u;
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40);
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return (uint16_t)(u >> 16);
}
__host__ __device__ inline float bf16_bits_to_f32(uint16_t b) {
  union { float f; uint32_t u; } v;
  v.u = ((uint32_t)b) << 16;
  return v.f;
}

// Wavefront-wide sum (64 lanes) of a double / float with DPP-free shuffles.
__device__ inline double wave_sum(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}
__device__ inline float wave_sum(float x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

}  // namespace rid
