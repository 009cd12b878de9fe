// CPU stand-in (test infrastructure only): the bfloat16 storage type.
#pragma once
#include <cstdint>
struct __hip_bfloat16 {
  uint16_t x;
};
