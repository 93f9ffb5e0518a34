// Two-term bf16 split of fp32 values: hi = bf16(x), lo = bf16(x - hi), both rounded to nearest
// even (x - hi is exact in fp32).  Shared by the projector-table generator, which stores the
// planes once, and the GEMM loaders, which split their fp32 operands on the fly; both must
// produce identical bits for identical inputs.
#pragma once

#include <hip/hip_runtime.h>

namespace pw {

struct Split2 {
  unsigned short h, l;
};

__device__ __forceinline__ unsigned short bf16_bits(float x) {
  const __bf16 b = (__bf16)x;  // round to nearest even
  return __builtin_bit_cast(unsigned short, b);
}
__device__ __forceinline__ float bf16_val(unsigned short u) {
  return __builtin_bit_cast(float, (unsigned int)u << 16);
}
__device__ __forceinline__ Split2 split(float x) {
  Split2 s;
  s.h = bf16_bits(x);
  s.l = bf16_bits(x - bf16_val(s.h));
  return s;
}
// Packs two bf16 values into one word, the first in the low half (memory order).
__device__ __forceinline__ unsigned int pack(unsigned short lo16, unsigned short hi16) {
  return (unsigned int)lo16 | ((unsigned int)hi16 << 16);
}

}  // namespace pw
