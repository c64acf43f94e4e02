// Storage of the Kahan compensation term in bfloat16 (FP32's exponent, 8
// significant bits).  The compensation holds the low-order part lost by the
// last FP32 addition; storing it with 8 significant bits changes what the
// next step corrects by at most 2^-8 of it, i.e. 2^-8 of one FP32 rounding
// per term, and halves the compensation's HBM traffic.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstring>

namespace tbs {

// Round-to-nearest-even of an FP32 value to its upper 16 bits (NaN stays NaN:
// the rounding increment never carries out of a NaN's exponent field, whose
// quiet bit is set).
__host__ __device__ inline uint32_t bf16_bits(float f) {
  uint32_t b;
#ifdef __HIP_DEVICE_COMPILE__
  b = __float_as_uint(f);
#else
  std::memcpy(&b, &f, 4);
#endif
  return (b + 0x7fffu + ((b >> 16) & 1u)) >> 16;
}

__host__ __device__ inline float bf16_value(uint32_t h) {
  const uint32_t b = h << 16;
#ifdef __HIP_DEVICE_COMPILE__
  return __uint_as_float(b);
#else
  float f;
  std::memcpy(&f, &b, 4);
  return f;
#endif
}

// A complex compensation (re, im) as one 32-bit word: re in the low half.
__host__ __device__ inline uint32_t bf16_pack(float re, float im) {
  return bf16_bits(re) | (bf16_bits(im) << 16);
}
__host__ __device__ inline void bf16_unpack(uint32_t w, float& re, float& im) {
  re = bf16_value(w & 0xffffu);
  im = bf16_value(w >> 16);
}

}  // namespace tbs
