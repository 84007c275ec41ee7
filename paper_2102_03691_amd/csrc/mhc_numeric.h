// Numeric helpers of the device code: bfloat16 splitting and compensated
// float64 summation.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mhc {

// Round a float to bfloat16 with round-to-nearest-even (finite inputs).
__device__ __forceinline__ uint16_t bf16_rne(float x) {
  uint32_t b = __float_as_uint(x);
  b += 0x7FFFu + ((b >> 16) & 1u);
  return (uint16_t)(b >> 16);
}

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// x ~= hi + lo with hi = bf16(x), lo = bf16(x - hi); |x - hi - lo| <= 2^-17 |x|.
__device__ __forceinline__ void split_bf16_from_f32(float x, uint16_t& hi, uint16_t& lo) {
  hi = bf16_rne(x);
  lo = bf16_rne(x - bf16_to_f32(hi));
}

__device__ __forceinline__ void split_bf16_from_f64(double x, uint16_t& hi, uint16_t& lo) {
  hi = bf16_rne((float)x);
  lo = bf16_rne((float)(x - (double)bf16_to_f32(hi)));
}

// Neumaier (improved Kahan-Babuska) addition: (sum + comp) tracks the exact
// running total to about one float64 rounding regardless of the count.
__device__ __forceinline__ void neumaier_add(double& sum, double& comp, double x) {
  const double t = sum + x;
  if (fabs(sum) >= fabs(x))
    comp += (sum - t) + x;
  else
    comp += (x - t) + sum;
  sum = t;
}

}  // namespace mhc
