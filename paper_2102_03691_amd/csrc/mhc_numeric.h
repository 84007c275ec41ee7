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

// OCP e4m3 (gfx950 native fp8): largest finite magnitude 448.  The hardware
// conversion returns NaN beyond that, so callers clamp first.
constexpr float FP8_MAX = 448.f;

// Round a pair of floats to e4m3 (round-to-nearest-even), packed in the low 16 bits.
__device__ __forceinline__ uint32_t fp8x2(float a, float b) {
  a = fminf(fmaxf(a, -FP8_MAX), FP8_MAX);
  b = fminf(fmaxf(b, -FP8_MAX), FP8_MAX);
  return (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false) & 0xFFFFu;
}

// Decode byte `sel` (0..3) of a packed e4m3 word.
__device__ __forceinline__ float fp8_to_f32(uint32_t w, int sel) {
  switch (sel) {
    case 0: return __builtin_amdgcn_cvt_f32_fp8((int)w, 0);
    case 1: return __builtin_amdgcn_cvt_f32_fp8((int)w, 1);
    case 2: return __builtin_amdgcn_cvt_f32_fp8((int)w, 2);
    default: return __builtin_amdgcn_cvt_f32_fp8((int)w, 3);
  }
}

// 16 scaled values -> 16 e4m3 bytes (hi), and optionally the e4m3 residuals
// (lo) so that x ~= hi + lo; written as two 16-byte words.
__device__ __forceinline__ void quant16_fp8(const float* x, uint32_t hi[4], uint32_t lo[4], bool want_lo) {
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    const uint32_t h01 = fp8x2(x[4 * w + 0], x[4 * w + 1]);
    const uint32_t h23 = fp8x2(x[4 * w + 2], x[4 * w + 3]);
    hi[w] = h01 | (h23 << 16);
    if (want_lo) {
      const float r0 = x[4 * w + 0] - fp8_to_f32(hi[w], 0);
      const float r1 = x[4 * w + 1] - fp8_to_f32(hi[w], 1);
      const float r2 = x[4 * w + 2] - fp8_to_f32(hi[w], 2);
      const float r3 = x[4 * w + 3] - fp8_to_f32(hi[w], 3);
      lo[w] = fp8x2(r0, r1) | (fp8x2(r2, r3) << 16);
    } else {
      lo[w] = 0;
    }
  }
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
