// Device helpers for gfx950 kernels: bfloat16 conversion, 64-lane wavefront reductions,
// MFMA operand types, GELU.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>
#include <utility>

namespace dr {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4_t __attribute__((ext_vector_type(4)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef uint16_t u16x8_t __attribute__((ext_vector_type(8)));
typedef uint16_t u16x4_t __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));  // 16-byte load/store unit

constexpr int WAVE = 64;

// Compile-time loop: f(std::integral_constant<int, i>) for i = 0 .. N-1.  Register arrays
// indexed only through it keep constant indices from the first optimisation pass on, so they
// stay in VGPRs (a runtime-indexed array can be placed in scratch or LDS, which turns every
// register prefetch into a round trip through memory).
template <class F, int... I>
__device__ __forceinline__ void static_for_impl(F& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));

// float -> bfloat16 bits, round to nearest even (NaN stays NaN): the conversion compiles to
// gfx950's v_cvt_pk_bf16_f32, one instruction per pair.
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }

__device__ __forceinline__ uint32_t pack_bf2(float a, float b) {
  const bf16x2_t v = {(__bf16)a, (__bf16)b};
  return __builtin_bit_cast(uint32_t, v);
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, WAVE));
  return v;
}

// Exact GELU: 0.5 z (1 + erf(z / sqrt(2))).
__device__ __forceinline__ float gelu_erf(float z) {
  return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f));
}

// GELU for the reduced-precision paths, whose result is rounded to bf16 or e4m3 next: erf
// from the rational approximation of Abramowitz & Stegun, Handbook of Mathematical Functions,
// formula 7.1.26 (erf x = 1 - (a1 t + a2 t^2 + a3 t^3 + a4 t^4 + a5 t^5) e^(-x^2),
// t = 1 / (1 + p x), x >= 0, |error| <= 1.5e-7), extended as an odd function.  One
// reciprocal, one exp2 and a handful of FMAs instead of the library erff.
__device__ __forceinline__ float gelu_fast(float z) {
  const float x = fabsf(z) * 0.70710678118654752f;
  const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, x, 1.0f));
  float p = fmaf(1.061405429f, t, -1.453152027f);
  p = fmaf(p, t, 1.421413741f);
  p = fmaf(p, t, -0.284496736f);
  p = fmaf(p, t, 0.254829592f);
  p *= t;
  const float e = __builtin_amdgcn_exp2f(-1.4426950408889634f * x * x);
  const float erf_z = __builtin_copysignf(fmaf(-p, e, 1.0f), z);
  const float hz = 0.5f * z;
  return fmaf(hz, erf_z, hz);
}

__device__ __forceinline__ float sigmoidf(float z) { return 1.0f / (1.0f + expf(-z)); }

}  // namespace dr
