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

// GELU for the reduced-precision paths, whose result is rounded to bf16 or e4m3 next:
// 0.5 z (1 + erf(z / sqrt 2)) with erf from an odd polynomial, erf x ~ x P(x^2) with P of
// degree 8, fitted here by iteratively reweighted least squares towards the minimax fit of
// erf on [0, 3] and evaluated in FP32 by Horner's rule on x clamped to [-3, 3] (beyond,
// |1 - erf x| < 2.3e-5).  Maximum absolute error of erf over the real line: 2.7e-5, so the
// GELU error is at most 1.4e-5 |z| (under 6e-5 for |z| <= 6) -- against a bf16 rounding of
// the result of 2^-9 relative, and a second linear that sums 4 C such values.  Thirteen full-rate VALU instructions, no
// transcendental: this epilogue runs once per hidden unit and query token, the largest
// element-wise cost of the network.
#define DR_ERF_P0 1.1282683610916138f
#define DR_ERF_P1 -0.3753148317337036f
#define DR_ERF_P2 0.11107926815748215f
#define DR_ERF_P3 -0.02510281279683113f
#define DR_ERF_P4 0.004235409200191498f
#define DR_ERF_P5 -0.0005110329948365688f
#define DR_ERF_P6 4.106005508219823e-05f
#define DR_ERF_P7 -1.944792757058167e-06f
#define DR_ERF_P8 4.074131609854703e-08f
#define DR_ERF_CLAMP 3.0f
__device__ __forceinline__ float gelu_fast(float z) {
  const float x = __builtin_amdgcn_fmed3f(z * 0.70710678118654752f, -DR_ERF_CLAMP, DR_ERF_CLAMP);
  const float t = x * x;
  float p = fmaf(DR_ERF_P8, t, DR_ERF_P7);
  p = fmaf(p, t, DR_ERF_P6);
  p = fmaf(p, t, DR_ERF_P5);
  p = fmaf(p, t, DR_ERF_P4);
  p = fmaf(p, t, DR_ERF_P3);
  p = fmaf(p, t, DR_ERF_P2);
  p = fmaf(p, t, DR_ERF_P1);
  p = fmaf(p, t, DR_ERF_P0);
  const float hz = 0.5f * z;
  return fmaf(hz, x * p, hz);
}

// The same GELU with its two constant factors moved into the neighbouring linears: for
// x = z / sqrt 2 (the first linear's weights and bias carry the 1/sqrt 2) it returns
// sqrt 2 GELU(z) = x (1 + erf x) (the second linear's weight carries the other 1/sqrt 2).
// Eleven full-rate instructions.
__device__ __forceinline__ float gelu_scaled(float x) {
  const float xc = __builtin_amdgcn_fmed3f(x, -DR_ERF_CLAMP, DR_ERF_CLAMP);
  const float t = xc * xc;
  float p = fmaf(DR_ERF_P8, t, DR_ERF_P7);
  p = fmaf(p, t, DR_ERF_P6);
  p = fmaf(p, t, DR_ERF_P5);
  p = fmaf(p, t, DR_ERF_P4);
  p = fmaf(p, t, DR_ERF_P3);
  p = fmaf(p, t, DR_ERF_P2);
  p = fmaf(p, t, DR_ERF_P1);
  p = fmaf(p, t, DR_ERF_P0);
  return fmaf(x, xc * p, x);
}

__device__ __forceinline__ float sigmoidf(float z) { return 1.0f / (1.0f + expf(-z)); }

}  // namespace dr
