// FP8 (OCP e4m3) path on gfx950: the Q/K/V, projection and MLP GEMMs take e4m3 operands with
// per-tensor scales and accumulate in FP32 on v_mfma_f32_16x16x128_f8f6f4; LayerNorm
// statistics, softmax and the residual stream stay FP32 (attention itself runs in BF16).
//
// Scaling: a tensor T is stored as e4m3(T / s) with s = amax(|T|) / 448 (s = 1 when amax is
// 0), round to nearest even; the GEMM epilogue multiplies by s_A * s_W.  Weight scales are
// fixed at load; activation scales come from the current call: an amax pass (or the epilogue
// of the producing kernel) max-reduces |T| into a per-block slot with an atomic max on the
// float bits (valid for non-negative floats), and the consumer reads the slot.
//
// MFMA 16x16x128 f8f6f4 operands: lane l supplies row/column (l % 16) with 32 consecutive
// k values in group (l / 16); A and B use the same k slots, so any k order common to both is
// legal.  The double-rate hazard rule of the BF16 kernels applies: MFMA groups are fenced.
#include "dr_device.h"
#include "dr_internal.h"

namespace dr {

typedef int i32x8_t __attribute__((ext_vector_type(8)));

__device__ __forceinline__ f32x4_t mfma_fp8(const i32x8_t& a, const i32x8_t& b, const f32x4_t& c) {
  // format 0 = e4m3 for both operands, no block scaling
  return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, c, 0, 0, 0, 0, 0, 0);
}

__device__ __forceinline__ void fp8_group_begin() { __builtin_amdgcn_sched_barrier(0); }
__device__ __forceinline__ void fp8_group_end() {
  __builtin_amdgcn_sched_barrier(0);
  asm volatile("s_nop 7" ::: "memory");
  __builtin_amdgcn_sched_barrier(0);
}

// two floats -> two e4m3 bytes (round to nearest even, hardware conversion); inputs are
// clamped to the finite range first so that rounding overshoot of a scaled value can never
// become NaN
__device__ __forceinline__ uint32_t f32x2_to_fp8(float a, float b) {
  a = fminf(fmaxf(a, -448.0f), 448.0f);
  b = fminf(fmaxf(b, -448.0f), 448.0f);
  return (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false) & 0xffffu;
}

__device__ __forceinline__ float scale_of(const float* amax_slot) {
  const float a = *amax_slot;
  return a > 0.f ? a / 448.0f : 1.0f;
}

__device__ __forceinline__ void atomic_amax(float* slot, float v) {
  // non-negative floats order like their bit patterns.  Read first: once the slot holds the
  // call's maximum, later blocks skip the atomic (many blocks contend for one address; a
  // stale read only costs an atomic that changes nothing)
  if (v > *reinterpret_cast<volatile float*>(slot))
    atomicMax(reinterpret_cast<unsigned int*>(slot), __float_as_uint(v));
}

__device__ __forceinline__ float wave_max_abs(float v) { return wave_max(fabsf(v)); }

// ------------------------------------------------------------------------------------------
// elementwise quantisation (weights at load, and the test hook)
// ------------------------------------------------------------------------------------------
__global__ void quantize_fp8_kernel(const float* __restrict__ in, uint8_t* __restrict__ out, size_t n,
                                    float inv_scale) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; 2 * i < n; i += (size_t)gridDim.x * blockDim.x) {
    const float a = in[2 * i] * inv_scale;
    const float b = (2 * i + 1 < n) ? in[2 * i + 1] * inv_scale : 0.f;
    const uint32_t pk = f32x2_to_fp8(a, b);
    out[2 * i] = (uint8_t)(pk & 0xff);
    if (2 * i + 1 < n) out[2 * i + 1] = (uint8_t)(pk >> 8);
  }
}

void launch_quantize_fp8(const float* in, uint8_t* out, size_t n, float inv_scale, hipStream_t s) {
  size_t grid = (n / 2 + 256) / 256;
  if (grid > 8192) grid = 8192;
  if (grid) quantize_fp8_kernel<<<(unsigned)grid, 256, 0, s>>>(in, out, n, inv_scale);
}

__global__ void zero_f32_kernel(float* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.f;
}

void launch_zero_f32(float* p, int n, hipStream_t s) {
  if (n > 0) zero_f32_kernel<<<(n + 255) / 256, 256, 0, s>>>(p, n);
}

// ------------------------------------------------------------------------------------------
// amax of LayerNorm outputs over rows x[rows[r]] (r < *nrows) or x[r] (r < nrows_max, only
// rows whose window has queries when wcount is given).  One wavefront per row.
// ------------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) ln_amax_kernel(const float* __restrict__ x, const int32_t* __restrict__ rows,
                                                      const int32_t* __restrict__ nrows_dev, int nrows_max,
                                                      const int32_t* __restrict__ wcount, int S, int C,
                                                      const float* __restrict__ g, const float* __restrict__ b,
                                                      float* slot) {
  const int lane = threadIdx.x & 63;
  const int nrows = nrows_dev ? nrows_dev[0] : nrows_max;
  float mx = 0.f;
  for (int r = blockIdx.x * 4 + (threadIdx.x >> 6); r < nrows; r += gridDim.x * 4) {
    if (wcount && wcount[r / S] == 0) continue;
    const float* xr = x + (size_t)(rows ? rows[r] : r) * C;
    const int per = C / 64;
    float v[16];
    float s = 0.f;
    for (int e = 0; e < per; ++e) {
      v[e] = xr[lane + 64 * e];
      s += v[e];
    }
    const float mean = wave_sum(s) / C;
    float q = 0.f;
    for (int e = 0; e < per; ++e) {
      const float d = v[e] - mean;
      q += d * d;
    }
    const float rstd = rsqrtf(wave_sum(q) / C + 1e-5f);
    for (int e = 0; e < per; ++e) {
      const int c = lane + 64 * e;
      mx = fmaxf(mx, fabsf((v[e] - mean) * rstd * g[c] + b[c]));
    }
  }
  // one atomic per block
  __shared__ float wred[4];
  mx = wave_max(mx);
  if (lane == 0) wred[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    mx = fmaxf(fmaxf(wred[0], wred[1]), fmaxf(wred[2], wred[3]));
    if (mx > 0.f) atomic_amax(slot, mx);
  }
}

void launch_ln_amax(const float* x, const int32_t* rows, const int32_t* nrows_dev, int nrows_max,
                    const int32_t* wcount, int S, int C, const float* g, const float* b, float* slot,
                    hipStream_t s) {
  if (nrows_max <= 0) return;
  int grid = (nrows_max + 3) / 4;
  if (grid > 2048) grid = 2048;
  ln_amax_kernel<<<grid, 256, 0, s>>>(x, rows, nrows_dev, nrows_max, wcount, S, C, g, b, slot);
}

// ------------------------------------------------------------------------------------------
// LayerNorm-fused FP8 panel GEMM.  Block = 512 threads = 8 waves (2 rows x 4 columns), tile
// 128 rows x BN columns, wave tile 64 x BN/4.  Prologue: LayerNorm of the 128 rows in FP32,
// divided by the activation scale and cast to e4m3 into an LDS panel holding the full K;
// weights (e4m3 [BN][K]) stream through a two-stage LDS ring of 128-byte k chunks.
// ------------------------------------------------------------------------------------------
constexpr int F8_PANEL_M = 128;
constexpr int F8_THREADS = 512;
constexpr int F8_BK = 128;                 // fp8 elements per stage = one MFMA k step
constexpr int F8_WST = F8_BK + 16;         // stage row stride in bytes

template <int BN>
__host__ __device__ constexpr size_t f8_panel_smem(int K) {
  return (size_t)F8_PANEL_M * (K + 16) + (size_t)2 * BN * F8_WST;
}

constexpr int F8_LN_BATCH = 8;

template <int PER2>
__device__ __forceinline__ void f8_ln_rows(const float* __restrict__ x, const int32_t* __restrict__ rows, int M,
                                           int m0, const float* __restrict__ lng, const float* __restrict__ lnb,
                                           float inv_sa, uint8_t* apanel, int KS) {
  constexpr int K = 128 * PER2;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int r0 = wv; r0 < F8_PANEL_M; r0 += F8_LN_BATCH * (F8_THREADS / 64)) {
    float2 v[F8_LN_BATCH][PER2];
#pragma unroll
    for (int j = 0; j < F8_LN_BATCH; ++j) {
      const int m = m0 + r0 + j * (F8_THREADS / 64);
      if (m < M) {
        const float* xr = x + (size_t)(rows ? rows[m] : m) * K;
#pragma unroll
        for (int e = 0; e < PER2; ++e) v[j][e] = *reinterpret_cast<const float2*>(xr + 2 * lane + 128 * e);
      } else {
#pragma unroll
        for (int e = 0; e < PER2; ++e) v[j][e] = make_float2(0.f, 0.f);
      }
    }
#pragma unroll
    for (int j = 0; j < F8_LN_BATCH; ++j) {
      const int r = r0 + j * (F8_THREADS / 64);
      uint8_t* arow = apanel + (size_t)r * KS;
      if (m0 + r >= M) {
#pragma unroll
        for (int e = 0; e < PER2; ++e) *reinterpret_cast<uint16_t*>(arow + 2 * lane + 128 * e) = 0;
        continue;
      }
      float sum = 0.f;
#pragma unroll
      for (int e = 0; e < PER2; ++e) sum += v[j][e].x + v[j][e].y;
      const float mean = wave_sum(sum) / K;
      float sq = 0.f;
#pragma unroll
      for (int e = 0; e < PER2; ++e) {
        const float d0 = v[j][e].x - mean, d1 = v[j][e].y - mean;
        sq += d0 * d0 + d1 * d1;
      }
      const float rstd = rsqrtf(wave_sum(sq) / K + 1e-5f);
#pragma unroll
      for (int e = 0; e < PER2; ++e) {
        const int c = 2 * lane + 128 * e;
        const float y0 = ((v[j][e].x - mean) * rstd * lng[c] + lnb[c]) * inv_sa;
        const float y1 = ((v[j][e].y - mean) * rstd * lng[c + 1] + lnb[c + 1]) * inv_sa;
        *reinterpret_cast<uint16_t*>(arow + c) = (uint16_t)f32x2_to_fp8(y0, y1);
      }
    }
  }
}

template <int BN, class Epi>
__device__ __forceinline__ void f8_panel_gemm(const float* __restrict__ x, const int32_t* __restrict__ rows, int M,
                                              int m0, int K, const float* __restrict__ lng,
                                              const float* __restrict__ lnb, float inv_sa,
                                              const uint8_t* __restrict__ W, int n0, uint8_t* smem, Epi& epi) {
  constexpr int FN = BN / 64;
  constexpr int W_CHUNKS = BN * F8_BK / 16 / F8_THREADS;  // 16-byte chunks per thread per stage
  static_assert(FN >= 1 && W_CHUNKS >= 1, "fp8 panel tile too small");
  const int KS = K + 16;
  uint8_t* apanel = smem;
  uint8_t* wst = smem + (size_t)F8_PANEL_M * KS;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int wm = wv >> 2, wn = wv & 3;
  const int l16 = lane & 15, kg = lane >> 4;

  u32x4_t rw[W_CHUNKS];
  auto load_w = [&](int k0) {
#pragma unroll
    for (int c = 0; c < W_CHUNKS; ++c) {
      const int id = t + F8_THREADS * c;
      rw[c] = *reinterpret_cast<const u32x4_t*>(W + (size_t)(n0 + (id >> 3)) * K + k0 + (id & 7) * 16);
    }
  };
  auto stash_w = [&](int buf) {
#pragma unroll
    for (int c = 0; c < W_CHUNKS; ++c) {
      const int id = t + F8_THREADS * c;
      *reinterpret_cast<u32x4_t*>(wst + ((size_t)buf * BN + (id >> 3)) * F8_WST + (id & 7) * 16) = rw[c];
    }
  };
  load_w(0);

  // LayerNorm prologue: lane handles channel pairs (2*lane + 128*e, +1); rows in batches whose
  // loads are issued before the first reduction
  switch (K / 128) {
    case 1: f8_ln_rows<1>(x, rows, M, m0, lng, lnb, inv_sa, apanel, KS); break;
    case 2: f8_ln_rows<2>(x, rows, M, m0, lng, lnb, inv_sa, apanel, KS); break;
    case 3: f8_ln_rows<3>(x, rows, M, m0, lng, lnb, inv_sa, apanel, KS); break;
    case 4: f8_ln_rows<4>(x, rows, M, m0, lng, lnb, inv_sa, apanel, KS); break;
    case 6: f8_ln_rows<6>(x, rows, M, m0, lng, lnb, inv_sa, apanel, KS); break;
    default: f8_ln_rows<8>(x, rows, M, m0, lng, lnb, inv_sa, apanel, KS); break;
  }
  stash_w(0);
  __syncthreads();

  f32x4_t acc[4][FN];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};

  const int nk = K / F8_BK;
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) load_w((kt + 1) * F8_BK);
    const uint8_t* wb = wst + (size_t)buf * BN * F8_WST;
    i32x8_t af[4], wf[FN];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint8_t* p = apanel + (size_t)(wm * 64 + i * 16 + l16) * KS + kt * F8_BK + kg * 32;
      const uint4 lo = *reinterpret_cast<const uint4*>(p), hi = *reinterpret_cast<const uint4*>(p + 16);
      af[i] = i32x8_t{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
    }
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const uint8_t* p = wb + (size_t)(wn * (BN / 4) + j * 16 + l16) * F8_WST + kg * 32;
      const uint4 lo = *reinterpret_cast<const uint4*>(p), hi = *reinterpret_cast<const uint4*>(p + 16);
      wf[j] = i32x8_t{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
    }
    fp8_group_begin();
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) acc[i][j] = mfma_fp8(wf[j], af[i], acc[i][j]);
    fp8_group_end();
    if (kt + 1 < nk) {
      stash_w(buf ^ 1);
      __syncthreads();
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int m = m0 + wm * 64 + i * 16 + l16;
    const bool ok = m < M;
#pragma unroll
    for (int j = 0; j < FN; ++j) epi(ok, m, n0 + wn * (BN / 4) + j * 16 + kg * 4, acc[i][j]);
  }
  epi.finish();
}

// Q rows [N][C] multiplied by qscale (log2(e)/sqrt(dh): the attention kernel takes Q scaled
// for base-2 exponentials), K [win][head][Spad][dh], V transposed [win][head][dh][spv] -- the
// layouts of the BF16 path, so both precisions share one attention kernel.
struct F8QkvEpi {
  const float* bias;
  const float* wscale;  // per block: [0] s_q, [1] s_k, [2] s_v
  float sa, qscale;
  bf16 *q, *k, *vt;
  int C, dh, heads, Spad, S, spv;
  __device__ __forceinline__ void operator()(bool ok, int m, int n, const f32x4_t& a) const {
    if (!ok) return;
    const int part = n < C ? 0 : (n < 2 * C ? 1 : 2);
    const float sc = sa * wscale[part];
    const float4 b4 = *reinterpret_cast<const float4*>(bias + n);
    float y0 = a[0] * sc + b4.x, y1 = a[1] * sc + b4.y, y2 = a[2] * sc + b4.z, y3 = a[3] * sc + b4.w;
    if (part == 0) {
      uint2 pk;
      pk.x = pack_bf2(y0 * qscale, y1 * qscale);
      pk.y = pack_bf2(y2 * qscale, y3 * qscale);
      *reinterpret_cast<uint2*>(q + (size_t)m * C + n) = pk;
      return;
    }
    const int c = n - part * C, hh = c / dh, d = c - hh * dh;
    const int w = m / S, s = m - w * S;
    if (part == 1) {
      uint2 pk;
      pk.x = pack_bf2(y0, y1);
      pk.y = pack_bf2(y2, y3);
      *reinterpret_cast<uint2*>(k + (((size_t)w * heads + hh) * Spad + s) * dh + d) = pk;
    } else {
      bf16* dst = vt + (((size_t)w * heads + hh) * dh + d) * spv + s;
      dst[0] = f2bf(y0);
      dst[spv] = f2bf(y1);
      dst[2 * spv] = f2bf(y2);
      dst[3 * spv] = f2bf(y3);
    }
  }
  __device__ __forceinline__ void finish() const {}
};

template <int BN>
__global__ void __launch_bounds__(F8_THREADS) ln_qkv_fp8_kernel(Geo g, int C, int heads, int Spad,
                                                                const float* __restrict__ x,
                                                                const uint8_t* __restrict__ flag,
                                                                const int32_t* __restrict__ wcount,
                                                                const float* __restrict__ lng,
                                                                const float* __restrict__ lnb,
                                                                const uint8_t* __restrict__ W,
                                                                const float* __restrict__ wscale,
                                                                const float* __restrict__ bias,
                                                                const float* __restrict__ amax_u, float qscale,
                                                                int spv, bf16* q, bf16* k, bf16* vt) {
  extern __shared__ __align__(16) uint8_t smem_f8[];
  const int M = g.N;
  const int n0 = blockIdx.x * BN, m0 = blockIdx.y * F8_PANEL_M;
  const bool is_q = n0 < C;
  int need = 0;
  if (threadIdx.x < F8_PANEL_M && m0 + threadIdx.x < M) {
    const int m = m0 + threadIdx.x;
    need = is_q ? flag[m] != 0 : wcount[m / g.S] > 0;
  }
  if (!__syncthreads_or(need)) return;
  const float sa = scale_of(amax_u);
  F8QkvEpi epi{bias, wscale, sa, qscale, q, k, vt, C, C / heads, heads, Spad, g.S, spv};
  f8_panel_gemm<BN>(x, nullptr, M, m0, C, lng, lnb, 1.0f / sa, W, n0, smem_f8, epi);
}

// GELU epilogue writing bf16 h and max-reducing |h| into a slot.
struct F8GeluEpi {
  const float* bias;
  float sc;
  bf16* h;
  float* amax_h;
  int R;
  float mx;
  __device__ __forceinline__ void operator()(bool ok, int m, int n, const f32x4_t& a) {
    if (!ok) return;
    const float4 b4 = *reinterpret_cast<const float4*>(bias + n);
    const float y0 = gelu_fast(a[0] * sc + b4.x), y1 = gelu_fast(a[1] * sc + b4.y);
    const float y2 = gelu_fast(a[2] * sc + b4.z), y3 = gelu_fast(a[3] * sc + b4.w);
    mx = fmaxf(mx, fmaxf(fmaxf(fabsf(y0), fabsf(y1)), fmaxf(fabsf(y2), fabsf(y3))));
    uint2 pk;
    pk.x = pack_bf2(y0, y1);
    pk.y = pack_bf2(y2, y3);
    *reinterpret_cast<uint2*>(h + (size_t)m * R + n) = pk;
  }
  __device__ __forceinline__ void finish() {
    const float w = wave_max(mx);
    if ((threadIdx.x & 63) == 0 && w > 0.f) atomic_amax(amax_h, w);
  }
};

template <int BN>
__global__ void __launch_bounds__(F8_THREADS) ln_fc1_fp8_kernel(int C, int R, const float* __restrict__ x,
                                                                const int32_t* __restrict__ idx,
                                                                const int32_t* __restrict__ nq,
                                                                const float* __restrict__ lng,
                                                                const float* __restrict__ lnb,
                                                                const uint8_t* __restrict__ W, float s_w,
                                                                const float* __restrict__ bias,
                                                                const float* __restrict__ amax_u, bf16* h,
                                                                float* amax_h) {
  extern __shared__ __align__(16) uint8_t smem_f8[];
  const int M = nq[0];
  const int n0 = blockIdx.x * BN, m0 = blockIdx.y * F8_PANEL_M;
  if (m0 >= M) return;
  const float sa = scale_of(amax_u);
  F8GeluEpi epi{bias, sa * s_w, h, amax_h, R, 0.f};
  f8_panel_gemm<BN>(x, idx, M, m0, C, lng, lnb, 1.0f / sa, W, n0, smem_f8, epi);
}

template <class Kern>
static void f8_allow(Kern k, size_t smem, size_t& granted) {
  if (smem > 65536 && smem > granted) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k), hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    granted = smem;
  }
}

template <int BN>
static void qkv_fp8_launch(const Geo& g, int C, int heads, int Spad, const float* x, const uint8_t* flag,
                           const int32_t* wcount, const float* lng, const float* lnb, const uint8_t* w,
                           const float* wscale, const float* bias, const float* amax_u, float qscale, int spv,
                           bf16* q, bf16* k, bf16* vt, hipStream_t s) {
  static size_t granted = 0;
  const size_t smem = f8_panel_smem<BN>(C);
  f8_allow(ln_qkv_fp8_kernel<BN>, smem, granted);
  dim3 grid(3 * C / BN, (g.N + F8_PANEL_M - 1) / F8_PANEL_M);
  ln_qkv_fp8_kernel<BN><<<grid, F8_THREADS, smem, s>>>(g, C, heads, Spad, x, flag, wcount, lng, lnb, w, wscale,
                                                        bias, amax_u, qscale, spv, q, k, vt);
}

void launch_ln_qkv_fp8(const Geo& g, int C, int heads, int Spad, const float* x, const uint8_t* flag,
                       const int32_t* wcount, const float* lng, const float* lnb, const uint8_t* w,
                       const float* wscale, const float* bias, const float* amax_u, float qscale, int spv, bf16* q,
                       bf16* k, bf16* vt, hipStream_t s) {
  if (C % 256 == 0)
    qkv_fp8_launch<256>(g, C, heads, Spad, x, flag, wcount, lng, lnb, w, wscale, bias, amax_u, qscale, spv, q, k, vt, s);
  else if (C % 128 == 0)
    qkv_fp8_launch<128>(g, C, heads, Spad, x, flag, wcount, lng, lnb, w, wscale, bias, amax_u, qscale, spv, q, k, vt, s);
  else
    qkv_fp8_launch<64>(g, C, heads, Spad, x, flag, wcount, lng, lnb, w, wscale, bias, amax_u, qscale, spv, q, k, vt, s);
}

template <int BN>
static void fc1_fp8_launch(int m_max, int C, int R, const float* x, const int32_t* idx, const int32_t* nq,
                           const float* lng, const float* lnb, const uint8_t* w, float s_w, const float* bias,
                           const float* amax_u, bf16* h, float* amax_h, hipStream_t s) {
  static size_t granted = 0;
  const size_t smem = f8_panel_smem<BN>(C);
  f8_allow(ln_fc1_fp8_kernel<BN>, smem, granted);
  dim3 grid(R / BN, (m_max + F8_PANEL_M - 1) / F8_PANEL_M);
  ln_fc1_fp8_kernel<BN><<<grid, F8_THREADS, smem, s>>>(C, R, x, idx, nq, lng, lnb, w, s_w, bias, amax_u, h, amax_h);
}

void launch_ln_fc1_fp8(int m_max, int C, int R, const float* x, const int32_t* idx, const int32_t* nq,
                       const float* lng, const float* lnb, const uint8_t* w, float s_w, const float* bias,
                       const float* amax_u, bf16* h, float* amax_h, hipStream_t s) {
  if (m_max <= 0) return;
  if (R % 256 == 0)
    fc1_fp8_launch<256>(m_max, C, R, x, idx, nq, lng, lnb, w, s_w, bias, amax_u, h, amax_h, s);
  else if (R % 128 == 0)
    fc1_fp8_launch<128>(m_max, C, R, x, idx, nq, lng, lnb, w, s_w, bias, amax_u, h, amax_h, s);
  else
    fc1_fp8_launch<64>(m_max, C, R, x, idx, nq, lng, lnb, w, s_w, bias, amax_u, h, amax_h, s);
}

// ------------------------------------------------------------------------------------------
// FP8 GEMM over compact bf16 rows with a residual epilogue: x[res_rows[m], n] += s_a s_w
// (e4m3(A/s_a) . e4m3(W)^T)[m, n] + bias[n].  256 threads = 2 x 2 waves, tile 64 x 128,
// 128-wide k stages; A is converted bf16 -> e4m3 while it is staged into LDS.
// ------------------------------------------------------------------------------------------
constexpr int G8_BM = 64, G8_BN = 128;

__global__ void __launch_bounds__(256) gemm_fp8_resid_kernel(const bf16* __restrict__ A, const int32_t* __restrict__ m_dev,
                                                             int K, const uint8_t* __restrict__ W, float s_w,
                                                             const float* __restrict__ amax_a,
                                                             const float* __restrict__ bias, int Nout,
                                                             float* __restrict__ x, const int32_t* __restrict__ res_rows) {
  __shared__ __align__(16) uint8_t As[2][G8_BM][F8_WST];
  __shared__ __align__(16) uint8_t Ws[2][G8_BN][F8_WST];
  const int M = m_dev[0];
  const int m0 = blockIdx.x * G8_BM, n0 = blockIdx.y * G8_BN;
  if (m0 >= M) return;
  const float sa = scale_of(amax_a);
  const float inv_sa = 1.0f / sa;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int wm = wv >> 1, wn = wv & 1;
  const int l16 = lane & 15, kg = lane >> 4;
  // A stage: 64 rows x 128 k = 1024 chunks of 8 bf16 -> 4 per thread; W stage: 128 rows x
  // 128 B = 1024 chunks of 16 B -> 4 per thread
  u32x4_t ra[4], rw[4];
  auto load = [&](int k0) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int id = t + 256 * c;
      const int row = id >> 4, col = (id & 15) * 8;
      const int m = m0 + row;
      ra[c] = m < M ? *reinterpret_cast<const u32x4_t*>(A + (size_t)m * K + k0 + col) : u32x4_t{0u, 0u, 0u, 0u};
      const int wr = id >> 3, wc = (id & 7) * 16;
      rw[c] = *reinterpret_cast<const u32x4_t*>(W + (size_t)(n0 + wr) * K + k0 + wc);
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int id = t + 256 * c;
      const int row = id >> 4, col = (id & 15) * 8;
      const uint32_t w4[4] = {ra[c].x, ra[c].y, ra[c].z, ra[c].w};
      uint32_t lo = 0, hi = 0;
      lo = f32x2_to_fp8(bf2f(w4[0] & 0xffff) * inv_sa, bf2f(w4[0] >> 16) * inv_sa) |
           (f32x2_to_fp8(bf2f(w4[1] & 0xffff) * inv_sa, bf2f(w4[1] >> 16) * inv_sa) << 16);
      hi = f32x2_to_fp8(bf2f(w4[2] & 0xffff) * inv_sa, bf2f(w4[2] >> 16) * inv_sa) |
           (f32x2_to_fp8(bf2f(w4[3] & 0xffff) * inv_sa, bf2f(w4[3] >> 16) * inv_sa) << 16);
      *reinterpret_cast<uint2*>(&As[buf][row][col]) = make_uint2(lo, hi);
      const int wr = id >> 3, wc = (id & 7) * 16;
      *reinterpret_cast<u32x4_t*>(&Ws[buf][wr][wc]) = rw[c];
    }
  };
  f32x4_t acc[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};
  load(0);
  stash(0);
  __syncthreads();
  const int nk = K / F8_BK;
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) load((kt + 1) * F8_BK);
    i32x8_t af[2], wf[4];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const uint8_t* p = &As[buf][wm * 32 + i * 16 + l16][kg * 32];
      const uint4 lo = *reinterpret_cast<const uint4*>(p), hi = *reinterpret_cast<const uint4*>(p + 16);
      af[i] = i32x8_t{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint8_t* p = &Ws[buf][wn * 64 + j * 16 + l16][kg * 32];
      const uint4 lo = *reinterpret_cast<const uint4*>(p), hi = *reinterpret_cast<const uint4*>(p + 16);
      wf[j] = i32x8_t{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
    }
    fp8_group_begin();
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = mfma_fp8(wf[j], af[i], acc[i][j]);
    fp8_group_end();
    if (kt + 1 < nk) {
      stash(buf ^ 1);
      __syncthreads();
    }
  }
  const float sc = sa * s_w;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int m = m0 + wm * 32 + i * 16 + l16;
    if (m >= M) continue;
    const int dst = res_rows[m];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int n = n0 + wn * 64 + j * 16 + kg * 4;
      const float4 b4 = *reinterpret_cast<const float4*>(bias + n);
      float4* p = reinterpret_cast<float4*>(x + (size_t)dst * Nout + n);
      float4 xv = *p;
      xv.x += acc[i][j][0] * sc + b4.x;
      xv.y += acc[i][j][1] * sc + b4.y;
      xv.z += acc[i][j][2] * sc + b4.z;
      xv.w += acc[i][j][3] * sc + b4.w;
      *p = xv;
    }
  }
}

void launch_gemm_fp8_resid(const bf16* A, const int32_t* m_dev, int m_max, int K, const uint8_t* W, float s_w,
                           const float* amax_a, const float* bias, int Nout, float* x, const int32_t* res_rows,
                           hipStream_t s) {
  if (m_max <= 0) return;
  dim3 grid((m_max + G8_BM - 1) / G8_BM, Nout / G8_BN);
  gemm_fp8_resid_kernel<<<grid, 256, 0, s>>>(A, m_dev, K, W, s_w, amax_a, bias, Nout, x, res_rows);
}

bool fp8_supported(int C, int R) { return C % 128 == 0 && R % 128 == 0; }

}  // namespace dr
