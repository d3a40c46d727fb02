// Window attention of the training passes on the FP32 matrix cores (v_mfma_f32_16x16x4_f32).
//
// Forward with saved row statistics, then a reverse pass in two kernels that recompute the
// probabilities from Q, K and the saved (max, sum) instead of storing them: P never leaves
// the registers.  One workgroup of four wavefronts per (window, head):
//
//   fwd:  K, V of the window in LDS; per 16-query tile S^T = K Q^T, P = exp(S/sqrt(dh) - m)/l,
//         O^T = V^T P^T; writes O and (m, l) per query and head.
//   dq:   K, V in LDS; per 16-query tile P (recomputed), dP^T = V dO^T, D = rowsum(P dP),
//         dS = P (dP - D), dQ^T = K^T dS^T / sqrt(dh); writes dQ and D.
//   dkv:  Q, dO, (m, l, D) of the window's queries in LDS; per 16-key tile P and dS again
//         (query tiles in order), dV^T = dO^T P, dK^T = Q^T dS / sqrt(dh); writes dK, dV.
//
// Every sum runs in a fixed order (no atomics), so the results are deterministic.
//
// MFMA 16x16x4 (FP32): lane l supplies A[l % 16][k = l / 16] and B[k = l / 16][l % 16]; the
// result lane l holds D[4 (l / 16) + r][l % 16], r = 0..3.  Only the pairing of A's and B's
// k slots matters, so a 64-wide contraction over channels uses k-step (j, e) with lane group
// g = l / 16 supplying channel 16 j + 4 g + e (one 16-byte read per lane and j), and a
// contraction over keys (or queries) held in result layout uses k-step (tile, r) with lane
// group g supplying index 16 tile + 4 g + r -- the probabilities feed the next product
// straight from the registers.
//
// LDS rows of dh floats hold their 16-byte chunks XOR-swizzled by row (chunk c of row s at
// c ^ (s mod dh/4)), so the 16 rows read by one lane group at a fixed logical chunk fall on
// distinct banks.
#include "dr_device.h"
#include "dr_internal.h"

namespace dr {

constexpr int TA_THREADS = 256;
constexpr int TA_MAX_S = 304;  // keys (or queries) per window the LDS tiles hold

__device__ __forceinline__ f32x4_t mfma_f32_4(float a, float b, const f32x4_t& c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ void ta_fence_begin() { __builtin_amdgcn_sched_barrier(0); }
__device__ __forceinline__ void ta_fence_end() {
  __builtin_amdgcn_sched_barrier(0);
  asm volatile("s_nop 7" ::: "memory");
  __builtin_amdgcn_sched_barrier(0);
}

// element (row s, channel d) of a swizzled [rows][DH] tile
template <int DH>
__device__ __forceinline__ int ta_off(int s, int d) {
  constexpr int NCH = DH / 4;
  return s * DH + 4 * ((d >> 2) ^ (s & (NCH - 1))) + (d & 3);
}

// 16-byte chunk c of row s
template <int DH>
__device__ __forceinline__ const float4& ta_chunk(const float* t, int s, int c) {
  constexpr int NCH = DH / 4;
  return *reinterpret_cast<const float4*>(t + s * DH + 4 * (c ^ (s & (NCH - 1))));
}

// rows [0, npad) of a [rows][DH] tile from global rows src + i * ld (i < n), zero beyond n
template <int DH>
__device__ __forceinline__ void ta_stage(const float* __restrict__ src, size_t ld, int n, int npad, float* dst) {
  constexpr int NCH = DH / 4;
  for (int e = threadIdx.x; e < npad * NCH; e += TA_THREADS) {
    const int s = e / NCH, c = e - s * NCH;
    const float4 v = s < n ? *reinterpret_cast<const float4*>(src + (size_t)s * ld + 4 * c) : make_float4(0.f, 0.f, 0.f, 0.f);
    *reinterpret_cast<float4*>(dst + s * DH + 4 * (c ^ (s & (NCH - 1)))) = v;
  }
}

// The B operand of a 16-row tile of a row-major [rows][ld] matrix (rows at base + i * ld,
// channels h*DH ..): lane supplies row (l % 16) with channels 16 j + 4 g + e, i.e. one
// float4 per j.  Rows past n read as zero.
template <int DH>
__device__ __forceinline__ void ta_rows_operand(const float* __restrict__ base, size_t ld, int row0, int n,
                                                float4 (&v)[DH / 16]) {
  const int lane = threadIdx.x & 63, l16 = lane & 15, g = lane >> 4;
  const int row = row0 + l16;
#pragma unroll
  for (int j = 0; j < DH / 16; ++j)
    v[j] = row < n ? *reinterpret_cast<const float4*>(base + (size_t)row * ld + 16 * j + 4 * g)
                   : make_float4(0.f, 0.f, 0.f, 0.f);
}

// D = A B over a 64-wide (DH) channel contraction: A rows from an LDS tile (row a0 + l % 16),
// B from registers (the caller's float4 per j).  Result: D[4 g + r][l % 16].
template <int DH>
__device__ __forceinline__ f32x4_t ta_dot_tile(const float* At, int a0, const float4 (&b)[DH / 16]) {
  const int lane = threadIdx.x & 63, l16 = lane & 15, g = lane >> 4;
  float4 a[DH / 16];
#pragma unroll
  for (int j = 0; j < DH / 16; ++j) a[j] = ta_chunk<DH>(At, a0 + l16, 4 * j + g);
  f32x4_t acc = f32x4_t{0.f, 0.f, 0.f, 0.f};
  ta_fence_begin();
#pragma unroll
  for (int j = 0; j < DH / 16; ++j) {
    acc = mfma_f32_4(a[j].x, b[j].x, acc);
    acc = mfma_f32_4(a[j].y, b[j].y, acc);
    acc = mfma_f32_4(a[j].z, b[j].z, acc);
    acc = mfma_f32_4(a[j].w, b[j].w, acc);
  }
  ta_fence_end();
  return acc;
}

// acc[dt] += T^T X over the 16 rows x0 + 4 g + r of tile T (LDS, channels 16 dt + l % 16) with
// X[r] the caller's per-lane values for rows x0 + 4 g + r (k-step r): accumulates
// D[channel 16 dt + 4 g' + r'][l % 16].
template <int DH>
__device__ __forceinline__ void ta_accum_T(const float* Tt, int x0, const float (&x)[4], f32x4_t (&acc)[DH / 16]) {
  const int lane = threadIdx.x & 63, l16 = lane & 15, g = lane >> 4;
  float a[4][DH / 16];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int dt = 0; dt < DH / 16; ++dt) a[r][dt] = Tt[ta_off<DH>(x0 + 4 * g + r, 16 * dt + l16)];
  ta_fence_begin();
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int dt = 0; dt < DH / 16; ++dt) acc[dt] = mfma_f32_4(a[r][dt], x[r], acc[dt]);
  ta_fence_end();
}

// ------------------------------------------------------------------------------------------
// forward with (m, l)
// ------------------------------------------------------------------------------------------
template <int DH, int NT>
__global__ void __launch_bounds__(TA_THREADS) attn_train_fwd_kernel(int S, int C, int heads, const float* __restrict__ q,
                                                                    const float* __restrict__ kv,
                                                                    const int32_t* __restrict__ woff,
                                                                    float* __restrict__ o, float2* __restrict__ stats) {
  extern __shared__ __align__(16) float ta_lds[];
  float* Ks = ta_lds;
  float* Vs = ta_lds + 16 * NT * DH;
  const int w = blockIdx.x / heads, h = blockIdx.x - w * heads;
  const int q0 = woff[w], nq = woff[w + 1] - q0;
  if (nq == 0) return;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, l16 = lane & 15, g = lane >> 4;
  const float* kbase = kv + (size_t)w * S * 2 * C + h * DH;
  ta_stage<DH>(kbase, 2 * C, S, 16 * NT, Ks);
  ta_stage<DH>(kbase + C, 2 * C, S, 16 * NT, Vs);
  __syncthreads();
  const float scale = rsqrtf((float)DH);
  for (int qt = wv; qt * 16 < nq; qt += TA_THREADS / 64) {
    float4 qf[DH / 16];
    ta_rows_operand<DH>(q + (size_t)q0 * C + h * DH, C, qt * 16, nq, qf);
    float sc[NT][4];
    float mx = -INFINITY;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const f32x4_t a = ta_dot_tile<DH>(Ks, 16 * t, qf);  // key 16 t + 4 g + r, query l16
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const bool ok = 16 * t + 4 * g + r < S;
        sc[t][r] = ok ? a[r] * scale : -INFINITY;
        mx = fmaxf(mx, sc[t][r]);
      }
    }
    mx = fmaxf(mx, __shfl_xor(mx, 16, 64));
    mx = fmaxf(mx, __shfl_xor(mx, 32, 64));
    float sum = 0.f;
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float p = expf(sc[t][r] - mx);
        sc[t][r] = p;
        sum += p;
      }
    sum += __shfl_xor(sum, 16, 64);
    sum += __shfl_xor(sum, 32, 64);
    f32x4_t acc[DH / 16];
#pragma unroll
    for (int dt = 0; dt < DH / 16; ++dt) acc[dt] = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < NT; ++t) ta_accum_T<DH>(Vs, 16 * t, sc[t], acc);  // O^T[d][query]
    const int qi = qt * 16 + l16;
    if (qi < nq) {
      const float inv = 1.0f / sum;
      float* orow = o + (size_t)(q0 + qi) * C + h * DH;
#pragma unroll
      for (int dt = 0; dt < DH / 16; ++dt)
        *reinterpret_cast<float4*>(orow + 16 * dt + 4 * g) =
            make_float4(acc[dt][0] * inv, acc[dt][1] * inv, acc[dt][2] * inv, acc[dt][3] * inv);
      if (g == 0) stats[(size_t)(q0 + qi) * heads + h] = make_float2(mx, sum);
    }
  }
}

// ------------------------------------------------------------------------------------------
// reverse, query side: dQ and D = rowsum(P dP)
// ------------------------------------------------------------------------------------------
template <int DH, int NT>
__global__ void __launch_bounds__(TA_THREADS) attn_train_dq_kernel(int S, int C, int heads, const float* __restrict__ q,
                                                                   const float* __restrict__ kv,
                                                                   const float* __restrict__ dout,
                                                                   const float2* __restrict__ stats,
                                                                   const int32_t* __restrict__ woff,
                                                                   float* __restrict__ dq, float* __restrict__ dsum) {
  extern __shared__ __align__(16) float ta_lds[];
  float* Ks = ta_lds;
  float* Vs = ta_lds + 16 * NT * DH;
  const int w = blockIdx.x / heads, h = blockIdx.x - w * heads;
  const int q0 = woff[w], nq = woff[w + 1] - q0;
  if (nq == 0) return;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, l16 = lane & 15, g = lane >> 4;
  const float* kbase = kv + (size_t)w * S * 2 * C + h * DH;
  ta_stage<DH>(kbase, 2 * C, S, 16 * NT, Ks);
  ta_stage<DH>(kbase + C, 2 * C, S, 16 * NT, Vs);
  __syncthreads();
  const float scale = rsqrtf((float)DH);
  for (int qt = wv; qt * 16 < nq; qt += TA_THREADS / 64) {
    const int qi = qt * 16 + l16;
    float4 qf[DH / 16], gf[DH / 16];
    ta_rows_operand<DH>(q + (size_t)q0 * C + h * DH, C, qt * 16, nq, qf);
    ta_rows_operand<DH>(dout + (size_t)q0 * C + h * DH, C, qt * 16, nq, gf);
    const float2 st = qi < nq ? stats[(size_t)(q0 + qi) * heads + h] : make_float2(INFINITY, 1.f);
    const float inv_l = 1.0f / st.y;
    float p[NT][4], dp[NT][4];
    float D = 0.f;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const f32x4_t a = ta_dot_tile<DH>(Ks, 16 * t, qf);
      const f32x4_t b = ta_dot_tile<DH>(Vs, 16 * t, gf);  // dP^T[key][query]
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const bool ok = 16 * t + 4 * g + r < S;
        p[t][r] = ok ? expf(a[r] * scale - st.x) * inv_l : 0.f;
        dp[t][r] = b[r];
        D += p[t][r] * dp[t][r];
      }
    }
    D += __shfl_xor(D, 16, 64);
    D += __shfl_xor(D, 32, 64);
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) dp[t][r] = p[t][r] * (dp[t][r] - D);  // dS
    f32x4_t acc[DH / 16];
#pragma unroll
    for (int dt = 0; dt < DH / 16; ++dt) acc[dt] = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < NT; ++t) ta_accum_T<DH>(Ks, 16 * t, dp[t], acc);  // dQ^T[d][query]
    if (qi < nq) {
      float* row = dq + (size_t)(q0 + qi) * C + h * DH;
#pragma unroll
      for (int dt = 0; dt < DH / 16; ++dt)
        *reinterpret_cast<float4*>(row + 16 * dt + 4 * g) =
            make_float4(acc[dt][0] * scale, acc[dt][1] * scale, acc[dt][2] * scale, acc[dt][3] * scale);
      if (g == 0) dsum[(size_t)(q0 + qi) * heads + h] = D;
    }
  }
}

// ------------------------------------------------------------------------------------------
// reverse, key side: dK and dV of every key of the window (zero without queries)
// ------------------------------------------------------------------------------------------
template <int DH, int NT>
__global__ void __launch_bounds__(TA_THREADS) attn_train_dkv_kernel(int S, int C, int heads, const float* __restrict__ q,
                                                                    const float* __restrict__ kv,
                                                                    const float* __restrict__ dout,
                                                                    const float2* __restrict__ stats,
                                                                    const float* __restrict__ dsum,
                                                                    const int32_t* __restrict__ woff,
                                                                    float* __restrict__ dkv) {
  extern __shared__ __align__(16) float ta_lds[];
  constexpr int QP = 16 * NT;  // query rows the tiles hold (queries of a window <= its keys)
  float* Qs = ta_lds;
  float* Gs = ta_lds + QP * DH;
  float* Ms = Gs + QP * DH;
  float* Ls = Ms + QP;
  float* Ds = Ls + QP;
  const int w = blockIdx.x / heads, h = blockIdx.x - w * heads;
  const int q0 = woff[w], nq = woff[w + 1] - q0;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, l16 = lane & 15, g = lane >> 4;
  const int nqt = (nq + 15) / 16;
  ta_stage<DH>(q + (size_t)q0 * C + h * DH, C, nq, 16 * nqt, Qs);
  ta_stage<DH>(dout + (size_t)q0 * C + h * DH, C, nq, 16 * nqt, Gs);
  for (int i = threadIdx.x; i < 16 * nqt; i += TA_THREADS) {
    // padding queries: m = +inf makes their probabilities 0
    const float2 st = i < nq ? stats[(size_t)(q0 + i) * heads + h] : make_float2(INFINITY, 1.f);
    Ms[i] = st.x;
    Ls[i] = 1.0f / st.y;
    Ds[i] = i < nq ? dsum[(size_t)(q0 + i) * heads + h] : 0.f;
  }
  __syncthreads();
  const float scale = rsqrtf((float)DH);
  const float* kbase = kv + (size_t)w * S * 2 * C + h * DH;
  for (int kt = wv; kt < NT; kt += TA_THREADS / 64) {
    float4 kf[DH / 16], vf[DH / 16];
    ta_rows_operand<DH>(kbase, 2 * C, kt * 16, S, kf);
    ta_rows_operand<DH>(kbase + C, 2 * C, kt * 16, S, vf);
    f32x4_t dk[DH / 16], dvv[DH / 16];
#pragma unroll
    for (int dt = 0; dt < DH / 16; ++dt) dk[dt] = dvv[dt] = f32x4_t{0.f, 0.f, 0.f, 0.f};
    for (int qt = 0; qt < nqt; ++qt) {
      const f32x4_t a = ta_dot_tile<DH>(Qs, 16 * qt, kf);  // S[query 16 qt + 4 g + r][key l16]
      const f32x4_t b = ta_dot_tile<DH>(Gs, 16 * qt, vf);  // dP[query][key]
      float p[4], ds[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int qi = 16 * qt + 4 * g + r;
        p[r] = expf(a[r] * scale - Ms[qi]) * Ls[qi];
        ds[r] = p[r] * (b[r] - Ds[qi]);
      }
      ta_accum_T<DH>(Gs, 16 * qt, p, dvv);  // dV^T[d][key]
      ta_accum_T<DH>(Qs, 16 * qt, ds, dk);  // dK^T[d][key] (times the scale below)
    }
    const int s = kt * 16 + l16;
    if (s < S) {
      float* row = dkv + ((size_t)w * S + s) * 2 * C + h * DH;
#pragma unroll
      for (int dt = 0; dt < DH / 16; ++dt) {
        *reinterpret_cast<float4*>(row + 16 * dt + 4 * g) =
            make_float4(dk[dt][0] * scale, dk[dt][1] * scale, dk[dt][2] * scale, dk[dt][3] * scale);
        *reinterpret_cast<float4*>(row + C + 16 * dt + 4 * g) =
            make_float4(dvv[dt][0], dvv[dt][1], dvv[dt][2], dvv[dt][3]);
      }
    }
  }
}

// ------------------------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------------------------
template <class K>
static void ta_allow(K kernel, size_t bytes) {
  if (bytes > 65536)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)bytes);
}

bool attn_train_supported(int dh, int S) { return (dh == 32 || dh == 64) && S >= 1 && S <= TA_MAX_S; }

template <int DH, int NT>
static void ta_launch(int which, const Geo& g, int C, int heads, const float* q, const float* kv, const float* dout,
                      float* o, float2* stats, const float2* cstats, float* dq, float* dsum, const float* cdsum,
                      const int32_t* woff, float* dkv, hipStream_t s) {
  const size_t kvb = (size_t)2 * 16 * NT * DH * 4;
  const size_t dkvb = kvb + (size_t)3 * 16 * NT * 4;
  const dim3 grid(g.nwin * heads);
  if (which == 0) {
    static bool a = false;
    if (!a) { ta_allow(attn_train_fwd_kernel<DH, NT>, kvb); a = true; }
    attn_train_fwd_kernel<DH, NT><<<grid, TA_THREADS, kvb, s>>>(g.S, C, heads, q, kv, woff, o, stats);
  } else if (which == 1) {
    static bool a = false;
    if (!a) { ta_allow(attn_train_dq_kernel<DH, NT>, kvb); a = true; }
    attn_train_dq_kernel<DH, NT><<<grid, TA_THREADS, kvb, s>>>(g.S, C, heads, q, kv, dout, cstats, woff, dq, dsum);
  } else {
    static bool a = false;
    if (!a) { ta_allow(attn_train_dkv_kernel<DH, NT>, dkvb); a = true; }
    attn_train_dkv_kernel<DH, NT><<<grid, TA_THREADS, dkvb, s>>>(g.S, C, heads, q, kv, dout, cstats, cdsum, woff, dkv);
  }
}

// key tiles per window (16 NT >= S), instantiated for the configured windows: 64 keys
// (8 x 8 x 1), 225 (5 x 9 x 5) and 300 (6 x 10 x 5); other sizes up to TA_MAX_S use the
// next instantiated tile count
template <int DH>
static void ta_dispatch(int which, const Geo& g, int C, int heads, const float* q, const float* kv, const float* dout,
                        float* o, float2* stats, const float2* cstats, float* dq, float* dsum, const float* cdsum,
                        const int32_t* woff, float* dkv, hipStream_t s) {
  const int nt = (g.S + 15) / 16;
  if (nt <= 4)
    ta_launch<DH, 4>(which, g, C, heads, q, kv, dout, o, stats, cstats, dq, dsum, cdsum, woff, dkv, s);
  else if (nt <= 8)
    ta_launch<DH, 8>(which, g, C, heads, q, kv, dout, o, stats, cstats, dq, dsum, cdsum, woff, dkv, s);
  else if (nt <= 15)
    ta_launch<DH, 15>(which, g, C, heads, q, kv, dout, o, stats, cstats, dq, dsum, cdsum, woff, dkv, s);
  else
    ta_launch<DH, 19>(which, g, C, heads, q, kv, dout, o, stats, cstats, dq, dsum, cdsum, woff, dkv, s);
}

static void ta_run(int which, const Geo& g, int C, int heads, const float* q, const float* kv, const float* dout,
                   float* o, float2* stats, const float2* cstats, float* dq, float* dsum, const float* cdsum,
                   const int32_t* woff, float* dkv, hipStream_t s) {
  if (g.nwin <= 0) return;
  if (C / heads == 64)
    ta_dispatch<64>(which, g, C, heads, q, kv, dout, o, stats, cstats, dq, dsum, cdsum, woff, dkv, s);
  else
    ta_dispatch<32>(which, g, C, heads, q, kv, dout, o, stats, cstats, dq, dsum, cdsum, woff, dkv, s);
}

void launch_attn_train_fwd(const Geo& g, int C, int heads, const float* q, const float* kv, const int32_t* woff,
                           float* o, float2* stats, hipStream_t s) {
  ta_run(0, g, C, heads, q, kv, nullptr, o, stats, nullptr, nullptr, nullptr, nullptr, woff, nullptr, s);
}

void launch_attn_train_dq(const Geo& g, int C, int heads, const float* q, const float* kv, const float* dout,
                          const float2* stats, const int32_t* woff, float* dq, float* dsum, hipStream_t s) {
  ta_run(1, g, C, heads, q, kv, dout, nullptr, nullptr, stats, dq, dsum, nullptr, woff, nullptr, s);
}

void launch_attn_train_dkv(const Geo& g, int C, int heads, const float* q, const float* kv, const float* dout,
                           const float2* stats, const float* dsum, const int32_t* woff, float* dkv, hipStream_t s) {
  ta_run(2, g, C, heads, q, kv, dout, nullptr, nullptr, stats, nullptr, nullptr, dsum, woff, dkv, s);
}

}  // namespace dr
