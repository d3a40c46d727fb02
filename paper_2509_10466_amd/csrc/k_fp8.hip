// FP8 (OCP e4m3) path on gfx950: the Q/K/V, projection and MLP GEMMs take e4m3 operands with
// per-tensor scales and accumulate in FP32 on v_mfma_f32_16x16x128_f8f6f4; LayerNorm
// statistics, softmax and the residual stream stay FP32 (attention itself runs in BF16).
//
// Scaling: a tensor T is stored as e4m3(T / s) with s = amax(|T|) / 448 (s = 1 when amax is
// 0), round to nearest even; the GEMM epilogue multiplies by s_A * s_W.  Weight scales are
// fixed at load; activation scales come from the current call: the LayerNorm pass (or the
// epilogue of the producing kernel) max-reduces |T| into a per-block slot with an atomic max
// on the float bits (valid for non-negative floats), and the consumer reads the slot.
//
// Per transformer block: LayerNorm 1 (FP32 statistics, affine) of every token in a window
// with queries -> bf16 rows + amax; Q/K/V GEMM; attention (BF16, amax of O); projection +
// residual; LayerNorm 2 of the query rows -> bf16 rows + amax; first MLP linear + GELU (amax
// of h); second MLP linear + residual.  Every GEMM is the kernel below: bf16 rows quantised
// to e4m3 while they are staged, e4m3 weights, FP32 accumulation.
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
                                    float inv_scale, const float* __restrict__ scale) {
  if (scale) inv_scale = 1.0f / *scale;
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
  if (grid) quantize_fp8_kernel<<<(unsigned)grid, 256, 0, s>>>(in, out, n, inv_scale, nullptr);
}

void launch_quantize_fp8_dev(const float* in, uint8_t* out, size_t n, const float* scale, hipStream_t s) {
  size_t grid = (n / 2 + 256) / 256;
  if (grid > 8192) grid = 8192;
  if (grid) quantize_fp8_kernel<<<(unsigned)grid, 256, 0, s>>>(in, out, n, 1.f, scale);
}

__global__ void zero_f32_kernel(float* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.f;
}

void launch_zero_f32(float* p, int n, hipStream_t s) {
  if (n > 0) zero_f32_kernel<<<(n + 255) / 256, 256, 0, s>>>(p, n);
}

// ------------------------------------------------------------------------------------------
// LayerNorm rows: out[r] = LN(x[rows[r]]) (r < *nrows, compact output) or LN(x[r]) (r <
// nrows_max, only rows whose window has queries when wcount is given; output at row r), in
// bf16, and amax |out| of the call into *slot.  Sixteen lanes per row, four rows per
// wavefront; lane j of a row holds columns 4 (j + 16 e) .. +3 (16-byte loads).  FP32
// statistics (mean, then the centred sum of squares; biased variance, eps 1e-5).
// ------------------------------------------------------------------------------------------
constexpr int LNR_PER_MAX = 16;  // float4 groups per lane: C <= 1024

__device__ __forceinline__ float sum16(float v) {
  v += __shfl_xor(v, 1, 64);
  v += __shfl_xor(v, 2, 64);
  v += __shfl_xor(v, 4, 64);
  v += __shfl_xor(v, 8, 64);
  return v;
}

__global__ void __launch_bounds__(256) ln_rows_amax_kernel(const float* __restrict__ x, const int32_t* __restrict__ rows,
                                                           const int32_t* __restrict__ nrows_dev, int nrows_max,
                                                           const int32_t* __restrict__ wcount, int S, int C,
                                                           const float* __restrict__ g, const float* __restrict__ b,
                                                           bf16* __restrict__ out, float* slot) {
  const int lane = threadIdx.x & 63, j = lane & 15;
  const int nrows = nrows_dev ? nrows_dev[0] : nrows_max;
  const int per = C / 64;
  float mx = 0.f;
  // the loop bound is uniform per wavefront: 16-lane shuffles stay inside the wavefront
  for (int r0 = (blockIdx.x * 4 + (threadIdx.x >> 6)) * 4; r0 < nrows; r0 += gridDim.x * 16) {
    const int r = r0 + (lane >> 4);
    bool ok = r < nrows;
    if (ok && wcount) ok = wcount[r / S] > 0;
    const float* xr = x + (size_t)(ok ? (rows ? rows[r] : r) : 0) * C;
    float4 v[LNR_PER_MAX];
    float s = 0.f;
#pragma unroll
    for (int e = 0; e < LNR_PER_MAX; ++e)
      if (e < per) {
        v[e] = ok ? *reinterpret_cast<const float4*>(xr + 4 * (j + 16 * e)) : make_float4(0.f, 0.f, 0.f, 0.f);
        s += (v[e].x + v[e].y) + (v[e].z + v[e].w);
      }
    const float mean = sum16(s) / C;
    float q = 0.f;
#pragma unroll
    for (int e = 0; e < LNR_PER_MAX; ++e)
      if (e < per) {
        const float d0 = v[e].x - mean, d1 = v[e].y - mean, d2 = v[e].z - mean, d3 = v[e].w - mean;
        q += (d0 * d0 + d1 * d1) + (d2 * d2 + d3 * d3);
      }
    const float rstd = rsqrtf(sum16(q) / C + 1e-5f);
    if (ok) {
      bf16* orow = out + (size_t)r * C;
#pragma unroll
      for (int e = 0; e < LNR_PER_MAX; ++e)
        if (e < per) {
          const int c = 4 * (j + 16 * e);
          const float4 g4 = *reinterpret_cast<const float4*>(g + c), b4 = *reinterpret_cast<const float4*>(b + c);
          const float y0 = (v[e].x - mean) * rstd * g4.x + b4.x, y1 = (v[e].y - mean) * rstd * g4.y + b4.y;
          const float y2 = (v[e].z - mean) * rstd * g4.z + b4.z, y3 = (v[e].w - mean) * rstd * g4.w + b4.w;
          uint2 pk;
          pk.x = pack_bf2(y0, y1);
          pk.y = pack_bf2(y2, y3);
          *reinterpret_cast<uint2*>(orow + c) = pk;
          mx = fmaxf(mx, fmaxf(fmaxf(fabsf(y0), fabsf(y1)), fmaxf(fabsf(y2), fabsf(y3))));
        }
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

void launch_ln_rows_amax(const float* x, const int32_t* rows, const int32_t* nrows_dev, int nrows_max,
                         const int32_t* wcount, int S, int C, const float* g, const float* b, bf16* out, float* slot,
                         hipStream_t s) {
  if (nrows_max <= 0) return;
  int grid = (nrows_max + 15) / 16;
  if (grid > 4096) grid = 4096;
  ln_rows_amax_kernel<<<grid, 256, 0, s>>>(x, rows, nrows_dev, nrows_max, wcount, S, C, g, b, out, slot);
}

// ------------------------------------------------------------------------------------------
// FP8 GEMM over bf16 rows: Y[m, n] = s_a (e4m3(A/s_a) . e4m3(W)^T)[m, n], handed with s_a to
// an epilogue (which applies s_w, the bias and the destination).  256 threads = 2 x 2 waves,
// tile 64 x 128, 128-wide k stages, A converted bf16 -> e4m3 while it is staged into LDS.
// Rows: M = *m_dev when given, else m_host.  Without a tile list a tile runs only if
// epi.need(m, n0) holds for one of its rows; with one (Q/K/V), block x takes row tile
// tiles[list * mt + x] of list epi.list(n0) (lists built with the window order, ROW_TILE rows).
// ------------------------------------------------------------------------------------------
constexpr int F8_BK = 128;          // fp8 elements per stage = one MFMA k step
constexpr int F8_WST = F8_BK + 16;  // stage row stride in bytes
// Tile: BM x BN outputs, WM x WN wavefronts (each TM x TN), two LDS stages of 128-wide k.
template <int BM_, int BN_, int WM_, int WN_>
struct F8Tile {
  static constexpr int BM = BM_, BN = BN_, WM = WM_, WN = WN_;
  static constexpr int THREADS = 64 * WM * WN;
  static constexpr int TM = BM / WM, TN = BN / WN, FM = TM / 16, FN = TN / 16;
  static constexpr int LA = BM * 16 / THREADS;  // 16-byte bf16 chunks of A per thread per stage
  static constexpr int LW = BN * 8 / THREADS;   // 16-byte e4m3 chunks of W per thread per stage
  static constexpr size_t LDS_BYTES = (size_t)2 * (BM + BN) * F8_WST;
  static_assert(TM % 16 == 0 && TN % 16 == 0, "fragment multiples");
  static_assert(BM * 16 % THREADS == 0 && BN * 8 % THREADS == 0, "whole chunks per thread");
};
using F8Small = F8Tile<64, 128, 2, 2>;  // 4 wavefronts; the Q/K/V row-tile lists use its 64 rows
static_assert(F8Small::BM == ROW_TILE, "row tiles are listed in ROW_TILE units");

template <class TL, class Epi>
__global__ void __launch_bounds__(TL::THREADS) gemm_fp8_kernel(const bf16* __restrict__ A,
                                                               const int32_t* __restrict__ m_dev, int m_host, int K,
                                                               const uint8_t* __restrict__ W,
                                                               const float* __restrict__ amax_a,
                                                               const int32_t* __restrict__ tiles,
                                                               const int32_t* __restrict__ ntiles, Epi epi) {
  extern __shared__ __align__(16) uint8_t f8_lds[];
  uint8_t(*As)[TL::BM][F8_WST] = reinterpret_cast<uint8_t(*)[TL::BM][F8_WST]>(f8_lds);
  uint8_t(*Ws)[TL::BN][F8_WST] = reinterpret_cast<uint8_t(*)[TL::BN][F8_WST]>(f8_lds + 2 * TL::BM * F8_WST);
  const int M = m_dev ? m_dev[0] : m_host;
  const int n0 = blockIdx.y * TL::BN;
  int m0 = blockIdx.x * TL::BM;
  if (tiles) {  // (launched with F8Small only)
    const int l = epi.list(n0);
    if ((int)blockIdx.x >= ntiles[l]) return;
    m0 = tiles[l * ((m_host + TL::BM - 1) / TL::BM) + blockIdx.x] * TL::BM;
  } else {
    if (m0 >= M) return;
    int nd = 0;
    if ((int)threadIdx.x < TL::BM && m0 + (int)threadIdx.x < M) nd = epi.need(m0 + threadIdx.x, n0);
    if (!__syncthreads_or(nd)) return;
  }
  const float sa = scale_of(amax_a);
  const float inv_sa = 1.0f / sa;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int wm = wv / TL::WN, wn = wv % TL::WN;
  const int l16 = lane & 15, kg = lane >> 4;
  // A stage: BM rows x 128 k = 16 chunks of 8 bf16 per row; W stage: BN rows x 128 B = 8
  // chunks of 16 B per row
  u32x4_t ra[TL::LA], rw[TL::LW];
  auto load = [&](int k0) {
#pragma unroll
    for (int c = 0; c < TL::LA; ++c) {
      const int id = t + TL::THREADS * c;
      const int row = id >> 4, col = (id & 15) * 8;
      const int m = m0 + row;
      ra[c] = m < M ? *reinterpret_cast<const u32x4_t*>(A + (size_t)m * K + k0 + col) : u32x4_t{0u, 0u, 0u, 0u};
    }
#pragma unroll
    for (int c = 0; c < TL::LW; ++c) {
      const int id = t + TL::THREADS * c;
      const int wr = id >> 3, wc = (id & 7) * 16;
      rw[c] = *reinterpret_cast<const u32x4_t*>(W + (size_t)(n0 + wr) * K + k0 + wc);
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int c = 0; c < TL::LA; ++c) {
      const int id = t + TL::THREADS * c;
      const int row = id >> 4, col = (id & 15) * 8;
      const uint32_t w4[4] = {ra[c].x, ra[c].y, ra[c].z, ra[c].w};
      uint32_t lo = 0, hi = 0;
      lo = f32x2_to_fp8(bf2f(w4[0] & 0xffff) * inv_sa, bf2f(w4[0] >> 16) * inv_sa) |
           (f32x2_to_fp8(bf2f(w4[1] & 0xffff) * inv_sa, bf2f(w4[1] >> 16) * inv_sa) << 16);
      hi = f32x2_to_fp8(bf2f(w4[2] & 0xffff) * inv_sa, bf2f(w4[2] >> 16) * inv_sa) |
           (f32x2_to_fp8(bf2f(w4[3] & 0xffff) * inv_sa, bf2f(w4[3] >> 16) * inv_sa) << 16);
      *reinterpret_cast<uint2*>(&As[buf][row][col]) = make_uint2(lo, hi);
    }
#pragma unroll
    for (int c = 0; c < TL::LW; ++c) {
      const int id = t + TL::THREADS * c;
      const int wr = id >> 3, wc = (id & 7) * 16;
      *reinterpret_cast<u32x4_t*>(&Ws[buf][wr][wc]) = rw[c];
    }
  };
  f32x4_t acc[TL::FM][TL::FN];
#pragma unroll
  for (int i = 0; i < TL::FM; ++i)
#pragma unroll
    for (int j = 0; j < TL::FN; ++j) acc[i][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};
  // what the epilogue reads from memory (the residual rows), requested before the product so
  // that its latency hides behind it
  typename Epi::Pre pre[TL::FM][TL::FN];
#pragma unroll
  for (int i = 0; i < TL::FM; ++i) {
    const int m = m0 + wm * TL::TM + i * 16 + l16;
#pragma unroll
    for (int j = 0; j < TL::FN; ++j) pre[i][j] = epi.pre(min(m, M - 1), n0 + wn * TL::TN + j * 16 + kg * 4);
  }
  load(0);
  stash(0);
  __syncthreads();
  const int nk = K / F8_BK;
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) load((kt + 1) * F8_BK);
    i32x8_t af[TL::FM], wf[TL::FN];
#pragma unroll
    for (int i = 0; i < TL::FM; ++i) {
      const uint8_t* p = &As[buf][wm * TL::TM + i * 16 + l16][kg * 32];
      const uint4 lo = *reinterpret_cast<const uint4*>(p), hi = *reinterpret_cast<const uint4*>(p + 16);
      af[i] = i32x8_t{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
    }
#pragma unroll
    for (int j = 0; j < TL::FN; ++j) {
      const uint8_t* p = &Ws[buf][wn * TL::TN + j * 16 + l16][kg * 32];
      const uint4 lo = *reinterpret_cast<const uint4*>(p), hi = *reinterpret_cast<const uint4*>(p + 16);
      wf[j] = i32x8_t{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
    }
    fp8_group_begin();
#pragma unroll
    for (int i = 0; i < TL::FM; ++i)
#pragma unroll
      for (int j = 0; j < TL::FN; ++j) acc[i][j] = mfma_fp8(wf[j], af[i], acc[i][j]);
    fp8_group_end();
    if (kt + 1 < nk) {
      stash(buf ^ 1);
      __syncthreads();
    }
  }
#pragma unroll
  for (int i = 0; i < TL::FM; ++i) {
    const int m = m0 + wm * TL::TM + i * 16 + l16;
    if (m >= M) continue;
#pragma unroll
    for (int j = 0; j < TL::FN; ++j) epi(m, n0 + wn * TL::TN + j * 16 + kg * 4, acc[i][j], sa, pre[i][j]);
  }
  epi.finish();
}

template <class TL, class Epi>
static void gemm_fp8_launch(const bf16* A, const int32_t* m_dev, int m_max, int K, int Nout, const uint8_t* W,
                            const float* amax_a, const Epi& epi, hipStream_t s, const int32_t* tiles = nullptr,
                            const int32_t* ntiles = nullptr) {
  if (m_max <= 0) return;
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(gemm_fp8_kernel<TL, Epi>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)TL::LDS_BYTES);
    attr = true;
  }
  dim3 grid((m_max + TL::BM - 1) / TL::BM, Nout / TL::BN);
  gemm_fp8_kernel<TL, Epi><<<grid, TL::THREADS, TL::LDS_BYTES, s>>>(A, m_dev, m_max, K, W, amax_a, tiles, ntiles, epi);
}

// Row count from which the first MLP linear uses the 8-wavefront FP8 tile (as for BF16).
constexpr int F8_BIG_M = 32768;

// x[res_rows[m], n] += s_a s_w Y + bias[n]
struct F8ResidEpi {
  const float* bias;
  const float* s_w;  // device: the weight's scale
  float* x;
  const int32_t* res_rows;
  int Nout;
  __device__ __forceinline__ int need(int, int) const { return 1; }
  __device__ __forceinline__ int list(int) const { return 0; }
  using Pre = float4;  // x[res_rows[m], n .. n + 3]
  __device__ __forceinline__ Pre pre(int m, int n) const {
    return *reinterpret_cast<const float4*>(x + (size_t)res_rows[m] * Nout + n);
  }
  __device__ __forceinline__ void operator()(int m, int n, const f32x4_t& a, float sa, const Pre& xin) const {
    const float sc = sa * *s_w;
    const float4 b4 = *reinterpret_cast<const float4*>(bias + n);
    float4* p = reinterpret_cast<float4*>(x + (size_t)res_rows[m] * Nout + n);
    float4 xv = xin;
    xv.x += a[0] * sc + b4.x;
    xv.y += a[1] * sc + b4.y;
    xv.z += a[2] * sc + b4.z;
    xv.w += a[3] * sc + b4.w;
    *p = xv;
  }
  __device__ __forceinline__ void finish() const {}
};

void launch_gemm_fp8_resid(const bf16* A, const int32_t* m_dev, int m_max, int K, const uint8_t* W, const float* s_w,
                           const float* amax_a, const float* bias, int Nout, float* x, const int32_t* res_rows,
                           hipStream_t s) {
  // (a 128 x 128 tile on 8 wavefronts measured slower here at 720p)
  gemm_fp8_launch<F8Small>(A, m_dev, m_max, K, Nout, W, amax_a, F8ResidEpi{bias, s_w, x, res_rows, Nout}, s);
}

// Q rows [N][C] multiplied by qscale (log2(e)/sqrt(dh): the attention kernel takes Q scaled
// for base-2 exponentials), K [win][head][Spad][dh], V transposed [win][head][dh][spv] -- the
// layouts of the BF16 path, so both precisions share one attention kernel.  Q tiles run over
// the listed row tiles with a query, K/V tiles over those touching a window with queries.
struct F8QkvEpi {
  const float* bias;
  const float* wscale;  // [0] s_q, [1] s_k, [2] s_v
  float qscale;
  bf16 *q, *k, *vt;
  int C, dh, heads, Spad, S, spv;
  __device__ __forceinline__ int need(int, int) const { return 1; }
  __device__ __forceinline__ int list(int n0) const { return n0 < C ? 0 : 1; }
  struct Pre {  // the bias of the fragment's channels and the token's window and slot
    float4 b4;
    int w, s;
  };
  __device__ __forceinline__ Pre pre(int m, int n) const {
    const int w = m / S;
    return {*reinterpret_cast<const float4*>(bias + n), w, m - w * S};
  }
  __device__ __forceinline__ void operator()(int m, int n, const f32x4_t& a, float sa, const Pre& pr) const {
    const int part = n < C ? 0 : (n < 2 * C ? 1 : 2);
    const float sc = sa * wscale[part];
    const float4 b4 = pr.b4;
    const float y0 = a[0] * sc + b4.x, y1 = a[1] * sc + b4.y, y2 = a[2] * sc + b4.z, y3 = a[3] * sc + b4.w;
    if (part == 0) {
      uint2 pk;
      pk.x = pack_bf2(y0 * qscale, y1 * qscale);
      pk.y = pack_bf2(y2 * qscale, y3 * qscale);
      *reinterpret_cast<uint2*>(q + (size_t)m * C + n) = pk;
      return;
    }
    const int c = n - part * C, hh = c / dh, d = c - hh * dh;
    const int w = pr.w, s = pr.s;
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

void launch_qkv_fp8(const Geo& g, int C, int heads, int Spad, int spv, const bf16* u, const int32_t* tiles,
                    const int32_t* ntiles, const uint8_t* w, const float* wscale, const float* bias,
                    const float* amax_u, float qscale, bf16* q, bf16* k, bf16* vt, hipStream_t s) {
  const F8QkvEpi epi{bias, wscale, qscale, q, k, vt, C, C / heads, heads, Spad, g.S, spv};
  gemm_fp8_launch<F8Small>(u, nullptr, g.N, C, 3 * C, w, amax_u, epi, s, tiles, ntiles);
}

// h = GELU(s_a s_w Y + b1) in bf16, amax |h| of the call into *amax_h (one atomic per wave)
struct F8GeluEpi {
  const float* bias;
  const float* s_w;  // device: the weight's scale
  bf16* h;
  float* amax_h;
  int R;
  float mx;
  __device__ __forceinline__ int need(int, int) const { return 1; }
  __device__ __forceinline__ int list(int) const { return 0; }
  struct Pre {};
  __device__ __forceinline__ Pre pre(int, int) const { return {}; }
  __device__ __forceinline__ void operator()(int m, int n, const f32x4_t& a, float sa, const Pre&) {
    const float sc = sa * *s_w;
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

void launch_fc1_fp8(int m_max, const int32_t* m_dev, int C, int R, const bf16* u, const uint8_t* w, const float* s_w,
                    const float* bias, const float* amax_u, bf16* h, float* amax_h, hipStream_t s) {
  const F8GeluEpi epi{bias, s_w, h, amax_h, R, 0.f};
  if (m_max >= F8_BIG_M && R % 256 == 0)
    gemm_fp8_launch<F8Tile<128, 256, 2, 4>>(u, m_dev, m_max, C, R, w, amax_u, epi, s);
  else
    gemm_fp8_launch<F8Small>(u, m_dev, m_max, C, R, w, amax_u, epi, s);
}

bool fp8_supported(int C, int R) { return C % 128 == 0 && R % 128 == 0 && C / 64 <= LNR_PER_MAX; }

}  // namespace dr
