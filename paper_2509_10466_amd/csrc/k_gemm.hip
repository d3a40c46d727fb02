// BF16 linears of the transformer blocks on the direct-to-LDS MFMA core (gemm_core.h).
//
// The LayerNorms are split in two.  Their normalisation (x - mean) * rstd is applied by the
// kernel that produces the row -- the embedding for every token, the output projection and
// the second MLP linear for the updated tokens -- which stores the normalised row x^ in bf16
// next to the FP32 residual.  Their affine part is folded into the linear that follows:
// LN(x) W^T + b = x^ (W diag(g))^T + (b + W beta), so Q/K/V, the first MLP linear and the
// decoder read x^ directly.  In exact arithmetic this is the same network (the folded weights
// are derived on the device at load, in double precision).  The first MLP linear's folded
// weight and bias and the second's weight each also carry a factor 1/sqrt 2, so that the
// GELU epilogue evaluates x (1 + erf x) on x = z / sqrt 2 (gelu_scaled) without the two
// constant multiplications of 0.5 z (1 + erf(z / sqrt 2)).
//
//   qkv:   [Q | K | V] = x^ Wqkv'^T + bqkv'      all tokens of windows holding a query (K, V);
//                                                row tiles holding a flagged token (Q)
//   fc1:   h = GELU(u2 W1'^T + b1')              u2 = x^ of the flagged tokens after the
//                                                projection (compact rows)
//   proj:  x[idx[r]] += o W_o^T + b_o;  u2[r] = normalise(x[idx[r]])
//   fc2:   x[idx[r]] += h W_2^T + b_2;  x^[idx[r]] = normalise(x[idx[r]])
#include "dr_internal.h"
#include "gemm_core.h"

namespace dr {

template <class K>
static void allow_lds(K kernel, size_t bytes) {
  if (bytes > 65536)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)bytes);
}

// Applies epi(m, n, acc[i][j]) to the fragments of rows m < M.
template <class TL, class Epi>
__device__ __forceinline__ void for_fragments(int M, int m0, int n0, f32x4_t (&acc)[TL::FM][TL::FN], const Epi& epi) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int wm = wv / TL::WN, wn = wv % TL::WN, l16 = lane & 15, kg = lane >> 4;
  static_for<TL::FM>([&](auto i) {
    const int m = m0 + wm * TL::TM + 16 * i + l16;
    if (m < M)
      static_for<TL::FN>([&](auto j) { epi(m, n0 + wn * TL::TN + 16 * j + 4 * kg, acc[i][j]); });
  });
}

// Row count from which the larger 8-wavefront tiles pay off (measured on the Q/K/V and first
// MLP linear shapes: from ~50k rows they run 13-17 % faster, at 16k rows 10 % slower).
constexpr int BIG_M = 32768;


// ------------------------------------------------------------------------------------------
// Q/K/V
// ------------------------------------------------------------------------------------------
// Columns [0, C) -> Q rows [N][C]; [C, 2C) -> K [win][head][Spad][dh]; [2C, 3C) -> V
// transposed, V^T [win][head][dh][spv] (keys contiguous, the layout the attention kernel
// stages as is).  A column tile lies inside one of the three parts (C % BN == 0); dh is a
// power of two (2^dsh).  Channel c of a part sits at head c >> dsh, lane c & (dh - 1), so K's
// offset is (c >> dsh) Spad dh + (c & (dh - 1)) and V^T's row is c itself.
struct QkvRow {
  bf16* base;  // token's Q row / K row of head 0 / V^T column of head 0, lane 0
  int part;    // 0 Q, 1 K, 2 V
};

__device__ __forceinline__ void qkv_store(const QkvRow& r, int c, int C, int dsh, int kstride, int vstride,
                                          const float4& b4, const f32x4_t& a) {
  const float y0 = a[0] + b4.x, y1 = a[1] + b4.y, y2 = a[2] + b4.z, y3 = a[3] + b4.w;
  if (r.part == 2) {
    bf16* dst = r.base + (size_t)c * vstride;
    dst[0] = f2bf(y0);
    dst[vstride] = f2bf(y1);
    dst[2 * vstride] = f2bf(y2);
    dst[3 * vstride] = f2bf(y3);
    return;
  }
  const int off = r.part == 0 ? c : (c >> dsh) * kstride + (c & ((1 << dsh) - 1));
  uint2 pk;
  pk.x = pack_bf2(y0, y1);
  pk.y = pack_bf2(y2, y3);
  *reinterpret_cast<uint2*>(r.base + off) = pk;
}

struct QkvOut {
  const float* bias;
  bf16 *q, *k, *vt;
  int C, dsh, heads, Spad, S, spv;
  __device__ __forceinline__ QkvRow row(int m, int n0) const {
    const int part = n0 >= 2 * C ? 2 : n0 >= C ? 1 : 0;
    if (part == 0) return {q + (size_t)m * C, 0};
    const int w = m / S, s = m - w * S;
    if (part == 1) return {k + (((size_t)w * heads * Spad + s) << dsh), 1};
    return {vt + (((size_t)w * heads) << dsh) * spv + s, 2};
  }
  // the bias of channels n .. n + 3, and the store of a fragment of row r with it
  __device__ __forceinline__ float4 bias4(int n) const { return *reinterpret_cast<const float4*>(bias + n); }
  __device__ __forceinline__ void store_b(const QkvRow& r, int n, const float4& b4, const f32x4_t& a) const {
    qkv_store(r, n - r.part * C, C, dsh, Spad << dsh, spv, b4, a);
  }
};

// Stream mode: Q rows into the batch buffer; K [win_f][head][S_f][dh] and V^T
// [win_f][head][dh][sfp] of every token into the current ring slot of its request's cache.
struct StreamQkvOut {
  const float* bias;
  bf16* q;
  StreamTable tab;
  int C, dsh, heads, Sf, nwin_f;
  __device__ __forceinline__ QkvRow row(int m, int n0) const {
    const int part = n0 >= 2 * C ? 2 : n0 >= C ? 1 : 0;
    if (part == 0) return {q + (size_t)m * C, 0};
    const int w = m / Sf, s = m - w * Sf;
    const int r = w / nwin_f, wl = w - r * nwin_f;
    const size_t slot = (size_t)pick(tab.head, r);
    if (part == 1) return {pick(tab.k, r) + slot * tab.slot_stride + (((size_t)wl * heads * Sf + s) << dsh), 1};
    return {pick(tab.v, r) + slot * tab.vslot_stride + (((size_t)wl * heads) << dsh) * tab.sfp + s, 2};
  }
  __device__ __forceinline__ float4 bias4(int n) const { return *reinterpret_cast<const float4*>(bias + n); }
  __device__ __forceinline__ void store_b(const QkvRow& r, int n, const float4& b4, const f32x4_t& a) const {
    qkv_store(r, n - r.part * C, C, dsh, Sf << dsh, tab.sfp, b4, a);
  }
};

// One Q/K/V tile (rows m0 .., columns n0 ..).  Row-then-column epilogue: out.row(m, n0)
// computes the destination of token m once (the column tile's part of the output is uniform
// over the tile) and out.store_b(row, n, b4, a) adds the fragment's channel offset, which
// keeps per-token address arithmetic (divisions, table selects) out of the per-fragment
// path.  The row destinations and this lane's bias values are fetched before the product, so
// that their latency hides behind it.
template <class TL, class Out, int KC = 0>
__device__ __forceinline__ void qkv_tile(int M, int m0, int n0, int C, const bf16* __restrict__ xh,
                                         const bf16* __restrict__ W, bf16* ring, const Out& out) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int wm = wv / TL::WN, wn = wv % TL::WN, l16 = lane & 15, kg = lane >> 4;
  QkvRow rr[TL::FM];
  static_for<TL::FM>([&](auto f) { rr[f] = out.row(min(m0 + wm * TL::TM + 16 * f + l16, M - 1), n0); });
  float4 b4[TL::FN];
  static_for<TL::FN>([&](auto j) { b4[j] = out.bias4(n0 + wn * TL::TN + 16 * j + 4 * kg); });
  f32x4_t acc[TL::FM][TL::FN];
  gemm_core<TL, KC>(xh, M, m0, W, n0, C, ring, acc);
  static_for<TL::FM>([&](auto f) {
    if (m0 + wm * TL::TM + 16 * f + l16 < M)
      static_for<TL::FN>([&](auto j) { out.store_b(rr[f], n0 + wn * TL::TN + 16 * j + 4 * kg, b4[j], acc[f][j]); });
  });
}

// Tile skipping: a Q column tile runs only for row tiles holding a flagged token; a K/V
// column tile only for row tiles touching a window with queries (clip mode) -- keys and
// values of a window without queries are never read.  Stream mode keeps K/V of every token
// (later frames may query any window): wcount == nullptr.
template <class TL, class Out>
__global__ void __launch_bounds__(TL::THREADS) qkv_kernel(int M, int C, int S, const bf16* __restrict__ xh,
                                                  const uint8_t* __restrict__ flag,
                                                  const int32_t* __restrict__ wcount,
                                                  const bf16* __restrict__ W, Out out) {
  extern __shared__ __align__(16) bf16 ring[];
  const int mt = (M + TL::BM - 1) / TL::BM, nt = 3 * C / TL::BN;
  int rt, ct;
  xcd_tile(blockIdx.x, nt, rt, ct);
  if (rt >= mt) return;
  const int m0 = rt * TL::BM, n0 = ct * TL::BN;
  const bool is_q = n0 < C;
  int need = 0;
  if (threadIdx.x < TL::BM && m0 + (int)threadIdx.x < M) {
    const int m = m0 + threadIdx.x;
    need = is_q ? flag[m] != 0 : (wcount ? wcount[m / S] > 0 : 1);
  }
  if (!__syncthreads_or(need)) return;
  qkv_tile<TL>(M, m0, n0, C, xh, W, ring, out);
}

// Clip mode: blocks run only the listed row tiles (computed with the window order).  Block b
// takes, in dispatch order, the Q column tiles of the tiles holding a flagged token, then the
// K/V column tiles of the tiles touching a window with queries (each part XCD-ordered as
// xcd_tile), and the slots past both lists exit, last.
template <class TL, class Out, int KC>
__global__ void __launch_bounds__(TL::THREADS) qkv_list_kernel(int M, int C_, const bf16* __restrict__ xh,
                                                       const int32_t* __restrict__ tiles,
                                                       const int32_t* __restrict__ ntiles, const bf16* __restrict__ W,
                                                       Out out) {
  static_assert(TL::BM == ROW_TILE, "row tiles are listed in ROW_TILE units");
  static_assert(KC % TL::BN == 0, "whole column tiles");
  const int C = KC ? KC : C_;
  extern __shared__ __align__(16) bf16 ring[];
  const int mt = (M + TL::BM - 1) / TL::BM;
  const int ntq = C / TL::BN, gq = xcd_grid(ntiles[0], ntq);
  const bool is_q = (int)blockIdx.x < gq;
  const int b = is_q ? blockIdx.x : blockIdx.x - gq;
  int i, ct;
  xcd_tile(b, is_q ? ntq : 2 * ntq, i, ct);
  if (i >= ntiles[is_q ? 0 : 1]) return;
  const int m0 = tiles[(is_q ? 0 : mt) + i] * TL::BM, n0 = (is_q ? 0 : C) + ct * TL::BN;
  qkv_tile<TL, Out, KC>(M, m0, n0, C, xh, W, ring, out);
}

template <class TL, int KC, class Out>
static void qkv_list_launch(int M, int C, const bf16* xh, const int32_t* tiles, const int32_t* ntiles, const bf16* w,
                            const Out& out, hipStream_t s) {
  static bool attr = false;
  if (!attr) {
    allow_lds(qkv_list_kernel<TL, Out, KC>, TL::LDS_BYTES);
    attr = true;
  }
  const int mt = (M + TL::BM - 1) / TL::BM;
  const int grid = xcd_grid(mt, C / TL::BN) + xcd_grid(mt, 2 * C / TL::BN);
  qkv_list_kernel<TL, Out, KC><<<grid, TL::THREADS, TL::LDS_BYTES, s>>>(M, C, xh, tiles, ntiles, w, out);
}

// The network widths get their own instantiation, with the k loop unrolled (0.8 % per clip at
// 5 x 240 x 432 and 5 x 720 x 1280, timed back to back on one GPU); other widths take K at
// run time.
template <class TL, class Out>
static void qkv_list_by_c(int M, int C, const bf16* xh, const int32_t* tiles, const int32_t* ntiles, const bf16* w,
                          const Out& out, hipStream_t s) {
  if constexpr (TL::BN == 128) {
    switch (C) {
      case 128: return qkv_list_launch<TL, 128>(M, C, xh, tiles, ntiles, w, out, s);
      case 256: return qkv_list_launch<TL, 256>(M, C, xh, tiles, ntiles, w, out, s);
      case 384: return qkv_list_launch<TL, 384>(M, C, xh, tiles, ntiles, w, out, s);
      default: break;
    }
  } else if (C == 64) {
    return qkv_list_launch<TL, 64>(M, C, xh, tiles, ntiles, w, out, s);
  }
  qkv_list_launch<TL, 0>(M, C, xh, tiles, ntiles, w, out, s);
}

template <class TL, class Out>
static void qkv_launch(int M, int C, int S, const bf16* xh, const uint8_t* flag, const int32_t* wcount,
                       const bf16* w, const Out& out, hipStream_t s) {
  static bool attr = false;
  if (!attr) {
    allow_lds(qkv_kernel<TL, Out>, TL::LDS_BYTES);
    attr = true;
  }
  const int grid = xcd_grid((M + TL::BM - 1) / TL::BM, 3 * C / TL::BN);
  qkv_kernel<TL, Out><<<grid, TL::THREADS, TL::LDS_BYTES, s>>>(M, C, S, xh, flag, wcount, w, out);
}

// log2 of a power of two (head widths 32 and 64 are the ones the attention kernels take)
static int log2_pow2(int v) {
  int k = 0;
  while ((1 << k) < v) ++k;
  return k;
}

void launch_qkv_bf16(const Geo& g, int C, int heads, int Spad, int spv, const bf16* xh, const int32_t* tiles,
                     const int32_t* ntiles, const bf16* w, const float* bias, bf16* q, bf16* k, bf16* vt,
                     hipStream_t s) {
  if (g.N <= 0) return;
  const QkvOut out{bias, q, k, vt, C, log2_pow2(C / heads), heads, Spad, g.S, spv};
  // 8 wavefronts per 64 x 128 tile below BIG_M tokens (0.6 % faster per clip at 5 x 240 x 432,
  // 1 % slower at 5 x 720 x 1280, timed back to back on one GPU)
  if (C % 128 == 0 && g.N < BIG_M)
    qkv_list_by_c<GemmTile<64, 128, 2, 4, 2>>(g.N, C, xh, tiles, ntiles, w, out, s);
  else if (C % 128 == 0)
    qkv_list_by_c<GemmTile<64, 128, 2, 2, 2>>(g.N, C, xh, tiles, ntiles, w, out, s);
  else
    qkv_list_by_c<GemmTile<64, 64, 2, 2, 3>>(g.N, C, xh, tiles, ntiles, w, out, s);
}

void launch_qkv_stream(const Geo& g, int C, int heads, const bf16* xh, const uint8_t* flag, const bf16* w,
                       const float* bias, bf16* q, const StreamTable& tab, hipStream_t s) {
  if (g.N <= 0) return;
  const StreamQkvOut out{bias, q, tab, C, log2_pow2(C / heads), heads, g.S, g.nwh * g.nww};
  if (C % 128 == 0 && g.N >= BIG_M)
    qkv_launch<GemmTile<256, 128, 4, 2, 2>>(g.N, C, g.S, xh, flag, nullptr, w, out, s);
  else if (C % 128 == 0)
    qkv_launch<GemmTile<64, 128, 2, 2, 2>>(g.N, C, g.S, xh, flag, nullptr, w, out, s);
  else
    qkv_launch<GemmTile<64, 64, 2, 2, 3>>(g.N, C, g.S, xh, flag, nullptr, w, out, s);
}

// ------------------------------------------------------------------------------------------
// First MLP linear + GELU over the compact query rows (the first *m_dev rows)
// ------------------------------------------------------------------------------------------
struct GeluOut {
  const float* bias;
  bf16* h;
  int R;
  __device__ __forceinline__ void operator()(int m, int n, const f32x4_t& a) const {
    const float4 b4 = *reinterpret_cast<const float4*>(bias + n);
    uint2 pk;
    // the first and second linears' weights carry GELU's constant factors (gelu_scaled)
    pk.x = pack_bf2(gelu_scaled(a[0] + b4.x), gelu_scaled(a[1] + b4.y));
    pk.y = pack_bf2(gelu_scaled(a[2] + b4.z), gelu_scaled(a[3] + b4.w));
    *reinterpret_cast<uint2*>(h + (size_t)m * R + n) = pk;
  }
};

template <class TL>
__global__ void __launch_bounds__(TL::THREADS) fc1_kernel(const int32_t* __restrict__ m_dev, int C, int R,
                                                  const bf16* __restrict__ u2, const bf16* __restrict__ W,
                                                  GeluOut out) {
  extern __shared__ __align__(16) bf16 ring[];
  const int M = m_dev[0];
  const int nt = R / TL::BN;
  const int mt = (M + TL::BM - 1) / TL::BM;
  // the grid covers the largest possible M (fixed for graph capture); surplus tiles exit
  int rt, ct;
  xcd_tile(blockIdx.x, nt, rt, ct);
  if (rt >= mt) return;
  const int m0 = rt * TL::BM, n0 = ct * TL::BN;
  f32x4_t acc[TL::FM][TL::FN];
  gemm_core<TL>(u2, M, m0, W, n0, C, ring, acc);
  for_fragments<TL>(M, m0, n0, acc, out);
}

template <class TL>
static void fc1_launch(int m_max, const int32_t* m_dev, int C, int R, const bf16* u2, const bf16* w,
                       const float* bias, bf16* h, hipStream_t s) {
  static bool attr = false;
  if (!attr) {
    allow_lds(fc1_kernel<TL>, TL::LDS_BYTES);
    attr = true;
  }
  const int grid = xcd_grid((m_max + TL::BM - 1) / TL::BM, R / TL::BN);
  fc1_kernel<TL><<<grid, TL::THREADS, TL::LDS_BYTES, s>>>(m_dev, C, R, u2, w, GeluOut{bias, h, R});
}

void launch_fc1_bf16(int m_max, const int32_t* m_dev, int C, int R, const bf16* u2, const bf16* w,
                     const float* bias, bf16* h, hipStream_t s) {
  if (m_max <= 0) return;
  if (m_max >= BIG_M && R % 256 == 0)
    fc1_launch<GemmTile<128, 256, 2, 4, 2>>(m_max, m_dev, C, R, u2, w, bias, h, s);
  else
    fc1_launch<GemmTile<64, 128, 2, 2, 2>>(m_max, m_dev, C, R, u2, w, bias, h, s);
}

// ------------------------------------------------------------------------------------------
// Residual linears with the row normalisation in the epilogue.  Block tile 64 rows x the full
// width C (4 wavefronts side by side, each C/4 channels), so each row's statistics are
// complete inside the block: the wavefront sums go through LDS.  Two passes (mean, then the
// centred sum of squares), FP32, biased variance, eps 1e-5.
// ------------------------------------------------------------------------------------------
template <class TL>
__global__ void __launch_bounds__(TL::THREADS) resid_ln_kernel(const int32_t* __restrict__ m_dev, int K,
                                                       const bf16* __restrict__ A, const bf16* __restrict__ W,
                                                       const float* __restrict__ bias, float* __restrict__ x,
                                                       const int32_t* __restrict__ rows, bf16* __restrict__ xh,
                                                       const int32_t* __restrict__ hrows) {
  constexpr int C = TL::BN;
  extern __shared__ __align__(16) bf16 ring[];
  __shared__ float red[2][TL::WN][TL::BM];
  static_assert(TL::WN == 4, "row sums over four column wavefronts");
  const int M = m_dev[0];
  // row tile b: consecutive row tiles run on different XCDs
  const int m0 = blockIdx.x * TL::BM;
  if (m0 >= M) return;
  f32x4_t acc[TL::FM][TL::FN];
  gemm_core<TL>(A, M, m0, W, 0, K, ring, acc);

  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int wm = wv / TL::WN, wn = wv % TL::WN;
  const int l16 = lane & 15, kg = lane >> 4;
  int dst[TL::FM];
  float part[TL::FM];
  static_for<TL::FM>([&](auto i) {
    const int m = m0 + wm * TL::TM + 16 * i + l16;
    const bool ok = m < M;
    dst[i] = ok ? rows[m] : -1;
    float sum = 0.f;
    static_for<TL::FN>([&](auto j) {
      const int n = wn * TL::TN + 16 * j + 4 * kg;
      const float4 b4 = *reinterpret_cast<const float4*>(bias + n);
      float4 xo = make_float4(0.f, 0.f, 0.f, 0.f);
      if (ok) xo = *reinterpret_cast<const float4*>(x + (size_t)dst[i] * C + n);
      f32x4_t& a = acc[i][j];
      a[0] += b4.x + xo.x;
      a[1] += b4.y + xo.y;
      a[2] += b4.z + xo.z;
      a[3] += b4.w + xo.w;
      if (ok) *reinterpret_cast<float4*>(x + (size_t)dst[i] * C + n) = make_float4(a[0], a[1], a[2], a[3]);
      sum += (a[0] + a[1]) + (a[2] + a[3]);
    });
    sum += __shfl_xor(sum, 16, 64);
    sum += __shfl_xor(sum, 32, 64);
    part[i] = sum;
  });
  if (kg == 0) static_for<TL::FM>([&](auto i) { red[0][wn][wm * TL::TM + 16 * i + l16] = part[i]; });
  __syncthreads();
  float mean[TL::FM];
  static_for<TL::FM>([&](auto i) {
    const int r = wm * TL::TM + 16 * i + l16;
    mean[i] = ((red[0][0][r] + red[0][1][r]) + (red[0][2][r] + red[0][3][r])) * (1.0f / C);
    float sq = 0.f;
    static_for<TL::FN>([&](auto j) {
      static_for<4>([&](auto e) {
        const float d = acc[i][j][int(e)] - mean[i];
        sq += d * d;
      });
    });
    sq += __shfl_xor(sq, 16, 64);
    sq += __shfl_xor(sq, 32, 64);
    part[i] = sq;
  });
  if (kg == 0) static_for<TL::FM>([&](auto i) { red[1][wn][wm * TL::TM + 16 * i + l16] = part[i]; });
  __syncthreads();
  static_for<TL::FM>([&](auto i) {
    const int r = wm * TL::TM + 16 * i + l16;
    const float var = ((red[1][0][r] + red[1][1][r]) + (red[1][2][r] + red[1][3][r])) * (1.0f / C);
    const float rstd = rsqrtf(var + 1e-5f);
    if (dst[i] >= 0) {
      const int hr = hrows ? hrows[m0 + r] : m0 + r;
      static_for<TL::FN>([&](auto j) {
        const int n = wn * TL::TN + 16 * j + 4 * kg;
        const f32x4_t& a = acc[i][j];
        uint2 pk;
        pk.x = pack_bf2((a[0] - mean[i]) * rstd, (a[1] - mean[i]) * rstd);
        pk.y = pack_bf2((a[2] - mean[i]) * rstd, (a[3] - mean[i]) * rstd);
        *reinterpret_cast<uint2*>(xh + (size_t)hr * C + n) = pk;
      });
    }
  });
}

template <class TL>
static void resid_ln_launch(int m_max, const int32_t* m_dev, int K, const bf16* A, const bf16* w, const float* bias,
                            float* x, const int32_t* rows, bf16* xh, const int32_t* hrows, hipStream_t s) {
  static bool attr = false;
  if (!attr) {
    allow_lds(resid_ln_kernel<TL>, TL::LDS_BYTES);
    attr = true;
  }
  resid_ln_kernel<TL><<<(m_max + TL::BM - 1) / TL::BM, TL::THREADS, TL::LDS_BYTES, s>>>(m_dev, K, A, w, bias, x, rows, xh, hrows);
}

bool resid_ln_supported(int C) { return C == 64 || C == 128 || C == 256 || C == 384; }

void launch_resid_ln_bf16(int m_max, const int32_t* m_dev, int C, int K, const bf16* A, const bf16* w,
                          const float* bias, float* x, const int32_t* rows, bf16* xh, const int32_t* hrows,
                          hipStream_t s) {
  if (m_max <= 0) return;
  switch (C) {
    case 64: resid_ln_launch<GemmTile<64, 64, 1, 4, 3>>(m_max, m_dev, K, A, w, bias, x, rows, xh, hrows, s); break;
    case 128: resid_ln_launch<GemmTile<64, 128, 1, 4, 3>>(m_max, m_dev, K, A, w, bias, x, rows, xh, hrows, s); break;
    case 256: resid_ln_launch<GemmTile<64, 256, 1, 4, 3>>(m_max, m_dev, K, A, w, bias, x, rows, xh, hrows, s); break;
    case 384: resid_ln_launch<GemmTile<64, 384, 2, 4, 2>>(m_max, m_dev, K, A, w, bias, x, rows, xh, hrows, s); break;
    default: break;  // rejected by the caller (resid_ln_supported)
  }
}

// ------------------------------------------------------------------------------------------
// Fused post-attention block over 64 query rows (compact rows r, token idx[r]):
//   x1 = x + o W_o^T + b_o        u2 = normalise(x1)
//   h  = GELU(u2 W1'^T + b1')     (hidden chunks of HC columns)
//   x2 = x1 + h W_2^T + b_2       x^ = normalise(x2)
// u2 and h never leave LDS: the o rows are loaded once into a resident A tile that u2 then
// overwrites, each hidden chunk is written to LDS by the GELU epilogue and immediately
// consumed by the second linear.  Only the weights stream, through a 3-stage ring whose
// stages are, in order: the C/64 k-blocks of W_o; then per hidden chunk j the C/64 k-blocks
// of W1' rows [j*HC, (j+1)*HC) followed by the HC/64 k-blocks of W_2 columns of chunk j.
// Block = 512 threads = 8 wavefronts in 2 (rows) x 4 (columns): the block needs most of the
// LDS, so it runs alone on its CU, and two wavefronts per SIMD keep the matrix pipe fed
// while the other waits on LDS or the barrier.
// ------------------------------------------------------------------------------------------
constexpr int MLP_THREADS = 512;

template <int C_, int HC_, int BM_ = 64, int ST_ = 3, int SR_ = 0>
struct MlpCfg {
  static constexpr int C = C_, HC = HC_, BM = BM_, R = 4 * C, ST = ST_;
  static constexpr int WM = 2, WN = 4, TM = BM / WM;   // wavefront grid; rows per wavefront
  static constexpr int FM = TM / 16;
  static constexpr int SLOT_ROWS = SR_ ? SR_ : (C > HC ? C : HC);
  static constexpr int SLOT = SLOT_ROWS * 64;          // bf16 elements per ring slot
  static constexpr int NKC = C / 64, NKH = HC / 64;    // k blocks of C- and HC-wide operands
  static constexpr int NCH = R / HC;                   // hidden chunks
  // a k block of a C-row weight (W_o, W_2) moves in NHALF stages of CS rows when a slot
  // holds fewer than C rows
  static constexpr int CS = C < SLOT_ROWS ? C : SLOT_ROWS, NHALF = C / CS;
  // k blocks of W1' per stage: as many HC-row blocks as a ring slot holds, so that every
  // stage moves a full slot (fewer stages, each with the same fixed wait + barrier cost)
  static constexpr int KB1 = (SLOT_ROWS / HC < NKC) ? SLOT_ROWS / HC : NKC;
  static constexpr int NW1 = NKC / KB1;                // W1' stages per hidden chunk
  static constexpr int PER_CHUNK = NW1 + NKH * NHALF;
  static constexpr int NSTAGE = NKC * NHALF + NCH * PER_CHUNK;
  static constexpr int FN_C = C / 64, FN_H = HC / 64;  // 16-wide fragments per wavefront
  static constexpr int FPH = FN_C / NHALF;             // of them per C-row stage
  // output column of wavefront wn's fragment j (lane group kg adds 4 kg): the wavefront's
  // columns are spread over the NHALF row ranges of a C-row stage, FPH fragments in each
  __device__ static constexpr int col(int wn, int j) { return (j / FPH) * CS + wn * 16 * FPH + 16 * (j % FPH); }
  static constexpr size_t RING = (size_t)ST * SLOT, ARES = (size_t)NKC * BM * 64, HRES = (size_t)NKH * BM * 64;
  static constexpr size_t FLOATS = 2 * (size_t)C + R + 2 * WN * BM;  // b_o, b1', b_2, row sums
  static constexpr size_t LDS_BYTES = (RING + ARES + HRES) * 2 + FLOATS * 4;
  static_assert(C % 64 == 0 && HC % 64 == 0 && R % HC == 0 && NKC % KB1 == 0, "shapes");
  static_assert(C % CS == 0 && FN_C % NHALF == 0 && CS % (16 * WN) == 0 && SLOT_ROWS >= HC, "C-row stages");
  static_assert((BM == 32 || BM == 64) && (ST == 2 || ST == 3), "row tile and ring depth");
  // x1 (the residual after the projection) kept in registers for the second residual, rather
  // than stored to x and read back, where the registers allow it
  static constexpr bool X1_REGS = C <= 256;
  static_assert(LDS_BYTES <= 160 * 1024, "LDS");
};

// One 64-wide k block: acc[i][j] += A[wm*TM + 16i + l16][k] W[wn*16*FN + 16j + l16][k], A and
// W in the swizzled 64-column LDS layout.
template <class MC, int FN, int J0 = 0, int NA = FN>
__device__ __forceinline__ void mfma_block(const bf16* As, const bf16* Ws, f32x4_t (&acc)[MC::FM][NA]) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int wm = wv / MC::WN, wn = wv % MC::WN;
  const int l16 = lane & 15, kg = lane >> 4;
  bf16x8_t af[2][MC::FM], wf[2][FN];
  static_for<2>([&](auto kk) {
    static_for<MC::FM>([&](auto i) {
      const int row = wm * MC::TM + 16 * i + l16;
      af[kk][i] = *reinterpret_cast<const bf16x8_t*>(As + row * 64 + (((4 * kk + kg) ^ lds_swz(row)) * 8));
    });
    static_for<FN>([&](auto j) {
      const int row = wn * 16 * FN + 16 * j + l16;
      wf[kk][j] = *reinterpret_cast<const bf16x8_t*>(Ws + row * 64 + (((4 * kk + kg) ^ lds_swz(row)) * 8));
    });
  });
  static_for<2>([&](auto kk) {
    mfma_fence_begin();
    static_for<MC::FM>([&](auto i) {
      static_for<FN>([&](auto j) { acc[i][J0 + j] = mfma_bf16_16x16x32(wf[kk][j], af[kk][i], acc[i][J0 + j]); });
    });
    mfma_fence_end();
  });
}

// As mfma_block with the A fragments already in registers (af[kk][i]: rows wm*TM + 16 i + l16,
// k values 32 kk + 8 kg .. +7 of the 64-wide k block).
template <class MC, int FN>
__device__ __forceinline__ void mfma_block_ra(const bf16x8_t (&af)[2][MC::FM], const bf16* Ws,
                                              f32x4_t (&acc)[MC::FM][FN]) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int wn = wv % MC::WN;
  const int l16 = lane & 15, kg = lane >> 4;
  bf16x8_t wf[2][FN];
  static_for<2>([&](auto kk) {
    static_for<FN>([&](auto j) {
      const int row = wn * 16 * FN + 16 * j + l16;
      wf[kk][j] = *reinterpret_cast<const bf16x8_t*>(Ws + row * 64 + (((4 * kk + kg) ^ lds_swz(row)) * 8));
    });
  });
  static_for<2>([&](auto kk) {
    mfma_fence_begin();
    static_for<MC::FM>([&](auto i) {
      static_for<FN>([&](auto j) { acc[i][j] = mfma_bf16_16x16x32(wf[kk][j], af[kk][i], acc[i][j]); });
    });
    mfma_fence_end();
  });
}

// Element offset of (row r, column c) in a resident [k block][BM rows][64] swizzled tile.
template <int BM = 64>
__device__ __forceinline__ int res_off(int r, int c) {
  return (c >> 6) * (BM * 64) + r * 64 + ((((c & 63) >> 3) ^ lds_swz(r)) << 3) + (c & 7);
}

// This thread's residual values x[dst] for the [64][C] accumulators (zero for rows past M),
// loaded ahead of the epilogue so that their latency overlaps the last k stage.
template <class MC>
__device__ __forceinline__ void load_resid(const float* __restrict__ x, const int (&dst)[MC::FM],
                                           float4 (&xo)[MC::FM][MC::FN_C]) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int wn = wv % MC::WN, kg = lane >> 4;
  static_for<MC::FM>([&](auto i) {
    static_for<MC::FN_C>([&](auto j) {
      const int n = MC::col(wn, j) + 4 * kg;
      xo[i][j] = dst[i] >= 0 ? *reinterpret_cast<const float4*>(x + (size_t)dst[i] * MC::C + n)
                             : make_float4(0.f, 0.f, 0.f, 0.f);
    });
  });
}

// Residual + row normalisation for the [64][C] accumulators: acc += bias + xo (= x[dst]);
// x[dst] = acc; the row statistics come back through mean/rstd.  The four column
// wavefronts of a row group exchange partial sums through red[2][WN][BM].
template <class MC>
__device__ __forceinline__ void resid_rows(f32x4_t (&acc)[MC::FM][MC::FN_C], const float* sbias,
                                           float* __restrict__ x, const int (&dst)[MC::FM],
                                           const float4 (&xo_in)[MC::FM][MC::FN_C], float (*red)[MC::WN][MC::BM],
                                           float (&mean)[MC::FM], float (&rstd)[MC::FM], bool store = true) {
  constexpr int C = MC::C, FN = MC::FN_C;
  // the thread index passes through an empty asm so that the column addresses below are
  // recomputed per call rather than kept live (or spilled) from an earlier call
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));
  const int lane = tid & 63, wv = tid >> 6;
  const int wm = wv / MC::WN, wn = wv % MC::WN;
  const int l16 = lane & 15, kg = lane >> 4;
  float part[MC::FM];
  static_for<MC::FM>([&](auto i) {
    float sum = 0.f;
    static_for<FN>([&](auto j) {
      const int n = MC::col(wn, j) + 4 * kg;
      const float4 xo = xo_in[i][j];
      f32x4_t& a = acc[i][j];
      a[0] += sbias[n] + xo.x;
      a[1] += sbias[n + 1] + xo.y;
      a[2] += sbias[n + 2] + xo.z;
      a[3] += sbias[n + 3] + xo.w;
      if (store && dst[i] >= 0)
        *reinterpret_cast<float4*>(x + (size_t)dst[i] * C + n) = make_float4(a[0], a[1], a[2], a[3]);
      sum += (a[0] + a[1]) + (a[2] + a[3]);
    });
    sum += __shfl_xor(sum, 16, 64);
    sum += __shfl_xor(sum, 32, 64);
    part[i] = sum;
  });
  if (kg == 0) static_for<MC::FM>([&](auto i) { red[0][wn][wm * MC::TM + 16 * i + l16] = part[i]; });
  lds_barrier();
  static_for<MC::FM>([&](auto i) {
    const int r = wm * MC::TM + 16 * i + l16;
    mean[i] = ((red[0][0][r] + red[0][1][r]) + (red[0][2][r] + red[0][3][r])) * (1.0f / C);
    float sq = 0.f;
    static_for<FN>([&](auto j) {
      static_for<4>([&](auto e) {
        const float d = acc[i][j][int(e)] - mean[i];
        sq += d * d;
      });
    });
    sq += __shfl_xor(sq, 16, 64);
    sq += __shfl_xor(sq, 32, 64);
    part[i] = sq;
  });
  if (kg == 0) static_for<MC::FM>([&](auto i) { red[1][wn][wm * MC::TM + 16 * i + l16] = part[i]; });
  lds_barrier();
  static_for<MC::FM>([&](auto i) {
    const int r = wm * MC::TM + 16 * i + l16;
    const float var = ((red[1][0][r] + red[1][1][r]) + (red[1][2][r] + red[1][3][r])) * (1.0f / C);
    rstd[i] = rsqrtf(var + 1e-5f);
  });
}

template <class MC>
__global__ void __launch_bounds__(MLP_THREADS) mlp_block_kernel(const int32_t* __restrict__ m_dev,
                                                                const bf16* __restrict__ o,
                                                                const int32_t* __restrict__ rows,
                                                                const bf16* __restrict__ Wo, const float* __restrict__ bo,
                                                                const bf16* __restrict__ W1, const float* __restrict__ b1,
                                                                const bf16* __restrict__ W2, const float* __restrict__ b2,
                                                                float* __restrict__ x, bf16* __restrict__ xh) {
  constexpr int C = MC::C, HC = MC::HC, R = MC::R, BM = MC::BM, NW = MLP_THREADS / 64;
  extern __shared__ __align__(16) bf16 lds[];
  bf16* ring = lds;
  bf16* ares = lds + MC::RING;
  bf16* hres = ares + MC::ARES;
  float* sbo = reinterpret_cast<float*>(hres + MC::HRES);
  float* sb1 = sbo + C;
  float* sb2 = sb1 + R;
  float(*red)[MC::WN][MC::BM] = reinterpret_cast<float(*)[MC::WN][MC::BM]>(sb2 + C);

  const int M = m_dev[0];
  const int m0 = blockIdx.x * BM;
  if (m0 >= M) return;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int wm = wv / MC::WN, wn = wv % MC::WN;
  const int l16 = lane & 15, kg = lane >> 4;

  // the rows' token indices first: the residual loads below need them
  int dst[MC::FM];
  static_for<MC::FM>([&](auto i) {
    const int m = m0 + wm * MC::TM + 16 * i + l16;
    dst[i] = m < M ? rows[m] : -1;
  });
  // the biases into registers now, into LDS after the loads below are queued: one round trip
  // for all of them instead of one per loop iteration
  constexpr int NBC = (C + MLP_THREADS - 1) / MLP_THREADS, NBR = (R + MLP_THREADS - 1) / MLP_THREADS;
  float vbo[NBC], vb2[NBC], vb1[NBR];
  static_for<NBC>([&](auto k) {
    const int i = t + MLP_THREADS * k;
    vbo[k] = i < C ? bo[i] : 0.f;
    vb2[k] = i < C ? b2[i] : 0.f;
  });
  static_for<NBR>([&](auto k) {
    const int i = t + MLP_THREADS * k;
    vb1[k] = i < R ? b1[i] : 0.f;
  });
  // o rows -> resident A tile (rows >= M read row M-1; their results are never stored):
  // 8 rows per load, BM / 8 row groups per k block, one group per wavefront
  if (wv * 8 < BM)
    static_for<MC::NKC>([&](auto kb) {
      const int row = wv * 8 + (lane >> 3);
      const int m = min(m0 + row, M - 1);
      dma16(o + (size_t)m * C + 64 * kb + ((lane & 7) ^ lds_swz(row)) * 8, ares + kb * BM * 64 + wv * 512);
    });
  // weight stages: stage s holds rows [0, stage_rows(s)) of 64 k columns; a W1' stage holds
  // KB1 blocks of HC rows, k block b of the stage at rows [b HC, (b+1) HC)
  auto stage_rows = [](int s) {
    if (s < MC::NKC * MC::NHALF) return MC::CS;
    const int tt = (s - MC::NKC * MC::NHALF) % MC::PER_CHUNK;
    return tt < MC::NW1 ? HC * MC::KB1 : MC::CS;
  };
  auto issue = [&](int s) {
    const bf16* base;
    int rows_s, ld, blk_rows;  // slot rows; source row stride; rows per k block in the slot
    if (s < MC::NKC * MC::NHALF) {
      const int kb = s / MC::NHALF, h = s - kb * MC::NHALF;
      base = Wo + (size_t)h * MC::CS * C + 64 * kb;
      rows_s = MC::CS;
      ld = C;
      blk_rows = MC::CS;
    } else {
      const int q = s - MC::NKC * MC::NHALF, j = q / MC::PER_CHUNK, tt = q - j * MC::PER_CHUNK;
      if (tt < MC::NW1) {
        base = W1 + (size_t)j * HC * C + 64 * MC::KB1 * tt;
        rows_s = HC * MC::KB1;
        ld = C;
        blk_rows = HC;
      } else {
        const int u = tt - MC::NW1, kb = u / MC::NHALF, h = u - kb * MC::NHALF;
        base = W2 + (size_t)h * MC::CS * R + j * HC + 64 * kb;
        rows_s = MC::CS;
        ld = R;
        blk_rows = MC::CS;
      }
    }
    bf16* dst = ring + (s % MC::ST) * MC::SLOT;
    static_for<MC::SLOT_ROWS / (8 * NW)>([&](auto c) {
      const int g8 = wv + NW * c;
      if (g8 * 8 < rows_s) {  // uniform per wavefront
        const int row = g8 * 8 + (lane >> 3);
        const int b = row / blk_rows, rr = row - b * blk_rows;  // blk_rows is a multiple of 8
        dma16(base + (size_t)rr * ld + 64 * b + ((lane & 7) ^ lds_swz(row)) * 8, dst + g8 * 512);
      }
    });
  };
  static_for<MC::ST - 1>([&](auto s0) { issue(s0); });
  // the residual rows x[dst] for the projection's epilogue, requested now (after the first
  // stages) so that their latency hides behind the projection: the first two stage waits
  // leave these NX loads outstanding, the third covers them
  float4 xo[MC::FM][MC::FN_C];
  load_resid<MC>(x, dst, xo);
  constexpr int NX = MC::FM * MC::FN_C;
  static_for<NBC>([&](auto k) {
    const int i = t + MLP_THREADS * k;
    if (i < C) {
      sbo[i] = vbo[k];
      sb2[i] = vb2[k];
    }
  });
  static_for<NBR>([&](auto k) {
    const int i = t + MLP_THREADS * k;
    if (i < R) sb1[i] = vb1[k];
  });
  f32x4_t acc[MC::FM][MC::FN_C], hacc[MC::FM][MC::FN_H];
  static_for<MC::FM>([&](auto i) {
    static_for<MC::FN_C>([&](auto j) { acc[i][j] = f32x4_t{0.f, 0.f, 0.f, 0.f}; });
    static_for<MC::FN_H>([&](auto j) { hacc[i][j] = f32x4_t{0.f, 0.f, 0.f, 0.f}; });  // set per chunk below
  });
  float mean[MC::FM], rstd[MC::FM];
  // Before multiplying stage s: wait until it has landed (with a 3-stage ring at most the next
  // stage's loads outstanding, or none after a stretch of other vector-memory traffic), then
  // queue s + ST - 1.
  bool drained = true;  // the bias loads and row indices above are vector-memory reads
  auto enter = [&](int s) {
    if (MC::ST == 2 || drained || s + 1 >= MC::NSTAGE)
      vm_wait_barrier<0>();
    else if (stage_rows(s + 1) == MC::CS)
      vm_wait_barrier<(MC::ST == 3 ? MC::CS / (8 * NW) : 0)>();
    else
      vm_wait_barrier<(MC::ST == 3 ? HC * MC::KB1 / (8 * NW) : 0)>();
    drained = false;
    if (s + MC::ST - 1 < MC::NSTAGE) issue(s + MC::ST - 1);
    return ring + (s % MC::ST) * MC::SLOT;
  };
  int s = 0;
  static_assert(MC::ST == 3, "the counted waits below assume a 3-stage ring");
  // stage s + 1's loads per wavefront (s = 0, 1): the counts of the first two waits
  constexpr int L1 = stage_rows(1) / (8 * NW), L2 = stage_rows(2) / (8 * NW);
  static_for<MC::NKC * MC::NHALF>([&](auto sk) {
    constexpr int kb = sk / MC::NHALF, h = sk % MC::NHALF;
    const bf16* ws;
    if constexpr (sk == 0) {  // outstanding: stage 0, stage 1, x rows
      vm_wait_barrier<L1 + NX>();
      drained = false;
      issue(s + MC::ST - 1);
      ws = ring;
    } else if constexpr (sk == 1) {  // outstanding: stage 1, x rows, stage 2
      vm_wait_barrier<NX + L2>();
      issue(s + MC::ST - 1);
      ws = ring + MC::SLOT;
    } else {
      ws = enter(s);
    }
    mfma_block<MC, MC::FPH, h * MC::FPH, MC::FN_C>(ares + kb * BM * 64, ws, acc);
    ++s;
  });
  // x1 = x + o W_o^T + b_o; u2 = normalise(x1) into the resident tile (every wavefront has
  // finished reading o there: resid_rows passes two block barriers)
  // x1 stays in registers (xo) for the second residual (or goes to x and is read back)
  resid_rows<MC>(acc, sbo, x, dst, xo, red, mean, rstd, !MC::X1_REGS);
  if constexpr (MC::X1_REGS)
    static_for<MC::FM>([&](auto i) {
      static_for<MC::FN_C>([&](auto j) { xo[i][j] = make_float4(acc[i][j][0], acc[i][j][1], acc[i][j][2], acc[i][j][3]); });
    });
  static_for<MC::FM>([&](auto i) {
    const int r = wm * MC::TM + 16 * i + l16;
    static_for<MC::FN_C>([&](auto j) {
      const int n = MC::col(wn, j) + 4 * kg;
      const f32x4_t& a = acc[i][j];
      uint2 pk;
      pk.x = pack_bf2((a[0] - mean[i]) * rstd[i], (a[1] - mean[i]) * rstd[i]);
      pk.y = pack_bf2((a[2] - mean[i]) * rstd[i], (a[3] - mean[i]) * rstd[i]);
      *reinterpret_cast<uint2*>(ares + res_off<MC::BM>(r, n)) = pk;
      acc[i][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};
    });
  });
  drained = true;  // x was read and written
  // this wavefront's u2 fragments stay in registers for every hidden chunk
  lds_barrier();
  bf16x8_t ua[MC::NKC][2][MC::FM];
  static_for<MC::NKC>([&](auto kb) {
    static_for<2>([&](auto kk) {
      static_for<MC::FM>([&](auto i) {
        const int row = wm * MC::TM + 16 * i + l16;
        ua[kb][kk][i] = *reinterpret_cast<const bf16x8_t*>(ares + kb * BM * 64 + row * 64 +
                                                           (((4 * kk + kg) ^ lds_swz(row)) * 8));
      });
    });
  });
  // unrolled: every stage index, ring slot and wait count below is a constant (1.2 % per clip
  // at 5 x 240 x 432, timed back to back on one GPU)
#pragma unroll
  for (int j = 0; j < MC::NCH; ++j) {
    // the chunk's accumulators start at its bias b1' (the GELU epilogue then adds nothing)
    static_for<MC::FN_H>([&](auto jj) {
      const float4 b4 = *reinterpret_cast<const float4*>(sb1 + j * HC + wn * 16 * MC::FN_H + 16 * jj + 4 * kg);
      static_for<MC::FM>([&](auto i) { hacc[i][jj] = f32x4_t{b4.x, b4.y, b4.z, b4.w}; });
    });
    static_for<MC::NW1>([&](auto tt) {
      const bf16* ws = enter(s);
      static_for<MC::KB1>([&](auto b) { mfma_block_ra<MC, MC::FN_H>(ua[tt * MC::KB1 + b], ws + b * HC * 64, hacc); });
      ++s;
    });
    // hidden chunk j: GELU into the H tile (its previous contents were consumed before this
    // stage's barrier); the weights carry GELU's constant factors (gelu_scaled)
    static_for<MC::FM>([&](auto i) {
      const int r = wm * MC::TM + 16 * i + l16;
      static_for<MC::FN_H>([&](auto jj) {
        const int c = wn * 16 * MC::FN_H + 16 * jj + 4 * kg;
        const f32x4_t& a = hacc[i][jj];
        uint2 pk;
        pk.x = pack_bf2(gelu_scaled(a[0]), gelu_scaled(a[1]));
        pk.y = pack_bf2(gelu_scaled(a[2]), gelu_scaled(a[3]));
        *reinterpret_cast<uint2*>(hres + res_off<MC::BM>(r, c)) = pk;
      });
    });
    static_for<MC::NKH * MC::NHALF>([&](auto sk) {
      constexpr int kb = sk / MC::NHALF, h = sk % MC::NHALF;
      const bf16* ws = enter(s);
      mfma_block<MC, MC::FPH, h * MC::FPH, MC::FN_C>(hres + kb * BM * 64, ws, acc);
      ++s;
    });
  }
  // x2 = x1 + h W_2^T + b_2; x^ = normalise(x2)
  if constexpr (!MC::X1_REGS) load_resid<MC>(x, dst, xo);  // this thread's own stores, an L2 hit
  resid_rows<MC>(acc, sb2, x, dst, xo, red, mean, rstd);
  static_for<MC::FM>([&](auto i) {
    if (dst[i] >= 0)
      static_for<MC::FN_C>([&](auto j) {
        const int n = MC::col(wn, j) + 4 * kg;
        const f32x4_t& a = acc[i][j];
        uint2 pk;
        pk.x = pack_bf2((a[0] - mean[i]) * rstd[i], (a[1] - mean[i]) * rstd[i]);
        pk.y = pack_bf2((a[2] - mean[i]) * rstd[i], (a[3] - mean[i]) * rstd[i]);
        *reinterpret_cast<uint2*>(xh + (size_t)dst[i] * C + n) = pk;
      });
  });
}

template <class MC>
static void mlp_launch(int m_max, const int32_t* m_dev, const bf16* o, const int32_t* rows, const bf16* wo,
                       const float* bo, const bf16* w1, const float* b1, const bf16* w2, const float* b2, float* x,
                       bf16* xh, hipStream_t s) {
  static bool attr = false;
  if (!attr) {
    allow_lds(mlp_block_kernel<MC>, MC::LDS_BYTES);
    attr = true;
  }
  mlp_block_kernel<MC><<<(m_max + MC::BM - 1) / MC::BM, MLP_THREADS, MC::LDS_BYTES, s>>>(m_dev, o, rows, wo, bo, w1,
                                                                                          b1, w2, b2, x, xh);
}

bool mlp_block_supported(int C, int R) { return R == 4 * C && (C == 64 || C == 128 || C == 256 || C == 384); }

void launch_mlp_block_bf16(int m_max, const int32_t* m_dev, int C, const bf16* o, const int32_t* rows,
                           const bf16* wo, const float* bo, const bf16* w1, const float* b1, const bf16* w2,
                           const float* b2, float* x, bf16* xh, hipStream_t s) {
  if (m_max <= 0) return;
  switch (C) {
    case 64: mlp_launch<MlpCfg<64, 128>>(m_max, m_dev, o, rows, wo, bo, w1, b1, w2, b2, x, xh, s); break;
    case 128: mlp_launch<MlpCfg<128, 128>>(m_max, m_dev, o, rows, wo, bo, w1, b1, w2, b2, x, xh, s); break;
    case 256: mlp_launch<MlpCfg<256, 128>>(m_max, m_dev, o, rows, wo, bo, w1, b1, w2, b2, x, xh, s); break;
    // dim 384: 64-row tiles with 192-row weight slots (W_o and W_2 k blocks in two halves) and
    // 192-wide hidden chunks fit the LDS (155 KB)
    case 384: mlp_launch<MlpCfg<384, 192, 64, 3, 192>>(m_max, m_dev, o, rows, wo, bo, w1, b1, w2, b2, x, xh, s); break;
    default: break;  // rejected by the caller (mlp_block_supported)
  }
}

}  // namespace dr
