// BF16 path on gfx950 matrix cores: v_mfma_f32_16x16x32_bf16 (FP32 accumulation) for the
// Q/K/V projection, the output projection and both MLP linears, and a fused window-attention
// kernel with K and V^T staged in LDS and the softmax max/sum in FP32 across lanes.
//
// MFMA 16x16x32 operand layout (wave64): lane l supplies row (l % 16) of A and column
// (l % 16) of B, each with 8 consecutive k values; the k group is (l / 16).  The result lane
// l holds C[4*(l/16) + i][l % 16], i = 0..3.  Only the pairing of A's and B's k slots matters
// for the sum, so any k permutation applied to both operands alike is legal; the attention
// kernel uses that to feed P straight from the score registers.
//
// Hazard rule.  The double-rate v_mfma_f32_16x16x32_bf16 keeps reading its A/B source VGPRs
// for a few cycles after issue, and a VALU write to one of those VGPRs right after the issue
// corrupts the product (seen as run-to-run differences of single output elements).  The
// compiler does not pad that write-after-read case, so every group of these MFMAs is fenced:
// scheduling barriers keep VALU code out of the group and an s_nop after the group gives the
// last MFMA time to read its operands.  Inside a group, each MFMA waits for the matrix pipe,
// which covers the operand reads of the one before it.  The attention kernel instead uses the
// single-rate 16x16x16 form, whose operands are read at issue.
#include "dr_device.h"
#include "dr_internal.h"

namespace dr {

__device__ __forceinline__ f32x4_t mfma16(const bf16x8_t& a, const bf16x8_t& b, const f32x4_t& c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Fences around a group of double-rate MFMAs (see the hazard rule above).
__device__ __forceinline__ void mfma_group_begin() { __builtin_amdgcn_sched_barrier(0); }
__device__ __forceinline__ void mfma_group_end() {
  __builtin_amdgcn_sched_barrier(0);
  asm volatile("s_nop 7" ::: "memory");
  __builtin_amdgcn_sched_barrier(0);
}

// k = 32 product from two single-rate 16x16x16 MFMAs (k slots 0-3, then 4-7).
__device__ __forceinline__ f32x4_t mfma16_x2(const bf16x8_t& a, const bf16x8_t& b, const f32x4_t& c) {
  const bf16x4_t a0 = {a[0], a[1], a[2], a[3]}, a1 = {a[4], a[5], a[6], a[7]};
  const bf16x4_t b0 = {b[0], b[1], b[2], b[3]}, b1 = {b[4], b[5], b[6], b[7]};
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a1, b1, __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a0, b0, c, 0, 0, 0), 0, 0, 0);
}

__device__ __forceinline__ f32x4_t mfma16k16(const bf16x4_t& a, const bf16x4_t& b, const f32x4_t& c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

template <typename T, typename S>
__device__ __forceinline__ T bitcast(const S& s) {
  static_assert(sizeof(T) == sizeof(S), "size");
  T t;
  __builtin_memcpy(&t, &s, sizeof(T));
  return t;
}

// ------------------------------------------------------------------------------------------
// Tiled GEMM core.  Block = 256 threads = 4 waves in a 2 x 2 grid; block tile BM x BN
// (tokens x output channels), each wave (BM/2) x (BN/2); BK = 64 per LDS stage, the next
// stage prefetched into registers while the current one is multiplied.
//
// Orientation: with CH_ROWS = true the MFMA's A operand is the weight tile, so each lane ends
// with 4 consecutive output channels of one token (row-major stores); with CH_ROWS = false
// each lane ends with 4 consecutive tokens of one channel (used for V^T).
// ------------------------------------------------------------------------------------------
constexpr int BK = 64;
constexpr int LDS_STRIDE = BK + 8;  // bf16 elements; 144 B rows keep ds_read_b128 conflict free

template <int BM, int BN>
struct GemmSmem {
  bf16 a[2][BM][LDS_STRIDE];
  bf16 w[2][BN][LDS_STRIDE];
};

template <int BM, int BN, bool CH_ROWS>
__device__ __forceinline__ void gemm_tile(const bf16* __restrict__ A, int M, int m0, int K,
                                          const bf16* __restrict__ W, int n0,
                                          GemmSmem<BM, BN>& sm, f32x4_t (&acc)[BM / 32][BN / 32]) {
  constexpr int TM = BM / 2, TN = BN / 2;        // wave tile
  constexpr int FM = TM / 16, FN = TN / 16;      // 16x16 fragments per wave
  constexpr int A_CHUNKS = BM * BK / 8 / 256;    // 16-byte chunks per thread
  constexpr int W_CHUNKS = BN * BK / 8 / 256;
  static_assert(A_CHUNKS >= 1 && W_CHUNKS >= 1, "tile too small");
  const int t = threadIdx.x;
  const int lane = t & 63, wv = t >> 6;
  const int wm = wv >> 1, wn = wv & 1;
  const int l16 = lane & 15, kg = lane >> 4;

#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};

  u32x4_t ra[A_CHUNKS], rw[W_CHUNKS];
  auto load = [&](int k0) {
    static_for<A_CHUNKS>([&](auto c) {
      const int id = t + 256 * c;
      const int row = id >> 3, col = (id & 7) * 8;
      const int m = m0 + row;
      ra[c] = (m < M) ? *reinterpret_cast<const u32x4_t*>(A + (size_t)m * K + k0 + col)
                      : u32x4_t{0u, 0u, 0u, 0u};
    });
    static_for<W_CHUNKS>([&](auto c) {
      const int id = t + 256 * c;
      const int row = id >> 3, col = (id & 7) * 8;
      rw[c] = *reinterpret_cast<const u32x4_t*>(W + (size_t)(n0 + row) * K + k0 + col);
    });
  };
  auto stash = [&](int buf) {
    static_for<A_CHUNKS>([&](auto c) {
      const int id = t + 256 * c;
      *reinterpret_cast<u32x4_t*>(&sm.a[buf][id >> 3][(id & 7) * 8]) = ra[c];
    });
    static_for<W_CHUNKS>([&](auto c) {
      const int id = t + 256 * c;
      *reinterpret_cast<u32x4_t*>(&sm.w[buf][id >> 3][(id & 7) * 8]) = rw[c];
    });
  };

  load(0);
  stash(0);
  __syncthreads();
  const int nk = K / BK;
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) load((kt + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 32) {
      bf16x8_t af[FM], wf[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i)
        af[i] = *reinterpret_cast<const bf16x8_t*>(&sm.a[buf][wm * TM + i * 16 + l16][kk + kg * 8]);
#pragma unroll
      for (int j = 0; j < FN; ++j)
        wf[j] = *reinterpret_cast<const bf16x8_t*>(&sm.w[buf][wn * TN + j * 16 + l16][kk + kg * 8]);
      mfma_group_begin();
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          acc[i][j] = CH_ROWS ? mfma16(wf[j], af[i], acc[i][j]) : mfma16(af[i], wf[j], acc[i][j]);
      mfma_group_end();
    }
    if (kt + 1 < nk) {
      stash(buf ^ 1);
      __syncthreads();
    }
  }
}

// ------------------------------------------------------------------------------------------
// Generic GEMM over compact rows: out = A W^T + bias with an epilogue.
//   EPI_STORE: bf16 out[m, n];  EPI_GELU: bf16 GELU;  EPI_RESID: f32 x[res_rows[m], n] += y.
// ------------------------------------------------------------------------------------------
template <int BM, int BN>
__global__ void __launch_bounds__(256) gemm_bf16_kernel(const bf16* __restrict__ A, const int32_t* __restrict__ m_dev,
                                                        int m_max, int K, const bf16* __restrict__ W,
                                                        const float* __restrict__ bias, int Nout, int epi,
                                                        void* __restrict__ out, const int32_t* __restrict__ res_rows) {
  __shared__ GemmSmem<BM, BN> sm;
  const int M = m_dev ? m_dev[0] : m_max;
  const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
  if (m0 >= M) return;
  f32x4_t acc[BM / 32][BN / 32];
  gemm_tile<BM, BN, true>(A, M, m0, K, W, n0, sm, acc);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int wm = wv >> 1, wn = wv & 1;
  const int l16 = lane & 15, kg = lane >> 4;
#pragma unroll
  for (int i = 0; i < BM / 32; ++i) {
    const int m = m0 + wm * (BM / 2) + i * 16 + l16;
    if (m >= M) continue;
#pragma unroll
    for (int j = 0; j < BN / 32; ++j) {
      const int n = n0 + wn * (BN / 2) + j * 16 + kg * 4;
      const float4 b4 = *reinterpret_cast<const float4*>(bias + n);
      float y0 = acc[i][j][0] + b4.x, y1 = acc[i][j][1] + b4.y;
      float y2 = acc[i][j][2] + b4.z, y3 = acc[i][j][3] + b4.w;
      if (epi == EPI_RESID) {
        const int dst = res_rows ? res_rows[m] : m;
        float4* p = reinterpret_cast<float4*>(static_cast<float*>(out) + (size_t)dst * Nout + n);
        float4 xv = *p;
        xv.x += y0; xv.y += y1; xv.z += y2; xv.w += y3;
        *p = xv;
      } else {
        if (epi == EPI_GELU) {
          y0 = gelu_erf(y0); y1 = gelu_erf(y1); y2 = gelu_erf(y2); y3 = gelu_erf(y3);
        }
        uint2 pk;
        pk.x = pack_bf2(y0, y1);
        pk.y = pack_bf2(y2, y3);
        *reinterpret_cast<uint2*>(static_cast<bf16*>(out) + (size_t)m * Nout + n) = pk;
      }
    }
  }
}

void launch_gemm_bf16(const bf16* A, const int32_t* m_dev, int m_max, int K, const bf16* W,
                      const float* bias, int Nout, int epi, void* out, const int32_t* res_rows,
                      hipStream_t s) {
  if (m_max <= 0) return;
  // 64-row tiles: the gathered row count is often only a few thousand
  if (Nout % 128 == 0) {
    dim3 grid((m_max + 63) / 64, Nout / 128);
    gemm_bf16_kernel<64, 128><<<grid, 256, 0, s>>>(A, m_dev, m_max, K, W, bias, Nout, epi, out, res_rows);
  } else {
    dim3 grid((m_max + 63) / 64, Nout / 64);
    gemm_bf16_kernel<64, 64><<<grid, 256, 0, s>>>(A, m_dev, m_max, K, W, bias, Nout, epi, out, res_rows);
  }
}

// ------------------------------------------------------------------------------------------
// LayerNorm-fused panel GEMM.  Block = 512 threads = 8 waves in 2 (rows) x 4 (columns); block
// tile 128 rows x BN output columns, wave tile 64 x BN/4.  The prologue normalises the block's
// 128 rows of the FP32 residual stream (one wavefront per row, FP32 statistics, biased
// variance, eps 1e-5) straight into a bf16 A panel holding the full K = C in LDS; the weight
// tile [BN][K] then streams through a two-stage LDS ring, the next stage prefetched into
// registers while the current one is multiplied.  Rows come from x[rows[r]] (gathered) or
// x[r]; the first *m_dev (or m_max) rows are valid.
// ------------------------------------------------------------------------------------------
constexpr int PANEL_M = 128;
constexpr int PANEL_THREADS = 512;

template <int BN>
__host__ __device__ constexpr size_t panel_smem_bytes(int K) {
  return (size_t)PANEL_M * (K + 8) * 2 + (size_t)2 * BN * LDS_STRIDE * 2;
}

constexpr int LN_BATCH = 8;

// 128 panel rows -> LayerNorm -> bf16; K = 64 * KPER channels; lane owns channels lane + 64 e.
template <int KPER>
__device__ __forceinline__ void ln_rows_to_panel(const float* __restrict__ x, const int32_t* __restrict__ rows,
                                                 int M, int m0, const float* __restrict__ lng,
                                                 const float* __restrict__ lnb, bf16* apanel, int KS) {
  constexpr int K = 64 * KPER;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  float g[KPER], b[KPER];
#pragma unroll
  for (int e = 0; e < KPER; ++e) {
    g[e] = lng[lane + 64 * e];
    b[e] = lnb[lane + 64 * e];
  }
  for (int r0 = wv; r0 < PANEL_M; r0 += LN_BATCH * (PANEL_THREADS / 64)) {
    float v[LN_BATCH][KPER];
#pragma unroll
    for (int j = 0; j < LN_BATCH; ++j) {
      const int r = r0 + j * (PANEL_THREADS / 64);
      const int m = m0 + r;
      if (r < PANEL_M && m < M) {
        const float* xr = x + (size_t)(rows ? rows[m] : m) * K;
#pragma unroll
        for (int e = 0; e < KPER; ++e) v[j][e] = xr[lane + 64 * e];
      } else {
#pragma unroll
        for (int e = 0; e < KPER; ++e) v[j][e] = 0.f;
      }
    }
#pragma unroll
    for (int j = 0; j < LN_BATCH; ++j) {
      const int r = r0 + j * (PANEL_THREADS / 64);
      if (r >= PANEL_M) break;
      bf16* arow = apanel + (size_t)r * KS;
      if (m0 + r >= M) {
#pragma unroll
        for (int e = 0; e < KPER; ++e) arow[lane + 64 * e] = 0;
        continue;
      }
      float sum = 0.f;
#pragma unroll
      for (int e = 0; e < KPER; ++e) sum += v[j][e];
      const float mean = wave_sum(sum) / K;
      float sq = 0.f;
#pragma unroll
      for (int e = 0; e < KPER; ++e) {
        const float d = v[j][e] - mean;
        sq += d * d;
      }
      const float rstd = rsqrtf(wave_sum(sq) / K + 1e-5f);
#pragma unroll
      for (int e = 0; e < KPER; ++e) arow[lane + 64 * e] = f2bf((v[j][e] - mean) * rstd * g[e] + b[e]);
    }
  }
}

// any K (multiple of 64, at most 1024): one row at a time
__device__ __forceinline__ void ln_rows_to_panel_any(const float* __restrict__ x, const int32_t* __restrict__ rows,
                                                     int M, int m0, int K, const float* __restrict__ lng,
                                                     const float* __restrict__ lnb, bf16* apanel, int KS) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int per = K / 64;
  for (int r = wv; r < PANEL_M; r += PANEL_THREADS / 64) {
    const int m = m0 + r;
    bf16* arow = apanel + (size_t)r * KS;
    if (m < M) {
      const float* xr = x + (size_t)(rows ? rows[m] : m) * K;
      float v[16];
      float sum = 0.f;
      for (int e = 0; e < per; ++e) {
        v[e] = xr[lane + 64 * e];
        sum += v[e];
      }
      const float mean = wave_sum(sum) / K;
      float sq = 0.f;
      for (int e = 0; e < per; ++e) {
        const float d = v[e] - mean;
        sq += d * d;
      }
      const float rstd = rsqrtf(wave_sum(sq) / K + 1e-5f);
      for (int e = 0; e < per; ++e) {
        const int c = lane + 64 * e;
        arow[c] = f2bf((v[e] - mean) * rstd * lng[c] + lnb[c]);
      }
    } else {
      for (int e = 0; e < per; ++e) arow[lane + 64 * e] = 0;
    }
  }
}

template <int BN, class Epi>
__device__ __forceinline__ void panel_gemm(const float* __restrict__ x, const int32_t* __restrict__ rows,
                                           int M, int m0, int K, const float* __restrict__ lng,
                                           const float* __restrict__ lnb, const bf16* __restrict__ W, int n0,
                                           bf16* smem, Epi& epi) {
  constexpr int FN = BN / 64;              // 16-wide fragments per wave in N
  constexpr int W_CHUNKS = BN * BK / 8 / PANEL_THREADS;
  static_assert(FN >= 1 && W_CHUNKS >= 1, "panel tile too small");
  const int KS = K + 8;                    // A panel row stride (bf16)
  bf16* apanel = smem;
  bf16* wst = smem + (size_t)PANEL_M * KS;  // [2][BN][LDS_STRIDE]
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int wm = wv >> 2, wn = wv & 3;
  const int l16 = lane & 15, kg = lane >> 4;

  u32x4_t rw[W_CHUNKS];
  auto load_w = [&](int k0) {
    static_for<W_CHUNKS>([&](auto c) {
      const int id = t + PANEL_THREADS * c;
      rw[c] = *reinterpret_cast<const u32x4_t*>(W + (size_t)(n0 + (id >> 3)) * K + k0 + (id & 7) * 8);
    });
  };
  auto stash_w = [&](int buf) {
    static_for<W_CHUNKS>([&](auto c) {
      const int id = t + PANEL_THREADS * c;
      *reinterpret_cast<u32x4_t*>(wst + ((size_t)buf * BN + (id >> 3)) * LDS_STRIDE + (id & 7) * 8) = rw[c];
    });
  };
  load_w(0);

  // LayerNorm prologue: wave wv normalises rows wv, wv + 8, ... in batches of LN_BATCH rows
  // whose loads are all issued before the first reduction (hides the load latency).
  switch (K / 64) {
    case 1: ln_rows_to_panel<1>(x, rows, M, m0, lng, lnb, apanel, KS); break;
    case 2: ln_rows_to_panel<2>(x, rows, M, m0, lng, lnb, apanel, KS); break;
    case 4: ln_rows_to_panel<4>(x, rows, M, m0, lng, lnb, apanel, KS); break;
    case 6: ln_rows_to_panel<6>(x, rows, M, m0, lng, lnb, apanel, KS); break;
    default: ln_rows_to_panel_any(x, rows, M, m0, K, lng, lnb, apanel, KS); break;
  }
  stash_w(0);
  __syncthreads();

  f32x4_t acc[4][FN];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};

  const int nk = K / BK;
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) load_w((kt + 1) * BK);
    const bf16* wb = wst + (size_t)buf * BN * LDS_STRIDE;
#pragma unroll
    for (int kk = 0; kk < BK; kk += 32) {
      bf16x8_t af[4], wf[FN];
#pragma unroll
      for (int i = 0; i < 4; ++i)
        af[i] = *reinterpret_cast<const bf16x8_t*>(apanel + (size_t)(wm * 64 + i * 16 + l16) * KS + kt * BK + kk + kg * 8);
#pragma unroll
      for (int j = 0; j < FN; ++j)
        wf[j] = *reinterpret_cast<const bf16x8_t*>(wb + (size_t)(wn * (BN / 4) + j * 16 + l16) * LDS_STRIDE + kk + kg * 8);
      mfma_group_begin();
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = mfma16(wf[j], af[i], acc[i][j]);
      mfma_group_end();
    }
    if (kt + 1 < nk) {
      stash_w(buf ^ 1);
      __syncthreads();
    }
  }
  // lane holds output channels n .. n+3 of token m
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int m = m0 + wm * 64 + i * 16 + l16;
    if (m >= M) continue;
#pragma unroll
    for (int j = 0; j < FN; ++j) epi(m, n0 + wn * (BN / 4) + j * 16 + kg * 4, acc[i][j]);
  }
}

// Q/K/V epilogue: columns [0, C) -> Q rows [N, C]; [C, 2C) -> K, [2C, 3C) -> V, both
// [win][head][Spad][dh].
struct QkvEpi {
  const float* bias;
  bf16 *q, *k, *v;
  int C, dh, heads, Spad, S;
  __device__ __forceinline__ void operator()(int m, int n, const f32x4_t& a) const {
    const float4 b4 = *reinterpret_cast<const float4*>(bias + n);
    uint2 pk;
    pk.x = pack_bf2(a[0] + b4.x, a[1] + b4.y);
    pk.y = pack_bf2(a[2] + b4.z, a[3] + b4.w);
    bf16* dst;
    if (n < C) {
      dst = q + (size_t)m * C + n;
    } else {
      const int part = n < 2 * C ? 1 : 2;
      const int c = n - part * C, hh = c / dh, d = c - hh * dh;
      const int w = m / S, s = m - w * S;
      dst = (part == 1 ? k : v) + (((size_t)w * heads + hh) * Spad + s) * dh + d;
    }
    *reinterpret_cast<uint2*>(dst) = pk;
  }
};

// LN1 + Q/K/V over all N tokens.  Column blocks of Q run only for row tiles holding a
// flagged token; K/V blocks only for row tiles touching a window that has queries (keys and
// values of a window without queries are never read).
template <int BN>
__global__ void __launch_bounds__(PANEL_THREADS) ln_qkv_kernel(Geo g, int C, int heads, int Spad,
                                                               const float* __restrict__ x,
                                                               const uint8_t* __restrict__ flag,
                                                               const int32_t* __restrict__ wcount,
                                                               const float* __restrict__ lng,
                                                               const float* __restrict__ lnb,
                                                               const bf16* __restrict__ W,
                                                               const float* __restrict__ bias, bf16* q,
                                                               bf16* k, bf16* v) {
  extern __shared__ __align__(16) bf16 smem_panel[];
  const int M = g.N;
  const int n0 = blockIdx.x * BN, m0 = blockIdx.y * PANEL_M;
  const bool is_q = n0 < C;
  int need = 0;
  if (threadIdx.x < PANEL_M && m0 + threadIdx.x < M) {
    const int m = m0 + threadIdx.x;
    need = is_q ? flag[m] != 0 : wcount[m / g.S] > 0;
  }
  if (!__syncthreads_or(need)) return;
  QkvEpi epi{bias, q, k, v, C, C / heads, heads, Spad, g.S};
  panel_gemm<BN>(x, nullptr, M, m0, C, lng, lnb, W, n0, smem_panel, epi);
}

template <class K>
static void allow_smem(K kernel, size_t bytes) {
  if (bytes > 65536)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)bytes);
}

template <int BN>
static void qkv_launch(const Geo& g, int C, int heads, int Spad, const float* x, const uint8_t* flag,
                       const int32_t* wcount, const float* lng, const float* lnb, const bf16* w,
                       const float* bias, bf16* q, bf16* k, bf16* v, hipStream_t s) {
  const size_t smem = panel_smem_bytes<BN>(C);
  static size_t granted = 0;
  if (smem > granted) {
    allow_smem(ln_qkv_kernel<BN>, smem);
    granted = smem;
  }
  dim3 grid(3 * C / BN, (g.N + PANEL_M - 1) / PANEL_M);
  ln_qkv_kernel<BN><<<grid, PANEL_THREADS, smem, s>>>(g, C, heads, Spad, x, flag, wcount, lng, lnb, w, bias, q, k, v);
}

void launch_ln_qkv_bf16(const Geo& g, int C, int heads, int Spad, const float* x, const uint8_t* flag,
                        const int32_t* wcount, const float* lng, const float* lnb, const bf16* w,
                        const float* bias, bf16* q, bf16* k, bf16* v, hipStream_t s) {
  if (C % 256 == 0 && panel_smem_bytes<256>(C) <= 160 * 1024)
    qkv_launch<256>(g, C, heads, Spad, x, flag, wcount, lng, lnb, w, bias, q, k, v, s);
  else if (C % 128 == 0)
    qkv_launch<128>(g, C, heads, Spad, x, flag, wcount, lng, lnb, w, bias, q, k, v, s);
  else
    qkv_launch<64>(g, C, heads, Spad, x, flag, wcount, lng, lnb, w, bias, q, k, v, s);
}

// Entry r of a per-request table held in the kernel arguments, read through selects: a
// runtime index into the argument struct would copy the whole table to scratch memory.
template <class T>
__device__ __forceinline__ T pick(const T (&a)[STREAM_MAXB], int r) {
  T v = a[0];
  static_for<STREAM_MAXB>([&](auto i) {
    if (i == r) v = a[i];
  });
  return v;
}

// Stream-mode Q/K/V epilogue: Q rows into the batch buffer; K and V of every token into the
// current ring slot of its request's cache ([win_f][head][S_f][dh] per block and slot).
struct StreamQkvEpi {
  const float* bias;
  bf16* q;
  StreamTable tab;
  int C, dh, heads, Sf, nwin_f;
  __device__ __forceinline__ void operator()(int m, int n, const f32x4_t& a) const {
    const float4 b4 = *reinterpret_cast<const float4*>(bias + n);
    uint2 pk;
    pk.x = pack_bf2(a[0] + b4.x, a[1] + b4.y);
    pk.y = pack_bf2(a[2] + b4.z, a[3] + b4.w);
    bf16* dst;
    if (n < C) {
      dst = q + (size_t)m * C + n;
    } else {
      const int part = n < 2 * C ? 1 : 2;
      const int c = n - part * C, hh = c / dh, d = c - hh * dh;
      const int w = m / Sf, s = m - w * Sf;
      const int r = w / nwin_f, wl = w - r * nwin_f;
      dst = (part == 1 ? pick(tab.k, r) : pick(tab.v, r)) + (size_t)pick(tab.head, r) * tab.slot_stride +
            (((size_t)wl * heads + hh) * Sf + s) * dh + d;
    }
    *reinterpret_cast<uint2*>(dst) = pk;
  }
};

// LN1 + Q/K/V for a batch of new frames: K/V of every token (later frames may query any
// window), Q only for row tiles holding a flagged token.
template <int BN>
__global__ void __launch_bounds__(PANEL_THREADS) ln_qkv_stream_kernel(Geo g, int C, int heads,
                                                                      const float* __restrict__ x,
                                                                      const uint8_t* __restrict__ flag,
                                                                      const float* __restrict__ lng,
                                                                      const float* __restrict__ lnb,
                                                                      const bf16* __restrict__ W,
                                                                      const float* __restrict__ bias, bf16* q,
                                                                      StreamTable tab) {
  extern __shared__ __align__(16) bf16 smem_panel[];
  const int M = g.N;
  const int n0 = blockIdx.x * BN, m0 = blockIdx.y * PANEL_M;
  if (n0 < C) {
    int need = 0;
    if (threadIdx.x < PANEL_M && m0 + threadIdx.x < M) need = flag[m0 + threadIdx.x] != 0;
    if (!__syncthreads_or(need)) return;
  }
  StreamQkvEpi epi{bias, q, tab, C, C / heads, heads, g.S, g.nwh * g.nww};
  panel_gemm<BN>(x, nullptr, M, m0, C, lng, lnb, W, n0, smem_panel, epi);
}

template <int BN>
static void qkv_stream_launch(const Geo& g, int C, int heads, const float* x, const uint8_t* flag,
                              const float* lng, const float* lnb, const bf16* w, const float* bias, bf16* q,
                              const StreamTable& tab, hipStream_t s) {
  const size_t smem = panel_smem_bytes<BN>(C);
  static size_t granted = 0;
  if (smem > granted) {
    allow_smem(ln_qkv_stream_kernel<BN>, smem);
    granted = smem;
  }
  dim3 grid(3 * C / BN, (g.N + PANEL_M - 1) / PANEL_M);
  ln_qkv_stream_kernel<BN><<<grid, PANEL_THREADS, smem, s>>>(g, C, heads, x, flag, lng, lnb, w, bias, q, tab);
}

void launch_ln_qkv_stream(const Geo& g, int C, int heads, const float* x, const uint8_t* flag, const float* lng,
                          const float* lnb, const bf16* w, const float* bias, bf16* q, const StreamTable& tab,
                          hipStream_t s) {
  if (C % 256 == 0 && panel_smem_bytes<256>(C) <= 160 * 1024)
    qkv_stream_launch<256>(g, C, heads, x, flag, lng, lnb, w, bias, q, tab, s);
  else if (C % 128 == 0)
    qkv_stream_launch<128>(g, C, heads, x, flag, lng, lnb, w, bias, q, tab, s);
  else
    qkv_stream_launch<64>(g, C, heads, x, flag, lng, lnb, w, bias, q, tab, s);
}

// GELU epilogue: h[m, n] = bf16(GELU(acc + b)).
struct GeluEpi {
  const float* bias;
  bf16* h;
  int R;
  __device__ __forceinline__ void operator()(int m, int n, const f32x4_t& a) const {
    const float4 b4 = *reinterpret_cast<const float4*>(bias + n);
    uint2 pk;
    pk.x = pack_bf2(gelu_erf(a[0] + b4.x), gelu_erf(a[1] + b4.y));
    pk.y = pack_bf2(gelu_erf(a[2] + b4.z), gelu_erf(a[3] + b4.w));
    *reinterpret_cast<uint2*>(h + (size_t)m * R + n) = pk;
  }
};

// LN2 + first MLP linear + GELU over the gathered query rows x[idx[r]], r < *nq.
template <int BN>
__global__ void __launch_bounds__(PANEL_THREADS) ln_fc1_kernel(int C, int R, const float* __restrict__ x,
                                                               const int32_t* __restrict__ idx,
                                                               const int32_t* __restrict__ nq,
                                                               const float* __restrict__ lng,
                                                               const float* __restrict__ lnb,
                                                               const bf16* __restrict__ W,
                                                               const float* __restrict__ bias, bf16* h) {
  extern __shared__ __align__(16) bf16 smem_panel[];
  const int M = nq[0];
  const int n0 = blockIdx.x * BN, m0 = blockIdx.y * PANEL_M;
  if (m0 >= M) return;
  GeluEpi epi{bias, h, R};
  panel_gemm<BN>(x, idx, M, m0, C, lng, lnb, W, n0, smem_panel, epi);
}

template <int BN>
static void fc1_launch(int m_max, int C, int R, const float* x, const int32_t* idx, const int32_t* nq,
                       const float* lng, const float* lnb, const bf16* w, const float* bias, bf16* h,
                       hipStream_t s) {
  const size_t smem = panel_smem_bytes<BN>(C);
  static size_t granted = 0;
  if (smem > granted) {
    allow_smem(ln_fc1_kernel<BN>, smem);
    granted = smem;
  }
  dim3 grid(R / BN, (m_max + PANEL_M - 1) / PANEL_M);
  ln_fc1_kernel<BN><<<grid, PANEL_THREADS, smem, s>>>(C, R, x, idx, nq, lng, lnb, w, bias, h);
}

void launch_ln_fc1_bf16(int m_max, int C, int R, const float* x, const int32_t* idx, const int32_t* nq,
                        const float* lng, const float* lnb, const bf16* w, const float* bias, bf16* h,
                        hipStream_t s) {
  if (m_max <= 0) return;
  if (R % 256 == 0 && panel_smem_bytes<256>(C) <= 160 * 1024)
    fc1_launch<256>(m_max, C, R, x, idx, nq, lng, lnb, w, bias, h, s);
  else if (R % 128 == 0)
    fc1_launch<128>(m_max, C, R, x, idx, nq, lng, lnb, w, bias, h, s);
  else
    fc1_launch<64>(m_max, C, R, x, idx, nq, lng, lnb, w, bias, h, s);
}

// ------------------------------------------------------------------------------------------
// Window attention on MFMA.  Block = 4 waves = 64 queries of one (window, head); K and V of
// the window/head ([Spad][dh] each in global memory) are staged in LDS once, V transposed to
// V^T [dh][keys] on the way in.  Each wave: 16 queries.
//   S^T tile (16 keys x 16 queries) = K_tile (16 x dh) . Q^T  -> lane l holds the scores of
//   query l%16 for keys 16t + 4*(l/16) + i.  Softmax statistics stay FP32: max/sum over
//   registers, then across the 4 lane groups with two xor shuffles.
//   O^T (16 dh x 16 queries) = V^T (dh x keys) . P^T, with P taken from the score registers
//   (the k slots of both operands use the same key permutation).
// ------------------------------------------------------------------------------------------
template <int DH, int NT>
struct AttnTile {
  static constexpr int SP = NT * 16;   // padded window length
  static constexpr int KST = DH + 8;   // LDS row stride of K (bf16)
  static constexpr int VST = SP + 4;   // LDS row stride of V^T: rows spread over distinct bank
                                       // pairs, 8-byte aligned
};

// Stage `nrows` keys/values (rows of [.][DH] in global memory) into LDS rows row0.. of K and
// columns row0.. of V^T.
template <int DH, int NT>
__device__ __forceinline__ void attn_stage(bf16* Ks, bf16* Vs, const bf16* __restrict__ kg_,
                                           const bf16* __restrict__ vg_, int row0, int nrows) {
  using AT = AttnTile<DH, NT>;
  const int t = threadIdx.x;
  for (int c = t; c < nrows * DH / 8; c += 256) {
    const int row = c / (DH / 8), col = (c % (DH / 8)) * 8;
    *reinterpret_cast<uint4*>(&Ks[(row0 + row) * AT::KST + col]) = *reinterpret_cast<const uint4*>(kg_ + row * DH + col);
  }
  for (int c = t; c < nrows * DH / 8; c += 256) {
    const int key = c / (DH / 8), d0 = (c % (DH / 8)) * 8;
    const uint4 v = *reinterpret_cast<const uint4*>(vg_ + key * DH + d0);
    const uint32_t wds[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      Vs[(d0 + 2 * e) * AT::VST + row0 + key] = (bf16)(wds[e] & 0xffffu);
      Vs[(d0 + 2 * e + 1) * AT::VST + row0 + key] = (bf16)(wds[e] >> 16);
    }
  }
}

// Queries of one (window, head, 64-query tile) against the S keys staged in LDS (rows >= S of
// K and columns >= S of V^T must be finite; their scores are masked to -inf).
template <int DH, int NT>
__device__ __forceinline__ void attn_compute(const bf16* Ks, const bf16* Vs, int S, int C, int h,
                                             const bf16* __restrict__ q, const int32_t* __restrict__ idx,
                                             int q0, int nqw, int qbase, bf16* __restrict__ o,
                                             float* __restrict__ amax_o) {
  constexpr int KST = AttnTile<DH, NT>::KST;
  constexpr int VST = AttnTile<DH, NT>::VST;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int l16 = lane & 15, kg = lane >> 4;
  const int qi = qbase + wv * 16 + l16;  // this lane's query (column of S^T)
  if (qbase + wv * 16 >= nqw) return;    // whole wave idle (no block barrier follows)
  const bool valid = qi < nqw;
  const int r = q0 + (valid ? qi : 0);
  const int n = idx[r];

  // Q^T operand: lane holds q[n][kk*32 + 8*kg .. +7]
  bf16x8_t qf[DH / 32];
#pragma unroll
  for (int kk = 0; kk < DH / 32; ++kk) {
    uint4 v = valid ? *reinterpret_cast<const uint4*>(q + (size_t)n * C + h * DH + kk * 32 + kg * 8)
                    : make_uint4(0, 0, 0, 0);
    qf[kk] = bitcast<bf16x8_t>(v);
  }

  const float sl2 = 1.4426950408889634f / sqrtf((float)DH);  // log2(e) / sqrt(dh)
  float sc[NT][4];
#pragma unroll
  for (int tt = 0; tt < NT; ++tt) {
    f32x4_t a = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kk = 0; kk < DH / 32; ++kk) {
      const bf16x8_t kf = *reinterpret_cast<const bf16x8_t*>(&Ks[(tt * 16 + l16) * KST + kk * 32 + kg * 8]);
      a = mfma16_x2(kf, qf[kk], a);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int key = tt * 16 + kg * 4 + i;
      sc[tt][i] = key < S ? a[i] * sl2 : -INFINITY;
    }
  }
  float mx = -INFINITY;
#pragma unroll
  for (int tt = 0; tt < NT; ++tt)
#pragma unroll
    for (int i = 0; i < 4; ++i) mx = fmaxf(mx, sc[tt][i]);
  mx = fmaxf(mx, __shfl_xor(mx, 16, 64));
  mx = fmaxf(mx, __shfl_xor(mx, 32, 64));
  float sum = 0.f;
#pragma unroll
  for (int tt = 0; tt < NT; ++tt)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float p = exp2f(sc[tt][i] - mx);
      sc[tt][i] = p;
      sum += p;
    }
  sum += __shfl_xor(sum, 16, 64);
  sum += __shfl_xor(sum, 32, 64);
  const float inv = 1.0f / sum;
  float omax = 0.f;

#pragma unroll
  for (int dt = 0; dt < DH / 16; ++dt) {
    f32x4_t a = {0.f, 0.f, 0.f, 0.f};
    const bf16* vrow = &Vs[(dt * 16 + l16) * VST];
#pragma unroll
    for (int tt = 0; tt + 1 < NT; tt += 2) {
      const uint2 v0 = *reinterpret_cast<const uint2*>(vrow + tt * 16 + kg * 4);
      const uint2 v1 = *reinterpret_cast<const uint2*>(vrow + tt * 16 + 16 + kg * 4);
      uint4 pv;
      pv.x = pack_bf2(sc[tt][0], sc[tt][1]);
      pv.y = pack_bf2(sc[tt][2], sc[tt][3]);
      pv.z = pack_bf2(sc[tt + 1][0], sc[tt + 1][1]);
      pv.w = pack_bf2(sc[tt + 1][2], sc[tt + 1][3]);
      const uint4 vv = make_uint4(v0.x, v0.y, v1.x, v1.y);
      a = mfma16_x2(bitcast<bf16x8_t>(vv), bitcast<bf16x8_t>(pv), a);
    }
    if (NT & 1) {
      constexpr int tt = NT - 1;
      const uint2 v0 = *reinterpret_cast<const uint2*>(vrow + tt * 16 + kg * 4);
      uint2 pv;
      pv.x = pack_bf2(sc[tt][0], sc[tt][1]);
      pv.y = pack_bf2(sc[tt][2], sc[tt][3]);
      a = mfma16k16(bitcast<bf16x4_t>(v0), bitcast<bf16x4_t>(pv), a);
    }
    if (valid) {
      uint2 pk;
      pk.x = pack_bf2(a[0] * inv, a[1] * inv);
      pk.y = pack_bf2(a[2] * inv, a[3] * inv);
      *reinterpret_cast<uint2*>(o + (size_t)r * C + h * DH + dt * 16 + kg * 4) = pk;
      omax = fmaxf(omax, fmaxf(fmaxf(fabsf(a[0]), fabsf(a[1])), fmaxf(fabsf(a[2]), fabsf(a[3]))) * inv);
    }
  }
  if (amax_o) {
    // max |O| of this wave into the per-call slot (non-negative floats order like their bits)
    const float wmx = wave_max(omax);
    if (lane == 0 && wmx > 0.f) atomicMax(reinterpret_cast<unsigned int*>(amax_o), __float_as_uint(wmx));
  }
}

template <int DH, int NT>
__global__ void __launch_bounds__(256) attn_bf16_kernel(Geo g, int C, int heads, const bf16* __restrict__ q,
                                                        const bf16* __restrict__ kmat, const bf16* __restrict__ vmat,
                                                        const int32_t* __restrict__ idx,
                                                        const int32_t* __restrict__ woff, bf16* __restrict__ o,
                                                        float* __restrict__ amax_o) {
  using AT = AttnTile<DH, NT>;
  __shared__ bf16 Ks[AT::SP * AT::KST];
  __shared__ bf16 Vs[DH * AT::VST];
  const int w = blockIdx.x / heads, h = blockIdx.x - w * heads;
  const int q0 = woff[w], nqw = woff[w + 1] - q0;
  const int qbase = blockIdx.y * 64;
  if (qbase >= nqw) return;
  // K and V of (w, h) hold SP rows, the pad rows zero in memory
  attn_stage<DH, NT>(Ks, Vs, kmat + ((size_t)w * heads + h) * AT::SP * DH, vmat + ((size_t)w * heads + h) * AT::SP * DH,
                     0, AT::SP);
  __syncthreads();
  attn_compute<DH, NT>(Ks, Vs, g.S, C, h, q, idx, q0, nqw, qbase, o, amax_o);
}

// Stream mode: the keys of window (request r, window wl) are the window's rows in the
// request's cached frames (oldest first) followed by the new frame, each frame block being
// S_f = wh*ww rows of a ring slot [win_f][head][S_f][dh].
template <int DH, int NT>
__global__ void __launch_bounds__(256) attn_stream_kernel(StreamTable tab, int C, int heads, int Sf, int nwin_f,
                                                          const bf16* __restrict__ q, const int32_t* __restrict__ idx,
                                                          const int32_t* __restrict__ woff, bf16* __restrict__ o) {
  using AT = AttnTile<DH, NT>;
  __shared__ bf16 Ks[AT::SP * AT::KST];
  __shared__ bf16 Vs[DH * AT::VST];
  const int w = blockIdx.x / heads, h = blockIdx.x - w * heads;
  const int q0 = woff[w], nqw = woff[w + 1] - q0;
  const int qbase = blockIdx.y * 64;
  if (qbase >= nqw) return;
  const int r = w / nwin_f, wl = w - r * nwin_f;
  const int np = pick(tab.npast, r), hd = pick(tab.head, r), nT = pick(tab.T, r);
  const bf16* kr = pick(tab.k, r);
  const bf16* vr = pick(tab.v, r);
  const size_t off = ((size_t)wl * heads + h) * Sf * DH;
  for (int j = 0; j <= np; ++j) {
    const int slot = (hd - np + j + nT) % nT;
    attn_stage<DH, NT>(Ks, Vs, kr + (size_t)slot * tab.slot_stride + off, vr + (size_t)slot * tab.slot_stride + off,
                       j * Sf, Sf);
  }
  const int S = (np + 1) * Sf;
  // zero the pad keys (rows of K, columns of V^T) so that P = 0 meets finite values
  for (int e = threadIdx.x; e < (AT::SP - S) * DH; e += 256) {
    const int row = S + e / DH, d = e % DH;
    Ks[row * AT::KST + d] = 0;
    Vs[d * AT::VST + row] = 0;
  }
  __syncthreads();
  attn_compute<DH, NT>(Ks, Vs, S, C, h, q, idx, q0, nqw, qbase, o, nullptr);
}

void launch_attn_bf16(const Geo& g, int C, int heads, int Spad, const bf16* q, const bf16* k,
                      const bf16* vt, const int32_t* idx, const int32_t* woff, bf16* o, float* amax_o,
                      hipStream_t s) {
  const int dh = C / heads;
  dim3 grid(g.nwin * heads, (g.S + 63) / 64);
  const int nt = Spad / 16;
#define DR_ATTN_CASE(DH_, NT_)                                                          \
  if (dh == DH_ && nt == NT_) {                                                         \
    attn_bf16_kernel<DH_, NT_><<<grid, 256, 0, s>>>(g, C, heads, q, k, vt, idx, woff, o, amax_o); \
    return;                                                                             \
  }
  DR_ATTN_CASE(32, 4)
  DR_ATTN_CASE(64, 4)
  DR_ATTN_CASE(64, 15)
  DR_ATTN_CASE(64, 19)
  DR_ATTN_CASE(32, 15)
  DR_ATTN_CASE(32, 19)
#undef DR_ATTN_CASE
}

void launch_attn_stream(const StreamTable& tab, const Geo& g, int C, int heads, int Spad, const bf16* q,
                        const int32_t* idx, const int32_t* woff, bf16* o, hipStream_t s) {
  const int dh = C / heads;
  dim3 grid(g.nwin * heads, (g.S + 63) / 64);
  const int nt = Spad / 16;
  const int nwin_f = g.nwh * g.nww;
#define DR_ATTN_CASE(DH_, NT_)                                                                      \
  if (dh == DH_ && nt == NT_) {                                                                     \
    attn_stream_kernel<DH_, NT_><<<grid, 256, 0, s>>>(tab, C, heads, g.S, nwin_f, q, idx, woff, o); \
    return;                                                                                         \
  }
  DR_ATTN_CASE(32, 4)
  DR_ATTN_CASE(64, 4)
  DR_ATTN_CASE(64, 15)
  DR_ATTN_CASE(64, 19)
  DR_ATTN_CASE(32, 15)
  DR_ATTN_CASE(32, 19)
#undef DR_ATTN_CASE
}

bool attn_bf16_supported(int dh, int spad) {
  const int nt = spad / 16;
  return (dh == 32 || dh == 64) && (nt == 4 || nt == 15 || nt == 19);
}

// ------------------------------------------------------------------------------------------
__global__ void f32_to_bf16_kernel(const float* __restrict__ a, bf16* __restrict__ b, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    b[i] = f2bf(a[i]);
}

void launch_f32_to_bf16(const float* a, bf16* b, size_t n, hipStream_t s) {
  size_t grid = (n + 255) / 256;
  if (grid > 8192) grid = 8192;
  if (grid) f32_to_bf16_kernel<<<(unsigned)grid, 256, 0, s>>>(a, b, n);
}

}  // namespace dr
