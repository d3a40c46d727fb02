// Training kernels (FP32): the pieces of the hand-written reverse pass of the inpainting
// network.  Weight gradients are reductions over tokens; they are computed deterministically
// (fixed chunks of rows, then the chunk partials summed in order), so a gradient does not
// depend on launch timing or on which other clips share the batch.
#include "dr_device.h"
#include "dr_internal.h"

namespace dr {

constexpr int RED_CHUNK = 2048;  // rows per partial of a token reduction

// ------------------------------------------------------------------------------------------
// Y[r, :] = X[rows[r], :] for r < *n (gather of residual rows)
// ------------------------------------------------------------------------------------------
__global__ void gather_rows_kernel(const float* __restrict__ X, const int32_t* __restrict__ rows,
                                   const int32_t* __restrict__ n_dev, int n_max, int C, float* __restrict__ Y) {
  const int n = n_dev ? n_dev[0] : n_max;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < (size_t)n * C; e += (size_t)gridDim.x * blockDim.x) {
    const size_t r = e / C, c = e - r * C;
    Y[e] = X[(size_t)rows[r] * C + c];
  }
}

void launch_gather_rows(const float* X, const int32_t* rows, const int32_t* n_dev, int n_max, int C, float* Y,
                        hipStream_t s) {
  size_t grid = ((size_t)n_max * C + 255) / 256;
  if (grid > 8192) grid = 8192;
  if (grid) gather_rows_kernel<<<(unsigned)grid, 256, 0, s>>>(X, rows, n_dev, n_max, C, Y);
}

// X[rows[r], :] = Y[r, :] (scatter-replace)
__global__ void scatter_rows_kernel(const float* __restrict__ Y, const int32_t* __restrict__ rows,
                                    const int32_t* __restrict__ n_dev, int C, float* __restrict__ X) {
  const int n = n_dev[0];
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < (size_t)n * C; e += (size_t)gridDim.x * blockDim.x) {
    const size_t r = e / C, c = e - r * C;
    X[(size_t)rows[r] * C + c] = Y[e];
  }
}

void launch_scatter_rows(const float* Y, const int32_t* rows, const int32_t* n_dev, int n_max, int C, float* X,
                         hipStream_t s) {
  size_t grid = ((size_t)n_max * C + 255) / 256;
  if (grid > 8192) grid = 8192;
  if (grid) scatter_rows_kernel<<<(unsigned)grid, 256, 0, s>>>(Y, rows, n_dev, C, X);
}

// ------------------------------------------------------------------------------------------
// elementwise: a = GELU(h);  dh = da * GELU'(h),  GELU'(z) = Phi(z) + z phi(z)
// ------------------------------------------------------------------------------------------
__global__ void gelu_fwd_kernel(const float* __restrict__ h, const int32_t* __restrict__ n_dev, int R,
                                float* __restrict__ a) {
  const size_t n = (size_t)n_dev[0] * R;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
    a[e] = gelu_erf(h[e]);
}

__global__ void gelu_bwd_kernel(const float* __restrict__ h, const float* __restrict__ da,
                                const int32_t* __restrict__ n_dev, int R, float* __restrict__ dh) {
  const size_t n = (size_t)n_dev[0] * R;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    const float z = h[e];
    const float cdf = 0.5f * (1.0f + erff(z * 0.70710678118654752f));
    const float pdf = 0.3989422804014327f * expf(-0.5f * z * z);
    dh[e] = da[e] * (cdf + z * pdf);
  }
}

void launch_gelu_fwd(const float* h, const int32_t* n_dev, int n_max, int R, float* a, hipStream_t s) {
  size_t grid = ((size_t)n_max * R + 255) / 256;
  if (grid > 8192) grid = 8192;
  if (grid) gelu_fwd_kernel<<<(unsigned)grid, 256, 0, s>>>(h, n_dev, R, a);
}

void launch_gelu_bwd(const float* h, const float* da, const int32_t* n_dev, int n_max, int R, float* dh,
                     hipStream_t s) {
  size_t grid = ((size_t)n_max * R + 255) / 256;
  if (grid > 8192) grid = 8192;
  if (grid) gelu_bwd_kernel<<<(unsigned)grid, 256, 0, s>>>(h, da, n_dev, R, dh);
}

// ------------------------------------------------------------------------------------------
// LayerNorm backward, one wavefront per row r < *n (or n_max): rows of x at rows[r] (or r);
// dx[r] = rstd * (dxh - mean(dxh) - xh * mean(dxh * xh)), dxh = dy * gamma, written or added
// (accumulate) at dst row (rows ? rows[r] : r) or compact r (dst_compact).  dgamma/dbeta
// partials per block of 64 rows: part[blk][0..C) = sum dy*xh, part[blk][C..2C) = sum dy.
// ------------------------------------------------------------------------------------------
constexpr int LNB_ROWS = 64;

__global__ void __launch_bounds__(256) ln_bwd_kernel(const float* __restrict__ x, const int32_t* __restrict__ rows,
                                                     const int32_t* __restrict__ n_dev, int n_max, int C,
                                                     const float* __restrict__ g, const float* __restrict__ dy,
                                                     float* __restrict__ dx, int accumulate, int dst_compact,
                                                     float* __restrict__ part) {
  extern __shared__ float red[];  // [4][2C]
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int n = n_dev ? n_dev[0] : n_max;
  const int per = C / 64;
  float pg[16], pb[16];
  for (int e = 0; e < per; ++e) pg[e] = pb[e] = 0.f;
  for (int rr = 0; rr < LNB_ROWS / 4; ++rr) {
    const int r = blockIdx.x * LNB_ROWS + rr * 4 + wv;
    if (r >= n) break;
    const size_t src = rows ? (size_t)rows[r] : (size_t)r;
    const float* xr = x + src * C;
    const float* dyr = dy + (size_t)r * C;
    float v[16], d[16];
    float s = 0.f;
    for (int e = 0; e < per; ++e) {
      v[e] = xr[lane + 64 * e];
      s += v[e];
    }
    const float mean = wave_sum(s) / C;
    float q = 0.f;
    for (int e = 0; e < per; ++e) {
      const float t = v[e] - mean;
      q += t * t;
    }
    const float rstd = rsqrtf(wave_sum(q) / C + 1e-5f);
    float s1 = 0.f, s2 = 0.f;
    for (int e = 0; e < per; ++e) {
      const int c = lane + 64 * e;
      const float xh = (v[e] - mean) * rstd;
      const float dyv = dyr[c];
      d[e] = dyv * g[c];
      s1 += d[e];
      s2 += d[e] * xh;
      pg[e] += dyv * xh;
      pb[e] += dyv;
      v[e] = xh;
    }
    s1 = wave_sum(s1) / C;
    s2 = wave_sum(s2) / C;
    float* out = dx + (dst_compact ? (size_t)r : src) * C;
    for (int e = 0; e < per; ++e) {
      const int c = lane + 64 * e;
      const float val = rstd * (d[e] - s1 - v[e] * s2);
      out[c] = accumulate ? out[c] + val : val;
    }
  }
  // fixed-order block reduction of the dgamma / dbeta partials
  for (int e = 0; e < per; ++e) {
    red[wv * 2 * C + lane + 64 * e] = pg[e];
    red[wv * 2 * C + C + lane + 64 * e] = pb[e];
  }
  __syncthreads();
  for (int c = threadIdx.x; c < 2 * C; c += blockDim.x)
    part[(size_t)blockIdx.x * 2 * C + c] = red[c] + red[2 * C + c] + red[4 * C + c] + red[6 * C + c];
}

void launch_ln_bwd(const float* x, const int32_t* rows, const int32_t* n_dev, int n_max, int C, const float* g,
                   const float* dy, float* dx, int accumulate, int dst_compact, float* part, hipStream_t s) {
  const int blocks = (n_max + LNB_ROWS - 1) / LNB_ROWS;
  if (blocks <= 0) return;
  ln_bwd_kernel<<<blocks, 256, 4 * 2 * C * sizeof(float), s>>>(x, rows, n_dev, n_max, C, g, dy, dx, accumulate,
                                                              dst_compact, part);
}

int ln_bwd_blocks(int n_max) { return (n_max + LNB_ROWS - 1) / LNB_ROWS; }

// out[c] (+)= sum over b < nparts of part[b][c] (in order)
__global__ void sum_parts_kernel(const float* __restrict__ part, int nparts, int width, float* __restrict__ out,
                                 int accumulate) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= width) return;
  // four interleaved partial sums (loads in flight together), combined in a fixed order
  float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
  int b = 0;
  for (; b + 3 < nparts; b += 4) {
    a0 += part[(size_t)b * width + c];
    a1 += part[(size_t)(b + 1) * width + c];
    a2 += part[(size_t)(b + 2) * width + c];
    a3 += part[(size_t)(b + 3) * width + c];
  }
  for (; b < nparts; ++b) a0 += part[(size_t)b * width + c];
  const float acc = (a0 + a1) + (a2 + a3);
  out[c] = accumulate ? out[c] + acc : acc;
}

void launch_sum_parts(const float* part, int nparts, int width, float* out, int accumulate, hipStream_t s) {
  if (width <= 0) return;
  sum_parts_kernel<<<(width + 255) / 256, 256, 0, s>>>(part, nparts, width, out, accumulate);
}

// ------------------------------------------------------------------------------------------
// Token reductions.  TN product: out[i][j] = sum_m A[arow(m)][i] * B[brow(m)][j], m < *M (or
// M_max), A row stride lda, B row stride ldb, i < I, j < J.  Partials per chunk of RED_CHUNK
// rows: part[chunk][i][j]; a 64 x 64 output tile per block, 4 x 4 per thread.
// Column sums: out[j] = sum_m B[m][j] (same chunking).
// ------------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) tn_partial_kernel(const float* __restrict__ A, const int32_t* __restrict__ arow,
                                                         int lda, const float* __restrict__ B,
                                                         const int32_t* __restrict__ brow, int ldb,
                                                         const int32_t* __restrict__ M_dev, int M_max, int I, int J,
                                                         float* __restrict__ part) {
  __shared__ float As[16][64];
  __shared__ float Bs[16][64];
  const int M = M_dev ? M_dev[0] : M_max;
  const int i0 = blockIdx.x * 64, j0 = blockIdx.y * 64, chunk = blockIdx.z;
  const int m_begin = chunk * RED_CHUNK;
  const int m_end = min(M, m_begin + RED_CHUNK);
  const int t = threadIdx.x, ty = t >> 4, tx = t & 15;
  float acc[4][4] = {};
  for (int m0 = m_begin; m0 < m_end; m0 += 16) {
    // 16 rows x 64 columns of A and of B: 1024 values each, 4 per thread
    for (int e = t; e < 1024; e += 256) {
      const int rr = e >> 6, cc = e & 63;
      const int m = m0 + rr;
      float av = 0.f, bv = 0.f;
      if (m < m_end) {
        const size_t ra = arow ? (size_t)arow[m] : (size_t)m;
        const size_t rb = brow ? (size_t)brow[m] : (size_t)m;
        if (i0 + cc < I) av = A[ra * lda + i0 + cc];
        if (j0 + cc < J) bv = B[rb * ldb + j0 + cc];
      }
      As[rr][cc] = av;
      Bs[rr][cc] = bv;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      float a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = As[k][ty + 16 * u];
        b[u] = Bs[k][tx + 16 * u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = fmaf(a[u], b[v], acc[u][v]);
    }
    __syncthreads();
  }
  float* P = part + (size_t)chunk * I * J;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int i = i0 + ty + 16 * u;
    if (i >= I) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int j = j0 + tx + 16 * v;
      if (j < J) P[(size_t)i * J + j] = acc[u][v];
    }
  }
}

// ------------------------------------------------------------------------------------------
// BF16-operand products for mixed-precision training: FP32 master weights, activations and
// gradients; every operand is rounded to bf16 (round to nearest even) as it is loaded, and
// the products accumulate in FP32 on MFMA 16x16x32.  A 64 x 64 output tile per block of four
// wavefronts, each wavefront 2 x 2 fragments of 16 x 16.
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ void tr_mfma_fence() {
  __builtin_amdgcn_sched_barrier(0);
  asm volatile("s_nop 7" ::: "memory");
  __builtin_amdgcn_sched_barrier(0);
}

// 8 consecutive FP32 values (32-byte aligned) as bf16, or zeros
__device__ __forceinline__ bf16x8_t tr_load8(const float* p, bool ok) {
  bf16x8_t r;
  if (ok) {
    const float4 a = *reinterpret_cast<const float4*>(p), b = *reinterpret_cast<const float4*>(p + 4);
    r[0] = (__bf16)a.x; r[1] = (__bf16)a.y; r[2] = (__bf16)a.z; r[3] = (__bf16)a.w;
    r[4] = (__bf16)b.x; r[5] = (__bf16)b.y; r[6] = (__bf16)b.z; r[7] = (__bf16)b.w;
  } else {
#pragma unroll
    for (int e = 0; e < 8; ++e) r[e] = (__bf16)0.f;
  }
  return r;
}

// Y[m, n] = sum_k A[arow(m), k] W[n, k] + bias[n] with the epilogues of the FP32 GEMM
// (store, exact GELU, or add into out[res_rows(m)]); K % 8 == 0, a k chunk past K reads zeros.
// Per 32-wide k step the block loads the 64 rows of A and of W once (two 16-byte loads per
// thread each), rounds them to bf16 into LDS (rows padded to 40), and each wavefront reads
// its operand fragments from there.
constexpr int GB_LD = 40;
__global__ void __launch_bounds__(256) gemm_bf16ops_kernel(const float* __restrict__ A, const int32_t* __restrict__ arows,
                                                           const int32_t* __restrict__ m_dev, int m_max, int K,
                                                           const float* __restrict__ W, const float* __restrict__ bias,
                                                           int Nout, int epi, float* __restrict__ out,
                                                           const int32_t* __restrict__ res_rows) {
  __shared__ __align__(16) __bf16 As[64][GB_LD];
  __shared__ __align__(16) __bf16 Ws[64][GB_LD];
  const int M = m_dev ? m_dev[0] : m_max;
  const int m0 = blockIdx.x * 64, n0 = blockIdx.y * 64;
  if (m0 >= M) return;  // uniform per block
  const int t = threadIdx.x;
  const int lane = t & 63, wv = t >> 6;
  const int l16 = lane & 15, kg = lane >> 4;
  const int wm = wv >> 1, wn = wv & 1;
  // loader: row lr of the tile, k columns lk .. lk + 7 of the step
  const int lr = t >> 2, lk = (t & 3) * 8;
  const int am = m0 + lr, wnr = n0 + lr;
  const bool aok = am < M, wok = wnr < Nout;
  const float* arow = A + (size_t)(aok ? (arows ? arows[am] : am) : 0) * K;
  const float* wrow = W + (size_t)(wok ? wnr : 0) * K;
  f32x4_t acc[2][2];
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int i = 0; i < 2; ++i) acc[j][i] = f32x4_t{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += 32) {
    const int k = k0 + lk;
    *reinterpret_cast<bf16x8_t*>(&As[lr][lk]) = tr_load8(arow + k, aok && k < K);
    *reinterpret_cast<bf16x8_t*>(&Ws[lr][lk]) = tr_load8(wrow + k, wok && k < K);
    __syncthreads();
    bf16x8_t a[2], w[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) a[i] = *reinterpret_cast<const bf16x8_t*>(&As[32 * wm + 16 * i + l16][8 * kg]);
#pragma unroll
    for (int j = 0; j < 2; ++j) w[j] = *reinterpret_cast<const bf16x8_t*>(&Ws[32 * wn + 16 * j + l16][8 * kg]);
    __syncthreads();
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int i = 0; i < 2; ++i) acc[j][i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w[j], a[i], acc[j][i], 0, 0, 0);
    tr_mfma_fence();
  }
  // lane holds Y[m = .. + l16][n = .. + 4 kg + e]
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int m = m0 + 32 * wm + 16 * i + l16;
    if (m >= M) continue;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int n = n0 + 32 * wn + 16 * j + 4 * kg + e;
        if (n >= Nout) continue;
        const float y = acc[j][i][e] + bias[n];
        if (epi == EPI_STORE) {
          out[(size_t)m * Nout + n] = y;
        } else if (epi == EPI_GELU) {
          out[(size_t)m * Nout + n] = gelu_erf(y);
        } else {
          const int dst = res_rows ? res_rows[m] : m;
          out[(size_t)dst * Nout + n] += y;
        }
      }
    }
  }
}

void launch_gemm_bf16ops(const float* A, const int32_t* arows, const int32_t* m_dev, int m_max, int K,
                         const float* W, const float* bias, int Nout, int epi, float* out,
                         const int32_t* res_rows, hipStream_t s) {
  if (m_max <= 0) return;
  dim3 grid((m_max + 63) / 64, (Nout + 63) / 64);
  gemm_bf16ops_kernel<<<grid, 256, 0, s>>>(A, arows, m_dev, m_max, K, W, bias, Nout, epi, out, res_rows);
}

// TN partials with bf16 operands: part[chunk][i][j] = sum over the chunk's rows m of
// A[arow(m)][i] B[brow(m)][j] (the same partial layout as tn_partial_kernel).  A 64 x 64
// output tile per block of four wavefronts (32 x 32 each).  Per step of 32 rows, the block
// loads the rows' 64 columns of A and of B with 16-byte loads, rounds them to bf16 and stores
// them transposed in LDS ([column][row], rows padded to 40), so that each lane's operand --
// 8 consecutive rows of one column -- is one 16-byte LDS read.
constexpr int TN_T = 64, TN_LD = 40;
__global__ void __launch_bounds__(256) tn_bf16ops_kernel(const float* __restrict__ A, const int32_t* __restrict__ arow,
                                                         int lda, const float* __restrict__ B,
                                                         const int32_t* __restrict__ brow, int ldb,
                                                         const int32_t* __restrict__ M_dev, int M_max, int I, int J,
                                                         float* __restrict__ part) {
  __shared__ __align__(16) __bf16 As[TN_T][TN_LD];
  __shared__ __align__(16) __bf16 Bs[TN_T][TN_LD];
  const int M = M_dev ? M_dev[0] : M_max;
  const int i0 = blockIdx.x * TN_T, j0 = blockIdx.y * TN_T, chunk = blockIdx.z;
  const int m_begin = chunk * RED_CHUNK;
  const int m_end = min(M, m_begin + RED_CHUNK);
  const int t = threadIdx.x;
  const int lane = t & 63, wv = t >> 6;
  const int l16 = lane & 15, kg = lane >> 4;
  const int wi = wv >> 1, wj = wv & 1;
  const int lr = t >> 3, lc = (t & 7) * 8;  // loader: row of the step, first of 8 columns
  f32x4_t acc[2][2];
#pragma unroll
  for (int fj = 0; fj < 2; ++fj)
#pragma unroll
    for (int fi = 0; fi < 2; ++fi) acc[fj][fi] = f32x4_t{0.f, 0.f, 0.f, 0.f};
  for (int m0 = m_begin; m0 < m_end; m0 += 32) {
    const int m = m0 + lr;
    float va[8], vb[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) va[e] = vb[e] = 0.f;
    if (m < m_end) {
      const float* pa = A + (arow ? (size_t)arow[m] : (size_t)m) * lda + i0 + lc;
      const float* pb = B + (brow ? (size_t)brow[m] : (size_t)m) * ldb + j0 + lc;
      if (i0 + lc + 8 <= I && ((reinterpret_cast<uintptr_t>(pa) & 15) == 0)) {
        const float4 a0 = *reinterpret_cast<const float4*>(pa), a1 = *reinterpret_cast<const float4*>(pa + 4);
        va[0] = a0.x; va[1] = a0.y; va[2] = a0.z; va[3] = a0.w; va[4] = a1.x; va[5] = a1.y; va[6] = a1.z; va[7] = a1.w;
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) va[e] = i0 + lc + e < I ? pa[e] : 0.f;
      }
      if (j0 + lc + 8 <= J && ((reinterpret_cast<uintptr_t>(pb) & 15) == 0)) {
        const float4 b0 = *reinterpret_cast<const float4*>(pb), b1 = *reinterpret_cast<const float4*>(pb + 4);
        vb[0] = b0.x; vb[1] = b0.y; vb[2] = b0.z; vb[3] = b0.w; vb[4] = b1.x; vb[5] = b1.y; vb[6] = b1.z; vb[7] = b1.w;
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) vb[e] = j0 + lc + e < J ? pb[e] : 0.f;
      }
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      As[lc + e][lr] = (__bf16)va[e];
      Bs[lc + e][lr] = (__bf16)vb[e];
    }
    __syncthreads();
    bf16x8_t x[2], y[2];
#pragma unroll
    for (int fi = 0; fi < 2; ++fi) x[fi] = *reinterpret_cast<const bf16x8_t*>(&As[32 * wi + 16 * fi + l16][8 * kg]);
#pragma unroll
    for (int fj = 0; fj < 2; ++fj) y[fj] = *reinterpret_cast<const bf16x8_t*>(&Bs[32 * wj + 16 * fj + l16][8 * kg]);
    __syncthreads();
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int fj = 0; fj < 2; ++fj)
#pragma unroll
      for (int fi = 0; fi < 2; ++fi) acc[fj][fi] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(y[fj], x[fi], acc[fj][fi], 0, 0, 0);
    tr_mfma_fence();
  }
  // lane holds D[j = .. + 4 kg + e][i = .. + l16]
  float* P = part + (size_t)chunk * I * J;
#pragma unroll
  for (int fi = 0; fi < 2; ++fi) {
    const int i = i0 + 32 * wi + 16 * fi + l16;
    if (i >= I) continue;
#pragma unroll
    for (int fj = 0; fj < 2; ++fj)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int j = j0 + 32 * wj + 16 * fj + 4 * kg + e;
        if (j < J) P[(size_t)i * J + j] = acc[fj][fi][e];
      }
  }
}

void launch_tn_bf16ops(const float* A, const int32_t* arow, int lda, const float* B, const int32_t* brow, int ldb,
                       const int32_t* M_dev, int M_max, int I, int J, float* part, hipStream_t s) {
  const int chunks = (M_max + RED_CHUNK - 1) / RED_CHUNK;
  if (chunks <= 0) return;
  dim3 grid((I + TN_T - 1) / TN_T, (J + TN_T - 1) / TN_T, chunks);
  tn_bf16ops_kernel<<<grid, 256, 0, s>>>(A, arow, lda, B, brow, ldb, M_dev, M_max, I, J, part);
}

int tn_chunks(int M_max) { return (M_max + RED_CHUNK - 1) / RED_CHUNK; }

void launch_tn_partial(const float* A, const int32_t* arow, int lda, const float* B, const int32_t* brow, int ldb,
                       const int32_t* M_dev, int M_max, int I, int J, float* part, hipStream_t s) {
  const int chunks = tn_chunks(M_max);
  if (chunks <= 0) return;
  dim3 grid((I + 63) / 64, (J + 63) / 64, chunks);
  tn_partial_kernel<<<grid, 256, 0, s>>>(A, arow, lda, B, brow, ldb, M_dev, M_max, I, J, part);
}

// One block per (64 columns, chunk): 16 row groups of 64 lanes, each lane summing every 16th
// row of its column with 8 independent partial sums (loads in flight together), then a fixed
// order reduction of the groups in LDS (deterministic).
__global__ void __launch_bounds__(1024) colsum_partial_kernel(const float* __restrict__ B, int ldb,
                                                              const int32_t* __restrict__ M_dev, int M_max, int J,
                                                              float* __restrict__ part) {
  __shared__ float red[16][64];
  const int M = M_dev ? M_dev[0] : M_max;
  const int col = threadIdx.x & 63, grp = threadIdx.x >> 6;
  const int j = blockIdx.x * 64 + col;
  const int chunk = blockIdx.y;
  const int m_begin = chunk * RED_CHUNK, m_end = min(M, m_begin + RED_CHUNK);
  float acc[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) acc[u] = 0.f;
  if (j < J) {
    int m = m_begin + grp;
    for (; m + 7 * 16 < m_end; m += 8 * 16)
#pragma unroll
      for (int u = 0; u < 8; ++u) acc[u] += B[(size_t)(m + 16 * u) * ldb + j];
    for (; m < m_end; m += 16) acc[0] += B[(size_t)m * ldb + j];
  }
  red[grp][col] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  __syncthreads();
  if (grp == 0 && j < J) {
    float t = 0.f;
    for (int g = 0; g < 16; ++g) t += red[g][col];
    part[(size_t)chunk * J + j] = t;
  }
}

void launch_colsum_partial(const float* B, int ldb, const int32_t* M_dev, int M_max, int J, float* part,
                           hipStream_t s) {
  const int chunks = tn_chunks(M_max);
  if (chunks <= 0) return;
  colsum_partial_kernel<<<dim3((J + 63) / 64, chunks), 1024, 0, s>>>(B, ldb, M_dev, M_max, J, part);
}

// ------------------------------------------------------------------------------------------
// Pixel-side pieces.  Patches of the cut-out input [N][48] (k = (ky*4 + kx)*3 + c), and the
// decoder's pre-activation gradient per token: dyt[n][k] = dpred * pred * (1 - pred) at the
// token's pixels.  Also the full-frame decoder (all tokens) for the training forward:
// pred = sigmoid(z W_dec + b) written to every pixel.
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ size_t tok_pixel(const Geo& g, int n) {
  int w = n / g.S, s = n - w * g.S;
  int v = w % g.nww;
  int r = w / g.nww;
  int u = r % g.nwh;
  r /= g.nwh;
  int nT = g.T / g.wt;
  int a = r % nT;
  int b = r / nT;
  int dj = s % g.ww;
  int q = s / g.ww;
  int di = q % g.wh;
  int dt = q / g.wh;
  int t = a * g.wt + dt, i = u * g.wh + di, j = v * g.ww + dj;
  return (((size_t)b * g.T + t) * g.H + (size_t)4 * i) * g.W + (size_t)4 * j;
}

__global__ void patches_kernel(Geo g, const float* __restrict__ frames, const uint8_t* __restrict__ masks,
                               float* __restrict__ P) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < (size_t)g.N * 48; e += (size_t)gridDim.x * blockDim.x) {
    const int n = (int)(e / 48), k = (int)(e % 48);
    const int pix = k / 3, c = k - 3 * pix, ky = pix >> 2, kx = pix & 3;
    const size_t px = tok_pixel(g, n) + (size_t)ky * g.W + kx;
    P[e] = masks[px] ? 0.f : frames[px * 3 + c];
  }
}

void launch_patches(const Geo& g, const float* frames, const uint8_t* masks, float* P, hipStream_t s) {
  size_t grid = ((size_t)g.N * 48 + 255) / 256;
  if (grid > 8192) grid = 8192;
  patches_kernel<<<(unsigned)grid, 256, 0, s>>>(g, frames, masks, P);
}

__global__ void decoder_full_kernel(Geo g, int C, const float* __restrict__ z, const float* __restrict__ dw,
                                    const float* __restrict__ db, float* __restrict__ pred) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < (size_t)g.N * 48; e += (size_t)gridDim.x * blockDim.x) {
    const int n = (int)(e / 48), k = (int)(e % 48);
    const int pix = k / 3, c = k - 3 * pix, ky = pix >> 2, kx = pix & 3;
    const float* zr = z + (size_t)n * C;
    float acc = db[c];
    for (int i = 0; i < C; ++i) acc = fmaf(zr[i], dw[i * 48 + k], acc);
    const size_t px = tok_pixel(g, n) + (size_t)ky * g.W + kx;
    pred[px * 3 + c] = 1.0f / (1.0f + expf(-acc));
  }
}

void launch_decoder_full(const Geo& g, int C, const float* z, const float* dw, const float* db, float* pred,
                         hipStream_t s) {
  size_t grid = ((size_t)g.N * 48 + 255) / 256;
  if (grid > 16384) grid = 16384;
  decoder_full_kernel<<<(unsigned)grid, 256, 0, s>>>(g, C, z, dw, db, pred);
}

__global__ void dec_grad_tok_kernel(Geo g, const float* __restrict__ pred, const float* __restrict__ dpred,
                                    float* __restrict__ dyt) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < (size_t)g.N * 48; e += (size_t)gridDim.x * blockDim.x) {
    const int n = (int)(e / 48), k = (int)(e % 48);
    const int pix = k / 3, c = k - 3 * pix, ky = pix >> 2, kx = pix & 3;
    const size_t i = (tok_pixel(g, n) + (size_t)ky * g.W + kx) * 3 + c;
    const float p = pred[i];
    dyt[e] = dpred[i] * p * (1.0f - p);
  }
}

void launch_dec_grad_tok(const Geo& g, const float* pred, const float* dpred, float* dyt, hipStream_t s) {
  size_t grid = ((size_t)g.N * 48 + 255) / 256;
  if (grid > 8192) grid = 8192;
  dec_grad_tok_kernel<<<(unsigned)grid, 256, 0, s>>>(g, pred, dpred, dyt);
}

// ------------------------------------------------------------------------------------------
// L1 training loss: L = w_in mean_{m!=0}|pred - gt| + w_out mean_{m==0}|pred - gt| over
// pixel-channel values, and dL/dpred = w * sign(pred - gt) / count (sign(0) = 0; an empty
// region contributes nothing).  Two passes: counts and partial sums per block (fixed order),
// then the gradient.  acc[0..3] = (sum_in, sum_out, n_in, n_out) after the reduction.
// ------------------------------------------------------------------------------------------
constexpr int L1_BLOCKS = 1024;

__global__ void l1_partial_kernel(const float* __restrict__ pred, const float* __restrict__ gt,
                                  const uint8_t* __restrict__ masks, size_t npix, float* __restrict__ part) {
  __shared__ float sh[4][256];
  float si = 0.f, so = 0.f, ni = 0.f, no = 0.f;
  for (size_t p = blockIdx.x * (size_t)blockDim.x + threadIdx.x; p < npix; p += (size_t)gridDim.x * blockDim.x) {
    const bool in = masks[p] != 0;
    float e = 0.f;
    for (int c = 0; c < 3; ++c) e += fabsf(pred[3 * p + c] - gt[3 * p + c]);
    if (in) {
      si += e;
      ni += 3.f;
    } else {
      so += e;
      no += 3.f;
    }
  }
  sh[0][threadIdx.x] = si;
  sh[1][threadIdx.x] = so;
  sh[2][threadIdx.x] = ni;
  sh[3][threadIdx.x] = no;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st)
      for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x < 4) part[blockIdx.x * 4 + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ void l1_final_kernel(const float* __restrict__ part, int nb, float w_in, float w_out,
                                float* __restrict__ acc, float* __restrict__ loss) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s[4] = {0, 0, 0, 0};
  for (int b = 0; b < nb; ++b)
    for (int k = 0; k < 4; ++k) s[k] += part[b * 4 + k];
  for (int k = 0; k < 4; ++k) acc[k] = (float)s[k];
  double L = 0.0;
  if (s[2] > 0) L += w_in * s[0] / s[2];
  if (s[3] > 0) L += w_out * s[1] / s[3];
  loss[0] = (float)L;
}

__global__ void l1_grad_kernel(const float* __restrict__ pred, const float* __restrict__ gt,
                               const uint8_t* __restrict__ masks, size_t npix, float w_in, float w_out,
                               const float* __restrict__ acc, float* __restrict__ dpred) {
  const float gi = acc[2] > 0.f ? w_in / acc[2] : 0.f;
  const float go = acc[3] > 0.f ? w_out / acc[3] : 0.f;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < 3 * npix; e += (size_t)gridDim.x * blockDim.x) {
    const float d = pred[e] - gt[e];
    const float sg = d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f);
    dpred[e] = sg * (masks[e / 3] ? gi : go);
  }
}

void launch_l1_loss(const float* pred, const float* gt, const uint8_t* masks, size_t npix, float w_in, float w_out,
                    float* part, float* acc, float* loss, float* dpred, hipStream_t s) {
  l1_partial_kernel<<<L1_BLOCKS, 256, 0, s>>>(pred, gt, masks, npix, part);
  l1_final_kernel<<<1, 64, 0, s>>>(part, L1_BLOCKS, w_in, w_out, acc, loss);
  if (dpred) {
    size_t grid = (3 * npix + 255) / 256;
    if (grid > 8192) grid = 8192;
    l1_grad_kernel<<<(unsigned)grid, 256, 0, s>>>(pred, gt, masks, npix, w_in, w_out, acc, dpred);
  }
}

}  // namespace dr
