// The plain FP32 path: one simple kernel per operation (LayerNorm, SIMT-tiled GEMM with a
// bias/GELU/residual epilogue, and per-query window attention).  It is the baseline the
// MFMA paths are measured against and the FP32 reference of the library itself.
#include "dr_device.h"
#include "dr_internal.h"

namespace dr {

// ------------------------------------------------------------------------------------------
// LayerNorm over C channels, biased variance, eps = 1e-5; one wavefront per row.
// Input row r is x[rows ? rows[r] : r]; output row r is compact.
// ------------------------------------------------------------------------------------------
template <typename OutT>
__device__ __forceinline__ void store_val(OutT* p, float v);
template <>
__device__ __forceinline__ void store_val<float>(float* p, float v) { *p = v; }
template <>
__device__ __forceinline__ void store_val<bf16>(bf16* p, float v) { *p = f2bf(v); }

template <typename OutT>
__global__ void __launch_bounds__(256) ln_kernel(const float* __restrict__ x, const int32_t* __restrict__ rows,
                                                 const int32_t* __restrict__ nrows_dev, int nrows_max, int C,
                                                 const float* __restrict__ g, const float* __restrict__ b,
                                                 OutT* __restrict__ y) {
  const int lane = threadIdx.x & 63;
  const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int nrows = nrows_dev ? nrows_dev[0] : nrows_max;
  if (r >= nrows) return;
  const int src = rows ? rows[r] : r;
  const float* xr = x + (size_t)src * C;
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
  OutT* yr = y + (size_t)r * C;
  for (int e = 0; e < per; ++e) {
    const int c = lane + 64 * e;
    store_val<OutT>(yr + c, (v[e] - mean) * rstd * g[c] + b[c]);
  }
}

void launch_ln_f32(const float* x, const int32_t* rows, const int32_t* nrows_dev, int nrows_max,
                   int C, const float* g, const float* b, float* y, hipStream_t s) {
  if (nrows_max <= 0) return;
  ln_kernel<float><<<(nrows_max + 3) / 4, 256, 0, s>>>(x, rows, nrows_dev, nrows_max, C, g, b, y);
}


// ------------------------------------------------------------------------------------------
// SIMT GEMM: Y[m, n] = sum_k A[arow(m), k] * W[n, k] + bias[n]; 64x64 tile, BK = 16,
// 256 threads with 4x4 outputs each.
// ------------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) gemm_f32_kernel(const float* __restrict__ A, const int32_t* __restrict__ arows,
                                                       const int32_t* __restrict__ m_dev, int m_max, int K,
                                                       const float* __restrict__ W, const float* __restrict__ bias,
                                                       int Nout, int epi, float* __restrict__ out,
                                                       const int32_t* __restrict__ res_rows) {
  __shared__ float As[16][64 + 4];
  __shared__ float Ws[16][64 + 4];
  const int M = m_dev ? m_dev[0] : m_max;
  const int m0 = blockIdx.x * 64, n0 = blockIdx.y * 64;
  if (m0 >= M) return;
  const int t = threadIdx.x;
  const int lr = t >> 2, lk = (t & 3) * 4;  // loader: row in tile, k offset
  const int am = m0 + lr;
  const bool a_ok = am < M;
  const float* arow = A + (size_t)(a_ok ? (arows ? arows[am] : am) : 0) * K;
  const int wn = n0 + lr;
  const bool w_ok = wn < Nout;
  const float* wrow = W + (size_t)(w_ok ? wn : 0) * K;
  const int ty = t >> 4, tx = t & 15;
  float acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.f;
  for (int k0 = 0; k0 < K; k0 += 16) {
    float4 av = a_ok ? *reinterpret_cast<const float4*>(arow + k0 + lk) : make_float4(0, 0, 0, 0);
    float4 wv = w_ok ? *reinterpret_cast<const float4*>(wrow + k0 + lk) : make_float4(0, 0, 0, 0);
    As[lk + 0][lr] = av.x; As[lk + 1][lr] = av.y; As[lk + 2][lr] = av.z; As[lk + 3][lr] = av.w;
    Ws[lk + 0][lr] = wv.x; Ws[lk + 1][lr] = wv.y; Ws[lk + 2][lr] = wv.z; Ws[lk + 3][lr] = wv.w;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      float a[4], w[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[k][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) w[j] = Ws[k][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(a[i], w[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int m = m0 + ty + 16 * i;
    if (m >= M) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int n = n0 + tx + 16 * j;
      if (n >= Nout) continue;
      const float y = acc[i][j] + bias[n];
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

void launch_gemm_f32(const float* A, const int32_t* arows, const int32_t* m_dev, int m_max, int K,
                     const float* W, const float* bias, int Nout, int epi, float* out,
                     const int32_t* res_rows, hipStream_t s) {
  if (m_max <= 0) return;
  dim3 grid((m_max + 63) / 64, (Nout + 63) / 64);
  gemm_f32_kernel<<<grid, 256, 0, s>>>(A, arows, m_dev, m_max, K, W, bias, Nout, epi, out, res_rows);
}

// ------------------------------------------------------------------------------------------
// Window attention, FP32: one wavefront per (window, head, query).  Scores over all S keys of
// the window, softmax with the row max subtracted, then O = P V.
//   q  : compact query rows [Nq, C]          (row woff[w] + j is window w's j-th query)
//   kv : all tokens [N, 2C] window-major     (K in columns [0, C), V in [C, 2C))
//   o  : compact [Nq, C]
// ------------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) attn_f32_kernel(Geo g, int C, int heads, const float* __restrict__ q,
                                                       const float* __restrict__ kv,
                                                       const int32_t* __restrict__ woff, float* __restrict__ o) {
  __shared__ float qs[4][64];
  __shared__ float ps[4][320];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int w = blockIdx.x / heads, h = blockIdx.x - w * heads;
  const int j = blockIdx.y * 4 + wv;
  const int q0 = woff[w], nqw = woff[w + 1] - q0;
  if (j >= nqw) return;
  const int dh = C / heads;
  const int r = q0 + j;
  const float scale = rsqrtf((float)dh);
  if (lane < dh) qs[wv][lane] = q[(size_t)r * C + h * dh + lane];
  __builtin_amdgcn_wave_barrier();
  const float* kbase = kv + (size_t)w * g.S * 2 * C + h * dh;
  float mx = -INFINITY;
  for (int s = lane; s < g.S; s += 64) {
    const float* kr = kbase + (size_t)s * 2 * C;
    float d = 0.f;
    for (int e = 0; e < dh; ++e) d = fmaf(qs[wv][e], kr[e], d);
    d *= scale;
    ps[wv][s] = d;
    mx = fmaxf(mx, d);
  }
  mx = wave_max(mx);
  float sum = 0.f;
  for (int s = lane; s < g.S; s += 64) {
    const float e = expf(ps[wv][s] - mx);
    ps[wv][s] = e;
    sum += e;
  }
  sum = wave_sum(sum);
  __builtin_amdgcn_wave_barrier();
  if (lane < dh) {
    const float* vbase = kbase + C + lane;
    float acc = 0.f;
    for (int s = 0; s < g.S; ++s) acc = fmaf(ps[wv][s], vbase[(size_t)s * 2 * C], acc);
    o[(size_t)r * C + h * dh + lane] = acc / sum;
  }
}

void launch_attn_f32(const Geo& g, int C, int heads, const float* q, const float* kv,
                     const int32_t* woff, float* o, hipStream_t s) {
  dim3 grid(g.nwin * heads, (g.S + 3) / 4);
  attn_f32_kernel<<<grid, 256, 0, s>>>(g, C, heads, q, kv, woff, o);
}

}  // namespace dr
