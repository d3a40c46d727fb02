// Pixel-side steps of the path: cut-out + patch embedding (first step after the token
// gather), and final LayerNorm + transposed-conv decoder + sigmoid + composite (last step).
//
// The network input is the frame with private pixels set to 0 (thesis, Methods,
// "Inpainting Manager"); the output keeps every non-private pixel of the input and takes
// generated content only inside the mask.  Both steps are FP32 in every precision mode:
// together they are well under 1 % of the path's arithmetic.
#include "dr_device.h"
#include "dr_internal.h"
#include "gemm_core.h"
#include "tokens_dev.h"

namespace dr {

__device__ __forceinline__ void token_coords(const Geo& g, int n, int& b, int& t, int& i, int& j) {
  int w = n / g.S, s = n - w * g.S;
  int v = w % g.nww;
  int r = w / g.nww;
  int u = r % g.nwh;
  r /= g.nwh;
  int nT = g.T / g.wt;
  int a = r % nT;
  b = r / nT;
  int dj = s % g.ww;
  int q = s / g.ww;
  int di = q % g.wh;
  int dt = q / g.wh;
  t = a * g.wt + dt;
  i = u * g.wh + di;
  j = v * g.ww + dj;
}

// ------------------------------------------------------------------------------------------
// Cut-out + patch embedding: x[n, o] = b[o] + sum_k wT[k, o] * patch_n[k],
// k = (ky*4 + kx)*3 + c, patch value = 0 where the mask is set.  Block = C threads, 64
// tokens per block; thread o keeps its 48 weights in registers.
// ------------------------------------------------------------------------------------------
constexpr int EMB_TOK = 64;

__global__ void embed_kernel(Geo g, int C, const float* __restrict__ frames,
                             const uint8_t* __restrict__ masks, const float* __restrict__ wT,
                             const float* __restrict__ bias, float* __restrict__ x) {
  __shared__ float P[EMB_TOK][48];
  const int n0 = blockIdx.x * EMB_TOK;
  for (int seg = threadIdx.x; seg < EMB_TOK * 4; seg += blockDim.x) {
    const int tok = seg >> 2, ky = seg & 3;
    const int n = n0 + tok;
    float vals[12];
    if (n < g.N) {
      int b, t, i, j;
      token_coords(g, n, b, t, i, j);
      const size_t px = (((size_t)b * g.T + t) * g.H + 4 * i + ky) * g.W + 4 * j;
      const float4* src = reinterpret_cast<const float4*>(frames + px * 3);
      const float4 f0 = src[0], f1 = src[1], f2 = src[2];
      const uint32_t m = *reinterpret_cast<const uint32_t*>(masks + px);
      vals[0] = f0.x; vals[1] = f0.y; vals[2] = f0.z; vals[3] = f0.w;
      vals[4] = f1.x; vals[5] = f1.y; vals[6] = f1.z; vals[7] = f1.w;
      vals[8] = f2.x; vals[9] = f2.y; vals[10] = f2.z; vals[11] = f2.w;
#pragma unroll
      for (int kx = 0; kx < 4; ++kx) {
        if ((m >> (8 * kx)) & 0xffu) {
          vals[kx * 3 + 0] = 0.f;
          vals[kx * 3 + 1] = 0.f;
          vals[kx * 3 + 2] = 0.f;
        }
      }
    } else {
#pragma unroll
      for (int k = 0; k < 12; ++k) vals[k] = 0.f;
    }
#pragma unroll
    for (int k = 0; k < 12; ++k) P[tok][ky * 12 + k] = vals[k];
  }
  __syncthreads();
  for (int o = threadIdx.x; o < C; o += blockDim.x) {
    float w[48];
#pragma unroll
    for (int k = 0; k < 48; ++k) w[k] = wT[k * C + o];
    const float bo = bias[o];
    const int ntok = min(EMB_TOK, g.N - n0);
    for (int tok = 0; tok < ntok; ++tok) {
      float acc = bo;
#pragma unroll
      for (int k = 0; k < 48; ++k) acc = fmaf(P[tok][k], w[k], acc);
      x[(size_t)(n0 + tok) * C + o] = acc;
    }
  }
}

void launch_embed(const Geo& g, int C, const float* frames, const uint8_t* masks, const float* wT,
                  const float* b, float* x, hipStream_t s) {
  const int blocks = (g.N + EMB_TOK - 1) / EMB_TOK;
  const int threads = C < 256 ? C : 256;
  embed_kernel<<<blocks, threads, 0, s>>>(g, C, frames, masks, wT, b, x);
}

// ------------------------------------------------------------------------------------------
// Final LayerNorm + decoder + sigmoid, then the masked pixels of each flagged token are
// written.  One wavefront per flagged token; the decoder matrix [C][48] lives in LDS.
// ------------------------------------------------------------------------------------------
constexpr int DEC_GRID = 1024;

__global__ void __launch_bounds__(256) decode_kernel(Geo g, int C, const float* __restrict__ x,
                                                     const int32_t* __restrict__ idx,
                                                     const int32_t* __restrict__ nq,
                                                     const float* __restrict__ lng,
                                                     const float* __restrict__ lnb,
                                                     const float* __restrict__ dw,
                                                     const float* __restrict__ db,
                                                     const uint8_t* __restrict__ masks,
                                                     float* __restrict__ out) {
  extern __shared__ float sm[];
  float* Wd = sm;                      // [C][48]
  float* Z = sm + (size_t)C * 48;      // [4][C]
  for (int e = threadIdx.x; e < C * 48; e += blockDim.x) Wd[e] = dw[e];
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  float* z = Z + wv * C;
  const int total = nq[0];
  const int per = C / 64;
  for (int r = blockIdx.x * 4 + wv; r < total; r += gridDim.x * 4) {
    const int n = idx[r];
    const float* xr = x + (size_t)n * C;
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
      z[c] = (v[e] - mean) * rstd * lng[c] + lnb[c];
    }
    __builtin_amdgcn_wave_barrier();
    if (lane < 48) {
      float acc = db[lane % 3];
      for (int c = 0; c < C; ++c) acc = fmaf(z[c], Wd[c * 48 + lane], acc);
      const float pred = 1.0f / (1.0f + expf(-acc));
      int b, t, i, j;
      token_coords(g, n, b, t, i, j);
      const int pix = lane / 3, ch = lane - 3 * pix;
      const int ky = pix >> 2, kx = pix & 3;
      const size_t px = (((size_t)b * g.T + t) * g.H + 4 * i + ky) * g.W + 4 * j + kx;
      if (masks[px]) out[px * 3 + ch] = pred;
    }
    __builtin_amdgcn_wave_barrier();
  }
}

void launch_decode(const Geo& g, int C, const float* x, const int32_t* idx, const int32_t* nq,
                   const float* lng, const float* lnb, const float* dw, const float* db,
                   const uint8_t* masks, float* out, hipStream_t s) {
  const size_t smem = (size_t)C * 48 * sizeof(float) + 4 * (size_t)C * sizeof(float);
  int grid = (g.N + 3) / 4;
  if (grid > DEC_GRID) grid = DEC_GRID;
  static size_t granted = 0;
  if (smem > 65536 && smem > granted) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(decode_kernel),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    granted = smem;
  }
  decode_kernel<<<grid, 256, smem, s>>>(g, C, x, idx, nq, lng, lnb, dw, db, masks, out);
}

// ------------------------------------------------------------------------------------------
// BF16 mode: patch embedding and decoder on MFMA (v_mfma_f32_16x16x32_bf16, FP32
// accumulation).  Each wavefront handles 16 tokens; lane l works on token l % 16 and k chunk
// l / 16 of each 32-wide k slice (the operand layout of the GEMM core), so a wavefront holds
// every channel of its tokens and the row statistics need no block-level exchange.
// ------------------------------------------------------------------------------------------

// x = patch W_e^T + b_e (FP32 residual) and x^ = normalise(x) (bf16).  Lane (token l16, row
// group kg) loads patch row ky = kg of its token: 4 pixels x 3 channels (three 16-byte loads)
// and the row's 4 mask bytes, cut out.  The 48 patch values enter the two 32-wide k slices in
// a permuted order -- slice 0: values 12 kg .. 12 kg + 7, slice 1: 12 kg + 8 .. 12 kg + 11 and
// four zeros -- and wT16 [C][64] holds the embedding weight in that same order, so each
// lane's MFMA operands come straight from its own loads.
// Only what later steps read is stored: x^ of tokens in windows with queries (of every token
// when wcount is null: stream mode keeps K/V of all tokens), x of flagged tokens.
// The kernel is a chain of memory round trips, so every load a token needs (its window's query
// count, its flag, the patch row and mask bytes) is issued at once at the start, and the
// weight [C][64] is staged once per block by direct global->LDS loads in 128-byte rows with
// 16-byte chunk c at c ^ (row & 7) (loads into VGPRs move a quarter of the bytes per cycle).
// (the body for 64-token group blk; a block of 256 threads; emb_w holds C x 64 bf16 of LDS
// and then the C bias floats)
template <int C>
__device__ __forceinline__ void embed_tokens(const Geo& g, int blk, const float* __restrict__ frames,
                                             const uint8_t* __restrict__ masks, const uint8_t* __restrict__ flag,
                                             const int32_t* __restrict__ wcount, const bf16* __restrict__ wT16,
                                             const float* __restrict__ bias, float* __restrict__ x,
                                             bf16* __restrict__ xh, bf16* emb_w) {
  constexpr int FN = C / 16;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int l16 = lane & 15, kg = lane >> 4;
  const int n = (blk * 4 + wv) * 16 + l16;
  const bool in = n < g.N;
  float v[12];
#pragma unroll
  for (int e = 0; e < 12; ++e) v[e] = 0.f;
  uint32_t m = 0;
  int wc = 0, fl = 0;
  if (in) {
    wc = wcount == nullptr ? 1 : wcount[n / g.S];
    fl = flag[n];
    int b, t, i, j;
    token_coords(g, n, b, t, i, j);
    const size_t px = (((size_t)b * g.T + t) * g.H + 4 * i + kg) * g.W + 4 * j;
    const float4* src = reinterpret_cast<const float4*>(frames + px * 3);
    const float4 f0 = src[0], f1 = src[1], f2 = src[2];
    m = *reinterpret_cast<const uint32_t*>(masks + px);
    v[0] = f0.x; v[1] = f0.y; v[2] = f0.z; v[3] = f0.w;
    v[4] = f1.x; v[5] = f1.y; v[6] = f1.z; v[7] = f1.w;
    v[8] = f2.x; v[9] = f2.y; v[10] = f2.z; v[11] = f2.w;
  }
  const bool need_h = in && wc > 0;
  if (!__syncthreads_or(need_h)) return;  // uniform per block
  static_for<C / 32>([&](auto c) {  // C rows, 8 per load, over the four wavefronts
    const int g8 = wv + 4 * c;
    const int row = g8 * 8 + (lane >> 3);
    dma16(wT16 + (size_t)row * 64 + ((lane & 7) ^ lds_swz(row)) * 8, emb_w + g8 * 512);
  });
  // the bias (C floats, 256-byte aligned) after the weight, 64 16-byte chunks per wavefront
  float* emb_b = reinterpret_cast<float*>(emb_w + C * 64);
  if (wv * 64 < C / 4 && wv * 64 + lane < C / 4)
    dma16(bias + 4 * (wv * 64 + lane), reinterpret_cast<bf16*>(emb_b + wv * 256));
  vm_wait_barrier<0>();
  if (!__any(need_h)) return;  // wave-uniform; no barrier follows
  const bool need_x = need_h && fl != 0;
#pragma unroll
  for (int kx = 0; kx < 4; ++kx)
    if ((m >> (8 * kx)) & 0xffu) v[3 * kx] = v[3 * kx + 1] = v[3 * kx + 2] = 0.f;
  bf16x8_t p0, p1;
#pragma unroll
  for (int e = 0; e < 8; ++e) p0[e] = (__bf16)v[e];
#pragma unroll
  for (int e = 0; e < 4; ++e) p1[e] = (__bf16)v[8 + e];
#pragma unroll
  for (int e = 4; e < 8; ++e) p1[e] = (__bf16)0.f;
  // each fragment's weight slices and bias are read from LDS one fragment ahead of its fenced
  // MFMA pair (inside the fences every fragment had waited for its own round trips in turn)
  f32x4_t acc[FN];
  float sum = 0.f;
  auto wslice = [&](int f, bf16x8_t& w0, bf16x8_t& w1, float4& b4) {
    const int row = 16 * f + l16;
    w0 = *reinterpret_cast<const bf16x8_t*>(emb_w + row * 64 + ((kg ^ lds_swz(row)) * 8));
    w1 = *reinterpret_cast<const bf16x8_t*>(emb_w + row * 64 + (((4 + kg) ^ lds_swz(row)) * 8));
    b4 = *reinterpret_cast<const float4*>(emb_b + 16 * f + 4 * kg);
  };
  bf16x8_t wa0, wa1, wb0, wb1;
  float4 ba, bb;
  wslice(0, wa0, wa1, ba);
  static_for<FN>([&](auto f) {
    bf16x8_t& c0 = (f & 1) ? wb0 : wa0;
    bf16x8_t& c1 = (f & 1) ? wb1 : wa1;
    const float4& b4 = (f & 1) ? bb : ba;
    if constexpr (f + 1 < FN) {
      if constexpr (f & 1)
        wslice(f + 1, wa0, wa1, ba);
      else
        wslice(f + 1, wb0, wb1, bb);
    }
    f32x4_t a = {0.f, 0.f, 0.f, 0.f};
    __builtin_amdgcn_sched_barrier(0);
    a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(c0, p0, a, 0, 0, 0);
    a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(c1, p1, a, 0, 0, 0);
    __builtin_amdgcn_sched_barrier(0);
    asm volatile("s_nop 7" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
    a[0] += b4.x; a[1] += b4.y; a[2] += b4.z; a[3] += b4.w;
    acc[f] = a;
    sum += (a[0] + a[1]) + (a[2] + a[3]);
  });
  sum += __shfl_xor(sum, 16, 64);
  sum += __shfl_xor(sum, 32, 64);
  const float mean = sum * (1.0f / C);
  float sq = 0.f;
#pragma unroll
  for (int f = 0; f < FN; ++f)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const float d = acc[f][e] - mean;
      sq += d * d;
    }
  sq += __shfl_xor(sq, 16, 64);
  sq += __shfl_xor(sq, 32, 64);
  const float rstd = rsqrtf(sq * (1.0f / C) + 1e-5f);
  if (!need_h) return;
#pragma unroll
  for (int f = 0; f < FN; ++f) {
    const int c = 16 * f + 4 * kg;
    const f32x4_t& a = acc[f];
    if (need_x) *reinterpret_cast<float4*>(x + (size_t)n * C + c) = make_float4(a[0], a[1], a[2], a[3]);
    uint2 pk;
    pk.x = pack_bf2((a[0] - mean) * rstd, (a[1] - mean) * rstd);
    pk.y = pack_bf2((a[2] - mean) * rstd, (a[3] - mean) * rstd);
    *reinterpret_cast<uint2*>(xh + (size_t)n * C + c) = pk;
  }
}

// One launch for the three steps of the BF16 path that need only the token flags and window
// counts: block 0 orders the windows and lists the Q/K/V row tiles, blocks 1 .. nwin gather
// each window's query tokens, the rest embed 64 tokens each.  They run side by side instead of
// one after the other with a launch gap between.  emb_wcount: window counts for the
// embedding's skip test (null: embed every token, as stream mode needs).
template <int C>
__global__ void __launch_bounds__(256) tokens_embed_bf16_kernel(
    Geo g, const float* __restrict__ frames, const uint8_t* __restrict__ masks, const uint8_t* __restrict__ flag,
    const int32_t* __restrict__ wcount, const int32_t* __restrict__ emb_wcount, const bf16* __restrict__ wT16,
    const float* __restrict__ bias, float* __restrict__ x, bf16* __restrict__ xh, int32_t* __restrict__ idx,
    int32_t* __restrict__ woff, int32_t* __restrict__ nq, int32_t* __restrict__ order, int32_t* __restrict__ tiles,
    int32_t* __restrict__ ntiles) {
  extern __shared__ __align__(16) int tok_lds[];
  const int b = blockIdx.x;
  if (b == 0) {
    order_windows<256>(g.nwin, g.S, g.N, wcount, flag, order, tiles, ntiles, tok_lds, tok_lds + (ORDER_MAX_S + 1),
                  tok_lds + 2 * (ORDER_MAX_S + 1));
  } else if (b <= g.nwin) {
    gather_window(g, b - 1, flag, wcount, idx, woff, nq);
  } else {
    embed_tokens<C>(g, b - 1 - g.nwin, frames, masks, flag, emb_wcount, wT16, bias, x, xh,
                    reinterpret_cast<bf16*>(tok_lds));
  }
}

void launch_tokens_embed_bf16(const Geo& g, int C, const float* frames, const uint8_t* masks, const uint8_t* flag,
                              const int32_t* wcount, const int32_t* emb_wcount, const bf16* wT16, const float* b,
                              float* x, bf16* xh, int32_t* idx, int32_t* woff, int32_t* nq, int32_t* order,
                              int32_t* tiles, int32_t* ntiles, hipStream_t s) {
  const int grid = 1 + g.nwin + (g.N + 63) / 64;
  const size_t order_lds = (2 * (size_t)(ORDER_MAX_S + 1) + 2) * 4;
  const size_t lds = std::max((size_t)C * 64 * 2 + (size_t)C * 4, order_lds);  // weight + bias, at most 49.5 KB
#define DR_TOK_EMB(C_)                                                                                        \
  case C_:                                                                                                    \
    tokens_embed_bf16_kernel<C_><<<grid, 256, lds, s>>>(g, frames, masks, flag, wcount, emb_wcount, wT16, b, x, \
                                                       xh, idx, woff, nq, order, tiles, ntiles);             \
    break;
  switch (C) {
    DR_TOK_EMB(64)
    DR_TOK_EMB(128)
    DR_TOK_EMB(256)
    DR_TOK_EMB(384)
    default: break;  // rejected by the caller (resid_ln_supported)
  }
#undef DR_TOK_EMB
}

// Decoder on x^ with the final LayerNorm's affine part folded in: logits[k] = bd'[k] +
// sum_c x^[c] Wd'[k][c] (Wd' [48][C] bf16, bd' [48] FP32), sigmoid, and the masked pixels of
// each flagged token written.  Output fragment f of lane l holds k = 16 f + 4 (l / 16) + e of
// token l % 16.  Blocks blk of nblk, 256 threads; wl holds 48 x C bf16 of LDS.  The weight is
// staged once per block by direct loads ([C/64][48][64], swizzled 128-byte rows) and every x^
// fragment of a 16-token group is requested before its MFMAs: with the loads inside the
// fenced k loop each slice waited for its own round trip.
template <int C>
__device__ __forceinline__ void decode_rows(const Geo& g, int blk, int nblk, const bf16* __restrict__ xh,
                                            const int32_t* __restrict__ idx, const int32_t* __restrict__ nq,
                                            const bf16* __restrict__ wd16, const float* __restrict__ bd,
                                            const uint8_t* __restrict__ masks, float* __restrict__ out, bf16* wl) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int l16 = lane & 15, kg = lane >> 4;
  const int total = nq[0];
  if (blk * 64 >= total) return;  // no rows here: skip the weight
  constexpr int NG = (C / 64) * 6;  // 8-row groups of the staged weight
  for (int gi = wv; gi < NG; gi += 4) {  // uniform per wavefront
    const int kb = gi / 6, g8 = gi - kb * 6;
    const int row = g8 * 8 + (lane >> 3);
    dma16(wd16 + (size_t)row * C + 64 * kb + ((lane & 7) ^ lds_swz(row)) * 8, wl + (kb * 48 + g8 * 8) * 64);
  }
  vm_wait_barrier<0>();
  for (int r0 = (blk * 4 + wv) * 16; r0 < total; r0 += nblk * 64) {
    const int r = r0 + l16;
    const bool ok = r < total;
    const int n = ok ? idx[r] : 0;
    bf16x8_t z[C / 32];
#pragma unroll
    for (int kk = 0; kk < C / 32; ++kk)
      z[kk] = ok ? *reinterpret_cast<const bf16x8_t*>(xh + (size_t)n * C + kk * 32 + 8 * kg) : bf16x8_t{};
    f32x4_t acc[3] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
#pragma unroll
    for (int kk = 0; kk < C / 32; ++kk) {
      bf16x8_t w[3];
#pragma unroll
      for (int f = 0; f < 3; ++f) {
        const int row = 16 * f + l16;
        w[f] = *reinterpret_cast<const bf16x8_t*>(wl + ((kk >> 1) * 48 + row) * 64 + ((((kk & 1) * 4 + kg) ^ lds_swz(row)) * 8));
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int f = 0; f < 3; ++f) acc[f] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w[f], z[kk], acc[f], 0, 0, 0);
      __builtin_amdgcn_sched_barrier(0);
      asm volatile("s_nop 7" ::: "memory");
      __builtin_amdgcn_sched_barrier(0);
    }
    if (!ok) continue;
    int b, t, i, j;
    token_coords(g, n, b, t, i, j);
#pragma unroll
    for (int f = 0; f < 3; ++f)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int k = 16 * f + 4 * kg + e;
        const int pix = k / 3, ch = k - 3 * pix;
        const int ky = pix >> 2, kx = pix & 3;
        const size_t px = (((size_t)b * g.T + t) * g.H + 4 * i + ky) * g.W + 4 * j + kx;
        if (masks[px]) out[px * 3 + ch] = 1.0f / (1.0f + expf(-(acc[f][e] + bd[k])));
      }
  }
}

// ------------------------------------------------------------------------------------------
// Overlapping variant: embedding Conv2d(3, C, 8, stride 4, padding 2) and the decoder as the
// matching transposed convolution, whose overlapping patches are summed (the fold) -- done
// here as a reduction: each token's 8 x 8 x 3 logit patch, then each private pixel sums the
// patches of the (at most 2 x 2) tokens whose footprint covers it.
// ------------------------------------------------------------------------------------------

// Window-major index of token (b, t, i, j) (inverse of token_coords).
__device__ __forceinline__ int token_index(const Geo& g, int b, int t, int i, int j) {
  const int nT = g.T / g.wt;
  const int a = t / g.wt, dt = t - a * g.wt;
  const int u = i / g.wh, di = i - u * g.wh;
  const int v = j / g.ww, dj = j - v * g.ww;
  const int w = ((b * nT + a) * g.nwh + u) * g.nww + v;
  return w * g.S + (dt * g.wh + di) * g.ww + dj;
}

// Lane (token l16, group kg) loads rows ky = kg and kg + 4 of its token's footprint (pixel
// rows 4i - 2 + ky, columns 4j - 2 .. 4j + 5; zero outside the frame and where the mask is
// set): 24 values per row, m = 3 kx + c.  32-wide k slice s takes values m = 8 (s % 3) .. + 7
// of row kg + 4 (s / 3) in the lane's 8 slots, and wT16 [C][192] holds the weight in the
// same slot order.  Columns come in pixel pairs (x0 and W are even), each pair wholly inside
// or outside the frame: three 8-byte loads and one 2-byte mask load per pair.
template <int C>
__global__ void __launch_bounds__(256) embed_ovl_bf16_kernel(Geo g, const float* __restrict__ frames,
                                                             const uint8_t* __restrict__ masks,
                                                             const uint8_t* __restrict__ flag,
                                                             const int32_t* __restrict__ wcount,
                                                             const bf16* __restrict__ wT16,
                                                             const float* __restrict__ bias, float* __restrict__ x,
                                                             bf16* __restrict__ xh) {
  constexpr int FN = C / 16, KS = 6;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int l16 = lane & 15, kg = lane >> 4;
  const int n = (blockIdx.x * 4 + wv) * 16 + l16;
  const bool need_h = n < g.N && (wcount == nullptr || wcount[n / g.S] > 0);
  if (!__any(need_h)) return;  // wave-uniform: no barrier in this kernel
  const bool need_x = need_h && flag[n] != 0;
  bf16x8_t pk[KS];
  int b = 0, t = 0, i = 0, j = 0;
  if (need_h) token_coords(g, n, b, t, i, j);
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    float v[24];
#pragma unroll
    for (int e = 0; e < 24; ++e) v[e] = 0.f;
    const int y = 4 * i - 2 + kg + 4 * r;
    if (need_h && y >= 0 && y < g.H) {
      const size_t rowpx = (((size_t)b * g.T + t) * g.H + y) * g.W;
      const int x0 = 4 * j - 2;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int xx = x0 + 2 * q;
        if (xx >= 0 && xx < g.W) {
          const float2* src = reinterpret_cast<const float2*>(frames + (rowpx + xx) * 3);
          const float2 f0 = src[0], f1 = src[1], f2 = src[2];
          const uint32_t m = *reinterpret_cast<const uint16_t*>(masks + rowpx + xx);
          const bool m0 = (m & 0xffu) != 0, m1 = (m >> 8) != 0;
          v[6 * q + 0] = m0 ? 0.f : f0.x;
          v[6 * q + 1] = m0 ? 0.f : f0.y;
          v[6 * q + 2] = m0 ? 0.f : f1.x;
          v[6 * q + 3] = m1 ? 0.f : f1.y;
          v[6 * q + 4] = m1 ? 0.f : f2.x;
          v[6 * q + 5] = m1 ? 0.f : f2.y;
        }
      }
    }
#pragma unroll
    for (int part = 0; part < 3; ++part)
#pragma unroll
      for (int e = 0; e < 8; ++e) pk[3 * r + part][e] = (__bf16)v[8 * part + e];
  }
  f32x4_t acc[FN];
  float sum = 0.f;
#pragma unroll
  for (int f = 0; f < FN; ++f) {
    const bf16* wr = wT16 + (size_t)(16 * f + l16) * (32 * KS) + 8 * kg;
    bf16x8_t w[KS];
#pragma unroll
    for (int sl = 0; sl < KS; ++sl) w[sl] = *reinterpret_cast<const bf16x8_t*>(wr + 32 * sl);
    f32x4_t a = {0.f, 0.f, 0.f, 0.f};
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int sl = 0; sl < KS; ++sl) a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w[sl], pk[sl], a, 0, 0, 0);
    __builtin_amdgcn_sched_barrier(0);
    asm volatile("s_nop 7" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
    const float4 b4 = *reinterpret_cast<const float4*>(bias + 16 * f + 4 * kg);
    a[0] += b4.x; a[1] += b4.y; a[2] += b4.z; a[3] += b4.w;
    acc[f] = a;
    sum += (a[0] + a[1]) + (a[2] + a[3]);
  }
  sum += __shfl_xor(sum, 16, 64);
  sum += __shfl_xor(sum, 32, 64);
  const float mean = sum * (1.0f / C);
  float sq = 0.f;
#pragma unroll
  for (int f = 0; f < FN; ++f)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const float d = acc[f][e] - mean;
      sq += d * d;
    }
  sq += __shfl_xor(sq, 16, 64);
  sq += __shfl_xor(sq, 32, 64);
  const float rstd = rsqrtf(sq * (1.0f / C) + 1e-5f);
  if (!need_h) return;
#pragma unroll
  for (int f = 0; f < FN; ++f) {
    const int c = 16 * f + 4 * kg;
    const f32x4_t& a = acc[f];
    if (need_x) *reinterpret_cast<float4*>(x + (size_t)n * C + c) = make_float4(a[0], a[1], a[2], a[3]);
    uint2 pw;
    pw.x = pack_bf2((a[0] - mean) * rstd, (a[1] - mean) * rstd);
    pw.y = pack_bf2((a[2] - mean) * rstd, (a[3] - mean) * rstd);
    *reinterpret_cast<uint2*>(xh + (size_t)n * C + c) = pw;
  }
}

void launch_embed_ovl_bf16(const Geo& g, int C, const float* frames, const uint8_t* masks, const uint8_t* flag,
                           const int32_t* wcount, const bf16* wT16, const float* b, float* x, bf16* xh,
                           hipStream_t s) {
  const int blocks = (g.N + 63) / 64;
  if (blocks == 0) return;
  switch (C) {
    case 64: embed_ovl_bf16_kernel<64><<<blocks, 256, 0, s>>>(g, frames, masks, flag, wcount, wT16, b, x, xh); break;
    case 128: embed_ovl_bf16_kernel<128><<<blocks, 256, 0, s>>>(g, frames, masks, flag, wcount, wT16, b, x, xh); break;
    case 256: embed_ovl_bf16_kernel<256><<<blocks, 256, 0, s>>>(g, frames, masks, flag, wcount, wT16, b, x, xh); break;
    case 384: embed_ovl_bf16_kernel<384><<<blocks, 256, 0, s>>>(g, frames, masks, flag, wcount, wT16, b, x, xh); break;
    default: break;  // rejected by the caller
  }
}

// Logit patch of each flagged token: contrib[n][k] = bd'[k] + sum_c x^[n][c] Wd'[k][c],
// k = (ky*8 + kx)*3 + ch; twelve 16-wide output fragments per 16 tokens.
template <int C>
__global__ void __launch_bounds__(256) decode_ovl_bf16_kernel(Geo g, const bf16* __restrict__ xh,
                                                              const int32_t* __restrict__ idx,
                                                              const int32_t* __restrict__ nq,
                                                              const bf16* __restrict__ wd16,
                                                              const float* __restrict__ bd,
                                                              float* __restrict__ contrib) {
  constexpr int NF = 12;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int l16 = lane & 15, kg = lane >> 4;
  const int total = nq[0];
  for (int r0 = (blockIdx.x * 4 + wv) * 16; r0 < total; r0 += gridDim.x * 64) {
    const int r = r0 + l16;
    const bool ok = r < total;
    const int n = ok ? idx[r] : 0;
    f32x4_t acc[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) acc[f] = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
    for (int kk = 0; kk < C / 32; ++kk) {
      const bf16x8_t z = ok ? *reinterpret_cast<const bf16x8_t*>(xh + (size_t)n * C + kk * 32 + 8 * kg)
                            : bf16x8_t{};
      bf16x8_t w[NF];
#pragma unroll
      for (int f = 0; f < NF; ++f)
        w[f] = *reinterpret_cast<const bf16x8_t*>(wd16 + (size_t)(16 * f + l16) * C + kk * 32 + 8 * kg);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int f = 0; f < NF; ++f) acc[f] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w[f], z, acc[f], 0, 0, 0);
      __builtin_amdgcn_sched_barrier(0);
      asm volatile("s_nop 7" ::: "memory");
      __builtin_amdgcn_sched_barrier(0);
    }
    if (!ok) continue;
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      const int k = 16 * f + 4 * kg;
      const float4 b4 = *reinterpret_cast<const float4*>(bd + k);
      *reinterpret_cast<float4*>(contrib + (size_t)n * 192 + k) =
          make_float4(acc[f][0] + b4.x, acc[f][1] + b4.y, acc[f][2] + b4.z, acc[f][3] + b4.w);
    }
  }
}

void launch_decode_ovl_bf16(const Geo& g, int C, const bf16* xh, const int32_t* idx, const int32_t* nq,
                            const bf16* wd16, const float* bd, float* contrib, hipStream_t s) {
  int grid = (g.N + 63) / 64;
  if (grid > DEC_GRID) grid = DEC_GRID;
  if (grid == 0) return;
  switch (C) {
    case 64: decode_ovl_bf16_kernel<64><<<grid, 256, 0, s>>>(g, xh, idx, nq, wd16, bd, contrib); break;
    case 128: decode_ovl_bf16_kernel<128><<<grid, 256, 0, s>>>(g, xh, idx, nq, wd16, bd, contrib); break;
    case 256: decode_ovl_bf16_kernel<256><<<grid, 256, 0, s>>>(g, xh, idx, nq, wd16, bd, contrib); break;
    case 384: decode_ovl_bf16_kernel<384><<<grid, 256, 0, s>>>(g, xh, idx, nq, wd16, bd, contrib); break;
    default: break;
  }
}

// Each private pixel (y, x): the covering tokens are rows i1 = (y + 2) / 4 (kernel row
// y + 2 - 4 i1 in 0..3) and i1 - 1 (kernel row + 4), likewise for columns, those inside the
// token grid (the crop); the pixel sums their logit patches at its kernel offset, adds the
// bias and applies the sigmoid.  Every covering token is flagged by the footprint rule, so
// its patch has been written.  Four pixels per thread (W % 4 == 0).
__global__ void __launch_bounds__(256) fold_ovl_kernel(Geo g, const float* __restrict__ contrib,
                                                       const float* __restrict__ db,
                                                       const uint8_t* __restrict__ masks, float* __restrict__ out) {
  const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t npix = (size_t)g.B * g.T * g.H * g.W;
  if (q * 4 >= npix) return;
  const size_t p0 = q * 4;
  const uint32_t m4 = *reinterpret_cast<const uint32_t*>(masks + p0);
  if (m4 == 0) return;
  const size_t plane = (size_t)g.H * g.W;
  const int bt = (int)(p0 / plane);
  const int b = bt / g.T, t = bt - b * g.T;
  const size_t in_plane = p0 - (size_t)bt * plane;
  const int y = (int)(in_plane / g.W), x0 = (int)(in_plane - (size_t)y * g.W);
  const int i1 = (y + 2) >> 2;
  const float b0 = db[0], b1 = db[1], b2 = db[2];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    if (!((m4 >> (8 * e)) & 0xffu)) continue;
    const int x = x0 + e;
    const int j1 = (x + 2) >> 2;
    float a0 = b0, a1 = b1, a2 = b2;
#pragma unroll
    for (int di = 0; di < 2; ++di) {
      const int i = i1 - di;
      if (i < 0 || i >= g.Ht) continue;
      const int ky = y + 2 - 4 * i;
#pragma unroll
      for (int dj = 0; dj < 2; ++dj) {
        const int j = j1 - dj;
        if (j < 0 || j >= g.Wt) continue;
        const int kx = x + 2 - 4 * j;
        const float* cp = contrib + (size_t)token_index(g, b, t, i, j) * 192 + (ky * 8 + kx) * 3;
        a0 += cp[0];
        a1 += cp[1];
        a2 += cp[2];
      }
    }
    float* o = out + (p0 + e) * 3;
    o[0] = 1.0f / (1.0f + expf(-a0));
    o[1] = 1.0f / (1.0f + expf(-a1));
    o[2] = 1.0f / (1.0f + expf(-a2));
  }
}

void launch_fold_ovl(const Geo& g, const float* contrib, const float* db, const uint8_t* masks, float* out,
                     hipStream_t s) {
  const size_t quads = (size_t)g.B * g.T * g.H * g.W / 4;
  if (quads == 0) return;
  fold_ovl_kernel<<<(unsigned)((quads + 255) / 256), 256, 0, s>>>(g, contrib, db, masks, out);
}

// ------------------------------------------------------------------------------------------
// out = frames wherever the mask is 0 (4 pixels per thread, vector loads and stores).
// ------------------------------------------------------------------------------------------
// (quads q0, q0 + stride, ...)
__device__ __forceinline__ void copy_quads(size_t q0, size_t stride, size_t nquad, const float4* __restrict__ frames,
                                           const uint32_t* __restrict__ masks, float4* __restrict__ out) {
  for (size_t q = q0; q < nquad; q += stride) {
    const uint32_t m = masks[q];
    if (m == 0x01010101u) continue;
    const float4 a = frames[3 * q], b = frames[3 * q + 1], c = frames[3 * q + 2];
    if (m == 0) {
      out[3 * q] = a;
      out[3 * q + 1] = b;
      out[3 * q + 2] = c;
    } else {
      float v[12] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w, c.x, c.y, c.z, c.w};
      float* o = reinterpret_cast<float*>(out + 3 * q);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (((m >> (8 * k)) & 0xffu) == 0) {
          o[3 * k] = v[3 * k];
          o[3 * k + 1] = v[3 * k + 1];
          o[3 * k + 2] = v[3 * k + 2];
        }
      }
    }
  }
}

__global__ void copy_unmasked_kernel(size_t nquad, const float4* __restrict__ frames,
                                     const uint32_t* __restrict__ masks, float4* __restrict__ out) {
  copy_quads(blockIdx.x * (size_t)blockDim.x + threadIdx.x, (size_t)gridDim.x * blockDim.x, nquad, frames, masks,
             out);
}

// The BF16 decoder (blocks below gd) and the copy of the unmasked pixels (the rest) in one
// launch: they write disjoint pixels.
template <int C>
__global__ void __launch_bounds__(256) decode_copy_bf16_kernel(Geo g, const bf16* __restrict__ xh,
                                                               const int32_t* __restrict__ idx,
                                                               const int32_t* __restrict__ nq,
                                                               const bf16* __restrict__ wd16,
                                                               const float* __restrict__ bd,
                                                               const uint8_t* __restrict__ masks,
                                                               float* __restrict__ out, int gd, size_t nquad,
                                                               const float4* __restrict__ frames) {
  extern __shared__ __align__(16) bf16 dec_w[];
  if ((int)blockIdx.x < gd)
    decode_rows<C>(g, blockIdx.x, gd, xh, idx, nq, wd16, bd, masks, out, dec_w);
  else
    copy_quads((blockIdx.x - gd) * (size_t)blockDim.x + threadIdx.x, (size_t)(gridDim.x - gd) * blockDim.x, nquad,
               frames, reinterpret_cast<const uint32_t*>(masks), reinterpret_cast<float4*>(out));
}

void launch_decode_copy_bf16(const Geo& g, int C, const bf16* xh, const int32_t* idx, const int32_t* nq,
                             const bf16* wd16, const float* bd, const uint8_t* masks, const float* frames,
                             float* out, size_t npix, hipStream_t s) {
  int gd = (g.N + 63) / 64;
  if (gd > DEC_GRID) gd = DEC_GRID;
  const size_t nquad = out != frames ? npix / 4 : 0;  // in place: nothing to copy
  size_t gc = (nquad + 255) / 256;
  if (gc > 4096) gc = 4096;
  const unsigned grid = (unsigned)(gd + gc);
  if (grid == 0) return;
  const float4* f4 = reinterpret_cast<const float4*>(frames);
#define DR_DEC_COPY(C_)                                                                                        \
  case C_:                                                                                                     \
    decode_copy_bf16_kernel<C_><<<grid, 256, 48 * C_ * 2, s>>>(g, xh, idx, nq, wd16, bd, masks, out, gd, nquad, f4); \
    break;
  switch (C) {
    DR_DEC_COPY(64)
    DR_DEC_COPY(128)
    DR_DEC_COPY(256)
    DR_DEC_COPY(384)
    default: break;
  }
#undef DR_DEC_COPY
}

void launch_copy_unmasked(size_t npix, const float* frames, const uint8_t* masks, float* out,
                          hipStream_t s) {
  const size_t nquad = npix / 4;
  size_t grid = (nquad + 255) / 256;
  if (grid > 4096) grid = 4096;
  if (grid == 0) return;
  copy_unmasked_kernel<<<(unsigned)grid, 256, 0, s>>>(nquad, reinterpret_cast<const float4*>(frames),
                                                      reinterpret_cast<const uint32_t*>(masks),
                                                      reinterpret_cast<float4*>(out));
}

}  // namespace dr

namespace dr {

// ------------------------------------------------------------------------------------------
// Stream mode: copy the batch's per-request frames and masks into contiguous staging buffers
// (request-major), and the staged outputs back.  One grid row per request, float4 / u32
// accesses (each frame holds a multiple of 4 pixels).
// ------------------------------------------------------------------------------------------
__global__ void gather_frames_kernel(FramePtrs p, size_t nquad, float4* __restrict__ fst,
                                     uint32_t* __restrict__ mst) {
  const int r = blockIdx.y;
  const float4* f = reinterpret_cast<const float4*>(p.f[r]);
  const uint32_t* m = reinterpret_cast<const uint32_t*>(p.m[r]);
  float4* fo = fst + (size_t)r * nquad * 3;
  uint32_t* mo = mst + (size_t)r * nquad;
  for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < nquad; q += (size_t)gridDim.x * blockDim.x) {
    fo[3 * q] = f[3 * q];
    fo[3 * q + 1] = f[3 * q + 1];
    fo[3 * q + 2] = f[3 * q + 2];
    mo[q] = m[q];
  }
}

__global__ void scatter_frames_kernel(FramePtrs p, size_t nquad, const float4* __restrict__ ost) {
  const int r = blockIdx.y;
  float4* o = reinterpret_cast<float4*>(p.o[r]);
  const float4* src = ost + (size_t)r * nquad * 3;
  for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < 3 * nquad; q += (size_t)gridDim.x * blockDim.x)
    o[q] = src[q];
}

void launch_gather_frames(const FramePtrs& p, size_t npix, float* fst, uint8_t* mst, hipStream_t s) {
  const size_t nquad = npix / 4;
  unsigned gx = (unsigned)((nquad + 255) / 256);
  if (gx > 512) gx = 512;
  gather_frames_kernel<<<dim3(gx, p.n), 256, 0, s>>>(p, nquad, reinterpret_cast<float4*>(fst),
                                                     reinterpret_cast<uint32_t*>(mst));
}

void launch_scatter_frames(const FramePtrs& p, size_t npix, const float* ost, hipStream_t s) {
  const size_t nquad = npix / 4;
  unsigned gx = (unsigned)((3 * nquad + 255) / 256);
  if (gx > 512) gx = 512;
  scatter_frames_kernel<<<dim3(gx, p.n), 256, 0, s>>>(p, nquad, reinterpret_cast<const float4*>(ost));
}

}  // namespace dr
