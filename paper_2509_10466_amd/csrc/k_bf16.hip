// Window attention on gfx950 matrix cores (BF16 operands, FP32 accumulation): K and V^T of a
// (window, head) staged in LDS, scores and softmax statistics in FP32 registers.
//
// MFMA 16x16 operand layout (wave64): lane l supplies row (l % 16) of A and column (l % 16)
// of B, each with consecutive k values; the k group is (l / 16).  The result lane l holds
// C[4*(l/16) + i][l % 16], i = 0..3.  Only the pairing of A's and B's k slots matters for
// the sum, so any k permutation applied to both operands alike is legal; the kernel uses
// that to feed P straight from the score registers.
//
// The score and output products (S^T = K Q^T, O^T = V^T P^T) use the double-rate
// v_mfma_f32_16x16x32_bf16 in fenced groups: that form keeps reading its source VGPRs for a
// few cycles after issue, and a VALU write to one of them right after the issue corrupts the
// product (seen as run-to-run differences of single output elements), a case the compiler
// does not pad; each group is therefore bracketed by scheduling barriers and followed by
// s_nop 7, with the next group's operands loaded into other registers beforehand.  The last
// key tile of an odd tile count, which has no partner for a 32-wide k step, uses the
// single-rate v_mfma_f32_16x16x16_bf16, whose operands are read at issue.
#include "dr_device.h"
#include "dr_internal.h"

namespace dr {

__device__ __forceinline__ f32x4_t mfma16k16(const bf16x4_t& a, const bf16x4_t& b, const f32x4_t& c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// Double-rate k = 32 product; groups of these are fenced (see above).
__device__ __forceinline__ f32x4_t mfma32(const bf16x8_t& a, const bf16x8_t& b, const f32x4_t& c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ void mfma_fence_begin() { __builtin_amdgcn_sched_barrier(0); }
__device__ __forceinline__ void mfma_fence_end() {
  __builtin_amdgcn_sched_barrier(0);
  asm volatile("s_nop 7" ::: "memory");
  __builtin_amdgcn_sched_barrier(0);
}

template <typename T, typename S>
__device__ __forceinline__ T bitcast(const S& s) {
  static_assert(sizeof(T) == sizeof(S), "size");
  T t;
  __builtin_memcpy(&t, &s, sizeof(T));
  return t;
}

// ------------------------------------------------------------------------------------------
// Window attention, clip mode (BF16 and FP8 paths): one block of 8 wavefronts per (window, head)
// runs every query of the window, so K and V of a (window, head) reach LDS exactly once.
// K [Spad][dh] arrives by direct global->LDS loads with its 16-byte chunks XOR-swizzled by
// row (chunk c of row r at c ^ (r mod dh/8)), V^T [dh][SPV] is stored transposed by the
// Q/K/V epilogue with an odd number of 16-byte chunks per row (SPV), so its 16 fragment
// rows fall on distinct banks, and is copied as one contiguous block.  Each wavefront
// takes query tiles of 16: S^T = K Q^T, row softmax in FP32 registers, O^T = V^T P^T.
// ------------------------------------------------------------------------------------------
constexpr int ATT_THREADS = 512;
// Blocks per (window, head) of the clip attention kernel.  Two (each staging the window and
// taking every other group of 8 query tiles) measured slower at 240 keys: 128 against
// 114 us of attention per clip, the second staging of the busiest windows costing more
// than their second pass over query tiles.
constexpr int ATT_SPLIT = 1;

__host__ __device__ constexpr int attn_vt_stride(int spad) { return (spad / 8) % 2 ? spad : spad + 8; }

// Copies `bytes` (a multiple of 16) from global to LDS, 1 KB per wavefront load; the
// K tile is swizzled on the way (dh/8 chunks per row), the V^T tile copied as is.
template <int CH, bool SWZ, int NTHR = ATT_THREADS>
__device__ __forceinline__ void attn_dma(const bf16* __restrict__ src, bf16* dst, int bytes) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int chunks = bytes / 16;
  for (int c0 = wv * 64; c0 < chunks; c0 += NTHR) {
    const int c = c0 + lane;
    if (c < chunks) {
      int sc = c;
      if (SWZ) {
        const int row = c / CH, pc = c % CH;
        sc = row * CH + (pc ^ (row & (CH - 1)));
      }
      __builtin_amdgcn_global_load_lds(src + (size_t)sc * 8, (__attribute__((address_space(3))) void*)(dst + c0 * 8),
                                       16, 0, 0);
    }
  }
}

// Q^T operand of query tile qt: lane holds q[idx[q0 + 16 qt + l16]][h*DH + 32 kk + 8 kg ..]
template <int DH>
__device__ __forceinline__ void attn_load_q(const bf16* __restrict__ q, const int32_t* __restrict__ idx, int q0,
                                            int nqw, int C, int h, int qt, bf16x8_t (&qf)[DH / 32]) {
  const int lane = threadIdx.x & 63, l16 = lane & 15, kg = lane >> 4;
  const int qi = qt * 16 + l16;
  const bool ok = qi < nqw;
  const int n = idx[q0 + (ok ? qi : 0)];
#pragma unroll
  for (int kk = 0; kk < DH / 32; ++kk) {
    const uint4 v = ok ? *reinterpret_cast<const uint4*>(q + (size_t)n * C + h * DH + kk * 32 + kg * 8)
                       : make_uint4(0, 0, 0, 0);
    qf[kk] = bitcast<bf16x8_t>(v);
  }
}

// Clip mode: keys 0 .. S-1 of the window; only the last tile can hold padding keys
// (S > 16 (NT - 1)).  V^T rows of stride SPV.
template <int NT, int SPV>
struct ClipKeys {
  int S;
  __device__ __forceinline__ bool valid(int tt, int j) const { return tt < NT - 1 || tt * 16 + j < S; }
  __device__ __forceinline__ const bf16* vt(const bf16* Vt, int d, int tt, int off) const {
    return Vt + d * SPV + tt * 16 + off;
  }
};

// Stream mode: NF frame blocks of SFP keys (the frame's SF window tokens, then padding);
// frame f exists when f <= np (np cached frames, then the new one).  V^T is frame-major,
// [NF][DH][VST].  A 16-key tile never straddles frames (SFP is a multiple of 16).
template <int DH, int SF, int SFP, int VST>
struct RingKeys {
  int np;
  __device__ __forceinline__ bool valid(int tt, int j) const {
    const int f = tt * 16 / SFP, within = tt * 16 - f * SFP + j;
    return f <= np && within < SF;
  }
  __device__ __forceinline__ const bf16* vt(const bf16* Vt, int d, int tt, int off) const {
    const int f = tt * 16 / SFP;
    return Vt + (f * DH + d) * VST + (tt * 16 - f * SFP) + off;
  }
};

// Every query tile of one (window, head): K (rows = keys, swizzled) and V^T staged in LDS.
// `keys` decides which keys exist (valid(tt, j): key 16 tt + j) and where V^T row d of the
// 4 keys from 16 tt + off sits (vt).  qnext holds the first tile's Q operand, loaded by the
// caller before staging.
// MODE selects the keys a query sees inside its window (tokens ordered (frame, row, column),
// A = tokens per frame, wt frames, wbase = the window's first token): 0 all of them, 1 those of
// the query's own frame (spatial attention of a decoupled network).  Masked keys score -inf,
// like padding; the query's own key is always visible.  (Temporal attention, the query's own
// position in every frame, has its own kernel: attn_temporal_kernel.)
struct KeyMask {
  int A, wbase;
};

template <int DH, int NT, class Keys, int MODE = 0, int QSTEP = ATT_THREADS / 64>
__device__ __forceinline__ float attn_query_tiles(const bf16* Ks, const bf16* Vt, const Keys& keys, int C, int h,
                                                 const bf16* __restrict__ q, const int32_t* __restrict__ idx,
                                                 int q0, int nqw, bf16* __restrict__ o, bf16x8_t (&qnext)[DH / 32],
                                                 bool want_amax, KeyMask km = KeyMask{0, 0}, int qt_base = 0) {
  constexpr int CH = DH / 8;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int l16 = lane & 15, kg = lane >> 4;
  float omax = 0.f;
  // query tiles qt_base + wv, then every QSTEP-th (the caller loaded the first one's Q)
  for (int qt = qt_base + wv; qt * 16 < nqw; qt += QSTEP) {
    // K and V^T fragments are re-read from LDS per query tile: hoisting them out of the loop
    // would hold the whole window in registers
    asm volatile("" ::: "memory");
    const int qi = qt * 16 + l16;
    const bool valid = qi < nqw;
    const int r = q0 + (valid ? qi : 0);
    // MODE 1: bit p of vis = key slot p of this lane (key 16 (p / 4) + 4 kg + p % 4) is
    // visible to its query; built once per query tile, three registers at most
    static_assert(MODE == 0 || MODE == 1, "key mask mode");
    constexpr int MW = (4 * NT + 31) / 32;
    uint32_t vis[MW];
    // key tiles tlo .. thi hold every key the tile's queries see (wave-uniform); MODE 1 skips
    // the products, exponentials and V^T reads of the others
    int tlo = 0, thi = NT - 1;
    if (MODE != 0) {
      const int sq = idx[r] - km.wbase;
      {
        // the query's frame [klo, klo + A) maps to a contiguous run of slots (key order is
        // monotone in p): slots below key x number 4 floor(y / 16) + min(y mod 16, 4),
        // y = x - 4 kg
        const int klo = (sq / km.A) * km.A;
        auto below = [&](int x) {
          const int y = x - kg * 4;
          return y <= 0 ? 0 : min(4 * NT, (y >> 4) * 4 + min(y & 15, 4));
        };
        const int plo = below(klo), phi = below(klo + km.A);
        int lo = klo, hi = klo + km.A - 1;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
          lo = min(lo, __shfl_xor(lo, off, 64));
          hi = max(hi, __shfl_xor(hi, off, 64));
        }
        tlo = __builtin_amdgcn_readfirstlane(lo) >> 4;
        thi = __builtin_amdgcn_readfirstlane(hi) >> 4;
#pragma unroll
        for (int j = 0; j < MW; ++j) {
          const int lo = min(max(plo - 32 * j, 0), 32), hi = min(max(phi - 32 * j, 0), 32);
          vis[j] = (uint32_t)(((1ull << hi) - 1ull) & ~((1ull << lo) - 1ull));
        }
      }
    }
    bf16x8_t qf[DH / 32];
#pragma unroll
    for (int kk = 0; kk < DH / 32; ++kk) qf[kk] = qnext[kk];
    // (nqw <= 16 NT: with QSTEP >= NT no wavefront has a second tile)
    if (QSTEP < NT && (qt + QSTEP) * 16 < nqw) attn_load_q<DH>(q, idx, q0, nqw, C, h, qt + QSTEP, qnext);
    // S^T = K Q^T: key tiles in groups of TG, each tile's k slices chained, the chains of a
    // group interleaved; a group's K fragments are read while the previous group multiplies
    constexpr int KS = DH / 32;  // 32-wide k slices
    constexpr int TG = 3;
    float sc[NT][4];
    bf16x8_t kf[2][TG][KS];
    auto read_k = [&](int g0, bf16x8_t (&dst)[TG][KS]) {
#pragma unroll
      for (int u = 0; u < TG; ++u) {
        const int tt = g0 + u;
        if (tt < NT) {
          const int row = tt * 16 + l16;
#pragma unroll
          for (int kk = 0; kk < KS; ++kk)
            dst[u][kk] = *reinterpret_cast<const bf16x8_t*>(Ks + row * DH + (((kk * 4 + kg) ^ (row & (CH - 1))) * 8));
        }
      }
    };
    auto group_live = [&](int g0) { return MODE == 0 || (g0 <= thi && g0 + TG - 1 >= tlo); };
    read_k(0, kf[0]);
#pragma unroll
    for (int g0 = 0; g0 < NT; g0 += TG) {
      const int cur = (g0 / TG) & 1;
      if (g0 + TG < NT) read_k(g0 + TG, kf[cur ^ 1]);
      if (!group_live(g0)) {
#pragma unroll
        for (int u = 0; u < TG; ++u)
          if (g0 + u < NT)
#pragma unroll
            for (int i = 0; i < 4; ++i) sc[g0 + u][i] = -INFINITY;
        continue;
      }
      f32x4_t a[TG];
      mfma_fence_begin();
#pragma unroll
      for (int kk = 0; kk < KS; ++kk)
#pragma unroll
        for (int u = 0; u < TG; ++u)
          if (g0 + u < NT) a[u] = mfma32(kf[cur][u][kk], qf[kk], kk ? a[u] : f32x4_t{0.f, 0.f, 0.f, 0.f});
      mfma_fence_end();
      // scores are already in base 2 (Q carries log2(e) / sqrt(dh)); padding keys and keys of
      // frames that do not exist yet score -inf
#pragma unroll
      for (int u = 0; u < TG; ++u) {
        const int tt = g0 + u;
        if (tt < NT)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            // (a visible key of MODE 1 always exists: it lies inside the window)
            const bool ok = MODE == 0 ? keys.valid(tt, kg * 4 + i) : ((vis[tt >> 3] >> ((tt & 7) * 4 + i)) & 1u);
            sc[tt][i] = ok ? a[u][i] : -INFINITY;
          }
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
    for (int tt = 0; tt < NT; ++tt) {
      if (MODE != 0 && (tt < tlo || tt > thi)) {
#pragma unroll
        for (int i = 0; i < 4; ++i) sc[tt][i] = 0.f;
        continue;
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float p = __builtin_amdgcn_exp2f(sc[tt][i] - mx);  // argument <= 0
        sc[tt][i] = p;
        sum += p;
      }
    }
    sum += __shfl_xor(sum, 16, 64);
    sum += __shfl_xor(sum, 32, 64);
    const float inv = 1.0f / sum;

    // O^T = V^T P^T: per pair of key tiles one MFMA for each 16-row block of dh (independent
    // accumulators), P^T straight from the score registers (key order 4kg..+3 of each tile,
    // matched by the V^T reads)
    constexpr int DT = DH / 16, NP = NT / 2;
    f32x4_t acc[DT];
#pragma unroll
    for (int dt = 0; dt < DT; ++dt) acc[dt] = f32x4_t{0.f, 0.f, 0.f, 0.f};
    bf16x8_t vf[DT];
    // (V^T fragments are read per pair, not double-buffered: the spare registers let two
    // blocks share a CU at 240 keys)
    auto read_v = [&](int p, bf16x8_t (&dst)[DT]) {
#pragma unroll
      for (int dt = 0; dt < DT; ++dt) {
        const uint2 v0 = *reinterpret_cast<const uint2*>(keys.vt(Vt, dt * 16 + l16, 2 * p, kg * 4));
        const uint2 v1 = *reinterpret_cast<const uint2*>(keys.vt(Vt, dt * 16 + l16, 2 * p + 1, kg * 4));
        dst[dt] = bitcast<bf16x8_t>(make_uint4(v0.x, v0.y, v1.x, v1.y));
      }
    };
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      if (MODE != 0 && (2 * p + 1 < tlo || 2 * p > thi)) continue;  // P = 0 on both tiles
      read_v(p, vf);
      uint4 pv;
      pv.x = pack_bf2(sc[2 * p][0], sc[2 * p][1]);
      pv.y = pack_bf2(sc[2 * p][2], sc[2 * p][3]);
      pv.z = pack_bf2(sc[2 * p + 1][0], sc[2 * p + 1][1]);
      pv.w = pack_bf2(sc[2 * p + 1][2], sc[2 * p + 1][3]);
      const bf16x8_t pb = bitcast<bf16x8_t>(pv);
      mfma_fence_begin();
#pragma unroll
      for (int dt = 0; dt < DT; ++dt) acc[dt] = mfma32(vf[dt], pb, acc[dt]);
      mfma_fence_end();
    }
    if ((NT & 1) && (MODE == 0 || NT - 1 <= thi)) {  // last key tile alone: single-rate k = 16
      constexpr int tt = NT - 1;
      uint2 pv;
      pv.x = pack_bf2(sc[tt][0], sc[tt][1]);
      pv.y = pack_bf2(sc[tt][2], sc[tt][3]);
#pragma unroll
      for (int dt = 0; dt < DT; ++dt) {
        const uint2 v0 = *reinterpret_cast<const uint2*>(keys.vt(Vt, dt * 16 + l16, tt, kg * 4));
        acc[dt] = mfma16k16(bitcast<bf16x4_t>(v0), bitcast<bf16x4_t>(pv), acc[dt]);
      }
    }
    if (valid) {
#pragma unroll
      for (int dt = 0; dt < DT; ++dt) {
        uint2 pk;
        pk.x = pack_bf2(acc[dt][0] * inv, acc[dt][1] * inv);
        pk.y = pack_bf2(acc[dt][2] * inv, acc[dt][3] * inv);
        *reinterpret_cast<uint2*>(o + (size_t)r * C + h * DH + dt * 16 + kg * 4) = pk;
        if (want_amax)
          omax = fmaxf(omax, fmaxf(fmaxf(fabsf(acc[dt][0]), fabsf(acc[dt][1])),
                                   fmaxf(fabsf(acc[dt][2]), fabsf(acc[dt][3]))) * inv);
      }
    }
  }
  // max |O| of this wavefront's rows (the loop bound is uniform per wavefront)
  return want_amax ? wave_max(omax) : 0.f;
}

// At up to 240 keys the kernel fits 128 VGPRs: 4 wavefronts per SIMD, two blocks per CU.  The
// key masks of the decoupled patterns take a few more registers at 240 keys and dh = 64.
template <int NT, int MODE>
constexpr int attn_clip_waves_per_simd() { return NT <= 4 || (NT <= 15 && MODE == 0) ? 4 : 3; }
// Threads of a clip attention block: 16 wavefronts where the kernel fits 4 per SIMD and a
// window has more query tiles than 8 wavefronts take in one pass, so that a full window's
// tiles (the longest blocks of the launch) run in one pass; otherwise 8.
template <int NT, int MODE>
constexpr int attn_clip_threads() { return attn_clip_waves_per_simd<NT, MODE>() == 4 && NT > 8 ? 1024 : ATT_THREADS; }

template <int DH, int NT, int MODE>
__global__ void __launch_bounds__((attn_clip_threads<NT, MODE>()), (attn_clip_waves_per_simd<NT, MODE>())) attn_clip_kernel(Geo g, int C, int heads, const bf16* __restrict__ q,
                                                                const bf16* __restrict__ kmat,
                                                                const bf16* __restrict__ vtmat,
                                                                const int32_t* __restrict__ idx,
                                                                const int32_t* __restrict__ woff,
                                                                const int32_t* __restrict__ worder,
                                                                bf16* __restrict__ o, float* __restrict__ amax_o) {
  constexpr int SP = NT * 16, CH = DH / 8, SPV = attn_vt_stride(SP);
  extern __shared__ __align__(16) bf16 att_lds[];
  bf16* Ks = att_lds;            // [SP][DH], swizzled chunks
  bf16* Vt = att_lds + SP * DH;  // [DH][SPV]
  // (window, head) work in order of decreasing query count; ATT_SPLIT blocks per (window,
  // head), block `part` taking query tiles 8 part + wv, then every 8 ATT_SPLIT-th, so a
  // window with more than 8 query tiles spreads over several CUs
  const int part = blockIdx.x % ATT_SPLIT, wh_ = blockIdx.x / ATT_SPLIT;
  const int rank = wh_ / heads, h = wh_ - rank * heads;
  const int w = worder[rank];
  const int q0 = woff[w], nqw = woff[w + 1] - q0;
  constexpr int NTHR = attn_clip_threads<NT, MODE>(), QW = NTHR / 64;  // query tiles per pass
  if (QW * part * 16 >= nqw) return;    // uniform per block
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  bf16x8_t qnext[DH / 32];
  if ((QW * part + wv) * 16 < nqw) attn_load_q<DH>(q, idx, q0, nqw, C, h, QW * part + wv, qnext);
  attn_dma<CH, true, NTHR>(kmat + ((size_t)w * heads + h) * SP * DH, Ks, SP * DH * 2);
  attn_dma<CH, false, NTHR>(vtmat + ((size_t)w * heads + h) * DH * SPV, Vt, DH * SPV * 2);
  asm volatile("s_waitcnt vmcnt(0)\n\ts_barrier" ::: "memory");
  const float wmx = attn_query_tiles<DH, NT, ClipKeys<NT, SPV>, MODE, QW * ATT_SPLIT>(
      Ks, Vt, ClipKeys<NT, SPV>{g.S}, C, h, q, idx, q0, nqw, o, qnext, amax_o != nullptr,
      KeyMask{g.wh * g.ww, w * g.S}, QW * part);
  if (amax_o) {
    // max |O| of the block into the per-call slot that scales O for an FP8 projection: one
    // atomic per block, skipped when the slot already holds more (non-negative floats order
    // like their bits)
    __shared__ float wred[NTHR / 64];
    if ((threadIdx.x & 63) == 0) wred[wv] = wmx;
    __syncthreads();
    if (threadIdx.x == 0) {
      float m = 0.f;
      for (int i = 0; i < NTHR / 64; ++i) m = fmaxf(m, wred[i]);
      if (m > 0.f && m > *reinterpret_cast<volatile float*>(amax_o))
        atomicMax(reinterpret_cast<unsigned int*>(amax_o), __float_as_uint(m));
    }
  }
}

// Temporal blocks of a decoupled network: a query sees only the wt keys at its own token
// position in the frames of its window (keys s mod A + f A), so there are no key tiles to
// multiply.  One block per (window, head), as in attn_clip_kernel: V^T of the window is
// staged in LDS, and four lanes per query each take DH/4 channels -- of Q and of the key rows
// (16-byte loads from global memory, all issued before the first product), combining their
// partial scores with two shuffles, and of O, read from the V^T columns.  Scores are in
// base 2 (Q carries log2(e) / sqrt(dh)).
template <int DH>
__global__ void __launch_bounds__(ATT_THREADS) attn_temporal_kernel(Geo g, int C, int heads, int Spad,
                                                                    const bf16* __restrict__ q,
                                                                    const bf16* __restrict__ kmat,
                                                                    const bf16* __restrict__ vtmat,
                                                                    const int32_t* __restrict__ idx,
                                                                    const int32_t* __restrict__ woff,
                                                                    const int32_t* __restrict__ worder,
                                                                    bf16* __restrict__ o, float* __restrict__ amax_o) {
  constexpr int DPL = DH / 4, NV = DPL / 8;  // channels per lane, 16-byte vectors per lane
  const int spv = attn_vt_stride(Spad);
  const int rank = blockIdx.x / heads, h = blockIdx.x - rank * heads;
  const int w = worder[rank];
  const int q0 = woff[w], nqw = woff[w + 1] - q0;
  if (nqw == 0) return;
  extern __shared__ __align__(16) bf16 att_lds[];
  bf16* Vt = att_lds;  // [DH][spv]
  attn_dma<DH / 8, false>(vtmat + ((size_t)w * heads + h) * DH * spv, Vt, DH * spv * 2);
  asm volatile("s_waitcnt vmcnt(0)\n\ts_barrier" ::: "memory");  // every thread, once
  const int A = g.wh * g.ww, part = threadIdx.x & 3;
  const bf16* kb = kmat + ((size_t)w * heads + h) * Spad * DH + part * DPL;
  float omax = 0.f;
  for (int qi = threadIdx.x >> 2; qi < nqw; qi += ATT_THREADS / 4) {  // uniform per 4 lanes
    const int r = q0 + qi;
    const int n = idx[r];
    const int kpos = (n - w * g.S) % A;
    u16x8_t qu[NV], ku[8][NV];
#pragma unroll
    for (int v = 0; v < NV; ++v)
      qu[v] = *reinterpret_cast<const u16x8_t*>(q + (size_t)n * C + h * DH + part * DPL + 8 * v);
#pragma unroll
    for (int f = 0; f < 8; ++f)
#pragma unroll
      for (int v = 0; v < NV; ++v)
        ku[f][v] = f < g.wt ? *reinterpret_cast<const u16x8_t*>(kb + (size_t)(kpos + f * A) * DH + 8 * v)
                            : u16x8_t{};
    float sc[8];
    float mx = -INFINITY;
#pragma unroll
    for (int f = 0; f < 8; ++f) {
      float d = -INFINITY;
      if (f < g.wt) {
        float acc = 0.f;
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
          for (int e = 0; e < 8; ++e) acc = fmaf(bf2f(qu[v][e]), bf2f(ku[f][v][e]), acc);
        acc += __shfl_xor(acc, 1, 64);
        acc += __shfl_xor(acc, 2, 64);
        d = acc;
      }
      sc[f] = d;
      mx = fmaxf(mx, d);
    }
    float sum = 0.f;
#pragma unroll
    for (int f = 0; f < 8; ++f) {
      const float p = f < g.wt ? __builtin_amdgcn_exp2f(sc[f] - mx) : 0.f;
      sc[f] = p;
      sum += p;
    }
    const float inv = 1.0f / sum;
    float ov[DPL];
#pragma unroll
    for (int e = 0; e < DPL; ++e) ov[e] = 0.f;
#pragma unroll
    for (int f = 0; f < 8; ++f) {
      if (f < g.wt) {
        const bf16* vc = Vt + (size_t)(part * DPL) * spv + kpos + f * A;
#pragma unroll
        for (int e = 0; e < DPL; ++e) ov[e] = fmaf(sc[f], bf2f(vc[(size_t)e * spv]), ov[e]);
      }
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      uint4 pk;
      pk.x = pack_bf2(ov[8 * v + 0] * inv, ov[8 * v + 1] * inv);
      pk.y = pack_bf2(ov[8 * v + 2] * inv, ov[8 * v + 3] * inv);
      pk.z = pack_bf2(ov[8 * v + 4] * inv, ov[8 * v + 5] * inv);
      pk.w = pack_bf2(ov[8 * v + 6] * inv, ov[8 * v + 7] * inv);
      *reinterpret_cast<uint4*>(o + (size_t)r * C + h * DH + part * DPL + 8 * v) = pk;
    }
    if (amax_o)
#pragma unroll
      for (int e = 0; e < DPL; ++e) omax = fmaxf(omax, fabsf(ov[e]) * inv);
  }
  if (amax_o) {
    const float wmx = wave_max(omax);
    __shared__ float wred[ATT_THREADS / 64];
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) wred[wv] = wmx;
    __syncthreads();
    if (threadIdx.x == 0) {
      float m = 0.f;
      for (int i = 0; i < ATT_THREADS / 64; ++i) m = fmaxf(m, wred[i]);
      if (m > 0.f && m > *reinterpret_cast<volatile float*>(amax_o))
        atomicMax(reinterpret_cast<unsigned int*>(amax_o), __float_as_uint(m));
    }
  }
}

// Stream mode: the keys of window (request r, window wl) are that window's tokens in the
// request's cached frames (oldest first) and in the new frame.  Each frame is a block of SFP
// key slots (its SF tokens, then padding); K of a frame is a contiguous [SF][dh] run of its
// ring slot and arrives by direct loads, V^T of a frame ([dh][SFP] in the ring) is copied
// into a frame-major LDS layout with rows padded to VST; frames that do not exist yet get
// zero V^T (their keys score -inf).
template <int SF>
struct RingShape {
  static constexpr int SFP = (SF + 15) / 16 * 16;  // key slots per frame (whole 16-key tiles)
  static constexpr int VST = SFP + 8;               // LDS row stride of V^T: odd 16-byte chunks
};

template <int DH, int SF, int NF>
__global__ void __launch_bounds__(ATT_THREADS) attn_ring_kernel(StreamTable tab, int C, int heads, int nwin_f,
                                                                const bf16* __restrict__ q,
                                                                const int32_t* __restrict__ idx,
                                                                const int32_t* __restrict__ woff,
                                                                const int32_t* __restrict__ worder,
                                                                bf16* __restrict__ o) {
  constexpr int SFP = RingShape<SF>::SFP, VST = RingShape<SF>::VST, NT = NF * SFP / 16, CH = DH / 8;
  extern __shared__ __align__(16) bf16 att_lds[];
  bf16* Ks = att_lds;                 // [NT*16][DH], swizzled chunks, key = frame * SFP + token
  bf16* Vt = att_lds + NT * 16 * DH;  // [NF][DH][VST]
  const int rank = blockIdx.x / heads, h = blockIdx.x - rank * heads;
  const int w = worder[rank];
  const int q0 = woff[w], nqw = woff[w + 1] - q0;
  if (nqw == 0) return;
  const int r = w / nwin_f, wl = w - r * nwin_f;
  const int np = pick(tab.npast, r), hd = pick(tab.head, r), nT = pick(tab.T, r);
  const bf16* kr = pick(tab.k, r);
  const bf16* vr = pick(tab.v, r);
  const int t = threadIdx.x, wv = t >> 6;
  bf16x8_t qnext[DH / 32];
  if (wv * 16 < nqw) attn_load_q<DH>(q, idx, q0, nqw, C, h, wv, qnext);
  for (int f = 0; f <= np; ++f) {
    const int slot = (hd - np + f + nT) % nT;
    attn_dma<CH, true>(kr + (size_t)slot * tab.slot_stride + ((size_t)wl * heads + h) * SF * DH, Ks + f * SFP * DH,
                       SF * DH * 2);
    const bf16* vsrc = vr + (size_t)slot * tab.vslot_stride + ((size_t)wl * heads + h) * DH * SFP;
    for (int c = t; c < DH * SFP / 8; c += ATT_THREADS) {
      const int d = c / (SFP / 8), ch = c - d * (SFP / 8);
      *reinterpret_cast<uint4*>(Vt + (f * DH + d) * VST + ch * 8) = *reinterpret_cast<const uint4*>(vsrc + d * SFP + ch * 8);
    }
  }
  for (int e = t; e < (NF - 1 - np) * DH * VST / 8; e += ATT_THREADS)
    *reinterpret_cast<uint4*>(Vt + (np + 1) * DH * VST + e * 8) = make_uint4(0, 0, 0, 0);
  asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)\n\ts_barrier" ::: "memory");
  attn_query_tiles<DH, NT>(Ks, Vt, RingKeys<DH, SF, SFP, VST>{np}, C, h, q, idx, q0, nqw, o, qnext, false);
}

int ring_vt_frame_stride(int sf) { return (sf + 15) / 16 * 16; }

bool attn_ring_supported(int dh, int sf, int nf) {
  return (dh == 32 || dh == 64) && (((sf == 45 || sf == 60) && (nf == 5 || nf == 1)) || (sf == 64 && nf == 1));
}

void launch_attn_ring(const StreamTable& tab, const Geo& g, int C, int heads, int nf, const bf16* q, const int32_t* idx,
                      const int32_t* woff, const int32_t* worder, bf16* o, hipStream_t s) {
  const int dh = C / heads, sf = g.S;
  const int nwin_f = g.nwh * g.nww;
#define DR_ATTN_RING(DH_, SF_, NF_)                                                                           \
  if (dh == DH_ && sf == SF_ && nf == NF_) {                                                                  \
    constexpr int SFP = RingShape<SF_>::SFP, VST = RingShape<SF_>::VST;                                       \
    const size_t lds = (size_t)NF_ * SFP * DH_ * 2 + (size_t)NF_ * DH_ * VST * 2;                             \
    static bool attr = false;                                                                                 \
    if (!attr) {                                                                                              \
      if (lds > 65536)                                                                                        \
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(attn_ring_kernel<DH_, SF_, NF_>),             \
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);                      \
      attr = true;                                                                                            \
    }                                                                                                         \
    attn_ring_kernel<DH_, SF_, NF_><<<g.nwin * heads, ATT_THREADS, lds, s>>>(tab, C, heads, nwin_f, q, idx, woff, \
                                                                             worder, o);                      \
    return;                                                                                                   \
  }
  DR_ATTN_RING(64, 45, 5)
  DR_ATTN_RING(64, 60, 5)
  DR_ATTN_RING(32, 45, 5)
  DR_ATTN_RING(32, 60, 5)
  DR_ATTN_RING(32, 64, 1)
  DR_ATTN_RING(64, 64, 1)
  DR_ATTN_RING(64, 45, 1)
  DR_ATTN_RING(64, 60, 1)
  DR_ATTN_RING(32, 45, 1)
  DR_ATTN_RING(32, 60, 1)
#undef DR_ATTN_RING
}

// Stream mode, temporal block of a decoupled network: the query at position p of window
// (request r, window wl) attends to the keys at position p of that window in the request's
// cached frames (oldest first) and in the new frame.  A handful of keys per query, so no
// matrix cores: four lanes per query, DH/4 channels each, an online softmax over the frames.
// K rows of a position are contiguous in the ring; V^T is read at stride sfp, which the
// neighbouring queries of a wave share cache lines of.
template <int DH>
__global__ void __launch_bounds__(ATT_THREADS) attn_ring_temporal_kernel(StreamTable tab, int C, int heads, int nwin_f,
                                                                         int sf, const bf16* __restrict__ q,
                                                                         const int32_t* __restrict__ idx,
                                                                         const int32_t* __restrict__ woff,
                                                                         const int32_t* __restrict__ worder,
                                                                         bf16* __restrict__ o) {
  constexpr int DPL = DH / 4, NV = DPL / 8;
  const int rank = blockIdx.x / heads, h = blockIdx.x - rank * heads;
  const int w = worder[rank];
  const int q0 = woff[w], nqw = woff[w + 1] - q0;
  if (nqw == 0) return;
  const int r = w / nwin_f, wl = w - r * nwin_f;
  const int np = pick(tab.npast, r), hd = pick(tab.head, r), nT = pick(tab.T, r);
  const int part = threadIdx.x & 3;
  const bf16* kb = pick(tab.k, r) + ((size_t)wl * heads + h) * sf * DH + part * DPL;
  const bf16* vb = pick(tab.v, r) + (((size_t)wl * heads + h) * DH + part * DPL) * tab.sfp;
  for (int qi = threadIdx.x >> 2; qi < nqw; qi += ATT_THREADS / 4) {  // uniform per 4 lanes
    const int row = q0 + qi;
    const int n = idx[row];
    const int p = n - w * sf;
    u16x8_t qu[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v)
      qu[v] = *reinterpret_cast<const u16x8_t*>(q + (size_t)n * C + h * DH + part * DPL + 8 * v);
    float m = -INFINITY, l = 0.f, ov[DPL];
#pragma unroll
    for (int e = 0; e < DPL; ++e) ov[e] = 0.f;
    for (int f = 0; f <= np; ++f) {
      const int slot = (hd - np + f + nT) % nT;
      const bf16* kf = kb + (size_t)slot * tab.slot_stride + (size_t)p * DH;
      float acc = 0.f;
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const u16x8_t ku = *reinterpret_cast<const u16x8_t*>(kf + 8 * v);
#pragma unroll
        for (int e = 0; e < 8; ++e) acc = fmaf(bf2f(qu[v][e]), bf2f(ku[e]), acc);
      }
      acc += __shfl_xor(acc, 1, 64);
      acc += __shfl_xor(acc, 2, 64);
      const float mn = fmaxf(m, acc);
      const float a = __builtin_amdgcn_exp2f(m - mn), pe = __builtin_amdgcn_exp2f(acc - mn);
      l = fmaf(l, a, pe);
      m = mn;
      const bf16* vf = vb + (size_t)slot * tab.vslot_stride + p;
#pragma unroll
      for (int e = 0; e < DPL; ++e) ov[e] = fmaf(pe, bf2f(vf[(size_t)e * tab.sfp]), ov[e] * a);
    }
    const float inv = 1.0f / l;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      uint4 pk;
      pk.x = pack_bf2(ov[8 * v + 0] * inv, ov[8 * v + 1] * inv);
      pk.y = pack_bf2(ov[8 * v + 2] * inv, ov[8 * v + 3] * inv);
      pk.z = pack_bf2(ov[8 * v + 4] * inv, ov[8 * v + 5] * inv);
      pk.w = pack_bf2(ov[8 * v + 6] * inv, ov[8 * v + 7] * inv);
      *reinterpret_cast<uint4*>(o + (size_t)row * C + h * DH + part * DPL + 8 * v) = pk;
    }
  }
}

bool attn_ring_temporal_supported(int dh) { return dh == 32 || dh == 64; }

void launch_attn_ring_temporal(const StreamTable& tab, const Geo& g, int C, int heads, const bf16* q,
                               const int32_t* idx, const int32_t* woff, const int32_t* worder, bf16* o,
                               hipStream_t s) {
  const int dh = C / heads, nwin_f = g.nwh * g.nww;
  if (dh == 64)
    attn_ring_temporal_kernel<64><<<g.nwin * heads, ATT_THREADS, 0, s>>>(tab, C, heads, nwin_f, g.S, q, idx, woff,
                                                                         worder, o);
  else if (dh == 32)
    attn_ring_temporal_kernel<32><<<g.nwin * heads, ATT_THREADS, 0, s>>>(tab, C, heads, nwin_f, g.S, q, idx, woff,
                                                                         worder, o);
}

int attn_clip_vt_stride(int spad) { return attn_vt_stride(spad); }

void launch_attn_clip(const Geo& g, int C, int heads, int Spad, const bf16* q, const bf16* k, const bf16* vt,
                      const int32_t* idx, const int32_t* woff, const int32_t* worder, bf16* o, float* amax_o,
                      int mode, hipStream_t s) {
  const int dh = C / heads;
  const int nt = Spad / 16;
  if (mode == 2) {  // temporal blocks of a decoupled network
    const size_t vlds = (size_t)dh * attn_vt_stride(Spad) * 2;  // V^T of one (window, head)
    if (dh == 64)
      attn_temporal_kernel<64><<<g.nwin * heads, ATT_THREADS, vlds, s>>>(g, C, heads, Spad, q, k, vt, idx, woff,
                                                                         worder, o, amax_o);
    else if (dh == 32)
      attn_temporal_kernel<32><<<g.nwin * heads, ATT_THREADS, vlds, s>>>(g, C, heads, Spad, q, k, vt, idx, woff,
                                                                         worder, o, amax_o);
    return;
  }
  const size_t lds = (size_t)Spad * dh * 2 + (size_t)dh * attn_vt_stride(Spad) * 2;
#define DR_ATTN_CLIP(DH_, NT_, MODE_)                                                                   \
  if (dh == DH_ && nt == NT_ && mode == MODE_) {                                                        \
    static bool attr = false;                                                                           \
    if (!attr) {                                                                                        \
      if (lds > 65536)                                                                                  \
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(attn_clip_kernel<DH_, NT_, MODE_>),     \
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);                \
      attr = true;                                                                                      \
    }                                                                                                   \
    attn_clip_kernel<DH_, NT_, MODE_><<<g.nwin * heads * ATT_SPLIT, attn_clip_threads<NT_, MODE_>(), lds, s>>>(g, C, heads, q, k, vt, idx, woff, \
                                                                               worder, o, amax_o);      \
    return;                                                                                             \
  }
#define DR_ATTN_CLIP_MODES(DH_, NT_) DR_ATTN_CLIP(DH_, NT_, 0) DR_ATTN_CLIP(DH_, NT_, 1)
  DR_ATTN_CLIP_MODES(32, 4)
  DR_ATTN_CLIP_MODES(64, 4)
  DR_ATTN_CLIP_MODES(64, 15)
  DR_ATTN_CLIP_MODES(64, 19)
  DR_ATTN_CLIP_MODES(32, 15)
  DR_ATTN_CLIP_MODES(32, 19)
#undef DR_ATTN_CLIP_MODES
#undef DR_ATTN_CLIP
}

bool attn_bf16_supported(int dh, int spad) {
  const int nt = spad / 16;
  return (dh == 32 || dh == 64) && (nt == 4 || nt == 15 || nt == 19);
}

}  // namespace dr
