// BF16 GEMM core for gfx950: C[m][n] = sum_k A[m][k] * W[n][k], FP32 accumulation on
// v_mfma_f32_16x16x32_bf16.
//
// Block = 64 WM WN threads (4 or 8 wavefronts) in a WM x WN grid; block tile BM tokens x BN
// output channels; K is consumed 64 at a time through an ST-stage ring in LDS.  Each stage holds the
// BM rows of A followed by the BN rows of W, 128 bytes (64 bf16) per row, and is filled by
// direct global->LDS loads (global_load_lds_dwordx4: each lane of a wavefront moves 16 bytes,
// lane i landing at byte 16*i of the wavefront's 1 KB destination, i.e. 8 rows per
// instruction) -- no VGPR staging, no LDS store instructions.  Stage kt+ST-1 is issued while
// stage kt is multiplied; a wavefront waits for its own loads of stage kt with an explicit
// vmcnt and the block barrier then makes every wavefront's loads visible.
//
// LDS layout: the 16-byte chunk c of row r sits at chunk position c ^ (r & 7).  The MFMA
// operand reads fetch 16 consecutive rows at one logical chunk; measured on gfx950 with the
// SQ_LDS_BANK_CONFLICT counter, this XOR pattern reads those 16 rows without bank conflicts
// (unswizzled 128-byte rows, 144-byte padded rows and an XOR with (r ^ (r >> 3)) & 7 all
// conflict).  The loads apply the same swizzle to the global addresses.
//
// MFMA operands: lane l supplies row (l % 16) of each operand with k values 8*(l/16)..+7 of
// the 32-wide k slice.  The W fragment is the MFMA's A operand, so result lane l holds output
// channels 4*(l/16)..+3 of token (l % 16) within the 16 x 16 fragment.  acc[i][j] covers
// tokens m0 + wm*TM + 16 i + (l % 16) and channels n0 + wn*TN + 16 j + 4 (l / 16) + e.
//
// Double-rate MFMA groups are fenced as everywhere in this library (scheduling barriers,
// then s_nop 7 after the group): a VALU write to a source VGPR of an in-flight
// v_mfma_f32_16x16x32_bf16 corrupts its product.
#pragma once

#include "dr_device.h"

namespace dr {

typedef uint16_t bf16_t;

__device__ __forceinline__ int lds_swz(int row) { return row & 7; }

__device__ __forceinline__ f32x4_t mfma_bf16_16x16x32(const bf16x8_t& a, const bf16x8_t& b, const f32x4_t& c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ void mfma_fence_begin() { __builtin_amdgcn_sched_barrier(0); }
__device__ __forceinline__ void mfma_fence_end() {
  __builtin_amdgcn_sched_barrier(0);
  asm volatile("s_nop 7" ::: "memory");
  __builtin_amdgcn_sched_barrier(0);
}

// Wait until at most N of this wavefront's vector-memory operations are outstanding and its
// LDS operations are done, then the block barrier.  Written as one asm statement with a
// memory clobber so that the compiler neither adds a full vmcnt(0) wait (as a fenced
// __syncthreads would) nor moves LDS accesses across the barrier.
template <int N>
__device__ __forceinline__ void vm_wait_barrier() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  asm volatile("s_waitcnt vmcnt(%0) lgkmcnt(0)\n\ts_barrier" ::"n"(N) : "memory");
}

__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

__device__ __forceinline__ void dma16(const void* gsrc, bf16_t* lds_dst) {
  __builtin_amdgcn_global_load_lds(gsrc, (__attribute__((address_space(3))) void*)lds_dst, 16, 0, 0);
}

template <int BM_, int BN_, int WM_, int WN_, int ST_>
struct GemmTile {
  static constexpr int BM = BM_, BN = BN_, WM = WM_, WN = WN_, ST = ST_;
  static constexpr int NW = WM * WN, THREADS = 64 * NW;  // wavefronts, threads per block
  static constexpr int TM = BM / WM, TN = BN / WN;  // wavefront tile
  static constexpr int FM = TM / 16, FN = TN / 16;  // 16 x 16 fragments per wavefront
  static constexpr int ROWS = BM + BN;              // LDS rows per stage
  static constexpr int LOADS = ROWS / (8 * NW);     // 1 KB loads per wavefront per stage
  static constexpr int STAGE = ROWS * 64;           // bf16 elements per stage
  static constexpr size_t LDS_BYTES = (size_t)ST * STAGE * 2;
  static_assert(NW == 4 || NW == 8, "4 or 8 wavefronts");
  static_assert(TM % 16 == 0 && TN % 16 == 0 && BM % 16 == 0, "fragment multiples");
  static_assert(ROWS % (8 * NW) == 0, "whole loads");
  static_assert(ST >= 2 && (ST - 2) * LOADS < 64, "vmcnt range");
};

// One block tile.  A: [M][K] rows (rows >= M are read from row M-1 and must be ignored by the
// caller), W: [*][K] rows n0 .. n0+BN-1; K a multiple of 64, M >= 1.  `lds` holds
// GemmTile::LDS_BYTES.  On return every wavefront has finished reading LDS only after the
// caller's next barrier.
// KC > 0: K = KC known at compile time (the k loop unrolled, its waits fixed); else K at run time.
template <class TL, int KC = 0>
__device__ __forceinline__ void gemm_core(const bf16_t* __restrict__ A, int M, int m0,
                                          const bf16_t* __restrict__ W, int n0, int K_, bf16_t* lds,
                                          f32x4_t (&acc)[TL::FM][TL::FN]) {
  const int K = KC ? KC : K_;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int wm = wv / TL::WN, wn = wv % TL::WN;
  const int l16 = lane & 15, kg = lane >> 4;

  static_for<TL::FM>([&](auto i) {
    static_for<TL::FN>([&](auto j) { acc[i][j] = f32x4_t{0.f, 0.f, 0.f, 0.f}; });
  });

  // global source of each of this lane's loads (fixed over K; advanced by 64 per stage)
  const bf16_t* src[TL::LOADS];
  static_for<TL::LOADS>([&](auto c) {
    const int row = (wv + TL::NW * c) * 8 + (lane >> 3);
    const int chunk = (lane & 7) ^ lds_swz(row);
    const bf16_t* base;
    if (row < TL::BM) {
      const int m = min(m0 + row, M - 1);
      base = A + (size_t)m * K;
    } else {
      base = W + (size_t)(n0 + row - TL::BM) * K;
    }
    src[c] = base + chunk * 8;
  });
  auto issue = [&](int kt, int buf) {
    bf16_t* dst = lds + buf * TL::STAGE;
    static_for<TL::LOADS>([&](auto c) { dma16(src[c] + kt * 64, dst + (wv + TL::NW * c) * 512); });
  };
  // per-lane LDS element offsets of the operand rows (chunk position applied per k slice)
  int arow[TL::FM], wrow[TL::FN];
  static_for<TL::FM>([&](auto i) { arow[i] = wm * TL::TM + 16 * i + l16; });
  static_for<TL::FN>([&](auto j) { wrow[j] = TL::BM + wn * TL::TN + 16 * j + l16; });

  const int nk = K / 64;
  static_for<TL::ST - 1>([&](auto s) {
    if (s < nk) issue(s, s);
  });
  auto stage = [&](int kt) {
    const int ahead = min(TL::ST - 2, nk - 1 - kt);  // later stages already in flight
    static_for<TL::ST - 1>([&](auto a) {
      if (a == ahead) vm_wait_barrier<a * TL::LOADS>();
    });
    if (kt + TL::ST - 1 < nk) issue(kt + TL::ST - 1, (kt + TL::ST - 1) % TL::ST);
    const bf16_t* sb = lds + (kt % TL::ST) * TL::STAGE;
    // both 32-wide k slices of the stage are read before the first MFMA group, so the
    // second slice's LDS latency hides behind the first group
    bf16x8_t af[2][TL::FM], wf[2][TL::FN];
    static_for<2>([&](auto kk) {
      static_for<TL::FM>([&](auto i) {
        const int c = (4 * kk + kg) ^ lds_swz(arow[i]);
        af[kk][i] = *reinterpret_cast<const bf16x8_t*>(sb + arow[i] * 64 + c * 8);
      });
      static_for<TL::FN>([&](auto j) {
        const int c = (4 * kk + kg) ^ lds_swz(wrow[j]);
        wf[kk][j] = *reinterpret_cast<const bf16x8_t*>(sb + wrow[j] * 64 + c * 8);
      });
    });
    static_for<2>([&](auto kk) {
      mfma_fence_begin();
      static_for<TL::FM>([&](auto i) {
        static_for<TL::FN>([&](auto j) { acc[i][j] = mfma_bf16_16x16x32(wf[kk][j], af[kk][i], acc[i][j]); });
      });
      mfma_fence_end();
    });
  };
  if constexpr (KC > 0)
    static_for<KC / 64>([&](auto kt) { stage(kt); });
  else
    for (int kt = 0; kt < nk; ++kt) stage(kt);
}

// Tile order: consecutive workgroups are dispatched round-robin over the 8 XCDs (each with
// its own L2).  Workgroup b runs on XCD b % 8; it is given row tile (k / nt) * 8 + b % 8 and
// column tile k % nt (k = b / 8), so each XCD owns every 8th row tile and computes all nt
// column tiles of a row tile back to back (its A rows are read into that XCD's L2 once), and
// the row tiles that exist for a data-dependent row count spread evenly over the XCDs.
// Grid: 8 * ceil(mt / 8) * nt workgroups; tiles with row >= mt exit.
__device__ __forceinline__ void xcd_tile(int b, int nt, int& rt, int& ct) {
  const int k = b >> 3;
  ct = k % nt;
  rt = (k / nt) * 8 + (b & 7);
}

__host__ __device__ constexpr int xcd_grid(int mt, int nt) { return 8 * ((mt + 7) / 8) * nt; }

}  // namespace dr
