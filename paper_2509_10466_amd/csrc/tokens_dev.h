// Device bodies of the token-list kernels (k_tokens.hip), shared with the fused launch of the
// BF16 path that runs them beside the patch embedding (k_pixels.hip).
#pragma once

#include "dr_device.h"
#include "dr_internal.h"

namespace dr {

// One workgroup per window: offset = flagged tokens in earlier windows, then an ordered
// compaction of this window's flagged tokens into idx (ranks from wavefront ballots).
// (the body of the kernel for window w; a block of 256 threads)
__device__ __forceinline__ void gather_window(const Geo& g, int w, const uint8_t* __restrict__ flag,
                                              const int32_t* __restrict__ wcount, int32_t* __restrict__ idx,
                                              int32_t* __restrict__ woff, int32_t* __restrict__ nq) {
  __shared__ int red[4];
  __shared__ int wave_tot[4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int part = 0;
  for (int k = threadIdx.x; k < w; k += blockDim.x) part += wcount[k];
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) part += __shfl_xor(part, o, 64);
  if (lane == 0) red[wv] = part;
  __syncthreads();
  const int off = red[0] + red[1] + red[2] + red[3];
  int running = 0;
  for (int base = 0; base < g.S; base += 256) {
    const int s = base + threadIdx.x;
    const int f = (s < g.S) ? flag[w * g.S + s] : 0;
    const unsigned long long bal = __ballot(f);
    const int below = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) wave_tot[wv] = __popcll(bal);
    __syncthreads();
    int before = running;
    for (int k = 0; k < wv; ++k) before += wave_tot[k];
    if (f) idx[off + before + below] = w * g.S + s;
    running += wave_tot[0] + wave_tot[1] + wave_tot[2] + wave_tot[3];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    woff[w] = off;
    if (w == g.nwin - 1) {
      woff[g.nwin] = off + running;
      nq[0] = off + running;
    }
  }
}

// Windows listed by decreasing query count (a counting sort over counts 0..S, one block):
// the attention kernel takes its (window, head) work in this order, so the longest windows
// start first and the short ones fill in behind them.  Windows of equal count may come in
// any order; that only changes scheduling, never a result.
constexpr int ORDER_MAX_S = 2048;

//
// The same block lists the Q/K/V GEMM's row tiles of ROW_TILE tokens that have work: tiles
// holding a flagged token (their Q rows are read) and tiles touching a window with queries
// (their K/V rows are read), so that the GEMM launches no block for the others.
static_assert(ROW_TILE == 64, "the flag scan reads a tile as four 16-byte words");

// (the body of the one-block kernel, at most MAXT threads; hist and start hold S + 1 ints
// each in LDS, nlist 2)
template <int MAXT>
__device__ __forceinline__ void order_windows(int nwin, int S, int N, const int32_t* __restrict__ wcount,
                                              const uint8_t* __restrict__ flag, int32_t* __restrict__ order,
                                              int32_t* __restrict__ tiles, int32_t* __restrict__ ntiles, int* hist,
                                              int* start, int* nlist) {
  for (int c = threadIdx.x; c <= S; c += blockDim.x) hist[c] = 0;
  if (threadIdx.x < 2) nlist[threadIdx.x] = 0;
  __syncthreads();
  const int mt = (N + ROW_TILE - 1) / ROW_TILE;
  for (int rt = threadIdx.x; rt < mt; rt += blockDim.x) {
    const int r0 = rt * ROW_TILE, r1 = min(N, r0 + ROW_TILE);  // rows [r0, r1)
    bool kv = false;
    for (int w = r0 / S; w <= (r1 - 1) / S; ++w) kv |= wcount[w] > 0;
    bool q = false;
    if (r1 - r0 == ROW_TILE) {  // whole tile: four independent 16-byte loads (64-byte aligned)
      const uint4* f4 = reinterpret_cast<const uint4*>(flag + r0);
      uint4 a = f4[0], b = f4[1], c = f4[2], d = f4[3];
      q = ((a.x | a.y | a.z | a.w) | (b.x | b.y | b.z | b.w) | (c.x | c.y | c.z | c.w) | (d.x | d.y | d.z | d.w)) != 0;
    } else {
      for (int r = r0; r < r1; ++r) q |= flag[r] != 0;
    }
    if (q) tiles[atomicAdd(&nlist[0], 1)] = rt;
    if (kv) tiles[mt + atomicAdd(&nlist[1], 1)] = rt;
  }
  for (int w = threadIdx.x; w < nwin; w += blockDim.x) atomicAdd(&hist[wcount[w]], 1);
  __syncthreads();
  // start[c] = number of windows with more than c queries: an exclusive scan of the counts
  // taken from c = S down.  Thread t sums a run of `per` consecutive positions of that order,
  // the run totals are scanned in LDS (log2(blockDim) steps), then each thread writes its
  // run's starts -- one serial pass over S + 1 counts had been the longest thread of the
  // launch.
  __shared__ int runsum[MAXT];
  const int n = S + 1, per = (n + (int)blockDim.x - 1) / (int)blockDim.x;
  int tot = 0;
  for (int k = 0; k < per; ++k) {
    const int p = (int)threadIdx.x * per + k;
    if (p < n) tot += hist[S - p];
  }
  runsum[threadIdx.x] = tot;
  __syncthreads();
  for (int off = 1; off < (int)blockDim.x; off <<= 1) {
    const int v = (int)threadIdx.x >= off ? runsum[threadIdx.x - off] : 0;
    __syncthreads();
    runsum[threadIdx.x] += v;
    __syncthreads();
  }
  int run = threadIdx.x ? runsum[threadIdx.x - 1] : 0;
  for (int k = 0; k < per; ++k) {
    const int p = (int)threadIdx.x * per + k;
    if (p < n) {
      start[S - p] = run;
      run += hist[S - p];
    }
  }
  __syncthreads();
  for (int w = threadIdx.x; w < nwin; w += blockDim.x) order[atomicAdd(&start[wcount[w]], 1)] = w;
  if (threadIdx.x < 2) ntiles[threadIdx.x] = nlist[threadIdx.x];
}

}  // namespace dr
