// Step 1 of the path: token flags and the gather lists of query tokens.
//
// A token is flagged when any pixel of its p x p patch is private (OR rule), i.e. when the
// cut-out of the private object (thesis, Methods, "Object Control") touches it.  Tokens are
// numbered window-major: window w = ((b*nT + a)*nwh + u)*nww + v, and inside a window
// s = (dt*wh + di)*ww + dj; token n = w*S + s.  All outputs are integers and are exact.
#include "dr_device.h"
#include "dr_internal.h"

namespace dr {

// Pixel offset (in pixels, not channels) of the top-left pixel of token n.
__device__ __forceinline__ size_t token_pixel(const Geo& g, int n) {
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
  return (((size_t)b * g.T + t) * g.H + (size_t)g.P * i) * g.W + (size_t)g.P * j;
}

// Halo rule of the overlapping embedding and decoder (kernel 8, stride 4, padding 2): the
// token's footprint is rows 4i - 2 .. 4i + 5 and columns 4j - 2 .. 4j + 5, clipped to the
// frame.  Per row: the upper two mask bytes of the word left of the patch, the patch's word
// and the lower two bytes of the word right of it (each read only when inside the frame).
__device__ __forceinline__ int footprint_any(const Geo& g, const uint8_t* __restrict__ masks, size_t px) {
  const size_t plane = (size_t)g.H * g.W;
  const size_t in_plane = px % plane;
  const int y = (int)(in_plane / g.W), x = (int)(in_plane - (size_t)y * g.W);
  const size_t base = px - in_plane;
  uint32_t any = 0;
  for (int dy = -2; dy < 6; ++dy) {
    const int yy = y + dy;
    if (yy < 0 || yy >= g.H) continue;
    const uint8_t* row = masks + base + (size_t)yy * g.W;
    any |= *reinterpret_cast<const uint32_t*>(row + x);
    if (x > 0) any |= *reinterpret_cast<const uint32_t*>(row + x - 4) >> 16;
    if (x + 4 < g.W) any |= *reinterpret_cast<const uint32_t*>(row + x + 4) & 0xffffu;
  }
  return any != 0;
}

// One workgroup per window: flag its S tokens and count them.  halo: 0 = the token's own
// 4 x 4 patch, 1 = the 8 x 8 footprint of the overlapping embedding and decoder.
__global__ void __launch_bounds__(256) token_flags_kernel(Geo g, const uint8_t* __restrict__ masks,
                                                          int all, int halo, uint8_t* __restrict__ flag,
                                                          int32_t* __restrict__ wcount) {
  __shared__ int cnt;
  const int w = blockIdx.x;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  int local = 0;
  for (int s = threadIdx.x; s < g.S; s += blockDim.x) {
    const int n = w * g.S + s;
    int f = 1;
    if (!all && halo) {
      f = footprint_any(g, masks, token_pixel(g, n));
    } else if (!all) {
      const size_t px = token_pixel(g, n);
      uint32_t any = 0;
      // p == 4 and W % 4 == 0: each patch row is one aligned 32-bit word of mask bytes.
      for (int ky = 0; ky < 4; ++ky)
        any |= *reinterpret_cast<const uint32_t*>(masks + px + (size_t)ky * g.W);
      f = any != 0;
    }
    flag[n] = (uint8_t)f;
    local += f;
  }
  if (local) atomicAdd(&cnt, local);
  __syncthreads();
  if (threadIdx.x == 0) wcount[w] = cnt;
}

// One workgroup per window: offset = flagged tokens in earlier windows, then an ordered
// compaction of this window's flagged tokens into idx (ranks from wavefront ballots).
__global__ void __launch_bounds__(256) token_gather_kernel(Geo g, const uint8_t* __restrict__ flag,
                                                           const int32_t* __restrict__ wcount,
                                                           int32_t* __restrict__ idx,
                                                           int32_t* __restrict__ woff,
                                                           int32_t* __restrict__ nq) {
  __shared__ int red[4];
  __shared__ int wave_tot[4];
  const int w = blockIdx.x;
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

__global__ void __launch_bounds__(1024) window_order_kernel(int nwin, int S, int N, const int32_t* __restrict__ wcount,
                                                            const uint8_t* __restrict__ flag,
                                                            int32_t* __restrict__ order, int32_t* __restrict__ tiles,
                                                            int32_t* __restrict__ ntiles) {
  __shared__ int hist[ORDER_MAX_S + 1];
  __shared__ int start[ORDER_MAX_S + 1];
  __shared__ int nlist[2];
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
  if (threadIdx.x == 0) {
    int run = 0;
    for (int c = S; c >= 0; --c) {
      start[c] = run;
      run += hist[c];
    }
  }
  __syncthreads();
  for (int w = threadIdx.x; w < nwin; w += blockDim.x) order[atomicAdd(&start[wcount[w]], 1)] = w;
  if (threadIdx.x < 2) ntiles[threadIdx.x] = nlist[threadIdx.x];
}

bool window_order_supported(int S) { return S <= ORDER_MAX_S; }

void launch_window_order(const Geo& g, const int32_t* wcount, const uint8_t* flag, int32_t* order, int32_t* tiles,
                         int32_t* ntiles, hipStream_t s) {
  window_order_kernel<<<1, 1024, 0, s>>>(g.nwin, g.S, g.N, wcount, flag, order, tiles, ntiles);
}

void launch_token_flags(const Geo& g, const uint8_t* masks, int all, uint8_t* flag,
                        int32_t* wcount, hipStream_t s, int halo) {
  token_flags_kernel<<<g.nwin, 256, 0, s>>>(g, masks, all, halo, flag, wcount);
}

void launch_token_gather(const Geo& g, const uint8_t* flag, const int32_t* wcount, int32_t* idx,
                         int32_t* woff, int32_t* nq, hipStream_t s) {
  token_gather_kernel<<<g.nwin, 256, 0, s>>>(g, flag, wcount, idx, woff, nq);
}

}  // namespace dr
