// Step 1 of the path: token flags and the gather lists of query tokens.
//
// A token is flagged when any pixel of its p x p patch is private (OR rule), i.e. when the
// cut-out of the private object (thesis, Methods, "Object Control") touches it.  Tokens are
// numbered window-major: window w = ((b*nT + a)*nwh + u)*nww + v, and inside a window
// s = (dt*wh + di)*ww + dj; token n = w*S + s.  All outputs are integers and are exact.
#include "dr_device.h"
#include "dr_internal.h"
#include "tokens_dev.h"

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

__global__ void __launch_bounds__(256) token_gather_kernel(Geo g, const uint8_t* __restrict__ flag,
                                                           const int32_t* __restrict__ wcount,
                                                           int32_t* __restrict__ idx,
                                                           int32_t* __restrict__ woff,
                                                           int32_t* __restrict__ nq) {
  gather_window(g, blockIdx.x, flag, wcount, idx, woff, nq);
}

__global__ void __launch_bounds__(1024) window_order_kernel(int nwin, int S, int N, const int32_t* __restrict__ wcount,
                                                            const uint8_t* __restrict__ flag,
                                                            int32_t* __restrict__ order, int32_t* __restrict__ tiles,
                                                            int32_t* __restrict__ ntiles) {
  __shared__ int hist[ORDER_MAX_S + 1];
  __shared__ int start[ORDER_MAX_S + 1];
  __shared__ int nlist[2];
  order_windows<1024>(nwin, S, N, wcount, flag, order, tiles, ntiles, hist, start, nlist);
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
