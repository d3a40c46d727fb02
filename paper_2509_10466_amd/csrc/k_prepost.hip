// Camera-resolution pre- and post-processing around the network (the thesis runs its models
// at half the camera resolution and scales the outputs by 2, and cuts the selected objects'
// masks out of the camera frame: Methods, "Object Control" and "Performance Optimisations --
// Upscaling").  Definitions, with the readings the thesis leaves open:
//
//   prep: camera frame u8 BGRA [H][W][4] and per-object instance masks u8 [K][H][W]
//     mask_full[y][x] = 1 if a selected instance covers a pixel within the square window of
//                       radius r around (y, x) (the union, dilated; outside pixels ignored)
//     mask_low[y][x]  = any of mask_full over the 2 x 2 block (2y.., 2x..)
//     frame_low[y][x] = mean of the block's RGB / 255, float32
//   post: out[y][x] = mask_full[y][x] ? (u8 B, G, R of pred_low[y/2][x/2], alpha of bgra)
//                                     : bgra[y][x] (bit for bit)
//     u8(v) = clamp(rint(255 v), 0, 255) with the product rounded in float32.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>

#include "dr_internal.h"

using namespace dr;

namespace {

constexpr int PP_TY = 32, PP_TX = 64;  // full-resolution output tile of one prep block
constexpr int PP_RMAX = 16;            // largest dilation radius
constexpr int PP_THREADS = 256;

// One block per PP_TY x PP_TX tile.  LDS: the selected-instance union over the tile plus an
// r-pixel halo, then its horizontal running max, then the tile's dilated mask.
__global__ void __launch_bounds__(PP_THREADS) prep_kernel(const uint8_t* __restrict__ bgra,
                                                          const uint8_t* __restrict__ inst, int K, uint32_t select,
                                                          int r, int H, int W, float* __restrict__ frame_low,
                                                          uint8_t* __restrict__ mask_low,
                                                          uint8_t* __restrict__ mask_full) {
  __shared__ uint8_t U[(PP_TY + 2 * PP_RMAX) * (PP_TX + 2 * PP_RMAX)];
  __shared__ uint8_t Hm[(PP_TY + 2 * PP_RMAX) * PP_TX];
  __shared__ uint8_t M[PP_TY * PP_TX];
  const int y0 = blockIdx.y * PP_TY, x0 = blockIdx.x * PP_TX;
  const int wy = PP_TY + 2 * r, wx = PP_TX + 2 * r;  // halo window
  const size_t plane = (size_t)H * W;
  for (int e = threadIdx.x; e < wy * wx; e += PP_THREADS) {
    const int yy = e / wx, xx = e - yy * wx;
    const int gy = y0 - r + yy, gx = x0 - r + xx;
    uint8_t u = 0;
    if (gy >= 0 && gy < H && gx >= 0 && gx < W) {
      const size_t p = (size_t)gy * W + gx;
      for (int k = 0; k < K; ++k)
        if ((select >> k) & 1u) u |= inst[k * plane + p] != 0;
    }
    U[e] = u;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < wy * PP_TX; e += PP_THREADS) {
    const int yy = e / PP_TX, x = e - yy * PP_TX;
    uint8_t m = 0;
    for (int d = 0; d <= 2 * r; ++d) m |= U[yy * wx + x + d];
    Hm[e] = m;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < PP_TY * PP_TX; e += PP_THREADS) {
    const int y = e / PP_TX, x = e - y * PP_TX;
    uint8_t m = 0;
    for (int d = 0; d <= 2 * r; ++d) m |= Hm[(y + d) * PP_TX + x];
    M[e] = m;
    const int gy = y0 + y, gx = x0 + x;
    if (gy < H && gx < W) mask_full[(size_t)gy * W + gx] = m;
  }
  __syncthreads();
  const int Wl = W / 2;
  for (int e = threadIdx.x; e < (PP_TY / 2) * (PP_TX / 2); e += PP_THREADS) {
    const int ly = e / (PP_TX / 2), lx = e - ly * (PP_TX / 2);
    const int gy = y0 + 2 * ly, gx = x0 + 2 * lx;  // H, W even: the whole 2 x 2 block is inside
    if (gy >= H || gx >= W) continue;
    const uint8_t ml = M[(2 * ly) * PP_TX + 2 * lx] | M[(2 * ly) * PP_TX + 2 * lx + 1] |
                       M[(2 * ly + 1) * PP_TX + 2 * lx] | M[(2 * ly + 1) * PP_TX + 2 * lx + 1];
    const uint2 a = *reinterpret_cast<const uint2*>(bgra + ((size_t)gy * W + gx) * 4);
    const uint2 b = *reinterpret_cast<const uint2*>(bgra + ((size_t)(gy + 1) * W + gx) * 4);
    // channel c of pixel word v: byte c (B = 0, G = 1, R = 2)
    auto ch = [](uint32_t v, int c) { return (int)((v >> (8 * c)) & 0xffu); };
    const size_t lo = (size_t)(gy / 2) * Wl + gx / 2;
    float* f = frame_low + lo * 3;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int s = ch(a.x, 2 - c) + ch(a.y, 2 - c) + ch(b.x, 2 - c) + ch(b.y, 2 - c);  // RGB order out
      f[c] = (float)s / 1020.0f;  // exact sum of four bytes, one rounding
    }
    mask_low[lo] = ml;
  }
}

__device__ __forceinline__ uint32_t to_u8(float v) {
  const float q = rintf(__fmul_rn(255.0f, v));
  return (uint32_t)fminf(fmaxf(q, 0.0f), 255.0f);
}

// Four pixels per thread (W % 4 == 0): one 16-byte load and store of BGRA.
__global__ void __launch_bounds__(256) post_kernel(const uint8_t* __restrict__ bgra, const float* __restrict__ pred_low,
                                                   const uint8_t* __restrict__ mask_full, int H, int W,
                                                   uint8_t* __restrict__ out) {
  const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;  // quad of pixels
  const size_t npix = (size_t)H * W;
  if (q * 4 >= npix) return;
  const size_t p0 = q * 4;
  const int y = (int)(p0 / W), x0 = (int)(p0 - (size_t)y * W);
  uint4 px = *reinterpret_cast<const uint4*>(bgra + p0 * 4);
  const uint32_t m4 = *reinterpret_cast<const uint32_t*>(mask_full + p0);
  uint32_t w[4] = {px.x, px.y, px.z, px.w};
  const int Wl = W / 2;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if ((m4 >> (8 * i)) & 0xffu) {
      const float* pr = pred_low + ((size_t)(y / 2) * Wl + (x0 + i) / 2) * 3;
      w[i] = to_u8(pr[2]) | (to_u8(pr[1]) << 8) | (to_u8(pr[0]) << 16) | (w[i] & 0xff000000u);
    }
  }
  *reinterpret_cast<uint4*>(out + p0 * 4) = make_uint4(w[0], w[1], w[2], w[3]);
}

#define PP_HIP_OK(ctx, expr)                                                                   \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess) return dr_fail(ctx, DR_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  const char* pa = static_cast<const char*>(a);
  const char* pb = static_cast<const char*>(b);
  return pa < pb + nb && pb < pa + na;
}

}  // namespace

extern "C" dr_status dr_prep_frame(dr_ctx* c, const uint8_t* bgra, const uint8_t* inst, int K, uint32_t select,
                                   int radius, int H, int W, float* frame_low, uint8_t* mask_low, uint8_t* mask_full,
                                   void* stream) {
  if (!c || !bgra || !frame_low || !mask_low || !mask_full || (K > 0 && !inst))
    return dr_fail(c, DR_EINVAL, "dr_prep_frame: null argument");
  if (K < 0 || K > 32) return dr_fail(c, DR_EINVAL, "dr_prep_frame: %d instance masks (0..32)", K);
  if (radius < 0 || radius > PP_RMAX) return dr_fail(c, DR_EINVAL, "dr_prep_frame: radius %d (0..%d)", radius, PP_RMAX);
  if (H <= 0 || W <= 0 || (H & 1) || (W & 1)) return dr_fail(c, DR_ESHAPE, "dr_prep_frame: frame %dx%d (even sizes)", H, W);
  if ((uintptr_t)bgra & 7) return dr_fail(c, DR_EINVAL, "dr_prep_frame: bgra must be 8-byte aligned");
  PP_HIP_OK(c, hipSetDevice(c->device));
  dim3 grid((W + PP_TX - 1) / PP_TX, (H + PP_TY - 1) / PP_TY);
  prep_kernel<<<grid, PP_THREADS, 0, (hipStream_t)stream>>>(bgra, inst, K, select, radius, H, W, frame_low, mask_low,
                                                            mask_full);
  PP_HIP_OK(c, hipGetLastError());
  return DR_OK;
}

extern "C" dr_status dr_post_frame(dr_ctx* c, const uint8_t* bgra, const float* pred_low, const uint8_t* mask_full,
                                   int H, int W, uint8_t* out, void* stream) {
  if (!c || !bgra || !pred_low || !mask_full || !out) return dr_fail(c, DR_EINVAL, "dr_post_frame: null argument");
  if (H <= 0 || W <= 0 || (H & 1) || (W & 3)) return dr_fail(c, DR_ESHAPE, "dr_post_frame: frame %dx%d (H even, W % 4 == 0)", H, W);
  if (((uintptr_t)bgra & 15) || ((uintptr_t)out & 15) || ((uintptr_t)mask_full & 3) || ((uintptr_t)pred_low & 3))
    return dr_fail(c, DR_EINVAL, "dr_post_frame: bgra/out must be 16-byte, mask 4-byte, pred 4-byte aligned");
  const size_t npix = (size_t)H * W;
  if (out != bgra && overlaps(out, npix * 4, bgra, npix * 4)) return dr_fail(c, DR_EINVAL, "dr_post_frame: out partially overlaps bgra");
  if (overlaps(out, npix * 4, mask_full, npix) || overlaps(out, npix * 4, pred_low, npix * 3))
    return dr_fail(c, DR_EINVAL, "dr_post_frame: out overlaps an input");
  PP_HIP_OK(c, hipSetDevice(c->device));
  const size_t quads = npix / 4;
  post_kernel<<<(unsigned)((quads + 255) / 256), 256, 0, (hipStream_t)stream>>>(bgra, pred_low, mask_full, H, W, out);
  PP_HIP_OK(c, hipGetLastError());
  return DR_OK;
}
