// Weight loading: the flat FP32 parameter vector lives on the device, and every layout the
// kernels read (transposes, concatenations, the patch-embedding and decoder permutations, the
// bf16 copies, the LayerNorm affine parts folded into the following linear, the e4m3 copies
// with their per-tensor scales) is derived from it on the device.
//
// The derivation is a plan built once per network shape on the host: for every element of
// the FP32 arena the index of its source parameter, for every element of the bf16 arena the
// indices of its one or two factors, and for every folded bias one row descriptor.  Loading
// then runs a handful of gather / fold / quantise kernels on the caller's stream, so
// dr_load_params (parameters already on the device, as in a training loop) copies nothing
// through the host and, once the arenas exist, allocates nothing.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "dr_internal.h"

using namespace dr;

namespace dr {
bool fp8_supported(int C, int R);
}

#define HIP_OK(ctx, expr)                                                                                   \
  do {                                                                                                      \
    hipError_t e_ = (expr);                                                                                 \
    if (e_ != hipSuccess) return dr_fail(ctx, DR_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));     \
  } while (0)

// ------------------------------------------------------------------------------------------
// the plan
// ------------------------------------------------------------------------------------------
struct FoldRow {     // dst = sc * (bias + sum_i W[i] * beta[i]), accumulated in double
  int32_t dst;       // f32 arena element
  int32_t bias;      // parameter index of the bias, or -1 (none)
  int32_t w, w_si;   // parameter index of W[0] and the stride between W[i] and W[i+1]
  int32_t beta;      // parameter index of beta[0] (contiguous)
  int32_t n;
  double sc;
};

struct dr_wplan {
  int K = 0;                        // embedding / decoder kernel size of this plan
  size_t nparams = 0;
  std::vector<int32_t> m32;         // f32 arena: source parameter, -1 = 0
  std::vector<int32_t> m16a, m16b;  // bf16 arena: value = a * b * scale (see gather16_kernel)
  std::vector<FoldRow> folds;
  // arena offsets (elements)
  size_t ewT, eb, dbf, lnfg, lnfb, dw, db, dbo;
  size_t e16, d16, eo16, dwo16;
  struct Blk { size_t f[26]; size_t h[6]; size_t p[16]; };
  std::vector<Blk> blk;
  size_t p_ew, p_eb, p_lnfg, p_lnfb, p_dw, p_db;  // parameter offsets
};

void dr::dr_wplan_free(dr_wplan* p) { delete p; }

size_t dr::dr_nparams(const Net& n, int K) {
  const size_t C = n.C, R = n.R;
  return 2 * (C * 3 * K * K) + C + 3 + 2 * C + n.cfg.blocks * (4 * C * C + 2 * R * C + 9 * C + R);
}

static dr_wplan* build_plan(const Net& n, int K) {
  dr_wplan* pl = new dr_wplan();
  pl->K = K;
  const int C = n.C, R = n.R, L = n.cfg.blocks, P = n.P;
  const size_t CC = (size_t)C * C, RC = (size_t)R * C;
  // parameter offsets in blob order
  size_t o = 0;
  pl->p_ew = o; o += (size_t)C * 3 * K * K;
  pl->p_eb = o; o += C;
  pl->blk.resize(L);
  const size_t sizes[16] = {(size_t)C, (size_t)C, CC, (size_t)C, CC, (size_t)C, CC, (size_t)C,
                            CC, (size_t)C, (size_t)C, (size_t)C, RC, (size_t)R, RC, (size_t)C};
  for (int l = 0; l < L; ++l)
    for (int k = 0; k < 16; ++k) {
      pl->blk[l].p[k] = o;
      o += sizes[k];
    }
  pl->p_lnfg = o; o += C;
  pl->p_lnfb = o; o += C;
  pl->p_dw = o; o += (size_t)C * 3 * K * K;
  pl->p_db = o; o += 3;
  pl->nparams = o;

  std::vector<int32_t>& f = pl->m32;
  std::vector<int32_t>&a16 = pl->m16a, &b16 = pl->m16b;
  auto pad32 = [&] { while (f.size() % 64) f.push_back(-1); };  // 256-byte alignment
  auto pad16 = [&] {
    while (a16.size() % 128) {
      a16.push_back(-1);
      b16.push_back((int32_t)0x80000000u);
    }
  };
  auto copy = [&](size_t src, size_t nel) {
    const size_t off = f.size();
    for (size_t e = 0; e < nel; ++e) f.push_back((int32_t)(src + e));
    pad32();
    return off;
  };
  // T[i][part*out_each + o] = W_part[o][i] for W [out][in]
  auto transpose = [&](std::initializer_list<size_t> parts, int out_each, int in) {
    const size_t off = f.size();
    const int np = (int)parts.size(), out_total = out_each * np;
    f.resize(off + (size_t)in * out_total);
    int pi = 0;
    for (size_t src : parts) {
      for (int oo = 0; oo < out_each; ++oo)
        for (int i = 0; i < in; ++i) f[off + (size_t)i * out_total + pi * out_each + oo] = (int32_t)(src + (size_t)oo * in + i);
      ++pi;
    }
    pad32();
    return off;
  };
  // second-factor code of the bf16 map: bit 31 set = no factor, bits 29-30 = scale class
  // (0: 1, 1: the softmax scale of Q, 2: 1/sqrt 2 of the GELU), bits 0-28 = factor index
  auto fcode = [](int64_t factor, int cls) -> int32_t {
    const uint32_t c = (uint32_t)cls << 29;
    return (int32_t)(factor < 0 ? (0x80000000u | c) : (c | (uint32_t)factor));
  };
  auto cast16 = [&](std::initializer_list<std::pair<size_t, size_t>> parts, int cls = 0) {
    const size_t off = a16.size();
    for (auto pr : parts)
      for (size_t e = 0; e < pr.second; ++e) {
        a16.push_back((int32_t)(pr.first + e));
        b16.push_back(fcode(-1, cls));
      }
    pad16();
    return off;
  };
  // W diag(g) for W [outs][in], scaled by class cls
  auto fold16 = [&](size_t w, int outs, int in, size_t g, int cls) {
    for (int oo = 0; oo < outs; ++oo)
      for (int i = 0; i < in; ++i) {
        a16.push_back((int32_t)(w + (size_t)oo * in + i));
        b16.push_back(fcode((int64_t)(g + i), cls));
      }
  };
  auto foldb = [&](size_t dst, size_t w, int outs, int in, size_t bias, size_t beta, double sc) {
    for (int oo = 0; oo < outs; ++oo)
      pl->folds.push_back({(int32_t)(dst + oo), (int32_t)(bias + oo), (int32_t)(w + (size_t)oo * in), 1,
                           (int32_t)beta, in, sc});
  };
  // patch-embedding weight transposed to [48][C] (row (ky*P + kx)*3 + c) and the decoder as
  // [C][48] (column (ky*P + kx)*3 + ch); zero for the overlapping variant, which has its own
  auto ew_idx = [&](int oc, int k) {  // embed.w element of output channel oc, patch value k
    const int pix = k / 3, ch = k % 3, ky = pix / P, kx = pix % P;
    return (int32_t)(pl->p_ew + ((size_t)(oc * 3 + ch) * P + ky) * P + kx);
  };
  auto dw_idx = [&](int ci, int k) {  // dec.w element of input channel ci, output value k
    const int pix = k / 3, ch = k % 3, ky = pix / P, kx = pix % P;
    return (int32_t)(pl->p_dw + ((size_t)(ci * 3 + ch) * P + ky) * P + kx);
  };
  pl->ewT = f.size();
  for (int k = 0; k < 48; ++k)
    for (int oc = 0; oc < C; ++oc) f.push_back(K == P ? ew_idx(oc, k) : -1);
  pad32();
  pl->eb = copy(pl->p_eb, C);
  const double qscale = 1.4426950408889634 / std::sqrt((double)n.dh);
  for (int l = 0; l < L; ++l) {
    dr_wplan::Blk& B = pl->blk[l];
    const size_t* s = B.p;
    for (int k = 0; k < 16; ++k) B.f[k] = copy(s[k], sizes[k]);
    B.f[16] = f.size();  // [Wk; Wv]
    for (size_t e = 0; e < CC; ++e) f.push_back((int32_t)(s[4] + e));
    for (size_t e = 0; e < CC; ++e) f.push_back((int32_t)(s[6] + e));
    pad32();
    B.f[17] = f.size();  // [bk; bv]
    for (int e = 0; e < C; ++e) f.push_back((int32_t)(s[5] + e));
    for (int e = 0; e < C; ++e) f.push_back((int32_t)(s[7] + e));
    pad32();
    B.f[18] = f.size();  // [bq; bk; bv]
    for (int e = 0; e < C; ++e) f.push_back((int32_t)(s[3] + e));
    for (int e = 0; e < C; ++e) f.push_back((int32_t)(s[5] + e));
    for (int e = 0; e < C; ++e) f.push_back((int32_t)(s[7] + e));
    pad32();
    B.f[19] = transpose({s[2]}, C, C);        // Wq^T
    B.f[20] = transpose({s[4], s[6]}, C, C);  // [Wk; Wv]^T [C][2C]
    B.f[21] = transpose({s[8]}, C, C);        // Wo^T
    B.f[22] = transpose({s[12]}, R, C);       // W1^T [C][R]
    B.f[23] = transpose({s[14]}, C, R);       // W2^T [R][C]
    B.h[0] = cast16({{s[2], CC}, {s[4], CC}, {s[6], CC}});
    B.h[1] = cast16({{s[8], CC}});
    B.h[2] = cast16({{s[12], RC}});
    // W2 carries one 1/sqrt 2 of the GELU (gelu_scaled)
    B.h[3] = cast16({{s[14], RC}}, 2);
    // LayerNorm affine parts folded into the next linear: W diag(g) and b + W beta; Q also
    // carries the softmax scale in base 2, log2(e) / sqrt(dh): the attention kernels of the
    // BF16 path exponentiate the scores with exp2 directly
    B.h[4] = a16.size();
    fold16(s[2], C, C, s[0], 1);
    fold16(s[4], C, C, s[0], 0);
    fold16(s[6], C, C, s[0], 0);
    pad16();
    B.f[24] = f.size();
    f.resize(f.size() + 3 * (size_t)C, -1);
    pad32();
    foldb(B.f[24], s[2], C, C, s[3], s[1], qscale);
    foldb(B.f[24] + C, s[4], C, C, s[5], s[1], 1.0);
    foldb(B.f[24] + 2 * C, s[6], C, C, s[7], s[1], 1.0);
    // the first MLP linear also carries the other 1/sqrt 2 of the GELU (gelu_scaled)
    B.h[5] = a16.size();
    fold16(s[12], R, C, s[10], 2);
    pad16();
    B.f[25] = f.size();
    f.resize(f.size() + (size_t)R, -1);
    pad32();
    foldb(B.f[25], s[12], R, C, s[13], s[11], 0.70710678118654752440);
  }
  // embedding weight [C][64] in the k slot order of the MFMA embedding's patch operand (slot
  // 32 s + 8 g + e holds patch value k = 12 g + 8 s + e for e < 8 - 4 s, zero otherwise), and
  // the decoder with the final LayerNorm folded in: Wd'[k][c] = gf[c] Wd[c][k],
  // bd'[k] = bd[k % 3] + sum_c bf[c] Wd[c][k]
  pl->e16 = a16.size();
  for (int oc = 0; oc < C; ++oc)
    for (int sl = 0; sl < 2; ++sl)
      for (int gq = 0; gq < 4; ++gq)
        for (int e = 0; e < 8; ++e) {
          const bool on = K == P && e < (sl ? 4 : 8);
          a16.push_back(on ? ew_idx(oc, 12 * gq + 8 * sl + e) : -1);
          b16.push_back(fcode(-1, 0));
        }
  pad16();
  pl->d16 = a16.size();
  for (int k = 0; k < 48; ++k)
    for (int ci = 0; ci < C; ++ci) {
      a16.push_back(K == P ? dw_idx(ci, k) : -1);
      b16.push_back(fcode(K == P ? (int64_t)(pl->p_lnfg + ci) : -1, 0));
    }
  pad16();
  pl->dbf = f.size();
  f.resize(f.size() + 48, -1);
  pad32();
  if (K == P)
    for (int k = 0; k < 48; ++k)
      pl->folds.push_back({(int32_t)(pl->dbf + k), (int32_t)(pl->p_db + k % 3), dw_idx(0, k), 3 * P * P,
                           (int32_t)pl->p_lnfb, C, 1.0});
  pl->lnfg = copy(pl->p_lnfg, C);
  pl->lnfb = copy(pl->p_lnfb, C);
  pl->dw = f.size();
  for (int ci = 0; ci < C; ++ci)
    for (int k = 0; k < 48; ++k) f.push_back(K == P ? dw_idx(ci, k) : -1);
  pad32();
  pl->db = copy(pl->p_db, 3);
  pl->eo16 = pl->dwo16 = pl->dbo = 0;
  if (K != P) {
    // overlapping variant: embedding weight [C][192] in the slot order of the overlapping MFMA
    // embedding (slot 32 s + 8 g + e holds footprint row ky = g + 4 (s / 3), value
    // m = 8 (s % 3) + e = 3 kx + c), decoder [192][C] (k = (ky*8 + kx)*3 + ch) with the final
    // LayerNorm gain folded in, and its shift through the decoder per token
    pl->eo16 = a16.size();
    for (int oc = 0; oc < C; ++oc)
      for (int sl = 0; sl < 6; ++sl)
        for (int gq = 0; gq < 4; ++gq)
          for (int e = 0; e < 8; ++e) {
            const int ky = gq + 4 * (sl / 3), m = 8 * (sl % 3) + e, kx = m / 3, ch = m % 3;
            a16.push_back((int32_t)(pl->p_ew + ((size_t)(oc * 3 + ch) * K + ky) * K + kx));
            b16.push_back(fcode(-1, 0));
          }
    pad16();
    auto dwo_idx = [&](int ci, int k) {
      const int ky = (k / 3) / 8, kx = (k / 3) % 8, ch = k % 3;
      return (int32_t)(pl->p_dw + ((size_t)(ci * 3 + ch) * K + ky) * K + kx);
    };
    pl->dwo16 = a16.size();
    for (int k = 0; k < 192; ++k)
      for (int ci = 0; ci < C; ++ci) {
        a16.push_back(dwo_idx(ci, k));
        b16.push_back(fcode((int64_t)(pl->p_lnfg + ci), 0));
      }
    pad16();
    pl->dbo = f.size();
    f.resize(f.size() + 192, -1);
    pad32();
    for (int k = 0; k < 192; ++k)
      pl->folds.push_back({(int32_t)(pl->dbo + k), -1, dwo_idx(0, k), 3 * K * K, (int32_t)pl->p_lnfb, C, 1.0});
  }
  return pl;
}

// ------------------------------------------------------------------------------------------
// device kernels
// ------------------------------------------------------------------------------------------
__global__ void gather32_kernel(const float* __restrict__ src, const int32_t* __restrict__ m, size_t n,
                                float* __restrict__ dst) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    const int32_t k = m[e];
    dst[e] = k >= 0 ? src[k] : 0.f;
  }
}

// dst = bf16(scale * a [* g]): a = src[ma] (0 when ma < 0); mb bit 31 clear: g = src[mb & (2^29 - 1)];
// mb bits 29-30: scale 1, qscale or hscale.  Products in double, rounded once to f32, then
// to bf16.
__global__ void gather16_kernel(const float* __restrict__ src, const int32_t* __restrict__ ma,
                                const int32_t* __restrict__ mb, double qscale, double hscale, size_t n,
                                bf16* __restrict__ dst) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    const int32_t a = ma[e];
    const uint32_t b = (uint32_t)mb[e];
    float v = 0.f;
    if (a >= 0) {
      const int cls = (b >> 29) & 3;
      const double sc = cls == 1 ? qscale : (cls == 2 ? hscale : 1.0);
      const double g = (b >> 31) ? 1.0 : (double)src[b & 0x1FFFFFFFu];
      v = (float)(sc * (double)src[a] * g);
    }
    dst[e] = f2bf(v);
  }
}

__global__ void fold_kernel(const float* __restrict__ src, const FoldRow* __restrict__ rows, int nrows,
                            float* __restrict__ dst) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrows) return;
  const FoldRow fr = rows[r];
  double acc = fr.bias >= 0 ? (double)src[fr.bias] : 0.0;
  for (int i = 0; i < fr.n; ++i) acc += (double)src[fr.w + (size_t)i * fr.w_si] * (double)src[fr.beta + i];
  dst[fr.dst] = (float)(fr.sc * acc);
}

// amax of 6 weight tensors per block (one workgroup per tensor), scale = amax / 448 (1 if 0)
__global__ __launch_bounds__(256) void weight_scale_kernel(const float* const* __restrict__ ptrs,
                                                           const size_t* __restrict__ counts,
                                                           float* __restrict__ scales) {
  const int t = blockIdx.x;  // tensor (block l = t / 6, k = t % 6)
  const float* p = ptrs[t];
  const size_t n = counts[t];
  float m = 0.f;
  for (size_t e = threadIdx.x; e < n; e += 256) m = fmaxf(m, fabsf(p[e]));
  __shared__ float red[256];
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) scales[(t / 6) * 8 + t % 6] = red[0] > 0.f ? red[0] / 448.0f : 1.0f;
}

// ------------------------------------------------------------------------------------------
// host side
// ------------------------------------------------------------------------------------------
static void assign_pointers(dr_ctx* c, const dr_wplan& pl) {
  Net& n = c->net;
  const float* F = c->wf32;
  const bf16* B16 = c->wb16;
  const int L = n.cfg.blocks;
  n.embed_wT = F + pl.ewT;
  n.embed_b = F + pl.eb;
  n.blk.assign(L, BlockW());
  for (int l = 0; l < L; ++l) {
    BlockW& w = n.blk[l];
    const size_t* O = pl.blk[l].f;
    const size_t* H = pl.blk[l].h;
    w.ln1g = F + O[0]; w.ln1b = F + O[1];
    w.wq = F + O[2]; w.bq = F + O[3];
    w.wk = F + O[4]; w.bk = F + O[5];
    w.wv = F + O[6]; w.bv = F + O[7];
    w.wo = F + O[8]; w.bo = F + O[9];
    w.ln2g = F + O[10]; w.ln2b = F + O[11];
    w.w1 = F + O[12]; w.b1 = F + O[13];
    w.w2 = F + O[14]; w.b2 = F + O[15];
    w.wkv = F + O[16]; w.bkv = F + O[17]; w.bqkv = F + O[18];
    w.wqT = F + O[19]; w.wkvT = F + O[20]; w.woT = F + O[21]; w.w1T = F + O[22]; w.w2T = F + O[23];
    w.wqkv16 = B16 + H[0];
    w.wo16 = B16 + H[1];
    w.w116 = B16 + H[2];
    w.w216 = B16 + H[3];
    w.wqkvf16 = B16 + H[4];
    w.w1f16 = B16 + H[5];
    w.bqkvf = F + O[24];
    w.b1f = F + O[25];
    w.wqkv8 = w.wo8 = w.w18 = w.w28 = nullptr;
    w.wscale8 = nullptr;
  }
  n.embed_wT16 = B16 + pl.e16;
  n.dec_wf16 = B16 + pl.d16;
  n.dec_bf = F + pl.dbf;
  n.lnfg = F + pl.lnfg;
  n.lnfb = F + pl.lnfb;
  n.dec_w = F + pl.dw;
  n.dec_b = F + pl.db;
  const bool ovl = pl.K != n.P;
  n.K = pl.K;
  n.embed_ovl16 = ovl ? B16 + pl.eo16 : nullptr;
  n.dec_ovl16 = ovl ? B16 + pl.dwo16 : nullptr;
  n.dec_ovl_bf = ovl ? F + pl.dbo : nullptr;
  n.dec_ovl_b = ovl ? F + pl.db : nullptr;
  if (c->w8) {
    const size_t CC = (size_t)n.C * n.C, RC = (size_t)n.R * n.C, per_blk = 4 * CC + 2 * RC;
    for (int l = 0; l < L; ++l) {
      BlockW& w = n.blk[l];
      uint8_t* base = c->w8 + per_blk * l;
      w.wqkv8 = base;
      w.wo8 = base + 3 * CC;
      w.w18 = base + 4 * CC;
      w.w28 = base + 4 * CC + RC;
      w.wscale8 = c->wscale8 + (size_t)l * 8;
    }
  }
}

static void free_arenas(dr_ctx* c) {
  for (void* p : c->weight_allocs) (void)hipFree(p);
  c->weight_allocs.clear();
  c->params = c->wf32 = nullptr;
  c->wf32_elems = 0;
  c->wb16 = nullptr;
  c->w8 = nullptr;
  c->wscale8 = nullptr;
  c->wmaps32 = c->wmaps16a = c->wmaps16b = nullptr;
  c->wfolds = nullptr;
  c->wjob_ptrs = nullptr;
  c->wjob_counts = nullptr;
  dr_wplan_free(c->wplan);
  c->wplan = nullptr;
  c->have_weights = false;
}

void dr::dr_weights_release(dr_ctx* c) { free_arenas(c); }

// Plan and device arenas for kernel size K (allocated once per K; a later load with the same
// K reuses them, so its pointers -- and the captured HIP graphs -- stay valid).
static dr_status ensure_arenas(dr_ctx* c, int K) {
  if (c->wplan && c->wplan->K == K) return DR_OK;
  HIP_OK(c, hipDeviceSynchronize());
  dr_invalidate_graphs(c);
  free_arenas(c);
  dr_wplan* pl = build_plan(c->net, K);
  c->wplan = pl;
  const Net& n = c->net;
  const int L = n.cfg.blocks;
  auto A = [&](size_t bytes) -> void* {
    void* p = nullptr;
    if (hipMalloc(&p, bytes ? bytes : 256) != hipSuccess) return nullptr;
    c->weight_allocs.push_back(p);
    return p;
  };
  c->params = (float*)A(pl->nparams * 4);
  c->wf32 = (float*)A(pl->m32.size() * 4);
  c->wf32_elems = pl->m32.size();
  c->wb16 = (bf16*)A(pl->m16a.size() * 2);
  c->wmaps32 = (int32_t*)A(pl->m32.size() * 4);
  c->wmaps16a = (int32_t*)A(pl->m16a.size() * 4);
  c->wmaps16b = (int32_t*)A(pl->m16b.size() * 4);
  c->wfolds = A(pl->folds.size() * sizeof(FoldRow));
  bool ok = c->params && c->wf32 && c->wb16 && c->wmaps32 && c->wmaps16a && c->wmaps16b && c->wfolds;
  if (ok && fp8_supported(n.C, n.R)) {
    const size_t CC = (size_t)n.C * n.C, RC = (size_t)n.R * n.C;
    c->w8 = (uint8_t*)A((4 * CC + 2 * RC) * L);
    c->wscale8 = (float*)A((size_t)L * 8 * 4);
    c->wjob_ptrs = (const float**)A((size_t)L * 6 * sizeof(float*));
    c->wjob_counts = (size_t*)A((size_t)L * 6 * sizeof(size_t));
    ok = c->w8 && c->wscale8 && c->wjob_ptrs && c->wjob_counts;
  }
  if (!ok) {
    free_arenas(c);
    return dr_fail(c, DR_ENOMEM, "weights: device allocation failed");
  }
  HIP_OK(c, hipMemcpy(c->wmaps32, pl->m32.data(), pl->m32.size() * 4, hipMemcpyHostToDevice));
  HIP_OK(c, hipMemcpy(c->wmaps16a, pl->m16a.data(), pl->m16a.size() * 4, hipMemcpyHostToDevice));
  HIP_OK(c, hipMemcpy(c->wmaps16b, pl->m16b.data(), pl->m16b.size() * 4, hipMemcpyHostToDevice));
  HIP_OK(c, hipMemcpy(c->wfolds, pl->folds.data(), pl->folds.size() * sizeof(FoldRow), hipMemcpyHostToDevice));
  assign_pointers(c, *pl);
  if (c->w8) {
    std::vector<const float*> ptrs;
    std::vector<size_t> counts;
    const size_t CC = (size_t)n.C * n.C, RC = (size_t)n.R * n.C;
    for (int l = 0; l < L; ++l) {
      const BlockW& w = n.blk[l];
      const float* p6[6] = {w.wq, w.wk, w.wv, w.wo, w.w1, w.w2};
      const size_t n6[6] = {CC, CC, CC, CC, RC, RC};
      for (int k = 0; k < 6; ++k) {
        ptrs.push_back(p6[k]);
        counts.push_back(n6[k]);
      }
    }
    HIP_OK(c, hipMemcpy(c->wjob_ptrs, ptrs.data(), ptrs.size() * sizeof(float*), hipMemcpyHostToDevice));
    HIP_OK(c, hipMemcpy(c->wjob_counts, counts.data(), counts.size() * sizeof(size_t), hipMemcpyHostToDevice));
  }
  return DR_OK;
}

// Every derived layout from c->params, enqueued on s.
static dr_status derive(dr_ctx* c, hipStream_t s) {
  const dr_wplan& pl = *c->wplan;
  const Net& n = c->net;
  const size_t n32 = pl.m32.size(), n16 = pl.m16a.size();
  const double qscale = 1.4426950408889634 / std::sqrt((double)n.dh);
  gather32_kernel<<<(unsigned)std::min<size_t>((n32 + 255) / 256, 8192), 256, 0, s>>>(c->params, c->wmaps32, n32, c->wf32);
  gather16_kernel<<<(unsigned)std::min<size_t>((n16 + 255) / 256, 8192), 256, 0, s>>>(
      c->params, c->wmaps16a, c->wmaps16b, qscale, 0.70710678118654752440, n16, c->wb16);
  const int nf = (int)pl.folds.size();
  fold_kernel<<<(nf + 127) / 128, 128, 0, s>>>(c->params, (const FoldRow*)c->wfolds, nf, c->wf32);
  HIP_OK(c, hipGetLastError());
  if (c->w8) {
    // FP8 e4m3 copies of the GEMM weights, one scale per tensor (amax / 448)
    const int L = n.cfg.blocks;
    weight_scale_kernel<<<L * 6, 256, 0, s>>>(c->wjob_ptrs, c->wjob_counts, c->wscale8);
    const size_t CC = (size_t)n.C * n.C, RC = (size_t)n.R * n.C;
    for (int l = 0; l < L; ++l) {
      const BlockW& w = n.blk[l];
      const float* src[6] = {w.wq, w.wk, w.wv, w.wo, w.w1, w.w2};
      const size_t nel[6] = {CC, CC, CC, CC, RC, RC};
      uint8_t* dst = const_cast<uint8_t*>(w.wqkv8);
      for (int k = 0; k < 6; ++k) {
        launch_quantize_fp8_dev(src[k], dst, nel[k], w.wscale8 + k, s);
        dst += nel[k];
      }
    }
    HIP_OK(c, hipGetLastError());
  }
  return DR_OK;
}

// ------------------------------------------------------------------------------------------
// C ABI
// ------------------------------------------------------------------------------------------
struct BlobRec {
  char name[48];
  uint32_t dtype, ndim, shape[4];
  uint64_t offset, nbytes;
};

extern "C" dr_status dr_load_weights(dr_ctx* c, const void* blob, size_t nbytes) {
  if (!c || !blob) return dr_fail(c, DR_EINVAL, "dr_load_weights: null argument");
  const char* b = (const char*)blob;
  const size_t head = 4 + 4 + sizeof(dr_netcfg) + 4;
  if (nbytes < head || std::memcmp(b, "DRW1", 4) != 0) return dr_fail(c, DR_EINVAL, "weight blob: bad magic");
  uint32_t version, count;
  dr_netcfg bc;
  std::memcpy(&version, b + 4, 4);
  std::memcpy(&bc, b + 8, sizeof bc);
  std::memcpy(&count, b + 8 + sizeof bc, 4);
  if (version != 1) return dr_fail(c, DR_EINVAL, "weight blob: unsupported version %u", version);
  if (std::memcmp(&bc, &c->net.cfg, sizeof bc) != 0)
    return dr_fail(c, DR_EINVAL, "weight blob: network config differs from the context's");
  const Net& n = c->net;
  const int C = n.C, R = n.R, L = n.cfg.blocks, P = n.P;
  // kernel size of the embedding and the decoder: P (non-overlapping) or 2P (overlapping,
  // stride P, padding P/2), read from the first tensor's shape
  int K = P;
  if (nbytes >= head + sizeof(BlobRec)) {
    BlobRec r0;
    std::memcpy(&r0, b + head, sizeof r0);
    if (r0.ndim == 4 && r0.shape[2] == (uint32_t)(2 * P) && r0.shape[3] == (uint32_t)(2 * P)) K = 2 * P;
  }
  if (K != P && P != 4) return dr_fail(c, DR_EINVAL, "weight blob: the overlapping embedding needs patch 4");
  struct Want { std::string name; std::vector<uint32_t> shape; };
  std::vector<Want> want;
  want.push_back({"embed.w", {(uint32_t)C, 3, (uint32_t)K, (uint32_t)K}});
  want.push_back({"embed.b", {(uint32_t)C}});
  for (int l = 0; l < L; ++l) {
    const std::string p = "blk" + std::to_string(l) + ".";
    const uint32_t c32 = C, r32 = R;
    for (const char* nm : {"ln1.g", "ln1.b"}) want.push_back({p + nm, {c32}});
    for (const char* nm : {"wq", "bq", "wk", "bk", "wv", "bv", "wo", "bo"})
      want.push_back({p + nm, nm[0] == 'w' ? std::vector<uint32_t>{c32, c32} : std::vector<uint32_t>{c32}});
    for (const char* nm : {"ln2.g", "ln2.b"}) want.push_back({p + nm, {c32}});
    want.push_back({p + "w1", {r32, c32}});
    want.push_back({p + "b1", {r32}});
    want.push_back({p + "w2", {c32, r32}});
    want.push_back({p + "b2", {c32}});
  }
  want.push_back({"lnf.g", {(uint32_t)C}});
  want.push_back({"lnf.b", {(uint32_t)C}});
  want.push_back({"dec.w", {(uint32_t)C, 3, (uint32_t)K, (uint32_t)K}});
  want.push_back({"dec.b", {3}});
  if (count != want.size())
    return dr_fail(c, DR_EINVAL, "weight blob: %u tensors, expected %zu", count, want.size());
  const size_t table = head + (size_t)count * sizeof(BlobRec);
  if (nbytes < table) return dr_fail(c, DR_EINVAL, "weight blob: truncated table");
  std::vector<float> flat;
  flat.reserve(dr_nparams(n, K));
  for (uint32_t i = 0; i < count; ++i) {
    BlobRec r;
    std::memcpy(&r, b + head + (size_t)i * sizeof(BlobRec), sizeof r);
    r.name[47] = 0;
    if (want[i].name != r.name)
      return dr_fail(c, DR_EINVAL, "weight blob: tensor %u is '%s', expected '%s'", i, r.name, want[i].name.c_str());
    if (r.dtype != 0) return dr_fail(c, DR_EINVAL, "weight blob: '%s' is not f32", r.name);
    if (r.ndim != want[i].shape.size()) return dr_fail(c, DR_EINVAL, "weight blob: '%s' has wrong rank", r.name);
    size_t elems = 1;
    for (uint32_t d = 0; d < r.ndim; ++d) {
      if (r.shape[d] != want[i].shape[d]) return dr_fail(c, DR_EINVAL, "weight blob: '%s' has wrong shape", r.name);
      elems *= r.shape[d];
    }
    if (r.nbytes != elems * 4 || table + r.offset + r.nbytes > nbytes || r.offset % 4)
      return dr_fail(c, DR_EINVAL, "weight blob: '%s' has a bad extent", r.name);
    const size_t o = flat.size();
    flat.resize(o + elems);
    std::memcpy(flat.data() + o, b + table + r.offset, r.nbytes);
  }
  HIP_OK(c, hipSetDevice(c->device));
  dr_status st = ensure_arenas(c, K);
  if (st != DR_OK) return st;
  c->have_weights = false;
  HIP_OK(c, hipMemcpy(c->params, flat.data(), flat.size() * 4, hipMemcpyHostToDevice));
  st = derive(c, nullptr);
  if (st != DR_OK) return st;
  HIP_OK(c, hipDeviceSynchronize());
  c->have_weights = true;
  return DR_OK;
}

extern "C" dr_status dr_load_params(dr_ctx* c, const float* params, void* stream) {
  if (!c || !params) return dr_fail(c, DR_EINVAL, "dr_load_params: null argument");
  const int K = c->wplan ? c->wplan->K : c->net.P;
  if (K != c->net.P) return dr_fail(c, DR_EINVAL, "dr_load_params: the overlapping embedding loads from a blob only");
  HIP_OK(c, hipSetDevice(c->device));
  dr_status st = ensure_arenas(c, K);
  if (st != DR_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  if (params != c->params)
    HIP_OK(c, hipMemcpyAsync(c->params, params, c->wplan->nparams * 4, hipMemcpyDeviceToDevice, s));
  st = derive(c, s);
  if (st != DR_OK) return st;
  c->have_weights = true;
  return DR_OK;
}
