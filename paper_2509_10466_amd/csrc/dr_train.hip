// Training entry points: a forward that keeps the activations the reverse pass needs, the
// hand-written reverse pass, the L1 training loss, and in-place weight updates from a flat
// device parameter vector.  FP32 throughout, or (dr_train_set_precision) with the weight
// products of both passes taking bf16 operands and accumulating in FP32, against FP32
// master weights, activations and gradients.
//
// The loss follows the thesis's region-weighted per-pixel L1 (Methods, "Model Training --
// Loss"), taken on the prediction before the composite.  Attention probabilities are not
// stored by the forward: the reverse pass recomputes them from Q, K and the saved row
// max / sum.
#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

#include "dr_internal.h"

using namespace dr;

namespace dr {
void launch_gather_rows(const float* X, const int32_t* rows, const int32_t* n_dev, int n_max, int C, float* Y, hipStream_t s);
void launch_scatter_rows(const float* Y, const int32_t* rows, const int32_t* n_dev, int n_max, int C, float* X, hipStream_t s);
void launch_gelu_fwd(const float* h, const int32_t* n_dev, int n_max, int R, float* a, hipStream_t s);
void launch_gelu_bwd(const float* h, const float* da, const int32_t* n_dev, int n_max, int R, float* dh, hipStream_t s);
bool attn_train_supported(int dh, int S);
void launch_attn_train_fwd(const Geo& g, int C, int heads, const float* q, const float* kv, const int32_t* woff,
                           float* o, float2* stats, hipStream_t s);
void launch_attn_train_dq(const Geo& g, int C, int heads, const float* q, const float* kv, const float* dout,
                          const float2* stats, const int32_t* woff, float* dq, float* dsum, hipStream_t s);
void launch_attn_train_dkv(const Geo& g, int C, int heads, const float* q, const float* kv, const float* dout,
                           const float2* stats, const float* dsum, const int32_t* woff, float* dkv, hipStream_t s);
void launch_ln_bwd(const float* x, const int32_t* rows, const int32_t* n_dev, int n_max, int C, const float* g,
                   const float* dy, float* dx, int accumulate, int dst_compact, float* part, hipStream_t s);
int ln_bwd_blocks(int n_max);
void launch_sum_parts(const float* part, int nparts, int width, float* out, int accumulate, hipStream_t s);
int tn_chunks(int M_max);
void launch_tn_partial(const float* A, const int32_t* arow, int lda, const float* B, const int32_t* brow, int ldb,
                       const int32_t* M_dev, int M_max, int I, int J, float* part, hipStream_t s);
void launch_tn_bf16ops(const float* A, const int32_t* arow, int lda, const float* B, const int32_t* brow, int ldb,
                       const int32_t* M_dev, int M_max, int I, int J, float* part, hipStream_t s);
void launch_gemm_bf16ops(const float* A, const int32_t* arows, const int32_t* m_dev, int m_max, int K,
                         const float* W, const float* bias, int Nout, int epi, float* out,
                         const int32_t* res_rows, hipStream_t s);
void launch_colsum_partial(const float* B, int ldb, const int32_t* M_dev, int M_max, int J, float* part, hipStream_t s);
void launch_patches(const Geo& g, const float* frames, const uint8_t* masks, float* P, hipStream_t s);
void launch_decoder_full(const Geo& g, int C, const float* z, const float* dw, const float* db, float* pred, hipStream_t s);
void launch_dec_grad_tok(const Geo& g, const float* pred, const float* dpred, float* dyt, hipStream_t s);
void launch_l1_loss(const float* pred, const float* gt, const uint8_t* masks, size_t npix, float w_in, float w_out,
                    float* part, float* acc, float* loss, float* dpred, hipStream_t s);
}  // namespace dr

#define HIP_OK(ctx, expr)                                                                                   \
  do {                                                                                                      \
    hipError_t e_ = (expr);                                                                                 \
    if (e_ != hipSuccess) return dr_fail(ctx, DR_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));     \
  } while (0)

#define KCHECK(what)                                                                                        \
  do {                                                                                                      \
    hipError_t e_ = hipGetLastError();                                                                      \
    if (e_ != hipSuccess) return dr_fail(c, DR_EHIP, "launch of %s failed: %s", what, hipGetErrorString(e_)); \
  } while (0)

// ------------------------------------------------------------------------------------------
// saved activations (one handle per forward) and the context's shared reverse-pass scratch
// ------------------------------------------------------------------------------------------
struct TrainBlock {
  float *x_in, *u, *kv, *q, *o, *x1, *n2, *hpre;
  float2* stats;
};

// Everything one forward leaves for its reverse pass, including a copy of the FP32 weight
// arena it ran with, so a later weight load does not change the gradient of an earlier
// forward.  Owned by the context; dr_saved_free returns it to the context's pool.
struct dr_saved {
  dr_ctx* owner = nullptr;
  bool live = false;  // handed out by dr_train_forward, not yet freed
  Geo g{};
  size_t cap = 0;     // tokens
  int S = 0;
  bool bf16 = false;  // precision of the products of its forward (and of its reverse pass)
  std::vector<void*> allocs;
  uint8_t* flag = nullptr;
  int32_t *wcount = nullptr, *woff = nullptr, *idx = nullptr, *nq = nullptr;
  std::vector<TrainBlock> blk;
  float *xf = nullptr, *z = nullptr, *pred = nullptr, *patches = nullptr;
  float* wsnap = nullptr;  // the FP32 weight arena of the forward
  size_t wsnap_elems = 0;
};

struct dr_train {
  Geo g{};
  size_t cap = 0;  // tokens
  int S = 0;
  std::vector<void*> allocs;
  // forward scratch
  float* x = nullptr;
  // reverse-pass scratch
  float *a = nullptr, *dx = nullptr, *dx2 = nullptr, *dx1 = nullptr, *da = nullptr, *dh = nullptr, *dn2 = nullptr,
        *dout = nullptr, *dq = nullptr, *dkv = nullptr, *du = nullptr, *dsum = nullptr, *dyt = nullptr,
        *dz = nullptr, *part = nullptr, *lnpart = nullptr, *zeros = nullptr, *tmp = nullptr;
  // loss scratch (allocated once)
  float *lpart = nullptr, *lacc = nullptr;
  std::vector<dr_saved*> saved;  // every handle of the context (live or pooled)
};

static void free_list(std::vector<void*>& l) {
  for (void* p : l) (void)hipFree(p);
  l.clear();
}

static void scratch_free(dr_train* t) {
  free_list(t->allocs);
  t->x = t->a = t->dx = t->dx2 = t->dx1 = t->da = t->dh = t->dn2 = t->dout = t->dq = t->dkv = t->du = t->dsum =
      t->dyt = t->dz = t->part = t->lnpart = t->zeros = t->tmp = nullptr;
  t->cap = 0;
}

static void saved_destroy(dr_saved* sv) {
  free_list(sv->allocs);
  delete sv;
}

// products of both passes: FP32 operands, or bf16 operands with FP32 accumulation
static void train_gemm(bool bf16, const float* A, const int32_t* arows, const int32_t* m_dev, int m_max, int K,
                       const float* W, const float* bias, int Nout, int epi, float* out, const int32_t* res_rows,
                       hipStream_t s) {
  (bf16 ? launch_gemm_bf16ops : launch_gemm_f32)(A, arows, m_dev, m_max, K, W, bias, Nout, epi, out, res_rows, s);
}

static dr_train* train_of(dr_ctx* c) {
  if (!c->train) c->train = new dr_train();
  return static_cast<dr_train*>(c->train);
}

void dr::dr_train_release(dr_ctx* c) {
  if (!c->train) return;
  dr_train* t = static_cast<dr_train*>(c->train);
  scratch_free(t);
  free_list(t->allocs);
  if (t->lpart) (void)hipFree(t->lpart);
  if (t->lacc) (void)hipFree(t->lacc);
  for (dr_saved* sv : t->saved) saved_destroy(sv);
  delete t;
  c->train = nullptr;
}

template <class F>
static bool alloc_all(std::vector<void*>& list, F&& fill) {
  bool ok = true;
  auto A = [&](size_t bytes) -> void* {
    void* p = nullptr;
    if (hipMalloc(&p, bytes ? bytes : 256) != hipSuccess) {
      ok = false;
      return nullptr;
    }
    list.push_back(p);
    return p;
  };
  fill(A);
  return ok;
}

// shared scratch for clips of g (grown, never shrunk)
static dr_status scratch_reserve(dr_ctx* c, dr_train* t, const Geo& g) {
  if ((size_t)g.N <= t->cap && t->S == g.S) return DR_OK;
  HIP_OK(c, hipDeviceSynchronize());
  scratch_free(t);
  const Net& n = c->net;
  const size_t N = g.N, C = n.C, R = n.R, H = n.cfg.heads;
  const bool ok = alloc_all(t->allocs, [&](auto& A) {
    t->x = (float*)A(N * C * 4);
    t->a = (float*)A(N * R * 4);
    t->dx = (float*)A(N * C * 4);
    t->dx2 = (float*)A(N * C * 4);
    t->dx1 = (float*)A(N * C * 4);
    t->da = (float*)A(N * R * 4);
    t->dh = (float*)A(N * R * 4);
    t->dn2 = (float*)A(N * C * 4);
    t->dout = (float*)A(N * C * 4);
    t->dq = (float*)A(N * C * 4);
    t->dkv = (float*)A(N * 2 * C * 4);
    t->du = (float*)A(N * C * 4);
    t->dsum = (float*)A(N * H * 4);
    t->dyt = (float*)A(N * 48 * 4);
    t->dz = (float*)A(N * C * 4);
    t->part = (float*)A((size_t)tn_chunks((int)N) * R * C * 4);
    t->lnpart = (float*)A((size_t)ln_bwd_blocks((int)N) * 2 * C * 4);
    t->zeros = (float*)A((2 * C + R + 64) * 4);
    t->tmp = (float*)A((R * C + 64) * 4);
  });
  if (!ok) {
    scratch_free(t);
    return dr_fail(c, DR_ENOMEM, "training workspace allocation failed");
  }
  HIP_OK(c, hipMemset(t->zeros, 0, (2 * C + R + 64) * 4));
  HIP_OK(c, hipDeviceSynchronize());
  t->cap = N;
  t->S = g.S;
  t->g = g;
  return DR_OK;
}

// a pooled handle that fits g, or a new one
static dr_status saved_acquire(dr_ctx* c, dr_train* t, const Geo& g, dr_saved** out) {
  *out = nullptr;
  const size_t wel = c->wf32_elems;
  dr_saved* best = nullptr;
  for (dr_saved* sv : t->saved)
    if (!sv->live && sv->cap >= (size_t)g.N && sv->S == g.S && sv->wsnap_elems == wel && (!best || sv->cap < best->cap))
      best = sv;
  if (!best) {
    const Net& n = c->net;
    const size_t N = g.N, C = n.C, R = n.R, L = n.cfg.blocks, H = n.cfg.heads, nw = g.nwin;
    dr_saved* sv = new dr_saved();
    const bool ok = alloc_all(sv->allocs, [&](auto& A) {
      sv->flag = (uint8_t*)A(N);
      sv->wcount = (int32_t*)A(nw * 4);
      sv->woff = (int32_t*)A((nw + 1) * 4);
      sv->idx = (int32_t*)A(N * 4);
      sv->nq = (int32_t*)A(256);
      sv->blk.resize(L);
      for (size_t l = 0; l < L; ++l) {
        TrainBlock& b = sv->blk[l];
        b.x_in = (float*)A(N * C * 4);
        b.u = (float*)A(N * C * 4);
        b.kv = (float*)A(N * 2 * C * 4);
        b.q = (float*)A(N * C * 4);
        b.o = (float*)A(N * C * 4);
        b.x1 = (float*)A(N * C * 4);
        b.n2 = (float*)A(N * C * 4);
        b.hpre = (float*)A(N * R * 4);
        b.stats = (float2*)A(N * H * 8);
      }
      sv->xf = (float*)A(N * C * 4);
      sv->z = (float*)A(N * C * 4);
      sv->pred = (float*)A(N * 16 * 12);
      sv->patches = (float*)A(N * 48 * 4);
      sv->wsnap = (float*)A(wel * 4);
    });
    if (!ok) {
      saved_destroy(sv);
      return dr_fail(c, DR_ENOMEM, "saved-activation allocation failed");
    }
    sv->owner = c;
    sv->cap = N;
    sv->S = g.S;
    sv->wsnap_elems = wel;
    t->saved.push_back(sv);
    best = sv;
  }
  best->g = g;
  best->live = true;
  *out = best;
  return DR_OK;
}

// flat parameter offsets (blob order)
struct ParamOffsets {
  size_t ew, eb, lnfg, lnfb, dw, db, total;
  struct B { size_t ln1g, ln1b, wq, bq, wk, bk, wv, bv, wo, bo, ln2g, ln2b, w1, b1, w2, b2; };
  std::vector<B> blk;
};

static ParamOffsets param_offsets(const Net& n) {
  ParamOffsets p;
  const size_t C = n.C, R = n.R;
  size_t o = 0;
  p.ew = o; o += C * 48;
  p.eb = o; o += C;
  p.blk.resize(n.cfg.blocks);
  for (auto& b : p.blk) {
    b.ln1g = o; o += C;
    b.ln1b = o; o += C;
    b.wq = o; o += C * C;
    b.bq = o; o += C;
    b.wk = o; o += C * C;
    b.bk = o; o += C;
    b.wv = o; o += C * C;
    b.bv = o; o += C;
    b.wo = o; o += C * C;
    b.bo = o; o += C;
    b.ln2g = o; o += C;
    b.ln2b = o; o += C;
    b.w1 = o; o += R * C;
    b.b1 = o; o += R;
    b.w2 = o; o += C * R;
    b.b2 = o; o += C;
  }
  p.lnfg = o; o += C;
  p.lnfb = o; o += C;
  p.dw = o; o += C * 48;
  p.db = o; o += 3;
  p.total = o;
  return p;
}

extern "C" size_t dr_param_count(dr_ctx* c) { return c ? param_offsets(c->net).total : 0; }

// ------------------------------------------------------------------------------------------
// forward with saved activations
// ------------------------------------------------------------------------------------------
static dr_status train_forward_into(dr_ctx* c, dr_train* t, dr_saved* sv, const float* frames, const uint8_t* masks,
                                    float* pred, hipStream_t s) {
  const Net& n = c->net;
  const Geo& g = sv->g;
  const int C = n.C, R = n.R, N = g.N, heads = n.cfg.heads;
  const bool b16 = sv->bf16;
  HIP_OK(c, hipMemcpyAsync(sv->wsnap, c->wf32, c->wf32_elems * 4, hipMemcpyDeviceToDevice, s));
  launch_token_flags(g, masks, 0, sv->flag, sv->wcount, s);
  launch_token_gather(g, sv->flag, sv->wcount, sv->idx, sv->woff, sv->nq, s);
  launch_embed(g, C, frames, masks, n.embed_wT, n.embed_b, t->x, s);
  launch_patches(g, frames, masks, sv->patches, s);
  KCHECK("embed");
  for (int l = 0; l < n.cfg.blocks; ++l) {
    const BlockW& b = n.blk[l];
    TrainBlock& tb = sv->blk[l];
    HIP_OK(c, hipMemcpyAsync(tb.x_in, t->x, (size_t)N * C * 4, hipMemcpyDeviceToDevice, s));
    launch_ln_f32(t->x, nullptr, nullptr, N, C, b.ln1g, b.ln1b, tb.u, s);
    train_gemm(b16, tb.u, nullptr, nullptr, N, C, b.wkv, b.bkv, 2 * C, EPI_STORE, tb.kv, nullptr, s);
    train_gemm(b16, tb.u, sv->idx, sv->nq, N, C, b.wq, b.bq, C, EPI_STORE, tb.q, nullptr, s);
    launch_attn_train_fwd(g, C, heads, tb.q, tb.kv, sv->woff, tb.o, tb.stats, s);
    train_gemm(b16, tb.o, nullptr, sv->nq, N, C, b.wo, b.bo, C, EPI_RESID, t->x, sv->idx, s);
    launch_gather_rows(t->x, sv->idx, sv->nq, N, C, tb.x1, s);
    launch_ln_f32(tb.x1, nullptr, sv->nq, N, C, b.ln2g, b.ln2b, tb.n2, s);
    train_gemm(b16, tb.n2, nullptr, sv->nq, N, C, b.w1, b.b1, R, EPI_STORE, tb.hpre, nullptr, s);
    launch_gelu_fwd(tb.hpre, sv->nq, N, R, t->a, s);
    train_gemm(b16, t->a, nullptr, sv->nq, N, R, b.w2, b.b2, C, EPI_RESID, t->x, sv->idx, s);
    KCHECK("block");
  }
  HIP_OK(c, hipMemcpyAsync(sv->xf, t->x, (size_t)N * C * 4, hipMemcpyDeviceToDevice, s));
  launch_ln_f32(t->x, nullptr, nullptr, N, C, n.lnfg, n.lnfb, sv->z, s);
  launch_decoder_full(g, C, sv->z, n.dec_w, n.dec_b, sv->pred, s);
  KCHECK("decoder");
  HIP_OK(c, hipMemcpyAsync(pred, sv->pred, (size_t)N * 16 * 12, hipMemcpyDeviceToDevice, s));
  return DR_OK;
}

extern "C" dr_status dr_train_forward(dr_ctx* c, const float* frames, const uint8_t* masks, float* pred, int B,
                                      int T, int H, int W, dr_saved** saved, void* stream) {
  if (!c || !frames || !masks || !pred || !saved) return dr_fail(c, DR_EINVAL, "dr_train_forward: null argument");
  *saved = nullptr;
  if (!c->have_weights) return dr_fail(c, DR_EINVAL, "no weights loaded");
  if (c->attn_pattern != 0) return dr_fail(c, DR_EINVAL, "training runs the joint-attention network");
  if (c->net.K != c->net.P) return dr_fail(c, DR_EINVAL, "training runs the non-overlapping embedding");
  if (!attn_train_supported(c->net.dh, c->net.S))
    return dr_fail(c, DR_ESHAPE, "training attention holds windows of at most 304 tokens, head dim 32 or 64");
  Geo g;
  dr_status st = dr_make_geo(c, B, T, H, W, c->net.cfg.win_t, g);
  if (st != DR_OK) return st;
  HIP_OK(c, hipSetDevice(c->device));
  dr_train* t = train_of(c);
  st = scratch_reserve(c, t, g);
  if (st != DR_OK) return st;
  dr_saved* sv = nullptr;
  st = saved_acquire(c, t, g, &sv);
  if (st != DR_OK) return st;
  sv->bf16 = c->train_bf16 != 0;
  st = train_forward_into(c, t, sv, frames, masks, pred, (hipStream_t)stream);
  if (st != DR_OK) {
    sv->live = false;  // back to the pool
    return st;
  }
  *saved = sv;
  return DR_OK;
}

extern "C" dr_status dr_saved_free(dr_ctx* c, dr_saved* sv) {
  if (!c || !sv) return dr_fail(c, DR_EINVAL, "dr_saved_free: null argument");
  if (!c->train) return dr_fail(c, DR_EINVAL, "dr_saved_free: not a handle of this context");
  dr_train* t = static_cast<dr_train*>(c->train);
  bool mine = false;
  for (dr_saved* x : t->saved) mine = mine || x == sv;
  if (!mine || sv->owner != c || !sv->live) return dr_fail(c, DR_EINVAL, "dr_saved_free: not a live handle of this context");
  sv->live = false;
  // keep at most two idle handles for reuse; free the others
  int idle = 0;
  for (size_t i = 0; i < t->saved.size();) {
    dr_saved* x = t->saved[i];
    if (!x->live && ++idle > 2) {
      saved_destroy(x);
      t->saved.erase(t->saved.begin() + i);
    } else {
      ++i;
    }
  }
  return DR_OK;
}

// grads[off .. off + I*J) = sum over chunks of TN partials
static void tn_grad(dr_train* t, bool bf16, const float* A, const int32_t* arow, int lda, const float* Bm, const int32_t* brow,
                    int ldb, const int32_t* M_dev, int M_max, int I, int J, float* out, hipStream_t s) {
  (bf16 ? launch_tn_bf16ops : launch_tn_partial)(A, arow, lda, Bm, brow, ldb, M_dev, M_max, I, J, t->part, s);
  launch_sum_parts(t->part, tn_chunks(M_max), I * J, out, 0, s);
}

static void colsum_grad(dr_train* t, const float* Bm, int ldb, const int32_t* M_dev, int M_max, int J, float* out,
                        hipStream_t s) {
  launch_colsum_partial(Bm, ldb, M_dev, M_max, J, t->part, s);
  launch_sum_parts(t->part, tn_chunks(M_max), J, out, 0, s);
}

// [C][48] (k = (ky*4 + kx)*3 + ch) -> [C][3][4][4]
__global__ void permute48_kernel(const float* __restrict__ src, int C, float* __restrict__ dst) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= C * 48) return;
  const int c = e / 48, k = e % 48;
  const int pix = k / 3, ch = k - 3 * pix, ky = pix >> 2, kx = pix & 3;
  dst[((c * 3 + ch) * 4 + ky) * 4 + kx] = src[e];
}

// sum of the 16 pixel columns of each channel: src[48] -> dst[3]
__global__ void fold48_kernel(const float* __restrict__ src, float* __restrict__ dst) {
  const int ch = threadIdx.x;
  if (ch >= 3) return;
  float acc = 0.f;
  for (int pix = 0; pix < 16; ++pix) acc += src[pix * 3 + ch];
  dst[ch] = acc;
}

// ------------------------------------------------------------------------------------------
// reverse pass
// ------------------------------------------------------------------------------------------
extern "C" dr_status dr_train_backward(dr_ctx* c, dr_saved* sv, const float* dpred, float* grads, void* stream) {
  if (!c || !sv || !dpred || !grads) return dr_fail(c, DR_EINVAL, "dr_train_backward: null argument");
  if (!c->train) return dr_fail(c, DR_EINVAL, "dr_train_backward: not a handle of this context");
  dr_train* t = static_cast<dr_train*>(c->train);
  bool mine = false;
  for (dr_saved* x : t->saved) mine = mine || x == sv;
  if (!mine || sv->owner != c || !sv->live)
    return dr_fail(c, DR_EINVAL, "dr_train_backward: not a live handle of this context");
  if (sv->wsnap_elems != c->wf32_elems)
    return dr_fail(c, DR_EINVAL, "dr_train_backward: the weights were reloaded with another layout");
  if ((size_t)sv->g.N > t->cap || sv->g.S != t->S)
    return dr_fail(c, DR_EINVAL, "dr_train_backward: workspace smaller than the handle's clip");
  HIP_OK(c, hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)stream;
  const Net& n = c->net;
  const Geo& g = sv->g;
  const int C = n.C, R = n.R, N = g.N, heads = n.cfg.heads;
  const bool b16 = sv->bf16;
  const ParamOffsets po = param_offsets(n);
  // the weights of the handle's forward: same arena layout, the handle's copy
  auto W = [&](const float* p) { return sv->wsnap + (p - c->wf32); };
  float* G = grads;
  // decoder: dyt = dpred * pred (1 - pred) per token and (ky, kx, ch)
  launch_dec_grad_tok(g, sv->pred, dpred, t->dyt, s);
  tn_grad(t, b16, sv->z, nullptr, C, t->dyt, nullptr, 48, nullptr, N, C, 48, t->tmp, s);
  permute48_kernel<<<(C * 48 + 255) / 256, 256, 0, s>>>(t->tmp, C, G + po.dw);
  colsum_grad(t, t->dyt, 48, nullptr, N, 48, t->tmp, s);
  fold48_kernel<<<1, 64, 0, s>>>(t->tmp, G + po.db);
  train_gemm(b16, t->dyt, nullptr, nullptr, N, 48, W(n.dec_w), t->zeros, C, EPI_STORE, t->dz, nullptr, s);
  // final LayerNorm
  launch_ln_bwd(sv->xf, nullptr, nullptr, N, C, W(n.lnfg), t->dz, t->dx, 0, 0, t->lnpart, s);
  launch_sum_parts(t->lnpart, ln_bwd_blocks(N), 2 * C, G + po.lnfg, 0, s);  // lnf.g then lnf.b
  KCHECK("decoder backward");
  for (int l = n.cfg.blocks - 1; l >= 0; --l) {
    const BlockW& b = n.blk[l];
    const TrainBlock& tb = sv->blk[l];
    const ParamOffsets::B& pb = po.blk[l];
    // x2 = x1 + W2 GELU(W1 LN2(x1) + b1) + b2 on the query rows
    launch_gather_rows(t->dx, sv->idx, sv->nq, N, C, t->dx2, s);
    launch_gelu_fwd(tb.hpre, sv->nq, N, R, t->a, s);
    tn_grad(t, b16, t->dx2, nullptr, C, t->a, nullptr, R, sv->nq, N, C, R, G + pb.w2, s);
    colsum_grad(t, t->dx2, C, sv->nq, N, C, G + pb.b2, s);
    train_gemm(b16, t->dx2, nullptr, sv->nq, N, C, W(b.w2T), t->zeros, R, EPI_STORE, t->da, nullptr, s);
    launch_gelu_bwd(tb.hpre, t->da, sv->nq, N, R, t->dh, s);
    tn_grad(t, b16, t->dh, nullptr, R, tb.n2, nullptr, C, sv->nq, N, R, C, G + pb.w1, s);
    colsum_grad(t, t->dh, R, sv->nq, N, R, G + pb.b1, s);
    train_gemm(b16, t->dh, nullptr, sv->nq, N, R, W(b.w1T), t->zeros, C, EPI_STORE, t->dn2, nullptr, s);
    HIP_OK(c, hipMemcpyAsync(t->dx1, t->dx2, (size_t)N * C * 4, hipMemcpyDeviceToDevice, s));
    launch_ln_bwd(tb.x1, nullptr, sv->nq, N, C, W(b.ln2g), t->dn2, t->dx1, 1, 1, t->lnpart, s);
    launch_sum_parts(t->lnpart, ln_bwd_blocks(N), 2 * C, G + pb.ln2g, 0, s);  // ln2.g then ln2.b
    // x1 = x + Wo O + bo
    tn_grad(t, b16, t->dx1, nullptr, C, tb.o, nullptr, C, sv->nq, N, C, C, G + pb.wo, s);
    colsum_grad(t, t->dx1, C, sv->nq, N, C, G + pb.bo, s);
    train_gemm(b16, t->dx1, nullptr, sv->nq, N, C, W(b.woT), t->zeros, C, EPI_STORE, t->dout, nullptr, s);
    launch_scatter_rows(t->dx1, sv->idx, sv->nq, N, C, t->dx, s);
    KCHECK("mlp/proj backward");
    // attention
    launch_attn_train_dq(g, C, heads, tb.q, tb.kv, t->dout, tb.stats, sv->woff, t->dq, t->dsum, s);
    launch_attn_train_dkv(g, C, heads, tb.q, tb.kv, t->dout, tb.stats, t->dsum, sv->woff, t->dkv, s);
    KCHECK("attention backward");
    // Q, K, V projections
    tn_grad(t, b16, t->dq, nullptr, C, tb.u, sv->idx, C, sv->nq, N, C, C, G + pb.wq, s);
    colsum_grad(t, t->dq, C, sv->nq, N, C, G + pb.bq, s);
    tn_grad(t, b16, t->dkv, nullptr, 2 * C, tb.u, nullptr, C, nullptr, N, C, C, G + pb.wk, s);
    tn_grad(t, b16, t->dkv + C, nullptr, 2 * C, tb.u, nullptr, C, nullptr, N, C, C, G + pb.wv, s);
    colsum_grad(t, t->dkv, 2 * C, nullptr, N, C, G + pb.bk, s);
    colsum_grad(t, t->dkv + C, 2 * C, nullptr, N, C, G + pb.bv, s);
    train_gemm(b16, t->dkv, nullptr, nullptr, N, 2 * C, W(b.wkvT), t->zeros, C, EPI_STORE, t->du, nullptr, s);
    train_gemm(b16, t->dq, nullptr, sv->nq, N, C, W(b.wqT), t->zeros, C, EPI_RESID, t->du, sv->idx, s);
    // LN1
    launch_ln_bwd(tb.x_in, nullptr, nullptr, N, C, W(b.ln1g), t->du, t->dx, 1, 0, t->lnpart, s);
    launch_sum_parts(t->lnpart, ln_bwd_blocks(N), 2 * C, G + pb.ln1g, 0, s);  // ln1.g then ln1.b
    KCHECK("qkv backward");
  }
  // patch embedding
  tn_grad(t, b16, t->dx, nullptr, C, sv->patches, nullptr, 48, nullptr, N, C, 48, t->tmp, s);
  permute48_kernel<<<(C * 48 + 255) / 256, 256, 0, s>>>(t->tmp, C, G + po.ew);
  colsum_grad(t, t->dx, C, nullptr, N, C, G + po.eb, s);
  KCHECK("embed backward");
  return DR_OK;
}

extern "C" dr_status dr_l1_loss(dr_ctx* c, const float* pred, const float* gt, const uint8_t* masks, size_t npix,
                                float w_in, float w_out, float* loss, float* dpred, void* stream) {
  if (!c || !pred || !gt || !masks || !loss) return dr_fail(c, DR_EINVAL, "dr_l1_loss: null argument");
  HIP_OK(c, hipSetDevice(c->device));
  dr_train* t = train_of(c);
  if (!t->lpart && hipMalloc(&t->lpart, 1024 * 4 * 4) != hipSuccess) {
    t->lpart = nullptr;
    return dr_fail(c, DR_ENOMEM, "loss scratch allocation failed");
  }
  if (!t->lacc && hipMalloc(&t->lacc, 64) != hipSuccess) {
    t->lacc = nullptr;
    return dr_fail(c, DR_ENOMEM, "loss scratch allocation failed");
  }
  launch_l1_loss(pred, gt, masks, npix, w_in, w_out, t->lpart, t->lacc, loss, dpred, (hipStream_t)stream);
  KCHECK("l1 loss");
  return DR_OK;
}

extern "C" dr_status dr_train_set_precision(dr_ctx* c, dr_precision prec) {
  if (!c) return DR_EINVAL;
  if (prec != DR_FP32 && prec != DR_BF16) return dr_fail(c, DR_EINVAL, "training precision must be FP32 or BF16");
  c->train_bf16 = prec == DR_BF16;
  return DR_OK;
}
