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
void launch_attn_f32_save(const Geo& g, int C, int heads, const float* q, const float* kv, const int32_t* woff,
                          float* o, float2* stats, hipStream_t s);
void launch_attn_bwd_q(const Geo& g, int C, int heads, const float* q, const float* kv, const float* dout,
                       const float2* stats, const int32_t* woff, float* dq, float* P, float* dS, hipStream_t s);
void launch_attn_bwd_kv(const Geo& g, int C, int heads, const float* q, const float* dout, const float* P,
                        const float* dS, const int32_t* woff, float* dkv, hipStream_t s);
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
// training workspace (kept in the context between forward and backward)
// ------------------------------------------------------------------------------------------
struct TrainBlock {
  float *x_in, *u, *kv, *q, *o, *x1, *n2, *hpre;
  float2* stats;
};

struct dr_train {
  Geo g{};
  size_t cap = 0;  // tokens
  std::vector<void*> allocs;
  // gather lists
  uint8_t* flag = nullptr;
  int32_t *wcount = nullptr, *woff = nullptr, *idx = nullptr, *nq = nullptr;
  std::vector<TrainBlock> blk;
  float *x = nullptr, *xf = nullptr, *z = nullptr, *pred = nullptr, *patches = nullptr;
  // backward scratch
  float *a = nullptr, *dx = nullptr, *dx2 = nullptr, *dx1 = nullptr, *da = nullptr, *dh = nullptr, *dn2 = nullptr,
        *dout = nullptr, *dq = nullptr, *dkv = nullptr, *du = nullptr, *P = nullptr, *dS = nullptr, *dyt = nullptr,
        *dz = nullptr, *part = nullptr, *lnpart = nullptr, *zeros = nullptr, *tmp = nullptr;
  float *lpart = nullptr, *lacc = nullptr;
  bool have_fwd = false;
  bool bf16 = false;  // precision of the products of the last forward (and of its reverse pass)
};

static void train_free(dr_train* t) {
  for (void* p : t->allocs) (void)hipFree(p);
  t->allocs.clear();
  t->blk.clear();
  t->cap = 0;
}

// products of both passes: FP32 operands, or bf16 operands with FP32 accumulation
static void train_gemm(const dr_train* t, const float* A, const int32_t* arows, const int32_t* m_dev, int m_max,
                       int K, const float* W, const float* bias, int Nout, int epi, float* out,
                       const int32_t* res_rows, hipStream_t s) {
  (t->bf16 ? launch_gemm_bf16ops : launch_gemm_f32)(A, arows, m_dev, m_max, K, W, bias, Nout, epi, out, res_rows, s);
}

static dr_train* train_of(dr_ctx* c) {
  if (!c->train) c->train = new dr_train();
  return static_cast<dr_train*>(c->train);
}

void dr::dr_train_release(dr_ctx* c) {
  if (!c->train) return;
  dr_train* t = static_cast<dr_train*>(c->train);
  train_free(t);
  delete t;
  c->train = nullptr;
}

static dr_status train_reserve(dr_ctx* c, dr_train* t, const Geo& g) {
  if ((size_t)g.N <= t->cap && t->g.S == g.S) {
    t->g = g;
    return DR_OK;
  }
  HIP_OK(c, hipDeviceSynchronize());
  train_free(t);
  const Net& n = c->net;
  const size_t N = g.N, C = n.C, R = n.R, L = n.cfg.blocks, H = n.cfg.heads, nw = g.nwin;
  auto A = [&](size_t bytes) -> void* {
    void* p = nullptr;
    if (hipMalloc(&p, bytes ? bytes : 256) != hipSuccess) return nullptr;
    t->allocs.push_back(p);
    return p;
  };
  bool ok = true;
#define TA(field, bytes)                         \
  do {                                           \
    t->field = (decltype(t->field))A(bytes);     \
    ok = ok && t->field;                         \
  } while (0)
  TA(flag, N);
  TA(wcount, nw * 4);
  TA(woff, (nw + 1) * 4);
  TA(idx, N * 4);
  TA(nq, 256);
  t->blk.resize(L);
  for (size_t l = 0; l < L; ++l) {
    TrainBlock& b = t->blk[l];
    b.x_in = (float*)A(N * C * 4);
    b.u = (float*)A(N * C * 4);
    b.kv = (float*)A(N * 2 * C * 4);
    b.q = (float*)A(N * C * 4);
    b.o = (float*)A(N * C * 4);
    b.x1 = (float*)A(N * C * 4);
    b.n2 = (float*)A(N * C * 4);
    b.hpre = (float*)A(N * R * 4);
    b.stats = (float2*)A(N * H * 8);
    ok = ok && b.x_in && b.u && b.kv && b.q && b.o && b.x1 && b.n2 && b.hpre && b.stats;
  }
  TA(x, N * C * 4);
  TA(xf, N * C * 4);
  TA(z, N * C * 4);
  TA(pred, N * 16 * 12);
  TA(patches, N * 48 * 4);
  TA(a, N * R * 4);
  TA(dx, N * C * 4);
  TA(dx2, N * C * 4);
  TA(dx1, N * C * 4);
  TA(da, N * R * 4);
  TA(dh, N * R * 4);
  TA(dn2, N * C * 4);
  TA(dout, N * C * 4);
  TA(dq, N * C * 4);
  TA(dkv, N * 2 * C * 4);
  TA(du, N * C * 4);
  TA(P, N * H * g.S * 4);
  TA(dS, N * H * g.S * 4);
  TA(dyt, N * 48 * 4);
  TA(dz, N * C * 4);
  TA(part, (size_t)tn_chunks((int)N) * R * C * 4);
  TA(lnpart, (size_t)ln_bwd_blocks((int)N) * 2 * C * 4);
  TA(zeros, (2 * C + R + 64) * 4);
  TA(tmp, (R * C + 64) * 4);
  TA(lpart, 1024 * 4 * 4);
  TA(lacc, 64);
#undef TA
  if (!ok) {
    train_free(t);
    return dr_fail(c, DR_ENOMEM, "training workspace allocation failed");
  }
  HIP_OK(c, hipMemset(t->zeros, 0, (2 * C + R + 64) * 4));
  HIP_OK(c, hipDeviceSynchronize());
  t->cap = N;
  t->g = g;
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
extern "C" dr_status dr_train_forward(dr_ctx* c, const float* frames, const uint8_t* masks, float* pred, int B,
                                      int T, int H, int W, void* stream) {
  if (!c || !frames || !masks || !pred) return dr_fail(c, DR_EINVAL, "dr_train_forward: null argument");
  if (!c->have_weights) return dr_fail(c, DR_EINVAL, "no weights loaded");
  if (c->attn_pattern != 0) return dr_fail(c, DR_EINVAL, "training runs the joint-attention network");
  if (c->net.K != c->net.P) return dr_fail(c, DR_EINVAL, "training runs the non-overlapping embedding");
  Geo g;
  dr_status st = dr_make_geo(c, B, T, H, W, c->net.cfg.win_t, g);
  if (st != DR_OK) return st;
  HIP_OK(c, hipSetDevice(c->device));
  dr_train* t = train_of(c);
  st = train_reserve(c, t, g);
  if (st != DR_OK) return st;
  t->bf16 = c->train_bf16 != 0;
  hipStream_t s = (hipStream_t)stream;
  const Net& n = c->net;
  const int C = n.C, R = n.R, N = g.N, heads = n.cfg.heads;
  launch_token_flags(g, masks, 0, t->flag, t->wcount, s);
  launch_token_gather(g, t->flag, t->wcount, t->idx, t->woff, t->nq, s);
  launch_embed(g, C, frames, masks, n.embed_wT, n.embed_b, t->x, s);
  launch_patches(g, frames, masks, t->patches, s);
  KCHECK("embed");
  for (int l = 0; l < n.cfg.blocks; ++l) {
    const BlockW& b = n.blk[l];
    TrainBlock& tb = t->blk[l];
    HIP_OK(c, hipMemcpyAsync(tb.x_in, t->x, (size_t)N * C * 4, hipMemcpyDeviceToDevice, s));
    launch_ln_f32(t->x, nullptr, nullptr, N, C, b.ln1g, b.ln1b, tb.u, s);
    train_gemm(t, tb.u, nullptr, nullptr, N, C, b.wkv, b.bkv, 2 * C, EPI_STORE, tb.kv, nullptr, s);
    train_gemm(t, tb.u, t->idx, t->nq, N, C, b.wq, b.bq, C, EPI_STORE, tb.q, nullptr, s);
    launch_attn_f32_save(g, C, heads, tb.q, tb.kv, t->woff, tb.o, tb.stats, s);
    train_gemm(t, tb.o, nullptr, t->nq, N, C, b.wo, b.bo, C, EPI_RESID, t->x, t->idx, s);
    launch_gather_rows(t->x, t->idx, t->nq, N, C, tb.x1, s);
    launch_ln_f32(tb.x1, nullptr, t->nq, N, C, b.ln2g, b.ln2b, tb.n2, s);
    train_gemm(t, tb.n2, nullptr, t->nq, N, C, b.w1, b.b1, R, EPI_STORE, tb.hpre, nullptr, s);
    launch_gelu_fwd(tb.hpre, t->nq, N, R, t->a, s);
    train_gemm(t, t->a, nullptr, t->nq, N, R, b.w2, b.b2, C, EPI_RESID, t->x, t->idx, s);
    KCHECK("block");
  }
  HIP_OK(c, hipMemcpyAsync(t->xf, t->x, (size_t)N * C * 4, hipMemcpyDeviceToDevice, s));
  launch_ln_f32(t->x, nullptr, nullptr, N, C, n.lnfg, n.lnfb, t->z, s);
  launch_decoder_full(g, C, t->z, n.dec_w, n.dec_b, t->pred, s);
  KCHECK("decoder");
  HIP_OK(c, hipMemcpyAsync(pred, t->pred, (size_t)N * 16 * 12, hipMemcpyDeviceToDevice, s));
  t->have_fwd = true;
  return DR_OK;
}

// grads[off .. off + I*J) = sum over chunks of TN partials
static void tn_grad(dr_train* t, const float* A, const int32_t* arow, int lda, const float* Bm, const int32_t* brow,
                    int ldb, const int32_t* M_dev, int M_max, int I, int J, float* out, hipStream_t s) {
  (t->bf16 ? launch_tn_bf16ops : launch_tn_partial)(A, arow, lda, Bm, brow, ldb, M_dev, M_max, I, J, t->part, s);
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
extern "C" dr_status dr_train_backward(dr_ctx* c, const float* dpred, float* grads, void* stream) {
  if (!c || !dpred || !grads) return dr_fail(c, DR_EINVAL, "dr_train_backward: null argument");
  dr_train* t = train_of(c);
  if (!t->have_fwd) return dr_fail(c, DR_EINVAL, "dr_train_backward needs a preceding dr_train_forward");
  HIP_OK(c, hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)stream;
  const Net& n = c->net;
  const Geo& g = t->g;
  const int C = n.C, R = n.R, N = g.N, heads = n.cfg.heads;
  const ParamOffsets po = param_offsets(n);
  float* G = grads;
  // decoder: dyt = dpred * pred (1 - pred) per token and (ky, kx, ch)
  launch_dec_grad_tok(g, t->pred, dpred, t->dyt, s);
  tn_grad(t, t->z, nullptr, C, t->dyt, nullptr, 48, nullptr, N, C, 48, t->tmp, s);
  permute48_kernel<<<(C * 48 + 255) / 256, 256, 0, s>>>(t->tmp, C, G + po.dw);
  colsum_grad(t, t->dyt, 48, nullptr, N, 48, t->tmp, s);
  fold48_kernel<<<1, 64, 0, s>>>(t->tmp, G + po.db);
  train_gemm(t, t->dyt, nullptr, nullptr, N, 48, n.dec_w, t->zeros, C, EPI_STORE, t->dz, nullptr, s);
  // final LayerNorm
  launch_ln_bwd(t->xf, nullptr, nullptr, N, C, n.lnfg, t->dz, t->dx, 0, 0, t->lnpart, s);
  launch_sum_parts(t->lnpart, ln_bwd_blocks(N), 2 * C, G + po.lnfg, 0, s);  // lnf.g then lnf.b
  KCHECK("decoder backward");
  for (int l = n.cfg.blocks - 1; l >= 0; --l) {
    const BlockW& b = n.blk[l];
    const TrainBlock& tb = t->blk[l];
    const ParamOffsets::B& pb = po.blk[l];
    // x2 = x1 + W2 GELU(W1 LN2(x1) + b1) + b2 on the query rows
    launch_gather_rows(t->dx, t->idx, t->nq, N, C, t->dx2, s);
    launch_gelu_fwd(tb.hpre, t->nq, N, R, t->a, s);
    tn_grad(t, t->dx2, nullptr, C, t->a, nullptr, R, t->nq, N, C, R, G + pb.w2, s);
    colsum_grad(t, t->dx2, C, t->nq, N, C, G + pb.b2, s);
    train_gemm(t, t->dx2, nullptr, t->nq, N, C, b.w2T, t->zeros, R, EPI_STORE, t->da, nullptr, s);
    launch_gelu_bwd(tb.hpre, t->da, t->nq, N, R, t->dh, s);
    tn_grad(t, t->dh, nullptr, R, tb.n2, nullptr, C, t->nq, N, R, C, G + pb.w1, s);
    colsum_grad(t, t->dh, R, t->nq, N, R, G + pb.b1, s);
    train_gemm(t, t->dh, nullptr, t->nq, N, R, b.w1T, t->zeros, C, EPI_STORE, t->dn2, nullptr, s);
    HIP_OK(c, hipMemcpyAsync(t->dx1, t->dx2, (size_t)N * C * 4, hipMemcpyDeviceToDevice, s));
    launch_ln_bwd(tb.x1, nullptr, t->nq, N, C, b.ln2g, t->dn2, t->dx1, 1, 1, t->lnpart, s);
    launch_sum_parts(t->lnpart, ln_bwd_blocks(N), 2 * C, G + pb.ln2g, 0, s);  // ln2.g then ln2.b
    // x1 = x + Wo O + bo
    tn_grad(t, t->dx1, nullptr, C, tb.o, nullptr, C, t->nq, N, C, C, G + pb.wo, s);
    colsum_grad(t, t->dx1, C, t->nq, N, C, G + pb.bo, s);
    train_gemm(t, t->dx1, nullptr, t->nq, N, C, b.woT, t->zeros, C, EPI_STORE, t->dout, nullptr, s);
    launch_scatter_rows(t->dx1, t->idx, t->nq, N, C, t->dx, s);
    KCHECK("mlp/proj backward");
    // attention
    launch_attn_bwd_q(g, C, heads, tb.q, tb.kv, t->dout, tb.stats, t->woff, t->dq, t->P, t->dS, s);
    launch_attn_bwd_kv(g, C, heads, tb.q, t->dout, t->P, t->dS, t->woff, t->dkv, s);
    KCHECK("attention backward");
    // Q, K, V projections
    tn_grad(t, t->dq, nullptr, C, tb.u, t->idx, C, t->nq, N, C, C, G + pb.wq, s);
    colsum_grad(t, t->dq, C, t->nq, N, C, G + pb.bq, s);
    tn_grad(t, t->dkv, nullptr, 2 * C, tb.u, nullptr, C, nullptr, N, C, C, G + pb.wk, s);
    tn_grad(t, t->dkv + C, nullptr, 2 * C, tb.u, nullptr, C, nullptr, N, C, C, G + pb.wv, s);
    colsum_grad(t, t->dkv, 2 * C, nullptr, N, C, G + pb.bk, s);
    colsum_grad(t, t->dkv + C, 2 * C, nullptr, N, C, G + pb.bv, s);
    train_gemm(t, t->dkv, nullptr, nullptr, N, 2 * C, b.wkvT, t->zeros, C, EPI_STORE, t->du, nullptr, s);
    train_gemm(t, t->dq, nullptr, t->nq, N, C, b.wqT, t->zeros, C, EPI_RESID, t->du, t->idx, s);
    // LN1
    launch_ln_bwd(tb.x_in, nullptr, nullptr, N, C, b.ln1g, t->du, t->dx, 1, 0, t->lnpart, s);
    launch_sum_parts(t->lnpart, ln_bwd_blocks(N), 2 * C, G + pb.ln1g, 0, s);  // ln1.g then ln1.b
    KCHECK("qkv backward");
  }
  // patch embedding
  tn_grad(t, t->dx, nullptr, C, t->patches, nullptr, 48, nullptr, N, C, 48, t->tmp, s);
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
  if (!t->lpart) {
    if (hipMalloc(&t->lpart, 1024 * 4 * 4) != hipSuccess || hipMalloc(&t->lacc, 64) != hipSuccess)
      return dr_fail(c, DR_ENOMEM, "loss scratch allocation failed");
    t->allocs.push_back(t->lpart);
    t->allocs.push_back(t->lacc);
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
