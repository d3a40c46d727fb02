// Host side of the C ABI: context, weight blob loading, workspace, and the launch sequence
// of the inpainting forward (see include/drinpaint.h for the contract of every call).
#include <algorithm>
#include <initializer_list>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "dr_internal.h"

namespace dr {
bool attn_bf16_supported(int dh, int spad);
}


using namespace dr;

static std::string g_create_err;

static dr_status vfail(dr_ctx* c, dr_status st, const char* fmt, va_list ap) {
  char buf[512];
  vsnprintf(buf, sizeof buf, fmt, ap);
  if (c)
    c->err = buf;
  else
    g_create_err = buf;
  return st;
}

static dr_status fail(dr_ctx* c, dr_status st, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  dr_status r = vfail(c, st, fmt, ap);
  va_end(ap);
  return r;
}

dr_status dr::dr_fail(dr_ctx* c, dr_status st, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  dr_status r = vfail(c, st, fmt, ap);
  va_end(ap);
  return r;
}

#define HIP_OK(ctx, expr)                                                              \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(ctx, DR_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));        \
  } while (0)

const char* const dr::kStageNames[ST_COUNT] = {"tokens", "embed", "ln1",  "qkv",    "attn", "proj",
                                            "ln2",    "fc1",   "fc2",  "mlp",    "decode", "copy"};

// ------------------------------------------------------------------------------------------
// small host helpers
// ------------------------------------------------------------------------------------------

static bool ranges_overlap(const void* a, size_t na, const void* b, size_t nb) {
  const char* pa = (const char*)a;
  const char* pb = (const char*)b;
  return pa < pb + nb && pb < pa + na;
}

static hipError_t dmalloc(dr_ctx* c, void** p, size_t n, std::vector<void*>& list) {
  *p = nullptr;
  if (n == 0) n = 256;
  hipError_t e = hipMalloc(p, n);
  if (e == hipSuccess) list.push_back(*p);
  return e;
}

// profiling brackets
void dr::dr_prof_begin(dr_ctx* c, hipStream_t s, hipEvent_t* a, hipEvent_t* b) {
  *a = *b = nullptr;
  if (!c->prof) return;
  for (hipEvent_t* e : {a, b}) {
    if (!c->event_pool.empty()) {
      *e = c->event_pool.back();
      c->event_pool.pop_back();
    } else {
      hipEventCreate(e);
    }
  }
  hipEventRecord(*a, s);
}

void dr::dr_prof_end(dr_ctx* c, int stage, hipStream_t s, hipEvent_t a, hipEvent_t b) {
  if (!c->prof || !a) return;
  hipEventRecord(b, s);
  c->recs.push_back({stage, a, b});
}

// ------------------------------------------------------------------------------------------
// create / destroy
// ------------------------------------------------------------------------------------------
// ------------------------------------------------------------------------------------------
// static scratch of the allocation-free token gather (dr_gather_tokens_noalloc): per-window
// query counts.  Every device the library runs on holds one copy until the process ends; its
// device address is resolved once per device, at the first dr_create there.
// ------------------------------------------------------------------------------------------
static constexpr int kScratchWindows = 1 << 16;
static __device__ __align__(256) int32_t scratch[kScratchWindows];
static std::mutex g_scratch_mu;
static int32_t* g_scratch_dev[64];  // device address of `scratch` per HIP device

static int32_t* scratch_address(int device) {
  if (device < 0 || device >= 64) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[device]) {
    void* p = nullptr;
    // the device must be current: each device holds its own copy at its own address
    if (hipSetDevice(device) == hipSuccess && hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess)
      g_scratch_dev[device] = static_cast<int32_t*>(p);
  }
  return g_scratch_dev[device];
}

extern "C" dr_status dr_create(dr_ctx** out, int device, const dr_netcfg* cfg) {
  if (!out || !cfg) return fail(nullptr, DR_EINVAL, "dr_create: null argument");
  *out = nullptr;
  const dr_netcfg& k = *cfg;
  if (k.dim <= 0 || k.dim % 64 || k.dim > 1024)
    return fail(nullptr, DR_ESHAPE, "dim must be a positive multiple of 64, at most 1024");
  if (k.heads <= 0 || k.dim % k.heads) return fail(nullptr, DR_ESHAPE, "dim %% heads != 0");
  const int dh = k.dim / k.heads;
  if (dh != 32 && dh != 64) return fail(nullptr, DR_ESHAPE, "head dim must be 32 or 64");
  if (k.blocks <= 0 || k.mlp_ratio <= 0) return fail(nullptr, DR_ESHAPE, "blocks and mlp_ratio must be >= 1");
  if (k.patch != 4) return fail(nullptr, DR_ESHAPE, "only patch 4 is supported");
  if (k.win_h <= 0 || k.win_w <= 0 || k.win_t <= 0) return fail(nullptr, DR_ESHAPE, "window extents must be >= 1");
  const int S = k.win_h * k.win_w * k.win_t;
  if (S > 320) return fail(nullptr, DR_ESHAPE, "window of %d tokens exceeds 320", S);
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
    return fail(nullptr, DR_EINVAL, "no HIP device %d", device);
  int32_t* scr = scratch_address(device);
  if (!scr) return fail(nullptr, DR_EHIP, "dr_create: cannot resolve the static scratch array on device %d", device);
  dr_ctx* c = new dr_ctx();
  c->device = device;
  c->scratch_wcount = scr;
  Net& n = c->net;
  n.cfg = k;
  n.C = k.dim;
  n.R = k.dim * k.mlp_ratio;
  n.dh = dh;
  n.S = S;
  n.Spad = (S + 15) / 16 * 16;
  n.P = k.patch;
  *out = c;
  return DR_OK;
}

void dr::dr_free_work(Work& w) {
  for (void* p : w.allocs) hipFree(p);
  w = Work();
}

// attention mode of block l (see launch_attn_clip)
static int attn_mode(const dr_ctx* c, int l) { return c->attn_pattern == 0 ? 0 : (l % 2 == 0 ? 1 : 2); }

void dr::dr_invalidate_graphs(dr_ctx* c) {
  for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
  c->graphs.clear();
  c->graph_seen.clear();
  c->graph_epoch++;
}

static void free_work(dr_ctx* c) {
  dr_invalidate_graphs(c);
  dr_free_work(c->work);
}

extern "C" void dr_destroy(dr_ctx* c) {
  if (!c) return;
  hipSetDevice(c->device);
  hipDeviceSynchronize();
  free_work(c);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  dr_train_release(c);
  for (auto& kv : c->swork) {
    dr_free_work(*kv.second);
    delete kv.second;
  }
  for (auto& kv : c->streams) {
    hipFree(kv.second.kc);
    hipFree(kv.second.vc);
  }
  dr_weights_release(c);
  for (auto& r : c->recs) {
    hipEventDestroy(r.a);
    hipEventDestroy(r.b);
  }
  for (auto e : c->event_pool) hipEventDestroy(e);
  delete c;
}

extern "C" const char* dr_last_error(dr_ctx* c) { return c ? c->err.c_str() : g_create_err.c_str(); }

extern "C" const char* dr_stage_name(int stage) {
  return (stage >= 0 && stage < ST_COUNT) ? kStageNames[stage] : nullptr;
}


// ------------------------------------------------------------------------------------------
// shapes and workspace
// ------------------------------------------------------------------------------------------
dr_status dr::dr_make_geo(dr_ctx* c, int B, int T, int H, int W, int wt, Geo& g) {
  const dr_netcfg& k = c->net.cfg;
  if (B <= 0 || T <= 0 || H <= 0 || W <= 0) return fail(c, DR_ESHAPE, "empty or negative shape");
  if (T != wt) return fail(c, DR_ESHAPE, "T=%d must equal the window length %d", T, wt);
  if (H % (k.patch * k.win_h) || W % (k.patch * k.win_w))
    return fail(c, DR_ESHAPE, "H=%d, W=%d must be multiples of %d and %d", H, W, k.patch * k.win_h,
                k.patch * k.win_w);
  g.B = B; g.T = T; g.H = H; g.W = W; g.P = k.patch;
  g.Ht = H / k.patch; g.Wt = W / k.patch;
  g.wt = wt; g.wh = k.win_h; g.ww = k.win_w;
  g.nwh = g.Ht / k.win_h; g.nww = g.Wt / k.win_w;
  g.S = wt * k.win_h * k.win_w;
  const long long N = (long long)B * T * g.Ht * g.Wt;
  if (N > (1LL << 30)) return fail(c, DR_ESHAPE, "too many tokens");
  g.N = (int)N;
  g.nwin = g.N / g.S;
  return DR_OK;
}

static dr_status make_geo(dr_ctx* c, int B, int T, int H, int W, Geo& g) {
  return dr_make_geo(c, B, T, H, W, c->net.cfg.win_t, g);
}

dr_status dr::dr_reserve_work(dr_ctx* c, Work& w, const Geo& g, bool stream_mode) {
  const bool need_contrib = !stream_mode && c->net.K != c->net.P;
  if ((size_t)g.N <= w.cap_tokens && (size_t)g.nwin <= w.cap_windows && w.stream_mode == stream_mode &&
      (!need_contrib || w.contrib))
    return DR_OK;
  HIP_OK(c, hipSetDevice(c->device));
  HIP_OK(c, hipDeviceSynchronize());
  dr_free_work(w);
  const Net& n = c->net;
  const size_t N = g.N, C = n.C, R = n.R, nw = g.nwin;
  const size_t kvlen = nw * n.cfg.heads * (size_t)n.Spad * n.dh;
  void* p;
#define ALLOC(field, bytes)                                                        \
  do {                                                                             \
    if (dmalloc(c, &p, (bytes), w.allocs) != hipSuccess) {                          \
      dr_free_work(w);                                                             \
      return fail(c, DR_ENOMEM, "workspace: cannot allocate %zu bytes", (size_t)(bytes)); \
    }                                                                              \
    w.field = (decltype(w.field))p;                                                \
  } while (0)
  ALLOC(flag, N);
  ALLOC(wcount, nw * 4);
  ALLOC(woff, (nw + 1) * 4);
  ALLOC(idx, N * 4);
  ALLOC(nq, 256);
  ALLOC(worder, nw * 4);
  ALLOC(tiles, 2 * ((N + ROW_TILE - 1) / ROW_TILE) * 4);
  ALLOC(ntiles, 256);
  ALLOC(x, N * C * 4);
  ALLOC(q16, N * C * 2);
  ALLOC(o16, N * C * 2);
  ALLOC(h16, N * R * 2);
  ALLOC(u16, N * C * 2);
  ALLOC(xh, N * C * 2);
  ALLOC(amax, (size_t)n.cfg.blocks * 4 * 4);
  if (stream_mode) {
    const size_t npix = N * 16;  // 4 x 4 pixels per token
    ALLOC(fst, npix * 12);
    ALLOC(mst, npix);
    ALLOC(ost, npix * 12);
  } else {
    ALLOC(u, N * C * 4);
    ALLOC(kv, N * 2 * C * 4);
    ALLOC(q, N * C * 4);
    ALLOC(o, N * C * 4);
    ALLOC(h, N * R * 4);
    ALLOC(k16, kvlen * 2);
    const size_t vtlen = nw * n.cfg.heads * (size_t)n.dh * attn_clip_vt_stride(n.Spad);
    ALLOC(vt16, vtlen * 2);
    if (need_contrib) ALLOC(contrib, N * 192 * 4);
    // padded key rows of K and V (columns of V^T) must read as zero
    HIP_OK(c, hipMemset(w.k16, 0, kvlen * 2));
    HIP_OK(c, hipMemset(w.vt16, 0, vtlen * 2));
  }
#undef ALLOC
  HIP_OK(c, hipDeviceSynchronize());
  w.cap_tokens = N;
  w.cap_windows = nw;
  w.stream_mode = stream_mode;
  return DR_OK;
}

static dr_status reserve_geo(dr_ctx* c, const Geo& g) {
  const bool grows = !((size_t)g.N <= c->work.cap_tokens && (size_t)g.nwin <= c->work.cap_windows &&
                       !c->work.stream_mode && (c->net.K == c->net.P || c->work.contrib));
  if (grows) dr_invalidate_graphs(c);
  return dr_reserve_work(c, c->work, g, false);
}

extern "C" dr_status dr_reserve(dr_ctx* c, int B, int T, int H, int W, dr_precision prec) {
  if (!c) return DR_EINVAL;
  if (prec != DR_FP32 && prec != DR_BF16 && prec != DR_FP8) return fail(c, DR_EINVAL, "unsupported precision %d", (int)prec);
  Geo g;
  dr_status st = make_geo(c, B, T, H, W, g);
  if (st != DR_OK) return st;
  return reserve_geo(c, g);
}

// ------------------------------------------------------------------------------------------
// forward
// ------------------------------------------------------------------------------------------
#define LAUNCH(stage, call)                                                     \
  do {                                                                          \
    hipEvent_t ea_, eb_;                                                        \
    dr_prof_begin(c, s, &ea_, &eb_);                                            \
    call;                                                                       \
    hipError_t e_ = hipGetLastError();                                          \
    if (e_ != hipSuccess)                                                       \
      return fail(c, DR_EHIP, "launch of %s failed: %s", kStageNames[stage], hipGetErrorString(e_)); \
    dr_prof_end(c, stage, s, ea_, eb_);                                         \
  } while (0)

static dr_status run_tokens(dr_ctx* c, const Geo& g, const uint8_t* masks, int all, hipStream_t s) {
  Work& w = c->work;
  LAUNCH(ST_TOKENS, launch_token_flags(g, masks, all, w.flag, w.wcount, s, c->net.K != c->net.P));
  LAUNCH(ST_TOKENS, launch_token_gather(g, w.flag, w.wcount, w.idx, w.woff, w.nq, s));
  LAUNCH(ST_TOKENS, launch_window_order(g, w.wcount, w.flag, w.worder, w.tiles, w.ntiles, s));
  return DR_OK;
}

extern "C" dr_status dr_gather_tokens(dr_ctx* c, const uint8_t* masks, int B, int T, int H, int W,
                                      dr_query_set qs, uint8_t* flag, int32_t* idx, int32_t* woff,
                                      int32_t* nq, void* stream) {
  if (!c || !masks || !flag || !idx || !woff || !nq) return fail(c, DR_EINVAL, "dr_gather_tokens: null argument");
  if (qs != DR_QUERY_MASKED && qs != DR_QUERY_ALL) return fail(c, DR_EINVAL, "bad query set");
  Geo g;
  dr_status st = make_geo(c, B, T, H, W, g);
  if (st != DR_OK) return st;
  HIP_OK(c, hipSetDevice(c->device));
  // wcount scratch comes from the workspace
  st = reserve_geo(c, g);
  if (st != DR_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  LAUNCH(ST_TOKENS, launch_token_flags(g, masks, qs == DR_QUERY_ALL, flag, c->work.wcount, s, c->net.K != c->net.P));
  LAUNCH(ST_TOKENS, launch_token_gather(g, flag, c->work.wcount, idx, woff, nq, s));
  return DR_OK;
}

extern "C" dr_status dr_gather_tokens_noalloc(dr_ctx* c, const uint8_t* masks, int B, int T, int H, int W,
                                              dr_query_set qs, uint8_t* flag, int32_t* idx, int32_t* woff,
                                              int32_t* nq, void* stream) {
  if (!c || !masks || !flag || !idx || !woff || !nq)
    return fail(c, DR_EINVAL, "dr_gather_tokens_noalloc: null argument");
  if (qs != DR_QUERY_MASKED && qs != DR_QUERY_ALL) return fail(c, DR_EINVAL, "bad query set");
  Geo g;
  dr_status st = make_geo(c, B, T, H, W, g);
  if (st != DR_OK) return st;
  if (g.nwin > kScratchWindows)
    return fail(c, DR_EINVAL, "dr_gather_tokens_noalloc: %d windows exceed the static scratch of %d", g.nwin,
                kScratchWindows);
  HIP_OK(c, hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)stream;
  // no profiling brackets here: they may create events.  Every count in scratch[0, nwin) is
  // written by the flag kernel before the gather kernel reads it, so nothing is cleared.
  launch_token_flags(g, masks, qs == DR_QUERY_ALL, flag, c->scratch_wcount, s, c->net.K != c->net.P);
  launch_token_gather(g, flag, c->scratch_wcount, idx, woff, nq, s);
  HIP_OK(c, hipGetLastError());
  return DR_OK;
}

// The per-block launch sequence.  It reads only the workspace and the weights, so the same
// sequence can be captured once per shape into a HIP graph and replayed.
static dr_status run_blocks(dr_ctx* c, const Geo& g, dr_precision prec, hipStream_t s) {
  const Net& n = c->net;
  Work& w = c->work;
  const int C = n.C, R = n.R, N = g.N;
  const int nblk = (c->debug_blocks >= 0 && c->debug_blocks < n.cfg.blocks) ? c->debug_blocks : n.cfg.blocks;
  for (int l = 0; l < nblk; ++l) {
    const BlockW& b = n.blk[l];
    if (prec == DR_FP32) {
      LAUNCH(ST_LN1, launch_ln_f32(w.x, nullptr, nullptr, N, C, b.ln1g, b.ln1b, w.u, s));
      LAUNCH(ST_QKV, launch_gemm_f32(w.u, nullptr, nullptr, N, C, b.wkv, b.bkv, 2 * C, EPI_STORE, w.kv, nullptr, s));
      LAUNCH(ST_QKV, launch_gemm_f32(w.u, w.idx, w.nq, N, C, b.wq, b.bq, C, EPI_STORE, w.q, nullptr, s));
      LAUNCH(ST_ATTN, launch_attn_f32(g, C, n.cfg.heads, w.q, w.kv, w.woff, w.o, s));
      LAUNCH(ST_PROJ, launch_gemm_f32(w.o, nullptr, w.nq, N, C, b.wo, b.bo, C, EPI_RESID, w.x, w.idx, s));
      LAUNCH(ST_LN2, launch_ln_f32(w.x, w.idx, w.nq, N, C, b.ln2g, b.ln2b, w.u, s));
      LAUNCH(ST_FC1, launch_gemm_f32(w.u, nullptr, w.nq, N, C, b.w1, b.b1, R, EPI_GELU, w.h, nullptr, s));
      LAUNCH(ST_FC2, launch_gemm_f32(w.h, nullptr, w.nq, N, R, b.w2, b.b2, C, EPI_RESID, w.x, w.idx, s));
    } else if (prec == DR_FP8) {
      float* am = w.amax + 4 * l;  // [0] LN1 out, [1] O, [2] LN2 out, [3] h
      LAUNCH(ST_LN1, launch_ln_rows_amax(w.x, nullptr, nullptr, N, w.wcount, g.S, C, b.ln1g, b.ln1b, w.u16, am + 0, s));
      LAUNCH(ST_QKV, launch_qkv_fp8(g, C, n.cfg.heads, n.Spad, attn_clip_vt_stride(n.Spad), w.u16, w.tiles, w.ntiles, b.wqkv8, b.wscale8, b.bqkv, am + 0, (float)(1.4426950408889634 / std::sqrt((double)n.dh)), w.q16, w.k16, w.vt16, s));
      LAUNCH(ST_ATTN, launch_attn_clip(g, C, n.cfg.heads, n.Spad, w.q16, w.k16, w.vt16, w.idx, w.woff, w.worder, w.o16, am + 1, attn_mode(c, l), s));
      LAUNCH(ST_PROJ, launch_gemm_fp8_resid(w.o16, w.nq, N, C, b.wo8, b.wscale8 + 3, am + 1, b.bo, C, w.x, w.idx, s));
      LAUNCH(ST_LN2, launch_ln_rows_amax(w.x, w.idx, w.nq, N, nullptr, g.S, C, b.ln2g, b.ln2b, w.u16, am + 2, s));
      LAUNCH(ST_FC1, launch_fc1_fp8(N, w.nq, C, R, w.u16, b.w18, b.wscale8 + 4, b.b1, am + 2, w.h16, am + 3, s));
      LAUNCH(ST_FC2, launch_gemm_fp8_resid(w.h16, w.nq, N, R, b.w28, b.wscale8 + 5, am + 3, b.b2, C, w.x, w.idx, s));
    } else {
      // x^ (normalised rows) feeds Q/K/V; the projection leaves x1^ of the query rows in u16
      // for the MLP; the second MLP linear refreshes x^ of the query rows
      LAUNCH(ST_QKV, launch_qkv_bf16(g, C, n.cfg.heads, n.Spad, attn_clip_vt_stride(n.Spad), w.xh, w.tiles, w.ntiles, b.wqkvf16, b.bqkvf, w.q16, w.k16, w.vt16, s));
      LAUNCH(ST_ATTN, launch_attn_clip(g, C, n.cfg.heads, n.Spad, w.q16, w.k16, w.vt16, w.idx, w.woff, w.worder, w.o16, nullptr, attn_mode(c, l), s));
      if (mlp_block_supported(C, R)) {
        LAUNCH(ST_MLP, launch_mlp_block_bf16(N, w.nq, C, w.o16, w.idx, b.wo16, b.bo, b.w1f16, b.b1f, b.w216, b.b2, w.x, w.xh, s));
      } else {
        LAUNCH(ST_PROJ, launch_resid_ln_bf16(N, w.nq, C, C, w.o16, b.wo16, b.bo, w.x, w.idx, w.u16, nullptr, s));
        LAUNCH(ST_FC1, launch_fc1_bf16(N, w.nq, C, R, w.u16, b.w1f16, b.b1f, w.h16, s));
        LAUNCH(ST_FC2, launch_resid_ln_bf16(N, w.nq, C, R, w.h16, b.w216, b.b2, w.x, w.idx, w.xh, w.idx, s));
      }
    }
  }
  return DR_OK;
}

static std::string graph_key(const Geo& g, dr_precision prec) {
  char buf[128];
  snprintf(buf, sizeof buf, "%d,%d,%d,%d,%d,%d", g.B, g.T, g.H, g.W, (int)prec, 0);
  return buf;
}

extern "C" dr_status dr_inpaint(dr_ctx* c, const float* frames, const uint8_t* masks, float* out,
                                int B, int T, int H, int W, dr_precision prec, dr_query_set qs,
                                void* stream) {
  if (!c) return DR_EINVAL;
  if (!frames || !masks || !out) return fail(c, DR_EINVAL, "dr_inpaint: null pointer");
  if (!c->have_weights) return fail(c, DR_EINVAL, "dr_inpaint: no weights loaded");
  if (prec != DR_FP32 && prec != DR_BF16 && prec != DR_FP8) return fail(c, DR_EINVAL, "unsupported precision %d", (int)prec);
  if (qs != DR_QUERY_MASKED && qs != DR_QUERY_ALL) return fail(c, DR_EINVAL, "bad query set");
  Geo g;
  dr_status st = make_geo(c, B, T, H, W, g);
  if (st != DR_OK) return st;
  const Net& n = c->net;
  if (prec != DR_FP32 && !attn_bf16_supported(n.dh, n.Spad))
    return fail(c, DR_ESHAPE, "BF16 attention has no kernel for %d-token windows", n.S);
  if (prec == DR_BF16 && (!resid_ln_supported(n.C) || n.cfg.patch != 4 || !window_order_supported(g.S)))
    return fail(c, DR_ESHAPE, "the BF16 path needs dim 64, 128, 256 or 384 and patch 4");
  if (prec == DR_FP8 && !fp8_supported(n.C, n.R))
    return fail(c, DR_ESHAPE, "the FP8 path needs dim and hidden width multiples of 128");
  if (prec == DR_FP32 && c->attn_pattern != 0)
    return fail(c, DR_EINVAL, "decoupled attention runs on the BF16 and FP8 paths");
  const bool ovl = n.K != n.P;
  if (ovl && prec != DR_BF16) return fail(c, DR_EINVAL, "the overlapping embedding and decoder run on the BF16 path");
  const size_t npix = (size_t)B * T * H * W;
  if (out != frames && ranges_overlap(out, npix * 12, frames, npix * 12))
    return fail(c, DR_EINVAL, "out partially overlaps frames");
  if (ranges_overlap(out, npix * 12, masks, npix)) return fail(c, DR_EINVAL, "out overlaps masks");
  if (((uintptr_t)frames & 15) || ((uintptr_t)masks & 3))
    return fail(c, DR_EINVAL, "frames must be 16-byte and masks 4-byte aligned");
  HIP_OK(c, hipSetDevice(c->device));
  st = reserve_geo(c, g);
  if (st != DR_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  Work& w = c->work;
  const int C = n.C, R = n.R, N = g.N;
  if (prec == DR_BF16 && !ovl) {
    // token lists, window order and the embedding in one launch after the flags
    LAUNCH(ST_TOKENS, launch_token_flags(g, masks, qs == DR_QUERY_ALL, w.flag, w.wcount, s, 0));
    LAUNCH(ST_TOKENS, launch_tokens_embed_bf16(g, C, frames, masks, w.flag, w.wcount, w.wcount, n.embed_wT16, n.embed_b,
                                               w.x, w.xh, w.idx, w.woff, w.nq, w.worder, w.tiles, w.ntiles, s));
  } else {
    st = run_tokens(c, g, masks, qs == DR_QUERY_ALL, s);
    if (st != DR_OK) return st;
    if (ovl)
      LAUNCH(ST_EMBED, launch_embed_ovl_bf16(g, C, frames, masks, w.flag, w.wcount, n.embed_ovl16, n.embed_b, w.x, w.xh, s));
    else
      LAUNCH(ST_EMBED, launch_embed(g, C, frames, masks, n.embed_wT, n.embed_b, w.x, s));
  }
  if (prec == DR_FP8) LAUNCH(ST_LN1, launch_zero_f32(w.amax, 4 * n.cfg.blocks, s));
  dr_status br = DR_OK;
  const bool graphable = c->use_graphs && !c->prof && c->debug_blocks < 0;
  if (graphable) {
    const std::string key = graph_key(g, prec) + "#" + std::to_string(c->graph_epoch);
    auto it = c->graphs.find(key);
    if (it != c->graphs.end()) {
      HIP_OK(c, hipGraphLaunch(it->second, s));
    } else if (!c->graph_seen.count(key)) {
      // first call of this shape runs eagerly (and sets kernel attributes); the next one
      // captures
      c->graph_seen.insert(key);
      br = run_blocks(c, g, prec, s);
    } else {
      if (!c->cap_stream) HIP_OK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
      HIP_OK(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed));
      br = run_blocks(c, g, prec, c->cap_stream);
      hipGraph_t graph = nullptr;
      hipError_t ec = hipStreamEndCapture(c->cap_stream, &graph);
      if (br != DR_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return br;
      }
      if (ec != hipSuccess) return fail(c, DR_EHIP, "graph capture failed: %s", hipGetErrorString(ec));
      hipGraphExec_t exec = nullptr;
      ec = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (ec != hipSuccess) return fail(c, DR_EHIP, "graph instantiation failed: %s", hipGetErrorString(ec));
      c->graphs[key] = exec;
      HIP_OK(c, hipGraphLaunch(exec, s));
    }
  } else {
    br = run_blocks(c, g, prec, s);
  }
  if (br != DR_OK) return br;
  if (ovl) {
    LAUNCH(ST_DECODE, launch_decode_ovl_bf16(g, C, w.xh, w.idx, w.nq, n.dec_ovl16, n.dec_ovl_bf, w.contrib, s));
    LAUNCH(ST_DECODE, launch_fold_ovl(g, w.contrib, n.dec_ovl_b, masks, out, s));
  } else if (prec == DR_BF16) {  // decoder and unmasked copy in one launch
    LAUNCH(ST_DECODE, launch_decode_copy_bf16(g, C, w.xh, w.idx, w.nq, n.dec_wf16, n.dec_bf, masks, frames, out,
                                              npix, s));
    return DR_OK;
  } else
    LAUNCH(ST_DECODE, launch_decode(g, C, w.x, w.idx, w.nq, n.lnfg, n.lnfb, n.dec_w, n.dec_b, masks, out, s));
  if (out != frames) LAUNCH(ST_COPY, launch_copy_unmasked(npix, frames, masks, out, s));
  return DR_OK;
}

// ------------------------------------------------------------------------------------------
// profiling
// ------------------------------------------------------------------------------------------
extern "C" dr_status dr_profile(dr_ctx* c, int enable) {
  if (!c) return DR_EINVAL;
  c->prof = enable != 0;
  return DR_OK;
}

extern "C" dr_status dr_profile_read(dr_ctx* c, double* ms, int64_t* count, int nstage) {
  if (!c || !ms || !count || nstage < 0) return fail(c, DR_EINVAL, "dr_profile_read: bad argument");
  for (int i = 0; i < nstage; ++i) {
    ms[i] = 0.0;
    count[i] = 0;
  }
  HIP_OK(c, hipSetDevice(c->device));
  dr_status st = DR_OK;
  for (auto& r : c->recs) {
    float t = 0.f;
    hipError_t e = hipEventSynchronize(r.b);
    if (e == hipSuccess) e = hipEventElapsedTime(&t, r.a, r.b);
    if (e != hipSuccess && st == DR_OK) st = fail(c, DR_EHIP, "profile events: %s", hipGetErrorString(e));
    if (r.stage < nstage) {
      ms[r.stage] += t;
      count[r.stage] += 1;
    }
    c->event_pool.push_back(r.a);
    c->event_pool.push_back(r.b);
  }
  c->recs.clear();
  return st;
}

// ------------------------------------------------------------------------------------------
// inspection
// ------------------------------------------------------------------------------------------
extern "C" dr_status dr_inspect(dr_ctx* c, const char* name, void* dst, size_t nbytes, void* stream) {
  if (!c || !name || !dst) return fail(c, DR_EINVAL, "dr_inspect: null argument");
  const Work& w = c->work;
  const size_t N = w.cap_tokens, C = c->net.C, R = c->net.R;
  const size_t kvlen = w.cap_windows * c->net.cfg.heads * (size_t)c->net.Spad * c->net.dh;
  struct Buf { const char* n; const void* p; size_t bytes; } bufs[] = {
      {"x", w.x, N * C * 4},       {"xh", w.xh, N * C * 2},     {"u16", w.u16, N * C * 2}, {"q16", w.q16, N * C * 2},
      {"k16", w.k16, kvlen * 2},
      {"vt16", w.vt16, w.cap_windows * c->net.cfg.heads * (size_t)c->net.dh * attn_clip_vt_stride(c->net.Spad) * 2}, {"o16", w.o16, N * C * 2},
      {"h16", w.h16, N * R * 2},   {"u", w.u, N * C * 4},     {"kv", w.kv, N * 2 * C * 4},
      {"q", w.q, N * C * 4},       {"o", w.o, N * C * 4},     {"h", w.h, N * R * 4},
      {"flag", w.flag, N},         {"idx", w.idx, N * 4},     {"nq", w.nq, 4},
      {"wcount", w.wcount, w.cap_windows * 4},                  {"worder", w.worder, w.cap_windows * 4},
      {"tiles", w.tiles, 2 * ((N + ROW_TILE - 1) / ROW_TILE) * 4}, {"ntiles", w.ntiles, 8}};
  for (const Buf& b : bufs) {
    if (std::strcmp(b.n, name) == 0) {
      if (!b.p) return fail(c, DR_EINVAL, "dr_inspect: no workspace yet");
      if (nbytes > b.bytes) return fail(c, DR_EINVAL, "dr_inspect: %zu bytes requested, buffer has %zu", nbytes, b.bytes);
      HIP_OK(c, hipMemcpyAsync(dst, b.p, nbytes, hipMemcpyDeviceToDevice, (hipStream_t)stream));
      return DR_OK;
    }
  }
  return fail(c, DR_EINVAL, "dr_inspect: unknown buffer '%s'", name);
}

extern "C" dr_status dr_set_attention_pattern(dr_ctx* c, int pattern) {
  if (!c) return DR_EINVAL;
  if (pattern != 0 && pattern != 1) return fail(c, DR_EINVAL, "attention pattern %d (0 joint, 1 decoupled)", pattern);
  if (pattern == 1 && c->net.cfg.win_t > 8) return fail(c, DR_EINVAL, "decoupled attention takes at most 8 frames per window");
  if (c->attn_pattern != pattern) {
    HIP_OK(c, hipSetDevice(c->device));
    HIP_OK(c, hipDeviceSynchronize());
    dr_invalidate_graphs(c);  // captured block sequences hold the previous attention kernels
    c->attn_pattern = pattern;
  }
  return DR_OK;
}

extern "C" dr_status dr_debug_set(dr_ctx* c, const char* key, int64_t value) {
  if (!c || !key) return fail(c, DR_EINVAL, "dr_debug_set: null argument");
  if (std::strcmp(key, "blocks") == 0) {
    c->debug_blocks = (int)value;
    return DR_OK;
  }
  if (std::strcmp(key, "graphs") == 0) {
    c->use_graphs = value != 0;
    return DR_OK;
  }
  return fail(c, DR_EINVAL, "dr_debug_set: unknown key '%s'", key);
}

extern "C" dr_status dr_fp8_encode(dr_ctx* c, const float* in, uint8_t* out, size_t n, float scale, void* stream) {
  if (!c || !in || !out || !(scale > 0.f)) return fail(c, DR_EINVAL, "dr_fp8_encode: bad argument");
  HIP_OK(c, hipSetDevice(c->device));
  launch_quantize_fp8(in, out, n, 1.0f / scale, (hipStream_t)stream);
  HIP_OK(c, hipGetLastError());
  return DR_OK;
}
