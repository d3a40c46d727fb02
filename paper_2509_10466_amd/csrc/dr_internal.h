// Internal declarations shared by the library's translation units (host side and device
// helpers).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <utility>
#include <vector>

#include "../../include/drinpaint.h"
#include "dr_device.h"

namespace dr {

typedef uint16_t bf16;  // raw bfloat16 bits

// ------------------------------------------------------------------------------------------
// Stages (profiling ids)
// ------------------------------------------------------------------------------------------
enum Stage {
  ST_TOKENS = 0,  // token flags, per-window counts, gather lists
  ST_EMBED,       // cut-out + patch embedding
  ST_LN1,         // LayerNorm before attention
  ST_QKV,         // Q/K/V projection
  ST_ATTN,        // window attention
  ST_PROJ,        // output projection + residual
  ST_LN2,         // LayerNorm before the MLP
  ST_FC1,         // first MLP linear + GELU
  ST_FC2,         // second MLP linear + residual
  ST_MLP,         // fused projection + residual + MLP + residual (BF16)
  ST_DECODE,      // final LayerNorm + decoder + sigmoid + masked store
  ST_COPY,        // unmasked pixels copied to the output
  ST_COUNT
};

// ------------------------------------------------------------------------------------------
// Device-side parameter views
// ------------------------------------------------------------------------------------------
struct BlockW {
  const float *ln1g, *ln1b, *ln2g, *ln2b;
  const float *wq, *wk, *wv, *wo, *w1, *w2;  // f32 [out, in]
  const float *bq, *bk, *bv, *bo, *b1, *b2;
  const float* wkv;                          // f32 [2C, C]  (Wk rows then Wv rows)
  const float* bkv;                          // f32 [2C]
  const float* bqkv;                         // f32 [3C]
  const bf16* wqkv16;                        // bf16 [3C, C]
  const bf16 *wo16, *w116, *w216;            // bf16 [out, in]
  // LayerNorm affine parts folded into the following linear (BF16 path):
  // W' = W diag(g), b' = b + W beta
  const bf16 *wqkvf16, *w1f16;               // bf16 [3C, C], [R, C]
  const float *bqkvf, *b1f;                  // f32 [3C], [R]
  const uint8_t* wqkv8;                      // e4m3 [3C, C] (Wq, Wk, Wv each / own scale)
  const uint8_t *wo8, *w18, *w28;            // e4m3 [out, in]
  const float* wscale8;                      // device: s_q, s_k, s_v, s_o, s_1, s_2
  // transposed FP32 copies for the input gradients of the backward pass ([in, out])
  const float *wqT, *wkvT, *woT, *w1T, *w2T;  // [C,C], [C,2C], [C,C], [C,R], [R,C]
};

struct Net {
  dr_netcfg cfg;
  int C, R, dh, S, Spad, P;  // dim, hidden, head dim, window tokens, padded window, patch
  const float* embed_wT;     // [48][C], row k = (ky*p + kx)*3 + c
  const float* embed_b;      // [C]
  std::vector<BlockW> blk;
  const float *lnfg, *lnfb;
  const float* dec_w;        // [C][48], column k = (ky*p + kx)*3 + ch
  const float* dec_b;        // [3]
  const bf16* embed_wT16;    // bf16 [C][64]: embedding weight, k slots permuted for the MFMA embedding
  const bf16* dec_wf16;      // bf16 [48][C]: decoder weight with the final LayerNorm gain folded in
  const float* dec_bf;       // f32 [48]: decoder bias + final LayerNorm shift through the decoder
  // overlapping embedding and decoder (K = 2P; K = P otherwise and these are null)
  int K = 4;
  const bf16* embed_ovl16 = nullptr;  // bf16 [C][192], slot order of the overlapping embedding
  const bf16* dec_ovl16 = nullptr;    // bf16 [192][C]: decoder with the final LayerNorm gain folded in
  const float* dec_ovl_bf = nullptr;  // f32 [192]: final LayerNorm shift through the decoder (per token)
  const float* dec_ovl_b = nullptr;   // f32 [3]: decoder bias (once per pixel)
};

struct Work {
  int B = 0, T = 0, H = 0, W = 0;
  int N = 0, nwin = 0;
  size_t cap_tokens = 0;  // capacity in tokens
  size_t cap_windows = 0;
  // token gather
  uint8_t* flag = nullptr;
  int32_t* wcount = nullptr;
  int32_t* woff = nullptr;
  int32_t* idx = nullptr;
  int32_t* nq = nullptr;
  int32_t* worder = nullptr;  // windows by decreasing query count
  int32_t* tiles = nullptr;   // [2][ceil(N / ROW_TILE)]: row tiles with a flagged token, then
                              // row tiles touching a window with queries (any order)
  int32_t* ntiles = nullptr;  // [2]: lengths of the two lists
  // residual stream, FP32, window-major rows
  float* x = nullptr;
  // FP32 path scratch
  float *u = nullptr, *kv = nullptr, *q = nullptr, *o = nullptr, *h = nullptr;
  // BF16 path: normalised residual rows x^ (window-major, all tokens)
  bf16* xh = nullptr;
  // BF16 path scratch (u16: normalised rows after the projection, compact)
  bf16 *u16 = nullptr, *q16 = nullptr, *k16 = nullptr, *o16 = nullptr,
       *h16 = nullptr;
  bf16* vt16 = nullptr;  // V^T [win][head][dh][vt stride] (BF16 clip mode)
  float* amax = nullptr;  // FP8 activation amax slots [blocks][4]
  float* contrib = nullptr;  // overlapping decoder: per-token logit patches [N][192]
  // stream mode: contiguous staging of the batch's frames, masks and outputs
  float* fst = nullptr;
  uint8_t* mst = nullptr;
  float* ost = nullptr;
  bool stream_mode = false;
  std::vector<void*> allocs;
};

// Stream mode: one ring of win_t K/V slots per stream; slot j, block l starts at element
// (j * blocks + l) * blk_elems, each block holding [win_f][head][S_f][dh] bf16.
constexpr int STREAM_MAXB = 16;
struct StreamTable {
  bf16* k[STREAM_MAXB];     // cache base of request r, advanced to the current block (slot 0)
  bf16* v[STREAM_MAXB];
  int head[STREAM_MAXB];    // slot receiving the new frame
  int npast[STREAM_MAXB];   // cached past frames (<= ring - 1)
  int T[STREAM_MAXB];       // frames in the request's ring (memory slots + 1)
  long long slot_stride;    // elements between slots of K
  long long vslot_stride;   // elements between slots of V^T
  int sfp;                  // key slots per frame in V^T rows ([win_f][head][dh][sfp] per slot)
};

// Entry r of a per-request table held in kernel arguments, read through selects: a runtime
// index into the argument struct would copy the whole table to scratch memory.
template <class T>
__device__ __forceinline__ T pick(const T (&a)[STREAM_MAXB], int r) {
  T v = a[0];
  static_for<STREAM_MAXB>([&](auto i) {
    if (i == r) v = a[i];
  });
  return v;
}

struct FramePtrs {          // per-request device buffers of a stream-mode batch
  const float* f[STREAM_MAXB];
  const uint8_t* m[STREAM_MAXB];
  float* o[STREAM_MAXB];
  int n;
};

}  // namespace dr

namespace dr {
struct StreamSt {
  int H = 0, W = 0;
  int slots = 0;        // past frames kept (memory slots); the ring holds slots + 1 frames
  bf16* kc = nullptr;
  bf16* vc = nullptr;
  int head = 0, npast = 0;
  size_t bytes = 0;
};
}  // namespace dr

struct dr_wplan;  // per-shape weight derivation plan (dr_weights.hip)

struct dr_ctx {
  int device = 0;
  int32_t* scratch_wcount = nullptr;  // this device's static gather scratch (device address)
  dr::Net net;
  bool have_weights = false;
  // weights: the flat FP32 parameters (blob order) and the arenas derived from them on the
  // device, with the plan's index maps (all in weight_allocs)
  std::vector<void*> weight_allocs;
  dr_wplan* wplan = nullptr;
  float* params = nullptr;
  float* wf32 = nullptr;
  size_t wf32_elems = 0;
  dr::bf16* wb16 = nullptr;
  uint8_t* w8 = nullptr;
  float* wscale8 = nullptr;
  int32_t *wmaps32 = nullptr, *wmaps16a = nullptr, *wmaps16b = nullptr;
  void* wfolds = nullptr;
  const float** wjob_ptrs = nullptr;
  size_t* wjob_counts = nullptr;
  dr::Work work;
  std::string err;
  // profiling
  bool prof = false;
  int debug_blocks = -1;  // inspection: run only this many blocks (-1 = all)
  int attn_pattern = 0;   // 0 joint window attention; 1 decoupled (even blocks spatial, odd temporal)
  int train_bf16 = 0;     // training products with bf16 operands (FP32 accumulation, master weights)
  struct Rec { int stage; hipEvent_t a, b; };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> event_pool;
  // stream mode
  std::mutex smu;                                   // guards streams, budget, swork
  std::map<int, dr::StreamSt> streams;
  int next_sid = 1;
  size_t budget = 0;                                // 0 = no limit
  size_t used = 0;                                  // bytes of open streams' caches
  std::map<std::pair<int, int>, dr::Work*> swork;   // stream-mode workspaces by (H, W)
  void* train = nullptr;                            // training workspace (activations, scratch)
  // HIP graphs of the per-block launch sequence, per shape and precision
  bool use_graphs = true;
  int graph_epoch = 0;                              // bumped when weights or workspace move
  std::map<std::string, hipGraphExec_t> graphs;
  std::set<std::string> graph_seen;
  hipStream_t cap_stream = nullptr;
};

namespace dr {

// ------------------------------------------------------------------------------------------
// Kernel launchers (one translation unit each; all enqueue on `s`, no synchronisation)
// ------------------------------------------------------------------------------------------
struct Geo {
  int B, T, H, W;      // pixel shape
  int Ht, Wt;          // token grid per frame
  int nwh, nww;        // windows per frame (rows, cols)
  int wt, wh, ww;      // window extent in tokens
  int S, N, nwin;      // tokens per window, total tokens, total windows
  int P;               // patch
};

// step 1 -- token flags and gather lists
// halo 1: a token is flagged when its 8 x 8 footprint (overlapping embedding) holds a
// private pixel
void launch_token_flags(const Geo& g, const uint8_t* masks, int all, uint8_t* flag,
                        int32_t* wcount, hipStream_t s, int halo = 0);
void launch_token_gather(const Geo& g, const uint8_t* flag, const int32_t* wcount,
                         int32_t* idx, int32_t* woff, int32_t* nq, hipStream_t s);
// step 2 -- cut-out + patch embedding, x [N, C] f32 window-major
void launch_embed(const Geo& g, int C, const float* frames, const uint8_t* masks,
                  const float* wT, const float* b, float* x, hipStream_t s);
// final step -- LN_f + decoder + sigmoid, masked pixels of flagged tokens written to out
void launch_decode(const Geo& g, int C, const float* x, const int32_t* idx, const int32_t* nq,
                   const float* lng, const float* lnb, const float* dw, const float* db,
                   const uint8_t* masks, float* out, hipStream_t s);
// unmasked pixels copied from frames to out (skipped when in place)
void launch_copy_unmasked(size_t npix, const float* frames, const uint8_t* masks, float* out,
                          hipStream_t s);

// FP32 path
void launch_ln_f32(const float* x, const int32_t* rows, const int32_t* nrows_dev, int nrows_max,
                   int C, const float* g, const float* b, float* y, hipStream_t s);
enum EpiKind { EPI_STORE = 0, EPI_GELU = 1, EPI_RESID = 2 };
// Y = A[rows] W^T + bias, A f32 [*, K] (row stride K), W f32 [Nout, K].
//   EPI_STORE: Y[r, :] stored to out (row stride Nout)
//   EPI_GELU : GELU(Y) stored to out
//   EPI_RESID: x[res_rows[r], :] += Y[r, :]  (out = x, row stride Nout)
void launch_gemm_f32(const float* A, const int32_t* arows, const int32_t* m_dev, int m_max,
                     int K, const float* W, const float* bias, int Nout, int epi, float* out,
                     const int32_t* res_rows, hipStream_t s);
void launch_attn_f32(const Geo& g, int C, int heads, const float* q, const float* kv,
                     const int32_t* woff, float* o, hipStream_t s);

// FP8 path (OCP e4m3 operands, per-tensor scales s = amax/448, FP32 accumulation)
bool fp8_supported(int C, int R);
void launch_quantize_fp8(const float* in, uint8_t* out, size_t n, float inv_scale, hipStream_t s);
// as launch_quantize_fp8 with the scale read from device memory (values / *scale)
void launch_quantize_fp8_dev(const float* in, uint8_t* out, size_t n, const float* scale, hipStream_t s);
void launch_zero_f32(float* p, int n, hipStream_t s);
// LayerNorm of rows (affine) into bf16 rows plus the call's amax: rows given -> compact output
// rows r < *nrows_dev from x[rows[r]]; else rows r < nrows_max of windows with queries.
void launch_ln_rows_amax(const float* x, const int32_t* rows, const int32_t* nrows_dev, int nrows_max,
                         const int32_t* wcount, int S, int C, const float* g, const float* b, bf16* out,
                         float* slot, hipStream_t s);
// Q/K/V from the LayerNorm rows u [N][C]: q [N][C] (times qscale), k [win][head][Spad][dh],
// vt [win][head][dh][spv]; row tiles from the lists of launch_window_order
void launch_qkv_fp8(const Geo& g, int C, int heads, int Spad, int spv, const bf16* u, const int32_t* tiles,
                    const int32_t* ntiles, const uint8_t* w, const float* wscale, const float* bias,
                    const float* amax_u, float qscale, bf16* q, bf16* k, bf16* vt, hipStream_t s);
// first MLP linear + GELU over compact rows u [*m_dev][C] -> h [.][R], amax of h
void launch_fc1_fp8(int m_max, const int32_t* m_dev, int C, int R, const bf16* u, const uint8_t* w, const float* s_w,
                    const float* bias, const float* amax_u, bf16* h, float* amax_h, hipStream_t s);
void launch_gemm_fp8_resid(const bf16* A, const int32_t* m_dev, int m_max, int K,
                           const uint8_t* W, const float* s_w, const float* amax_a, const float* bias,
                           int Nout, float* x, const int32_t* res_rows, hipStream_t s);

// BF16 path after the token flags, in one launch: the window order and Q/K/V row tiles, each
// window's query list, and the embedding: x (f32) of flagged tokens, x^ (bf16) of tokens in
// windows with queries (emb_wcount null: all)
void launch_tokens_embed_bf16(const Geo& g, int C, const float* frames, const uint8_t* masks, const uint8_t* flag,
                              const int32_t* wcount, const int32_t* emb_wcount, const bf16* wT16, const float* b,
                              float* x, bf16* xh, int32_t* idx, int32_t* woff, int32_t* nq, int32_t* order,
                              int32_t* tiles, int32_t* ntiles, hipStream_t s);
// decoder from x^ (Wd' [48][C] with the final LayerNorm's affine part folded in) writing the
// masked pixels of the flagged tokens, and out = frames at every unmasked pixel of the npix
// pixels (no copy when out == frames), in one launch
void launch_decode_copy_bf16(const Geo& g, int C, const bf16* xh, const int32_t* idx, const int32_t* nq,
                             const bf16* wd16, const float* bd, const uint8_t* masks, const float* frames,
                             float* out, size_t npix, hipStream_t s);
// overlapping variant (kernel 8, stride 4, padding 2): the embedding with wT16 [C][192] in
// the slot order of embed_ovl_bf16_kernel; the decoder as per-token logit patches
// contrib [N][192] of the flagged tokens (k = (ky*8 + kx)*3 + ch, wd16 [192][C] with the final
// LayerNorm folded in) and a per-pixel sum over the covering tokens + bias + sigmoid
void launch_embed_ovl_bf16(const Geo& g, int C, const float* frames, const uint8_t* masks, const uint8_t* flag,
                           const int32_t* wcount, const bf16* wT16, const float* b, float* x, bf16* xh,
                           hipStream_t s);
void launch_decode_ovl_bf16(const Geo& g, int C, const bf16* xh, const int32_t* idx, const int32_t* nq,
                            const bf16* wd16, const float* bd, float* contrib, hipStream_t s);
void launch_fold_ovl(const Geo& g, const float* contrib, const float* db, const uint8_t* masks, float* out,
                     hipStream_t s);
// clip mode: the row tiles listed by launch_window_order (Q tiles with a flagged token, K/V
// tiles touching a window with queries)
void launch_qkv_bf16(const Geo& g, int C, int heads, int Spad, int spv, const bf16* xh, const int32_t* tiles,
                     const int32_t* ntiles, const bf16* w, const float* bias, bf16* q, bf16* k, bf16* vt,
                     hipStream_t s);
int attn_clip_vt_stride(int spad);
// amax_o (nullable): max |O| of the call is max-reduced into *amax_o (FP8 path).  mode: 0 joint
// window attention, 1 spatial (keys of the query's frame), 2 temporal (keys at the query's
// position in every frame) -- the blocks of a decoupled network.
void launch_attn_clip(const Geo& g, int C, int heads, int Spad, const bf16* q, const bf16* k, const bf16* vt,
                      const int32_t* idx, const int32_t* woff, const int32_t* worder, bf16* o, float* amax_o,
                      int mode, hipStream_t s);
bool window_order_supported(int S);
// Rows of the Q/K/V GEMM tiles listed by the token step (the GEMM's row tile height).
constexpr int ROW_TILE = 64;
// windows by decreasing query count, plus the two row-tile lists (tiles [2][ceil(N/ROW_TILE)],
// counts ntiles[2])
void launch_window_order(const Geo& g, const int32_t* wcount, const uint8_t* flag, int32_t* order, int32_t* tiles,
                         int32_t* ntiles, hipStream_t s);
void launch_qkv_stream(const Geo& g, int C, int heads, const bf16* xh, const uint8_t* flag, const bf16* w,
                       const float* bias, bf16* q, const StreamTable& tab, hipStream_t s);
void launch_fc1_bf16(int m_max, const int32_t* m_dev, int C, int R, const bf16* u2, const bf16* w,
                     const float* bias, bf16* h, hipStream_t s);
bool resid_ln_supported(int C);
bool mlp_block_supported(int C, int R);
void launch_mlp_block_bf16(int m_max, const int32_t* m_dev, int C, const bf16* o, const int32_t* rows,
                           const bf16* wo, const float* bo, const bf16* w1, const float* b1, const bf16* w2,
                           const float* b2, float* x, bf16* xh, hipStream_t s);
void launch_resid_ln_bf16(int m_max, const int32_t* m_dev, int C, int K, const bf16* A, const bf16* w,
                          const float* bias, float* x, const int32_t* rows, bf16* xh, const int32_t* hrows,
                          hipStream_t s);

// stream mode
void launch_gather_frames(const FramePtrs& p, size_t npix, float* fst, uint8_t* mst, hipStream_t s);
void launch_scatter_frames(const FramePtrs& p, size_t npix, const float* ost, hipStream_t s);
int ring_vt_frame_stride(int sf);
bool attn_ring_supported(int dh, int sf, int nf);
void launch_attn_ring(const StreamTable& tab, const Geo& g, int C, int heads, int nf, const bf16* q, const int32_t* idx,
                      const int32_t* woff, const int32_t* worder, bf16* o, hipStream_t s);
bool attn_ring_temporal_supported(int dh);
void launch_attn_ring_temporal(const StreamTable& tab, const Geo& g, int C, int heads, const bf16* q,
                               const int32_t* idx, const int32_t* woff, const int32_t* worder, bf16* o,
                               hipStream_t s);

// host helpers shared by the API translation units
dr_status dr_fail(dr_ctx* c, dr_status st, const char* fmt, ...);
dr_status dr_make_geo(dr_ctx* c, int B, int T, int H, int W, int wt, Geo& g);
dr_status dr_reserve_work(dr_ctx* c, Work& w, const Geo& g, bool stream_mode);
void dr_free_work(Work& w);
void dr_train_release(dr_ctx* c);
void dr_invalidate_graphs(dr_ctx* c);
// weights (dr_weights.hip)
void dr_weights_release(dr_ctx* c);
void dr_wplan_free(dr_wplan* p);
size_t dr_nparams(const Net& n, int K);
void dr_prof_begin(dr_ctx* c, hipStream_t s, hipEvent_t* a, hipEvent_t* b);
void dr_prof_end(dr_ctx* c, int stage, hipStream_t s, hipEvent_t a, hipEvent_t b);
extern const char* const kStageNames[];

}  // namespace dr
