/*
 * drinpaint -- C ABI of the MI355X (gfx950) inpainting library.
 *
 * The library runs the forward pass of a windowed-attention transformer inpainting network
 * on one GPU: it fills the private (masked) regions of each video frame with generated
 * background and leaves every other pixel untouched.  The operation follows the thesis's
 * problem statement for its inpainting stage (Methods, "Inpainting Manager"): the network
 * receives a frame whose masked regions are set to 0 and returns the completed frame; the
 * masked regions are the private objects cut out of the frame (Methods, "Object Control").
 *
 * Network (per clip of T frames, patch p, dim C, h heads, L blocks, MLP ratio r):
 *   1. cut-out xc = frame with masked pixels set to 0; token flag = OR of the mask over the
 *      token's p x p pixels;
 *   2. patch embedding: Conv2d(3 -> C, kernel p, stride p);
 *   3. L pre-LN blocks: multi-head self-attention inside non-overlapping windows of
 *      win_t x win_h x win_w tokens (scaled dot product, as in the thesis's
 *      "Performance Optimisations -- Inpainting Model"), then an exact-erf GELU MLP; only
 *      flagged tokens are queries and are updated, keys/values are all window tokens;
 *   4. final LayerNorm, ConvTranspose2d(C -> 3, kernel p, stride p), sigmoid;
 *   5. composite: out = prediction where the mask is nonzero, else the input pixel, bit for
 *      bit.
 *
 * Conventions shared by every call
 *   - Every call returns a dr_status; nothing aborts or throws across the ABI.  After a
 *     non-DR_OK status, dr_last_error(ctx) holds a message (per context, valid until the
 *     next call on that context).
 *   - Device pointers are plain HIP device addresses on the context's device, owned by the
 *     caller.  Host pointers are marked "host".
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).  Work is
 *     enqueued asynchronously on it; the caller synchronises.  Kernel faults surface as
 *     DR_EHIP at a later call or at the caller's synchronisation.
 *   - A context is not thread-safe: calls that overlap on one context race.
 */
#ifndef DRINPAINT_H
#define DRINPAINT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DR_OK = 0,
  DR_EINVAL = 1, /* bad argument: null pointer, bad enum, partial aliasing, no weights   */
  DR_ESHAPE = 2, /* shape does not tile into whole windows / unsupported network shape   */
  DR_ENOMEM = 3, /* device allocation failed or a footprint budget would be exceeded      */
  DR_EHIP = 4,   /* a HIP runtime call or kernel launch failed                             */
  DR_EBUSY = 5   /* resource in use (e.g. stream id still has work in flight)              */
} dr_status;

/* Arithmetic of the attention/MLP GEMMs.  DR_FP32: plain FP32 kernels, one per operation.
 * DR_BF16: BF16 operands on MFMA with FP32 accumulation.  DR_FP8: the Q/K/V, projection and
 * MLP GEMMs take OCP e4m3 operands with per-tensor scales (amax/448; weights fixed at load,
 * activations from the current call) and FP32 accumulation, attention stays BF16; needs dim
 * and hidden width multiples of 128.  LayerNorm statistics, softmax max/sum and the residual
 * stream stay FP32 in every mode.  The patch embedding and the decoder run in FP32 in DR_FP32
 * and DR_FP8, and take bf16 operands on MFMA (FP32 accumulation) in DR_BF16. */
typedef enum { DR_FP32 = 0, DR_BF16 = 1, DR_FP8 = 2 } dr_precision;

/* Which tokens are attention queries and get updated.  DR_QUERY_MASKED: tokens whose patch
 * holds a masked pixel.  DR_QUERY_ALL: every token (dense). */
typedef enum { DR_QUERY_MASKED = 0, DR_QUERY_ALL = 1 } dr_query_set;

typedef struct {
  int32_t dim;       /* C, multiple of 64, <= 1024                                        */
  int32_t heads;     /* h, dim / heads in {32, 64}                                        */
  int32_t blocks;    /* L >= 1                                                            */
  int32_t mlp_ratio; /* r >= 1                                                            */
  int32_t patch;     /* p; only 4 is supported                                            */
  int32_t win_h;     /* window height in tokens                                           */
  int32_t win_w;     /* window width in tokens                                            */
  int32_t win_t;     /* window length in frames; clips must have T == win_t               */
} dr_netcfg;

typedef struct dr_ctx dr_ctx;

/* Create a context on HIP device `device` for network `cfg` (host pointer, copied).
 * Checks the network shape (DR_ESHAPE if unsupported).  The context owns every buffer it
 * allocates; release it with dr_destroy. */
dr_status dr_create(dr_ctx** out, int device, const dr_netcfg* cfg);

/* Load FP32 master weights from a host blob of `nbytes` bytes (not retained).  Blob layout
 * (little endian): char magic[4] = "DRW1"; uint32 version = 1; dr_netcfg cfg; uint32 count;
 * then `count` records {char name[48]; uint32 dtype (0 = f32); uint32 ndim; uint32 shape[4];
 * uint64 offset; uint64 nbytes;}; data offsets are relative to the end of the table.  The
 * tensors must be exactly the network's parameters, in order: embed.w [C,3,p,p] (OIHW),
 * embed.b [C]; per block l: blk{l}.ln1.g, .ln1.b, .wq, .bq, .wk, .bk, .wv, .bv, .wo, .bo,
 * .ln2.g, .ln2.b, .w1 [rC,C], .b1, .w2 [C,rC], .b2 (linear weights [out,in]); lnf.g, lnf.b,
 * dec.w [C,3,p,p] (IOHW), dec.b [3].  Derived BF16 copies are built on the device.
 * Kernels of size 2p in embed.w and dec.w ([C,3,2p,2p], p = 4) select the overlapping
 * variant, after the thesis's Vec2Patch change (Methods, "Performance Optimisations --
 * Modified Vec2Patch"): a Conv2d(3, C, 2p, stride p, padding p/2) embedding, and a decoder
 * whose overlapping 2p x 2p patches are summed (the fold), computed as a per-pixel reduction
 * over the covering tokens with the padding cropped.  Its queries are the tokens whose
 * 2p x 2p footprint holds a private pixel.  It runs in clip mode on the BF16 path
 * (dr_inpaint with another precision, stream mode and training return DR_EINVAL).
 * DR_EINVAL on a malformed blob or a config mismatch. */
dr_status dr_load_weights(dr_ctx* ctx, const void* blob, size_t nbytes);

/* Pre-allocate the workspace for clips of B x T x H x W so later dr_inpaint calls of that
 * size (or smaller) allocate nothing.  dr_inpaint grows the workspace itself if needed. */
dr_status dr_reserve(dr_ctx* ctx, int B, int T, int H, int W, dr_precision prec);

/* Inpaint B clips of T frames.
 *   frames: device f32 [B,T,H,W,3] (NHWC, values nominally in [0,1]), 16-byte aligned.
 *   masks:  device u8  [B,T,H,W], nonzero = private pixel to be filled, 4-byte aligned.
 *   out:    device f32 [B,T,H,W,3].  out == frames (in place) is allowed; any other overlap
 *           of out with frames or masks is DR_EINVAL.
 * Pixels whose mask is 0 are copied from `frames` bit for bit.  DR_EINVAL for misaligned
 * frames or masks.  DR_ESHAPE unless
 * T == win_t, H % (p*win_h) == 0 and W % (p*win_w) == 0.  DR_EINVAL without weights. */
dr_status dr_inpaint(dr_ctx* ctx, const float* frames, const uint8_t* masks, float* out,
                     int B, int T, int H, int W, dr_precision prec, dr_query_set qs,
                     void* stream);

/* Token gather of step 1 alone, for inspection and tests.  Token order is window-major:
 * windows in (clip, frame-block, window-row, window-col) order, tokens inside a window in
 * (frame, row, col) order.  Outputs (device): flag u8 [N] (N = B*T*H*W/p^2), idx int32 [N]
 * whose first Nq entries list the flagged tokens in ascending order, woff int32 [nwin+1]
 * (window w's queries are idx[woff[w] .. woff[w+1])), nq int32 [1] = Nq. */
dr_status dr_gather_tokens(dr_ctx* ctx, const uint8_t* masks, int B, int T, int H, int W,
                           dr_query_set qs, uint8_t* flag, int32_t* idx, int32_t* woff,
                           int32_t* nq, void* stream);

/* dr_gather_tokens for callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: same arguments, outputs and
 * errors, but it allocates nothing (no workspace is reserved).  Its only scratch, the
 * per-window query counts, is a static device array of 65,536 entries (256 KB) that every
 * device the library runs on holds until the process ends; more windows than that
 * (B*T*H*W / (p^2 * window tokens)) give DR_EINVAL.  The array is shared by every call on a
 * device, so calls that overlap in time on one device (any context, any stream) race. */
dr_status dr_gather_tokens_noalloc(dr_ctx* ctx, const uint8_t* masks, int B, int T, int H, int W,
                                   dr_query_set qs, uint8_t* flag, int32_t* idx, int32_t* woff,
                                   int32_t* nq, void* stream);

/* Per-kernel timing.  dr_profile(ctx, 1) makes every later launch record a HIP event pair
 * on its stream; dr_profile_read synchronises on those events, writes the summed time in
 * milliseconds and the launch count per stage into ms[] / count[] (host arrays of
 * `nstage` entries, stage ids as listed by dr_stage_name), and clears the record.
 * dr_profile(ctx, 0) stops recording. */
dr_status dr_profile(dr_ctx* ctx, int enable);
dr_status dr_profile_read(dr_ctx* ctx, double* ms, int64_t* count, int nstage);
/* Name of stage id `stage` (static string), or NULL past the last stage. */
const char* dr_stage_name(int stage);

/* Inspection, for tests: copy the first `nbytes` of the named workspace buffer into device
 * memory `dst` on `stream`.  Names: "x" (f32 residual [N,C], window-major; BF16 path: rows
 * of flagged tokens), "xh", "u16", "q16", "o16" (bf16 [N,C]), "k16" (bf16
 * [win][head][Spad][dh]), "vt16" (bf16 [win][head][dh][spv]), "h16" (bf16 [N,rC]), "u", "q",
 * "o" (f32 [N,C]), "kv" (f32 [N,2C]), "h" (f32 [N,rC]), "flag" (u8 [N]), "idx" (int32 [N]),
 * "nq" (int32), "wcount" (int32 [win]), "worder" (int32 [win]: windows by decreasing query
 * count), "tiles" (int32 [2][ceil(N/64)]: row tiles of 64 tokens with a flagged token, then
 * row tiles touching a window with queries, each list in any order), "ntiles" (int32 [2]).
 * DR_EINVAL for an unknown name or a size beyond the buffer. */
dr_status dr_inspect(dr_ctx* ctx, const char* name, void* dst, size_t nbytes, void* stream);

/* Inspection, for tests: key "blocks" = number of transformer blocks later dr_inpaint calls
 * run (-1 = all; the output then is not the network's); key "graphs" = 0 launches every
 * kernel directly instead of replaying the per-block sequence as a HIP graph (default 1:
 * the first call of a shape runs directly, the second captures, later ones replay). */
dr_status dr_debug_set(dr_ctx* ctx, const char* key, int64_t value);

/* Test hook of the FP8 path's quantiser: out[i] = e4m3(in[i] / scale) (OCP e4m3, round to
 * nearest even, clamped to +-448), device pointers, n elements. */
dr_status dr_fp8_encode(dr_ctx* ctx, const float* in, uint8_t* out, size_t n, float scale,
                        void* stream);

/* ---- Stream mode (one new frame per call, per-stream memory of past frames) -------------
 * Each stream keeps, per transformer block, the keys/values of its last win_t - 1 frames on
 * the device (the thesis's memory tensors kept from previous outputs, Methods, "Inpainting
 * Manager"); a new frame's flagged tokens attend to their spatial window (win_h x win_w
 * tokens) in those frames and in the new frame, then the new frame's K/V replace the oldest.
 * The first frames of a stream use the frames available (a decoupled network's blocks attend
 * as dr_set_attention_pattern states).  BF16 only. */

/* Footprint budget in bytes for all open streams' caches (0 = unlimited, the default). */
dr_status dr_set_budget(dr_ctx* ctx, size_t bytes);
/* Device bytes a stream of H x W frames holds while open. */
size_t dr_stream_footprint(dr_ctx* ctx, int H, int W);
/* Open a stream of H x W frames (H, W multiples of the window's pixel size); *sid receives
 * its id.  DR_ENOMEM if its footprint does not fit the budget (admit it later). */
dr_status dr_stream_open(dr_ctx* ctx, int H, int W, int32_t* sid);
/* As dr_stream_open with `slots` past frames kept (the thesis's memory slots, 0..win_t-1;
 * dr_stream_open keeps win_t - 1).  Footprint scales with slots + 1. */
dr_status dr_stream_open_slots(dr_ctx* ctx, int H, int W, int slots, int32_t* sid);
/* Close a stream (waits for the device) and release its memory. */
dr_status dr_stream_close(dr_ctx* ctx, int32_t sid);
/* Inpaint the newest frame of n (1..16) distinct streams of one resolution in one batch.
 * sids: host array; frames, masks, outs: host arrays of device pointers to f32 [H,W,3],
 * u8 [H,W], f32 [H,W,3] (out must not overlap frame or mask).  Asynchronous on `stream`;
 * prec must be DR_BF16.  A stream must not appear in two overlapping calls. */
dr_status dr_stream_step(dr_ctx* ctx, int n, const int32_t* sids, const float* const* frames,
                         const uint8_t* const* masks, float* const* outs, dr_precision prec,
                         dr_query_set qs, void* stream);

/* Attention pattern of the network (a context setting; the weights are the same):
 * 0 (default) every block attends over its whole window; 1 decoupled, in the manner of the
 * DSTT network the thesis builds on (Background, "Decoupled Spatial-Temporal Transformer"):
 * even blocks attend within one frame of the window, odd blocks across the window's frames
 * at one token position.  Pattern 1 runs on the BF16 and FP8 paths of dr_inpaint (FP32 and
 * training return DR_EINVAL) with at most 8 frames per window, and in stream mode, where an
 * even block attends within the new frame's window only and an odd block to its token
 * position in the cached frames and the new one.  Waits for the device when the pattern
 * changes. */
dr_status dr_set_attention_pattern(dr_ctx* ctx, int pattern);

/* ---- Camera-resolution pre/post-processing ----------------------------------------------
 * The thesis runs its models at half the camera resolution and scales their outputs by 2
 * (Methods, "Performance Optimisations -- Upscaling"); the server cuts the masks of the
 * objects the user selected out of the camera frame (Methods, "Object Control").  These two
 * calls put the steps around the network on the GPU.  Asynchronous on `stream`. */

/* Camera frame -> network input at half resolution.
 *   bgra:      device u8 [H,W,4] (B, G, R, alpha), 8-byte aligned.
 *   inst:      device u8 [K,H,W] per-object instance masks (nonzero = object), K in 0..32
 *              (may be NULL when K == 0); bit k of `select` selects instance k.
 *   radius:    dilation of the union by a square (2r+1)^2 window, 0..16; pixels outside the
 *              frame do not contribute.
 * Outputs (device, caller-owned): mask_full u8 [H,W] (1 = private: the selected union,
 * dilated), mask_low u8 [H/2,W/2] (1 where any pixel of the 2x2 block is private),
 * frame_low f32 [H/2,W/2,3] (RGB mean of the 2x2 block / 255).  DR_ESHAPE unless H and W are
 * even; DR_EINVAL for null pointers, K or radius out of range, a misaligned bgra. */
dr_status dr_prep_frame(dr_ctx* ctx, const uint8_t* bgra, const uint8_t* inst, int K, uint32_t select,
                        int radius, int H, int W, float* frame_low, uint8_t* mask_low, uint8_t* mask_full,
                        void* stream);
/* Half-resolution prediction -> camera frame: out[y][x] = mask_full[y][x] ? B, G, R of
 * pred_low[y/2][x/2] (nearest 2x upscale) as clamp(rint(255 v), 0, 255) with alpha kept :
 * bgra[y][x] unchanged.  bgra, out: device u8 [H,W,4], 16-byte aligned (out == bgra allowed,
 * other overlaps DR_EINVAL); pred_low f32 [H/2,W/2,3]; mask_full u8 [H,W], 4-byte aligned.
 * DR_ESHAPE unless H is even and W % 4 == 0. */
dr_status dr_post_frame(dr_ctx* ctx, const uint8_t* bgra, const float* pred_low, const uint8_t* mask_full,
                        int H, int W, uint8_t* out, void* stream);

/* ---- Serving loop ---------------------------------------------------------------------
 * A persistent native thread that batches submitted requests continuously: per resolution
 * class it launches the oldest pending requests (at most one per stream, up to max_batch)
 * whenever that class's executor (own workspace and HIP stream) is idle, so classes overlap
 * on the device and new requests join as soon as their class frees up.  Latency of a request
 * = completion (event observed by the loop) - entry into dr_server_submit. */
typedef struct dr_server dr_server;
/* Start a server on `ctx` batching up to max_batch (1..16) requests.  The executors (HIP
 * stream, event, workspace for max_batch frames) of the resolutions of the streams open at
 * this call are created here, so serving them allocates nothing; a resolution first seen
 * later gets its executor when its first request is launched (its requests fail with
 * DR_ENOMEM if that allocation fails).  DR_ENOMEM if an executor cannot be created. */
dr_status dr_server_create(dr_ctx* ctx, int max_batch, dr_server** out);
/* Queue one frame of an open stream; device buffers must stay valid until it completes. */
dr_status dr_server_submit(dr_server* srv, int32_t sid, const float* frame,
                           const uint8_t* mask, float* out, uint64_t* ticket);
/* Move up to `max` completed requests into host arrays (status may be NULL; a nonzero status
 * is the dr_status of a failed batch -- DR_EHIP when its completion event reports a device
 * error -- with latency -1).  *n_done receives the count. */
dr_status dr_server_poll(dr_server* srv, uint64_t* tickets, double* latency_ms,
                         int32_t* status, int max, int* n_done);
/* Batches launched, requests launched, requests still pending (any pointer may be NULL). */
dr_status dr_server_stats(dr_server* srv, int64_t* batches, int64_t* requests, int* pending);
/* Finish all queued work, stop the thread and free the executors. */
void dr_server_destroy(dr_server* srv);

/* ---- Training ----------------------------------------------------------------------------
 * Parameters are addressed as one flat f32 vector in the blob order of dr_load_weights
 * (embed.w OIHW, embed.b, per block ln1.g ... b2, lnf.g, lnf.b, dec.w IOHW, dec.b). */
size_t dr_param_count(dr_ctx* ctx);

/* Replace the weights from `params`: device f32 [dr_param_count] in that flat order (the
 * non-overlapping network).  Every layout the kernels read -- transposes, the bf16 copies,
 * the LayerNorm affine parts folded into the following linear, the e4m3 copies and their
 * per-tensor scales -- is derived from it on the device, enqueued on `stream`: nothing goes
 * through host memory, and after the first load of a context nothing is allocated.  The
 * caller keeps `params` valid until that work has run.  Enqueued forwards that read the
 * weights run with the new values if they are ordered after this call on the device.
 * DR_EINVAL for a null pointer or a context whose weights use the overlapping embedding. */
dr_status dr_load_params(dr_ctx* ctx, const float* params, void* stream);

/* Precision of the training passes (the reverse pass of the thesis's L1-trained network,
 * Methods, "Model Training"): DR_FP32 (default) or DR_BF16, mixed precision -- the weight
 * products of the forward (Q/K/V, projection, MLP) and of the reverse pass (input and weight
 * gradients) take operands rounded to bf16 and accumulate in FP32; weights, activations,
 * LayerNorm, attention, the loss and every gradient stay FP32.  Applies from the next
 * dr_train_forward (its handle's dr_train_backward uses the same precision).  DR_EINVAL
 * otherwise. */
dr_status dr_train_set_precision(dr_ctx* ctx, dr_precision prec);

/* Saved activations of one training forward (opaque, owned by the context). */
typedef struct dr_saved dr_saved;

/* Forward of B clips (as dr_inpaint, masked queries) that keeps what the reverse pass needs
 * in a new handle *saved: per block the block input, LN1 output, K/V, Q, attention output
 * and row max/sum, post-projection rows, LN2 output and MLP pre-activation, and a copy of
 * the FP32 weights the forward ran with (so a later dr_load_params does not change this
 * forward's gradient).  pred: device f32 [B,T,H,W,3], the sigmoid output of the decoder at
 * every pixel (before the composite).  Several handles may be live at once; each is released
 * with dr_saved_free.  A handle's buffers are reused by a later forward after it is freed, so
 * free it only once the work reading it is ordered before that forward (same stream, or the
 * caller synchronised).  DR_ENOMEM if its buffers cannot be allocated. */
dr_status dr_train_forward(dr_ctx* ctx, const float* frames, const uint8_t* masks, float* pred,
                           int B, int T, int H, int W, dr_saved** saved, void* stream);

/* Reverse pass of the forward that produced `saved`: dpred = dL/dpred (device, layout of its
 * pred); grads: device f32 [dr_param_count] receives dL/dparams at that forward's weights.
 * Attention probabilities are recomputed from Q, K and the saved row statistics.  Token
 * reductions run in fixed chunks, so the result is deterministic.  The handle stays live
 * (the pass may be repeated).  DR_EINVAL for a handle that is not live on this context. */
dr_status dr_train_backward(dr_ctx* ctx, dr_saved* saved, const float* dpred, float* grads,
                            void* stream);

/* Release a handle of dr_train_forward (its buffers go back to the context for reuse; the
 * context keeps at most two such idle sets and frees the rest).  DR_EINVAL if `saved` is not
 * a live handle of `ctx`.  dr_destroy releases every handle of the context. */
dr_status dr_saved_free(dr_ctx* ctx, dr_saved* saved);

/* Training loss (thesis, Methods, "Model Training -- Loss"): loss[0] = w_in * mean over
 * masked pixel-channel values |pred - gt| + w_out * mean over the others (an empty region adds
 * 0); dpred (may be NULL) receives dL/dpred with sign(0) = 0.  Device pointers; npix pixels. */
dr_status dr_l1_loss(dr_ctx* ctx, const float* pred, const float* gt, const uint8_t* masks,
                     size_t npix, float w_in, float w_out, float* loss, float* dpred,
                     void* stream);

/* Message of the last failed call on `ctx` ("" if none).  ctx may be NULL (then the
 * message of the last failed dr_create). */
const char* dr_last_error(dr_ctx* ctx);

/* Free everything the context owns.  Waits for the context's device to finish its work. */
void dr_destroy(dr_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* DRINPAINT_H */
