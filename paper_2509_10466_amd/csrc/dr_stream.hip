// Stream mode and the serving loop (host side).
//
// Stream mode keeps, per stream and per block, the keys and values of the last win_t - 1
// frames -- the memory tensors of the thesis's inpainting model, kept from previous outputs
// (Methods, "Inpainting Manager") -- in a ring of win_t slots on the device.  One step
// inpaints the newest frame of up to STREAM_MAXB streams of one resolution in a single batch
// of launches: its K/V go straight into each stream's current slot and its queries attend to
// the slots of the past frames plus the current one.
//
// The server is a persistent native thread that batches requests continuously: requests
// queue per resolution class; whenever a class's executor (own workspace, own HIP stream) is
// idle it takes the oldest pending requests of that class, at most one per stream, and
// launches them; completions are detected by polling an event, so classes run concurrently
// on the device and new requests join as soon as their class frees up.  Streams are admitted
// by HBM footprint (dr_stream_open fails with DR_ENOMEM beyond the context budget).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <set>
#include <thread>
#include <vector>

#include "dr_internal.h"

using namespace dr;

#define HIP_OK(ctx, expr)                                                               \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) return dr_fail(ctx, DR_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

#define LAUNCH(stage, call)                                                                               \
  do {                                                                                                    \
    hipEvent_t ea_, eb_;                                                                                  \
    dr_prof_begin(c, s, &ea_, &eb_);                                                                      \
    call;                                                                                                 \
    hipError_t e_ = hipGetLastError();                                                                    \
    if (e_ != hipSuccess)                                                                                 \
      return dr_fail(c, DR_EHIP, "launch of %s failed: %s", kStageNames[stage], hipGetErrorString(e_));   \
    dr_prof_end(c, stage, s, ea_, eb_);                                                                   \
  } while (0)

// Ring bytes per slot and block: K [win_f][head][S_f][dh] and V^T [win_f][head][dh][sfp]
// (sfp = S_f rounded up to whole 16-key tiles), bf16.
static void ring_elems(const dr_ctx* c, int H, int W, size_t& k_elems, size_t& v_elems) {
  const dr_netcfg& k = c->net.cfg;
  const size_t tok = (size_t)(H / c->net.P) * (W / c->net.P);
  const int sf = k.win_h * k.win_w;
  k_elems = tok * c->net.C;
  v_elems = tok / sf * c->net.C * ring_vt_frame_stride(sf);
}

static size_t stream_bytes(const dr_ctx* c, int H, int W, int slots) {
  size_t ke, ve;
  ring_elems(c, H, W, ke, ve);
  return (size_t)(slots + 1) * c->net.cfg.blocks * (ke + ve) * 2;
}

static dr_status check_frame_shape(dr_ctx* c, int H, int W) {
  const dr_netcfg& k = c->net.cfg;
  if (H <= 0 || W <= 0 || H % (k.patch * k.win_h) || W % (k.patch * k.win_w))
    return dr_fail(c, DR_ESHAPE, "frame %dx%d does not tile into %dx%d-pixel windows", H, W, k.patch * k.win_h,
                   k.patch * k.win_w);
  return DR_OK;
}

extern "C" dr_status dr_set_budget(dr_ctx* c, size_t bytes) {
  if (!c) return DR_EINVAL;
  std::lock_guard<std::mutex> lk(c->smu);
  c->budget = bytes;
  return DR_OK;
}

extern "C" size_t dr_stream_footprint(dr_ctx* c, int H, int W) {
  return c ? stream_bytes(c, H, W, c->net.cfg.win_t - 1) : 0;
}

extern "C" dr_status dr_stream_open_slots(dr_ctx* c, int H, int W, int slots, int32_t* sid) {
  if (!c || !sid) return dr_fail(c, DR_EINVAL, "dr_stream_open: null argument");
  if (slots < 0 || slots > c->net.cfg.win_t - 1)
    return dr_fail(c, DR_EINVAL, "memory slots must be in [0, %d]", c->net.cfg.win_t - 1);
  dr_status st = check_frame_shape(c, H, W);
  if (st != DR_OK) return st;
  const size_t bytes = stream_bytes(c, H, W, slots);
  std::lock_guard<std::mutex> lk(c->smu);
  if (c->budget && c->used + bytes > c->budget)
    return dr_fail(c, DR_ENOMEM, "stream of %zu bytes exceeds the budget (%zu of %zu in use)", bytes, c->used,
                   c->budget);
  HIP_OK(c, hipSetDevice(c->device));
  StreamSt s;
  s.H = H;
  s.W = W;
  s.slots = slots;
  s.bytes = bytes;
  size_t ke, ve;
  ring_elems(c, H, W, ke, ve);
  const size_t kbytes = (size_t)(slots + 1) * c->net.cfg.blocks * ke * 2;
  const size_t vbytes = (size_t)(slots + 1) * c->net.cfg.blocks * ve * 2;
  if (hipMalloc(&s.kc, kbytes) != hipSuccess) return dr_fail(c, DR_ENOMEM, "stream cache allocation failed");
  if (hipMalloc(&s.vc, vbytes) != hipSuccess) {
    (void)hipFree(s.kc);
    return dr_fail(c, DR_ENOMEM, "stream cache allocation failed");
  }
  // the padding key slots of V^T are never written and must read as zero
  if (hipMemset(s.vc, 0, vbytes) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
    (void)hipFree(s.kc);
    (void)hipFree(s.vc);
    return dr_fail(c, DR_EHIP, "stream cache initialisation failed");
  }
  const int id = c->next_sid++;
  c->streams[id] = s;
  c->used += bytes;
  *sid = id;
  return DR_OK;
}

extern "C" dr_status dr_stream_open(dr_ctx* c, int H, int W, int32_t* sid) {
  if (!c) return DR_EINVAL;
  return dr_stream_open_slots(c, H, W, c->net.cfg.win_t - 1, sid);
}

extern "C" dr_status dr_stream_close(dr_ctx* c, int32_t sid) {
  if (!c) return DR_EINVAL;
  std::lock_guard<std::mutex> lk(c->smu);
  auto it = c->streams.find(sid);
  if (it == c->streams.end()) return dr_fail(c, DR_EINVAL, "no stream %d", sid);
  HIP_OK(c, hipSetDevice(c->device));
  HIP_OK(c, hipDeviceSynchronize());
  (void)hipFree(it->second.kc);
  (void)hipFree(it->second.vc);
  c->used -= it->second.bytes;
  c->streams.erase(it);
  return DR_OK;
}

// One batched step on workspace `w` and HIP stream `s`.  Caller holds c->smu.
static dr_status stream_step_locked(dr_ctx* c, Work& w, int n, const int32_t* sids, const float* const* frames,
                                    const uint8_t* const* masks, float* const* outs, dr_query_set qs,
                                    hipStream_t s) {
  if (n < 1 || n > STREAM_MAXB) return dr_fail(c, DR_EINVAL, "batch of %d requests (1..%d)", n, STREAM_MAXB);
  if (!c->have_weights) return dr_fail(c, DR_EINVAL, "no weights loaded");
  if (c->net.K != c->net.P) return dr_fail(c, DR_EINVAL, "stream mode runs the non-overlapping embedding");
  const Net& net = c->net;
  const bool decoupled = c->attn_pattern != 0;
  const int sf = net.cfg.win_h * net.cfg.win_w;
  if (decoupled ? !(attn_ring_supported(net.dh, sf, 1) && attn_ring_temporal_supported(net.dh))
                : !attn_ring_supported(net.dh, sf, net.cfg.win_t))
    return dr_fail(c, DR_ESHAPE, "no stream attention kernel for this window");
  if (!resid_ln_supported(net.C) || net.cfg.patch != 4)
    return dr_fail(c, DR_ESHAPE, "stream mode needs dim 64, 128, 256 or 384 and patch 4");
  std::vector<StreamSt*> st(n);
  for (int r = 0; r < n; ++r) {
    auto it = c->streams.find(sids[r]);
    if (it == c->streams.end()) return dr_fail(c, DR_EINVAL, "no stream %d", sids[r]);
    st[r] = &it->second;
    for (int q = 0; q < r; ++q)
      if (sids[q] == sids[r]) return dr_fail(c, DR_EINVAL, "stream %d twice in one batch", sids[r]);
    if (st[r]->H != st[0]->H || st[r]->W != st[0]->W) return dr_fail(c, DR_ESHAPE, "mixed resolutions in one batch");
    if (!frames[r] || !masks[r] || !outs[r]) return dr_fail(c, DR_EINVAL, "null frame pointer");
  }
  const int H = st[0]->H, Wd = st[0]->W;
  Geo g;
  dr_status rc = dr_make_geo(c, n, 1, H, Wd, 1, g);
  if (rc != DR_OK) return rc;
  rc = dr_reserve_work(c, w, g, true);
  if (rc != DR_OK) return rc;
  const size_t npix = (size_t)H * Wd;
  FramePtrs fp{};
  for (int r = 0; r < n; ++r) {
    fp.f[r] = frames[r];
    fp.m[r] = masks[r];
    fp.o[r] = outs[r];
  }
  fp.n = n;
  const int C = net.C, R = net.R, N = g.N, L = net.cfg.blocks;
  size_t blk_elems, vblk_elems;  // K and V^T elements of one frame and block
  ring_elems(c, H, Wd, blk_elems, vblk_elems);
  LAUNCH(ST_COPY, launch_gather_frames(fp, npix, w.fst, w.mst, s));
  LAUNCH(ST_TOKENS, launch_token_flags(g, w.mst, qs == DR_QUERY_ALL, w.flag, w.wcount, s));
  // token lists, window order and the embedding of every token in one launch
  LAUNCH(ST_TOKENS, launch_tokens_embed_bf16(g, C, w.fst, w.mst, w.flag, w.wcount, nullptr, net.embed_wT16, net.embed_b,
                                             w.x, w.xh, w.idx, w.woff, w.nq, w.worder, w.tiles, w.ntiles, s));
  for (int l = 0; l < L; ++l) {
    const BlockW& b = net.blk[l];
    StreamTable tab{};
    for (int r = 0; r < n; ++r) {
      tab.k[r] = st[r]->kc + (size_t)l * blk_elems;
      tab.v[r] = st[r]->vc + (size_t)l * vblk_elems;
      tab.head[r] = st[r]->head;
      tab.npast[r] = st[r]->npast;
      tab.T[r] = st[r]->slots + 1;
    }
    tab.slot_stride = (long long)L * blk_elems;
    tab.vslot_stride = (long long)L * vblk_elems;
    tab.sfp = ring_vt_frame_stride(g.S);
    LAUNCH(ST_QKV, launch_qkv_stream(g, C, net.cfg.heads, w.xh, w.flag, b.wqkvf16, b.bqkvf, w.q16, tab, s));
    if (!decoupled) {
      LAUNCH(ST_ATTN, launch_attn_ring(tab, g, C, net.cfg.heads, net.cfg.win_t, w.q16, w.idx, w.woff, w.worder, w.o16, s));
    } else if (l % 2 == 0) {
      // spatial block: the new frame's window only (its K/V sit in the head slot)
      for (int r = 0; r < n; ++r) tab.npast[r] = 0;
      LAUNCH(ST_ATTN, launch_attn_ring(tab, g, C, net.cfg.heads, 1, w.q16, w.idx, w.woff, w.worder, w.o16, s));
    } else {
      LAUNCH(ST_ATTN, launch_attn_ring_temporal(tab, g, C, net.cfg.heads, w.q16, w.idx, w.woff, w.worder, w.o16, s));
    }
    if (mlp_block_supported(C, R)) {
      LAUNCH(ST_MLP, launch_mlp_block_bf16(N, w.nq, C, w.o16, w.idx, b.wo16, b.bo, b.w1f16, b.b1f, b.w216, b.b2, w.x, w.xh, s));
    } else {
      LAUNCH(ST_PROJ, launch_resid_ln_bf16(N, w.nq, C, C, w.o16, b.wo16, b.bo, w.x, w.idx, w.u16, nullptr, s));
      LAUNCH(ST_FC1, launch_fc1_bf16(N, w.nq, C, R, w.u16, b.w1f16, b.b1f, w.h16, s));
      LAUNCH(ST_FC2, launch_resid_ln_bf16(N, w.nq, C, R, w.h16, b.w216, b.b2, w.x, w.idx, w.xh, w.idx, s));
    }
  }
  LAUNCH(ST_DECODE, launch_decode_copy_bf16(g, C, w.xh, w.idx, w.nq, net.dec_wf16, net.dec_bf, w.mst, w.fst, w.ost,
                                            npix * n, s));
  LAUNCH(ST_COPY, launch_scatter_frames(fp, npix, w.ost, s));
  // the new frame now occupies the head slot
  for (int r = 0; r < n; ++r) {
    st[r]->head = (st[r]->head + 1) % (st[r]->slots + 1);
    st[r]->npast = std::min(st[r]->npast + 1, st[r]->slots);
  }
  return DR_OK;
}

extern "C" dr_status dr_stream_step(dr_ctx* c, int n, const int32_t* sids, const float* const* frames,
                                    const uint8_t* const* masks, float* const* outs, dr_precision prec,
                                    dr_query_set qs, void* stream) {
  if (!c || !sids || !frames || !masks || !outs) return dr_fail(c, DR_EINVAL, "dr_stream_step: null argument");
  if (prec != DR_BF16) return dr_fail(c, DR_EINVAL, "stream mode runs in BF16");
  if (qs != DR_QUERY_MASKED && qs != DR_QUERY_ALL) return dr_fail(c, DR_EINVAL, "bad query set");
  HIP_OK(c, hipSetDevice(c->device));
  std::lock_guard<std::mutex> lk(c->smu);
  auto it0 = c->streams.find(sids[0]);
  if (it0 == c->streams.end()) return dr_fail(c, DR_EINVAL, "no stream %d", sids[0]);
  auto key = std::make_pair(it0->second.H, it0->second.W);
  Work*& w = c->swork[key];
  if (!w) w = new Work();
  return stream_step_locked(c, *w, n, sids, frames, masks, outs, qs, (hipStream_t)stream);
}

// ------------------------------------------------------------------------------------------
// server
// ------------------------------------------------------------------------------------------
namespace {
struct Req {
  uint64_t ticket;
  int32_t sid;
  const float* f;
  const uint8_t* m;
  float* o;
  double t_arrive;
  int H, W;
};

struct Exec {
  int H = 0, W = 0;
  Work work;
  hipStream_t s = nullptr;
  hipEvent_t ev = nullptr;
  std::vector<Req> inflight;
  bool busy = false;
};

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}
}  // namespace

struct dr_server {
  dr_ctx* ctx = nullptr;
  int max_batch = STREAM_MAXB;
  std::thread th;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Req> pending;
  struct Done { uint64_t ticket; double ms; int32_t status; };
  std::vector<Done> done;
  bool stop = false;
  uint64_t next_ticket = 1;
  std::vector<Exec*> execs;
  std::set<int32_t> busy_streams;
  int64_t batches = 0, batched_requests = 0;
};

// An executor for frames of H x W: its own HIP stream, completion event and workspace (sized
// for max_batch frames).  Null on failure, with the reason in *why.
static Exec* new_exec(dr_server* sv, int H, int W, const char** why) {
  dr_ctx* c = sv->ctx;
  Exec* e = new Exec();
  e->H = H;
  e->W = W;
  *why = nullptr;
  if (hipStreamCreateWithFlags(&e->s, hipStreamNonBlocking) != hipSuccess) {
    e->s = nullptr;
    *why = "executor stream creation failed";
  } else if (hipEventCreateWithFlags(&e->ev, hipEventDisableTiming) != hipSuccess) {
    e->ev = nullptr;
    *why = "executor event creation failed";
  } else {
    Geo g;
    std::lock_guard<std::mutex> slk(c->smu);
    if (dr_make_geo(c, sv->max_batch, 1, H, W, 1, g) != DR_OK || dr_reserve_work(c, e->work, g, true) != DR_OK)
      *why = "executor workspace allocation failed";
  }
  if (*why) {
    dr_free_work(e->work);
    if (e->ev) (void)hipEventDestroy(e->ev);
    if (e->s) (void)hipStreamDestroy(e->s);
    delete e;
    return nullptr;
  }
  return e;
}

static Exec* find_exec(dr_server* sv, int H, int W) {
  for (Exec* x : sv->execs)
    if (x->H == H && x->W == W) return x;
  return nullptr;
}

// Server thread.  sv->mu guards the queues and counters; it is released while a batch's
// launches are enqueued, so submissions and polls are never held up by a launch.
static void server_loop(dr_server* sv) {
  dr_ctx* c = sv->ctx;
  (void)hipSetDevice(c->device);
  std::unique_lock<std::mutex> lk(sv->mu);
  while (true) {
    bool progressed = false;
    // completions: a batch whose event reports an error fails its requests with DR_EHIP
    for (Exec* e : sv->execs) {
      if (!e->busy) continue;
      const hipError_t q = hipEventQuery(e->ev);
      if (q == hipErrorNotReady) continue;
      const double t = now_s();
      for (const Req& r : e->inflight) {
        if (q == hipSuccess)
          sv->done.push_back({r.ticket, (t - r.t_arrive) * 1e3, DR_OK});
        else
          sv->done.push_back({r.ticket, -1.0, DR_EHIP});
        sv->busy_streams.erase(r.sid);
      }
      e->inflight.clear();
      e->busy = false;
      progressed = true;
    }
    // an executor for every resolution class with pending requests (the classes of the
    // streams open at dr_server_create already have one)
    for (auto it = sv->pending.begin(); it != sv->pending.end();) {
      if (find_exec(sv, it->H, it->W)) {
        ++it;
        continue;
      }
      const char* why = nullptr;
      Exec* e = new_exec(sv, it->H, it->W, &why);
      if (e) {
        sv->execs.push_back(e);
        ++it;
        continue;
      }
      const int H = it->H, W = it->W;
      for (auto jt = sv->pending.begin(); jt != sv->pending.end();) {
        if (jt->H == H && jt->W == W) {
          sv->done.push_back({jt->ticket, -1.0, DR_ENOMEM});
          jt = sv->pending.erase(jt);
        } else {
          ++jt;
        }
      }
      it = sv->pending.begin();
      progressed = true;
    }
    // launches: per idle executor, the oldest pending requests of its class, one per stream
    for (Exec* e : sv->execs) {
      if (e->busy) continue;
      std::vector<Req> batch;
      std::set<int32_t> taken;
      for (auto it = sv->pending.begin(); it != sv->pending.end() && (int)batch.size() < sv->max_batch;) {
        if (it->H == e->H && it->W == e->W && !sv->busy_streams.count(it->sid) && !taken.count(it->sid)) {
          taken.insert(it->sid);
          batch.push_back(*it);
          it = sv->pending.erase(it);
        } else {
          ++it;
        }
      }
      if (batch.empty()) continue;
      for (const Req& r : batch) sv->busy_streams.insert(r.sid);
      e->busy = true;
      const int n = (int)batch.size();
      std::vector<int32_t> sids(n);
      std::vector<const float*> fr(n);
      std::vector<const uint8_t*> ms(n);
      std::vector<float*> os(n);
      for (int r = 0; r < n; ++r) {
        sids[r] = batch[r].sid;
        fr[r] = batch[r].f;
        ms[r] = batch[r].m;
        os[r] = batch[r].o;
      }
      lk.unlock();
      dr_status st;
      {
        std::lock_guard<std::mutex> slk(c->smu);
        st = stream_step_locked(c, e->work, n, sids.data(), fr.data(), ms.data(), os.data(), DR_QUERY_MASKED, e->s);
      }
      if (st == DR_OK && hipEventRecord(e->ev, e->s) != hipSuccess) st = DR_EHIP;
      lk.lock();
      if (st != DR_OK) {
        for (const Req& r : batch) {
          sv->done.push_back({r.ticket, -1.0, (int32_t)st});
          sv->busy_streams.erase(r.sid);
        }
        e->busy = false;
      } else {
        e->inflight = std::move(batch);
        sv->batches += 1;
        sv->batched_requests += n;
      }
      progressed = true;
    }
    bool any_busy = false;
    for (Exec* e : sv->execs) any_busy = any_busy || e->busy;
    if (sv->stop && sv->pending.empty() && !any_busy) break;
    if (!progressed) {
      if (any_busy || !sv->pending.empty())
        sv->cv.wait_for(lk, std::chrono::microseconds(20));
      else
        sv->cv.wait_for(lk, std::chrono::milliseconds(2));
    }
  }
}

extern "C" dr_status dr_server_create(dr_ctx* c, int max_batch, dr_server** out) {
  if (!c || !out) return dr_fail(c, DR_EINVAL, "dr_server_create: null argument");
  *out = nullptr;
  if (max_batch < 1 || max_batch > STREAM_MAXB) return dr_fail(c, DR_EINVAL, "max_batch must be 1..%d", STREAM_MAXB);
  HIP_OK(c, hipSetDevice(c->device));
  dr_server* sv = new dr_server();
  sv->ctx = c;
  sv->max_batch = max_batch;
  // executors (stream, event, workspace for max_batch frames) for the resolutions of the
  // streams already open, so that serving them allocates nothing
  std::set<std::pair<int, int>> classes;
  {
    std::lock_guard<std::mutex> slk(c->smu);
    for (const auto& kv : c->streams) classes.insert({kv.second.H, kv.second.W});
  }
  for (const auto& hw : classes) {
    const char* why = nullptr;
    Exec* e = new_exec(sv, hw.first, hw.second, &why);
    if (!e) {
      for (Exec* x : sv->execs) {
        dr_free_work(x->work);
        (void)hipEventDestroy(x->ev);
        (void)hipStreamDestroy(x->s);
        delete x;
      }
      delete sv;
      return dr_fail(c, DR_ENOMEM, "dr_server_create: %s", why);
    }
    sv->execs.push_back(e);
  }
  sv->th = std::thread(server_loop, sv);
  *out = sv;
  return DR_OK;
}

extern "C" dr_status dr_server_submit(dr_server* sv, int32_t sid, const float* frame, const uint8_t* mask, float* out,
                                      uint64_t* ticket) {
  if (!sv || !frame || !mask || !out || !ticket) return DR_EINVAL;
  const double t_arrive = now_s();  // latency counts from here, before any lock is taken
  dr_ctx* c = sv->ctx;
  int H = 0, W = 0;
  {
    std::lock_guard<std::mutex> slk(c->smu);
    auto it = c->streams.find(sid);
    if (it == c->streams.end()) return dr_fail(c, DR_EINVAL, "no stream %d", sid);
    H = it->second.H;
    W = it->second.W;
  }
  std::lock_guard<std::mutex> lk(sv->mu);
  if (sv->stop) return DR_EBUSY;
  const uint64_t t = sv->next_ticket++;
  sv->pending.push_back({t, sid, frame, mask, out, t_arrive, H, W});
  *ticket = t;
  sv->cv.notify_one();
  return DR_OK;
}

extern "C" dr_status dr_server_poll(dr_server* sv, uint64_t* tickets, double* latency_ms, int32_t* status, int max,
                                    int* n_done) {
  if (!sv || !tickets || !latency_ms || !n_done || max < 0) return DR_EINVAL;
  std::lock_guard<std::mutex> lk(sv->mu);
  const int n = std::min<int>(max, (int)sv->done.size());
  for (int i = 0; i < n; ++i) {
    tickets[i] = sv->done[i].ticket;
    latency_ms[i] = sv->done[i].ms;
    if (status) status[i] = sv->done[i].status;
  }
  sv->done.erase(sv->done.begin(), sv->done.begin() + n);
  *n_done = n;
  return DR_OK;
}

extern "C" dr_status dr_server_stats(dr_server* sv, int64_t* batches, int64_t* requests, int* pending) {
  if (!sv) return DR_EINVAL;
  std::lock_guard<std::mutex> lk(sv->mu);
  if (batches) *batches = sv->batches;
  if (requests) *requests = sv->batched_requests;
  if (pending) *pending = (int)sv->pending.size();
  return DR_OK;
}

extern "C" void dr_server_destroy(dr_server* sv) {
  if (!sv) return;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
    sv->cv.notify_one();
  }
  sv->th.join();
  (void)hipSetDevice(sv->ctx->device);
  for (Exec* e : sv->execs) {
    (void)hipStreamSynchronize(e->s);
    dr_free_work(e->work);
    (void)hipEventDestroy(e->ev);
    (void)hipStreamDestroy(e->s);
    delete e;
  }
  delete sv;
}
