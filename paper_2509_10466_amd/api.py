"""Python face of the library: argument marshalling around the C ABI, nothing else.

torch provides device memory and the current HIP stream; every step of the forward runs in
the library's HIP kernels.
"""
from __future__ import annotations

import ctypes as ct

import numpy as np
import torch

from . import _lib
from . import weights as wblob


def _ptr(t: torch.Tensor):
    return ct.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ct.c_void_p(stream.cuda_stream)


class Inpainter:
    """One library context: a network configuration, its weights on one device, and the
    workspace of the largest clip seen so far."""

    def __init__(self, cfg, weights, device: int = 0):
        self.lib = _lib.load()
        self.cfg = cfg
        self.device = device
        self._ctx = ct.c_void_p()
        c = _lib.NetCfgC.from_cfg(cfg)
        st = self.lib.dr_create(ct.byref(self._ctx), device, ct.byref(c))
        _lib.check(self.lib, None, st)
        blob = wblob.pack(cfg, weights)
        buf = ct.create_string_buffer(blob, len(blob))
        _lib.check(self.lib, self._ctx, self.lib.dr_load_weights(self._ctx, buf, len(blob)))
        if getattr(cfg, "attn", "joint") == "decoupled":
            self.set_attention("decoupled")
        self.stages = _lib.stage_names(self.lib)

    def set_attention(self, pattern: str):
        """"joint" (every block over its whole window) or "decoupled" (even blocks within a
        frame of the window, odd blocks across its frames at one position)."""
        code = {"joint": 0, "decoupled": 1}[pattern]
        _lib.check(self.lib, self._ctx, self.lib.dr_set_attention_pattern(self._ctx, code))

    # ------------------------------------------------------------------------------------
    def _check_inputs(self, frames, masks):
        if not (frames.is_cuda and masks.is_cuda):
            raise ValueError("frames and masks must be device tensors")
        if frames.dtype != torch.float32 or masks.dtype != torch.uint8:
            raise ValueError("frames must be float32 and masks uint8")
        if frames.dim() != 5 or frames.shape[-1] != 3 or masks.shape != frames.shape[:-1]:
            raise ValueError("frames must be [B,T,H,W,3] and masks [B,T,H,W]")
        if not (frames.is_contiguous() and masks.is_contiguous()):
            raise ValueError("frames and masks must be contiguous")

    def reserve(self, B, T, H, W, precision="bf16"):
        _lib.check(self.lib, self._ctx, self.lib.dr_reserve(self._ctx, B, T, H, W, _lib.PRECISION[precision]))

    def __call__(self, frames: torch.Tensor, masks: torch.Tensor, precision: str = "bf16",
                 query_set: str = "masked", out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """Inpaint ``frames`` [B,T,H,W,3] f32 under ``masks`` [B,T,H,W] u8 (nonzero = private).
        Returns ``out`` (allocated if not given; may be ``frames`` for in-place use)."""
        self._check_inputs(frames, masks)
        if out is None:
            out = torch.empty_like(frames)
        elif out.shape != frames.shape or out.dtype != torch.float32 or not out.is_contiguous():
            raise ValueError("out must match frames")
        B, T, H, W, _ = frames.shape
        st = self.lib.dr_inpaint(self._ctx, _ptr(frames), _ptr(masks), _ptr(out), B, T, H, W,
                                 _lib.PRECISION[precision], _lib.QUERY_SET[query_set], _stream(stream))
        _lib.check(self.lib, self._ctx, st)
        return out

    def gather_tokens(self, masks: torch.Tensor, query_set: str = "masked", stream=None):
        """(flag u8 [N], idx int32 [Nq], woff int32 [nwin+1]) in window-major token order."""
        if not masks.is_cuda or masks.dtype != torch.uint8 or masks.dim() != 4 or not masks.is_contiguous():
            raise ValueError("masks must be a contiguous uint8 device tensor [B,T,H,W]")
        B, T, H, W = masks.shape
        p = self.cfg.patch
        N = B * T * (H // p) * (W // p)
        nwin = max(N // self.cfg.window_tokens, 0)
        dev = masks.device
        flag = torch.empty(N, dtype=torch.uint8, device=dev)
        idx = torch.empty(N, dtype=torch.int32, device=dev)
        woff = torch.empty(nwin + 1, dtype=torch.int32, device=dev)
        nq = torch.empty(1, dtype=torch.int32, device=dev)
        st = self.lib.dr_gather_tokens(self._ctx, _ptr(masks), B, T, H, W, _lib.QUERY_SET[query_set],
                                       _ptr(flag), _ptr(idx), _ptr(woff), _ptr(nq), _stream(stream))
        _lib.check(self.lib, self._ctx, st)
        n = int(nq.item())
        return flag, idx[:n], woff

    def prep_frame(self, bgra: torch.Tensor, instances: torch.Tensor | None = None, select: int = 0xFFFFFFFF,
                   radius: int = 0, stream=None):
        """Camera frame u8 BGRA [H,W,4] and instance masks u8 [K,H,W] -> (frame_low f32
        [H/2,W/2,3], mask_low u8 [H/2,W/2], mask_full u8 [H,W]); bit k of ``select`` picks
        instance k, the union is dilated by a (2 radius + 1)^2 square."""
        if not bgra.is_cuda or bgra.dtype != torch.uint8 or bgra.dim() != 3 or bgra.shape[2] != 4 \
                or not bgra.is_contiguous():
            raise ValueError("bgra must be a contiguous uint8 device tensor [H,W,4]")
        H, W, _ = bgra.shape
        K = 0
        if instances is not None:
            if instances.dtype != torch.uint8 or instances.dim() != 3 or tuple(instances.shape[1:]) != (H, W) \
                    or not instances.is_contiguous() or instances.device != bgra.device:
                raise ValueError("instances must be a contiguous uint8 tensor [K,H,W] on the frame's device")
            K = instances.shape[0]
        dev = bgra.device
        frame_low = torch.empty((H // 2, W // 2, 3), dtype=torch.float32, device=dev)
        mask_low = torch.empty((H // 2, W // 2), dtype=torch.uint8, device=dev)
        mask_full = torch.empty((H, W), dtype=torch.uint8, device=dev)
        st = self.lib.dr_prep_frame(self._ctx, _ptr(bgra), _ptr(instances) if K else None, K, select & 0xFFFFFFFF,
                                    radius, H, W, _ptr(frame_low), _ptr(mask_low), _ptr(mask_full), _stream(stream))
        _lib.check(self.lib, self._ctx, st)
        return frame_low, mask_low, mask_full

    def post_frame(self, bgra: torch.Tensor, pred_low: torch.Tensor, mask_full: torch.Tensor,
                   out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """Composite the half-resolution prediction f32 [H/2,W/2,3] into the camera frame
        (u8 BGRA [H,W,4]) where ``mask_full`` is set; other pixels are copied."""
        H, W, _ = bgra.shape
        for t, dt, shape in ((bgra, torch.uint8, (H, W, 4)), (pred_low, torch.float32, (H // 2, W // 2, 3)),
                             (mask_full, torch.uint8, (H, W))):
            if not t.is_cuda or t.dtype != dt or tuple(t.shape) != shape or not t.is_contiguous():
                raise ValueError(f"expected a contiguous {dt} device tensor {shape}")
        if out is None:
            out = torch.empty_like(bgra)
        st = self.lib.dr_post_frame(self._ctx, _ptr(bgra), _ptr(pred_low), _ptr(mask_full), H, W, _ptr(out),
                                    _stream(stream))
        _lib.check(self.lib, self._ctx, st)
        return out

    def inspect(self, name: str, nbytes: int, stream=None) -> torch.Tensor:
        """Copy of the first ``nbytes`` of a named workspace buffer (uint8 device tensor)."""
        dst = torch.empty(nbytes, dtype=torch.uint8, device=f"cuda:{self.device}")
        st = self.lib.dr_inspect(self._ctx, name.encode(), _ptr(dst), nbytes, _stream(stream))
        _lib.check(self.lib, self._ctx, st)
        return dst

    def fp8_encode(self, values: torch.Tensor, scale: float, stream=None) -> torch.Tensor:
        """e4m3 codes (uint8) of values / scale, as the FP8 path quantises."""
        if not values.is_cuda or values.dtype != torch.float32 or not values.is_contiguous():
            raise ValueError("values must be a contiguous float32 device tensor")
        out = torch.empty(values.shape, dtype=torch.uint8, device=values.device)
        st = self.lib.dr_fp8_encode(self._ctx, _ptr(values), _ptr(out), values.numel(), scale, _stream(stream))
        _lib.check(self.lib, self._ctx, st)
        return out

    def debug_set(self, key: str, value: int):
        _lib.check(self.lib, self._ctx, self.lib.dr_debug_set(self._ctx, key.encode(), value))

    # ------------------------------------------------------------------------------------
    def profile(self, enable: bool = True):
        _lib.check(self.lib, self._ctx, self.lib.dr_profile(self._ctx, int(enable)))

    def profile_read(self):
        """{stage: (total ms, launches)} accumulated since the last read."""
        n = len(self.stages)
        ms = (ct.c_double * n)()
        cnt = (ct.c_int64 * n)()
        _lib.check(self.lib, self._ctx, self.lib.dr_profile_read(self._ctx, ms, cnt, n))
        return {self.stages[i]: (ms[i], cnt[i]) for i in range(n) if cnt[i]}

    # ---- training ---------------------------------------------------------------------
    def param_count(self) -> int:
        return int(self.lib.dr_param_count(self._ctx))

    def load_params(self, flat: torch.Tensor, stream=None):
        """Replace the weights from a flat FP32 parameter vector on this context's device (blob
        order).  The library derives every layout it needs on the device, on ``stream``; no
        data passes through host memory."""
        if not flat.is_cuda or flat.dtype != torch.float32 or not flat.is_contiguous() \
                or flat.numel() != self.param_count():
            raise ValueError("params must be a contiguous float32 device tensor of param_count() values")
        _lib.check(self.lib, self._ctx, self.lib.dr_load_params(self._ctx, _ptr(flat), _stream(stream)))

    def train_precision(self, precision: str):
        """"fp32" (default) or "bf16": bf16 operands with FP32 accumulation for the weight
        products of the training forward and reverse passes (FP32 master weights and
        gradients); takes effect at the next train_forward."""
        _lib.check(self.lib, self._ctx, self.lib.dr_train_set_precision(self._ctx, _lib.PRECISION[precision]))

    def train_forward(self, frames: torch.Tensor, masks: torch.Tensor, stream=None):
        """(pred, saved): the decoder prediction at every pixel [B,T,H,W,3] (before the
        composite) and the handle of the activations (and weights) its reverse pass needs."""
        self._check_inputs(frames, masks)
        pred = torch.empty_like(frames)
        B, T, H, W, _ = frames.shape
        h = ct.c_void_p()
        st = self.lib.dr_train_forward(self._ctx, _ptr(frames), _ptr(masks), _ptr(pred), B, T, H, W, ct.byref(h),
                                       _stream(stream))
        _lib.check(self.lib, self._ctx, st)
        return pred, Saved(self, h)

    def train_backward(self, saved: "Saved", dpred: torch.Tensor, stream=None) -> torch.Tensor:
        """dL/dparams (flat FP32, blob order) of the forward that produced ``saved``."""
        if saved.eng is not self or not saved.handle:
            raise ValueError("saved activations of another context, or already released")
        dpred = dpred.contiguous().float()
        grads = torch.empty(self.param_count(), dtype=torch.float32, device=dpred.device)
        st = self.lib.dr_train_backward(self._ctx, saved.handle, _ptr(dpred), _ptr(grads), _stream(stream))
        _lib.check(self.lib, self._ctx, st)
        return grads

    def l1_loss(self, pred, gt, masks, w_in: float = 1.0, w_out: float = 0.1, stream=None):
        """(loss [1] device tensor, dL/dpred)."""
        loss = torch.empty(1, dtype=torch.float32, device=pred.device)
        dpred = torch.empty_like(pred)
        st = self.lib.dr_l1_loss(self._ctx, _ptr(pred), _ptr(gt), _ptr(masks), masks.numel(), w_in, w_out,
                                 _ptr(loss), _ptr(dpred), _stream(stream))
        _lib.check(self.lib, self._ctx, st)
        return loss, dpred

    # ---- stream mode ------------------------------------------------------------------
    def set_budget(self, nbytes: int):
        _lib.check(self.lib, self._ctx, self.lib.dr_set_budget(self._ctx, int(nbytes)))

    def stream_footprint(self, H: int, W: int) -> int:
        return int(self.lib.dr_stream_footprint(self._ctx, H, W))

    def stream_open(self, H: int, W: int, slots: int | None = None) -> int:
        """Open a stream of H x W frames keeping `slots` past frames (default win_t - 1)."""
        sid = ct.c_int32()
        if slots is None:
            st = self.lib.dr_stream_open(self._ctx, H, W, ct.byref(sid))
        else:
            st = self.lib.dr_stream_open_slots(self._ctx, H, W, int(slots), ct.byref(sid))
        _lib.check(self.lib, self._ctx, st)
        return sid.value

    def stream_close(self, sid: int):
        _lib.check(self.lib, self._ctx, self.lib.dr_stream_close(self._ctx, sid))

    def stream_step(self, sids, frames, masks, outs=None, query_set: str = "masked", stream=None):
        """Inpaint the newest frame [H,W,3] of each stream in ``sids`` (one batch)."""
        n = len(sids)
        if not (len(frames) == len(masks) == n):
            raise ValueError("one frame and one mask per stream")
        for f, m in zip(frames, masks):
            if not (f.is_cuda and m.is_cuda and f.dtype == torch.float32 and m.dtype == torch.uint8
                    and f.is_contiguous() and m.is_contiguous() and f.dim() == 3 and f.shape[-1] == 3
                    and m.shape == f.shape[:-1]):
                raise ValueError("frames must be contiguous f32 [H,W,3] and masks u8 [H,W] device tensors")
        if outs is None:
            outs = [torch.empty_like(f) for f in frames]
        sid_arr = (ct.c_int32 * n)(*sids)
        fp = (ct.c_void_p * n)(*[f.data_ptr() for f in frames])
        mp = (ct.c_void_p * n)(*[m.data_ptr() for m in masks])
        op = (ct.c_void_p * n)(*[o.data_ptr() for o in outs])
        st = self.lib.dr_stream_step(self._ctx, n, sid_arr, fp, mp, op, _lib.PRECISION["bf16"],
                                     _lib.QUERY_SET[query_set], _stream(stream))
        _lib.check(self.lib, self._ctx, st)
        return outs

    def close(self):
        if self._ctx:
            self.lib.dr_destroy(self._ctx)  # releases every saved-activation handle too
            self._ctx = ct.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def inpaint(frames, masks, weights, cfg, precision: str = "bf16", query_set: str = "masked"):
    """One-shot form of ``Inpainter(cfg, weights)(frames, masks, precision, query_set)``."""
    eng = Inpainter(cfg, weights, device=frames.device.index or 0)
    try:
        out = eng(frames, masks, precision, query_set)
        torch.cuda.current_stream().synchronize()
        return out
    finally:
        eng.close()


class Server:
    """The library's native serving loop on one Inpainter context."""

    def __init__(self, eng: Inpainter, max_batch: int = 16):
        self.eng = eng
        self.lib = eng.lib
        self._srv = ct.c_void_p()
        _lib.check(self.lib, eng._ctx, self.lib.dr_server_create(eng._ctx, max_batch, ct.byref(self._srv)))

    def submit(self, sid: int, frame: torch.Tensor, mask: torch.Tensor, out: torch.Tensor) -> int:
        t = ct.c_uint64()
        st = self.lib.dr_server_submit(self._srv, sid, _ptr(frame), _ptr(mask), _ptr(out), ct.byref(t))
        _lib.check(self.lib, self.eng._ctx, st)
        return t.value

    def poll(self, max_n: int = 4096):
        """[(ticket, latency_ms, status)] of requests completed since the last poll."""
        tk = (ct.c_uint64 * max_n)()
        lat = (ct.c_double * max_n)()
        sts = (ct.c_int32 * max_n)()
        n = ct.c_int()
        _lib.check(self.lib, self.eng._ctx, self.lib.dr_server_poll(self._srv, tk, lat, sts, max_n, ct.byref(n)))
        return [(tk[i], lat[i], sts[i]) for i in range(n.value)]

    def stats(self):
        b, r, p = ct.c_int64(), ct.c_int64(), ct.c_int()
        _lib.check(self.lib, self.eng._ctx, self.lib.dr_server_stats(self._srv, ct.byref(b), ct.byref(r), ct.byref(p)))
        return {"batches": b.value, "requests": r.value, "pending": p.value}

    def close(self):
        if self._srv:
            self.lib.dr_server_destroy(self._srv)
            self._srv = ct.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _shapes(cfg):
    C, p, R = cfg.dim, cfg.patch, cfg.mlp_ratio * cfg.dim
    out = [("embed.w", (C, 3, p, p)), ("embed.b", (C,))]
    for l in range(cfg.blocks):
        b = f"blk{l}."
        out += [(b + "ln1.g", (C,)), (b + "ln1.b", (C,)), (b + "wq", (C, C)), (b + "bq", (C,)),
                (b + "wk", (C, C)), (b + "bk", (C,)), (b + "wv", (C, C)), (b + "bv", (C,)),
                (b + "wo", (C, C)), (b + "bo", (C,)), (b + "ln2.g", (C,)), (b + "ln2.b", (C,)),
                (b + "w1", (R, C)), (b + "b1", (R,)), (b + "w2", (C, R)), (b + "b2", (C,))]
    return out + [("lnf.g", (C,)), ("lnf.b", (C,)), ("dec.w", (C, 3, p, p)), ("dec.b", (3,))]


def flatten_params(cfg, weights) -> torch.Tensor:
    """Flat FP32 parameter vector (blob order) from a name -> array mapping."""
    return torch.cat([torch.as_tensor(np.asarray(weights[n], np.float32)).reshape(-1) for n, _ in _shapes(cfg)])


def unflatten_params(cfg, flat):
    """name -> view of a flat parameter vector."""
    out, o = {}, 0
    for n, shp in _shapes(cfg):
        size = int(np.prod(shp))
        out[n] = flat[o:o + size].reshape(shp)
        o += size
    return out


class Saved:
    """Handle of one training forward's saved activations; released by ``close`` (or when
    garbage-collected).  Work already enqueued that reads it must be ordered before the next
    training forward on the same context, which may reuse its buffers."""

    def __init__(self, eng: Inpainter, handle: ct.c_void_p):
        self.eng = eng
        self.handle = handle

    def close(self):
        if self.handle and self.eng._ctx:
            _lib.check(self.eng.lib, self.eng._ctx, self.eng.lib.dr_saved_free(self.eng._ctx, self.handle))
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class InpaintFn(torch.autograd.Function):
    """pred = network(frames, masks; params) with the library's hand-written backward.

    ``params`` is the flat FP32 parameter vector (blob order) on the context's device; the
    prediction is the decoder output at every pixel, before the composite (the training loss
    is taken on it).  Each application keeps its own saved activations, so several forwards
    may precede their backwards.  The parameters are loaded on the device, and only when the
    tensor object, or its contents by torch's version counter, differs from the last load (the
    last loaded tensor is kept referenced, so its memory cannot be handed to another tensor)."""

    @staticmethod
    def forward(ctx, frames, masks, params, eng):
        last = getattr(eng, "_params_last", None)
        if last is None or last[0] is not params or last[1] != params._version:
            eng.load_params(params.detach().contiguous())
            eng._params_last = (params, params._version)
        pred, saved = eng.train_forward(frames.contiguous(), masks.contiguous())
        ctx.eng = eng
        ctx.saved = saved
        return pred

    @staticmethod
    def backward(ctx, dpred):
        grads = ctx.eng.train_backward(ctx.saved, dpred)
        ctx.saved.close()
        return None, None, grads, None
