"""Python face of the library: argument marshalling around the C ABI, nothing else.

torch provides device memory and the current HIP stream; every step of the forward runs in
the library's HIP kernels.
"""
from __future__ import annotations

import ctypes as ct

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
        self.stages = _lib.stage_names(self.lib)

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

    def inspect(self, name: str, nbytes: int, stream=None) -> torch.Tensor:
        """Copy of the first ``nbytes`` of a named workspace buffer (uint8 device tensor)."""
        dst = torch.empty(nbytes, dtype=torch.uint8, device=f"cuda:{self.device}")
        st = self.lib.dr_inspect(self._ctx, name.encode(), _ptr(dst), nbytes, _stream(stream))
        _lib.check(self.lib, self._ctx, st)
        return dst

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

    def close(self):
        if self._ctx:
            self.lib.dr_destroy(self._ctx)
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
