"""Stream mode of the inpainting network, FP64 -- test infrastructure only.

The thesis's inpainting model runs frame by frame: it takes the newest frame (private
regions set to 0) together with memory tensors kept from its previous outputs and returns
the completed frame plus a new memory tensor (Methods, "Inpainting Manager"; the number of
memory slots is the ablation of "Performance Optimisations -- Inpainting Model").  Stream
mode realises that memory for the windowed network:

* every block l keeps, per stream, the keys and values of the last ``win_t - 1`` frames,
  each cached when that frame was the newest one;
* for a new frame, block l computes Q/K/V of the new frame's tokens; the queries (flagged
  tokens of the new frame) attend to the keys/values of their spatial window in the cached
  frames followed by the new frame (win_h x win_w tokens per frame, no key mask);
* decoupled networks (``cfg.attn == "decoupled"``; even blocks within one frame of a
  window, odd blocks across its frames at one token position, as in clip mode): a spatial
  block's queries attend to their spatial window in the new frame only, a temporal block's
  to their own token position in the cached frames followed by the new frame;
* the projection, MLP, final LayerNorm, decoder and composite act on the new frame only;
* then the new frame's K/V of every block enter the cache, dropping the oldest frame.

The first frames of a stream attend to the frames available so far.  Stream mode is causal,
so its outputs are not the clip-mode outputs.
"""
from __future__ import annotations

import numpy as np

from . import network as on

F64 = np.float64


class StreamState:
    """Per-stream cache: kv[l] is a list (oldest first) of (K, V), each [Ht, Wt, C].  ``slots``
    is the number of past frames kept (the thesis's memory slots m); default win_t - 1."""

    def __init__(self, cfg, slots=None):
        self.cfg = cfg
        self.slots = cfg.win_t - 1 if slots is None else int(slots)
        if not 0 <= self.slots <= cfg.win_t - 1:
            raise ValueError("slots must be in [0, win_t - 1]")
        self.kv = [[] for _ in range(cfg.blocks)]


def _windows2d(a, cfg):
    """[Ht, Wt, C] -> [nH, nW, wh*ww, C] (spatial windows of one frame)."""
    Ht, Wt, C = a.shape
    wh, ww = cfg.win_h, cfg.win_w
    a = a.reshape(Ht // wh, wh, Wt // ww, ww, C).transpose(0, 2, 1, 3, 4)
    return a.reshape(Ht // wh, Wt // ww, wh * ww, C)


def _unwindows2d(a, cfg):
    nH, nW, Sf, C = a.shape
    wh, ww = cfg.win_h, cfg.win_w
    return a.reshape(nH, nW, wh, ww, C).transpose(0, 2, 1, 3, 4).reshape(nH * wh, nW * ww, C)


def step(state: StreamState, frame, mask, W, cfg, query_set="masked"):
    """Inpaint one new frame [H, W, 3] with mask [H, W]; updates ``state``.
    Returns (out [H, W, 3] FP64, pred [H, W, 3])."""
    if getattr(cfg, "overlap", False):
        raise NotImplementedError("the overlapping embedding/decoder runs in clip mode only")
    p = cfg.patch
    H, Wd, _ = frame.shape
    if H % (p * cfg.win_h) or Wd % (p * cfg.win_w):
        raise ValueError("frame does not tile into whole windows")
    f5 = frame[None, None]
    m4 = mask[None, None]
    xc = on.cut_out(f5, m4)
    flags = on.token_flags(m4, p)[0, 0]
    upd = flags if query_set == "masked" else np.ones_like(flags)
    x = on.patch_embed(xc, W["embed.w"], W["embed.b"], p)[0, 0]          # [Ht, Wt, C]
    heads = cfg.heads
    new_kv = []
    for l in range(cfg.blocks):
        pre = f"blk{l}."
        w = lambda n: np.asarray(W[pre + n], F64)  # noqa: E731
        u = on.layer_norm(x, w("ln1.g"), w("ln1.b"))
        q = on.linear(u, w("wq"), w("bq"))
        k = on.linear(u, w("wk"), w("bk"))
        v = on.linear(u, w("wv"), w("bv"))
        past = state.kv[l]
        kind = on.block_attention_kind(l, cfg)
        if kind == "temporal":
            # one token position across the cached frames and the new one: [Ht, Wt, F, C]
            keys = np.stack([kk for kk, _ in past] + [k], axis=2)
            vals = np.stack([vv for _, vv in past] + [v], axis=2)
            o = _cross_attention(q[:, :, None, :], keys, vals, heads)[:, :, 0, :]
        else:
            frames_kv = [] if kind == "spatial" else past
            keys = np.concatenate([_windows2d(kk, cfg) for kk, _ in frames_kv] + [_windows2d(k, cfg)], axis=2)
            vals = np.concatenate([_windows2d(vv, cfg) for _, vv in frames_kv] + [_windows2d(v, cfg)], axis=2)
            o_w = _cross_attention(_windows2d(q, cfg), keys, vals, heads)
            o = _unwindows2d(o_w, cfg)
        x1 = x + on.linear(o, w("wo"), w("bo"))
        h = on.linear(on.layer_norm(x1, w("ln2.g"), w("ln2.b")), w("w1"), w("b1"))
        x2 = x1 + on.linear(on.gelu(h), w("w2"), w("b2"))
        x = np.where(upd[..., None], x2, x)
        new_kv.append((k, v))
    for l in range(cfg.blocks):
        state.kv[l].append(new_kv[l])
        while len(state.kv[l]) > state.slots:
            state.kv[l].pop(0)
    z = on.layer_norm(x, np.asarray(W["lnf.g"], F64), np.asarray(W["lnf.b"], F64))
    pred = on.sigmoid(on.decode_logits(z[None, None], W["dec.w"], W["dec.b"], p))[0, 0]
    out = np.where(mask[..., None] != 0, pred, frame.astype(F64))
    return out, pred


def _cross_attention(q, k, v, heads):
    """q [..., Sq, C], k/v [..., Sk, C]: softmax(Q K^T / sqrt(dh)) V per head."""
    lead = q.shape[:-2]
    Sq, C = q.shape[-2:]
    Sk = k.shape[-2]
    dh = C // heads
    n = int(np.prod(lead))
    qf = q.reshape(n, Sq, heads, dh).transpose(0, 2, 1, 3)
    kf = k.reshape(n, Sk, heads, dh).transpose(0, 2, 1, 3)
    vf = v.reshape(n, Sk, heads, dh).transpose(0, 2, 1, 3)
    a = on.softmax(qf @ kf.transpose(0, 1, 3, 2) / np.sqrt(dh))
    o = a @ vf
    return o.transpose(0, 2, 1, 3).reshape(*lead, Sq, C)


def run_stream(frames, masks, W, cfg, query_set="masked", slots=None):
    """Replay a whole stream: frames [T, H, W, 3], masks [T, H, W] -> outputs [T, H, W, 3]."""
    st = StreamState(cfg, slots)
    return np.stack([step(st, frames[t], masks[t], W, cfg, query_set)[0] for t in range(len(frames))])
