"""Clip-mode forward of the inpainting network, FP64, written for reading, not speed.

Test infrastructure only (see the package docstring).  Weights are the FP32 master
tensors promoted exactly to FP64; every BF16/FP8 rounding of the GPU path therefore
counts as error of that path.

The thesis (Methods, "Inpainting Manager") fixes the interface of the network: it takes a
frame whose private regions are set to 0 and returns a completed frame whose redacted
regions are filled with generated background; the private regions come from the object
masks cut out of the frame (Methods, "Object Control").  The thesis names DSTT-style
windowed spatio-temporal attention and scaled-dot-product attention (Methods,
"Performance Optimisations -- Inpainting Model") but prints no layer sizes, so the layer
stack below is the evaluated network: a strided-conv patch embedding, pre-LN blocks of
windowed multi-head self-attention and a GELU MLP, a final LayerNorm, a transposed-conv
decoder with a sigmoid, and the mask composite.

Readings taken where the description is silent (each is also the GPU path's definition):

* query set: only *flagged* tokens (tokens whose patch holds any private pixel) are
  attention queries and are updated; keys and values are all tokens of the window, with no
  key mask.  ``query_set="all"`` makes every token a query (the flag is all ones).
* token flag: logical OR of the mask over the token's p x p pixels.
* network input: the 3-channel cut-out frame; no mask channel, no positional encoding.
* blocks: pre-LN, LayerNorm with biased variance and eps = 1e-5, affine.
* attention: scale 1/sqrt(dh), head k owns channels [k*dh, (k+1)*dh), QKV biases, no
  dropout, no relative bias, no shifted windows; windows tile the token grid from (0, 0).
* decoupled variant (``cfg.attn == "decoupled"``): even blocks attend within the per-frame
  windows (win_h x win_w tokens), odd blocks across the win_t frames of a window at one
  token position; everything else is the joint network.
* MLP: Linear(C, rC) -> exact-erf GELU -> Linear(rC, C).
* final LayerNorm before the decoder; decoder = ConvTranspose2d(C, 3, k=p, s=p) + sigmoid.
* composite: a per-pixel select, out = pred where the mask is nonzero, else the input.
* overlapping variant (``cfg.overlap``; the thesis's DSTT base embeds overlapping patches and
  rebuilds the frame with a fold that sums the overlaps, which the thesis replaced by a
  reduction convolution plus a crop for TensorRT; Methods, "Performance Optimisations --
  Modified Vec2Patch"): embedding Conv2d(3, C, k = 2p, s = p, padding p/2) with zero
  padding; decoder = each token's 2p x 2p x 3 patch of logits, folded (overlaps summed)
  onto the padded frame, cropped by p/2 on every side, plus the bias, then the sigmoid.  A
  token is a query when any pixel of its 2p x 2p footprint inside the frame is private, so
  every token that a private pixel's logit sums over is updated.
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf

F64 = np.float64
LN_EPS = 1e-5


def _w(W, name):
    return np.asarray(W[name], dtype=F64)


def check_shape(frames, masks, cfg):
    B, T, H, Wd, ch = frames.shape
    if ch != 3 or masks.shape != (B, T, H, Wd):
        raise ValueError("frames must be [B,T,H,W,3] and masks [B,T,H,W]")
    p = cfg.patch
    if H % (p * cfg.win_h) or Wd % (p * cfg.win_w) or T % cfg.win_t:
        raise ValueError("shape does not tile into whole windows")


def cut_out(frames, masks):
    """The network input: private pixels set to 0, all others unchanged (Methods, "Object
    Control" and "Inpainting Manager")."""
    return np.where(masks[..., None] != 0, 0.0, frames.astype(F64))


def token_flags(masks, p):
    """flag[b, t, i, j] is True iff any pixel in rows p*i..p*i+p-1, columns p*j..p*j+p-1 of
    frame t is private (OR rule)."""
    B, T, H, W = masks.shape
    return (masks != 0).reshape(B, T, H // p, p, W // p, p).any(axis=(3, 5))


def token_flags_overlap(masks, p):
    """flag[b, t, i, j] is True iff any pixel of rows p*i - p/2 .. p*i + 3p/2 - 1, columns
    likewise, that lies inside the frame is private (the footprint of a kernel-2p token)."""
    m = masks != 0
    B, T, H, W = m.shape
    h = p // 2
    mp = np.zeros((B, T, H + 2 * h, W + 2 * h), dtype=bool)
    mp[:, :, h:h + H, h:h + W] = m
    Ht, Wt = H // p, W // p
    out = np.zeros((B, T, Ht, Wt), dtype=bool)
    for ky in range(2 * p):
        for kx in range(2 * p):
            out |= mp[:, :, ky:ky + p * Ht:p, kx:kx + p * Wt:p]
    return out


def patch_embed_overlap(xc, w, b, p):
    """Conv2d(3 -> C, kernel 2p, stride p, padding p/2, zero padding) on each frame, w OIHW
    [C, 3, 2p, 2p]: x[.., i, j, o] = b[o] + sum w[o, c, ky, kx] * xpad[p*i + ky, p*j + kx, c]."""
    B, T, H, W, _ = xc.shape
    h = p // 2
    xp = np.zeros((B, T, H + 2 * h, W + 2 * h, 3))
    xp[:, :, h:h + H, h:h + W] = xc
    w = np.asarray(w, F64)
    Ht, Wt = H // p, W // p
    x = np.zeros((B, T, Ht, Wt, w.shape[0])) + np.asarray(b, F64)
    for ky in range(2 * p):
        for kx in range(2 * p):
            x += xp[:, :, ky:ky + p * Ht:p, kx:kx + p * Wt:p, :] @ w[:, :, ky, kx].T
    return x


def decode_logits_fold(z, wd, bd, p):
    """Vec2Patch by fold: token (i, j) projects z to a 2p x 2p x 3 patch
    patch[ky, kx, ch] = sum_c z[c] wd[c, ch, ky, kx] (wd IOHW [C, 3, 2p, 2p]); the patches are
    added onto the padded frame at (p*i, p*j) (overlaps summed), the p/2 border is cropped and
    the bias added.  Equals ConvTranspose2d(C, 3, 2p, stride p, padding p/2)."""
    B, T, Ht, Wt, _ = z.shape
    k, h = 2 * p, p // 2
    patches = np.einsum("btijc,cdyx->btijyxd", z, np.asarray(wd, F64))
    canvas = np.zeros((B, T, p * Ht + 2 * h, p * Wt + 2 * h, 3))
    for i in range(Ht):
        for j in range(Wt):
            canvas[:, :, p * i:p * i + k, p * j:p * j + k] += patches[:, :, i, j]
    return canvas[:, :, h:h + p * Ht, h:h + p * Wt] + np.asarray(bd, F64)


def patch_embed(xc, w, b, p):
    """Conv2d(3 -> C, kernel p, stride p, no padding) on each frame:
    x[b,t,i,j,o] = b[o] + sum_{c,ky,kx} w[o,c,ky,kx] * xc[b,t,p*i+ky,p*j+kx,c];  w is OIHW."""
    B, T, H, W, _ = xc.shape
    patches = xc.reshape(B, T, H // p, p, W // p, p, 3)  # b t i ky j kx c
    return np.einsum("btiyjxc,ocyx->btijo", patches, np.asarray(w, F64)) + np.asarray(b, F64)


def layer_norm(x, g, b, eps=LN_EPS):
    """Per-token LayerNorm over the channel axis: biased variance, eps inside the root."""
    mu = x.mean(axis=-1, keepdims=True)
    var = ((x - mu) ** 2).mean(axis=-1, keepdims=True)
    return (x - mu) / np.sqrt(var + eps) * g + b


def linear(x, w, b):
    """y = x w^T + b with w stored [out, in]."""
    return x @ w.T + b


def gelu(z):
    """Exact GELU: 0.5 z (1 + erf(z / sqrt 2))."""
    return 0.5 * z * (1.0 + erf(z / np.sqrt(2.0)))


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def to_windows(x, cfg):
    """[B, T, Ht, Wt, C] -> [B, nT, nH, nW, S, C].  Window (a, u, v) holds tokens of frames
    a*wt.., rows u*wh.., columns v*ww..; inside a window tokens are ordered (dt, di, dj)."""
    B, T, Ht, Wt, C = x.shape
    wt, wh, ww = cfg.win_t, cfg.win_h, cfg.win_w
    x = x.reshape(B, T // wt, wt, Ht // wh, wh, Wt // ww, ww, C)
    x = x.transpose(0, 1, 3, 5, 2, 4, 6, 7)
    return x.reshape(B, T // wt, Ht // wh, Wt // ww, wt * wh * ww, C)


def from_windows(xw, cfg):
    """Inverse of ``to_windows``."""
    B, nT, nH, nW, S, C = xw.shape
    wt, wh, ww = cfg.win_t, cfg.win_h, cfg.win_w
    x = xw.reshape(B, nT, nH, nW, wt, wh, ww, C).transpose(0, 1, 4, 2, 5, 3, 6, 7)
    return x.reshape(B, nT * wt, nH * wh, nW * ww, C)


def to_frame_windows(x, cfg):
    """[B, T, Ht, Wt, C] -> [B, T, nH, nW, wh*ww, C]: the spatial windows of one frame."""
    B, T, Ht, Wt, C = x.shape
    wh, ww = cfg.win_h, cfg.win_w
    x = x.reshape(B, T, Ht // wh, wh, Wt // ww, ww, C).transpose(0, 1, 2, 4, 3, 5, 6)
    return x.reshape(B, T, Ht // wh, Wt // ww, wh * ww, C)


def from_frame_windows(xw, cfg):
    """Inverse of ``to_frame_windows``."""
    B, T, nH, nW, _, C = xw.shape
    wh, ww = cfg.win_h, cfg.win_w
    x = xw.reshape(B, T, nH, nW, wh, ww, C).transpose(0, 1, 2, 4, 3, 5, 6)
    return x.reshape(B, T, nH * wh, nW * ww, C)


def to_time_windows(x, cfg):
    """[B, T, Ht, Wt, C] -> [B, T/wt, Ht, Wt, wt, C]: one token position across the win_t
    frames of a window."""
    B, T, Ht, Wt, C = x.shape
    wt = cfg.win_t
    return x.reshape(B, T // wt, wt, Ht, Wt, C).transpose(0, 1, 3, 4, 2, 5)


def from_time_windows(xw, cfg):
    """Inverse of ``to_time_windows``."""
    B, nT, Ht, Wt, wt, C = xw.shape
    return xw.transpose(0, 1, 4, 2, 3, 5).reshape(B, nT * wt, Ht, Wt, C)


def block_attention_kind(l, cfg):
    """"joint" for every block of a joint-attention network; for a decoupled one (DSTT-style,
    Background, "Decoupled Spatial-Temporal Transformer") block l attends "spatial"-ly
    (within one frame of its window) when l is even and "temporal"-ly (across the window's
    frames at one token position) when l is odd."""
    if getattr(cfg, "attn", "joint") == "joint":
        return "joint"
    return "spatial" if l % 2 == 0 else "temporal"


def softmax(s):
    """Row softmax over the last axis (the row max is subtracted first; this changes no
    value in exact arithmetic)."""
    e = np.exp(s - s.max(axis=-1, keepdims=True))
    return e / e.sum(axis=-1, keepdims=True)


def multi_head_attention(q, k, v, heads, chunk=64):
    """softmax(Q K^T / sqrt(dh)) V for every head of every window.

    q, k, v: [..., S, C]; each leading index is one window, every query attends to all S
    keys of its own window.  Windows are processed in groups of ``chunk`` only to bound
    memory.  Returns (O [..., S, C], P [..., heads, S, S] or None when large)."""
    lead = q.shape[:-2]
    S, C = q.shape[-2:]
    dh = C // heads
    nwin = int(np.prod(lead)) if lead else 1
    qf = q.reshape(nwin, S, heads, dh).transpose(0, 2, 1, 3)
    kf = k.reshape(nwin, S, heads, dh).transpose(0, 2, 1, 3)
    vf = v.reshape(nwin, S, heads, dh).transpose(0, 2, 1, 3)
    out = np.empty((nwin, heads, S, dh))
    keep_p = nwin * heads * S * S <= 4_000_000
    probs = np.empty((nwin, heads, S, S)) if keep_p else None
    for w0 in range(0, nwin, chunk):
        sl = slice(w0, w0 + chunk)
        a = softmax(qf[sl] @ kf[sl].transpose(0, 1, 3, 2) / np.sqrt(dh))
        out[sl] = a @ vf[sl]
        if keep_p:
            probs[sl] = a
    o = out.transpose(0, 2, 1, 3).reshape(*lead, S, C)
    if keep_p:
        probs = probs.reshape(*lead, heads, S, S)
    return o, probs


def block(x, upd, W, l, cfg, trace=None):
    """One pre-LN transformer block on the token grid x [B, T, Ht, Wt, C].

    Every token supplies keys and values; the attention output, the projection and the MLP
    are applied to the tokens selected by ``upd`` (boolean [B, T, Ht, Wt]); all other
    tokens pass through unchanged."""
    p = f"blk{l}."
    u = layer_norm(x, _w(W, p + "ln1.g"), _w(W, p + "ln1.b"))
    q = linear(u, _w(W, p + "wq"), _w(W, p + "bq"))
    k = linear(u, _w(W, p + "wk"), _w(W, p + "bk"))
    v = linear(u, _w(W, p + "wv"), _w(W, p + "bv"))
    kind = block_attention_kind(l, cfg)
    to, back = {"joint": (to_windows, from_windows), "spatial": (to_frame_windows, from_frame_windows),
                "temporal": (to_time_windows, from_time_windows)}[kind]
    o_w, probs = multi_head_attention(to(q, cfg), to(k, cfg), to(v, cfg), cfg.heads)
    o = back(o_w, cfg)
    x1 = x + linear(o, _w(W, p + "wo"), _w(W, p + "bo"))
    h = linear(layer_norm(x1, _w(W, p + "ln2.g"), _w(W, p + "ln2.b")), _w(W, p + "w1"),
               _w(W, p + "b1"))
    x2 = x1 + linear(gelu(h), _w(W, p + "w2"), _w(W, p + "b2"))
    if trace is not None:
        trace.append(dict(x=x, u=u, q=q, k=k, v=v, o=o, probs=probs, x1=x1, h=h, x2=x2))
    return np.where(upd[..., None], x2, x)


def decode_logits(z, wd, bd, p):
    """ConvTranspose2d(C -> 3, kernel p, stride p, no padding), wd stored IOHW [C, 3, p, p]:
    y[b, t, p*i+ky, p*j+kx, ch] = bd[ch] + sum_c z[b,t,i,j,c] * wd[c,ch,ky,kx]."""
    y = np.einsum("btijc,cdyx->btiyjxd", z, np.asarray(wd, F64)) + np.asarray(bd, F64)
    B, T, Ht, _, Wt, _, _ = y.shape
    return y.reshape(B, T, Ht * p, Wt * p, 3)


def composite(frames, masks, pred):
    """out = pred where the mask is nonzero, else the input pixel itself (a select, so every
    pixel outside the mask is the input bit for bit)."""
    return np.where(masks[..., None] != 0, pred, frames.astype(F64))


def forward_detail(frames, masks, W, cfg, query_set="masked", keep_blocks=False):
    """Run the whole clip-mode forward; returns a dict of the intermediate results (with the
    per-block tensors under "blocks" when ``keep_blocks``)."""
    check_shape(frames, masks, cfg)
    p = cfg.patch
    ovl = getattr(cfg, "overlap", False)
    xc = cut_out(frames, masks)
    flags = token_flags_overlap(masks, p) if ovl else token_flags(masks, p)
    upd = flags if query_set == "masked" else np.ones_like(flags)
    x0 = (patch_embed_overlap if ovl else patch_embed)(xc, W["embed.w"], W["embed.b"], p)
    x = x0
    trace = [] if keep_blocks else None
    for l in range(cfg.blocks):
        x = block(x, upd, W, l, cfg, trace)
    z = layer_norm(x, _w(W, "lnf.g"), _w(W, "lnf.b"))
    pred = sigmoid((decode_logits_fold if ovl else decode_logits)(z, W["dec.w"], W["dec.b"], p))
    out = composite(frames, masks, pred)
    return dict(xc=xc, flags=flags, upd=upd, x0=x0, x=x, z=z, pred=pred, out=out,
                blocks=trace)


def forward(frames, masks, W, cfg, query_set="masked"):
    """Inpainted frames [B, T, H, W, 3] in FP64."""
    return forward_detail(frames, masks, W, cfg, query_set)["out"]


# --------------------------------------------------------------------------------------------
# Integer outputs of the token gather, in window-major token order
# --------------------------------------------------------------------------------------------

def window_major_flags(masks, cfg):
    """Token flags listed in window-major order: windows in (b, a, u, v) order, tokens inside
    a window in (dt, di, dj) order.  Returns uint8 [num_windows * S]."""
    tf = token_flags_overlap if getattr(cfg, "overlap", False) else token_flags
    f = tf(masks, cfg.patch)[..., None].astype(np.uint8)
    fw = to_windows(f, cfg)
    return fw.reshape(-1).copy()


def gather_lists(masks, cfg, query_set="masked"):
    """(flag u8 [N], idx int32 [Nq], woff int32 [num_windows + 1]).

    ``idx`` lists the flagged tokens (window-major index) in ascending order; ``woff[w]`` is
    the number of flagged tokens in windows before w, so window w's queries are
    idx[woff[w]:woff[w+1]]."""
    flag = window_major_flags(masks, cfg)
    if query_set != "masked":
        flag = np.ones_like(flag)
    S = cfg.window_tokens
    idx = np.flatnonzero(flag).astype(np.int32)
    per_win = flag.reshape(-1, S).sum(axis=1)
    woff = np.concatenate([[0], np.cumsum(per_win)]).astype(np.int32)
    return flag, idx, woff
