"""An independent FP64 implementation of the network from torch library routines.

Used only to pin the oracle: it shares no code with it and takes a different route to
each result -- ``conv2d`` for the patch embedding, ``max_pool2d`` for the token flags,
``layer_norm``, full attention over *all* tokens of a clip with a boolean same-window mask
built from token coordinates (instead of window partitioning), ``gelu``, and
``conv_transpose2d`` for the decoder.
"""
import numpy as np
import torch
import torch.nn.functional as F


def _t(a):
    return torch.from_numpy(np.asarray(a, dtype=np.float64))


def reference_forward(frames, masks, W, cfg, query_set="masked"):
    """(out, pred, flags) as numpy arrays; W holds numpy arrays."""
    Wt = {k: _t(v) for k, v in W.items()}
    out, pred, flags = reference_forward_t(frames, masks, Wt, cfg, query_set)
    return out.detach().numpy(), pred.detach().numpy(), flags.numpy()


def reference_forward_t(frames, masks, params, cfg, query_set="masked"):
    """Same as reference_forward on torch FP64 parameter tensors (autograd-ready)."""
    W = params
    fr = _t(frames)
    m = torch.from_numpy(np.asarray(masks) != 0)
    B, T, H, Wd, _ = fr.shape
    p, C, heads = cfg.patch, cfg.dim, cfg.heads
    Ht, Wt = H // p, Wd // p
    dh = C // heads
    xc = fr.masked_fill(m[..., None], 0.0)
    img = xc.reshape(B * T, H, Wd, 3).permute(0, 3, 1, 2)
    x = F.conv2d(img, W["embed.w"], W["embed.b"], stride=p)  # [BT, C, Ht, Wt]
    x = x.permute(0, 2, 3, 1).reshape(B, T * Ht * Wt, C)
    flags = F.max_pool2d(m.reshape(B * T, 1, H, Wd).double(), p).reshape(B, T * Ht * Wt) > 0
    upd = flags if query_set == "masked" else torch.ones_like(flags)

    tt, ii, jj = torch.meshgrid(torch.arange(T), torch.arange(Ht), torch.arange(Wt), indexing="ij")
    wid = ((tt // cfg.win_t) * (Ht // cfg.win_h) + ii // cfg.win_h) * (Wt // cfg.win_w) + jj // cfg.win_w
    wid = wid.reshape(-1)
    allowed = wid[:, None] == wid[None, :]

    def heads_of(z):
        return z.reshape(B, -1, heads, dh).transpose(1, 2)

    for l in range(cfg.blocks):
        g = lambda n: W[f"blk{l}.{n}"]  # noqa: E731
        u = F.layer_norm(x, (C,), g("ln1.g"), g("ln1.b"), eps=1e-5)
        q = F.linear(u, g("wq"), g("bq"))
        k = F.linear(u, g("wk"), g("bk"))
        v = F.linear(u, g("wv"), g("bv"))
        o = F.scaled_dot_product_attention(heads_of(q), heads_of(k), heads_of(v), attn_mask=allowed)
        o = o.transpose(1, 2).reshape(B, -1, C)
        x1 = x + F.linear(o, g("wo"), g("bo"))
        hdn = F.gelu(F.linear(F.layer_norm(x1, (C,), g("ln2.g"), g("ln2.b"), eps=1e-5), g("w1"), g("b1")))
        x2 = x1 + F.linear(hdn, g("w2"), g("b2"))
        x = torch.where(upd[..., None], x2, x)

    z = F.layer_norm(x, (C,), W["lnf.g"], W["lnf.b"], eps=1e-5)
    z = z.reshape(B * T, Ht, Wt, C).permute(0, 3, 1, 2)
    pred = torch.sigmoid(F.conv_transpose2d(z, W["dec.w"], W["dec.b"], stride=p))
    pred = pred.permute(0, 2, 3, 1).reshape(B, T, H, Wd, 3)
    out = torch.where(m[..., None], pred, fr)
    return out, pred, flags.reshape(B, T, Ht, Wt)
