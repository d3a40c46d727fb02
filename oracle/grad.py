"""Training loss and its analytic gradient, FP64, by hand (reverse mode) -- test infrastructure.

Loss (thesis, Methods, "Model Training -- Loss": per-pixel L1 against the ground truth on the
masked region and on the rest, weighted towards the masked region).  Reading taken: weights
1 and 0.1, means over pixel-channel elements of each region, an empty region contributes 0,
and the loss is taken on the network prediction before the composite (after the composite
the unmasked pixels equal the ground truth and would carry no gradient):

    L = mean_{m != 0} |pred - gt| + 0.1 * mean_{m == 0} |pred - gt|,   d|e|/de := sign(e), sign(0) = 0

``gt`` is the uncut input frame.  Gradients are returned for every parameter (same names and
shapes as the weights).  The pass recomputes the attention probabilities from Q and K
rather than storing them.

Pins: central finite differences in FP64 over random parameter directions, and torch FP64
autograd of the independent reference implementation (tests only).
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf

from . import network as on

F64 = np.float64


def l1_loss(pred, gt, masks, w_in=1.0, w_out=0.1):
    """(L, dL/dpred)."""
    inside = np.repeat(masks[..., None] != 0, 3, axis=-1)
    e = pred - np.asarray(gt, F64)
    n_in, n_out = int(inside.sum()), int((~inside).sum())
    L = 0.0
    g = np.zeros_like(e)
    if n_in:
        L += w_in * np.abs(e[inside]).sum() / n_in
        g[inside] = w_in * np.sign(e[inside]) / n_in
    if n_out:
        L += w_out * np.abs(e[~inside]).sum() / n_out
        g[~inside] = w_out * np.sign(e[~inside]) / n_out
    return L, g


def _ln_backward(x, g, dy, eps=on.LN_EPS):
    """LayerNorm over the last axis: returns (dx, dgamma, dbeta)."""
    mu = x.mean(-1, keepdims=True)
    var = ((x - mu) ** 2).mean(-1, keepdims=True)
    r = 1.0 / np.sqrt(var + eps)
    xh = (x - mu) * r
    red = tuple(range(x.ndim - 1))
    dgam = (dy * xh).sum(axis=red)
    dbet = dy.sum(axis=red)
    dxh = dy * g
    dx = r * (dxh - dxh.mean(-1, keepdims=True) - xh * (dxh * xh).mean(-1, keepdims=True))
    return dx, dgam, dbet


def _linear_backward(x, w, dy):
    """y = x w^T + b: returns (dx, dw, db)."""
    C_in = x.shape[-1]
    x2 = x.reshape(-1, C_in)
    d2 = dy.reshape(-1, dy.shape[-1])
    return dy @ w, d2.T @ x2, d2.sum(axis=0)


def _gelu_grad(z):
    return 0.5 * (1.0 + erf(z / np.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / np.sqrt(2.0 * np.pi)


def _attention_backward(q, k, v, do, heads):
    """Per window: P = softmax(Q K^T / sqrt(dh)) recomputed, O = P V.
    dV = P^T dO,  dP = dO V^T,  dS = P * (dP - rowsum(dO * O)),  dQ = dS K / sqrt(dh),
    dK = dS^T Q / sqrt(dh).  Arrays are [..., S, C] with heads as channel slices."""
    lead = q.shape[:-2]
    S, C = q.shape[-2:]
    dh = C // heads
    nw = int(np.prod(lead)) if lead else 1

    def split(a):
        return a.reshape(nw, S, heads, dh).transpose(0, 2, 1, 3)

    qf, kf, vf, dof = split(q), split(k), split(v), split(do)
    sc = 1.0 / np.sqrt(dh)
    p = on.softmax(qf @ kf.transpose(0, 1, 3, 2) * sc)
    o = p @ vf
    dv = p.transpose(0, 1, 3, 2) @ dof
    dp = dof @ vf.transpose(0, 1, 3, 2)
    ds = p * (dp - (dof * o).sum(-1, keepdims=True))
    dq = ds @ kf * sc
    dk = ds.transpose(0, 1, 3, 2) @ qf * sc

    def merge(a):
        return a.transpose(0, 2, 1, 3).reshape(*lead, S, C)

    return merge(dq), merge(dk), merge(dv)


def loss_and_grad(frames, masks, W, cfg, query_set="masked", w_in=1.0, w_out=0.1):
    """(L, {name: dL/dname}) for the clip-mode forward on ``frames`` (also the ground truth)."""
    if getattr(cfg, "overlap", False):
        raise NotImplementedError("the overlapping embedding/decoder runs in clip mode only")
    if getattr(cfg, "attn", "joint") != "joint":
        # the reverse pass below partitions every block into joint windows
        raise NotImplementedError("the gradient covers joint window attention only")
    d = on.forward_detail(frames, masks, W, cfg, query_set, keep_blocks=True)
    L, dpred = l1_loss(d["pred"], frames, masks, w_in, w_out)
    G = {}
    p = cfg.patch
    pred = d["pred"]
    # decoder: pred = sigmoid(y), y[b,t,p*i+ky,p*j+kx,ch] = bd[ch] + sum_c z[b,t,i,j,c] Wd[c,ch,ky,kx]
    dy = dpred * pred * (1.0 - pred)
    B, T, H, Wd, _ = dy.shape
    dy7 = dy.reshape(B, T, H // p, p, Wd // p, p, 3)            # b t i ky j kx ch
    wd = np.asarray(W["dec.w"], F64)
    z = d["z"]
    dz = np.einsum("btiyjxd,cdyx->btijc", dy7, wd)
    G["dec.w"] = np.einsum("btijc,btiyjxd->cdyx", z, dy7)
    G["dec.b"] = dy7.sum(axis=(0, 1, 2, 3, 4, 5))
    dx, G["lnf.g"], G["lnf.b"] = _ln_backward(d["x"], np.asarray(W["lnf.g"], F64), dz)

    upd = d["upd"][..., None].astype(F64)
    for l in reversed(range(cfg.blocks)):
        t = d["blocks"][l]
        pre = f"blk{l}."
        w = lambda n: np.asarray(W[pre + n], F64)  # noqa: E731
        dx2 = dx * upd
        dx_in = dx * (1.0 - upd)
        # x2 = x1 + W2 gelu(W1 LN2(x1) + b1) + b2
        a = on.gelu(t["h"])
        da, G[pre + "w2"], G[pre + "b2"] = _linear_backward(a, w("w2"), dx2)
        dh = da * _gelu_grad(t["h"])
        n2 = on.layer_norm(t["x1"], w("ln2.g"), w("ln2.b"))
        dn2, G[pre + "w1"], G[pre + "b1"] = _linear_backward(n2, w("w1"), dh)
        dx1_ln, G[pre + "ln2.g"], G[pre + "ln2.b"] = _ln_backward(t["x1"], w("ln2.g"), dn2)
        dx1 = dx2 + dx1_ln
        # x1 = x + Wo O + bo
        do, G[pre + "wo"], G[pre + "bo"] = _linear_backward(t["o"], w("wo"), dx1)
        dx_in = dx_in + dx1
        dq_w, dk_w, dv_w = _attention_backward(on.to_windows(t["q"], cfg), on.to_windows(t["k"], cfg),
                                               on.to_windows(t["v"], cfg), on.to_windows(do, cfg), cfg.heads)
        dq, dk, dv = (on.from_windows(a_, cfg) for a_ in (dq_w, dk_w, dv_w))
        du = np.zeros_like(t["u"])
        for name, dd in (("q", dq), ("k", dk), ("v", dv)):
            dui, G[pre + "w" + name], G[pre + "b" + name] = _linear_backward(t["u"], w("w" + name), dd)
            du += dui
        dxl, G[pre + "ln1.g"], G[pre + "ln1.b"] = _ln_backward(t["x"], w("ln1.g"), du)
        dx = dx_in + dxl
    # patch embedding: x0[b,t,i,j,o] = be[o] + sum We[o,c,ky,kx] xc[b,t,p*i+ky,p*j+kx,c]
    xc = d["xc"]
    patches = xc.reshape(B, T, H // p, p, Wd // p, p, 3)
    G["embed.w"] = np.einsum("btijo,btiyjxc->ocyx", dx, patches)
    G["embed.b"] = dx.sum(axis=(0, 1, 2, 3))
    return L, {k: G[k] for k in W}


def loss(frames, masks, W, cfg, query_set="masked", w_in=1.0, w_out=0.1):
    pred = on.forward_detail(frames, masks, W, cfg, query_set)["pred"]
    return l1_loss(pred, frames, masks, w_in, w_out)[0]
