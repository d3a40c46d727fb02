"""Pins of the oracle's decoupled (spatial / temporal) attention against closed forms, the
pinned joint attention and brute force.  CPU only."""
import dataclasses

import numpy as np

import drsynth
from oracle import network as on

BASE = drsynth.NetCfg(dim=16, heads=2, blocks=2, mlp_ratio=2, patch=4, win_h=2, win_w=3, win_t=3,
                      attn="decoupled")


def _qkv(seed, B=1, T=3, Ht=4, Wt=6, C=16):
    rng = np.random.default_rng(seed)
    return [rng.standard_normal((B, T, Ht, Wt, C)) for _ in range(3)]


def _attend(kind, q, k, v, cfg):
    to, back = {"spatial": (on.to_frame_windows, on.from_frame_windows),
                "temporal": (on.to_time_windows, on.from_time_windows),
                "joint": (on.to_windows, on.from_windows)}[kind]
    o, _ = on.multi_head_attention(to(q, cfg), to(k, cfg), to(v, cfg), cfg.heads)
    return back(o, cfg)


def test_block_kinds_alternate():
    assert [on.block_attention_kind(l, BASE) for l in range(4)] == ["spatial", "temporal", "spatial", "temporal"]
    assert on.block_attention_kind(1, dataclasses.replace(BASE, attn="joint")) == "joint"


def test_temporal_over_one_frame_returns_v():
    cfg = dataclasses.replace(BASE, win_t=1)
    q, k, v = _qkv(0, T=1)
    assert np.array_equal(_attend("temporal", q, k, v, cfg), v)


def test_spatial_over_one_frame_equals_joint():
    cfg = dataclasses.replace(BASE, win_t=1)
    q, k, v = _qkv(1, T=1)
    assert np.array_equal(_attend("spatial", q, k, v, cfg), _attend("joint", q, k, v, cfg))


def test_spatial_equals_joint_attention_run_per_frame():
    q, k, v = _qkv(2)
    one = dataclasses.replace(BASE, win_t=1)
    got = _attend("spatial", q, k, v, BASE)
    for t in range(q.shape[1]):
        ref = _attend("joint", q[:, t:t + 1], k[:, t:t + 1], v[:, t:t + 1], one)
        np.testing.assert_allclose(got[:, t:t + 1], ref, rtol=0, atol=1e-13)


def test_temporal_brute_force():
    q, k, v = _qkv(3)
    got = _attend("temporal", q, k, v, BASE)
    B, T, Ht, Wt, C = q.shape
    dh = C // BASE.heads
    wt = BASE.win_t
    for b in range(B):
        for t in range(T):
            a0 = (t // wt) * wt
            for i in range(Ht):
                for j in range(Wt):
                    for h in range(BASE.heads):
                        sl = slice(h * dh, (h + 1) * dh)
                        s = [q[b, t, i, j, sl] @ k[b, a0 + u, i, j, sl] / np.sqrt(dh) for u in range(wt)]
                        e = np.exp(np.array(s) - max(s))
                        p = e / e.sum()
                        ref = sum(p[u] * v[b, a0 + u, i, j, sl] for u in range(wt))
                        np.testing.assert_allclose(got[b, t, i, j, sl], ref, rtol=0, atol=1e-13)


def test_decoupled_equals_masked_joint_window():
    """Both kinds are joint-window attention with the keys outside the query's frame
    (spatial) or outside its token position (temporal) removed."""
    q, k, v = _qkv(4)
    cfg = BASE
    qw, kw, vw = (on.to_windows(a, cfg) for a in (q, k, v))
    S = qw.shape[-2]
    A = cfg.win_h * cfg.win_w
    s = np.arange(S)
    dh = cfg.dim // cfg.heads
    for kind, same in (("spatial", s[:, None] // A == s[None, :] // A),
                       ("temporal", s[:, None] % A == s[None, :] % A)):
        out = np.empty_like(qw)
        for h in range(cfg.heads):
            sl = slice(h * dh, (h + 1) * dh)
            sc = qw[..., sl] @ np.swapaxes(kw[..., sl], -1, -2) / np.sqrt(dh)
            sc = np.where(same, sc, -np.inf)
            out[..., sl] = on.softmax(sc) @ vw[..., sl]
        np.testing.assert_allclose(_attend(kind, q, k, v, cfg), on.from_windows(out, cfg), rtol=0, atol=1e-13)


def test_decoupled_forward_keeps_the_composite_and_differs_from_joint():
    cfg = BASE
    rng = np.random.default_rng(5)
    frames = rng.random((1, 3, 16, 24, 3)).astype(np.float32)
    masks = np.zeros((1, 3, 16, 24), np.uint8)
    masks[0, :, 4:10, 6:15] = 1
    W = drsynth.make_weights(cfg, 0)
    out = on.forward(frames, masks, W, cfg)
    assert np.array_equal(out[masks == 0], frames[masks == 0].astype(np.float64))
    joint = on.forward(frames, masks, W, dataclasses.replace(cfg, attn="joint"))
    assert not np.allclose(out[masks != 0], joint[masks != 0])


def test_gradient_and_stream_reject_decoupled_attention():
    """The reverse pass and stream mode partition every block into joint windows: a decoupled
    configuration must raise rather than silently return the joint network's result."""
    import pytest

    from oracle import grad as og
    from oracle import stream as ost
    rng = np.random.default_rng(0)
    cfg = BASE
    W = drsynth.make_weights(cfg, 0)
    frames = rng.random((1, cfg.win_t, 8, 12, 3))
    masks = (rng.random((1, cfg.win_t, 8, 12)) < 0.3).astype(np.uint8)
    with pytest.raises(NotImplementedError):
        og.loss_and_grad(frames, masks, W, cfg)
    with pytest.raises(NotImplementedError):
        ost.step(ost.StreamState(cfg), frames[0, 0], masks[0, 0], W, cfg)
