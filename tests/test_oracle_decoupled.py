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


def test_gradient_rejects_decoupled_attention():
    """The reverse pass partitions every block into joint windows: a decoupled configuration
    must raise rather than silently return the joint network's gradient."""
    import pytest

    from oracle import grad as og
    rng = np.random.default_rng(0)
    cfg = BASE
    W = drsynth.make_weights(cfg, 0)
    frames = rng.random((1, cfg.win_t, 8, 12, 3))
    masks = (rng.random((1, cfg.win_t, 8, 12)) < 0.3).astype(np.uint8)
    with pytest.raises(NotImplementedError):
        og.loss_and_grad(frames, masks, W, cfg)


# ------------------------------------------------------------------------------------------
# stream mode with the decoupled pattern
# ------------------------------------------------------------------------------------------
def _stream_frames(seed, T, H=8, W=12):
    rng = np.random.default_rng(seed)
    return rng.random((T, H, W, 3)), np.zeros((T, H, W), np.uint8)


def test_stream_decoupled_equals_clip_mode_when_past_frames_are_unmasked():
    """Past frames without private pixels are never updated in either mode, so their keys and
    values are the same; the newest frame's spatial blocks see its own frame and its temporal
    blocks its position in every frame, in both modes."""
    from oracle import stream as ost
    cfg = BASE
    W = drsynth.make_weights(cfg, 1, std=0.2)
    f, m = _stream_frames(2, cfg.win_t)
    m[-1, 1:7, 2:10] = 1
    outs = ost.run_stream(f, m, W, cfg)
    clip = on.forward(f[None], m[None], W, cfg)[0]
    np.testing.assert_allclose(outs[-1], clip[-1], rtol=1e-12, atol=1e-13)
    assert not np.allclose(outs[-1], ost.run_stream(f, m, W, dataclasses.replace(cfg, attn="joint"))[-1])


def test_stream_decoupled_identical_frames_equal_clip_mode():
    """A stream of identical frames (and masks) gives the clip-mode result of a clip of those
    frames: every frame's activations agree at every block in both modes, so a temporal block
    averages identical values either way."""
    from oracle import stream as ost
    cfg = BASE
    W = drsynth.make_weights(cfg, 2, std=0.2)
    f1, m1 = _stream_frames(3, 1)
    m1[0, 2:6, 1:9] = 1
    f = np.repeat(f1, cfg.win_t, axis=0)
    m = np.repeat(m1, cfg.win_t, axis=0)
    outs = ost.run_stream(f, m, W, cfg)
    clip = on.forward(f[None], m[None], W, cfg)[0]
    for t in range(cfg.win_t):
        np.testing.assert_allclose(outs[t], clip[t], rtol=1e-11, atol=1e-12)


def test_stream_decoupled_spatial_blocks_ignore_the_cache_and_history_is_bounded():
    """With one block (spatial only) the stream is per-frame; with two, a frame older than
    the memory slots no longer matters."""
    from oracle import stream as ost
    one = dataclasses.replace(BASE, blocks=1)
    W1 = drsynth.make_weights(one, 3, std=0.2)
    f, m = _stream_frames(4, 3)
    m[:, 2:6, 1:9] = 1
    f2 = f.copy()
    f2[0] = 0.3
    assert np.array_equal(ost.run_stream(f, m, W1, one)[-1], ost.run_stream(f2, m, W1, one)[-1])
    W = drsynth.make_weights(BASE, 3, std=0.2)
    a = ost.run_stream(f, m, W, BASE, slots=1)
    b = ost.run_stream(f2, m, W, BASE, slots=1)
    assert np.array_equal(a[-1], b[-1])   # frame 0 dropped by frame 2 (one memory slot)
    assert not np.array_equal(ost.run_stream(f, m, W, BASE, slots=2)[-1], ost.run_stream(f2, m, W, BASE, slots=2)[-1])


def test_stream_decoupled_planted_mistake_is_caught():
    """A temporal block that forgot the cache (attending to the new frame only) breaks the
    unmasked-history equivalence above."""
    from oracle import stream as ost
    cfg = BASE
    W = drsynth.make_weights(cfg, 1, std=0.2)
    f, m = _stream_frames(5, cfg.win_t)
    m[-1, 1:7, 2:10] = 1
    clip = on.forward(f[None], m[None], W, cfg)[0]
    orig = on.block_attention_kind
    try:
        # temporal blocks computed as spatial ones without the cache
        on.block_attention_kind = lambda l, c: "spatial" if orig(l, c) == "temporal" else orig(l, c)
        bad = ost.run_stream(f, m, W, cfg)
    finally:
        on.block_attention_kind = orig
    assert not np.allclose(bad[-1], clip[-1], atol=1e-6)
