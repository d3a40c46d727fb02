"""Pins of the stream-mode oracle: reductions to clip mode, cache eviction, causality."""
import numpy as np

import drsynth
from oracle import network as on
from oracle import stream as ost

# temporal windows of 3 frames, 2x3 tokens spatially, 16 x 24 px frames
SCFG = drsynth.NetCfg(dim=32, heads=2, blocks=2, mlp_ratio=4, patch=4, win_h=2, win_w=3, win_t=3)


def _frames(seed, T=3, H=16, W=24):
    rng = np.random.default_rng(seed)
    f = rng.random((T, H, W, 3)).astype(np.float32)
    m = np.zeros((T, H, W), np.uint8)
    return f, m


def test_single_frame_window_equals_clip_mode():
    """With win_t = 1 there is no cache: each stream step is the clip-mode forward of that frame."""
    cfg = drsynth.NETS["tiny64"]
    W = drsynth.make_weights(cfg, 0)
    frames = np.concatenate([drsynth.tiny_frame(s)[0] for s in range(3)], axis=1)[0]
    masks = np.concatenate([drsynth.tiny_frame(s)[1] for s in range(3)], axis=1)[0]
    outs = ost.run_stream(frames, masks, W, cfg)
    for t in range(3):
        ref = on.forward(frames[None, t:t + 1], masks[None, t:t + 1], W, cfg)[0, 0]
        np.testing.assert_allclose(outs[t], ref, rtol=0, atol=1e-13)


def test_last_frame_equals_clip_mode_when_past_frames_are_unmasked():
    """Past frames without private pixels are never updated in either mode, so their keys and
    values coincide, and the newest frame attends to the same window in both."""
    cfg = SCFG
    W = drsynth.make_weights(cfg, 1, std=0.2)
    f, m = _frames(2)
    m[-1, 3:11, 5:17] = 1
    outs = ost.run_stream(f, m, W, cfg)
    clip = on.forward(f[None], m[None], W, cfg)[0]
    np.testing.assert_allclose(outs[-1], clip[-1], rtol=1e-12, atol=1e-13)
    # and the same check with a later frame that is only partly masked
    m[-1] = 0
    m[-1, 0:4, 0:4] = 1
    np.testing.assert_allclose(ost.run_stream(f, m, W, cfg)[-1], on.forward(f[None], m[None], W, cfg)[0, -1],
                               rtol=1e-12, atol=1e-13)


def test_cache_keeps_only_the_last_frames():
    """A frame older than win_t - 1 steps no longer influences the output."""
    cfg = SCFG
    W = drsynth.make_weights(cfg, 1, std=0.2)
    f, m = _frames(3, T=4)
    m[-1, 3:11, 5:17] = 1
    f2 = f.copy()
    f2[0] = np.random.default_rng(9).random(f2[0].shape)
    m2 = m.copy()
    m2[0, 2:6, 2:6] = 1
    a = ost.run_stream(f, m, W, cfg)
    b = ost.run_stream(f2, m2, W, cfg)
    assert np.array_equal(a[-1], b[-1])
    assert not np.array_equal(a[0], b[0])


def test_stream_is_causal_and_differs_from_clip_mode():
    cfg = SCFG
    W = drsynth.make_weights(cfg, 1, std=0.2)
    f, m = _frames(4)
    m[:, 3:11, 5:17] = 1
    outs = ost.run_stream(f, m, W, cfg)
    # causal: the first frame's output does not depend on later frames
    f2 = f.copy()
    f2[1:] = 0.5
    assert np.array_equal(ost.run_stream(f2, m, W, cfg)[0], outs[0])
    # masked past frames are updated in clip mode, so the two modes differ in general
    clip = on.forward(f[None], m[None], W, cfg)[0]
    assert not np.allclose(outs[-1], clip[-1], atol=1e-6)
    # outside the mask the input is returned bit for bit
    assert np.array_equal(outs[:, :, :][m == 0], f[m == 0].astype(np.float64))


def test_memory_slots_bound_the_history():
    """With m memory slots, frames older than m steps no longer matter; m = 0 is per-frame."""
    cfg = SCFG
    W = drsynth.make_weights(cfg, 1, std=0.2)
    f, m = _frames(5, T=3)
    m[-1, 3:11, 5:17] = 1
    f2 = f.copy()
    f2[0] = 0.25
    a = ost.run_stream(f, m, W, cfg, slots=1)
    b = ost.run_stream(f2, m, W, cfg, slots=1)
    assert np.array_equal(a[-1], b[-1])  # frame 0 dropped by frame 2
    c = ost.run_stream(f2, m, W, cfg, slots=2)
    assert not np.array_equal(a[-1], c[-1])
    single = drsynth.NetCfg(**{**SCFG.__dict__, "win_t": 1})
    z = ost.run_stream(f, m, W, cfg, slots=0)[-1]
    ref = on.forward(f[None, -1:], m[None, -1:], W, single)[0, 0]
    np.testing.assert_allclose(z, ref, rtol=0, atol=1e-13)
