"""Seeded synthetic inputs: determinism, value ranges, coverage bounds."""
import numpy as np

import drsynth


def test_clip_deterministic_and_in_range():
    f1, m1, c1 = drsynth.make_clip(0, 5, 240, 432)
    f2, m2, c2 = drsynth.make_clip(0, 5, 240, 432)
    assert np.array_equal(f1, f2) and np.array_equal(m1, m2) and c1 == c2
    assert f1.dtype == np.float32 and m1.dtype == np.uint8
    assert f1.min() >= 0.0 and f1.max() <= 1.0
    assert set(np.unique(m1)) <= {0, 1}
    f3, _, _ = drsynth.make_clip(1, 5, 240, 432)
    assert not np.array_equal(f1, f3)


def test_clip_mask_coverage_reaches_target():
    for seed in range(3):
        f, m, c = drsynth.make_clip(seed, 5, 240, 432)
        assert 0.10 <= c <= 0.40
        cov = m.reshape(5, -1).mean(axis=1)
        assert np.all(cov >= c) and np.all(cov <= c + 0.25)


def test_tiny_frame_rectangle_coverage():
    f, m = drsynth.tiny_frame(0)
    assert f.shape == (1, 1, 64, 64, 3) and m.shape == (1, 1, 64, 64)
    assert abs(m.mean() - 0.15) < 0.03


def test_weights_order_and_stats():
    cfg = drsynth.NETS["clip240"]
    w = drsynth.make_weights(cfg, 0)
    assert list(w) == [n for n, _ in drsynth.weight_order(cfg)]
    assert all(a.dtype == np.float32 for a in w.values())
    assert abs(w["blk0.w1"].std() - 0.02) < 1e-3
    assert abs(w["blk3.ln2.g"].mean() - 1.0) < 1e-2
    n = sum(a.size for a in w.values())
    assert 6.2e6 < n < 6.5e6


def test_scene_masks_move_with_objects():
    sc = drsynth.Scene(5, 240, 432)
    assert not np.array_equal(sc.mask(0), sc.mask(4))
    assert np.array_equal(sc.mask(7), sc.mask(7))
