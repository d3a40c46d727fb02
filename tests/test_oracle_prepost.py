"""Pins of the pre/post-processing oracle against library routines, brute force and closed
forms.  CPU only."""
import numpy as np
import pytest
import torch
import torch.nn.functional as F
from scipy.ndimage import maximum_filter

from oracle import prepost as pp


def _rng(seed):
    return np.random.default_rng(seed)


def test_bgra_channel_order_and_scale():
    bgra = np.zeros((2, 3, 4), np.uint8)
    bgra[..., 0] = 10   # B
    bgra[..., 1] = 20   # G
    bgra[..., 2] = 255  # R
    bgra[..., 3] = 7    # alpha is ignored
    rgb = pp.bgra_to_rgb(bgra)
    assert np.allclose(rgb[..., 0], 1.0) and np.allclose(rgb[..., 1], 20 / 255) and np.allclose(rgb[..., 2], 10 / 255)


def test_union_respects_selection():
    inst = np.zeros((3, 4, 5), np.uint8)
    inst[0, 0, 0] = 3
    inst[1, 1, 1] = 1
    inst[2, 2, 2] = 255
    u = pp.mask_union(inst, [True, False, True])
    assert u[0, 0] == 1 and u[1, 1] == 0 and u[2, 2] == 1 and u.sum() == 2


@pytest.mark.parametrize("r", [0, 1, 3, 7])
def test_dilation_matches_scipy_max_filter(r):
    m = (_rng(r).random((23, 31)) < 0.05).astype(np.uint8)
    ref = maximum_filter(m, size=2 * r + 1, mode="constant", cval=0)
    assert np.array_equal(pp.dilate(m, r), ref)


def test_dilation_of_corner_pixel_is_clipped_square():
    m = np.zeros((10, 12), np.uint8)
    m[0, 11] = 1
    d = pp.dilate(m, 2)
    assert d.sum() == 3 * 3 and d[:3, 9:].all()


def test_downscale_matches_torch_avg_pool():
    rgb = _rng(1).random((8, 12, 3))
    ref = F.avg_pool2d(torch.from_numpy(rgb).permute(2, 0, 1)[None], 2)[0].permute(1, 2, 0).numpy()
    assert np.allclose(pp.downscale2(rgb), ref, rtol=0, atol=1e-15)


def test_mask_downscale_matches_torch_max_pool():
    m = (_rng(2).random((8, 12)) < 0.2).astype(np.uint8)
    ref = F.max_pool2d(torch.from_numpy(m.astype(np.float32))[None, None], 2)[0, 0].numpy().astype(np.uint8)
    assert np.array_equal(pp.downscale2_mask(m), ref)


def test_upscale_matches_torch_nearest():
    img = _rng(3).random((5, 7, 3))
    ref = F.interpolate(torch.from_numpy(img).permute(2, 0, 1)[None], scale_factor=2, mode="nearest")[0].permute(1, 2, 0).numpy()
    assert np.array_equal(pp.upscale2(img), ref)


def test_u8_round_trip_and_clamp():
    u = np.arange(256, dtype=np.uint8)
    assert np.array_equal(pp.to_u8((u.astype(np.float32) / np.float32(255.0))), u)
    assert pp.to_u8(np.array([-0.5, 1.5], np.float32)).tolist() == [0, 255]
    # half-way cases round to even: 255 * v = 0.5 -> 0, 1.5 -> 2
    v = np.array([0.5, 1.5], np.float32) / np.float32(255.0)
    assert np.float32(255.0) * v[0] == np.float32(0.5) and pp.to_u8(v[:1]).tolist() == [0]


def test_post_copies_unmasked_pixels_bit_exactly_and_writes_masked():
    rng = _rng(4)
    bgra = rng.integers(0, 256, (6, 8, 4), dtype=np.uint8)
    pred = rng.random((3, 4, 3)).astype(np.float32)
    mask = np.zeros((6, 8), np.uint8)
    mask[2:4, 4:8] = 1
    out = pp.post(bgra, pred, mask)
    assert np.array_equal(out[mask == 0], bgra[mask == 0])
    assert np.array_equal(out[..., 3], bgra[..., 3])
    # pixel (3, 5) takes low-res (1, 2), RGB -> BGR
    exp = pp.to_u8(pred[1, 2])
    assert out[3, 5, 0] == exp[2] and out[3, 5, 1] == exp[1] and out[3, 5, 2] == exp[0]


def test_prep_then_post_of_unmasked_frame_is_identity():
    rng = _rng(5)
    bgra = rng.integers(0, 256, (8, 10, 4), dtype=np.uint8)
    inst = np.zeros((2, 8, 10), np.uint8)
    low, mlow, mfull = pp.prep(bgra, inst, [True, True], 2)
    assert mlow.sum() == 0 and mfull.sum() == 0
    assert np.array_equal(pp.post(bgra, low.astype(np.float32), mfull), bgra)


def test_low_res_mask_covers_every_private_pixel():
    rng = _rng(6)
    inst = (rng.random((3, 12, 16)) < 0.02).astype(np.uint8)
    bgra = rng.integers(0, 256, (12, 16, 4), dtype=np.uint8)
    _, mlow, mfull = pp.prep(bgra, inst, [True, False, True], 1)
    assert np.all(pp.upscale2(mlow[..., None])[..., 0] >= mfull)
