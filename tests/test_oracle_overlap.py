"""Pins of the oracle's overlapping patch embedding and fold decoder (kernel 2p, stride p,
padding p/2) against torch's conv2d / conv_transpose2d, a per-pixel reduction over the
covering tokens written out by hand, brute-force flags, and the pinned non-overlapping
network as a special case.  CPU only."""
import dataclasses

import numpy as np
import pytest

import drsynth
from oracle import network as on

torch = pytest.importorskip("torch")
F = torch.nn.functional

CFG = drsynth.NetCfg(dim=16, heads=2, blocks=2, mlp_ratio=2, patch=4, win_h=2, win_w=3, win_t=2, overlap=True)


def test_embed_matches_conv2d():
    rng = np.random.default_rng(0)
    xc = rng.random((1, 2, 16, 24, 3))
    w = rng.standard_normal((7, 3, 8, 8))
    b = rng.standard_normal(7)
    x = on.patch_embed_overlap(xc, w, b, 4)
    ref = F.conv2d(torch.from_numpy(xc[0]).permute(0, 3, 1, 2), torch.from_numpy(w), torch.from_numpy(b),
                   stride=4, padding=2).permute(0, 2, 3, 1).numpy()
    assert x.shape == (1, 2, 4, 6, 7)
    np.testing.assert_allclose(x[0], ref, rtol=1e-12, atol=1e-12)


def test_embed_corner_brute_force():
    """Token (0, 0) reads rows and columns -2 .. 5: the padding contributes nothing."""
    rng = np.random.default_rng(1)
    xc = rng.random((1, 1, 8, 8, 3))
    w = rng.standard_normal((2, 3, 8, 8))
    b = np.zeros(2)
    x = on.patch_embed_overlap(xc, w, b, 4)
    for (i, j) in [(0, 0), (1, 1), (0, 1)]:
        acc = 0.0
        for c in range(3):
            for ky in range(8):
                for kx in range(8):
                    y, xx = 4 * i - 2 + ky, 4 * j - 2 + kx
                    if 0 <= y < 8 and 0 <= xx < 8:
                        acc += w[1, c, ky, kx] * xc[0, 0, y, xx, c]
        assert abs(acc - x[0, 0, i, j, 1]) < 1e-12


def test_fold_matches_conv_transpose2d():
    rng = np.random.default_rng(2)
    z = rng.standard_normal((1, 2, 4, 6, 5))
    wd = rng.standard_normal((5, 3, 8, 8))
    bd = rng.standard_normal(3)
    y = on.decode_logits_fold(z, wd, bd, 4)
    ref = F.conv_transpose2d(torch.from_numpy(z[0]).permute(0, 3, 1, 2), torch.from_numpy(wd), torch.from_numpy(bd),
                             stride=4, padding=2).permute(0, 2, 3, 1).numpy()
    assert y.shape == (1, 2, 16, 24, 3)
    np.testing.assert_allclose(y[0], ref, rtol=1e-12, atol=1e-12)


def test_fold_equals_reduction_over_covering_tokens():
    """The reduction form: pixel (y, x) sums the logit contributions of the tokens whose
    2p x 2p footprint covers it (at most 2 x 2), at kernel offset (y + p/2 - p i, ...)."""
    rng = np.random.default_rng(3)
    Ht, Wt, C, p = 3, 4, 5, 4
    z = rng.standard_normal((1, 1, Ht, Wt, C))
    wd = rng.standard_normal((C, 3, 8, 8))
    bd = rng.standard_normal(3)
    y = on.decode_logits_fold(z, wd, bd, p)
    for py in range(p * Ht):
        for px in range(p * Wt):
            acc = bd.copy()
            n_tok = 0
            for i in range(Ht):
                for j in range(Wt):
                    ky, kx = py + 2 - p * i, px + 2 - p * j
                    if 0 <= ky < 8 and 0 <= kx < 8:
                        acc += z[0, 0, i, j] @ wd[:, :, ky, kx]
                        n_tok += 1
            assert n_tok in (1, 2, 4)
            np.testing.assert_allclose(y[0, 0, py, px], acc, rtol=1e-12, atol=1e-12)


def test_overlap_flags_brute_force_and_cover():
    rng = np.random.default_rng(4)
    m = (rng.random((1, 2, 16, 24)) < 0.03).astype(np.uint8)
    fl = on.token_flags_overlap(m, 4)
    for t in range(2):
        for i in range(4):
            for j in range(6):
                y0, y1 = max(0, 4 * i - 2), min(16, 4 * i + 6)
                x0, x1 = max(0, 4 * j - 2), min(24, 4 * j + 6)
                assert fl[0, t, i, j] == bool(m[0, t, y0:y1, x0:x1].any())
    # every token a private pixel's logit sums over is a query
    for t, py, px in zip(*np.nonzero(m[0])):
        for i in range(4):
            for j in range(6):
                if 0 <= py + 2 - 4 * i < 8 and 0 <= px + 2 - 4 * j < 8:
                    assert fl[0, t, i, j]
    assert np.all(fl >= on.token_flags(m, 4))


def _center_weights(Wp, cfg_ovl, seed):
    """Kernel-2p weights that are zero outside the central p x p taps and equal ``Wp``'s
    kernel-p weights there; every other tensor shared."""
    W = dict(Wp)
    for name in ("embed.w", "dec.w"):
        k = np.zeros(Wp[name].shape[:2] + (8, 8), np.float32)
        k[:, :, 2:6, 2:6] = Wp[name]
        W[name] = k
    return W


def test_center_only_kernels_reduce_to_the_plain_network():
    """With taps only at the central p x p of the 2p kernel, the overlapping network is the
    non-overlapping one: the embedding reads exactly the token's own patch and each pixel's
    logit comes from its own token alone.  (Every token a query: in masked mode the wider
    flag rule updates more tokens, which then feed later blocks as keys and values.)"""
    plain = dataclasses.replace(CFG, overlap=False)
    Wp = drsynth.make_weights(plain, 5)
    Wo = _center_weights(Wp, CFG, 5)
    f, m = drsynth.make_clip_batch([0], 2, 16, 24)
    a = on.forward(f, m, Wo, CFG, "all")
    b = on.forward(f, m, Wp, plain, "all")
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-12)


def test_center_only_kernels_masked_mode_matches_plain_blocks_on_the_wider_query_set():
    """Masked mode with centre-only kernels: the plain network's steps run on the overlap
    flag set give the same picture."""
    plain = dataclasses.replace(CFG, overlap=False)
    Wp = drsynth.make_weights(plain, 7)
    Wo = _center_weights(Wp, CFG, 7)
    f, m = drsynth.make_clip_batch([3], 2, 16, 24)
    a = on.forward(f, m, Wo, CFG, "masked")
    upd = on.token_flags_overlap(m, 4)
    x = on.patch_embed(on.cut_out(f, m), Wp["embed.w"], Wp["embed.b"], 4)
    for l in range(plain.blocks):
        x = on.block(x, upd, Wp, l, plain)
    z = on.layer_norm(x, np.float64(Wp["lnf.g"]), np.float64(Wp["lnf.b"]))
    b = on.composite(f, m, on.sigmoid(on.decode_logits(z, Wp["dec.w"], Wp["dec.b"], 4)))
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-12)


def test_overlap_network_differs_and_keeps_outside_pixels():
    Wo = drsynth.make_weights(CFG, 6)
    f, m = drsynth.make_clip_batch([1], 2, 16, 24)
    out = on.forward(f, m, Wo, CFG)
    inside = np.repeat(m[..., None] != 0, 3, axis=-1)
    assert np.array_equal(out[~inside], f[~inside].astype(np.float64))
    plain = dataclasses.replace(CFG, overlap=False)
    Wp = drsynth.make_weights(plain, 6)
    assert np.abs(out - on.forward(f, m, Wp, plain))[inside].max() > 1e-4


def test_gather_lists_use_the_overlap_rule():
    f, m = drsynth.make_clip_batch([2], 2, 16, 24)
    flag, idx, woff = on.gather_lists(m, CFG)
    ref = on.to_windows(on.token_flags_overlap(m, 4)[..., None].astype(np.uint8), CFG).reshape(-1)
    assert np.array_equal(flag, ref)
    assert woff[-1] == idx.size == int(ref.sum())


# ------------------------------------------------------------------------------------------
# the pins above have teeth: plausible mistakes planted in the oracle are caught
# ------------------------------------------------------------------------------------------
_orig_fold = on.decode_logits_fold
_orig_embed = on.patch_embed_overlap
_orig_flags = on.token_flags_overlap


def _fold_crop_shifted(z, wd, bd, p):
    y = _orig_fold(z, wd, bd, p) - np.asarray(bd)
    y = np.roll(y, 1, axis=2)  # crop taken one row too early
    return y + np.asarray(bd)


def _fold_kernel_transposed(z, wd, bd, p):
    return _orig_fold(z, np.asarray(wd).transpose(0, 1, 3, 2), bd, p)


def _embed_pad_one_side(xc, w, b, p):
    pad = np.zeros_like(xc)
    pad[:, :, :-2] = xc[:, :, 2:]  # the frame shifted up by the padding
    return _orig_embed(pad, w, b, p)


def _flags_no_halo(masks, p):
    return on.token_flags(masks, p)


_OVL_MUTATIONS = {
    "fold crop shifted": ("decode_logits_fold", _fold_crop_shifted, test_fold_matches_conv_transpose2d),
    "fold kernel transposed": ("decode_logits_fold", _fold_kernel_transposed,
                               test_fold_equals_reduction_over_covering_tokens),
    "embedding padding on one side": ("patch_embed_overlap", _embed_pad_one_side, test_embed_matches_conv2d),
    "flags without the footprint halo": ("token_flags_overlap", _flags_no_halo, test_overlap_flags_brute_force_and_cover),
}


@pytest.mark.parametrize("name", sorted(_OVL_MUTATIONS))
def test_planted_overlap_mistake_is_caught(name, monkeypatch):
    attr, fn, pin = _OVL_MUTATIONS[name]
    monkeypatch.setattr(on, attr, fn)
    with pytest.raises(AssertionError):
        pin()
