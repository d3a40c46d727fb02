"""Pins of the FP64 oracle against things other than itself: library routines, brute force,
closed forms and invariants of the method.  CPU only."""
import math

import numpy as np
import pytest
import torch
import torch.nn.functional as F

import drsynth
from oracle import network as on
from tests.torchref import reference_forward

SMALL = drsynth.NetCfg(dim=32, heads=2, blocks=2, mlp_ratio=4, patch=4, win_h=2, win_w=3, win_t=2)


def small_inputs(seed=0, B=2, T=2, H=16, W=24, cov=0.3):
    rng = np.random.default_rng(seed)
    frames = rng.random((B, T, H, W, 3)).astype(np.float32)
    masks = (rng.random((B, T, H, W)) < cov * 0.2).astype(np.uint8)
    # a solid block so some tokens are fully private, others untouched
    masks[:, :, 4:9, 5:13] = 1
    return frames, masks


# ------------------------------------------------------------------------------------------
# token flags and gather lists: brute force
# ------------------------------------------------------------------------------------------

def test_token_flags_brute_force():
    frames, masks = small_inputs(1)
    fl = on.token_flags(masks, 4)
    B, T, H, W = masks.shape
    for b in range(B):
        for t in range(T):
            for i in range(H // 4):
                for j in range(W // 4):
                    anyp = False
                    for y in range(4 * i, 4 * i + 4):
                        for x in range(4 * j, 4 * j + 4):
                            anyp = anyp or masks[b, t, y, x] != 0
                    assert fl[b, t, i, j] == anyp


def test_gather_lists_brute_force():
    frames, masks = small_inputs(2)
    cfg = SMALL
    flag, idx, woff = on.gather_lists(masks, cfg)
    B, T, H, W = masks.shape
    Ht, Wt = H // 4, W // 4
    S = cfg.window_tokens
    # enumerate windows and their tokens directly from coordinates
    expect_flag = []
    for b in range(B):
        for a in range(T // cfg.win_t):
            for u in range(Ht // cfg.win_h):
                for v in range(Wt // cfg.win_w):
                    for dt in range(cfg.win_t):
                        for di in range(cfg.win_h):
                            for dj in range(cfg.win_w):
                                t, i, j = a * cfg.win_t + dt, u * cfg.win_h + di, v * cfg.win_w + dj
                                expect_flag.append(int(masks[b, t, 4 * i:4 * i + 4, 4 * j:4 * j + 4].any()))
    assert flag.tolist() == expect_flag
    assert idx.tolist() == [n for n, f in enumerate(expect_flag) if f]
    nwin = len(expect_flag) // S
    assert woff.tolist() == [sum(expect_flag[:w * S]) for w in range(nwin + 1)]
    assert len(idx) >= math.ceil(int((masks != 0).sum()) / 16)


def test_windows_roundtrip_and_membership():
    cfg = SMALL
    x = np.arange(2 * 2 * 4 * 6, dtype=np.float64).reshape(2, 2, 4, 6, 1)
    xw = on.to_windows(x, cfg)
    assert np.array_equal(on.from_windows(xw, cfg), x)
    # window (b=1, a=0, u=1, v=1), token (dt=1, di=0, dj=2) is frame 1, row 2, col 5
    S_idx = (1 * cfg.win_h + 0) * cfg.win_w + 2
    assert xw[1, 0, 1, 1, S_idx, 0] == x[1, 1, 2, 5, 0]


# ------------------------------------------------------------------------------------------
# cut-out and composite
# ------------------------------------------------------------------------------------------

def test_composite_outside_mask_is_input_bitwise():
    cfg = drsynth.NETS["tiny64"]
    frames, masks = drsynth.tiny_frame(0)
    W = drsynth.make_weights(cfg, 0)
    out = on.forward(frames, masks, W, cfg)
    outside = masks[..., None].repeat(3, -1) == 0
    assert np.array_equal(out[outside].astype(np.float32), frames[outside])
    inside = ~outside
    assert np.all((out[inside] > 0) & (out[inside] < 1))


def test_empty_mask_is_identity_and_full_mask_is_pred():
    cfg = drsynth.NETS["tiny64"]
    frames, _ = drsynth.tiny_frame(3)
    W = drsynth.make_weights(cfg, 0)
    zero = np.zeros(frames.shape[:-1], np.uint8)
    d0 = on.forward_detail(frames, zero, W, cfg)
    assert np.array_equal(d0["out"], frames.astype(np.float64))
    assert not d0["flags"].any()
    ones = np.ones_like(zero)
    d1 = on.forward_detail(frames, ones, W, cfg)
    assert np.array_equal(d1["out"], d1["pred"])


def test_cut_out_sets_private_pixels_to_zero():
    frames, masks = small_inputs(4)
    xc = on.cut_out(frames, masks)
    assert np.all(xc[masks != 0] == 0)
    assert np.array_equal(xc[masks == 0], frames[masks == 0].astype(np.float64))


# ------------------------------------------------------------------------------------------
# convolutions
# ------------------------------------------------------------------------------------------

def test_patch_embed_matches_conv2d_and_brute_force():
    rng = np.random.default_rng(5)
    xc = rng.random((1, 2, 8, 12, 3))
    w = rng.standard_normal((7, 3, 4, 4))
    b = rng.standard_normal(7)
    x = on.patch_embed(xc, w, b, 4)
    ref = F.conv2d(torch.from_numpy(xc.reshape(2, 8, 12, 3)).permute(0, 3, 1, 2), torch.from_numpy(w),
                   torch.from_numpy(b), stride=4).permute(0, 2, 3, 1).numpy()
    np.testing.assert_allclose(x.reshape(ref.shape), ref, rtol=1e-12, atol=1e-12)
    # six-deep loop for one output
    t, i, j, o = 1, 1, 2, 3
    acc = b[o]
    for c in range(3):
        for ky in range(4):
            for kx in range(4):
                acc += w[o, c, ky, kx] * xc[0, t, 4 * i + ky, 4 * j + kx, c]
    assert abs(acc - x[0, t, i, j, o]) < 1e-12


def test_decoder_matches_conv_transpose2d():
    rng = np.random.default_rng(6)
    z = rng.standard_normal((1, 2, 3, 4, 5))
    wd = rng.standard_normal((5, 3, 4, 4))
    bd = rng.standard_normal(3)
    y = on.decode_logits(z, wd, bd, 4)
    ref = F.conv_transpose2d(torch.from_numpy(z.reshape(2, 3, 4, 5)).permute(0, 3, 1, 2),
                             torch.from_numpy(wd), torch.from_numpy(bd), stride=4)
    np.testing.assert_allclose(y.reshape(2, 12, 16, 3), ref.permute(0, 2, 3, 1).numpy(),
                               rtol=1e-12, atol=1e-12)


def test_embed_decoder_adjoint_identity():
    rng = np.random.default_rng(7)
    w = rng.standard_normal((6, 3, 4, 4))
    xin = rng.standard_normal((1, 1, 8, 12, 3))
    y = rng.standard_normal((1, 1, 2, 3, 6))
    conv = on.patch_embed(xin, w, np.zeros(6), 4)
    convT = on.decode_logits(y, w, np.zeros(3), 4)
    lhs = float((conv * y).sum())
    rhs = float((xin * convT).sum())
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)


# ------------------------------------------------------------------------------------------
# LayerNorm, GELU
# ------------------------------------------------------------------------------------------

def test_layer_norm_moments_and_library():
    rng = np.random.default_rng(8)
    x = rng.standard_normal((10, 33)) * 3 + 1
    y = on.layer_norm(x, np.ones(33), np.zeros(33), eps=0.0)
    np.testing.assert_allclose(y.mean(-1), 0, atol=1e-12)
    np.testing.assert_allclose((y ** 2).mean(-1), 1, atol=1e-12)
    g, b = rng.standard_normal(33), rng.standard_normal(33)
    ref = F.layer_norm(torch.from_numpy(x), (33,), torch.from_numpy(g), torch.from_numpy(b), eps=1e-5)
    np.testing.assert_allclose(on.layer_norm(x, g, b), ref.numpy(), rtol=1e-12, atol=1e-12)


def test_gelu_scalar_loop_and_identities():
    z = np.linspace(-6, 6, 101)
    ref = np.array([0.5 * t * (1 + math.erf(t / math.sqrt(2))) for t in z])
    np.testing.assert_allclose(on.gelu(z), ref, rtol=1e-14, atol=1e-15)
    assert on.gelu(np.array(0.0)) == 0.0
    np.testing.assert_allclose(on.gelu(z) - on.gelu(-z), z, atol=1e-13)


# ------------------------------------------------------------------------------------------
# attention
# ------------------------------------------------------------------------------------------

def test_attention_rows_sum_to_one_and_match_sdpa():
    rng = np.random.default_rng(9)
    q, k, v = (rng.standard_normal((3, 12, 16)) for _ in range(3))
    o, p = on.multi_head_attention(q, k, v, heads=2)
    np.testing.assert_allclose(p.sum(-1), 1.0, atol=1e-12)
    tq = lambda a: torch.from_numpy(a).reshape(3, 12, 2, 8).transpose(1, 2)  # noqa: E731
    ref = F.scaled_dot_product_attention(tq(q), tq(k), tq(v)).transpose(1, 2).reshape(3, 12, 16)
    np.testing.assert_allclose(o, ref.numpy(), rtol=1e-12, atol=1e-12)


def test_window_attention_equals_masked_full_attention():
    """Per-window attention == brute-force full attention over all tokens with -inf outside
    the query's window, on a tiny multi-frame grid."""
    cfg = SMALL
    rng = np.random.default_rng(10)
    shape = (1, 2, 4, 6, cfg.dim)
    q, k, v = (rng.standard_normal(shape) for _ in range(3))
    o_w, _ = on.multi_head_attention(on.to_windows(q, cfg), on.to_windows(k, cfg),
                                     on.to_windows(v, cfg), cfg.heads)
    o = on.from_windows(o_w, cfg).reshape(-1, cfg.dim)
    coords = [(t, i, j) for t in range(2) for i in range(4) for j in range(6)]
    wid = [((t // 2) * 2 + i // 2) * 2 + j // 3 for (t, i, j) in coords]
    qf, kf, vf = (a.reshape(-1, cfg.dim) for a in (q, k, v))
    dh = cfg.dim // cfg.heads
    for n in range(len(coords)):
        for h in range(cfg.heads):
            sl = slice(h * dh, (h + 1) * dh)
            s = np.array([qf[n, sl] @ kf[m, sl] / math.sqrt(dh) if wid[m] == wid[n] else -np.inf
                          for m in range(len(coords))])
            a = np.exp(s - s.max())
            a /= a.sum()
            np.testing.assert_allclose(o[n, sl], a @ vf[:, sl], rtol=1e-12, atol=1e-12)


def test_uniform_attention_closed_form():
    """With Wq = 0 and bq = 0 all scores are 0, so every query returns the window mean of V."""
    rng = np.random.default_rng(11)
    k, v = rng.standard_normal((2, 4, 9, 8)), rng.standard_normal((2, 4, 9, 8))
    q = np.zeros_like(k)
    o, _ = on.multi_head_attention(q, k, v, heads=2)
    np.testing.assert_allclose(o, np.broadcast_to(v.mean(-2, keepdims=True), o.shape), atol=1e-14)


def test_attention_permutation_equivariance():
    rng = np.random.default_rng(12)
    q, k, v = (rng.standard_normal((1, 10, 8)) for _ in range(3))
    perm = rng.permutation(10)
    o, _ = on.multi_head_attention(q, k, v, heads=2)
    op, _ = on.multi_head_attention(q[:, perm], k[:, perm], v[:, perm], heads=2)
    np.testing.assert_allclose(op, o[:, perm], atol=1e-13)


# ------------------------------------------------------------------------------------------
# whole network
# ------------------------------------------------------------------------------------------

@pytest.mark.parametrize("query_set", ["masked", "all"])
def test_forward_matches_independent_torch_reference(query_set):
    cfg = SMALL
    frames, masks = small_inputs(13)
    W = drsynth.make_weights(cfg, 3, std=0.2)  # larger weights: every term matters
    d = on.forward_detail(frames, masks, W, cfg, query_set)
    out, pred, flags = reference_forward(frames, masks, W, cfg, query_set)
    assert np.array_equal(d["flags"], flags)
    np.testing.assert_allclose(d["pred"], pred, rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(d["out"], out, rtol=1e-11, atol=1e-12)


def test_tiny64_matches_independent_torch_reference():
    cfg = drsynth.NETS["tiny64"]
    frames, masks = drsynth.tiny_frame(0)
    W = drsynth.make_weights(cfg, 0, qk_std=0.2)
    d = on.forward_detail(frames, masks, W, cfg)
    out, pred, _ = reference_forward(frames, masks, W, cfg)
    np.testing.assert_allclose(d["out"], out, rtol=1e-11, atol=1e-12)


def test_masked_with_full_mask_equals_all_queries():
    cfg = SMALL
    frames, _ = small_inputs(14)
    masks = np.ones(frames.shape[:-1], np.uint8)
    W = drsynth.make_weights(cfg, 1)
    a = on.forward(frames, masks, W, cfg, "masked")
    b = on.forward(frames, masks, W, cfg, "all")
    np.testing.assert_allclose(a, b, atol=1e-12, rtol=0)


def test_unflagged_tokens_keep_embedding():
    cfg = SMALL
    frames, masks = small_inputs(15)
    W = drsynth.make_weights(cfg, 1)
    d = on.forward_detail(frames, masks, W, cfg)
    keep = ~d["flags"]
    assert np.array_equal(d["x"][keep], d["x0"][keep])
    assert not np.allclose(d["x"][~keep], d["x0"][~keep])


def test_window_locality_bitwise():
    """Changing pixels outside window w's pixel footprint leaves w's outputs bit-identical."""
    cfg = SMALL
    frames, masks = small_inputs(16, B=1)
    W = drsynth.make_weights(cfg, 2)
    out0 = on.forward(frames, masks, W, cfg)
    f2, m2 = frames.copy(), masks.copy()
    # window (u=0, v=0) covers token rows 0..1, cols 0..2 -> pixel rows 0..7, cols 0..11
    f2[:, :, 8:, :] = np.random.default_rng(0).random(f2[:, :, 8:, :].shape)
    m2[:, :, 8:, 12:] ^= 1
    out1 = on.forward(f2, m2, W, cfg)
    assert np.array_equal(out0[:, :, :8, :12], out1[:, :, :8, :12])
    assert not np.array_equal(out0[:, :, 8:], out1[:, :, 8:])


def test_batch_independence():
    cfg = SMALL
    frames, masks = small_inputs(17, B=3)
    W = drsynth.make_weights(cfg, 2)
    full = on.forward(frames, masks, W, cfg)
    for b in range(3):
        one = on.forward(frames[b:b + 1], masks[b:b + 1], W, cfg)
        np.testing.assert_array_equal(one, full[b:b + 1])


def test_translation_by_window_stride_commutes_with_crop():
    """No positional encoding + aligned non-overlapping windows: the forward of a crop at a
    window boundary equals the crop of the forward."""
    cfg = SMALL
    frames, masks = small_inputs(18, B=1, H=16, W=24)
    W = drsynth.make_weights(cfg, 2)
    full = on.forward(frames, masks, W, cfg)
    # window footprint is 8 x 12 pixels; crop the window (u=1, v=1)
    crop = on.forward(frames[:, :, 8:16, 12:24], masks[:, :, 8:16, 12:24], W, cfg)
    np.testing.assert_allclose(crop, full[:, :, 8:16, 12:24], rtol=0, atol=1e-13)


def test_frame_permutation_within_temporal_window():
    """Windows span every frame of the clip and carry no positional encoding, so permuting
    the frames permutes the outputs."""
    cfg = SMALL
    frames, masks = small_inputs(19, B=1)
    W = drsynth.make_weights(cfg, 2)
    out = on.forward(frames, masks, W, cfg)
    outp = on.forward(frames[:, ::-1], masks[:, ::-1], W, cfg)
    np.testing.assert_allclose(outp, out[:, ::-1], atol=1e-12)
