"""GPU parity of the overlapping embedding and fold decoder (kernel 8, stride 4, padding 2)
against the FP64 oracle, through the C ABI."""
import dataclasses
import sys

import numpy as np
import pytest

import drsynth
from oracle import network as on
from tests.gpu_util import TOL, case_inputs, compare

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def ovl(cfg):
    return dataclasses.replace(cfg, overlap=True)


_ENG = {}


def engine(cfg, seed=0, qk_std=None):
    from paper_2509_10466_amd import Inpainter
    key = (cfg, seed, qk_std)
    if key not in _ENG:
        W = drsynth.make_weights(cfg, seed, qk_std=qk_std)
        _ENG[key] = (Inpainter(cfg, W), W)
    return _ENG[key]


def run(eng, frames, masks, precision="bf16", qs="masked"):
    out = eng(torch.from_numpy(frames).cuda(), torch.from_numpy(masks).cuda(), precision, qs)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("case", ["tiny64", "mid", "mid_b2", "clip240"])
@pytest.mark.parametrize("qs", ["masked", "all"])
def test_overlap_flags_bit_exact(dev, case, qs):
    cfg, frames, masks = case_inputs(case)
    cfg = ovl(cfg)
    _say(f"[ovl gather] case={case} qs={qs}")
    eng, _ = engine(cfg)
    flag, idx, woff = eng.gather_tokens(torch.from_numpy(masks).cuda(), qs)
    torch.cuda.synchronize()
    rf, ri, rw = on.gather_lists(masks, cfg, qs)
    assert np.array_equal(flag.cpu().numpy(), rf)
    assert np.array_equal(idx.cpu().numpy(), ri)
    assert np.array_equal(woff.cpu().numpy(), rw)


@pytest.mark.parametrize("case", ["tiny64", "mid", "mid_b2"])
@pytest.mark.parametrize("qs", ["masked", "all"])
def test_overlap_parity_small(dev, case, qs):
    """tiny64 is one 64 x 64 frame (one window): the padding and the crop act on every side."""
    cfg, frames, masks = case_inputs(case)
    cfg = ovl(cfg)
    _say(f"[ovl] case={case} qs={qs} shape={frames.shape}")
    eng, W = engine(cfg)
    out = run(eng, frames, masks, "bf16", qs)
    ref = on.forward(frames, masks, W, cfg, qs)
    mx, n = compare(out, ref, frames, masks, TOL["bf16"])
    _say(f"    max abs err {mx:.3e} over {n} in-mask values")


def test_overlap_stress_weights(dev):
    cfg, frames, masks = case_inputs("mid")
    cfg = ovl(cfg)
    eng, W = engine(cfg, seed=1, qk_std=0.2)
    out = run(eng, frames, masks)
    compare(out, on.forward(frames, masks, W, cfg), frames, masks, TOL["bf16"])


def test_overlap_full_size_whole_clip(dev):
    """The 5 x 240 x 432 clip with the 256-dim overlapping network, every pixel compared with
    the oracle on the whole clip (windows are no longer independent: the embedding and the
    decoder reach 2 pixels into the neighbouring windows)."""
    cfg, frames, masks = case_inputs("clip240")
    cfg = ovl(cfg)
    assert cfg == drsynth.NETS["clip240_ovl"]
    _say(f"[ovl full-size] shape={frames.shape}")
    eng, W = engine(cfg)
    out = run(eng, frames, masks)
    ref = on.forward(frames, masks, W, cfg)
    mx, n = compare(out, ref, frames, masks, TOL["bf16"])
    _say(f"    max abs err {mx:.3e} over {n} in-mask values")


def test_overlap_edge_masks(dev):
    """Masks on the frame border and on window borders (the padding, the crop and the
    windows' neighbours), and an empty mask (output = input)."""
    cfg, frames, _ = case_inputs("mid")
    cfg = ovl(cfg)
    eng, W = engine(cfg)
    m = np.zeros(frames.shape[:-1], np.uint8)
    m[:, :, 0:3, :] = 1            # top rows
    m[:, :, :, -2:] = 1            # right columns
    m[:, 2, 18:23, 34:39] = 1      # across a window corner (windows are 20 x 36 pixels)
    out = run(eng, frames, m)
    compare(out, on.forward(frames, m, W, cfg), frames, m, TOL["bf16"])
    z = np.zeros_like(m)
    assert np.array_equal(run(eng, frames, z), frames)


def test_overlap_in_place_and_determinism(dev):
    cfg, frames, masks = case_inputs("mid")
    cfg = ovl(cfg)
    eng, _ = engine(cfg)
    a = run(eng, frames, masks)
    f = torch.from_numpy(frames).cuda()
    m = torch.from_numpy(masks).cuda()
    eng(f, m, "bf16", out=f)
    torch.cuda.synchronize()
    assert np.array_equal(f.cpu().numpy(), a)
    assert np.array_equal(run(eng, frames, masks), a)


def test_overlap_rejects_other_paths(dev):
    from paper_2509_10466_amd._lib import DrError
    cfg, frames, masks = case_inputs("mid")
    eng, _ = engine(ovl(cfg))
    f = torch.from_numpy(frames).cuda()
    m = torch.from_numpy(masks).cuda()
    for prec in ("fp32", "fp8"):
        with pytest.raises(DrError, match="DR_EINVAL"):
            eng(f, m, prec)
    with pytest.raises(DrError, match="DR_EINVAL"):
        eng.train_forward(f, m)
    H, W = frames.shape[2:4]
    sid = eng.stream_open(H, W)
    try:
        out = torch.empty(f[0, 0].shape, dtype=torch.float32, device="cuda")
        with pytest.raises(DrError, match="DR_EINVAL"):
            eng.stream_step([sid], [f[0, 0].contiguous()], [m[0, 0].contiguous()], [out])
    finally:
        eng.stream_close(sid)


def test_reloading_plain_weights_switches_back(dev):
    """One context: overlapping weights, then the plain network's weights (kernel 4) give
    the plain network's output."""
    import ctypes as ct
    from paper_2509_10466_amd import Inpainter, _lib
    from paper_2509_10466_amd import weights as wblob
    cfg, frames, masks = case_inputs("mid")
    Wp = drsynth.make_weights(cfg, 0)
    plain = run(Inpainter(cfg, Wp), frames, masks)
    eng = Inpainter(ovl(cfg), drsynth.make_weights(ovl(cfg), 0))
    first = run(eng, frames, masks)
    blob = wblob.pack(cfg, Wp)
    buf = ct.create_string_buffer(blob, len(blob))
    _lib.check(eng.lib, eng._ctx, eng.lib.dr_load_weights(eng._ctx, buf, len(blob)))
    assert np.array_equal(run(eng, frames, masks), plain)
    assert not np.array_equal(first, plain)
    eng.close()


@pytest.mark.parametrize("qs", ["masked", "all"])
def test_overlap_with_decoupled_attention(dev, qs):
    """The two variants together: kernel-8 embedding and fold decoder around decoupled blocks."""
    cfg, frames, masks = case_inputs("mid")
    cfg = dataclasses.replace(cfg, overlap=True, attn="decoupled")
    _say(f"[ovl+dec] qs={qs}")
    eng, W = engine(cfg)
    out = run(eng, frames, masks, "bf16", qs)
    mx, n = compare(out, on.forward(frames, masks, W, cfg, qs), frames, masks, TOL["bf16"])
    _say(f"    max abs err {mx:.3e} over {n} in-mask values")


@pytest.mark.parametrize("qs", ["masked", "all"])
def test_overlap_clip720_network(dev, qs):
    """The 384-dim, 12-block clip720 network with the kernel-8 embedding and fold decoder on
    a 5 x 48 x 80 clip (2 x 2 windows of 6 x 10 tokens), whole clip against the oracle."""
    f, m, _ = drsynth.make_clip(4, 5, 48, 80, cov_range=(0.2, 0.4))
    cfg = ovl(drsynth.NETS["clip720"])
    _say(f"[ovl clip720 net] qs={qs}")
    eng, W = engine(cfg)
    out = run(eng, f, m, "bf16", qs)
    mx, n = compare(out, on.forward(f, m, W, cfg, qs), f, m, TOL["bf16"])
    _say(f"    max abs err {mx:.3e} over {n} in-mask values")


def test_overlap_graph_replay_equals_direct_launches(dev):
    from paper_2509_10466_amd import Inpainter
    cfg, fa, ma = case_inputs("clip240", 0)
    _, fb, mb = case_inputs("clip240", 1)
    cfg = ovl(cfg)
    eng = Inpainter(cfg, drsynth.make_weights(cfg, 0))
    eng.debug_set("graphs", 0)
    ra = run(eng, fa, ma)
    rb = run(eng, fb, mb)
    eng.debug_set("graphs", 1)
    for rep in range(4):
        assert np.array_equal(run(eng, fa, ma), ra), ("a", rep)
        _ = torch.ones(1000, device="cuda").sum().item()
        assert np.array_equal(run(eng, fb, mb), rb), ("b", rep)
    eng.close()
