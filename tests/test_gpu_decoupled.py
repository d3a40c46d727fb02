"""GPU parity of the decoupled attention pattern (even blocks within one frame of a window,
odd blocks across its frames at one token position) against the FP64 oracle."""
import dataclasses
import sys

import numpy as np
import pytest

import drsynth
from oracle import network as on
from tests.gpu_util import TOL, case_inputs, compare, sample_windows

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


def dec(cfg):
    return dataclasses.replace(cfg, attn="decoupled")


_ENG = {}


def engine(cfg, seed=0, qk_std=None):
    from paper_2509_10466_amd import Inpainter
    key = (cfg, seed, qk_std)
    if key not in _ENG:
        W = drsynth.make_weights(cfg, seed, qk_std=qk_std)
        _ENG[key] = (Inpainter(cfg, W), W)
    return _ENG[key]


def run(eng, frames, masks, precision, qs="masked"):
    out = eng(torch.from_numpy(frames).cuda(), torch.from_numpy(masks).cuda(), precision, qs)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("case,precision", [("tiny64", "bf16"), ("mid", "bf16"), ("mid_b2", "bf16"),
                                            ("mid", "fp8"), ("mid_b2", "fp8")])
@pytest.mark.parametrize("qs", ["masked", "all"])
def test_decoupled_parity_small(dev, case, precision, qs):
    """tiny64 has one frame per window: its temporal blocks see only the query's own key."""
    cfg, frames, masks = case_inputs(case)
    cfg = dec(cfg)
    _say(f"[decoupled] case={case} prec={precision} qs={qs} shape={frames.shape}")
    eng, W = engine(cfg)
    out = run(eng, frames, masks, precision, qs)
    ref = on.forward(frames, masks, W, cfg, qs)
    mx, n = compare(out, ref, frames, masks, TOL[precision])
    _say(f"    max abs err {mx:.3e} over {n} in-mask values")


@pytest.mark.parametrize("precision", ["bf16", "fp8"])
def test_decoupled_stress_weights(dev, precision):
    """Peaked softmax over the short per-frame and per-position key sets."""
    cfg, frames, masks = case_inputs("mid")
    cfg = dec(cfg)
    _say(f"[decoupled stress] prec={precision}")
    eng, W = engine(cfg, seed=1, qk_std=0.2)
    out = run(eng, frames, masks, precision)
    compare(out, on.forward(frames, masks, W, cfg), frames, masks, TOL[precision])


@pytest.mark.parametrize("precision", ["bf16", "fp8"])
def test_decoupled_full_size_sampled(dev, precision):
    """The 5 x 240 x 432 clip with the 256-dim decoupled network; sampled windows recomputed
    by the oracle from their pixel footprints."""
    cfg, frames, masks = case_inputs("clip240")
    cfg = dec(cfg)
    assert cfg == drsynth.NETS["clip240_dec"]
    _say(f"[decoupled full-size] prec={precision} shape={frames.shape}")
    eng, W = engine(cfg)
    out = run(eng, frames, masks, precision)
    inside = np.repeat(masks[..., None] != 0, 3, axis=-1)
    assert np.array_equal(out[~inside], frames[~inside])
    worst = 0.0
    for b, rs, cs in sample_windows(cfg, masks, k=6):
        ref = on.forward(frames[b:b + 1, :, rs, cs], masks[b:b + 1, :, rs, cs], W, cfg)
        mx, _ = compare(out[b:b + 1, :, rs, cs], ref, frames[b:b + 1, :, rs, cs], masks[b:b + 1, :, rs, cs],
                        TOL[precision])
        worst = max(worst, mx)
    _say(f"    worst sampled max abs err {worst:.3e}")


def test_pattern_switch_and_graphs(dev):
    """Switching the pattern on one context: joint -> decoupled -> joint gives the joint bits
    back (captured block graphs are dropped on a switch) and the decoupled result of a fresh
    decoupled context; the two patterns give different pictures."""
    from paper_2509_10466_amd import Inpainter
    cfg, frames, masks = case_inputs("mid")
    W = drsynth.make_weights(cfg, 0)
    eng = Inpainter(cfg, W)
    joint = run(eng, frames, masks, "bf16")
    joint2 = run(eng, frames, masks, "bf16")  # a replay of the captured graphs
    eng.set_attention("decoupled")
    d = run(eng, frames, masks, "bf16")
    d2 = run(eng, frames, masks, "bf16")
    eng.set_attention("joint")
    back = run(eng, frames, masks, "bf16")
    eng.close()
    fresh, _ = engine(dec(cfg))
    assert np.array_equal(joint, joint2) and np.array_equal(joint, back)
    assert np.array_equal(d, d2)
    assert np.array_equal(d, run(fresh, frames, masks, "bf16"))
    inside = masks != 0
    assert np.abs(d - joint)[inside].max() > 1e-3


def test_decoupled_rejects_fp32_and_training(dev):
    """Stream mode runs the decoupled pattern (its own tests compare it with the stream
    oracle); the FP32 path and training do not."""
    from paper_2509_10466_amd._lib import DrError
    cfg, frames, masks = case_inputs("mid")
    eng, _ = engine(dec(cfg))
    f = torch.from_numpy(frames).cuda()
    m = torch.from_numpy(masks).cuda()
    with pytest.raises(DrError, match="DR_EINVAL"):
        eng(f, m, "fp32")
    with pytest.raises(DrError, match="DR_EINVAL"):
        eng.train_forward(f, m)
    from paper_2509_10466_amd import _lib
    with pytest.raises(DrError, match="DR_EINVAL"):
        _lib.check(eng.lib, eng._ctx, eng.lib.dr_set_attention_pattern(eng._ctx, 2))


def _clip720_net_small(seed=3):
    """The 384-dim, 12-block clip720 network (6 x 10 x 5-token windows: 300 keys, padded to
    304) on a 5 x 48 x 80 clip of 2 x 2 windows, small enough for the whole-clip oracle."""
    f, m, _ = drsynth.make_clip(seed, 5, 48, 80, cov_range=(0.2, 0.4))
    return drsynth.NETS["clip720"], f, m


@pytest.mark.parametrize("precision", ["bf16", "fp8"])
@pytest.mark.parametrize("qs", ["masked", "all"])
def test_decoupled_clip720_network(dev, precision, qs):
    cfg, frames, masks = _clip720_net_small()
    cfg = dec(cfg)
    _say(f"[decoupled clip720 net] prec={precision} qs={qs}")
    eng, W = engine(cfg)
    out = run(eng, frames, masks, precision, qs)
    mx, n = compare(out, on.forward(frames, masks, W, cfg, qs), frames, masks, TOL[precision])
    _say(f"    max abs err {mx:.3e} over {n} in-mask values")


@pytest.mark.parametrize("precision", ["bf16", "fp8"])
def test_decoupled_graph_replay_equals_direct_launches(dev, precision):
    """The decoupled block sequence replayed as a HIP graph gives the bits of direct launches,
    on every replay, with inputs changing between calls."""
    from paper_2509_10466_amd import Inpainter
    cfg, fa, ma = case_inputs("clip240", 0)
    _, fb, mb = case_inputs("clip240", 1)
    cfg = dec(cfg)
    eng = Inpainter(cfg, drsynth.make_weights(cfg, 0))
    eng.debug_set("graphs", 0)
    ra = run(eng, fa, ma, precision)
    rb = run(eng, fb, mb, precision)
    eng.debug_set("graphs", 1)
    for rep in range(4):  # eager, capture, replay, replay (per clip)
        assert np.array_equal(run(eng, fa, ma, precision), ra), ("a", rep)
        _ = torch.ones(1000, device="cuda").sum().item()  # unrelated eager work + sync
        assert np.array_equal(run(eng, fb, mb, precision), rb), ("b", rep)
    eng.close()
