"""Whole-clip parity at full size: every window that holds a private pixel is recomputed by
the FP64 oracle from its own pixel footprint and compared with the GPU result; every pixel
outside the mask (which covers all windows without one) must be the input bit for bit.

5 x 240 x 432 clips (clip240 network) on two seeds in FP32, BF16 and FP8; 5 x 720 x 1280 clips
(clip720 network) in BF16 on seed 0 and in FP8 on seeds 0, 1 and 2.  Each case reports the
max and RMS error over the in-mask values and the spread of the oracle's in-mask prediction,
so the size of each tolerance can be read against the values it bounds."""
import sys

import numpy as np
import pytest

import drsynth
from oracle import network as on
from tests.gpu_util import TOL, active_windows, case_inputs, error_stats, oracle_windows

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


_ENG = {}
_REF = {}


def _engine(cfg):
    from paper_2509_10466_amd import Inpainter
    if cfg not in _ENG:
        W = drsynth.make_weights(cfg, 0)
        _ENG[cfg] = (Inpainter(cfg, W), W)
    return _ENG[cfg]


def _reference(case, seed):
    """(cfg, frames, masks, footprints, [(out, pred)] per footprint), cached per clip."""
    key = (case, seed)
    if key not in _REF:
        cfg, frames, masks = case_inputs(case, seed)
        _, W = _engine(cfg)
        fps = active_windows(cfg, masks)
        _say(f"  oracle: {case} seed {seed}, {len(fps)} windows with queries")
        _REF.clear()  # one clip's reference at a time bounds host memory
        _REF[key] = (cfg, frames, masks, fps, oracle_windows(on, cfg, frames, masks, W, fps))
    return _REF[key]


def _check(case, seed, precision):
    cfg, frames, masks, fps, refs = _reference(case, seed)
    eng, _ = _engine(cfg)
    _say(f"[whole clip] {case} seed {seed} {precision}")
    out = eng(torch.from_numpy(frames).cuda(), torch.from_numpy(masks).cuda(), precision)
    torch.cuda.synchronize()
    out = out.cpu().numpy()
    inside = np.repeat(masks[..., None] != 0, 3, axis=-1)
    assert np.array_equal(out[~inside], frames[~inside]), "pixels outside the mask changed"
    # gather every window's in-mask errors, then one verdict over the whole clip
    d, p = [], []
    for (b, rs, cs), (ro, rp) in zip(fps, refs):
        m = np.repeat(masks[b, :, rs, cs][..., None] != 0, 3, axis=-1)
        d.append(out[b, :, rs, cs][m].astype(np.float64) - ro[m])
        p.append(rp[m])
    d, p = np.concatenate(d), np.concatenate(p)
    assert d.size == int(inside.sum()), "the windows with queries must cover every private pixel"
    s = {"max": float(np.abs(d).max()), "rms": float(np.sqrt(np.mean(d * d))),
         "spread": float(p.max() - p.min()), "n": int(d.size), "windows": len(fps)}
    _say(f"    {s}")
    assert s["max"] <= TOL[precision], s


@pytest.mark.parametrize("precision", ["fp32", "bf16", "fp8"])
@pytest.mark.parametrize("seed", [0, 1])
def test_clip240_whole_clip(dev, seed, precision):
    _check("clip240", seed, precision)


def test_clip720_whole_clip_bf16(dev):
    _check("clip720", 0, "bf16")


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_clip720_whole_clip_fp8(dev, seed):
    _check("clip720", seed, "fp8")

