"""GPU stream mode with the decoupled attention pattern (even blocks within the new frame's
window, odd blocks at one token position across the cached frames and the new frame) against
the stream-mode oracle, through cache eviction, with fewer memory slots, and batched."""
import dataclasses
import sys

import numpy as np
import pytest

import drsynth
from oracle import stream as ost
from tests.gpu_util import MID, TOL, error_stats

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

# (network, frame H, frame W): head dims 64 and 32 at 45 keys per frame window, and the 720p
# network's 6 x 10 windows (60 keys, head dim 64)
NETS = {
    "mid": (dataclasses.replace(MID, attn="decoupled"), 40, 72),
    "mid_dh32": (dataclasses.replace(MID, heads=4, attn="decoupled"), 40, 72),
    "clip720": (dataclasses.replace(drsynth.NETS["clip720"], attn="decoupled"), 48, 80),
}
_ENG = {}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def engine(name):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if name not in _ENG:
        from paper_2509_10466_amd import Inpainter
        cfg = NETS[name][0]
        W = drsynth.make_weights(cfg, 0)
        _ENG[name] = (Inpainter(cfg, W), W)
    return _ENG[name]


def video(seed, T, H, W):
    sc = drsynth.Scene(seed, H, W, cov_range=(0.15, 0.4), cover_frames=T)
    return np.stack([sc.frame(t) for t in range(T)]), np.stack([sc.mask(t) for t in range(T)])


def _step(eng, sids, fr, ms, qs="masked"):
    outs = eng.stream_step(sids, [torch.from_numpy(f).cuda() for f in fr],
                           [torch.from_numpy(m).cuda() for m in ms], query_set=qs)
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in outs]


@pytest.mark.parametrize("name", list(NETS))
@pytest.mark.parametrize("qs", ["masked", "all"])
def test_stream_decoupled_matches_oracle_over_eviction(name, qs):
    """7 frames: the first see a partial history, the last two evict the oldest cached frame."""
    eng, W = engine(name)
    cfg, H, Wd = NETS[name]
    f, m = video(41, 7, H, Wd)
    sid = eng.stream_open(H, Wd)
    st = ost.StreamState(cfg)
    worst = 0.0
    try:
        for t in range(7):
            _say(f"[stream decoupled] net={name} qs={qs} frame {t}")
            out = _step(eng, [sid], [f[t]], [m[t]], qs)[0]
            ref, pred = ost.step(st, f[t], m[t], W, cfg, query_set=qs)
            s = error_stats(out, ref, pred, f[t], m[t], TOL["bf16"])
            worst = max(worst, s["max"])
    finally:
        eng.stream_close(sid)
    _say(f"  max abs err {worst:.3e}")


@pytest.mark.parametrize("slots", [0, 2])
def test_stream_decoupled_memory_slots(slots):
    """Fewer memory slots: a temporal block sees at most `slots` cached frames."""
    eng, W = engine("mid")
    cfg, H, Wd = NETS["mid"]
    f, m = video(43, 6, H, Wd)
    sid = eng.stream_open(H, Wd, slots=slots)
    st = ost.StreamState(cfg, slots)
    try:
        for t in range(6):
            _say(f"[stream decoupled] slots={slots} frame {t}")
            out = _step(eng, [sid], [f[t]], [m[t]])[0]
            ref, pred = ost.step(st, f[t], m[t], W, cfg)
            error_stats(out, ref, pred, f[t], m[t], TOL["bf16"])
    finally:
        eng.stream_close(sid)


def test_stream_decoupled_alone_equals_in_batch():
    """A stream's outputs are the same bitwise stepped alone or batched with streams that
    are at other points of their history."""
    eng, W = engine("mid")
    cfg, H, Wd = NETS["mid"]
    fa, ma = video(45, 6, H, Wd)
    fb, mb = video(46, 6, H, Wd)
    alone, s1, s2 = (eng.stream_open(H, Wd) for _ in range(3))
    try:
        _step(eng, [s2], [fb[0]], [mb[0]])  # s2 is one frame ahead
        for t in range(6):
            _say(f"[stream decoupled batch] frame {t}")
            a = _step(eng, [alone], [fa[t]], [ma[t]])[0]
            b = _step(eng, [s2, s1], [fb[(t + 1) % 6], fa[t]], [mb[(t + 1) % 6], ma[t]])[1]
            assert np.array_equal(a, b), t
    finally:
        for s in (alone, s1, s2):
            eng.stream_close(s)
