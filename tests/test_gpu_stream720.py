"""GPU stream mode on the 720p network (dim 384, 6 heads, 12 blocks, 6 x 10-token windows, 60
keys per frame and window): parity with the stream-mode oracle through cache eviction, on a
whole small stream and on sampled windows of a 360 x 640 stream, plus the native server
against direct steps at that network."""
import sys
import time

import numpy as np
import pytest

import drsynth
from oracle import stream as ost
from tests.gpu_util import TOL, error_stats

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

NET = drsynth.NETS["clip720"]


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def eng():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_10466_amd import Inpainter
    W = drsynth.make_weights(NET, 0)
    e = Inpainter(NET, W)
    e.W = W
    yield e
    e.close()


def video(seed, T, H, W, cov=(0.15, 0.4)):
    sc = drsynth.Scene(seed, H, W, cov_range=cov, cover_frames=T)
    return np.stack([sc.frame(t) for t in range(T)]), np.stack([sc.mask(t) for t in range(T)])


def _step(eng, sids, fr, ms):
    outs = eng.stream_step(sids, [torch.from_numpy(f).cuda() for f in fr], [torch.from_numpy(m).cuda() for m in ms])
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in outs]


def test_stream720_whole_stream_over_eviction(eng):
    """48 x 80 frames (2 x 2 windows), 7 frames: the first four see a partial history, the
    last two evict the oldest cached frame of every block."""
    f, m = video(31, 7, 48, 80)
    sid = eng.stream_open(48, 80)
    st = ost.StreamState(NET)
    worst = 0.0
    for t in range(7):
        _say(f"stream720 48x80 frame {t}")
        out = _step(eng, [sid], [f[t]], [m[t]])[0]
        ref, pred = ost.step(st, f[t], m[t], eng.W, NET)
        s = error_stats(out, ref, pred, f[t], m[t], TOL["bf16"])
        _say(f"  frame {t}: {s}")
        worst = max(worst, s["max"])
    eng.stream_close(sid)
    _say(f"stream720 48x80 max abs err {worst:.3e}")


def test_stream720_sampled_windows_360x640(eng):
    """360 x 640 frames (15 x 16 windows), 6 frames.  A window's outputs depend only on its own
    pixel footprint in the current and cached frames, so the oracle replays the stream of
    each sampled window's 24 x 40-pixel crop."""
    T, H, Wd = 6, 360, 640
    f, m = video(32, T, H, Wd)
    sid = eng.stream_open(H, Wd)
    outs = []
    for t in range(T):
        _say(f"stream720 360x640 frame {t}")
        outs.append(_step(eng, [sid], [f[t]], [m[t]])[0])
    eng.stream_close(sid)
    outs = np.stack(outs)
    ph, pw = NET.patch * NET.win_h, NET.patch * NET.win_w
    fps = [(u, v) for u in range(H // ph) for v in range(Wd // pw)]
    cov = np.array([m[:, u * ph:(u + 1) * ph, v * pw:(v + 1) * pw].mean() for u, v in fps])
    rng = np.random.default_rng(0)
    pick = list(np.argsort(-cov)[:4]) + list(np.flatnonzero(cov == 0)[:1])
    rest = [i for i in range(len(fps)) if i not in pick]
    pick += list(rng.choice(rest, size=4, replace=False))
    # outside the mask every pixel of the frame is the input, bit for bit
    inside = np.repeat(m[..., None] != 0, 3, -1)
    assert np.array_equal(outs[~inside], f[~inside])
    worst = 0.0
    for i in pick:
        u, v = fps[i]
        rs, cs = slice(u * ph, (u + 1) * ph), slice(v * pw, (v + 1) * pw)
        st = ost.StreamState(NET)
        for t in range(T):
            ref, pred = ost.step(st, f[t, rs, cs], m[t, rs, cs], eng.W, NET)
            s = error_stats(outs[t, rs, cs], ref, pred, f[t, rs, cs], m[t, rs, cs], TOL["bf16"])
            worst = max(worst, s["max"])
        _say(f"  window ({u},{v}) coverage {cov[i]:.2f}: last frame {s}")
    _say(f"stream720 360x640 sampled max abs err {worst:.3e}")


def test_stream720_alone_equals_in_batch(eng):
    """Bitwise: a 720p-network stream stepped alone or batched with two others."""
    fa, ma = video(41, 6, 48, 80)
    fb, mb = video(42, 6, 48, 80)
    fc, mc = video(43, 6, 48, 80)
    alone = eng.stream_open(48, 80)
    s1, s2, s3 = (eng.stream_open(48, 80) for _ in range(3))
    for t in range(6):
        a = _step(eng, [alone], [fa[t]], [ma[t]])[0]
        b = _step(eng, [s2, s1, s3], [fb[t], fa[t], fc[t]], [mb[t], ma[t], mc[t]])[1]
        assert np.array_equal(a, b), t
    for s in (alone, s1, s2, s3):
        eng.stream_close(s)


def test_stream720_server_equals_direct(eng):
    """Three 48 x 80 streams and one 96 x 160 stream through the native server, frames
    submitted interleaved across streams: every result equals the direct step bitwise."""
    from paper_2509_10466_amd.api import Server
    T = 6
    vids = {0: video(51, T, 48, 80), 1: video(52, T, 48, 80), 2: video(53, T, 48, 80), 3: video(54, T, 96, 160)}
    ref = {}
    for k, (f, m) in vids.items():
        sid = eng.stream_open(*f.shape[1:3])
        ref[k] = [_step(eng, [sid], [f[t]], [m[t]])[0] for t in range(T)]
        eng.stream_close(sid)
    sids = {k: eng.stream_open(*vids[k][0].shape[1:3]) for k in vids}
    dev_in = {k: ([torch.from_numpy(x).cuda() for x in vids[k][0]], [torch.from_numpy(x).cuda() for x in vids[k][1]])
              for k in vids}
    outs = {k: [torch.empty_like(x) for x in dev_in[k][0]] for k in vids}
    torch.cuda.synchronize()
    srv = Server(eng, max_batch=4)
    tickets = {}
    for t in range(T):
        for k in (3, 1, 0, 2):
            tk = srv.submit(sids[k], dev_in[k][0][t], dev_in[k][1][t], outs[k][t])
            tickets[tk] = (k, t)
    done = []
    t0 = time.time()
    while len(done) < len(tickets) and time.time() - t0 < 60:
        done += srv.poll()
        time.sleep(0.002)
    stats = srv.stats()
    srv.close()
    assert len(done) == len(tickets)
    assert all(s == 0 for _, _, s in done)
    _say(f"server stats {stats}")
    torch.cuda.synchronize()
    for k in vids:
        for t in range(T):
            assert np.array_equal(outs[k][t].cpu().numpy(), ref[k][t]), (k, t)
    for k in sids:
        eng.stream_close(sids[k])
