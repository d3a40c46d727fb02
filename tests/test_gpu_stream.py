"""GPU stream mode and serving loop: parity with the stream-mode oracle, batch invariance,
and the native server's results equal to direct steps."""
import sys
import time

import numpy as np
import pytest

import drsynth
from oracle import stream as ost
from tests.gpu_util import MID, TOL

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


@pytest.fixture(scope="module")
def eng(dev):
    from paper_2509_10466_amd import Inpainter
    W = drsynth.make_weights(MID, 0)
    e = Inpainter(MID, W)
    e.W = W
    return e


def video(seed, T, H=40, W=72):
    sc = drsynth.Scene(seed, H, W, cov_range=(0.15, 0.4), cover_frames=T)
    return np.stack([sc.frame(t) for t in range(T)]), np.stack([sc.mask(t) for t in range(T)])


def _step(eng, sids, fr, ms):
    outs = eng.stream_step(sids, [torch.from_numpy(f).cuda() for f in fr], [torch.from_numpy(m).cuda() for m in ms])
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in outs]


def test_stream_matches_oracle_over_eviction(eng):
    """7 frames: the first frames see a partial history, later ones evict the oldest."""
    f, m = video(3, 7)
    sid = eng.stream_open(40, 72)
    st = ost.StreamState(MID)
    worst = 0.0
    for t in range(7):
        out = _step(eng, [sid], [f[t]], [m[t]])[0]
        ref, _ = ost.step(st, f[t], m[t], eng.W, MID)
        inside = np.repeat(m[t][..., None] != 0, 3, -1)
        assert np.array_equal(out[~inside], f[t][~inside])
        err = float(np.abs(out[inside] - ref[inside]).max()) if inside.any() else 0.0
        assert err <= TOL["bf16"], (t, err)
        worst = max(worst, err)
    _say(f"stream max abs err {worst:.3e}")
    eng.stream_close(sid)


def test_stream_alone_equals_in_batch(eng):
    """A stream's outputs are the same bitwise whether stepped alone or batched with others."""
    fa, ma = video(5, 6)
    fb, mb = video(6, 6)
    fc, mc = video(7, 6)
    alone = eng.stream_open(40, 72)
    s1, s2, s3 = (eng.stream_open(40, 72) for _ in range(3))
    for t in range(6):
        a = _step(eng, [alone], [fa[t]], [ma[t]])[0]
        if t % 2 == 0:
            b = _step(eng, [s2, s1, s3], [fb[t], fa[t], fc[t]], [mb[t], ma[t], mc[t]])[1]
        else:
            b = _step(eng, [s1, s2], [fa[t], fb[t]], [ma[t], mb[t]])[0]
            _step(eng, [s3], [fc[t]], [mc[t]])
        assert np.array_equal(a, b), t
    for s in (alone, s1, s2, s3):
        eng.stream_close(s)


def test_stream_budget_admission(eng):
    from paper_2509_10466_amd._lib import DrError
    fp = eng.stream_footprint(40, 72)
    eng.set_budget(2 * fp)
    a = eng.stream_open(40, 72)
    b = eng.stream_open(40, 72)
    with pytest.raises(DrError, match="DR_ENOMEM"):
        eng.stream_open(40, 72)
    eng.stream_close(a)
    c = eng.stream_open(40, 72)  # admitted once memory frees up
    eng.stream_close(b)
    eng.stream_close(c)
    eng.set_budget(0)


def test_server_results_equal_direct_steps(eng):
    """Two resolutions, four streams, frames submitted out of order across streams: every
    result equals the direct step of the same stream history (bitwise)."""
    from paper_2509_10466_amd.api import Server
    T = 5
    vids = {0: video(11, T), 1: video(12, T), 2: video(13, T, 80, 144), 3: video(14, T, 80, 144)}
    # reference: direct single-stream steps
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
        for k in (2, 0, 3, 1):
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
    _say(f"server stats {stats}, median latency {np.median([l for _, l, _ in done]):.2f} ms")
    torch.cuda.synchronize()
    for k in vids:
        for t in range(T):
            assert np.array_equal(outs[k][t].cpu().numpy(), ref[k][t]), (k, t)
    for k in sids:
        eng.stream_close(sids[k])


@pytest.mark.parametrize("slots", [1, 2, 3])
def test_stream_memory_slots_match_oracle(eng, slots):
    f, m = video(21 + slots, 5)
    sid = eng.stream_open(40, 72, slots=slots)
    st = ost.StreamState(MID, slots)
    for t in range(5):
        out = _step(eng, [sid], [f[t]], [m[t]])[0]
        ref, _ = ost.step(st, f[t], m[t], eng.W, MID)
        inside = np.repeat(m[t][..., None] != 0, 3, -1)
        assert np.array_equal(out[~inside], f[t][~inside])
        if inside.any():
            assert float(np.abs(out[inside] - ref[inside]).max()) <= TOL["bf16"], (slots, t)
    eng.stream_close(sid)
