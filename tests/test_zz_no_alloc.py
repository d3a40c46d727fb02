"""The allocation-free token gather (dr_gather_tokens_noalloc) against dr_gather_tokens, through
the C ABI: bit-exact integer outputs on two calls in a row, the second with a smaller input
(the static scratch keeps the first call's counts), and the size limit."""
import ctypes as ct
import sys

import numpy as np
import pytest

import drsynth
from tests.gpu_util import MID

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _noalloc(eng, masks, qs=0):
    B, T, H, W = masks.shape
    p = eng.cfg.patch
    N = B * T * (H // p) * (W // p)
    nwin = N // eng.cfg.window_tokens
    dev = masks.device
    flag = torch.full((N,), 7, dtype=torch.uint8, device=dev)
    idx = torch.full((N,), -5, dtype=torch.int32, device=dev)
    woff = torch.full((nwin + 1,), -5, dtype=torch.int32, device=dev)
    nq = torch.full((1,), -5, dtype=torch.int32, device=dev)
    st = eng.lib.dr_gather_tokens_noalloc(eng._ctx, masks.data_ptr(), B, T, H, W, qs, flag.data_ptr(), idx.data_ptr(),
                                          woff.data_ptr(), nq.data_ptr(), ct.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0, eng.lib.dr_last_error(eng._ctx)
    torch.cuda.synchronize()
    n = int(nq.item())
    return flag.cpu().numpy(), idx[:n].cpu().numpy(), woff.cpu().numpy()


def test_gather_noalloc_matches_gather_on_two_calls():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_10466_amd import Inpainter
    cfg = drsynth.NETS["clip240"]
    eng = Inpainter(cfg, drsynth.make_weights(cfg, 0))
    big = drsynth.make_clip_batch([0, 1], 5, 240, 432)[1]          # 2 clips: 288 windows
    small = drsynth.make_clip(2, 5, 40, 72, cov_range=(0.2, 0.4))[1]  # 1 clip: 4 windows (MID-size frames)
    for name, m in (("2 x 5 x 240 x 432", big), ("1 x 5 x 40 x 72", small)):
        _say(f"[noalloc gather] {name}")
        mt = torch.from_numpy(m).cuda()
        for qs_name, qs in (("masked", 0), ("all", 1)):
            rf, ri, rw = eng.gather_tokens(mt, qs_name)
            torch.cuda.synchronize()
            f, i, w = _noalloc(eng, mt, qs)
            assert np.array_equal(f, rf.cpu().numpy()), (name, qs_name)
            assert np.array_equal(i, ri.cpu().numpy()), (name, qs_name)
            assert np.array_equal(w, rw.cpu().numpy()), (name, qs_name)
    eng.close()


def test_gather_noalloc_rejects_more_windows_than_its_scratch():
    """65,537 windows of 8 x 8 tokens (64 x 64-pixel frames of the tiny network) exceed the
    static array; the call is refused before anything is launched."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_10466_amd import Inpainter
    cfg = drsynth.NETS["tiny64"]
    eng = Inpainter(cfg, drsynth.make_weights(cfg, 0))
    tiny = torch.zeros(16, dtype=torch.int32, device="cuda")
    B = 16385  # frames of 4 windows each
    st = eng.lib.dr_gather_tokens_noalloc(eng._ctx, tiny.data_ptr(), B, 1, 64, 64, 0, tiny.data_ptr(), tiny.data_ptr(),
                                          tiny.data_ptr(), tiny.data_ptr(), None)
    assert st == 1  # DR_EINVAL
    assert b"static scratch" in eng.lib.dr_last_error(eng._ctx)
    eng.close()


def test_mid_network_gather_noalloc_all_ones_and_empty():
    """Degenerate masks: nothing private (Nq = 0) and everything private (every token)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_10466_amd import Inpainter
    eng = Inpainter(MID, drsynth.make_weights(MID, 0))
    for fill in (0, 1):
        m = torch.full((1, 5, 40, 72), fill, dtype=torch.uint8, device="cuda")
        rf, ri, rw = eng.gather_tokens(m)
        f, i, w = _noalloc(eng, m)
        assert np.array_equal(f, rf.cpu().numpy()) and np.array_equal(i, ri.cpu().numpy())
        assert np.array_equal(w, rw.cpu().numpy())
    eng.close()
