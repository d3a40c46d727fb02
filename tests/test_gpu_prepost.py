"""GPU parity of the camera-resolution pre/post-processing against the oracle: masks and u8
frames bit-exact, the half-resolution RGB within one float32 rounding."""
import sys

import numpy as np
import pytest

import drsynth
from oracle import prepost as pp

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def eng():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_10466_amd import Inpainter
    cfg = drsynth.NETS["tiny64"]
    e = Inpainter(cfg, drsynth.make_weights(cfg, 0))
    yield e
    e.close()


def _inputs(seed, H, W, K, density=0.002):
    rng = np.random.default_rng(seed)
    bgra = rng.integers(0, 256, (H, W, 4), dtype=np.uint8)
    inst = np.zeros((K, H, W), np.uint8)
    for k in range(K):
        inst[k] = (rng.random((H, W)) < density) * rng.integers(1, 256)
        y, x = rng.integers(0, H - 8), rng.integers(0, W - 8)
        inst[k, y:y + 7, x:x + 5] = 255  # a solid object too
    return bgra, inst


# sizes: whole tiles, ragged tiles in both directions, a frame smaller than one tile
@pytest.mark.parametrize("H,W,K,radius,select", [
    (64, 128, 3, 2, 0b101), (70, 134, 5, 0, 0xFFFFFFFF), (90, 150, 1, 16, 1), (10, 12, 2, 3, 0b10),
    (360, 640, 4, 7, 0b1011), (40, 72, 0, 5, 0xFFFFFFFF)])
def test_prep_matches_oracle(eng, H, W, K, radius, select):
    _say(f"[prep] H={H} W={W} K={K} r={radius} select={select:#x}")
    bgra, inst = _inputs(H * 7 + W, H, W, K)
    low, mlow, mfull = eng.prep_frame(torch.from_numpy(bgra).cuda(), torch.from_numpy(inst).cuda() if K else None,
                                      select, radius)
    torch.cuda.synchronize()
    sel = [(select >> k) & 1 for k in range(K)]
    rlow, rmlow, rmfull = pp.prep(bgra, inst, sel, radius)
    assert np.array_equal(mfull.cpu().numpy(), rmfull)
    assert np.array_equal(mlow.cpu().numpy(), rmlow)
    np.testing.assert_allclose(low.cpu().numpy(), rlow, rtol=0, atol=6e-8)  # one f32 rounding of a value < 1


@pytest.mark.parametrize("H,W", [(64, 128), (70, 132), (360, 640), (720, 1280)])
def test_post_matches_oracle(eng, H, W):
    _say(f"[post] H={H} W={W}")
    rng = np.random.default_rng(H + W)
    bgra = rng.integers(0, 256, (H, W, 4), dtype=np.uint8)
    pred = rng.random((H // 2, W // 2, 3)).astype(np.float32)
    pred[0, 0] = [-0.25, 1.5, 0.5 / 255]  # clamping and a half-way product
    mask = (rng.random((H, W)) < 0.3).astype(np.uint8)
    mask[0, 0] = 1
    out = eng.post_frame(torch.from_numpy(bgra).cuda(), torch.from_numpy(pred).cuda(), torch.from_numpy(mask).cuda())
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), pp.post(bgra, pred, mask))


def test_post_in_place_and_empty_mask(eng):
    rng = np.random.default_rng(9)
    bgra = rng.integers(0, 256, (32, 64, 4), dtype=np.uint8)
    pred = rng.random((16, 32, 3)).astype(np.float32)
    mask = np.zeros((32, 64), np.uint8)
    f = torch.from_numpy(bgra).cuda()
    out = eng.post_frame(f, torch.from_numpy(pred).cuda(), torch.from_numpy(mask).cuda(), out=f)
    torch.cuda.synchronize()
    assert out.data_ptr() == f.data_ptr() and np.array_equal(out.cpu().numpy(), bgra)


def test_prepost_rejects_bad_arguments(eng):
    from paper_2509_10466_amd._lib import DrError
    f = torch.zeros((33, 64, 4), dtype=torch.uint8, device="cuda")
    with pytest.raises(DrError):
        eng.prep_frame(f)  # odd height
    g = torch.zeros((32, 64, 4), dtype=torch.uint8, device="cuda")
    with pytest.raises(DrError):
        eng.prep_frame(g, radius=17)
    h = torch.zeros((32, 66, 4), dtype=torch.uint8, device="cuda")
    with pytest.raises(DrError):
        eng.post_frame(h, torch.zeros((16, 33, 3), device="cuda"), torch.zeros((32, 66), dtype=torch.uint8, device="cuda"))
