"""GPU reverse pass against the oracle's FP64 analytic gradient, the autograd wrapper, and
determinism."""
import sys

import numpy as np
import pytest

import drsynth
from oracle import grad as og
from tests.gpu_util import MID, case_inputs

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


def _gpu_grad(eng, frames, masks):
    f = torch.from_numpy(frames).cuda()
    m = torch.from_numpy(masks).cuda()
    pred, saved = eng.train_forward(f, m)
    loss, dpred = eng.l1_loss(pred, f, m)
    g = eng.train_backward(saved, dpred)
    torch.cuda.synchronize()
    saved.close()
    return float(loss.item()), g.cpu().numpy().astype(np.float64), pred.cpu().numpy()


def _flat(cfg, G):
    from paper_2509_10466_amd.api import _shapes
    return np.concatenate([np.asarray(G[n], np.float64).ravel() for n, _ in _shapes(cfg)])


@pytest.mark.parametrize("case", ["tiny64", "mid"])
def test_backward_matches_oracle_gradient(dev, case):
    from paper_2509_10466_amd import Inpainter
    cfg, frames, masks = case_inputs(case)
    W = drsynth.make_weights(cfg, 0)
    eng = Inpainter(cfg, W)
    L, g, pred = _gpu_grad(eng, frames, masks)
    Lr, Gr = og.loss_and_grad(frames, masks, W, cfg)
    gr = _flat(cfg, Gr)
    _say(f"[grad] {case}: loss gpu {L:.7f} oracle {Lr:.7f}; |g| {np.linalg.norm(gr):.4e}")
    assert abs(L - Lr) <= 1e-5 * abs(Lr)
    rel = np.linalg.norm(g - gr) / np.linalg.norm(gr)
    _say(f"    normwise relative error {rel:.3e}")
    assert rel <= 1e-3
    rng = np.random.default_rng(0)
    worst = 0.0
    for _ in range(200):
        v = rng.standard_normal(g.size)
        v /= np.linalg.norm(v)
        err = abs(g @ v - gr @ v) / np.linalg.norm(gr)
        worst = max(worst, err)
    _say(f"    worst directional error / |g| {worst:.3e}")
    assert worst <= 1e-3
    eng.close()


def test_backward_is_deterministic(dev):
    from paper_2509_10466_amd import Inpainter
    cfg, frames, masks = case_inputs("mid_b2")
    eng = Inpainter(cfg, drsynth.make_weights(cfg, 0))
    _, g1, _ = _gpu_grad(eng, frames, masks)
    _, g2, _ = _gpu_grad(eng, frames, masks)
    assert np.array_equal(g1, g2)
    eng.close()


def test_autograd_function_and_sgd_step(dev):
    """loss.backward() through InpaintFn fills params.grad with the library's gradient, and a
    small step against it lowers the loss."""
    from paper_2509_10466_amd import Inpainter
    from paper_2509_10466_amd.api import InpaintFn, flatten_params
    cfg, frames, masks = case_inputs("mid")
    W = drsynth.make_weights(cfg, 0)
    eng = Inpainter(cfg, W)
    f = torch.from_numpy(frames).cuda()
    m = torch.from_numpy(masks).cuda()
    params = flatten_params(cfg, W).cuda().requires_grad_(True)
    inside = (m != 0).unsqueeze(-1).expand_as(f)

    def loss_of(pred):
        e = (pred - f).abs()
        return e[inside].mean() + 0.1 * e[~inside].mean()

    pred = InpaintFn.apply(f, m, params, eng)
    loss = loss_of(pred)
    loss.backward()
    pred_d, saved = eng.train_forward(f, m)
    direct = eng.train_backward(saved, eng.l1_loss(pred_d, f, m)[1])
    torch.cuda.synchronize()
    saved.close()
    rel = float((params.grad - direct).norm() / direct.norm())
    assert rel < 1e-5, rel
    with torch.no_grad():
        stepped = params - 0.05 * params.grad / params.grad.norm()
    loss2 = loss_of(InpaintFn.apply(f, m, stepped, eng))
    _say(f"loss {float(loss):.6f} -> {float(loss2):.6f} after one normalised step")
    assert float(loss2) < float(loss)
    eng.close()


# ------------------------------------------------------------------------------------------
# mixed precision: bf16 operands, FP32 accumulation, FP32 master weights and gradients
# ------------------------------------------------------------------------------------------
# Every weight product rounds both operands to bf16 (unit roundoff u = 2^-9); a gradient entry
# of a 2-block network passes through about ten such products in the forward and reverse
# passes, so its relative error is bounded by roughly 10 * 2u = 4e-2 (first order), and the
# rounding errors of different products are independent, so the normwise error sits well
# inside that.  The forward prediction is held to the BF16 inference bound.
BF16_GRAD_TOL = 4e-2


@pytest.mark.parametrize("case", ["tiny64", "mid"])
def test_bf16_backward_matches_oracle_gradient(dev, case):
    from paper_2509_10466_amd import Inpainter
    cfg, frames, masks = case_inputs(case)
    W = drsynth.make_weights(cfg, 0)
    eng = Inpainter(cfg, W)
    _, _, pred32 = _gpu_grad(eng, frames, masks)
    eng.train_precision("bf16")
    L, g, pred = _gpu_grad(eng, frames, masks)
    Lr, Gr = og.loss_and_grad(frames, masks, W, cfg)
    gr = _flat(cfg, Gr)
    assert np.abs(pred - pred32).max() <= 2e-2
    assert abs(L - Lr) <= 1e-2 * abs(Lr)
    rel = np.linalg.norm(g - gr) / np.linalg.norm(gr)
    cos = float(g @ gr / (np.linalg.norm(g) * np.linalg.norm(gr)))
    _say(f"[bf16 grad] {case}: loss gpu {L:.7f} oracle {Lr:.7f}; normwise relative error {rel:.3e}, cosine {cos:.6f}")
    assert rel <= BF16_GRAD_TOL
    eng.train_precision("fp32")
    _, g32, _ = _gpu_grad(eng, frames, masks)
    assert np.linalg.norm(g32 - gr) / np.linalg.norm(gr) <= 1e-3  # switching back restores FP32
    eng.close()


def test_bf16_backward_is_deterministic(dev):
    from paper_2509_10466_amd import Inpainter
    cfg, frames, masks = case_inputs("mid_b2")
    eng = Inpainter(cfg, drsynth.make_weights(cfg, 0))
    eng.train_precision("bf16")
    _, g1, _ = _gpu_grad(eng, frames, masks)
    _, g2, _ = _gpu_grad(eng, frames, masks)
    assert np.array_equal(g1, g2)
    eng.close()


def test_train_precision_rejects_fp8(dev):
    from paper_2509_10466_amd import Inpainter
    from paper_2509_10466_amd._lib import DrError
    cfg, _, _ = case_inputs("tiny64")
    eng = Inpainter(cfg, drsynth.make_weights(cfg, 0))
    with pytest.raises(DrError, match="DR_EINVAL"):
        eng.train_precision("fp8")
    eng.close()


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_backward_clip720_network(dev, precision):
    """The 384-dim, 12-block network with 300-key windows (6 x 10 x 5), on a 5 x 48 x 80 clip
    (2 x 2 windows), against the oracle's FP64 gradient."""
    from paper_2509_10466_amd import Inpainter
    cfg = drsynth.NETS["clip720"]
    frames, masks, _ = drsynth.make_clip(5, 5, 48, 80, cov_range=(0.2, 0.4))
    W = drsynth.make_weights(cfg, 0)
    eng = Inpainter(cfg, W)
    eng.train_precision(precision)
    L, g, _ = _gpu_grad(eng, frames, masks)
    Lr, Gr = og.loss_and_grad(frames, masks, W, cfg)
    gr = _flat(cfg, Gr)
    rel = np.linalg.norm(g - gr) / np.linalg.norm(gr)
    _say(f"[grad clip720 net] {precision}: loss gpu {L:.7f} oracle {Lr:.7f}; normwise relative error {rel:.3e}")
    assert abs(L - Lr) <= (1e-5 if precision == "fp32" else 1e-2) * abs(Lr)
    # 12 blocks put about five bf16-operand products per block on a gradient's path; their
    # rounding errors (2u = 2^-8 each) are independent, so they add in quadrature:
    # 2u sqrt(60) ~ 3e-2, held at twice that
    assert rel <= (1e-3 if precision == "fp32" else 6e-2)
    eng.close()


# ------------------------------------------------------------------------------------------
# the training boundary: saved-activation handles and parameters loaded on the device
# ------------------------------------------------------------------------------------------
def test_two_forwards_then_one_backward_sum_gradients(dev):
    """Two InpaintFn applications (different clips) before a single backward: the gradient is
    the sum of the two separate gradients, because each application keeps its own handle."""
    from paper_2509_10466_amd import Inpainter
    from paper_2509_10466_amd.api import InpaintFn, flatten_params
    cfg = MID
    fa, ma, _ = drsynth.make_clip(3, 5, 40, 72, cov_range=(0.2, 0.4))
    fb, mb, _ = drsynth.make_clip(4, 5, 40, 72, cov_range=(0.2, 0.4))
    W = drsynth.make_weights(cfg, 0)
    eng = Inpainter(cfg, W)
    sep = []
    for f, m in ((fa, ma), (fb, mb)):
        _, g, _ = _gpu_grad(eng, f, m)
        sep.append(g)
    params = flatten_params(cfg, W).cuda().requires_grad_(True)
    losses = []
    for f, m in ((fa, ma), (fb, mb)):
        ft, mt = torch.from_numpy(f).cuda(), torch.from_numpy(m).cuda()
        pred = InpaintFn.apply(ft, mt, params, eng)
        inside = (mt != 0).unsqueeze(-1).expand_as(ft)
        e = (pred - ft).abs()
        losses.append(e[inside].mean() + 0.1 * e[~inside].mean())
    (losses[0] + losses[1]).backward()
    torch.cuda.synchronize()
    got = params.grad.cpu().numpy().astype(np.float64)
    want = sep[0] + sep[1]
    rel = np.linalg.norm(got - want) / np.linalg.norm(want)
    _say(f"[two forwards] relative difference to the summed gradients {rel:.3e}")
    assert rel < 1e-5
    eng.close()


def test_handle_keeps_the_weights_of_its_forward(dev):
    """A forward, then new parameters loaded, then that forward's backward: the gradient is the
    one at the forward's weights."""
    from paper_2509_10466_amd import Inpainter
    from paper_2509_10466_amd.api import flatten_params
    cfg, frames, masks = case_inputs("mid")
    W0 = drsynth.make_weights(cfg, 0)
    W1 = drsynth.make_weights(cfg, 1)
    eng = Inpainter(cfg, W0)
    _, g_ref, _ = _gpu_grad(eng, frames, masks)
    f = torch.from_numpy(frames).cuda()
    m = torch.from_numpy(masks).cuda()
    pred, saved = eng.train_forward(f, m)
    eng.load_params(flatten_params(cfg, W1).cuda())
    g = eng.train_backward(saved, eng.l1_loss(pred, f, m)[1])
    torch.cuda.synchronize()
    saved.close()
    assert np.array_equal(g.cpu().numpy().astype(np.float64), g_ref)
    eng.close()


def test_device_parameter_load_equals_blob_load(dev):
    """Inference after dr_load_params (flat parameters already on the device) is bitwise the
    inference after dr_load_weights of the same values, in every precision."""
    from paper_2509_10466_amd import Inpainter
    from paper_2509_10466_amd.api import flatten_params
    cfg, frames, masks = case_inputs("mid")
    W0 = drsynth.make_weights(cfg, 0)
    W1 = drsynth.make_weights(cfg, 1)
    a = Inpainter(cfg, W1)
    b = Inpainter(cfg, W0)
    b.load_params(flatten_params(cfg, W1).cuda())
    f = torch.from_numpy(frames).cuda()
    m = torch.from_numpy(masks).cuda()
    for prec in ("fp32", "bf16", "fp8"):
        oa = a(f, m, prec)
        ob = b(f, m, prec)
        torch.cuda.synchronize()
        assert torch.equal(oa, ob), prec
    a.close()
    b.close()


def test_training_step_copies_nothing_to_the_host(dev, monkeypatch):
    """An InpaintFn forward and backward with new parameters every step moves no tensor to host
    memory: the parameters go to the library as a device pointer."""
    from paper_2509_10466_amd import Inpainter
    from paper_2509_10466_amd.api import InpaintFn, flatten_params
    cfg, frames, masks = case_inputs("tiny64")
    W = drsynth.make_weights(cfg, 0)
    eng = Inpainter(cfg, W)
    f = torch.from_numpy(frames).cuda()
    m = torch.from_numpy(masks).cuda()
    params = flatten_params(cfg, W).cuda().requires_grad_(True)
    opt = torch.optim.SGD([params], lr=1e-3)

    def no_host(*a, **k):
        raise AssertionError("a tensor was copied to host memory")

    monkeypatch.setattr(torch.Tensor, "cpu", no_host)
    monkeypatch.setattr(torch.Tensor, "numpy", no_host)
    monkeypatch.setattr(torch.Tensor, "tolist", no_host)
    for _ in range(3):
        opt.zero_grad()
        pred = InpaintFn.apply(f, m, params, eng)
        (pred - f).abs().mean().backward()
        opt.step()
    monkeypatch.undo()
    torch.cuda.synchronize()
    assert torch.isfinite(params).all().item()
    eng.close()


def test_saved_handle_misuse_is_an_error(dev):
    from paper_2509_10466_amd import Inpainter
    cfg, frames, masks = case_inputs("tiny64")
    eng = Inpainter(cfg, drsynth.make_weights(cfg, 0))
    other = Inpainter(cfg, drsynth.make_weights(cfg, 0))
    f = torch.from_numpy(frames).cuda()
    m = torch.from_numpy(masks).cuda()
    pred, saved = eng.train_forward(f, m)
    dpred = eng.l1_loss(pred, f, m)[1]
    grads = torch.empty(eng.param_count(), dtype=torch.float32, device=f.device)
    # another context's handle is refused before any work is enqueued
    assert other.lib.dr_train_backward(other._ctx, saved.handle, dpred.data_ptr(), grads.data_ptr(), None) == 1
    st = other.lib.dr_saved_free(other._ctx, saved.handle)
    assert st == 1  # DR_EINVAL: not a handle of that context
    g1 = eng.train_backward(saved, dpred)
    g2 = eng.train_backward(saved, dpred)  # a live handle can be used again
    torch.cuda.synchronize()
    assert torch.equal(g1, g2)
    h = saved.handle
    saved.close()
    assert eng.lib.dr_saved_free(eng._ctx, h) == 1  # double free
    assert eng.lib.dr_train_backward(eng._ctx, h, dpred.data_ptr(), g1.data_ptr(), None) == 1
    eng.close()
    other.close()


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_backward_clip240_network_batch2(dev, precision):
    """The training network of the 4-clip workload (dim 256, 4 heads, 8 blocks, 225-key
    windows) on a batch of two 5 x 40 x 72 clips (2 x 2 windows each), against the oracle's
    FP64 gradient."""
    from paper_2509_10466_amd import Inpainter
    cfg = drsynth.NETS["clip240"]
    frames, masks = drsynth.make_clip_batch([7, 8], 5, 40, 72)
    W = drsynth.make_weights(cfg, 0)
    eng = Inpainter(cfg, W)
    eng.train_precision(precision)
    L, g, _ = _gpu_grad(eng, frames, masks)
    Lr, Gr = og.loss_and_grad(frames, masks, W, cfg)
    gr = _flat(cfg, Gr)
    rel = np.linalg.norm(g - gr) / np.linalg.norm(gr)
    _say(f"[grad clip240 net, batch 2] {precision}: loss gpu {L:.7f} oracle {Lr:.7f}; normwise relative error {rel:.3e}")
    assert abs(L - Lr) <= (1e-5 if precision == "fp32" else 1e-2) * abs(Lr)
    # eight blocks: about forty bf16-operand products on a gradient's path, 2u sqrt(40) ~ 2.5e-2
    assert rel <= (1e-3 if precision == "fp32" else 5e-2)
    eng.close()
