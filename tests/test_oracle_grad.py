"""Pins of the oracle's analytic gradient: FP64 central finite differences along seeded
random parameter directions, and torch FP64 autograd of the independent reference."""
import numpy as np
import pytest
import torch

import drsynth
from oracle import grad as og
from oracle import network as on
from tests.test_oracle_pins import SMALL, small_inputs
from tests.torchref import reference_forward_t


def _flat(G, names):
    return np.concatenate([np.asarray(G[n], np.float64).ravel() for n in names])


def _unflat(vec, W):
    out, o = {}, 0
    for n, a in W.items():
        out[n] = vec[o:o + a.size].reshape(a.shape)
        o += a.size
    return out


def test_loss_hand_example():
    """Two pixels, one masked: |0.9-0.5| on the masked 3 values, |0.2-0.4| on the rest."""
    import json, os
    fx = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "l1_loss_example.json")))
    pred = np.array(fx["pred"], np.float64)
    gt = np.array(fx["gt"], np.float64)
    m = np.array(fx["mask"], np.uint8)
    L, g = og.l1_loss(pred, gt, m)
    assert abs(L - fx["loss"]) < 1e-15
    np.testing.assert_allclose(g, np.array(fx["dloss_dpred"]), atol=1e-15)


def test_gradient_matches_torch_autograd():
    cfg = SMALL
    frames, masks = small_inputs(21)
    W = drsynth.make_weights(cfg, 4, std=0.2)
    L, G = og.loss_and_grad(frames, masks, W, cfg)
    Wt = {k: torch.tensor(np.asarray(v, np.float64), requires_grad=True) for k, v in W.items()}
    _, pred, _ = reference_forward_t(frames, masks, Wt, cfg)
    gt = torch.from_numpy(frames.astype(np.float64))
    inside = torch.from_numpy(np.repeat(masks[..., None] != 0, 3, axis=-1))
    e = (pred - gt).abs()
    Lt = e[inside].mean() + 0.1 * e[~inside].mean()
    Lt.backward()
    assert abs(float(Lt) - L) < 1e-12
    for k in W:
        np.testing.assert_allclose(G[k], Wt[k].grad.numpy(), rtol=1e-9, atol=1e-12, err_msg=k)


@pytest.mark.parametrize("ndir,seed", [(200, 0)])
def test_gradient_finite_differences_tiny64(ndir, seed):
    """Analytic FP64 gradient vs central differences (h = 1e-6) along `ndir` seeded unit
    directions in parameter space, on the 64x64 single-frame network."""
    cfg = drsynth.NETS["tiny64"]
    frames, masks = drsynth.tiny_frame(0)
    W = {k: v.astype(np.float64) for k, v in drsynth.make_weights(cfg, 0).items()}
    L0, G = og.loss_and_grad(frames, masks, W, cfg)
    names = list(W)
    g = _flat(G, names)
    theta = _flat(W, names)
    rng = np.random.default_rng(seed)
    h = 1e-6
    sign0 = np.sign(on.forward_detail(frames, masks, W, cfg)["pred"] - frames)
    checked = 0
    while checked < ndir:
        v = rng.standard_normal(theta.size)
        v /= np.linalg.norm(v)
        Wp, Wm = _unflat(theta + h * v, W), _unflat(theta - h * v, W)
        dp = on.forward_detail(frames, masks, Wp, cfg)["pred"]
        dm = on.forward_detail(frames, masks, Wm, cfg)["pred"]
        if not (np.array_equal(np.sign(dp - frames), sign0) and np.array_equal(np.sign(dm - frames), sign0)):
            continue  # an L1 kink inside [-h, h]: redraw
        lp = og.l1_loss(dp, frames, masks)[0]
        lm = og.l1_loss(dm, frames, masks)[0]
        fd = (lp - lm) / (2 * h)
        an = float(g @ v)
        # relative 1e-6, plus the rounding floor of an FP64 central difference:
        # |L| * 2^-52 / h ~ 3e-11 for L ~ 0.15, h = 1e-6 (floor taken at 1e-10)
        assert abs(an - fd) <= 1e-6 * abs(an) + 1e-10, (checked, an, fd)
        checked += 1
