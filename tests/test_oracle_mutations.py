"""The pins have teeth: plant a plausible mistake in the oracle (on the CPU, via monkeypatch)
and check that the comparison with the independent torch reference catches it."""
import numpy as np
import pytest
from scipy.special import erf

import drsynth
from oracle import network as on
from tests.test_oracle_pins import SMALL, small_inputs
from tests.torchref import reference_forward


def _no_scale_mha(q, k, v, heads, chunk=64):
    C = q.shape[-1]
    return _orig_mha(q * np.sqrt(C // heads), k, v, heads, chunk)


def _unbiased_ln(x, g, b, eps=1e-5):
    mu = x.mean(-1, keepdims=True)
    var = x.var(-1, ddof=1, keepdims=True)
    return (x - mu) / np.sqrt(var + eps) * g + b


def _tanh_gelu(z):
    return 0.5 * z * (1 + np.tanh(np.sqrt(2 / np.pi) * (z + 0.044715 * z ** 3)))


def _transposed_linear(x, w, b):
    return x @ (w if w.shape[0] == w.shape[1] else w.T) + b


def _wrong_windows(x, cfg):
    B, T, Ht, Wt, C = x.shape
    S = cfg.window_tokens
    return x.reshape(B, T // cfg.win_t, Ht // cfg.win_h, Wt // cfg.win_w, S, C)


def _wrong_unwindows(xw, cfg):
    B, nT, nH, nW, S, C = xw.shape
    return xw.reshape(B, nT * cfg.win_t, nH * cfg.win_h, nW * cfg.win_w, C)


def _flipped_decoder(z, wd, bd, p):
    return _orig_dec(z, np.asarray(wd).transpose(0, 1, 3, 2), bd, p)


def _and_flags(masks, p):
    B, T, H, W = masks.shape
    return (masks != 0).reshape(B, T, H // p, p, W // p, p).all(axis=(3, 5))


def _erf_gelu_wrong_sign(z):
    return 0.5 * z * (1.0 - erf(z / np.sqrt(2.0)))


_orig_mha = on.multi_head_attention
_orig_dec = on.decode_logits

MUTATIONS = {
    "attention scale dropped": ("multi_head_attention", _no_scale_mha),
    "unbiased LN variance": ("layer_norm", _unbiased_ln),
    "tanh GELU": ("gelu", _tanh_gelu),
    "GELU sign": ("gelu", _erf_gelu_wrong_sign),
    "transposed square weights": ("linear", _transposed_linear),
    "window partition without transpose": ("to_windows", _wrong_windows),
    "decoder kernel transposed": ("decode_logits", _flipped_decoder),
    "AND token flags": ("token_flags", _and_flags),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, monkeypatch):
    attr, fn = MUTATIONS[name]
    monkeypatch.setattr(on, attr, fn)
    if attr == "to_windows":
        monkeypatch.setattr(on, "from_windows", _wrong_unwindows)
    cfg = SMALL
    frames, masks = small_inputs(13)
    W = drsynth.make_weights(cfg, 3, std=0.2)
    d = on.forward_detail(frames, masks, W, cfg)
    out, pred, flags = reference_forward(frames, masks, W, cfg)
    same = (np.array_equal(d["flags"], flags) and np.allclose(d["pred"], pred, rtol=1e-11, atol=1e-12)
            and np.allclose(d["out"], out, rtol=1e-11, atol=1e-12))
    assert not same, f"planted mistake '{name}' went unnoticed"
