"""The polynomial erf inside the reduced-precision GELU epilogues, evaluated on the CPU the way
the kernels evaluate it (FP32 Horner with fused multiply-adds), against scipy's erf: the
error bound stated next to the coefficients must hold over the whole real line."""
import os
import re

import numpy as np
from scipy.special import erf

HDR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2509_10466_amd", "csrc",
                   "dr_device.h")


def _consts():
    text = open(HDR).read()
    vals = dict(re.findall(r"#define (DR_ERF_\w+) ([-0-9.e+]+)f", text))
    coef = [np.float32(float(vals[f"DR_ERF_P{k}"])) for k in range(9)]
    return coef, np.float32(float(vals["DR_ERF_CLAMP"]))


def _fma32(a, b, c):
    # a*b is exact in double for float32 operands; one rounding to float32 after the add
    return (a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64)).astype(np.float32)


def _gelu_kernel(z):
    coef, clamp = _consts()
    z = z.astype(np.float32)
    x = np.clip((z * np.float32(0.70710678118654752)).astype(np.float32), -clamp, clamp)
    t = (x * x).astype(np.float32)
    p = _fma32(np.full_like(t, coef[8]), t, np.full_like(t, coef[7]))
    for k in range(6, -1, -1):
        p = _fma32(p, t, np.full_like(t, coef[k]))
    hz = (np.float32(0.5) * z).astype(np.float32)
    return _fma32(hz, (x * p).astype(np.float32), hz), (x * p).astype(np.float32)


def test_polynomial_erf_error_bound():
    x = np.linspace(-8.0, 8.0, 4_000_001)
    _, e = _gelu_kernel(x / np.float32(0.70710678118654752))
    err = np.abs(e.astype(np.float64) - erf(x))
    assert err.max() <= 2.8e-5, err.max()


def test_gelu_error_bound():
    z = np.linspace(-12.0, 12.0, 2_000_001)
    g, _ = _gelu_kernel(z)
    exact = 0.5 * z * (1.0 + erf(z / np.sqrt(2.0)))
    err = np.abs(g.astype(np.float64) - exact)
    # |erf error| / 2 times |z|, plus the FP32 rounding of the last steps
    assert np.all(err <= 1.4e-5 * np.abs(z) + 2e-7)
    assert err[np.abs(z) <= 6.0].max() <= 6e-5


def test_special_values():
    g, e = _gelu_kernel(np.array([0.0, 1e-6, -1e-6, 30.0, -30.0]))
    assert g[0] == 0.0 and e[0] == 0.0
    assert e[1] == -e[2]  # odd
    assert abs(g[3] - 30.0) < 30.0 * 1.4e-5 and abs(g[4]) < 30.0 * 1.4e-5
