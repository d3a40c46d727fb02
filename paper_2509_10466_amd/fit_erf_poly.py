"""Coefficients of the polynomial erf used by the reduced-precision GELU epilogues
(csrc/dr_device.h, DR_ERF_P0..P8): erf x ~ x P(x^2) on [0, 3] with P of degree 8, by
iteratively reweighted least squares (Lawson's algorithm towards the minimax fit) on
Chebyshev nodes in x^2, rounded to FP32.  Prints the coefficients and the maximum error of
the FP32 Horner evaluation with the argument clamped to [-3, 3].

    python -m paper_2509_10466_amd.fit_erf_poly
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf

CLAMP = 3.0
DEGREE = 8


def fit(clamp: float = CLAMP, degree: int = DEGREE, nodes: int = 6000, iters: int = 60) -> np.ndarray:
    t = (np.cos(np.pi * (np.arange(nodes) + 0.5) / nodes) + 1.0) / 2.0 * clamp * clamp
    x = np.sqrt(t)
    V = np.vander(t, degree + 1, increasing=True) * x[:, None]
    y = erf(x)
    w = np.ones_like(t)
    c, *_ = np.linalg.lstsq(V, y, rcond=None)
    for _ in range(iters):
        w = w * np.sqrt(np.abs(V @ c - y) + 1e-30)
        w /= w.mean()
        c, *_ = np.linalg.lstsq(V * w[:, None], y * w, rcond=None)
    return c.astype(np.float32)


def max_error(c32: np.ndarray, clamp: float = CLAMP) -> float:
    x = np.linspace(0.0, 8.0, 2_000_001).astype(np.float32)
    xc = np.minimum(x, np.float32(clamp))
    t = (xc * xc).astype(np.float32)
    acc = np.full_like(t, c32[-1])
    for k in range(len(c32) - 2, -1, -1):
        acc = (acc.astype(np.float64) * t + np.float64(c32[k])).astype(np.float32)
    e = (xc * acc).astype(np.float64)
    return float(np.abs(e - erf(x.astype(np.float64))).max())


if __name__ == "__main__":
    c = fit()
    for k, v in enumerate(c):
        print(f"#define DR_ERF_P{k} {float(v)!r}f")
    print(f"max |error| of erf: {max_error(c):.3e}")
