"""Seeded synthetic inputs for the inpainting path: network shapes, frames, masks, weights.

This module holds no arithmetic of the inpainting method itself.  It only draws the
inputs that both the FP64 oracle and the GPU library consume, so that the two sides
see bit-identical frames, masks and FP32 master weights.

Workload shapes (all random numbers come from NumPy's PCG64 ``default_rng(seed)``):

* ``tiny64``  -- one 64x64 RGB frame, patch 4 (16x16 tokens), dim 64, 2 heads, 2 blocks,
  8x8x1 token windows.  Frame = (uniform noise + smooth per-channel plane) / 2; the mask is
  one random rectangle covering about 15 % of the pixels.
* ``clip240`` -- a 5-frame clip at 240x432, dim 256, 4 heads, 8 blocks, 5x9x5 windows
  (225 tokens).  Frame = panning Perlin background with three moving rectangular objects;
  masks = random-walk brush strokes anchored on the objects, dilated 7 px.
* ``clip480`` -- 480x864 frames on the ``clip240`` network.
* ``clip720`` -- 5 frames at 720x1280, dim 384, 6 heads, 12 blocks, 6x10x5 windows (300
  tokens).

The mask recipe follows the thesis's training-mask description (Methods, "Mask
generation": random strokes, stable or moving with the object, dilated to a coverage
range); the coverage range used here is 10-40 % for clips and 5-40 % for served streams.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "NetCfg", "NETS", "SHAPES", "weight_order", "make_weights", "tiny_frame",
    "Scene", "make_clip", "make_clip_batch",
]


@dataclasses.dataclass(frozen=True)
class NetCfg:
    """Network hyper-parameters.  ``dim`` = C, ``heads`` = h, ``blocks`` = L, ``mlp_ratio`` = r,
    ``patch`` = p (conv kernel = stride), window = win_t x win_h x win_w tokens.  ``attn``:
    "joint" (every block attends over the whole window) or "decoupled" (even blocks attend
    within one frame of the window, odd blocks across its frames at one token position).
    ``overlap``: the patch embedding and the decoder use kernel 2p at stride p with p/2
    padding (neighbouring patches overlap, and the decoder sums the overlaps) instead of
    kernel p."""
    dim: int
    heads: int
    blocks: int
    mlp_ratio: int
    patch: int
    win_h: int
    win_w: int
    win_t: int
    attn: str = "joint"
    overlap: bool = False

    @property
    def kernel(self) -> int:
        """Kernel size of the patch embedding and the decoder."""
        return 2 * self.patch if self.overlap else self.patch

    @property
    def head_dim(self) -> int:
        return self.dim // self.heads

    @property
    def window_tokens(self) -> int:
        return self.win_h * self.win_w * self.win_t


NETS = {
    "tiny64": NetCfg(dim=64, heads=2, blocks=2, mlp_ratio=4, patch=4, win_h=8, win_w=8, win_t=1),
    "clip240": NetCfg(dim=256, heads=4, blocks=8, mlp_ratio=4, patch=4, win_h=5, win_w=9, win_t=5),
    "clip720": NetCfg(dim=384, heads=6, blocks=12, mlp_ratio=4, patch=4, win_h=6, win_w=10, win_t=5),
    "clip240_dec": NetCfg(dim=256, heads=4, blocks=8, mlp_ratio=4, patch=4, win_h=5, win_w=9, win_t=5,
                          attn="decoupled"),
    "clip240_ovl": NetCfg(dim=256, heads=4, blocks=8, mlp_ratio=4, patch=4, win_h=5, win_w=9, win_t=5,
                          overlap=True),
}

# (net name, B, T, H, W) of each named workload.
SHAPES = {
    "tiny64": ("tiny64", 1, 1, 64, 64),
    "clip240": ("clip240", 1, 5, 240, 432),
    "clip480": ("clip240", 1, 5, 480, 864),
    "clip720": ("clip720", 1, 5, 720, 1280),
}


# --------------------------------------------------------------------------------------------
# Weights
# --------------------------------------------------------------------------------------------

def weight_order(cfg: NetCfg):
    """(name, shape) of every parameter in draw order.

    Linear weights are [out, in]; the patch-embed conv is OIHW [C, 3, k, k]; the
    transposed-conv decoder is IOHW [C, 3, k, k] (k = cfg.kernel)."""
    C, p, R = cfg.dim, cfg.kernel, cfg.mlp_ratio * cfg.dim
    out = [("embed.w", (C, 3, p, p)), ("embed.b", (C,))]
    for l in range(cfg.blocks):
        b = f"blk{l}."
        out += [
            (b + "ln1.g", (C,)), (b + "ln1.b", (C,)),
            (b + "wq", (C, C)), (b + "bq", (C,)),
            (b + "wk", (C, C)), (b + "bk", (C,)),
            (b + "wv", (C, C)), (b + "bv", (C,)),
            (b + "wo", (C, C)), (b + "bo", (C,)),
            (b + "ln2.g", (C,)), (b + "ln2.b", (C,)),
            (b + "w1", (R, C)), (b + "b1", (R,)),
            (b + "w2", (C, R)), (b + "b2", (C,)),
        ]
    out += [("lnf.g", (C,)), ("lnf.b", (C,)), ("dec.w", (C, 3, p, p)), ("dec.b", (3,))]
    return out


def make_weights(cfg: NetCfg, seed: int = 0, std: float = 0.02, qk_std: float | None = None):
    """FP32 master weights drawn from N(0, std^2) in ``weight_order``; LayerNorm gains are
    1 + N(0, std^2).  ``qk_std`` (the "stress" set) redraws Wq and Wk with a larger std so the
    softmax is peaked."""
    rng = np.random.default_rng(seed)
    w = {}
    for name, shape in weight_order(cfg):
        s = std
        if qk_std is not None and (name.endswith(".wq") or name.endswith(".wk")):
            s = qk_std
        a = rng.standard_normal(shape) * s
        if name.endswith(".g"):
            a = a + 1.0
        w[name] = a.astype(np.float32)
    return w


# --------------------------------------------------------------------------------------------
# tiny64 frames
# --------------------------------------------------------------------------------------------

def tiny_frame(seed: int = 0, H: int = 64, W: int = 64, coverage: float = 0.15):
    """One frame [1,1,H,W,3] f32 and its mask [1,1,H,W] u8 (1 = private pixel)."""
    rng = np.random.default_rng(seed)
    u = rng.random((H, W, 3))
    yy, xx = np.mgrid[0:H, 0:W]
    g = np.empty((H, W, 3))
    for c in range(3):
        a, b, cc = rng.random(3)
        plane = a + b * xx / W + cc * yy / H
        lo, hi = plane.min(), plane.max()
        g[..., c] = (plane - lo) / (hi - lo) if hi > lo else 0.0
    frame = ((u + g) / 2).astype(np.float32)
    area = coverage * H * W
    aspect = rng.uniform(0.5, 2.0)
    rh = max(1, min(H, int(round(math.sqrt(area * aspect)))))
    rw = max(1, min(W, int(round(area / rh))))
    y0 = int(rng.integers(0, H - rh + 1))
    x0 = int(rng.integers(0, W - rw + 1))
    mask = np.zeros((H, W), np.uint8)
    mask[y0:y0 + rh, x0:x0 + rw] = 1
    return frame[None, None], mask[None, None]


# --------------------------------------------------------------------------------------------
# Perlin-textured moving scenes with stroke masks
# --------------------------------------------------------------------------------------------

_GRADS = np.array([[1, 0], [-1, 0], [0, 1], [0, -1],
                   [1, 1], [-1, 1], [1, -1], [-1, -1]], np.float64)
_GRADS[4:] /= math.sqrt(2.0)


def _fade(t):
    # Perlin's improved-noise interpolant 6t^5 - 15t^4 + 10t^3 (Perlin, SIGGRAPH 2002).
    return t * t * t * (t * (t * 6 - 15) + 10)


def _gradient_noise(xs, ys, perm):
    """2-D improved Perlin gradient noise on the grid of column coordinates ``xs`` (1-D) and
    row coordinates ``ys`` (1-D), in lattice units.  Returns [len(ys), len(xs)]."""
    xi = np.floor(xs).astype(np.int64)
    yi = np.floor(ys).astype(np.int64)
    xf = (xs - xi)[None, :]
    yf = (ys - yi)[:, None]
    u = _fade(xf)
    v = _fade(yf)
    gx_t, gy_t = _GRADS[:, 0], _GRADS[:, 1]

    def corner(ix, iy, dx, dy):
        h = perm[(perm[ix & 255][None, :] + iy[:, None]) & 255] & 7
        return gx_t[h] * dx + gy_t[h] * dy

    n00 = corner(xi, yi, xf, yf)
    n10 = corner(xi + 1, yi, xf - 1, yf)
    n01 = corner(xi, yi + 1, xf, yf - 1)
    n11 = corner(xi + 1, yi + 1, xf - 1, yf - 1)
    nx0 = n00 + u * (n10 - n00)
    nx1 = n01 + u * (n11 - n01)
    return nx0 + v * (nx1 - nx0)


def _reflect(p, lo, hi):
    """Position p bounced between lo and hi (triangle wave)."""
    span = hi - lo
    if span <= 0:
        return np.full_like(p, lo)
    q = np.mod(p - lo, 2 * span)
    return lo + np.where(q > span, 2 * span - q, q)


class Scene:
    """An endless synthetic video: panning Perlin background (4 octaves, base period 64 px,
    persistence 0.5, per-channel offsets) with three moving rectangular objects (side 8-25 %
    of the width, solid colour plus 0.05 Gaussian noise, 2-6 px/frame, bouncing off the
    borders).  The private mask is a set of random-walk brush strokes (step 6-14 px, heading
    change N(0, 0.6 rad), brush radius 3-8 px) anchored on the objects and moving with them,
    dilated by a 7 px disc; strokes are added until every one of the first ``cover_frames``
    frames reaches the target coverage.

    ``frame(t)`` -> [H, W, 3] float32 in [0, 1];  ``mask(t)`` -> [H, W] uint8 in {0, 1}."""

    def __init__(self, seed: int, H: int, W: int, coverage: float | None = None,
                 cov_range=(0.10, 0.40), cover_frames: int = 5, dilate: int = 7):
        self.H, self.W = H, W
        rng = np.random.default_rng(seed)
        self.perm = rng.permutation(256).astype(np.int64)
        self.offsets = rng.uniform(0, 256, size=(3, 2))
        ang = rng.uniform(0, 2 * math.pi)
        speed = rng.uniform(1, 3)
        self.pan = np.array([speed * math.cos(ang), speed * math.sin(ang)])
        self.objects = []
        for _ in range(3):
            ow = int(rng.uniform(0.08, 0.25) * W)
            oh = int(rng.uniform(0.08, 0.25) * W)
            oh = min(oh, H - 1)
            ow = min(ow, W - 1)
            x0 = rng.uniform(0, W - ow)
            y0 = rng.uniform(0, H - oh)
            a = rng.uniform(0, 2 * math.pi)
            s = rng.uniform(2, 6)
            colour = rng.random(3)
            self.objects.append(dict(w=ow, h=oh, x0=x0, y0=y0, vx=s * math.cos(a),
                                     vy=s * math.sin(a), colour=colour,
                                     noise_seed=int(rng.integers(0, 2 ** 31))))
        self.coverage = float(rng.uniform(*cov_range)) if coverage is None else float(coverage)
        self._norm = None
        self._raw_cache = {}
        self._mask_cache = {}
        self.strokes = []  # (object index, rasterised stroke relative to the object origin)
        self._build_strokes(rng, cover_frames, dilate)

    # -- geometry ---------------------------------------------------------------------------
    def object_origin(self, k, t):
        o = self.objects[k]
        x = _reflect(np.asarray(o["x0"] + o["vx"] * t, np.float64), 0.0, self.W - o["w"])
        y = _reflect(np.asarray(o["y0"] + o["vy"] * t, np.float64), 0.0, self.H - o["h"])
        return float(x), float(y)

    # -- background ---------------------------------------------------------------------------
    def _background_raw(self, t):
        H, W = self.H, self.W
        xs = np.arange(W, dtype=np.float64) + self.pan[0] * t
        ys = np.arange(H, dtype=np.float64) + self.pan[1] * t
        out = np.zeros((H, W, 3))
        for c in range(3):
            acc = np.zeros((H, W))
            amp, period = 1.0, 64.0
            for _ in range(4):
                acc += amp * _gradient_noise(xs / period + self.offsets[c, 0],
                                             ys / period + self.offsets[c, 1], self.perm)
                amp *= 0.5
                period /= 2.0
            out[..., c] = acc
        return out

    def _normaliser(self):
        if self._norm is None:
            # Min-max over the first five frames (fixed for the whole video).
            self._raw_cache = {t: self._background_raw(t) for t in range(5)}
            stack = np.stack([self._raw_cache[t] for t in range(5)])
            lo = stack.min(axis=(0, 1, 2))
            hi = stack.max(axis=(0, 1, 2))
            self._norm = (lo, np.where(hi > lo, hi - lo, 1.0))
        return self._norm

    def frame(self, t: int) -> np.ndarray:
        lo, span = self._normaliser()
        raw = self._raw_cache.get(t) if t in self._raw_cache else self._background_raw(t)
        img = np.clip((raw - lo) / span, 0.0, 1.0)
        for k, o in enumerate(self.objects):
            x, y = self.object_origin(k, t)
            xi, yi = int(round(x)), int(round(y))
            nrng = np.random.default_rng(o["noise_seed"] + 7919 * t)
            patch = o["colour"][None, None, :] + 0.05 * nrng.standard_normal((o["h"], o["w"], 3))
            img[yi:yi + o["h"], xi:xi + o["w"]] = np.clip(patch, 0.0, 1.0)[: self.H - yi, : self.W - xi]
        return img.astype(np.float32)

    # -- masks --------------------------------------------------------------------------------
    def _stroke(self, rng):
        k = int(rng.integers(0, len(self.objects)))
        o = self.objects[k]
        p = np.array([rng.uniform(0, o["w"]), rng.uniform(0, o["h"])])
        heading = rng.uniform(0, 2 * math.pi)
        pts = [p.copy()]
        for _ in range(int(rng.integers(4, 13))):
            heading += rng.normal(0.0, 0.6)
            step = rng.uniform(6, 14)
            q = p + step * np.array([math.cos(heading), math.sin(heading)])
            n = max(1, int(math.ceil(step / 2.0)))
            for s in range(1, n + 1):
                pts.append(p + (q - p) * s / n)
            p = q
        return k, np.array(pts), float(rng.uniform(3, 8))

    @staticmethod
    def _bitmap(pts, radius):
        """Rasterise the union of discs of radius ``radius`` centred on ``pts`` (coordinates
        relative to the object's integer origin).  Returns (x0, y0, bool bitmap)."""
        ri = int(math.ceil(radius))
        x0 = int(math.floor(pts[:, 0].min())) - ri
        y0 = int(math.floor(pts[:, 1].min())) - ri
        x1 = int(math.ceil(pts[:, 0].max())) + ri + 1
        y1 = int(math.ceil(pts[:, 1].max())) + ri + 1
        yy, xx = np.mgrid[y0:y1, x0:x1].astype(np.float64)
        bm = np.zeros(xx.shape, bool)
        r2 = radius * radius
        for px, py in pts:
            cx0, cx1 = int(math.floor(px - ri)) - x0, int(math.ceil(px + ri)) + 1 - x0
            cy0, cy1 = int(math.floor(py - ri)) - y0, int(math.ceil(py + ri)) + 1 - y0
            sub = (xx[cy0:cy1, cx0:cx1] - px) ** 2 + (yy[cy0:cy1, cx0:cx1] - py) ** 2 <= r2
            bm[cy0:cy1, cx0:cx1] |= sub
        return x0, y0, bm

    def _paint(self, canvas, k, stamp, t):
        """OR a stroke bitmap into ``canvas``, placed on object k's integer origin at frame t."""
        H, W = canvas.shape
        bx, by, bm = stamp
        ox, oy = self.object_origin(k, t)
        X0 = int(round(ox)) + bx
        Y0 = int(round(oy)) + by
        h, w = bm.shape
        xa, ya = max(0, X0), max(0, Y0)
        xb, yb = min(W, X0 + w), min(H, Y0 + h)
        if xa >= xb or ya >= yb:
            return
        canvas[ya:yb, xa:xb] |= bm[ya - Y0:yb - Y0, xa - X0:xb - X0]

    def _build_strokes(self, rng, cover_frames, dilate):
        # Dilating a union of discs by a disc of radius d is the union of the discs grown by d,
        # so each stroke is painted with radius (brush + dilate).
        canv = [np.zeros((self.H, self.W), bool) for _ in range(cover_frames)]
        counts = [0] * cover_frames
        target = self.coverage * self.H * self.W
        for _ in range(20000):
            if min(counts) >= target:
                break
            k, pts, r = self._stroke(rng)
            stamp = self._bitmap(pts, r + dilate)
            self.strokes.append((k, stamp))
            for t in range(cover_frames):
                self._paint(canv[t], k, stamp, t)
                counts[t] = int(canv[t].sum())
        self._mask_cache = {t: canv[t].astype(np.uint8) for t in range(cover_frames)}

    def mask(self, t: int) -> np.ndarray:
        if t in self._mask_cache:
            return self._mask_cache[t].copy()
        canvas = np.zeros((self.H, self.W), bool)
        for k, stamp in self.strokes:
            self._paint(canvas, k, stamp, t)
        return canvas.astype(np.uint8)


def make_clip(seed: int, T: int, H: int, W: int, coverage: float | None = None,
              cov_range=(0.10, 0.40)):
    """One clip: frames [1,T,H,W,3] f32, masks [1,T,H,W] u8, target coverage."""
    sc = Scene(seed, H, W, coverage=coverage, cov_range=cov_range, cover_frames=T)
    frames = np.stack([sc.frame(t) for t in range(T)])[None]
    masks = np.stack([sc.mask(t) for t in range(T)])[None]
    return frames, masks, sc.coverage


def make_clip_batch(seeds, T, H, W):
    """Clips for several seeds stacked along the batch axis."""
    fs, ms = [], []
    for s in seeds:
        f, m, _ = make_clip(s, T, H, W)
        fs.append(f)
        ms.append(m)
    return np.concatenate(fs), np.concatenate(ms)


def make_workload(name: str, seed: int = 0):
    """(cfg, frames, masks) for a named workload shape."""
    net, B, T, H, W = SHAPES[name]
    cfg = NETS[net]
    if name == "tiny64":
        frames, masks = tiny_frame(seed, H, W)
    else:
        frames, masks = make_clip_batch(range(seed, seed + B), T, H, W)
    return cfg, frames, masks
