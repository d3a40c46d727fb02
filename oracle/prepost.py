"""Pre- and post-processing around the network at camera resolution, FP64 / exact integer.

Test infrastructure only (see the package docstring).

The thesis runs its segmentation and inpainting models at 640x360 and scales their outputs by
2 to the 1280x720 camera frame, accepting slight pixelation inside inpainted regions and
slightly jagged object outlines (Methods, "Performance Optimisations -- Upscaling"); the
server takes the masks of the objects the user selected and cuts those objects out of the
frame (Methods, "Object Control"); the camera-to-tensor conversion is part of the measured
frame time (Results, memory-slot table) and CPU pre/post-processing is the largest part of
the inpainting stage (Results, system timing breakdown).

Readings taken where the description is silent (each is also the GPU path's definition):

* camera frame: u8 BGRA [H, W, 4]; the network input is RGB value / 255.
* private mask: the union of the selected per-object instance masks (nonzero = object),
  dilated by a square (2r + 1) x (2r + 1) window (r = 0: no dilation); pixels outside the
  frame do not contribute.
* downscale by 2: RGB is the mean of each 2 x 2 block; a low-resolution pixel is private if
  any of its 2 x 2 full-resolution pixels is (no private pixel is lost).
* upscale by 2: nearest neighbour (each low-resolution pixel covers its 2 x 2 block), the
  pixelation the thesis describes.
* composite at full resolution: private pixels get the upscaled prediction converted to u8
  as clamp(rint(255 * v), 0, 255), computed in float32 (the same precision as the GPU path,
  since it decides an integer), alpha copied; every other pixel is copied unchanged.
"""
from __future__ import annotations

import numpy as np

F64 = np.float64


def bgra_to_rgb(bgra: np.ndarray) -> np.ndarray:
    """u8 BGRA [H, W, 4] -> RGB [H, W, 3] in [0, 1], float64."""
    assert bgra.dtype == np.uint8 and bgra.shape[-1] == 4
    return bgra[..., [2, 1, 0]].astype(F64) / 255.0


def mask_union(instances: np.ndarray, select) -> np.ndarray:
    """u8 [K, H, W] instance masks and K selection flags -> u8 [H, W] (1 = private)."""
    K = instances.shape[0]
    out = np.zeros(instances.shape[1:], dtype=np.uint8)
    for k in range(K):
        if select[k]:
            out |= (instances[k] != 0).astype(np.uint8)
    return out


def dilate(mask: np.ndarray, r: int) -> np.ndarray:
    """Square (2r+1)^2 dilation of a 0/1 mask; pixels outside the frame do not contribute."""
    H, W = mask.shape
    out = np.zeros_like(mask)
    for y in range(H):
        for x in range(W):
            y0, y1 = max(0, y - r), min(H, y + r + 1)
            x0, x1 = max(0, x - r), min(W, x + r + 1)
            out[y, x] = 1 if mask[y0:y1, x0:x1].any() else 0
    return out


def downscale2(rgb: np.ndarray) -> np.ndarray:
    """Mean of 2 x 2 blocks: [H, W, 3] -> [H/2, W/2, 3]."""
    H, W, _ = rgb.shape
    return rgb.reshape(H // 2, 2, W // 2, 2, 3).mean(axis=(1, 3))


def downscale2_mask(mask: np.ndarray) -> np.ndarray:
    """Any of each 2 x 2 block: [H, W] -> [H/2, W/2]."""
    H, W = mask.shape
    return mask.reshape(H // 2, 2, W // 2, 2).max(axis=(1, 3))


def upscale2(img: np.ndarray) -> np.ndarray:
    """Nearest neighbour: [h, w, ...] -> [2h, 2w, ...]."""
    return np.repeat(np.repeat(img, 2, axis=0), 2, axis=1)


def to_u8(v: np.ndarray) -> np.ndarray:
    """clamp(rint(255 v), 0, 255) with the product and the rounding in float32."""
    q = np.rint(np.float32(255.0) * v.astype(np.float32))
    return np.clip(q, 0, 255).astype(np.uint8)


def prep(bgra: np.ndarray, instances: np.ndarray, select, r: int):
    """Camera frame -> (RGB at half resolution, private mask at half resolution, private mask
    at full resolution)."""
    full = dilate(mask_union(instances, select), r)
    return downscale2(bgra_to_rgb(bgra)), downscale2_mask(full), full


def post(bgra: np.ndarray, pred_low: np.ndarray, mask_full: np.ndarray) -> np.ndarray:
    """Composite the half-resolution prediction (RGB f32 in [0, 1]) into the camera frame."""
    up = to_u8(upscale2(pred_low))  # [H, W, 3] RGB
    out = bgra.copy()
    m = mask_full != 0
    out[..., 0][m] = up[..., 2][m]
    out[..., 1][m] = up[..., 1][m]
    out[..., 2][m] = up[..., 0][m]
    return out
