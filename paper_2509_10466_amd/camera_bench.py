"""Camera-path benchmark: one collaborator's 1280x720 camera stream through the whole GPU path.

    python -m paper_2509_10466_amd.camera_bench [--frames 200] [--warmup 20] [--objects 4]

Per frame: u8 BGRA camera frame + per-object instance masks -> dr_prep_frame (union of the
selected objects, dilated by 5 px, 2x downscale to 640x360) -> dr_stream_step (the 384-dim,
12-block network with 6x10-token windows, whose 24x40-pixel windows tile 640x360; 4 past
frames kept) -> dr_post_frame (nearest 2x upscale, u8 composite into the camera frame).
The thesis runs its models at 640x360 and scales the outputs to 1280x720, and measures more
than 20 ms for its inpainting stage (CPU pre/post-processing plus ~10.5 ms of inference).

Inputs are synthetic: seeded video frames converted to BGRA, object masks from the seeded
stroke generator split into K instances, half of them selected.  GPU time per stage from HIP
events on the launch stream; prints one JSON line with mean / p50 / p99 ms per frame.
"""
from __future__ import annotations

import argparse
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--frames", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--objects", type=int, default=4)
    ap.add_argument("--radius", type=int, default=5)
    ap.add_argument("--pool", type=int, default=8, help="distinct camera frames, cycled")
    args = ap.parse_args()

    import torch
    import drsynth
    from paper_2509_10466_amd import Inpainter

    H, W = 720, 1280
    cfg = drsynth.NETS["clip720"]
    eng = Inpainter(cfg, drsynth.make_weights(cfg, 0))
    sc = drsynth.Scene(11, H, W, cover_frames=args.pool)
    bgras, insts = [], []
    rng = np.random.default_rng(11)
    K = args.objects
    for t in range(args.pool):
        rgb = sc.frame(t)
        bgra = np.empty((H, W, 4), np.uint8)
        bgra[..., :3] = np.clip(np.rint(rgb[..., ::-1] * 255.0), 0, 255).astype(np.uint8)
        bgra[..., 3] = 255
        m = sc.mask(t) != 0
        # split the private region into K instances by vertical bands; only the selected
        # ones (bits 0 and 2) are removed
        inst = np.zeros((K, H, W), np.uint8)
        band = rng.integers(0, K, size=W)
        for k in range(K):
            inst[k] = (m & (band[None, :] == k)).astype(np.uint8) * (k + 1)
        bgras.append(torch.from_numpy(bgra).cuda())
        insts.append(torch.from_numpy(inst).cuda())
    select = 0b0101
    sid = eng.stream_open(H // 2, W // 2)
    out = torch.empty_like(bgras[0])
    pred = torch.empty((H // 2, W // 2, 3), dtype=torch.float32, device="cuda")

    def frame(t, ev=None):
        i = t % args.pool
        if ev: ev[0].record()
        low, mlow, mfull = eng.prep_frame(bgras[i], insts[i], select, args.radius)
        if ev: ev[1].record()
        eng.stream_step([sid], [low], [mlow], [pred])
        if ev: ev[2].record()
        eng.post_frame(bgras[i], pred, mfull, out=out)
        if ev: ev[3].record()

    for t in range(args.warmup):
        frame(t)
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.frames)]
    for t in range(args.frames):
        frame(args.warmup + t, evs[t])
    torch.cuda.synchronize()
    prep = np.array([e[0].elapsed_time(e[1]) for e in evs])
    net = np.array([e[1].elapsed_time(e[2]) for e in evs])
    post = np.array([e[2].elapsed_time(e[3]) for e in evs])
    tot = np.array([e[0].elapsed_time(e[3]) for e in evs])
    eng.stream_close(sid)

    def st(a):
        return {"mean": round(float(a.mean()), 4), "p50": round(float(np.percentile(a, 50)), 4),
                "p99": round(float(np.percentile(a, 99)), 4)}

    print(json.dumps({"metric": "camera path ms per 1280x720 frame (GPU time)", "network_resolution": "640x360",
                      "objects": K, "selected": bin(select), "dilation_px": args.radius, "frames": args.frames,
                      "coverage": round(float(sc.coverage), 3), "dtype": "bf16",
                      "prep_ms": st(prep), "network_ms": st(net), "post_ms": st(post), "total_ms": st(tot),
                      "frames_per_s": round(1000.0 / float(tot.mean()), 1)}), flush=True)


if __name__ == "__main__":
    main()
