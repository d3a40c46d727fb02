"""FP8 vs BF16 vs plain FP32 on the same GPU, clip mode.

    python -m paper_2509_10466_amd.precision_bench [--shape clip720] [--clips 3] [--steps 10]
                                                   [--attn joint|decoupled] [--overlap]

Runs seeded clips of the chosen shape (default 5 x 720 x 1280 on the 384-dim, 12-block
network with 6x10x5-token windows, seeds 0..clips-1) in each precision and reports frames/s,
p50/p99 ms per clip (HIP events between calls on the launch stream) and the largest
absolute difference of the in-mask pixels from the FP32 path's output.  With --attn
decoupled (even blocks within one frame of a window, odd blocks across its frames) only BF16
and FP8 run, and FP8 is compared with BF16; with --overlap (kernel-8 embedding and fold
decoder) only BF16 runs.  Prints one JSON line.
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
    ap.add_argument("--shape", default="clip720")
    ap.add_argument("--clips", type=int, default=3)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--attn", default="joint", choices=["joint", "decoupled"])
    ap.add_argument("--overlap", action="store_true")
    args = ap.parse_args()

    import torch
    import drsynth
    from paper_2509_10466_amd import Inpainter

    net, B, T, H, W = drsynth.SHAPES[args.shape]
    cfg = drsynth.NETS[net]
    if args.overlap:
        import dataclasses
        cfg = dataclasses.replace(cfg, overlap=True)
    eng = Inpainter(cfg, drsynth.make_weights(cfg, 0))
    eng.set_attention(args.attn)
    precs = ("bf16",) if args.overlap else ("fp32", "bf16", "fp8") if args.attn == "joint" else ("bf16", "fp8")
    base = precs[0]
    clips = []
    for seed in range(args.clips):
        f, m, _ = drsynth.make_clip(seed, T, H, W)
        clips.append((torch.from_numpy(f).cuda(), torch.from_numpy(m).cuda()))
    res, outs = {}, {}
    for prec in precs:
        eng.reserve(B, T, H, W, prec)
        o = [torch.empty_like(f) for f, _ in clips]
        for i in range(args.warmup):
            f, m = clips[i % len(clips)]
            eng(f, m, prec, out=o[i % len(clips)])
        torch.cuda.synchronize()
        steps = args.steps if prec != "fp32" else max(3, args.steps // 3)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        ev[0].record()
        for i in range(steps):
            f, m = clips[i % len(clips)]
            eng(f, m, prec, out=o[i % len(clips)])
            ev[i + 1].record()
        torch.cuda.synchronize()
        lat = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(steps)])
        outs[prec] = [x.clone() for x in o]
        # per-stage GPU time (HIP events around each launch, eager, after the timed region)
        eng.profile(True)
        for i in range(len(clips)):
            f, m = clips[i]
            eng(f, m, prec, out=o[i])
        torch.cuda.synchronize()
        stages = {k: round(v[0] / len(clips), 4) for k, v in sorted(eng.profile_read().items(), key=lambda kv: -kv[1][0])}
        eng.profile(False)
        res[prec] = {"frames_per_s": round(T * 1000.0 / float(lat.mean()), 2),
                     "p50_ms_per_clip": round(float(np.percentile(lat, 50)), 3),
                     "p99_ms_per_clip": round(float(np.percentile(lat, 99)), 3), "steps": steps,
                     "stage_ms_per_clip": stages}
    for prec in precs[1:]:
        d = 0.0
        for (f, m), a, b in zip(clips, outs[prec], outs[base]):
            sel = m.bool()
            d = max(d, float((a - b).abs()[sel].max()) if sel.any() else 0.0)
            outside = ~sel
            assert torch.equal(a[outside], f[outside]), "pixels outside the mask must be the input"
        res[prec][f"max_abs_diff_vs_{base}_in_mask"] = round(d, 5)
        res[prec][f"speedup_vs_{base}"] = round(res[prec]["frames_per_s"] / res[base]["frames_per_s"], 3)
    print(json.dumps({"workload": f"{args.shape}: {B}x{T}x{H}x{W}, {cfg.dim}-dim {cfg.heads}-head {cfg.blocks}-block "
                                  f"net, {cfg.win_t}x{cfg.win_h}x{cfg.win_w}-token windows, masked-query mode, {args.attn} attention"
                                  + (", overlapping kernel-8 embedding and fold decoder" if args.overlap else ""),
                      "clips": args.clips, "results": res}), flush=True)


if __name__ == "__main__":
    main()
