"""Memory-slot sweep in stream mode: time per frame against the number of past frames kept.

    python -m paper_2509_10466_amd.slot_sweep [--frames 200] [--warmup 20]

The thesis's only in-network ablation varies the number of memory slots of its inpainting
model (2, 3, 4) and reports frame time and frames/s ("Performance Optimisations -- Inpainting
Model").  This sweep runs one 240x432 stream (256-dim, 8-block network, 5x9-token windows,
BF16) with m = 1..4 past frames kept and reports the GPU time per frame (HIP events around
each step, on the launch stream) and frames/s.  Prints one JSON line.
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
    ap.add_argument("--H", type=int, default=240)
    ap.add_argument("--W", type=int, default=432)
    args = ap.parse_args()

    import torch
    import drsynth
    from paper_2509_10466_amd import Inpainter

    cfg = drsynth.NETS["clip240"]
    eng = Inpainter(cfg, drsynth.make_weights(cfg, 0))
    sc = drsynth.Scene(7, args.H, args.W, cover_frames=10)
    frames = [torch.from_numpy(sc.frame(t)).cuda() for t in range(10)]
    masks = [torch.from_numpy(sc.mask(t)).cuda() for t in range(10)]
    out = torch.empty_like(frames[0])
    rows = []
    for m in (1, 2, 3, 4):
        sid = eng.stream_open(args.H, args.W, slots=m)
        for t in range(args.warmup):
            eng.stream_step([sid], [frames[t % 10]], [masks[t % 10]], [out])
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.frames + 1)]
        ev[0].record()
        for t in range(args.frames):
            eng.stream_step([sid], [frames[t % 10]], [masks[t % 10]], [out])
            ev[t + 1].record()
        torch.cuda.synchronize()
        lat = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(args.frames)])
        rows.append({"slots": m, "ms_per_frame": round(float(lat.mean()), 4),
                     "p99_ms": round(float(np.percentile(lat, 99)), 4),
                     "frames_per_s": round(1000.0 / float(lat.mean()), 1),
                     "footprint_MB": round(eng.stream_footprint(args.H, args.W) * (m + 1) / cfg.win_t / 1e6, 1)})
        eng.stream_close(sid)
    print(json.dumps({"metric": "stream-mode time per frame vs memory slots", "resolution": f"{args.H}x{args.W}",
                      "dtype": "bf16", "coverage": round(sc.coverage, 3), "rows": rows}), flush=True)


if __name__ == "__main__":
    main()
