"""Training-step timing: forward with saved activations, weighted L1 loss, hand-written
backward, on 4 clips of 5 x 240 x 432 (seeds 0..3, ground truth = the uncut frames), in
FP32 or mixed precision (bf16 operands of the weight products, FP32 accumulation and master
weights and gradients).

    python -m paper_2509_10466_amd.train_bench [--steps 5] [--precision fp32|bf16]

Prints one JSON line with the per-step time split (forward, loss, backward) from HIP events
on the launch stream, and the parameter-gradient norm as a sanity figure.
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
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--clips", type=int, default=4)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16"])
    args = ap.parse_args()

    import torch
    import drsynth
    from paper_2509_10466_amd import Inpainter

    cfg = drsynth.NETS["clip240"]
    eng = Inpainter(cfg, drsynth.make_weights(cfg, 0))
    eng.train_precision(args.precision)
    fs, ms = [], []
    for seed in range(args.clips):
        f, m, _ = drsynth.make_clip(seed, 5, 240, 432)
        fs.append(f[0])
        ms.append(m[0])
    gt = torch.from_numpy(np.stack(fs)).cuda()          # [4, 5, H, W, 3]
    masks = torch.from_numpy(np.stack(ms)).cuda()
    frames = gt * (1 - masks[..., None].float())         # private pixels cut out
    t_f, t_l, t_b = [], [], []
    gnorm = None
    for step in range(args.steps + 1):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        e[0].record()
        pred, saved = eng.train_forward(frames, masks)
        e[1].record()
        loss, dpred = eng.l1_loss(pred, gt, masks)
        e[2].record()
        grads = eng.train_backward(saved, dpred)
        e[3].record()
        torch.cuda.synchronize()
        saved.close()
        if step == 0:
            continue  # first step allocates the training workspace
        t_f.append(e[0].elapsed_time(e[1]))
        t_l.append(e[1].elapsed_time(e[2]))
        t_b.append(e[2].elapsed_time(e[3]))
        gnorm = float(grads.norm())
    tot = np.array(t_f) + np.array(t_l) + np.array(t_b)
    print(json.dumps({"workload": f"{args.clips} clips x 5 x 240 x 432, clip240 net, {args.precision} forward + backward",
                      "ms_per_step": round(float(tot.mean()), 3), "forward_ms": round(float(np.mean(t_f)), 3),
                      "loss_ms": round(float(np.mean(t_l)), 3), "backward_ms": round(float(np.mean(t_b)), 3),
                      "frames_per_s": round(args.clips * 5 * 1000.0 / float(tot.mean()), 2),
                      "loss": round(float(loss), 6), "grad_norm": round(gnorm, 6), "steps": args.steps}), flush=True)


if __name__ == "__main__":
    main()
