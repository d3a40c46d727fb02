"""Inpainting throughput on one MI355X: frames/s and p99 latency of the 5x240x432 clip
forward, BF16 MFMA path against the plain FP32 path, plus the roofline of the dominant
kernel and the FP64 oracle timed on the host cores.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

One step = one call of the library's inpainting forward on one 5-frame clip (token gather,
patch embedding, 8 window-attention blocks, decoder and composite).  Ten seeded clips
(coverage 10-40 %) are resident in device memory before timing and are cycled.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "inpainted frames/s + p99 ms/frame, 5×240×432 BF16 vs plain FP32, same GPU"
PEAK = {"bf16": 2500.0, "fp8": 5000.0, "fp32": 157.3}  # dense TFLOP/s, MI355X
HBM_PEAK = 8000.0  # GB/s


def stage_flops(stage, cfg, N, Nq, Na):
    """Algorithmic FLOPs of one launch of each stage (padding and skipped work not counted):
    N tokens, Nq query tokens, Na tokens in windows that have queries (only their keys and
    values are ever read)."""
    C, R, S = cfg.dim, cfg.dim * cfg.mlp_ratio, cfg.window_tokens
    return {
        "qkv": 2 * Na * C * 2 * C + 2 * Nq * C * C,
        "attn": 4 * Nq * S * C,
        "proj": 2 * Nq * C * C,
        "fc1": 2 * Nq * C * R,
        "fc2": 2 * Nq * R * C,
        "mlp": 2 * Nq * C * C + 4 * Nq * C * R,  # fused projection + MLP
        "embed": 2 * N * 48 * C,
        "decode": 2 * Nq * C * 48,
    }.get(stage)


def stage_bytes(stage, cfg, N, Nq, Na):
    """Algorithmic HBM bytes of one launch of each BF16-path stage: every operand read once,
    every result written once (bf16 activations, FP32 residual, bf16 weights)."""
    C, R = cfg.dim, cfg.dim * cfg.mlp_ratio
    return {
        "qkv": Na * C * 2 + Nq * C * 2 + 2 * Na * C * 2 + 3 * C * C * 2,   # x^ in; Q, K, V out; W
        "attn": Nq * C * 2 + 2 * Na * C * 2 + Nq * C * 2,                    # Q, K, V in; O out
        "mlp": Nq * C * 2 + 2 * Nq * C * 4 + Nq * C * 2 + (C * C + 2 * C * R) * 2,  # o, x in/out, x^ out, W
        "embed": N * 16 * (12 + 1) + N * C * (4 + 2),                        # pixels + mask in; x, x^ out
        "decode": Nq * C * 2 + Nq * 16 * (1 + 12) + 48 * C * 2,              # x^, masks in; pixels out
    }.get(stage)


def time_path(eng, clips, precision, steps, warmup, torch):
    """Warm up, then time `steps` calls bracketed by synchronisation; per-call latency from
    HIP events recorded between calls on the launch stream."""
    outs = [torch.empty_like(f) for f, _ in clips]
    for i in range(warmup):
        f, m = clips[i % len(clips)]
        eng(f, m, precision, out=outs[i % len(clips)])
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    ev[0].record()
    for i in range(steps):
        f, m = clips[i % len(clips)]
        eng(f, m, precision, out=outs[i % len(clips)])
        ev[i + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(steps)])
    gpu_ms = ev[0].elapsed_time(ev[steps])
    return wall, gpu_ms, lat


def latency_pass(eng, clips, precision, calls, torch):
    """Per-request latency: `calls` calls, each submitted alone and waited for, timed on the
    host clock from submission to completion (launch overhead included), and on HIP events
    around the call on the launch stream (device time of that request)."""
    outs = [torch.empty_like(f) for f, _ in clips]
    host_ms, dev_ms = [], []
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    for i in range(calls):
        f, m = clips[i % len(clips)]
        t0 = time.perf_counter()
        e0.record()
        eng(f, m, precision, out=outs[i % len(clips)])
        e1.record()
        e1.synchronize()
        host_ms.append((time.perf_counter() - t0) * 1e3)
        dev_ms.append(e0.elapsed_time(e1))
    h, d = np.array(host_ms), np.array(dev_ms)
    pct = lambda a, q: round(float(np.percentile(a, q)), 4)  # noqa: E731
    return {"samples": calls, "p50_ms": pct(h, 50), "p99_ms": pct(h, 99), "max_ms": round(float(h.max()), 4),
            "device_p50_ms": pct(d, 50), "device_p99_ms": pct(d, 99),
            "method": "each call submitted alone and waited for; host clock from submission to completion "
                      "(device_*: HIP events around the call on its stream)"}


def profile_path(eng, clips, precision, steps, torch):
    eng.profile(True)
    for i in range(steps):
        f, m = clips[i % len(clips)]
        eng(f, m, precision)
    torch.cuda.synchronize()
    rec = eng.profile_read()
    eng.profile(False)
    return rec


def _oracle_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        return len(os.sched_getaffinity(0))


def cpu_baseline(cfg, frames, masks, W, n_windows=None, seed_note="clip seed 0"):
    """The FP64 oracle on a bounded sample: `n_windows` windows of one clip (default all of
    them, i.e. the whole clip), each computed from its own pixel footprint (exact, since a
    window's outputs depend only on it)."""
    from oracle import network as on
    B, T, H, Wd, _ = frames.shape
    ph, pw = cfg.patch * cfg.win_h, cfg.patch * cfg.win_w
    wins = [(u, v) for u in range(H // ph) for v in range(Wd // pw)]
    n_windows = len(wins) if n_windows is None else n_windows
    rng = np.random.default_rng(0)
    pick = [wins[i] for i in rng.choice(len(wins), size=n_windows, replace=False)]
    t0 = time.perf_counter()
    for u, v in pick:
        rs, cs = slice(u * ph, (u + 1) * ph), slice(v * pw, (v + 1) * pw)
        on.forward(frames[:1, :, rs, cs], masks[:1, :, rs, cs], W, cfg)
    dt = time.perf_counter() - t0
    frac = n_windows / len(wins)
    return {"value": round(T * frac / dt, 4), "unit": "frames/s", "cores": int(_oracle_threads()), "kind": "oracle",
            "sample": f"{n_windows} of {len(wins)} windows of {seed_note} (all {T} frames, footprint "
                      f"{ph}x{pw} px each), {dt:.1f} s; frames/s scaled by the window fraction"}


def cpu_baseline_small():
    """The oracle on the 64x64 single-frame network (one frame, whole), median of 10 runs."""
    import drsynth
    from oracle import network as on
    cfg = drsynth.NETS["tiny64"]
    f, m = drsynth.tiny_frame(0)
    W = drsynth.make_weights(cfg, 0)
    ts = []
    for _ in range(10):
        t0 = time.perf_counter()
        on.forward(f, m, W, cfg)
        ts.append(time.perf_counter() - t0)
    med = float(np.median(ts))
    return {"value": round(1.0 / med, 3), "unit": "frames/s", "cores": int(_oracle_threads()), "kind": "oracle",
            "sample": f"1x64x64 frame, tiny64 network (dim 64, 2 blocks), median of 10 runs: {med * 1e3:.1f} ms"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--fp32-steps", type=int, default=40)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--latency-calls", type=int, default=1000,
                    help="calls of the per-request latency pass (independent of --steps)")
    ap.add_argument("--precision", default="bf16", choices=["bf16", "fp32", "fp8"])
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 256 MiB device copy (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this path has no multi-GPU mode "
              "(clips and windows shard with no exchange; see the design notes).", file=sys.stderr)
        sys.exit(2)

    import torch
    import drsynth
    from paper_2509_10466_amd import Inpainter

    name = "clip240"
    net, B, T, H, Wd = drsynth.SHAPES[name]
    cfg = drsynth.NETS[net]
    W = drsynth.make_weights(cfg, 0)
    eng = Inpainter(cfg, W)
    eng.reserve(B, T, H, Wd, "bf16")
    host = []
    for seed in range(10):
        f, m, cov = drsynth.make_clip(seed, T, H, Wd)
        host.append((f, m, cov))
    clips = [(torch.from_numpy(f).cuda(), torch.from_numpy(m).cuda()) for f, m, _ in host]
    p = cfg.patch
    tok_cov = [float(m.reshape(B, T, H // p, p, Wd // p, p).any(axis=(3, 5)).mean()) for _, m, _ in host]
    act_cov = []  # fraction of windows holding a query token (from the library's own gather)
    for _, m in clips:
        _, _, woff = eng.gather_tokens(m)
        act_cov.append(float((torch.diff(woff) > 0).float().mean()))
    pix_cov = [float(m.mean()) for _, m, _ in host]
    N = B * T * (H // p) * (Wd // p)

    # headline precision and the plain FP32 path
    wall, gpu_ms, lat = time_path(eng, clips, args.precision, args.steps, args.warmup, torch)
    wall32, gpu32, lat32 = time_path(eng, clips, "fp32", args.fp32_steps, 5, torch)
    fps = T * args.steps / wall
    fps32 = T * args.fp32_steps / wall32
    latency = latency_pass(eng, clips, args.precision, args.latency_calls, torch)

    # per-kernel events over the same workload -> roofline of the dominant kernel
    prof = profile_path(eng, clips, args.precision, len(clips) * 2, torch)
    nsteps_prof = len(clips) * 2
    mean_nq = float(np.mean([tc * N for tc in tok_cov]))
    mean_na = float(np.mean([ac * N for ac in act_cov]))
    best = None
    for st, (ms, cnt) in prof.items():
        if best is None or ms > best[1]:
            best = (st, ms, cnt)
    st, ms, cnt = best
    fl = stage_flops(st, cfg, N, mean_nq, mean_na)
    by = stage_bytes(st, cfg, N, mean_nq, mean_na)
    avg_s = ms / cnt / 1e3
    # the binding roof is the one with the longer ideal time at this launch's size
    t_mfma = fl / (PEAK[args.precision] * 1e12) if fl else 0.0
    t_hbm = by / (HBM_PEAK * 1e9) if by else 0.0
    if t_mfma >= t_hbm:
        ach = fl / avg_s / 1e12
        roof = {"kernel": st, "bound": "mfma", "achieved": round(ach, 2), "peak": PEAK[args.precision],
                "unit": "TFLOP/s", "frac": round(ach / PEAK[args.precision], 4)}
    else:
        ach = by / avg_s / 1e9
        roof = {"kernel": st, "bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK, 4)}
    from paper_2509_10466_amd.profile_summary import read_traffic
    tr = read_traffic(os.path.join(ROOT, "profiles", f"{st}_clip240_traffic.txt"))
    roof["traffic"] = round(tr[1]) if tr else None
    roof.update({"algorithmic_flops": fl, "algorithmic_bytes": by, "avg_launch_us": round(avg_s * 1e6, 2),
                 "launches": cnt, "timing": "HIP events around each launch on the launch stream, "
                                            "eager pass over the same clips after the timed region"})
    stages = {k: {"ms_per_step": round(v[0] / nsteps_prof, 4), "launches_per_step": v[1] / nsteps_prof}
              for k, v in sorted(prof.items(), key=lambda kv: -kv[1][0])}

    if args.calib_copy:
        src = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()

    cpu = cpu_other = None
    if not args.no_cpu:
        f0, m0, _ = host[0]
        cpu = cpu_baseline(cfg, f0, m0, W)
        # the oracle on the other single-GPU workloads: the 64x64 frame, and a sample of
        # windows of a 5x720x1280 clip on the 384-dim, 12-block network
        cfg720 = drsynth.NETS["clip720"]
        f7, m7, _ = drsynth.make_clip(0, 5, 720, 1280)
        cpu_other = {"tiny64": cpu_baseline_small(),
                     "clip720": cpu_baseline(cfg720, f7, m7, drsynth.make_weights(cfg720, 0), n_windows=12,
                                             seed_note="a 5x720x1280 clip (seed 0)")}

    line = {
        "metric": METRIC,
        "value": round(fps, 2),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {
            "workload": "clip240: 1 clip x 5 frames x 240x432 RGB f32, masked-query mode, dim 256, "
                        "4 heads, 8 blocks, MLP x4, 5x9x5-token windows, random-init N(0,0.02^2) weights",
            "clips": "10 seeded Perlin+moving-object clips, random-walk stroke masks dilated 7 px, cycled",
            "pixel_coverage_mean": round(float(np.mean(pix_cov)), 4),
            "token_coverage_mean": round(float(np.mean(tok_cov)), 4),
            "active_window_fraction_mean": round(float(np.mean(act_cov)), 4),
        },
        "p50_ms_per_clip": latency["p50_ms"],
        "p99_ms_per_clip": latency["p99_ms"],
        "p99_ms_per_frame": latency["p99_ms"],
        "p99_ms_per_frame_note": "all 5 frames of a clip complete together, so a frame's latency is its clip's",
        "latency": latency,
        "pipelined_gap_ms": {"samples": args.steps, "p50": round(float(np.percentile(lat, 50)), 4),
                             "p99": round(float(np.percentile(lat, 99)), 4),
                             "note": "HIP-event gaps between back-to-back calls of the throughput pass"},
        "fp32_plain": {"value": round(fps32, 2), "unit": "frames/s",
                       "p50_ms_per_clip": round(float(np.percentile(lat32, 50)), 4),
                       "p99_ms_per_clip": round(float(np.percentile(lat32, 99)), 4),
                       "steps": args.fp32_steps},
        "speedup_vs_fp32": round(fps / fps32, 3),
        "roofline": roof,
        "stages": stages,
        "cpu_baseline": cpu,
        "cpu_baseline_other": cpu_other,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
