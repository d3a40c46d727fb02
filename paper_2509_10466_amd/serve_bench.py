"""Serving benchmark: simulated collaborators streaming frames into the native serving loop.

    python -m paper_2509_10466_amd.serve_bench [--seconds 30] [--warmup 5] [--streams 16]

Sixteen collaborators each send frames as a Poisson process at 30 frames/s (exponential
gaps, seeded).  Resolutions are 240x432, 480x864 and 720x1280 in the ratio 2:1:1; the first
two run on the 256-dim / 8-block network with 5x9-token windows, 720x1280 on the 384-dim /
12-block network with 6x10-token windows (their frame sizes tile only those windows).  Each
stream keeps its last four frames' keys/values on the device (stream mode) and has a
random-walk stroke mask with coverage drawn from U[5 %, 40 %].  Frames come from a pool of
seeded synthetic video frames per stream, resident on the device, cycled.

Prints one JSON line: completed frames/s and p50/p99 latency (submission to completion,
ms) per resolution and overall, over the measured window after the warm-up.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

RES = [(240, 432), (240, 432), (480, 864), (720, 1280)]  # 2:1:1


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--seconds", type=float, default=30.0)
    ap.add_argument("--warmup", type=float, default=5.0)
    ap.add_argument("--streams", type=int, default=16)
    ap.add_argument("--fps", type=float, default=30.0)
    ap.add_argument("--pool", type=int, default=5, help="distinct frames per stream")
    ap.add_argument("--max-batch", type=int, default=8)
    ap.add_argument("--seed", type=int, default=0)
    args = ap.parse_args()

    import torch
    import drsynth
    from paper_2509_10466_amd import Inpainter
    from paper_2509_10466_amd.api import Server

    nets = {"clip240": drsynth.NETS["clip240"], "clip720": drsynth.NETS["clip720"]}
    engines = {k: Inpainter(cfg, drsynth.make_weights(cfg, 0)) for k, cfg in nets.items()}

    rng = np.random.default_rng(args.seed)
    streams = []
    t_gen = time.time()
    for i in range(args.streams):
        H, W = RES[(i * len(RES)) // args.streams] if args.streams >= len(RES) else RES[i % len(RES)]
        net = "clip720" if H == 720 else "clip240"
        sc = drsynth.Scene(1000 + i, H, W, cov_range=(0.05, 0.40), cover_frames=args.pool)
        frames = [torch.from_numpy(sc.frame(t)).cuda() for t in range(args.pool)]
        masks = [torch.from_numpy(sc.mask(t)).cuda() for t in range(args.pool)]
        outs = [torch.empty_like(frames[0]) for _ in range(8)]
        sid = engines[net].stream_open(H, W)
        streams.append(dict(i=i, H=H, W=W, net=net, sid=sid, frames=frames, masks=masks, outs=outs,
                            cov=sc.coverage, k=0))
    torch.cuda.synchronize()
    # servers start after the streams are open, so every executor's workspace is allocated
    # before the first request
    servers = {k: Server(e, max_batch=args.max_batch) for k, e in engines.items()}
    t_gen = time.time() - t_gen

    # arrival timeline: per stream exponential gaps at `fps`
    total = args.warmup + args.seconds
    events = []
    for s in streams:
        t = float(rng.exponential(1.0 / args.fps))
        while t < total:
            events.append((t, s["i"]))
            t += float(rng.exponential(1.0 / args.fps))
    events.sort()

    meta = {}
    results = []
    t0 = time.perf_counter()
    for t_ev, i in events:
        while time.perf_counter() - t0 < t_ev:
            pass
        s = streams[i]
        k = s["k"]
        s["k"] += 1
        tk = servers[s["net"]].submit(s["sid"], s["frames"][k % args.pool], s["masks"][k % args.pool],
                                      s["outs"][k % len(s["outs"])])
        meta[(s["net"], tk)] = (t_ev, i)
        for net, srv in servers.items():
            for tkt, lat, st in srv.poll():
                results.append((net, tkt, lat, st))
    # drain
    deadline = time.perf_counter() + 60
    while len(results) < len(events) and time.perf_counter() < deadline:
        for net, srv in servers.items():
            for tkt, lat, st in srv.poll():
                results.append((net, tkt, lat, st))
        time.sleep(0.001)
    stats = {k: v.stats() for k, v in servers.items()}
    for srv in servers.values():
        srv.close()

    per_res = {}
    failed = 0
    measured = 0
    for net, tkt, lat, st in results:
        t_ev, i = meta[(net, tkt)]
        if st != 0:
            failed += 1
            continue
        if t_ev < args.warmup:
            continue
        measured += 1
        key = f"{streams[i]['H']}x{streams[i]['W']}"
        per_res.setdefault(key, []).append(lat)
    allv = [v for vals in per_res.values() for v in vals]
    report = {
        "metric": "serving: completed frames/s and p50/p99 latency ms (submission to completion)",
        "streams": args.streams, "fps_per_stream": args.fps, "seconds": args.seconds, "warmup": args.warmup,
        "frames_per_s": round(measured / args.seconds, 2),
        "offered_frames_per_s": round(sum(1 for t, _ in events if t >= args.warmup) / args.seconds, 2),
        "p50_ms": round(float(np.percentile(allv, 50)), 3) if allv else None,
        "p99_ms": round(float(np.percentile(allv, 99)), 3) if allv else None,
        "per_resolution": {k: {"frames": len(v), "p50_ms": round(float(np.percentile(v, 50)), 3),
                               "p99_ms": round(float(np.percentile(v, 99)), 3),
                               "max_ms": round(float(np.max(v)), 3)} for k, v in sorted(per_res.items())},
        "failed": failed, "lost": len(events) - len(results),
        "batches": {k: v for k, v in stats.items()},
        "coverage": [round(s["cov"], 3) for s in streams],
        "setup_s": round(t_gen, 1), "dtype": "bf16", "data": "synthetic",
    }
    for s in streams:
        engines[s["net"]].stream_close(s["sid"])
    print(json.dumps(report), flush=True)


if __name__ == "__main__":
    main()
