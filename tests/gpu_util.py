"""Helpers shared by the GPU parity tests (no GPU work at import time)."""
import numpy as np

import drsynth

# A small network whose windows span all 5 frames with S = 225 (four query tiles, the last
# ragged), on 5 x 40 x 72 clips (2 x 2 windows).
MID = drsynth.NetCfg(dim=128, heads=2, blocks=2, mlp_ratio=4, patch=4, win_h=5, win_w=9, win_t=5)

TOL = {"fp32": 1e-4, "bf16": 2e-2, "fp8": 5e-2}


def case_inputs(case, seed=0):
    """(cfg, frames, masks) for a named parity case."""
    if case == "tiny64":
        cfg = drsynth.NETS["tiny64"]
        f, m = drsynth.tiny_frame(seed)
        return cfg, f, m
    if case == "mid":
        f, m, _ = drsynth.make_clip(seed, 5, 40, 72, cov_range=(0.2, 0.4))
        return MID, f, m
    if case == "mid_b2":
        f, m = drsynth.make_clip_batch([seed, seed + 1], 5, 40, 72)
        return MID, f, m
    name = {"clip240": "clip240", "clip480": "clip480", "clip720": "clip720"}[case]
    cfg, f, m = drsynth.make_workload(name, seed)
    return cfg, f, m


def window_footprints(cfg, frames_shape):
    """List of (b, row slice, col slice) of every window's pixel footprint (all frames)."""
    B, T, H, W, _ = frames_shape
    ph, pw = cfg.patch * cfg.win_h, cfg.patch * cfg.win_w
    return [(b, slice(u * ph, (u + 1) * ph), slice(v * pw, (v + 1) * pw))
            for b in range(B) for u in range(H // ph) for v in range(W // pw)]


def sample_windows(cfg, masks, k=8, seed=0):
    """k window footprints: the most-masked ones, unmasked ones and random ones."""
    fps = window_footprints(cfg, masks.shape + (3,))
    cov = np.array([masks[b, :, rs, cs].mean() for b, rs, cs in fps])
    order = np.argsort(-cov)
    rng = np.random.default_rng(seed)
    pick = list(order[: k // 2]) + list(np.flatnonzero(cov == 0)[:1])
    rest = [i for i in range(len(fps)) if i not in pick]
    pick += list(rng.choice(rest, size=min(len(rest), k - len(pick)), replace=False))
    return [fps[i] for i in pick]


def compare(out_gpu, out_ref, frames, masks, tol):
    """Outside the mask: bit-exact with the input.  Inside: max |gpu - ref| <= tol.
    Returns (max abs error inside, number of inside values)."""
    inside = np.repeat(masks[..., None] != 0, 3, axis=-1)
    assert np.array_equal(out_gpu[~inside], frames[~inside]), "pixels outside the mask changed"
    if not inside.any():
        return 0.0, 0
    err = np.abs(out_gpu[inside].astype(np.float64) - out_ref[inside])
    mx = float(err.max())
    assert mx <= tol, f"max abs error {mx:.3g} > {tol}"
    return mx, int(inside.sum())


def error_stats(out_gpu, out_ref, pred_ref, frames, masks, tol):
    """Checks one result against the oracle and returns its error statistics.

    Outside the mask the result must equal the input bit for bit; inside, the max abs error
    against the oracle must be within ``tol``.  Besides the max this reports the RMS error and
    the spread (max - min) of the oracle's in-mask prediction, which shows how far the
    tolerance is from a vacuous one (a constant prediction would miss by about half of it)."""
    inside = np.repeat(masks[..., None] != 0, 3, axis=-1)
    assert np.array_equal(out_gpu[~inside], frames[~inside]), "pixels outside the mask changed"
    if not inside.any():
        return {"max": 0.0, "rms": 0.0, "spread": 0.0, "n": 0}
    d = out_gpu[inside].astype(np.float64) - out_ref[inside]
    p = pred_ref[inside]
    s = {"max": float(np.abs(d).max()), "rms": float(np.sqrt(np.mean(d * d))),
         "spread": float(p.max() - p.min()), "n": int(inside.sum())}
    assert s["max"] <= tol, f"max abs error {s['max']:.3g} > {tol}"
    return s


def active_windows(cfg, masks):
    """Footprints of every window that holds a private pixel (the windows with queries)."""
    return [fp for fp in window_footprints(cfg, masks.shape + (3,))
            if masks[fp[0], :, fp[1], fp[2]].any()]


_POOL_STATE = {}


def _pool_init(cfg, W):
    from threadpoolctl import threadpool_limits
    _POOL_STATE["cfg"], _POOL_STATE["W"] = cfg, W
    _POOL_STATE["limits"] = threadpool_limits(1)


def _pool_group(args):
    from oracle import network as on
    f, m = args
    fwd = on.forward_detail(f, m, _POOL_STATE["W"], _POOL_STATE["cfg"])
    return fwd["out"], fwd["pred"]


def oracle_windows(on, cfg, frames, masks, W, fps, chunk=8, workers=None):
    """The oracle's (out, pred) on each window footprint in ``fps``, computed from the
    footprint's own pixels (a window's outputs depend on nothing else).  Footprints go to the
    oracle as batches of small clips, spread over worker processes (one BLAS thread each: most
    of the oracle's time is element-wise work that one process runs on one core)."""
    import concurrent.futures as cf
    import multiprocessing as mp
    import os
    groups = []
    for i in range(0, len(fps), chunk):
        grp = fps[i:i + chunk]
        groups.append((np.stack([frames[b, :, rs, cs] for b, rs, cs in grp]),
                       np.stack([masks[b, :, rs, cs] for b, rs, cs in grp])))
    if workers is None:
        workers = min(16, len(os.sched_getaffinity(0)), len(groups))
    if workers <= 1:
        res = [(lambda d: (d["out"], d["pred"]))(on.forward_detail(f, m, W, cfg)) for f, m in groups]
    else:
        # spawned workers import only numpy and the oracle; a worker that dies raises here
        with cf.ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn"),
                                    initializer=_pool_init, initargs=(cfg, W)) as pool:
            res = list(pool.map(_pool_group, groups))
    outs = []
    for o, p in res:
        outs += [(o[j], p[j]) for j in range(len(o))]
    return outs
