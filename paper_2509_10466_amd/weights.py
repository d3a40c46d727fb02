"""Versioned FP32 weight blob (the format ``dr_load_weights`` reads).

Layout, little endian: ``b"DRW1"``, uint32 version (1), the network config as 8 int32
(dim, heads, blocks, mlp_ratio, patch, win_h, win_w, win_t), uint32 tensor count, then one
88-byte record per tensor -- char name[48], uint32 dtype (0 = f32), uint32 ndim,
uint32 shape[4], uint64 offset, uint64 nbytes -- and finally the FP32 data, each tensor
256-byte aligned, offsets counted from the end of the record table.
"""
from __future__ import annotations

import struct

import numpy as np

MAGIC = b"DRW1"
VERSION = 1
_REC = struct.Struct("<48sII4IQQ")


def param_names(cfg):
    names = ["embed.w", "embed.b"]
    for l in range(cfg.blocks):
        names += [f"blk{l}.{n}" for n in ("ln1.g", "ln1.b", "wq", "bq", "wk", "bk", "wv", "bv",
                                          "wo", "bo", "ln2.g", "ln2.b", "w1", "b1", "w2", "b2")]
    return names + ["lnf.g", "lnf.b", "dec.w", "dec.b"]


def pack(cfg, weights) -> bytes:
    """Serialise ``weights`` (name -> array) for network ``cfg``."""
    names = param_names(cfg)
    head = MAGIC + struct.pack("<I8iI", VERSION, cfg.dim, cfg.heads, cfg.blocks, cfg.mlp_ratio,
                               cfg.patch, cfg.win_h, cfg.win_w, cfg.win_t, len(names))
    recs, blobs, off = [], [], 0
    for n in names:
        a = np.ascontiguousarray(np.asarray(weights[n], dtype=np.float32))
        if a.ndim > 4:
            raise ValueError(f"{n}: rank {a.ndim} > 4")
        shape = list(a.shape) + [0] * (4 - a.ndim)
        recs.append(_REC.pack(n.encode(), 0, a.ndim, *shape, off, a.nbytes))
        pad = (-a.nbytes) % 256
        blobs.append(a.tobytes() + b"\0" * pad)
        off += a.nbytes + pad
    return head + b"".join(recs) + b"".join(blobs)


def unpack(blob: bytes):
    """Inverse of ``pack``: (config tuple, name -> float32 array)."""
    if blob[:4] != MAGIC:
        raise ValueError("bad magic")
    version, *cfg, count = struct.unpack_from("<I8iI", blob, 4)
    if version != VERSION:
        raise ValueError(f"unsupported version {version}")
    table = 4 + 4 + 32 + 4
    data0 = table + count * _REC.size
    out = {}
    for i in range(count):
        name, dtype, ndim, s0, s1, s2, s3, offset, nbytes = _REC.unpack_from(blob, table + i * _REC.size)
        shape = (s0, s1, s2, s3)[:ndim]
        arr = np.frombuffer(blob, np.float32, count=nbytes // 4, offset=data0 + offset)
        out[name.rstrip(b"\0").decode()] = arr.reshape(shape).copy()
    return tuple(cfg), out
