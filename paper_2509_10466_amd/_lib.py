"""ctypes view of ``libdrinpaint.so`` (the C ABI declared in include/drinpaint.h).

torch is imported before the library is opened so that the process holds exactly one HIP
runtime: the library's ``libamdhip64.so.7`` dependency then resolves to the runtime torch
already loaded.  A missing library is an error; there is no fallback path.
"""
from __future__ import annotations

import ctypes as ct
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdrinpaint.so")

DR_OK, DR_EINVAL, DR_ESHAPE, DR_ENOMEM, DR_EHIP, DR_EBUSY = range(6)
STATUS_NAMES = {0: "DR_OK", 1: "DR_EINVAL", 2: "DR_ESHAPE", 3: "DR_ENOMEM", 4: "DR_EHIP", 5: "DR_EBUSY"}
PRECISION = {"fp32": 0, "bf16": 1, "fp8": 2}
QUERY_SET = {"masked": 0, "all": 1}


class NetCfgC(ct.Structure):
    _fields_ = [(n, ct.c_int32) for n in
                ("dim", "heads", "blocks", "mlp_ratio", "patch", "win_h", "win_w", "win_t")]

    @classmethod
    def from_cfg(cls, cfg):
        return cls(cfg.dim, cfg.heads, cfg.blocks, cfg.mlp_ratio, cfg.patch, cfg.win_h,
                   cfg.win_w, cfg.win_t)


class DrError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load():
    """Open the library (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  -- load torch's HIP runtime first
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2509_10466_amd.build`")
    lib = ct.CDLL(LIB_PATH)
    P, I, Z = ct.c_void_p, ct.c_int, ct.c_size_t
    sig = {
        "dr_create": (I, [ct.POINTER(P), I, ct.POINTER(NetCfgC)]),
        "dr_load_weights": (I, [P, P, Z]),
        "dr_reserve": (I, [P, I, I, I, I, I]),
        "dr_inpaint": (I, [P, P, P, P, I, I, I, I, I, I, P]),
        "dr_gather_tokens": (I, [P, P, I, I, I, I, I, P, P, P, P, P]),
        "dr_gather_tokens_noalloc": (I, [P, P, I, I, I, I, I, P, P, P, P, P]),
        "dr_profile": (I, [P, I]),
        "dr_profile_read": (I, [P, ct.POINTER(ct.c_double), ct.POINTER(ct.c_int64), I]),
        "dr_stage_name": (ct.c_char_p, [I]),
        "dr_inspect": (I, [P, ct.c_char_p, P, Z, P]),
        "dr_debug_set": (I, [P, ct.c_char_p, ct.c_int64]),
        "dr_fp8_encode": (I, [P, P, P, Z, ct.c_float, P]),
        "dr_set_budget": (I, [P, Z]),
        "dr_stream_footprint": (Z, [P, I, I]),
        "dr_stream_open": (I, [P, I, I, ct.POINTER(ct.c_int32)]),
        "dr_stream_open_slots": (I, [P, I, I, I, ct.POINTER(ct.c_int32)]),
        "dr_stream_close": (I, [P, ct.c_int32]),
        "dr_stream_step": (I, [P, I, P, P, P, P, I, I, P]),
        "dr_server_create": (I, [P, I, ct.POINTER(P)]),
        "dr_server_submit": (I, [P, ct.c_int32, P, P, P, ct.POINTER(ct.c_uint64)]),
        "dr_server_poll": (I, [P, P, P, P, I, ct.POINTER(I)]),
        "dr_server_stats": (I, [P, ct.POINTER(ct.c_int64), ct.POINTER(ct.c_int64), ct.POINTER(I)]),
        "dr_server_destroy": (None, [P]),
        "dr_param_count": (Z, [P]),
        "dr_load_params": (I, [P, P, P]),
        "dr_train_forward": (I, [P, P, P, P, I, I, I, I, ct.POINTER(P), P]),
        "dr_train_backward": (I, [P, P, P, P, P]),
        "dr_saved_free": (I, [P, P]),
        "dr_l1_loss": (I, [P, P, P, P, Z, ct.c_float, ct.c_float, P, P, P]),
        "dr_set_attention_pattern": (I, [P, I]),
        "dr_train_set_precision": (I, [P, I]),
        "dr_prep_frame": (I, [P, P, P, I, ct.c_uint32, I, I, I, P, P, P, P]),
        "dr_post_frame": (I, [P, P, P, P, I, I, P, P]),
        "dr_last_error": (ct.c_char_p, [P]),
        "dr_destroy": (None, [P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(lib, ctx, status):
    if status != DR_OK:
        raise DrError(status, lib.dr_last_error(ctx).decode(errors="replace"))


def stage_names(lib):
    out = []
    i = 0
    while True:
        s = lib.dr_stage_name(i)
        if s is None:
            return out
        out.append(s.decode())
        i += 1
