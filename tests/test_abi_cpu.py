"""C ABI checks that need no GPU: the library loads, exports every declared symbol, rejects
bad arguments before touching a device, and the weight blob round-trips."""
import ctypes as ct
import os
import re

import numpy as np
import pytest

import drsynth
from paper_2509_10466_amd import weights as wblob

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "drinpaint.h")
LIB = os.path.join(ROOT, "paper_2509_10466_amd", "libdrinpaint.so")


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w\s\*]*?\b(dr_\w+)\s*\(", text, re.M)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for s in ("dr_create", "dr_load_weights", "dr_reserve", "dr_inpaint", "dr_gather_tokens",
              "dr_profile", "dr_profile_read", "dr_stage_name", "dr_last_error", "dr_destroy"):
        assert s in syms


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    import torch  # noqa: F401  (same runtime order as the product binding)
    return ct.CDLL(LIB)


def test_library_exports_every_declared_symbol(lib):
    for s in declared_symbols():
        assert hasattr(lib, s), f"{s} not exported"


def test_stage_names_and_null_handling(lib):
    lib.dr_stage_name.restype = ct.c_char_p
    names = []
    i = 0
    while lib.dr_stage_name(i) is not None:
        names.append(lib.dr_stage_name(i).decode())
        i += 1
    assert names[:5] == ["tokens", "embed", "ln1", "qkv", "attn"]
    lib.dr_create.argtypes = [ct.c_void_p, ct.c_int, ct.c_void_p]
    assert lib.dr_create(None, 0, None) == 1  # DR_EINVAL, no device touched
    lib.dr_last_error.restype = ct.c_char_p
    lib.dr_last_error.argtypes = [ct.c_void_p]
    assert b"null" in lib.dr_last_error(None)
    lib.dr_inpaint.argtypes = [ct.c_void_p] * 4 + [ct.c_int] * 6 + [ct.c_void_p]
    assert lib.dr_inpaint(None, None, None, None, 1, 1, 1, 1, 0, 0, None) == 1


def test_create_rejects_unsupported_networks(lib):
    from paper_2509_10466_amd._lib import NetCfgC
    lib.dr_create.argtypes = [ct.c_void_p, ct.c_int, ct.c_void_p]
    ctx = ct.c_void_p()
    bad = [dict(dim=96), dict(heads=3), dict(heads=4), dict(patch=8), dict(win_h=41)]
    for b in bad:
        kw = dict(dim=64, heads=2, blocks=2, mlp_ratio=4, patch=4, win_h=8, win_w=8, win_t=1)
        kw.update(b)
        c = NetCfgC(*[kw[k] for k in ("dim", "heads", "blocks", "mlp_ratio", "patch", "win_h", "win_w", "win_t")])
        assert lib.dr_create(ct.byref(ctx), 0, ct.byref(c)) == 2, b  # DR_ESHAPE


def test_weight_blob_roundtrip():
    cfg = drsynth.NETS["tiny64"]
    W = drsynth.make_weights(cfg, 0)
    blob = wblob.pack(cfg, W)
    kcfg, back = wblob.unpack(blob)
    assert kcfg == (64, 2, 2, 4, 4, 8, 8, 1)
    assert list(back) == wblob.param_names(cfg) == [n for n, _ in drsynth.weight_order(cfg)]
    for k in W:
        assert np.array_equal(W[k], back[k])
