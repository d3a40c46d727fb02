"""Build the gfx950 shared library ``libdrinpaint.so`` in-tree with hipcc.

``python -m paper_2509_10466_amd.build`` compiles every ``csrc/*.hip`` translation unit for
gfx950 (object files under ``_build/``) and links ``paper_2509_10466_amd/libdrinpaint.so``.
"""
from __future__ import annotations

import concurrent.futures as cf
import json
import os
import re
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libdrinpaint.so")

ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
    "-Wno-unused-variable", "-Wno-unused-but-set-variable", "-Wno-unused-value",
    # keep the device code free of packed-FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    f"-I{os.path.join(ROOT, 'include')}",
    # per-kernel register, LDS and scratch figures as compiler remarks (parsed below)
    "-Rpass-analysis=kernel-resource-usage",
]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


_REMARK = re.compile(r"remark:\s+(Function Name|VGPRs|AGPRs|ScratchSize \[bytes/lane\]|"
                     r"Occupancy \[waves/SIMD\]|LDS Size \[bytes/block\]):\s+(\S+)")


def _resources(text):
    """Per-kernel resource table from the compiler's kernel-resource-usage remarks."""
    table, cur = {}, None
    for key, val in _REMARK.findall(text):
        if key == "Function Name":
            cur = table.setdefault(val, {})
        elif cur is not None:
            cur[key.split(" ")[0].lower()] = int(val) if val.isdigit() else val
    return table


def _compile(src):
    obj = os.path.join(BUILD, os.path.basename(src)[:-4] + ".o")
    cmd = [HIPCC, *FLAGS, "-c", src, "-o", obj]
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{p.stdout}\n{p.stderr}")
    text = p.stdout + p.stderr
    noise = ("'-packed-fp32-ops' is not a recognized feature", "remark:", "[-Rpass-analysis", "|")
    msgs = [ln for ln in text.splitlines()
            if ln.strip() and not any(n in ln for n in noise) and not ln.strip().isdigit()]
    return obj, msgs, _resources(text)


def build(verbose: bool = False) -> str:
    """Compile and link; returns the path of the shared library."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        results = list(ex.map(_compile, srcs))
    table = {}
    for obj, msgs, res in results:
        table.update(res)
        if verbose and msgs:
            print("\n".join(msgs), file=sys.stderr)
    with open(os.path.join(BUILD, "kernel_resources.json"), "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    # Register arrays that land in scratch turn prefetches into memory round trips; no kernel
    # of this library may use scratch.
    spilled = {k: v for k, v in table.items() if v.get("scratchsize", 0)}
    if spilled:
        raise RuntimeError("kernels using scratch memory: " + ", ".join(
            f"{k} ({v['scratchsize']} B/lane)" for k, v in sorted(spilled.items())))
    tmp = LIB + ".tmp"
    # every symbol must resolve at link time: a missing definition is a build error, not a
    # failure at load time
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-Wl,--no-undefined", "-o", tmp,
           *[r[0] for r in results]]
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError(f"link failed:\n{p.stdout}\n{p.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
