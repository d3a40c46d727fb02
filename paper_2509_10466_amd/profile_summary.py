"""Text summaries of rocprofv3 result databases (SQLite ``*_results.db``).

    python -m paper_2509_10466_amd.profile_summary kernels RESULTS_DB --command "CMD"
    python -m paper_2509_10466_amd.profile_summary traffic --fetch FETCH_DB --write WRITE_DB \\
        --kernel SUBSTRING --command-fetch "CMD" --command-write "CMD"
    python -m paper_2509_10466_amd.profile_summary counters DB [DB ...] --kernel SUB [--kernel SUB] \\
        --command "CMD" [--command "CMD"]

``kernels`` tabulates a --kernel-trace run: calls, average / min / max duration and share of
the traced GPU time per kernel.  ``traffic`` turns two --pmc runs (FETCH_SIZE, then
WRITE_SIZE; KiB per dispatch) into HBM bytes per launch of one kernel, each counter scaled by
what it reads for the plain 256 MiB device copy that ``bench.py --calib-copy`` performs
(torch's copy of a 64 Mi-element float32 tensor), and records a hash of the library
sources so that a later change of any kernel invalidates the figure.
"""
from __future__ import annotations

import argparse
import hashlib
import os
import re
import sqlite3
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
COPY_BYTES = 64 * 1024 * 1024 * 4  # bench.py --calib-copy: 64 Mi float32 elements


# Sources each profiled kernel is compiled from (its translation unit and the headers it
# includes); a traffic figure stays valid while these files are unchanged.
KERNEL_SOURCES = {
    "mlp_block_kernel": ["k_gemm.hip", "gemm_core.h", "dr_device.h", "dr_internal.h"],
    "qkv_list_kernel": ["k_gemm.hip", "gemm_core.h", "dr_device.h", "dr_internal.h"],
    "attn_clip_kernel": ["k_bf16.hip", "dr_device.h", "dr_internal.h"],
}


def source_hash(files=None) -> str:
    """sha256 over the named library sources (default: every HIP source and header), sorted."""
    csrc = os.path.join(HERE, "csrc")
    if files is None:
        files = [n for n in os.listdir(csrc) if n.endswith((".hip", ".h"))]
    h = hashlib.sha256()
    for name in sorted(files):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def short(name: str) -> str:
    return re.sub(r"\(.*", "", name).replace("void ", "")


def kernels(db: str, command: str) -> str:
    c = sqlite3.connect(db)
    rows = list(c.execute("select name, count(*), avg(end-start), min(end-start), max(end-start), "
                          "sum(end-start) from kernels group by name order by sum(end-start) desc"))
    tot = sum(r[5] for r in rows) or 1
    out = [f"command: {command}", "durations in microseconds (kernel trace, GPU timestamps)",
           f"{'kernel':72s} {'calls':>6s} {'avg':>9s} {'min':>9s} {'max':>9s} {'total_ms':>9s} {'pct':>6s}"]
    for name, cnt, avg, mn, mx, s in rows:
        out.append(f"{short(name)[:72]:72s} {cnt:6d} {avg / 1e3:9.2f} {mn / 1e3:9.2f} {mx / 1e3:9.2f} "
                   f"{s / 1e6:9.3f} {100 * s / tot:6.2f}")
    return "\n".join(out)


def _counter(db: str, counter: str):
    """kernel name -> list of per-dispatch counter values (KiB for the *_SIZE counters)."""
    c = sqlite3.connect(db)
    per = defaultdict(float)
    names = {}
    for name, ctr, val, did in c.execute("select kernel_name, counter_name, value, dispatch_id from counters_collection"):
        if ctr != counter:
            continue
        per[did] += val
        names[did] = name
    out = defaultdict(list)
    for did, v in per.items():
        out[names[did]].append(v)
    return out


def traffic(fetch_db, write_db, kernel, cmd_f, cmd_w) -> str:
    fetch = _counter(fetch_db, "FETCH_SIZE")
    write = _counter(write_db, "WRITE_SIZE")

    def pick(table, sub):
        hits = {k: v for k, v in table.items() if sub in k}
        if not hits:
            sys.exit(f"no kernel matching {sub!r}")
        return hits

    srcs = KERNEL_SOURCES.get(kernel)
    copy_f = [v for k, vs in fetch.items() if "copyBuffer" in k or "copy_kernel" in k for v in vs]
    copy_w = [v for k, vs in write.items() if "copyBuffer" in k or "copy_kernel" in k for v in vs]
    big_f = max(copy_f) if copy_f else None
    big_w = max(copy_w) if copy_w else None
    kf = pick(fetch, kernel)
    kw = pick(write, kernel)
    name = max(kf, key=lambda k: len(kf[k]))
    f_avg = sum(kf[name]) / len(kf[name])
    w_avg = sum(kw.get(name, [0.0])) / max(len(kw.get(name, [1])), 1)
    ref_kib = COPY_BYTES / 1024
    sf = ref_kib / big_f if big_f else 1.0
    sw = ref_kib / big_w if big_w else 1.0
    t = (f_avg * sf + w_avg * sw) * 1024
    lines = [
        f"command (FETCH_SIZE): {cmd_f}",
        f"command (WRITE_SIZE): {cmd_w}",
        f"kernel: {short(name)}",
        f"dispatches: {len(kf[name])}",
        f"FETCH_SIZE KiB per dispatch: {f_avg:.1f}",
        f"WRITE_SIZE KiB per dispatch: {w_avg:.1f}",
        f"copy calibration ({COPY_BYTES // (1 << 20)} MiB device copy): FETCH_SIZE {big_f} KiB, WRITE_SIZE {big_w} KiB "
        f"-> scale {sf:.4f} (fetch), {sw:.4f} (write)",
        f"traffic_bytes_per_launch: {t:.0f}",
        f"sources: {' '.join(srcs) if srcs else 'all'}",
        f"source_sha256: {source_hash(srcs)}",
    ]
    return "\n".join(lines)


def _counters_all(db: str):
    """kernel name -> counter -> list of per-dispatch values.  SQ counters are summed over
    their instances (shader engines, XCDs); GRBM counters, one per XCD for the same kernel
    interval, take the maximum (as rocprofv3's derived MfmaUtil does)."""
    c = sqlite3.connect(db)
    acc = defaultdict(lambda: defaultdict(float))
    names = {}
    for name, ctr, val, did in c.execute("select kernel_name, counter_name, value, dispatch_id from counters_collection"):
        key = (did, ctr)
        if ctr.startswith("GRBM_"):
            acc[did][ctr] = max(acc[did][ctr], val)
        else:
            acc[did][ctr] += val
        names[did] = name
    out = defaultdict(lambda: defaultdict(list))
    for did, d in acc.items():
        for ctr, v in d.items():
            out[names[did]][ctr].append(v)
    return out


SIMDS = 1024          # MI355X: 256 CUs x 4 SIMDs
CUS = 256
CLOCK_GHZ = 2.4


def trace_durations(summary: str):
    """kernel (short name) -> average duration in us, from a ``kernels`` summary file."""
    out = {}
    for ln in open(summary).read().splitlines():
        parts = ln.split()
        if len(parts) >= 7 and parts[-6].isdigit():
            try:
                out[" ".join(parts[:-6])] = float(parts[-5])
            except ValueError:
                pass
    return out


def counters(dbs, kernels, commands, trace_summary=None) -> str:
    """Per-kernel averages of the counters of one or more --pmc runs, with the derived figures
    normalised by the kernel's duration: its average in a kernel-trace summary of the same
    workload when given (a --pmc run serialises dispatches, so GRBM_GUI_ACTIVE there also
    counts the counter collection around each one), else GRBM_GUI_ACTIVE.  MFMA busy = sum
    SQ_VALU_MFMA_BUSY_CYCLES / (cycles x SIMDs) (rocprofv3's MfmaUtil); BF16 MFMA rate = 512
    SQ_INSTS_VALU_MFMA_MOPS_BF16 per second; VALU busy = 4 SQ_ACTIVE_INST_VALU / (cycles x
    SIMDs) (quad-cycles); LDS bank-conflict cycles per CU-cycle."""
    dur = trace_durations(trace_summary) if trace_summary else {}
    merged = defaultdict(lambda: defaultdict(list))
    for db in dbs:
        for k, d in _counters_all(db).items():
            for ctr, vals in d.items():
                merged[k][ctr] += vals
    lines = [f"command: {cmd}" for cmd in commands]
    lines.append("per-dispatch averages; derived figures from the averages")
    for sub in kernels:
        hits = [k for k in merged if sub in k]
        if not hits:
            lines.append(f"{sub}: no dispatch")
            continue
        name = max(hits, key=lambda k: len(next(iter(merged[k].values()))))
        d = {ctr: sum(v) / len(v) for ctr, v in merged[name].items()}
        n = max(len(v) for v in merged[name].values())
        lines.append(f"kernel: {short(name)}  (dispatches: {n})")
        for ctr in sorted(d):
            lines.append(f"  {ctr:32s} {d[ctr]:16.1f}")
        gui = d.get("GRBM_GUI_ACTIVE")
        us = next((v for k, v in dur.items() if k[:60] == short(name)[:60]), None)
        if us:
            gui = us * 1e3 * CLOCK_GHZ
            lines.append(f"  kernel time from the trace summary: {us:.2f} us")
        elif gui:
            lines.append(f"  kernel time from GRBM_GUI_ACTIVE: {gui / CLOCK_GHZ / 1e3:.2f} us")
        if gui:
            if "SQ_VALU_MFMA_BUSY_CYCLES" in d:
                lines.append(f"  MFMA busy: {100 * d['SQ_VALU_MFMA_BUSY_CYCLES'] / (gui * SIMDS):.1f} % of SIMD cycles")
            if "SQ_INSTS_VALU_MFMA_MOPS_BF16" in d:
                tf = 512 * d["SQ_INSTS_VALU_MFMA_MOPS_BF16"] / (gui / (CLOCK_GHZ * 1e9)) / 1e12
                lines.append(f"  BF16 MFMA rate: {tf:.1f} TFLOP/s ({100 * tf / 2500:.1f} % of 2.5 PFLOP/s), "
                             f"{512 * d['SQ_INSTS_VALU_MFMA_MOPS_BF16'] / 1e9:.3f} GFLOP issued")
            if "SQ_ACTIVE_INST_VALU" in d:
                lines.append(f"  VALU busy: {100 * 4 * d['SQ_ACTIVE_INST_VALU'] / (gui * SIMDS):.1f} % of SIMD cycles")
            if "SQ_VALU_MFMA_COEXEC_CYCLES" in d:
                lines.append(f"  VALU/MFMA co-execution: {100 * d['SQ_VALU_MFMA_COEXEC_CYCLES'] / (gui * SIMDS):.1f} % of SIMD cycles")
            if "SQ_LDS_BANK_CONFLICT" in d:
                lines.append(f"  LDS bank-conflict cycles: {100 * d['SQ_LDS_BANK_CONFLICT'] / (gui * CUS):.2f} % of CU cycles")
            if "SQ_ACTIVE_INST_LDS" in d:
                lines.append(f"  LDS instruction issue: {100 * 4 * d['SQ_ACTIVE_INST_LDS'] / (gui * SIMDS):.1f} % of SIMD cycles")
    return "\n".join(lines)


def read_traffic(path: str):
    """(kernel, bytes per launch) from a ``traffic`` summary if it was taken from the current
    sources, else None."""
    try:
        with open(path) as f:
            txt = f.read()
    except OSError:
        return None
    kv = dict(line.split(": ", 1) for line in txt.splitlines() if ": " in line)
    srcs = kv.get("sources", "all")
    if kv.get("source_sha256") != source_hash(None if srcs == "all" else srcs.split()):
        return None
    try:
        return kv["kernel"], float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    k = sub.add_parser("kernels")
    k.add_argument("db")
    k.add_argument("--command", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--kernel", required=True)
    t.add_argument("--command-fetch", required=True)
    t.add_argument("--command-write", required=True)
    cc = sub.add_parser("counters")
    cc.add_argument("dbs", nargs="+")
    cc.add_argument("--kernel", action="append", required=True)
    cc.add_argument("--command", action="append", required=True)
    cc.add_argument("--trace-summary", default=None, help="kernels summary of the same workload (durations)")
    a = ap.parse_args()
    if a.cmd == "kernels":
        print(kernels(a.db, a.command))
    elif a.cmd == "counters":
        print(counters(a.dbs, a.kernel, a.command, a.trace_summary))
    else:
        print(traffic(a.fetch, a.write, a.kernel, a.command_fetch, a.command_write))


if __name__ == "__main__":
    main()
