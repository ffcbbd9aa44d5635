"""rocprofv3 output helpers: per-kernel statistics of a kernel trace,
per-dispatch averages of --pmc counters, HBM traffic calibrated against a
plain copy kernel, and a digest of the kernel sources so stored counter
readings can be matched with the code they were taken on.

    python -m paper_2405_16237_amd.profiling stats --trace DIR --out FILE --command CMD
    python -m paper_2405_16237_amd.profiling traffic --fetch DIR --write DIR --copy-mib N \
        --out FILE --command-fetch CMD --command-write CMD
    python -m paper_2405_16237_amd.profiling counters --pmc DIR [DIR ...] --out FILE --command CMD ...

FETCH_SIZE and WRITE_SIZE are reported in KiB per dispatch; what one KiB of
a counter means in bytes moved is taken from the copy kernel (an elementwise
kernel reading and writing copy-mib MiB, launched by bench.py
--copy-kernel-mib) measured in the same runs.
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import os
import re
import sqlite3

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
COPY_KERNEL = "neg_kernel"


def source_digest() -> str:
    """sha256 over the HIP sources and the public header."""
    files = sorted(glob.glob(os.path.join(PKG, "csrc", "*.hip")) + glob.glob(os.path.join(PKG, "csrc", "*.h")))
    files.append(os.path.join(ROOT, "include", "nbvh.h"))
    h = hashlib.sha256()
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def short_name(full: str) -> str:
    """Kernel name without its argument list and return type."""
    depth, out = 0, []
    name = re.sub(r"^void ", "", full)
    # drop the trailing parameter list "(...)" at template depth 0
    for ch in name:
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            break
        out.append(ch)
    return "".join(out).strip()


def kernel_stats(trace_dir: str):
    """[(name, calls, total_us, avg_us)] sorted by total time, from a
    rocprofv3 --kernel-trace output directory (CSV or rocpd database)."""
    rows = collections.defaultdict(lambda: [0, 0.0])
    csvs = glob.glob(os.path.join(trace_dir, "**", "*kernel_trace.csv"), recursive=True)
    if csvs:
        for f in csvs:
            for r in csv.DictReader(open(f)):
                k = short_name(r["Kernel_Name"])
                rows[k][0] += 1
                rows[k][1] += (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
    else:
        for db in glob.glob(os.path.join(trace_dir, "**", "*_results.db"), recursive=True):
            con = sqlite3.connect(db)
            for name, calls, total, _avg, _pct in con.execute("select * from top_kernels"):
                k = short_name(name)
                rows[k][0] += int(calls)
                rows[k][1] += float(total)
    out = [(k, v[0], v[1], v[1] / max(1, v[0])) for k, v in rows.items()]
    out.sort(key=lambda r: -r[2])
    return out


def pmc_means(pmc_dir: str, counter: str) -> dict:
    """{kernel: (dispatches, mean value)} of one counter of a --pmc run."""
    vals = collections.defaultdict(list)
    for f in glob.glob(os.path.join(pmc_dir, "**", "*counter_collection.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            if r["Counter_Name"] == counter:
                vals[short_name(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    return {k: (len(v), sum(v) / len(v)) for k, v in vals.items()}


def traffic(fetch_dir: str, write_dir: str, copy_bytes: int) -> dict:
    """Bytes fetched from and written to memory per dispatch, per kernel,
    each counter scaled by its reading for the copy kernel."""
    fetch = pmc_means(fetch_dir, "FETCH_SIZE")
    write = pmc_means(write_dir, "WRITE_SIZE")
    cf = [v for k, v in fetch.items() if COPY_KERNEL in k]
    cw = [v for k, v in write.items() if COPY_KERNEL in k]
    if not cf or not cw:
        raise RuntimeError("the copy kernel is missing from the counter runs")
    f_factor = copy_bytes / (cf[0][1] * 1024.0)
    w_factor = copy_bytes / (cw[0][1] * 1024.0)
    kernels = {}
    for k in sorted(set(fetch) | set(write)):
        if COPY_KERNEL in k:
            continue
        fk = fetch.get(k, (0, 0.0))
        wk = write.get(k, (0, 0.0))
        kernels[k] = dict(dispatches=max(fk[0], wk[0]), fetch_kib=fk[1], write_kib=wk[1],
                          bytes=fk[1] * 1024.0 * f_factor + wk[1] * 1024.0 * w_factor)
    return dict(fetch_factor=f_factor, write_factor=w_factor, kernels=kernels)


def write_traffic(path: str, t: dict, copy_bytes: int, commands: list):
    with open(path, "w") as f:
        f.write("# HBM traffic per dispatch: rocprofv3 FETCH_SIZE and WRITE_SIZE (KiB per dispatch), each\n")
        f.write("# scaled by its reading for a copy kernel that reads and writes copy_bytes bytes.\n")
        for c in commands:
            f.write("command: %s\n" % c)
        f.write("source_digest: %s\n" % source_digest())
        f.write("copy_bytes: %d\n" % copy_bytes)
        f.write("fetch_factor: %.4f\n" % t["fetch_factor"])
        f.write("write_factor: %.4f\n" % t["write_factor"])
        for k, v in sorted(t["kernels"].items(), key=lambda kv: -kv[1]["bytes"]):
            f.write("kernel: %s | dispatches: %d | fetch_kib: %.1f | write_kib: %.1f | bytes: %.0f\n"
                    % (k, v["dispatches"], v["fetch_kib"], v["write_kib"], v["bytes"]))


def read_traffic(path: str) -> dict | None:
    """The summary written by write_traffic, or None if missing."""
    if not os.path.isfile(path):
        return None
    out = {"kernels": {}}
    for line in open(path):
        line = line.rstrip("\n")
        if line.startswith("#") or ": " not in line:
            continue
        key, val = line.split(": ", 1)
        if key == "kernel":
            parts = [p.strip() for p in val.split(" | ")]
            name = parts[0]
            kv = dict(p.split(": ", 1) for p in parts[1:])
            out["kernels"][name] = {k: float(v) for k, v in kv.items()}
        elif key == "command":
            out.setdefault("commands", []).append(val)
        else:
            out[key] = val
    return out


def write_stats(path: str, stats, command: str, top: int = 40):
    with open(path, "w") as f:
        f.write("# rocprofv3 --kernel-trace --stats: per-kernel device time\n")
        f.write("command: %s\n\n" % command)
        f.write("| kernel | calls | total us | avg us |\n|---|---|---|---|\n")
        for name, calls, total, avg in stats[:top]:
            f.write("| `%s` | %d | %.1f | %.2f |\n" % (name.replace("|", "/"), calls, total, avg))


def pmc_all(pmc_dir: str) -> dict:
    """{kernel: {counter: (dispatches, mean value)}} of every counter of a --pmc run."""
    vals = collections.defaultdict(lambda: collections.defaultdict(list))
    for f in glob.glob(os.path.join(pmc_dir, "**", "*counter_collection.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            vals[short_name(r["Kernel_Name"])][r["Counter_Name"]].append(float(r["Counter_Value"]))
    return {k: {c: (len(v), sum(v) / len(v)) for c, v in cs.items()} for k, cs in vals.items()}


def write_counters(path: str, dirs: list, commands: list, n_cu: int = 256):
    """Per-kernel means of the counters of several --pmc runs, with the
    per-compute-unit busy fractions that say what bounds a kernel: TA/TD busy
    cycles and stalls are summed over the compute units, GRBM_GUI_ACTIVE over
    the 8 accelerator dies."""
    merged = collections.defaultdict(dict)
    for d in dirs:
        for k, cs in pmc_all(d).items():
            merged[k].update(cs)
    with open(path, "w") as f:
        f.write("# rocprofv3 --pmc: per-dispatch means of hardware counters\n")
        for c in commands:
            f.write("command: %s\n" % c)
        f.write("source_digest: %s\n\n" % source_digest())
        for k in sorted(merged):
            cs = merged[k]
            f.write("## `%s`\n\n| counter | dispatches | mean per dispatch |\n|---|---|---|\n" % k)
            for c in sorted(cs):
                f.write("| %s | %d | %.4g |\n" % (c, cs[c][0], cs[c][1]))
            if "GRBM_GUI_ACTIVE" in cs:
                cyc = cs["GRBM_GUI_ACTIVE"][1] / 8.0
                f.write("\nkernel cycles per die: %.4g\n" % cyc)
                for c in ("TD_TD_BUSY_sum", "TA_TA_BUSY_sum", "TA_ADDR_STALLED_BY_TC_CYCLES_sum", "TD_TC_STALL_sum",
                          "TCP_PENDING_STALL_CYCLES_sum"):
                    if c in cs:
                        f.write("%s per compute unit: %.2f of the kernel's cycles\n" % (c, cs[c][1] / n_cu / cyc))
                # a compute unit issues at most one 64-lane VALU instruction per
                # cycle (4 SIMDs, 4 cycles each); MFMA busy cycles count per SIMD
                if "SQ_INSTS_VALU" in cs:
                    f.write("VALU instructions per compute unit and cycle: %.2f\n" % (cs["SQ_INSTS_VALU"][1] / n_cu / cyc))
                if "SQ_VALU_MFMA_BUSY_CYCLES" in cs:
                    f.write("matrix cores busy (SQ_VALU_MFMA_BUSY_CYCLES / (4 SIMDs x compute units x cycles)): %.3f\n"
                            % (cs["SQ_VALU_MFMA_BUSY_CYCLES"][1] / (4 * n_cu * cyc)))
            if "TCP_TOTAL_CACHE_ACCESSES_sum" in cs and "TCP_TCC_READ_REQ_sum" in cs:
                f.write("L1 miss fraction (TCP_TCC_READ_REQ / TCP_TOTAL_CACHE_ACCESSES): %.3f\n"
                        % (cs["TCP_TCC_READ_REQ_sum"][1] / cs["TCP_TOTAL_CACHE_ACCESSES_sum"][1]))
            if "TCC_HIT_sum" in cs and "TCC_MISS_sum" in cs:
                h, m = cs["TCC_HIT_sum"][1], cs["TCC_MISS_sum"][1]
                f.write("L2 hit fraction: %.3f\n" % (h / (h + m)))
            f.write("\n")


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("--trace", required=True)
    s.add_argument("--out", required=True)
    s.add_argument("--command", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--copy-mib", type=int, required=True)
    t.add_argument("--out", required=True)
    t.add_argument("--command-fetch", required=True)
    t.add_argument("--command-write", required=True)
    c = sub.add_parser("counters")
    c.add_argument("--pmc", nargs="+", required=True)
    c.add_argument("--out", required=True)
    c.add_argument("--command", action="append", required=True)
    a = ap.parse_args()
    if a.cmd == "counters":
        write_counters(a.out, a.pmc, a.command)
        return
    if a.cmd == "stats":
        write_stats(a.out, kernel_stats(a.trace), a.command)
    else:
        nbytes = a.copy_mib * (1 << 20)
        write_traffic(a.out, traffic(a.fetch, a.write, nbytes), nbytes, [a.command_fetch, a.command_write])


if __name__ == "__main__":
    main()
