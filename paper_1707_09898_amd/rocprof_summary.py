"""Short text summaries of rocprofv3 output (for the profiles/ folder), and
the lookup bench.py uses to attach measured HBM traffic to a kernel.

A summary holds, per kernel launch shape (name, element type, work items):
the launch count and mean duration from a --kernel-trace run, and the mean
FETCH_SIZE / WRITE_SIZE per dispatch from two --pmc runs, each scaled by the
factor that makes the same counter read the true size of a plain copy kernel
(a torch copy of --copy-mib MiB in the same program).  It also records a hash
of the HIP sources, so a reader can tell whether the kernels changed since
the counters were taken.

  python -m paper_1707_09898_amd.rocprof_summary --trace T.csv [--fetch F.csv --write W.csv
         --copy-mib N] --command "..." --title "..." --out profiles/NAME.md

With --sq S.csv (a pass of SQ_WAVES and SQ_INSTS_* counters) it writes
instead the instruction summary: VALU, LDS and vector-memory instructions
per wave and the VALU issue time over the chip next to each kernel's
duration.
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import json
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")


def code_tokens(text: str) -> str:
    """C/C++ source without its comments, whitespace runs collapsed to one
    space: what the compiler sees, so that an edit of a comment does not
    mark the counters as taken on other kernels."""
    out = []
    i, n = 0, len(text)
    while i < n:
        c = text[i]
        if c == "/" and i + 1 < n and text[i + 1] == "/":
            j = text.find("\n", i)
            i = n if j < 0 else j
            out.append(" ")
        elif c == "/" and i + 1 < n and text[i + 1] == "*":
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        elif c in "\"'":
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def source_hash() -> str:
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.h")) +
                    glob.glob(os.path.join(CSRC, "*.inc")) + glob.glob(os.path.join(CSRC, "*.cpp"))):
        h.update(os.path.basename(p).encode())
        with open(p, encoding="utf-8") as f:
            h.update(code_tokens(f.read()).encode())
    return h.hexdigest()[:16]


def kernel_key(name: str):
    """(base name, element type) of a demangled kernel name."""
    n = name.replace("(anonymous namespace)::", "").replace("void ", "").strip()
    base = re.split(r"[<(]", n, 1)[0].strip()
    m = re.match(r"[^<]*<\s*(float|double)", n)
    return base, (m.group(1) if m else "")


def read_trace(path):
    out = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        items = int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])
        base, ty = kernel_key(r["Kernel_Name"])
        out[(base, ty, items)].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3)
    return out


def read_counter(path, counter):
    out = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        base, ty = kernel_key(r["Kernel_Name"])
        out[(base, ty, int(r["Grid_Size"]))].append(float(r["Counter_Value"]))
    return out


def copy_factor(counts, copy_mib):
    """True KiB / counter KiB for the largest copyBuffer dispatch."""
    keys = [k for k in counts if "copyBuffer" in k[0]]
    if not keys or not copy_mib:
        return None
    k = max(keys, key=lambda k: k[2])
    v = sum(counts[k]) / len(counts[k])
    return copy_mib * 1024.0 / v


def summarize(args):
    trace = read_trace(args.trace)
    fetch = read_counter(args.fetch, "FETCH_SIZE") if args.fetch else {}
    write = read_counter(args.write, "WRITE_SIZE") if args.write else {}
    ff = copy_factor(fetch, args.copy_mib) if fetch else None
    wf = copy_factor(write, args.copy_mib) if write else None
    rows, data = [], {}
    for key in sorted(trace, key=lambda k: -sum(trace[k])):
        base, ty, items = key
        if not base.startswith("k_"):
            continue
        d = trace[key]
        avg = sum(d) / len(d)
        fb = wb = None
        if ff and key in fetch:
            fb = sum(fetch[key]) / len(fetch[key]) * ff * 1024.0
        if wf and key in write:
            wb = sum(write[key]) / len(write[key]) * wf * 1024.0
        rows.append((base, ty, items, len(d), avg, fb, wb))
        data[f"{base}|{ty}|{items}"] = {"calls": len(d), "avg_us": avg, "fetch_bytes": fb, "write_bytes": wb}
    lines = [f"# {args.title}", "", "Commands (from the repository root; rocprofv3 run from /tmp):", ""]
    lines += [f"    {c}" for c in args.command]
    lines += ["", f"HIP source hash: `{source_hash()}` (paper_1707_09898_amd/csrc).", ""]
    if ff or wf:
        lines += [f"Traffic calibration: a {args.copy_mib} MiB copy kernel in the same program reads "
                  f"FETCH_SIZE x {ff:.3f} and WRITE_SIZE x {wf:.3f} of its true size; the factors are applied below.", ""]
    lines += ["| kernel | type | work items | launches | mean us | FETCH MB/launch | WRITE MB/launch |",
              "|---|---|---:|---:|---:|---:|---:|"]
    for base, ty, items, n, avg, fb, wb in rows:
        f = f"{fb / 1e6:.1f}" if fb is not None else "-"
        w = f"{wb / 1e6:.1f}" if wb is not None else "-"
        lines.append(f"| {base} | {ty} | {items} | {n} | {avg:.2f} | {f} | {w} |")
    lines += ["", "<!-- traffic-json", json.dumps({"source_hash": source_hash(), "kernels": data}), "-->", ""]
    with open(args.out, "w") as fo:
        fo.write("\n".join(lines))


# VALU issue: a wave64 VALU instruction occupies a 16-lane SIMD for 4 cycles;
# 256 CUs x 4 SIMDs at 2.4 GHz
SIMDS = 256 * 4
CLOCK_HZ = 2.4e9
CYCLES_PER_WAVE_INSTR = 4


def summarize_sq(args):
    """Per kernel launch shape: waves, VALU / LDS / vector-memory instructions
    per wave (SQ counters), and the time the VALU instructions alone take to
    issue over the whole chip, next to the mean duration from the trace."""
    trace = read_trace(args.trace)
    cnt = {c: read_counter(args.sq, c) for c in ("SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_LDS",
                                                  "SQ_INSTS_VMEM_RD", "SQ_INSTS_VMEM_WR")}
    lines = [f"# {args.title}", "", "Commands (from the repository root; rocprofv3 run from /tmp):", ""]
    lines += [f"    {c}" for c in args.command]
    lines += ["", f"HIP source hash: `{source_hash()}` (paper_1707_09898_amd/csrc).", "",
              f"VALU issue time = VALU instructions x {CYCLES_PER_WAVE_INSTR} cycles / ({SIMDS} SIMDs x "
              f"{CLOCK_HZ / 1e9:.1f} GHz): the kernel's duration if VALU issue were its only limit.", "",
              "| kernel | type | work items | waves | VALU/wave | LDS/wave | VMEM rd+wr/wave | VALU issue us | mean us | issue / mean |",
              "|---|---|---:|---:|---:|---:|---:|---:|---:|---:|"]
    rows = []
    for key, waves_l in cnt["SQ_WAVES"].items():
        base, ty, items = key
        if not base.startswith("k_") or key not in trace:
            continue
        avg = lambda c: sum(cnt[c][key]) / len(cnt[c][key]) if key in cnt[c] else 0.0
        waves = avg("SQ_WAVES")
        if waves <= 0:
            continue
        valu = avg("SQ_INSTS_VALU")
        issue_us = valu * CYCLES_PER_WAVE_INSTR / (SIMDS * CLOCK_HZ) * 1e6
        mean_us = sum(trace[key]) / len(trace[key])
        rows.append((mean_us, f"| {base} | {ty} | {items} | {waves:.0f} | {valu / waves:.0f} | "
                              f"{avg('SQ_INSTS_LDS') / waves:.0f} | "
                              f"{(avg('SQ_INSTS_VMEM_RD') + avg('SQ_INSTS_VMEM_WR')) / waves:.0f} | "
                              f"{issue_us:.2f} | {mean_us:.2f} | {issue_us / mean_us:.2f} |"))
    lines += [r for _, r in sorted(rows, key=lambda t: -t[0])]
    lines.append("")
    with open(args.out, "w") as fo:
        fo.write("\n".join(lines))


def lookup(summary_path, base, ty, items):
    """(fetch + write bytes per launch, hash matches the sources) from a
    summary, or (None, False) when the summary or the kernel is not there."""
    if not os.path.exists(summary_path):
        return None, False
    text = open(summary_path).read()
    m = re.search(r"<!-- traffic-json\n(.*?)\n-->", text, re.S)
    if not m:
        return None, False
    d = json.loads(m.group(1))
    k = d["kernels"].get(f"{base}|{ty}|{items}")
    if not k or k.get("fetch_bytes") is None or k.get("write_bytes") is None:
        return None, False
    return k["fetch_bytes"] + k["write_bytes"], d["source_hash"] == source_hash()


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--copy-mib", type=int, default=0)
    ap.add_argument("--command", action="append", default=[])
    ap.add_argument("--title", default="rocprofv3 summary")
    ap.add_argument("--sq", help="counter CSV of an SQ_WAVES / SQ_INSTS_* pass: write the VALU summary")
    ap.add_argument("--out", required=True)
    a = ap.parse_args()
    summarize_sq(a) if a.sq else summarize(a)
