"""Summaries of rocprofv3 output for the profiles/ folder.

    python -m paper_2204_06204_amd.profiling stats <kernel_stats.csv> <steps> <title> <command>
    python -m paper_2204_06204_amd.profiling pmc <fetch_dir> <write_dir> <copy_bytes> <title> <command> [json_out]

`stats` turns a --kernel-trace --stats CSV into a table of kernels with calls,
average duration and share.  `pmc` combines a FETCH_SIZE run and a
WRITE_SIZE run (each also holding a plain copy kernel of known size, used to
scale the counters) into HBM bytes per launch of the apply kernels.
"""
from __future__ import annotations

import csv
import glob
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNEL_SOURCES = ("paper_2204_06204_amd/csrc/kernels.hip", "paper_2204_06204_amd/csrc/device.h")
PROJECT_SORT_SOURCES = ("paper_2204_06204_amd/csrc/project_sort.hip", "paper_2204_06204_amd/csrc/device.h")


def kernel_hash(sources=KERNEL_SOURCES) -> str:
    """Short hash of the sources that define the profiled kernels (the
    apply and outer-iteration kernels by default)."""
    h = hashlib.sha256()
    for s in sources:
        with open(os.path.join(ROOT, s), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stats_table(path: str, steps: float, title: str, command: str) -> str:
    """Per-kernel table of a --kernel-trace --stats run.  The streaming
    calibration kernel (torch's b = 2 a, run after the profiled work) is
    listed but left out of the per-step total."""
    rows = list(csv.DictReader(open(path)))
    tot = sum(float(r["TotalDurationNs"]) for r in rows if "AUnaryFunctor" not in r["Name"])
    out = [f"# {title}", "", f"Command: `{command}`", "",
           f"kernel-source hash: {kernel_hash()}", "",
           "| kernel | calls | avg us | per step us | share |", "|---|---:|---:|---:|---:|"]
    for r in rows:
        name = r["Name"].replace("|", "/")[:110]
        out.append(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                   f"{float(r['TotalDurationNs']) / steps / 1e3:.2f} | {float(r['Percentage']):.1f}% |")
    out.append("")
    out.append(f"Total kernel time per step: {tot / steps / 1e3:.1f} us")
    return "\n".join(out) + "\n"


def _counter_rows(d: str):
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    rows = []
    for f in files:
        rows += list(csv.DictReader(open(f)))
    return rows


def pmc_summary(fetch_dir: str, write_dir: str, copy_bytes: float, title: str, command: str) -> str:
    """Counter values are KiB per dispatch (summed over the agent).  The copy
    kernel moves copy_bytes in and out; its measured bytes give the scale."""
    res = {}
    for kind, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = _counter_rows(d)
        per = {}
        for r in rows:
            name = r.get("Kernel_Name", r.get("Kernel-Name", ""))
            if r.get("Counter_Name") != kind:
                continue
            per.setdefault(name, []).append(float(r["Counter_Value"]) * 1024.0)
        res[kind] = per
    def pick(per, key):
        vals = [v for n, vs in per.items() if key in n for v in vs]
        return sum(vals) / len(vals) if vals else None
    def calib(per):
        # the calibration kernel: b = 2 a over copy_bytes (torch's MulFunctor)
        vals = [sum(v) / len(v) for n, v in per.items() if "MulFunctor" in n]
        return max(vals) if vals else None
    copy_f = calib(res["FETCH_SIZE"])
    copy_w = calib(res["WRITE_SIZE"])
    sf = copy_bytes / copy_f if copy_f else None
    sw = copy_bytes / copy_w if copy_w else None
    lines = [f"# {title}", "", f"Command: `{command}`", "", f"kernel_hash: {kernel_hash()}",
             f"copy scale fetch: {sf}", f"copy scale write: {sw}", ""]
    data = {"kernel_hash": kernel_hash(), "scale_fetch": sf, "scale_write": sw, "kernels": {}}
    for n in sorted(set(res["FETCH_SIZE"]) | set(res["WRITE_SIZE"])):
        if "fbto::" not in n and "MulFunctor" not in n:
            continue  # torch's own set-up kernels
        f = pick(res["FETCH_SIZE"], n)
        w = pick(res["WRITE_SIZE"], n)
        fb = f * sf if (f is not None and sf) else None
        wb = w * sw if (w is not None and sw) else None
        data["kernels"][n if "fbto::" in n else n[:120]] = {"fetch_bytes": fb, "write_bytes": wb}
        lines.append(f"- `{n[:100]}`: fetch {fb} B, write {wb} B per dispatch")
    lines += ["", "```json", json.dumps(data, indent=1), "```", ""]
    return "\n".join(lines)


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        print(stats_table(sys.argv[2], float(sys.argv[3]), sys.argv[4], sys.argv[5]), end="")
    elif sys.argv[1] == "pmc":
        text = pmc_summary(sys.argv[2], sys.argv[3], float(sys.argv[4]), sys.argv[5], sys.argv[6])
        print(text, end="")
        if len(sys.argv) > 7:
            block = text.split("```json", 1)[1].split("```", 1)[0]
            with open(sys.argv[7], "w") as fh:
                fh.write(block.strip() + "\n")
