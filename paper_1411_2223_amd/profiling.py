"""Helpers that turn rocprofv3 CSV output into the short summaries kept under
profiles/, and that tie hardware-counter traffic to the kernel sources it was
measured on (a counter figure is only reported while those sources are unchanged).

    python -m paper_1411_2223_amd.profiling stats <kernel_stats.csv> [--top N]
    python -m paper_1411_2223_amd.profiling counters <fetch counter_collection.csv> <write counter_collection.csv>
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
KERNEL_SOURCES = ("csrc/dslash.hip", "csrc/asq_device.h", "csrc/asq_reduce.h", "csrc/asq_internal.h")
COUNTERS_FILE = os.path.join(ROOT, "profiles", "dslash_counters.json")


def kernel_source_hash() -> str:
    """SHA-256 over the sources that define the Dslash kernels."""
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def stats_table(path: str, top: int = 15) -> str:
    """Markdown table from a rocprofv3 --stats kernel_stats.csv."""
    rows = list(csv.DictReader(open(path)))
    out = ["| kernel | calls | avg us | min us | max us | % time |", "|---|---|---|---|---|---|"]
    for r in rows[:top]:
        out.append(f"| `{short_name(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                   f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | {float(r['Percentage']):.2f} |")
    return "\n".join(out)


def short_name(name: str) -> str:
    n = name.replace("asq::(anonymous namespace)::", "").replace("asq::", "").replace("void ", "")
    n = n.replace("(DslashArgs)", "").replace("(VecArgs)", "")
    return n[:110]


def counter_means(path: str, counter: str) -> dict:
    """kernel name -> (dispatches, mean counter value per dispatch) from counter_collection.csv."""
    acc = defaultdict(list)
    for r in csv.DictReader(open(path)):
        if r.get("Counter_Name", r.get("counter_name")) != counter:
            continue
        name = r.get("Kernel_Name", r.get("kernel_name"))
        acc[name].append(float(r.get("Counter_Value", r.get("value"))))
    return {k: (len(v), sum(v) / len(v)) for k, v in acc.items()}


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s1 = sub.add_parser("stats")
    s1.add_argument("csv")
    s1.add_argument("--top", type=int, default=15)
    s2 = sub.add_parser("counters")
    s2.add_argument("fetch_csv")
    s2.add_argument("write_csv")
    s3 = sub.add_parser("hash")
    a = ap.parse_args()
    if a.cmd == "stats":
        print(stats_table(a.csv, a.top))
    elif a.cmd == "hash":
        print(kernel_source_hash())
    else:
        fetch = counter_means(a.fetch_csv, "FETCH_SIZE")
        write = counter_means(a.write_csv, "WRITE_SIZE")
        res = {}
        for k in sorted(set(fetch) | set(write)):
            res[short_name(k)] = {"dispatches": fetch.get(k, (0, 0))[0], "FETCH_SIZE_KiB": fetch.get(k, (0, None))[1],
                                  "WRITE_SIZE_KiB": write.get(k, (0, None))[1]}
        print(json.dumps(res, indent=1))


if __name__ == "__main__":
    main()
