"""Helpers that turn rocprofv3 CSV output into the short summaries kept under
profiles/, and that tie hardware-counter traffic to the kernel sources it was
measured on (a counter figure is only reported while those sources are unchanged).

    python -m paper_1411_2223_amd.profiling stats <kernel_stats.csv> [--top N]
    python -m paper_1411_2223_amd.profiling counters <fetch counter_collection.csv> <write counter_collection.csv>
    python -m paper_1411_2223_amd.profiling write-counters <fetch csv> <write csv> --dir <run dir>
    python -m paper_1411_2223_amd.profiling write-stats <kernel_stats.csv> <bench log> --out <md> --title T --command C
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


# Dslash launches of `bench.py --kernels-only` at 20^3 x 64 (256 000 output sites),
# keyed like bench.py's roofline lookup: (vector tier)_(link tier)_1rhs.
KERNELS_ONLY = {
    "f32_f32_1rhs": ("dslash_kernel<LinkF32R18, VecF32, VecF32, ", (16 * 72 + 2 * 24) * 256000),
    "f64_f64_1rhs": ("dslash_kernel<LinkF64R18, VecF64, VecF64, ", (16 * 144 + 2 * 48) * 256000),
    "f16_f32_1rhs": ("dslash_kernel<LinkF32R18, VecF16, VecF16, ", (16 * 72 + 2 * 16) * 256000),
}
COPY_KERNEL = "copy_kernel"
COPY_BYTES = 1 << 30


def write_counters(fetch_csv: str, write_csv: str, run_dir: str) -> None:
    """profiles/dslash_counters.json (read by bench.py) and its Markdown summary."""
    fetch = counter_means(fetch_csv, "FETCH_SIZE")
    write = counter_means(write_csv, "WRITE_SIZE")

    def is_plain(name):
        # a plain-epilogue Dslash (template argument 5 is 0), or any other kernel
        n = short_name(name)
        return not n.startswith("dslash_kernel<") or n.split(", ")[4] == "0"

    def find(prefix):
        # the launch variant the timed loop used: the one with the most dispatches
        hits = [k for k in fetch if short_name(k).startswith(prefix) and is_plain(k)]
        if not hits:
            raise KeyError(prefix)
        return max(hits, key=lambda k: fetch[k][0])

    copy = find(COPY_KERNEL)
    ff = COPY_BYTES / 1024 / fetch[copy][1]
    wf = COPY_BYTES / 1024 / write[copy][1]
    h = kernel_source_hash()
    kernels = {}
    for key, (prefix, _) in KERNELS_ONLY.items():
        k = find(prefix)
        kernels[key] = {"FETCH_SIZE_KiB": fetch[k][1], "WRITE_SIZE_KiB": write[k][1], "dispatches": fetch[k][0],
                        "kernel": short_name(k)}
    cmds = [f"rocprofv3 --pmc FETCH_SIZE --output-format csv -d {run_dir}/fetch -o k -- python -u bench.py --kernels-only",
            f"rocprofv3 --pmc WRITE_SIZE --output-format csv -d {run_dir}/write -o k -- python -u bench.py --kernels-only",
            f"python -m paper_1411_2223_amd.profiling write-counters {fetch_csv} {write_csv} --dir {run_dir}"]
    out = {"kernel_source_sha": h, "lattice": "20x20x20x64", "fetch_factor": round(ff, 4), "write_factor": round(wf, 4),
           "calibration": {"copy_bytes_read": COPY_BYTES, "copy_bytes_written": COPY_BYTES,
                           "copy_FETCH_SIZE_KiB": fetch[copy][1], "copy_WRITE_SIZE_KiB": write[copy][1]},
           "commands": cmds, "kernels": kernels}
    with open(COUNTERS_FILE, "w") as f:
        json.dump(out, f, indent=1)
    lines = ["# Dslash HBM traffic from hardware counters, 20^3x64, 1 column", "",
             "Commands (repository root on the MI355X box, one counter per pass):", ""]
    lines += ["    " + c for c in cmds]
    lines += ["", f"Kernel sources hash (`python -m paper_1411_2223_amd.profiling hash`): `{h}`", "",
              f"Calibration with the plain copy kernel (`asq_copy_probe`, {COPY_BYTES >> 30} GiB read + "
              f"{COPY_BYTES >> 30} GiB written): FETCH_SIZE = {fetch[copy][1]:.1f} KiB, WRITE_SIZE = "
              f"{write[copy][1]:.1f} KiB per dispatch, so bytes = 1024 x ({ff:.4f} x FETCH_SIZE + {wf:.4f} x "
              f"WRITE_SIZE).", "",
              "| key | kernel (dispatches) | FETCH_SIZE KiB | WRITE_SIZE KiB | measured MB/launch | "
              "algorithmic MB/launch | measured / algorithmic |", "|---|---|---|---|---|---|---|"]
    for key, (prefix, alg) in KERNELS_ONLY.items():
        v = kernels[key]
        m = 1024 * (ff * v["FETCH_SIZE_KiB"] + wf * v["WRITE_SIZE_KiB"])
        lines.append(f"| `{key}` | `{v['kernel']}` ({v['dispatches']}) | {v['FETCH_SIZE_KiB']:.0f} | "
                     f"{v['WRITE_SIZE_KiB']:.0f} | {m / 1e6:.1f} | {alg / 1e6:.1f} | {m / alg:.3f} |")
    lines += ["", "Algorithmic bytes per output site: 16 links (72 B FP32 / 144 B FP64 18-real) + one input and one",
              "output colour vector (24 B FP32, 48 B FP64, 16 B FP16-with-norm); 256 000 output sites per launch.",
              "Reads above the algorithmic count are neighbour vectors fetched into more than one XCD's L2."]
    with open(os.path.join(ROOT, "profiles", "dslash_counters_20x20x20x64.md"), "w") as f:
        f.write("\n".join(lines) + "\n")


def write_stats(stats_csv: str, log: str, out: str, title: str, command: str, top: int = 14, note: str = "") -> None:
    bench = [l.rstrip() for l in open(log) if l.startswith("[bench]")]
    lines = [f"# {title}", "", "Command (repository root, MI355X box):", "", "    " + command,
             f"    python -m paper_1411_2223_amd.profiling stats {stats_csv} --top {top}", ""]
    if note:
        lines += [note, ""]
    lines += ["Template arguments of `dslash_kernel`: link tier, input tier, output (or residual) tier, columns",
              "per thread, epilogue (0 plain, 1 |out|^2, 2 update of r and x, 3 FP64 residual), software-pipelined",
              "hop loop.  Minimum durations near 1 us are masked no-op launches (columns that are converged or",
              "did not ask for a reliable update).", "", stats_table(stats_csv, top), "", "bench output of that run:", ""]
    lines += ["    " + l for l in bench]
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")


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
    s4 = sub.add_parser("write-counters")
    s4.add_argument("fetch_csv")
    s4.add_argument("write_csv")
    s4.add_argument("--dir", required=True)
    s5 = sub.add_parser("write-stats")
    s5.add_argument("csv")
    s5.add_argument("log")
    s5.add_argument("--out", required=True)
    s5.add_argument("--title", required=True)
    s5.add_argument("--command", required=True)
    s5.add_argument("--note", default="")
    s5.add_argument("--top", type=int, default=14)
    a = ap.parse_args()
    if a.cmd == "write-counters":
        write_counters(a.fetch_csv, a.write_csv, a.dir)
        return
    if a.cmd == "write-stats":
        write_stats(a.csv, a.log, a.out, a.title, a.command, a.top, a.note)
        return
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
