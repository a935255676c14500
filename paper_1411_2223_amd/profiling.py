"""Helpers that turn rocprofv3 CSV output into the short summaries kept under
profiles/, and that tie hardware-counter traffic to the kernel sources it was
measured on (a counter figure is only reported while those sources are unchanged).

    python -m paper_1411_2223_amd.profiling stats <kernel_stats.csv> [--top N]
    python -m paper_1411_2223_amd.profiling counters <fetch counter_collection.csv> <write counter_collection.csv>
    python -m paper_1411_2223_amd.profiling write-counters <fetch csv> <write csv> [--lattice L]
    python -m paper_1411_2223_amd.profiling write-stats <kernel_stats.csv> <bench log> --out <md> --title T --command C
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import re
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
KERNEL_SOURCES = ("csrc/dslash.hip", "csrc/dslash_impl.h", "csrc/dslash_mfma.h", "csrc/dslash_f64.hip", "csrc/dslash_f32.hip",
                  "csrc/dslash_r12.hip", "csrc/dslash_i16.hip", "csrc/dslash_f64f32.hip", "csrc/asq_device.h", "csrc/asq_reduce.h",
                  "csrc/asq_internal.h")


def counters_file(lattice: str) -> str:
    """Counter figures of one lattice's Dslash launches (read by bench.py)."""
    return os.path.join(ROOT, "profiles", f"dslash_counters_{lattice}.json")



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


def counter_means(path: str, counter: str, by_grid: bool = False, last: int = 0) -> dict:
    """kernel name (or (name, grid size in threads)) -> (dispatches, mean counter value per
    dispatch) from counter_collection.csv; with last > 0 over the last `last` dispatches
    only (the timed launches, after the autotuner's trials of other variants of the
    same kernel)."""
    acc = defaultdict(list)
    for r in csv.DictReader(open(path)):
        if r.get("Counter_Name", r.get("counter_name")) != counter:
            continue
        name = r.get("Kernel_Name", r.get("kernel_name"))
        key = (name, int(r["Grid_Size"])) if by_grid else name
        acc[key].append((int(r["Dispatch_Id"]), float(r.get("Counter_Value", r.get("value")))))
    out = {}
    for k, v in acc.items():
        vals = [x for _, x in sorted(v)]
        if last > 0:
            vals = vals[-last:]
        out[k] = (len(vals), sum(vals) / len(vals))
    return out


# Dslash launches of `bench.py [--workload ...] --kernels-only` per lattice, keyed
# like bench.py's traffic lookup: (vector tier)_(link tier)_(columns)rhs ->
# (kernel name prefix, algorithmic bytes per launch, columns).
H20 = 20 * 20 * 20 * 64 // 2
H48 = 48 * 48 * 48 * 96 // 2
HALF = {"20x20x20x64": H20, "48x48x48x96": H48}
KERNELS_ONLY = {
    "20x20x20x64": {
        "workload": "single_20x20x20x64",
        "f32_f32_1rhs": ("dslash_kernel<LinkF32R18, VecF32, VecF32, ", (16 * 72 + 2 * 24) * H20, 1, 20),
        "f64_f64_1rhs": ("dslash_kernel<LinkF64R18, VecF64, VecF64, ", (16 * 144 + 2 * 48) * H20, 1, 20),
        "f16_f32_1rhs": ("dslash_kernel<LinkF32R18, VecF16, VecF16, ", (16 * 72 + 2 * 16) * H20, 1, 20),
        "f16_f32_96rhs": ("dslash_kernel<LinkF32R18, VecF16, VecF16, ", (16 * 72 + 96 * 2 * 16) * H20, 96, 12),
    },
    "48x48x48x96": {
        "workload": "threelevel_48x48x48x96",
        "f16_f16r12_12rhs": ("dslash_kernel<LinkI16R12, VecF16, VecF16, ", (16 * 24 + 12 * 2 * 16) * H48, 12, 10),
        "f64_f64_12rhs": ("dslash_kernel<LinkF64R18, VecF64, VecF64, ", (16 * 144 + 12 * 2 * 48) * H48, 12, 5),
        "f32_f32_1rhs_r18": ("dslash_kernel<LinkF32R18, VecF32, VecF32, ", (16 * 72 + 2 * 24) * H48, 1, 20),
        "f64_f64_1rhs_r18": ("dslash_kernel<LinkF64R18, VecF64, VecF64, ", (16 * 144 + 2 * 48) * H48, 1, 20),
    },
}
COPY_KERNEL = "copy_kernel"
COPY_BYTES = 1 << 30


def write_counters(fetch_csv: str, write_csv: str, lattice: str = "20x20x20x64", tune_cache: str = "") -> None:
    """profiles/dslash_counters_<lattice>.json (read by bench.py) and its Markdown summary."""
    spec = KERNELS_ONLY[lattice]
    fetch = counter_means(fetch_csv, "FETCH_SIZE", by_grid=True)
    write = counter_means(write_csv, "WRITE_SIZE", by_grid=True)
    # the timed launches of each key: the last dispatches of its variant
    fetch_last = {key: counter_means(fetch_csv, "FETCH_SIZE", by_grid=True, last=spec[key][3])
                  for key in spec if key != "workload"}
    write_last = {key: counter_means(write_csv, "WRITE_SIZE", by_grid=True, last=spec[key][3])
                  for key in spec if key != "workload"}
    nblk = (HALF[lattice] + 255) // 256

    def is_plain(name):
        # a plain-epilogue Dslash (template argument 5 is 0), or any other kernel
        n = short_name(name)
        return not n.startswith("dslash_kernel<") or n.split(", ")[4] == "0"

    def tile(name):
        n = short_name(name)
        return int(n.split(", ")[3]) if n.startswith("dslash_kernel<") else 0

    def find(prefix, ncol=0):
        # the launch variant the timed loop used: among launches over ncol columns
        # (grid = site blocks x column tiles), the one with the most dispatches; a
        # link tier read with streaming loads counts as that tier
        hits = [(k, g) for (k, g) in fetch
                if re.sub(r"Streamed<(\w+)>", r"\1", short_name(k)).startswith(prefix) and is_plain(k)
                and (ncol == 0 or g == nblk * 256 * -(-ncol // tile(k)))]
        if not hits:
            raise KeyError(prefix)
        return max(hits, key=lambda k: fetch[k][0])

    copy = find(COPY_KERNEL)
    ff = COPY_BYTES / 1024 / fetch[copy][1]
    wf = COPY_BYTES / 1024 / write[copy][1]
    h = kernel_source_hash()
    kernels = {}
    keys = [k for k in spec if k != "workload"]
    for key in keys:
        k = find(spec[key][0], spec[key][2])
        fl, wl_ = fetch_last[key][k], write_last[key][k]
        kernels[key] = {"FETCH_SIZE_KiB": fl[1], "WRITE_SIZE_KiB": wl_[1], "dispatches": fl[0],
                        "kernel": short_name(k[0]), "grid_threads": k[1]}
    wl = "" if spec["workload"] == "single_20x20x20x64" else f"--workload {spec['workload']} "
    # each pass wrote its CSV into the directory given to -d
    # with a tune cache, an unprofiled run picks the launch variants first and both
    # counter passes take them from the file (no timing under the profiler)
    env = f"ASQ_TUNE_CACHE={tune_cache} " if tune_cache else ""
    cmds = ([f"{env}python -u bench.py {wl}--kernels-only"] if tune_cache else []) + [
        f"{env}rocprofv3 --pmc FETCH_SIZE --output-format csv -d {os.path.dirname(fetch_csv)} -o k -- "
        f"python -u bench.py {wl}--kernels-only",
        f"{env}rocprofv3 --pmc WRITE_SIZE --output-format csv -d {os.path.dirname(write_csv)} -o k -- "
        f"python -u bench.py {wl}--kernels-only",
        f"python -m paper_1411_2223_amd.profiling write-counters {fetch_csv} {write_csv} --lattice {lattice}"
        + (f" --tune-cache {tune_cache}" if tune_cache else "")]
    out = {"kernel_source_sha": h, "lattice": lattice, "fetch_factor": round(ff, 4), "write_factor": round(wf, 4),
           "calibration": {"copy_bytes_read": COPY_BYTES, "copy_bytes_written": COPY_BYTES,
                           "copy_FETCH_SIZE_KiB": fetch[copy][1], "copy_WRITE_SIZE_KiB": write[copy][1]},
           "commands": cmds, "kernels": kernels}
    with open(counters_file(lattice), "w") as f:
        json.dump(out, f, indent=1)
    lines = [f"# Dslash HBM traffic from hardware counters, {lattice}",
             "", "Commands (repository root on the MI355X box, one counter per pass):", ""]
    lines += ["    " + c for c in cmds]
    lines += ["", f"Kernel sources hash (`python -m paper_1411_2223_amd.profiling hash`): `{h}`", "",
              "Each row averages the timed launches of the variant the autotuner chose (the last",
              "dispatches of that kernel and grid; the tuner's trial launches come first)"
              + (", taken by both passes from the tune cache of the unprofiled first run." if tune_cache else "."),
              "",
              f"Calibration with the plain copy kernel (`asq_copy_probe`, {COPY_BYTES >> 30} GiB read + "
              f"{COPY_BYTES >> 30} GiB written): FETCH_SIZE = {fetch[copy][1]:.1f} KiB, WRITE_SIZE = "
              f"{write[copy][1]:.1f} KiB per dispatch, so bytes = 1024 x ({ff:.4f} x FETCH_SIZE + {wf:.4f} x "
              f"WRITE_SIZE).", "",
              "| key | kernel (dispatches) | FETCH_SIZE KiB | WRITE_SIZE KiB | measured MB/launch | "
              "algorithmic MB/launch | measured / algorithmic |", "|---|---|---|---|---|---|---|"]
    for key in keys:
        alg = spec[key][1]
        v = kernels[key]
        kernels[key]["alg_bytes"] = alg
        m = 1024 * (ff * v["FETCH_SIZE_KiB"] + wf * v["WRITE_SIZE_KiB"])
        lines.append(f"| `{key}` | `{v['kernel']}` ({v['dispatches']}) | {v['FETCH_SIZE_KiB']:.0f} | "
                     f"{v['WRITE_SIZE_KiB']:.0f} | {m / 1e6:.1f} | {alg / 1e6:.1f} | {m / alg:.3f} |")
    lines += ["", "Algorithmic bytes per output site: 16 links (144 B FP64 / 72 B FP32 18-real, 24 B 16-bit",
              "12-real) + one input and one output colour vector per column (48 B FP64, 24 B FP32, 16 B",
              "FP16-with-norm). Reads above the algorithmic count are neighbour vectors fetched into more",
              "than one XCD's L2."]
    with open(os.path.join(ROOT, "profiles", f"dslash_counters_{lattice}.md"), "w") as f:
        f.write("\n".join(lines) + "\n")


def trace_durations(trace_csv: str) -> dict:
    """(kernel name, grid size in threads) -> durations in ns, in dispatch order, from a
    rocprofv3 kernel_trace.csv."""
    acc = defaultdict(list)
    for r in csv.DictReader(open(trace_csv)):
        key = (r["Kernel_Name"], int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"]))
        acc[key].append((int(r["Dispatch_Id"]), int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
    return {k: [d for _, d in sorted(v)] for k, v in acc.items()}


def write_valu(counter_csv: str, trace_csv: str, out: str, command: str, lattice: str = "20x20x20x64",
               clock_ghz: float = 2.4, cus: int = 256) -> None:
    """VALU issue utilization of the timed Dslash launches: SQ_INSTS_VALU per launch (wave
    instructions; a wave64 VALU instruction occupies its 16-lane SIMD for 4 cycles, so a
    CU issues at most one per cycle) over cus x clock x the launch's duration, taken from a
    kernel-trace run of the same command (counter runs serialize and slow the kernels)."""
    spec = KERNELS_ONLY[lattice]
    nblk = (HALF[lattice] + 255) // 256
    durs = trace_durations(trace_csv)
    full = counter_means(counter_csv, "SQ_INSTS_VALU", by_grid=True)
    lines = [f"# Dslash VALU issue utilization, {lattice}", "", "Commands (repository root on the MI355X box):", "",
             "    " + command,
             f"    python -m paper_1411_2223_amd.profiling write-valu {counter_csv} {trace_csv} --out {out} "
             f"--command '...'", "",
             "Utilization = SQ_INSTS_VALU / (CUs x clock x duration): a CU issues at most one wave64 VALU",
             f"instruction per cycle (4 SIMDs, 4 cycles each); {cus} CUs at {clock_ghz} GHz.  Both figures are",
             "averages over the timed launches of the variant the autotuner chose (the last dispatches of",
             "that kernel and grid); durations come from the kernel-trace run.", "",
             "| key | kernel | VALU wave-instructions per launch | flops per VALU lane-op | duration us | VALU issue |",
             "|---|---|---|---|---|---|"]
    for key in [k for k in spec if k != "workload"]:
        prefix, alg, ncol, last = spec[key]

        def tile(name):
            return int(short_name(name).split(", ")[3])

        hits = [(k, g) for (k, g) in full
                if re.sub(r"Streamed<(\w+)>", r"\1", short_name(k)).startswith(prefix) and short_name(k).split(", ")[4] == "0"
                and g == nblk * 256 * -(-ncol // tile(k))]
        if not hits:
            continue
        k = max(hits, key=lambda h: full[h][0])
        n_valu = counter_means(counter_csv, "SQ_INSTS_VALU", by_grid=True, last=last)[k][1]
        d = durs.get(k, [])[-last:]
        d_us = sum(d) / len(d) / 1e3 if d else float("nan")
        util = n_valu / (cus * clock_ghz * 1e3 * d_us) if d else float("nan")
        flops = 1146.0 * HALF[lattice] * ncol
        lines.append(f"| `{key}` | `{short_name(k[0])}` | {n_valu:.3e} | {flops / (64 * n_valu):.2f} | {d_us:.1f} | "
                     f"{util:.2f} |")
    lines += ["", "Flops per VALU lane-operation counts 1146 flops per site and column; an FMA is 2."]
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")


def launches_by_grid(trace_csv: str, kernel: str) -> dict:
    """grid size in work-items -> (launches, mean, min, max duration in us) of the kernel
    whose short name is `kernel`, from a rocprofv3 kernel_trace.csv."""
    acc = defaultdict(list)
    for r in csv.DictReader(open(trace_csv)):
        if short_name(r["Kernel_Name"]) != kernel:
            continue
        acc[int(r["Grid_Size_X"])].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    return {g: (len(v), sum(v) / len(v), min(v), max(v)) for g, v in sorted(acc.items())}


def write_stats(stats_csv: str, log: str, out: str, title: str, command: str, top: int = 14, note: str = "",
                focus: str = "") -> None:
    bench = [l.rstrip() for l in open(log) if l.startswith("[bench]")]
    lines = [f"# {title}", "", "Command (repository root, MI355X box):", "", "    " + command,
             f"    python -m paper_1411_2223_amd.profiling stats {stats_csv} --top {top}", ""]
    if note:
        lines += [note, ""]
    if focus:
        trace = stats_csv.replace("_kernel_stats.csv", "_kernel_trace.csv")
        lines += [f"Launches of `{focus}` by grid size (work-items), from the kernel trace of the same run",
                  f"(`python -m paper_1411_2223_amd.profiling grid {trace} '{focus}'`):", "",
                  "| grid | launches | avg us | min us | max us |", "|---|---|---|---|---|"]
        for g, (n, avg, lo, hi) in launches_by_grid(trace, focus).items():
            lines.append(f"| {g} | {n} | {avg:.2f} | {lo:.2f} | {hi:.2f} |")
        lines.append("")
    lines += ["Template arguments of `dslash_kernel`: link tier, input tier, output (or residual) tier, columns",
              "per thread, epilogue (0 plain, 1 |out|^2, 2 update of r and x, 3 FP64 residual), software-pipelined",
              "hop loop, LDS window of x and y neighbours.  Minimum durations near 1 us are masked no-op launches",
              "(columns that are converged or did not ask for a reliable update).", "", stats_table(stats_csv, top), "", "bench output of that run:", ""]
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
    s4.add_argument("--lattice", default="20x20x20x64", choices=sorted(KERNELS_ONLY))
    s4.add_argument("--tune-cache", default="", help="the ASQ_TUNE_CACHE file the passes shared")
    s5 = sub.add_parser("write-stats")
    s5.add_argument("csv")
    s5.add_argument("log")
    s5.add_argument("--out", required=True)
    s5.add_argument("--title", required=True)
    s5.add_argument("--command", required=True)
    s5.add_argument("--note", default="")
    s5.add_argument("--top", type=int, default=14)
    s5.add_argument("--focus", default="", help="a kernel's short name: its launches by grid size")
    s7 = sub.add_parser("grid")
    s7.add_argument("trace_csv")
    s7.add_argument("kernel")
    s6 = sub.add_parser("write-valu")
    s6.add_argument("counter_csv")
    s6.add_argument("trace_csv")
    s6.add_argument("--out", required=True)
    s6.add_argument("--command", required=True)
    s6.add_argument("--lattice", default="20x20x20x64", choices=sorted(KERNELS_ONLY))
    a = ap.parse_args()
    if a.cmd == "write-valu":
        write_valu(a.counter_csv, a.trace_csv, a.out, a.command, a.lattice)
        return
    if a.cmd == "write-counters":
        write_counters(a.fetch_csv, a.write_csv, a.lattice, a.tune_cache)
        return
    if a.cmd == "write-stats":
        write_stats(a.csv, a.log, a.out, a.title, a.command, a.top, a.note, a.focus)
        return
    if a.cmd == "grid":
        for g, (n, avg, lo, hi) in launches_by_grid(a.trace_csv, a.kernel).items():
            print(f"grid {g}: {n} launches, avg {avg:.2f} us, min {lo:.2f}, max {hi:.2f}")
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
