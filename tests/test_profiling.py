"""The host arithmetic behind the bench line's `traffic` figure (CPU only): counter CSVs
are averaged over the timed dispatches, scaled by the copy kernel's calibration, and
used only while the Dslash sources hash matches the one recorded with them.

Synthetic counter files stand in for rocprofv3 output (same columns).
"""
import csv
import json
import os

import pytest

import bench
from paper_1411_2223_amd import profiling

FIELDS = ["Correlation_Id", "Dispatch_Id", "Grid_Size", "Kernel_Name", "Counter_Name", "Counter_Value"]


def dslash_name(link, vin, vout, cols, epi, pipe):
    return (f"void asq::(anonymous namespace)::dslash_kernel<asq::{link}, asq::{vin}, asq::{vout}, {cols}, {epi}, "
            f"{'true' if pipe else 'false'}>(asq::DslashArgs)")


def write_csv(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for i, (name, grid, value) in enumerate(rows, 1):
            w.writerow({"Correlation_Id": i, "Dispatch_Id": i, "Grid_Size": grid, "Kernel_Name": name,
                        "Counter_Name": counter, "Counter_Value": value})


def test_counter_means_last_dispatches(tmp_path):
    p = tmp_path / "c.csv"
    a = dslash_name("LinkF32R18", "VecF32", "VecF32", 1, 0, True)
    rows = [(a, 256000, 1000.0)] * 3 + [(a, 256000, 10.0), (a, 256000, 20.0), ("copy_kernel(x)", 64, 5.0)]
    write_csv(p, "FETCH_SIZE", rows)
    m = profiling.counter_means(str(p), "FETCH_SIZE", by_grid=True)
    assert m[(a, 256000)] == (5, (3000.0 + 30.0) / 5)
    last = profiling.counter_means(str(p), "FETCH_SIZE", by_grid=True, last=2)
    assert last[(a, 256000)] == (2, 15.0)
    assert profiling.counter_means(str(p), "WRITE_SIZE") == {}


def _counter_runs(tmp_path):
    """FETCH and WRITE files for the 20^3 x 64 kernels-only run: a 1 GiB copy read at
    524288 KiB (factor 2) and written at 1048576 KiB (factor 1), tuner trials first."""
    H = 20 * 20 * 20 * 64 // 2
    nblk = (H + 255) // 256
    spec = {
        "f32_f32_1rhs": (dslash_name("LinkF32R18", "VecF32", "VecF32", 1, 0, True), nblk * 256, 20, 150000.0, 6000.0),
        "f64_f64_1rhs": (dslash_name("LinkF64R18", "VecF64", "VecF64", 1, 0, False), nblk * 256, 20, 300000.0,
                         12000.0),
        "f16_f32_1rhs": (dslash_name("LinkF32R18", "VecF16", "VecF16", 1, 0, True), nblk * 256, 20, 148000.0,
                         4000.0),
        "f16_f32_96rhs": (dslash_name("LinkF32R18", "VecF16", "VecF16", 8, 0, True), nblk * 256 * 12, 12, 1.8e6,
                          384000.0),
    }
    fetch, write = [], []
    copy = "void asq::(anonymous namespace)::copy_kernel(uint4*, uint4 const*, unsigned long)"
    for key, (name, grid, n, f, w) in spec.items():
        # three trial launches of the same variant with other values, then the timed ones
        fetch += [(name, grid, 9e9)] * 3 + [(name, grid, f)] * n
        write += [(name, grid, 9e9)] * 3 + [(name, grid, w)] * n
        # a non-plain epilogue of the same tier must not be picked
        fetch.append((name.replace(", 0, ", ", 1, "), grid, 1.0))
        write.append((name.replace(", 0, ", ", 1, "), grid, 1.0))
    fetch.append((copy, 1 << 20, 524288.0))
    write.append((copy, 1 << 20, 1048576.0))
    fp, wp = tmp_path / "fetch.csv", tmp_path / "write.csv"
    write_csv(fp, "FETCH_SIZE", fetch)
    write_csv(wp, "WRITE_SIZE", write)
    return str(fp), str(wp), spec


def test_write_counters_calibration_and_bench_lookup(tmp_path, monkeypatch):
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(profiling, "ROOT", str(tmp_path))
    fp, wp, spec = _counter_runs(tmp_path)
    profiling.write_counters(fp, wp, "20x20x20x64")
    out = json.load(open(tmp_path / "profiles" / "dslash_counters_20x20x20x64.json"))
    assert out["fetch_factor"] == 2.0 and out["write_factor"] == 1.0
    assert out["kernel_source_sha"] == profiling.kernel_source_hash()
    for key, (name, grid, n, f, w) in spec.items():
        k = out["kernels"][key]
        assert (k["FETCH_SIZE_KiB"], k["WRITE_SIZE_KiB"], k["dispatches"], k["grid_threads"]) == (f, w, n, grid)
    assert os.path.exists(tmp_path / "profiles" / "dslash_counters_20x20x20x64.md")
    # bench.py's figure: bytes = 1024 (2 FETCH + WRITE) while the sources hash matches
    want = 1024.0 * (2.0 * 150000.0 + 6000.0)
    assert bench.measured_traffic("f32_f32_1rhs", 307200000) == pytest.approx(want)
    assert bench.measured_traffic("no_such_key", 1) is None
    # any change to the Dslash sources voids the counters
    monkeypatch.setattr(profiling, "kernel_source_hash", lambda: "0000000000000000")
    assert bench.measured_traffic("f32_f32_1rhs", 307200000) is None


def test_committed_counter_files_are_complete():
    # every key bench.py looks up is there, with a calibration near the copy kernel's 2 : 1
    for lattice, spec in profiling.KERNELS_ONLY.items():
        c = json.load(open(profiling.counters_file(lattice)))
        assert len(c["kernel_source_sha"]) == 16
        assert 1.9 < c["fetch_factor"] < 2.1 and 0.95 < c["write_factor"] < 1.05
        assert set(c["kernels"]) == {k for k in spec if k != "workload"}, lattice
