"""Benchmark of the even-odd asqtad CG on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]             # the headline line
    python bench.py --workload batched_20x20x20x64                  # 24 RHS x 4 masses, FP16 vectors
    python bench.py --workload threelevel_48x48x48x96               # 12 RHS, 12-real 16-bit links
    python bench.py --workload serving [--requests N]               # Poisson request stream
    python bench.py --workload asqtad_20x20x20x64                   # fat/long links built from thin links
    python bench.py --workload npr_20x20x20x64                      # Eq. (1) four-fermion contraction, FP64
    python bench.py --kernels-only                                  # fixed launches for counter runs

Headline step: one complete solve of A x = b (A = 4m^2 - D_eo D_oe, even
sites) to a relative FP64 true residual of 1e-10 with the mixed-precision
reliable-update CG, on synthetic fields shaped like the paper's 20^3 x 64
lattice, inputs already resident in HBM.  Rank 0 prints one JSON line with
solves/s, the time-to-1e-10, CG GFLOPS (1146 flops per site per Dslash), the
speed-up over the plain FP64 GPU CG, the Dslash HBM roofline (HIP events on
the launch stream) and the CPU oracle baseline on a bounded sample.  The other
workloads print their own JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

PEAK_HBM_GBS = 8000.0
# FP32 vector peak of MI355X with packed FP32 (157.3 TFLOP/s) and without it: the
# library is built without packed-FP32 instructions, so 256 CU x 2.4 GHz x 128
# FP32 flop/clk = 78.6 TFLOP/s is the arithmetic ceiling of its kernels.
PEAK_FP32_PACKED_TFLOPS = 157.3
PEAK_FP32_TFLOPS = 78.6
# FP64 vector peak: 256 CU x 2.4 GHz x 128 FP64 flop/clk
PEAK_FP64_TFLOPS = 78.6
# SU(3) products per (site, direction) of the nested-staple link construction:
# 6 x (4 x (2 x 2 + 2) + 2 + 2) for the fat link, 2 for the long link; 198 flops each
LINK_BUILD_PRODUCTS = 170
METRIC = "asqtad Dslash HBM GB/s; CG time-to-1e-10 at 20^3x64; solves/s + p99 latency"

LINK_BYTES = {"f64": 144, "f32": 72, "f32r12": 48, "f16r12": 24}
VEC_BYTES = {"f64": 48, "f32": 24, "f16": 16}


def measured_traffic(kernel_key, launches_bytes_alg, lattice="20x20x20x64"):
    """HBM bytes per launch from the committed counter run, or None when the Dslash
    sources changed since the counters were taken (or none were taken)."""
    from paper_1411_2223_amd import profiling

    try:
        with open(profiling.counters_file(lattice)) as f:
            c = json.load(f)
    except (OSError, ValueError):
        return None
    if c.get("kernel_source_sha") != profiling.kernel_source_hash():
        return None
    k = c.get("kernels", {}).get(kernel_key)
    if not k:
        return None
    return 1024.0 * (c["fetch_factor"] * k["FETCH_SIZE_KiB"] + c["write_factor"] * k["WRITE_SIZE_KiB"])


def dslash_bytes_per_site(link, vec, nrhs):
    """Algorithmic bytes of one half-Dslash per output site: 16 links, nrhs input and output vectors."""
    return 16 * LINK_BYTES[link] + nrhs * 2 * VEC_BYTES[vec]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="single_20x20x20x64",
                    choices=["single_20x20x20x64", "batched_20x20x20x64", "threelevel_48x48x48x96", "serving",
                             "asqtad_20x20x20x64", "npr_20x20x20x64"])
    ap.add_argument("--mode", default="mixed32", choices=["f64", "mixed32", "mixed16"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-multishift", action="store_true", help="batched: skip the shifted-CG line")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="bound on the oracle sample")
    ap.add_argument("--dslash-launches", type=int, default=200)
    ap.add_argument("--requests", type=int, default=2000, help="serving: measured requests (after warm-up)")
    ap.add_argument("--serve-warmup", type=int, default=100, help="serving: warm-up requests")
    ap.add_argument("--serve-cols", type=int, default=32, help="serving: column slots per run")
    ap.add_argument("--serve-streams", type=int, default=4, help="serving: concurrent runs (streams)")
    ap.add_argument("--rate", type=float, default=50.0, help="serving: Poisson arrival rate (requests/s)")
    ap.add_argument("--no-oracle-check", action="store_true",
                    help="three-level and asqtad: skip the host FP64 oracle residuals")
    ap.add_argument("--u0", type=float, default=1.0, help="asqtad: tadpole factor of the link construction")
    ap.add_argument("--kernels-only", action="store_true",
                    help="only launch the Dslash tiers and a 1 GiB copy probe (for hardware-counter runs)")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def time_dslash(asq, g, prec, nrhs, launches, stream, native=True):
    """Average duration of one Dslash launch (HIP events on the launch stream) -> seconds.

    native: the tuned kernel the solvers launch, on vectors in their native layout
    (asqtad_dslash_eo_variant with ASQ_VARIANT_NATIVE); otherwise the public operator on
    canonical vectors (asqtad_dslash_eo)."""
    import torch

    v = synth.make_sources(g.dims, nrhs, 99)
    vin = asq.vec_to_device(v, prec, stream=stream)
    if native:
        vin = g.to_native(vin, prec, nrhs, stream=stream)
    variant = asq.ASQ_VARIANT_NATIVE if native else None
    out = torch.empty_like(vin)
    for _ in range(5):
        g.dslash(1, vin, prec, nrhs, out=out, stream=stream, variant=variant)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(launches):
        g.dslash(1, vin, prec, nrhs, out=out, stream=stream, variant=variant)
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) * 1e-3 / launches


def tiled_dslash_rate(asq, dims, fat, lng, prec, link, stream, reps=(2, 2, 2, 2), launches=20):
    """1-RHS Dslash on the field tiled periodically reps times along (x, y, z, t): a lattice
    whose links are far beyond the 256 MB memory-side cache, so each launch streams them
    from HBM.  Returns (lattice, us per launch, algorithmic GB/s)."""
    import torch

    X, Y, Z, T = dims
    big = (X * reps[0], Y * reps[1], Z * reps[2], T * reps[3])

    def tile(a):
        d = asq.links_to_device(a).view(T, Z, Y, X, 72)
        return d.repeat(reps[3], reps[2], reps[1], reps[0], 1).reshape(-1).contiguous()

    gb = asq.Gauge(big, tile(fat), tile(lng), precs=(link,), recon=18, stream=stream)
    dt = time_dslash(asq, gb, prec, 1, launches, stream)
    half = int(np.prod(big)) // 2
    gbs = dslash_bytes_per_site(link, prec, 1) * half / dt / 1e9
    gb.close()
    del gb
    torch.cuda.empty_cache()
    return "x".join(map(str, big)), dt * 1e6, gbs


def copy_bandwidth(asq, stream, nbytes=1 << 30, reps=10):
    """Read+write GB/s of the library's plain copy kernel on a buffer far beyond the 256 MB MALL."""
    import torch

    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    sp = asq.stream_ptr(stream)
    for _ in range(2):
        asq.check(asq.asq_copy_probe(dst.data_ptr(), src.data_ptr(), nbytes, sp), "asq_copy_probe")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        asq.check(asq.asq_copy_probe(dst.data_ptr(), src.data_ptr(), nbytes, sp), "asq_copy_probe")
    e1.record(stream)
    e1.synchronize()
    dt = e0.elapsed_time(e1) * 1e-3 / reps
    del src, dst
    return 2 * nbytes / dt / 1e9


def read_bandwidth(asq, stream, nbytes=4 << 30, reps=10):
    """Read-only GB/s of the library's read probe on a buffer far beyond the 256 MB MALL."""
    import torch

    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    sink = torch.empty(asq.asq_read_probe_blocks(nbytes) * 16, dtype=torch.uint8, device="cuda")
    sp = asq.stream_ptr(stream)
    for _ in range(2):
        asq.check(asq.asq_read_probe(src.data_ptr(), nbytes, sink.data_ptr(), sp), "asq_read_probe")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        asq.check(asq.asq_read_probe(src.data_ptr(), nbytes, sink.data_ptr(), sp), "asq_read_probe")
    e1.record(stream)
    e1.synchronize()
    dt = e0.elapsed_time(e1) * 1e-3 / reps
    del src, sink
    return nbytes / dt / 1e9


CPU_RUNS = 10


def _oracle_cg_runs(dims, fat, lng, mass, b, tol, seconds):
    """Per-iteration time of the oracle's FP64 CG: CPU_RUNS runs of the first n
    iterations of one solve, n sized so that all runs take about ``seconds``."""
    import oracle

    oracle.lib()
    t0 = time.perf_counter()
    oracle.apply_A(dims, fat, lng, mass, b)  # one operator application to size the sample
    per_apply = time.perf_counter() - t0
    n = max(3, int(seconds / CPU_RUNS / max(per_apply, 1e-6)))
    per_iter = []
    for _ in range(CPU_RUNS):
        t0 = time.perf_counter()
        _, it, _, _ = oracle.cg(dims, fat, lng, mass, b, tol=tol, maxiter=n)
        dt = time.perf_counter() - t0
        # each run ends with one extra operator application (its true residual)
        per_iter.append(max(dt - per_apply, 1e-9) / max(it, 1))
    p = np.asarray(per_iter)
    return it, p


def _spread(p, scale):
    """median, mean and standard error of the mean of CPU_RUNS timings, scaled."""
    q = p * scale
    return {"median": float(np.median(q)), "mean": float(q.mean()),
            "se": float(q.std(ddof=1) / np.sqrt(len(q))) if len(q) > 1 else 0.0, "runs": len(q)}


def cpu_baseline(w, fat, lng, b, mass, iters_full, seconds):
    """Oracle CG on the same workload, bounded: CPU_RUNS timed prefixes of the solve,
    the median per-iteration time scaled to the full solve's iteration count."""
    import oracle

    dims = w["dims"]
    it, p = _oracle_cg_runs(dims, fat, lng, mass, b, w["tol"], seconds)
    t_solve = _spread(p, iters_full)
    # the oracle's half-Dslash (D_oe on the source), FP64, counted like the GPU's FP64 tier
    half = int(np.prod(dims)) // 2
    td = []
    for _ in range(CPU_RUNS):
        t0 = time.perf_counter()
        oracle.dslash(dims, fat, lng, 1, b)
        td.append(time.perf_counter() - t0)
    td = np.asarray(td)
    return {"value": 1.0 / t_solve["median"], "unit": "solves/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"oracle FP64 CG ({oracle.build_flags()}), {CPU_RUNS} runs of the first {it} of {iters_full} "
                      f"iterations at {dims[0]}^3x{dims[3]} (median {np.median(p) * 1e3:.1f} ms/iteration), "
                      f"scaled to the full solve",
            "seconds_per_solve": t_solve,
            "dslash_ms": _spread(td, 1e3),
            "dslash_gbs_effective": dslash_bytes_per_site("f64", "f64", 1) * half / float(np.median(td)) / 1e9}


def cpu_baseline_extrapolated(dims, fat, lng, b0, mass, col_iters, seconds, unit):
    """Oracle FP64 CG per-iteration time (median of CPU_RUNS timed prefixes of one
    column's solve), scaled to the batch: the oracle solves the columns one after
    another, each for the number of iterations the GPU needed for it (labelled
    extrapolated)."""
    import oracle

    it, p = _oracle_cg_runs(dims, fat, lng, mass, b0, 1e-10, seconds)
    total = _spread(p, sum(col_iters))
    med = total["median"]
    value = len(col_iters) / med if unit == "RHS-solves/s" else med * 1e3
    return {"value": value, "unit": unit, "cores": oracle.num_threads(), "kind": "oracle",
            "extrapolated": True,
            "sample": f"oracle FP64 CG ({oracle.build_flags()}), {CPU_RUNS} runs of the first {it} iterations "
                      f"of one column at {'x'.join(map(str, dims))} (median {np.median(p) * 1e3:.1f} ms/iteration), "
                      f"scaled to {len(col_iters)} columns x their GPU iteration counts ({sum(col_iters)} iterations)",
            "seconds_per_batch": total}


def kernels_only(asq, g, dims):
    """Fixed launches for counter collection: each 1-column Dslash tier 20 times, the
    96-column FP16 Dslash 12 times, then the copy probe."""
    import torch

    half = int(np.prod(dims)) // 2
    stream = torch.cuda.Stream()
    res = {}
    for prec, link, ncol, n in (("f32", "f32", 1, 20), ("f64", "f64", 1, 20), ("f16", "f32", 1, 20),
                                ("f16", "f32", 96, 12)):
        dt = time_dslash(asq, g, prec, ncol, n, stream)
        res[f"{prec}_{ncol}"] = {"us": dt * 1e6, "alg_bytes": dslash_bytes_per_site(link, prec, ncol) * half}
    n = 1 << 30
    src = torch.empty(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        asq.check(asq.asq_copy_probe(dst.data_ptr(), src.data_ptr(), n, asq.stream_ptr(stream)), "copy")
    torch.cuda.synchronize()
    res["copy"] = {"bytes_read": n, "bytes_written": n}
    print(json.dumps({"kernels_only": res}), flush=True)


def kernels_only_threelevel(asq, g, g18, dims, ncol):
    """Fixed launches at 48^3 x 96 for counter collection: the iterated 12-column Dslash
    (FP16-with-norm vectors, 16-bit 12-real links) 10 times and the 12-column FP64 Dslash of
    the reliable update 5 times; then, on 18-real links far beyond the memory-side cache,
    the one-column FP32 and FP64 Dslash 20 times each; then the copy probe."""
    import torch

    half = int(np.prod(dims)) // 2
    stream = torch.cuda.Stream()
    res = {}
    for prec, link, n in (("f16", "f16r12", 10), ("f64", "f64", 5)):
        dt = time_dslash(asq, g, prec, ncol, n, stream)
        res[prec] = {"us": dt * 1e6, "alg_bytes": dslash_bytes_per_site(link, prec, ncol) * half}
    for prec, n in (("f32", 20), ("f64", 20)):
        dt = time_dslash(asq, g18, prec, 1, n, stream)
        res[f"{prec}_1rhs"] = {"us": dt * 1e6, "alg_bytes": dslash_bytes_per_site(prec, prec, 1) * half}
    nb = 1 << 30
    src = torch.empty(nb, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        asq.check(asq.asq_copy_probe(dst.data_ptr(), src.data_ptr(), nb, asq.stream_ptr(stream)), "copy")
    torch.cuda.synchronize()
    res["copy"] = {"bytes_read": nb, "bytes_written": nb}
    print(json.dumps({"kernels_only": res}), flush=True)


def solve_series(g, masses, bd, mode, tol, steps, warmup, stream, work=None, x=None):
    """warm-up + timed solves; returns (seconds per solve over the whole timed region,
    per-solve seconds, last SolveResult).
    A solve returns once its FP64 true residual has been decided, so host clock
    differences between consecutive solves are whole solves."""
    import torch

    for k in range(warmup):
        r = g.solve(masses, bd, mode=mode, tol=tol, maxiter=50000, work=work, x=x, stream=stream)
        s0 = r.stats[0]
        log(f"warmup {k}: rc={r.rc} iters={s0['iters']} ru={s0['reliable_updates']} "
            f"resid={max(s['true_resid'] for s in r.stats):.3e} {s0['seconds'] * 1e3:.1f} ms")
    torch.cuda.synchronize()
    last = None
    times = []
    t_start = time.perf_counter()
    for _ in range(steps):
        t0 = time.perf_counter()
        last = g.solve(masses, bd, mode=mode, tol=tol, maxiter=50000, work=work, x=x, stream=stream)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        if last.rc != 0:
            raise SystemExit(f"solve failed rc={last.rc}")
    torch.cuda.synchronize()
    return (time.perf_counter() - t_start) / steps, times, last


def time_stats(times):
    """mean, median and standard error of the mean, in ms."""
    t = np.asarray(times) * 1e3
    se = float(t.std(ddof=1) / np.sqrt(len(t))) if len(t) > 1 else None
    return {"mean_ms": float(t.mean()), "median_ms": float(np.median(t)), "se_ms": se, "n": len(t)}


# ---------------------------------------------------------------------------


def run_single(args, asq, torch):
    w = synth.WORKLOADS["single_20x20x20x64"]
    dims, mass = w["dims"], w["masses"][0]
    half = int(np.prod(dims)) // 2
    log(f"workload single_20x20x20x64 dims={dims} m={mass} mode={args.mode}")
    fat, lng = synth.make_gauge(dims, w["eps"], synth.gauge_seed(w["index"]))
    b = synth.make_sources(dims, 1, synth.source_seed(w["index"]))
    g = asq.Gauge(dims, fat, lng, precs=("f64", "f32"), recon=18)
    if args.kernels_only:
        kernels_only(asq, g, dims)
        return
    stream = torch.cuda.Stream()
    bd = asq.vec_to_device(b, "f64")
    work = g.workspace(1, args.mode)
    x = torch.empty_like(bd)
    torch.cuda.synchronize()
    secs, times, last = solve_series(g, [mass], bd, args.mode, w["tol"], args.steps, args.warmup, stream, work,
                                     x)
    tst = time_stats(times)
    st = last.stats[0]
    log(f"timed {args.steps} solves: {secs * 1e3:.2f} ms each (median {tst['median_ms']:.2f}); iters={st['iters']} "
        f"ru={st['reliable_updates']} resid={st['true_resid']:.3e}")
    # plain FP64 GPU CG at the same accuracy (speed-up reference), outside the timed region
    work64 = g.workspace(1, "f64")
    t64, times64, r64 = solve_series(g, [mass], bd, "f64", w["tol"], 3, 1, stream, work64, x)
    log(f"f64 CG: iters={r64.stats[0]['iters']} resid={r64.stats[0]['true_resid']:.3e} {t64 * 1e3:.1f} ms")
    # the other sloppy tier for comparison: FP16-with-norm vectors, same FP32 links and arithmetic
    other = "mixed16" if args.mode == "mixed32" else None
    t_other = r_other = None
    if other:
        work_o = g.workspace(1, other)
        t_other, times_o, r_other = solve_series(g, [mass], bd, other, w["tol"], 5, 1, stream, work_o, x)
        log(f"{other} CG: iters={r_other.stats[0]['iters']} resid={r_other.stats[0]['true_resid']:.3e} "
            f"{t_other * 1e3:.1f} ms")

    # FP32 arithmetic on FP64-stored 18-real links (a field kept in FP64 only: the
    # sloppy Dslash rounds its links to FP32 on load), same solver and tolerance
    g64 = asq.Gauge(dims, fat, lng, precs=("f64",), recon=18)
    t_l64, times_l64, r_l64 = solve_series(g64, [mass], bd, "mixed32", w["tol"], 5, 1, stream, work, x)
    dt_l64 = time_dslash(asq, g64, "f32", 1, max(20, args.dslash_launches // 4), stream)
    l64_bytes = (16 * 144 + 2 * 24) * half
    log(f"mixed32 CG on FP64-stored links: iters={r_l64.stats[0]['iters']} "
        f"resid={r_l64.stats[0]['true_resid']:.3e} {t_l64 * 1e3:.1f} ms; its FP32 Dslash {dt_l64 * 1e6:.1f} us")
    g64.close()
    del g64

    # the optional link compression: the FP32 copy stored as 12 reals per link (two rows,
    # the third rebuilt in the kernel), same solver and tolerance; the bench line keeps
    # the 18-real links of its configuration
    g12 = asq.Gauge(dims, fat, lng, precs=("f64", "f32"), recon=12)
    t_r12, times_r12, r_r12 = solve_series(g12, [mass], bd, "mixed32", w["tol"], 5, 1, stream, work, x)
    dt_r12 = time_dslash(asq, g12, "f32", 1, max(20, args.dslash_launches // 4), stream)
    r12_bytes = dslash_bytes_per_site("f32r12", "f32", 1) * half
    log(f"mixed32 CG on FP32 12-real links: iters={r_r12.stats[0]['iters']} "
        f"resid={r_r12.stats[0]['true_resid']:.3e} {t_r12 * 1e3:.1f} ms; its FP32 Dslash {dt_r12 * 1e6:.1f} us")
    g12.close()
    del g12

    # the boundary's host-side costs, outside the timed region: importing the host FP64
    # links (once per gauge field), and a solve whose b starts and whose x ends in pinned
    # host memory (PCIe both ways)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g2 = asq.Gauge(dims, fat, lng, precs=("f64", "f32"), recon=18)
    torch.cuda.synchronize()
    import_ms = (time.perf_counter() - t0) * 1e3
    g2.close()
    del g2
    hb = torch.empty(bd.shape, dtype=bd.dtype, pin_memory=True)
    hb.copy_(bd.cpu())
    hx = torch.empty(bd.shape, dtype=bd.dtype, pin_memory=True)
    bd2 = torch.empty_like(bd)
    host_ms = []
    for k in range(4):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        with torch.cuda.stream(stream):
            bd2.copy_(hb, non_blocking=True)
        g.solve([mass], bd2, mode=args.mode, tol=w["tol"], maxiter=50000, work=work, x=x, stream=stream)
        with torch.cuda.stream(stream):
            hx.copy_(x, non_blocking=True)
        stream.synchronize()
        if k:
            host_ms.append((time.perf_counter() - t0) * 1e3)
    assert torch.equal(hx, x.cpu())
    log(f"gauge import from host: {import_ms:.1f} ms; solve with b and x in pinned host memory: "
        f"{np.median(host_ms):.2f} ms")

    # dominant kernel: the sloppy single-RHS Dslash
    tprec = {"mixed32": "f32", "f64": "f64", "mixed16": "f16"}[args.mode]
    link = "f64" if tprec == "f64" else "f32"
    dt = time_dslash(asq, g, tprec, 1, args.dslash_launches, stream)
    bytes_launch = dslash_bytes_per_site(link, tprec, 1) * half
    achieved = bytes_launch / dt / 1e9
    dt64 = time_dslash(asq, g, "f64", 1, max(20, args.dslash_launches // 4), stream)
    f64_gbs = dslash_bytes_per_site("f64", "f64", 1) * half / dt64 / 1e9
    dt_pub = time_dslash(asq, g, tprec, 1, args.dslash_launches, stream, native=False)
    log(f"dslash {tprec}: {dt * 1e6:.2f} us, {achieved:.0f} GB/s; f64: {dt64 * 1e6:.2f} us, {f64_gbs:.0f} GB/s; "
        f"public canonical-layout {tprec}: {dt_pub * 1e6:.2f} us")
    copy_gbs = copy_bandwidth(asq, stream)
    read_gbs = read_bandwidth(asq, stream)
    log(f"copy probe: {copy_gbs:.0f} GB/s; read probe: {read_gbs:.0f} GB/s")
    big, us_big, gbs_big = tiled_dslash_rate(asq, dims, fat, lng, tprec, link, stream)
    log(f"dslash {tprec} on {big} (links beyond the MALL): {us_big:.1f} us, {gbs_big:.0f} GB/s "
        f"({gbs_big / PEAK_HBM_GBS:.1%} of HBM peak)")

    ms = secs * 1e3
    iters = st["iters"]
    flops = half * ((2 * 1146 + 72) * iters + (2 * 1146 + 36) * st["reliable_updates"])
    out = {
        "metric": METRIC,
        "value": 1.0 / secs,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"mixed32": "f32", "f64": "f64", "mixed16": "f16"}[args.mode],
        "data": "synthetic",
        "config": {"workload": f"single_20x20x20x64: 20x20x20x64 even-odd asqtad CG, 1 RHS, m={mass}, "
                               f"eps={w['eps']} SU(3) links, tol 1e-10 FP64 true residual, {args.mode} "
                               f"reliable-update CG, FP32 and FP64 18-real links",
                   "global_batch": 1, "parallelism": "single GPU"},
        "time_to_solution_ms": ms,
        "time_to_solution": tst,
        "f64_time_to_solution": time_stats(times64),
        "iterations": iters,
        "reliable_updates": st["reliable_updates"],
        "true_resid": st["true_resid"],
        "cg_gflops": flops / secs / 1e9,
        "f64_cg_ms": t64 * 1e3,
        "f64_cg_iterations": r64.stats[0]["iters"],
        "speedup_vs_f64_cg": t64 / secs,
        "fp16_vectors_time_to_solution_ms": t_other * 1e3 if t_other else None,
        "fp64_links_fp32_arith": {"time_to_solution": time_stats(times_l64), "ms": t_l64 * 1e3,
                                  "iterations": r_l64.stats[0]["iters"],
                                  "true_resid": r_l64.stats[0]["true_resid"],
                                  "speedup_vs_f64_cg": t64 / t_l64,
                                  "dslash_us": dt_l64 * 1e6, "dslash_bytes_per_launch": l64_bytes,
                                  "dslash_gbs": l64_bytes / dt_l64 / 1e9},
        "fp32_12real_links": {"time_to_solution": time_stats(times_r12), "ms": t_r12 * 1e3,
                              "iterations": r_r12.stats[0]["iters"], "true_resid": r_r12.stats[0]["true_resid"],
                              "speedup_vs_f64_cg": t64 / t_r12, "dslash_us": dt_r12 * 1e6,
                              "dslash_bytes_per_launch": r12_bytes, "dslash_gbs": r12_bytes / dt_r12 / 1e9},
        "gauge_import_ms": import_ms,
        "pcie_inclusive_solve_ms": float(np.median(host_ms)),
        "fp16_vectors_iterations": r_other.stats[0]["iters"] if r_other else None,
        "dslash_gbs": achieved,
        "dslash_f64_gbs": f64_gbs,
        "dslash_public_canonical_us": dt_pub * 1e6,
        "copy_probe_gbs": copy_gbs,
        "read_probe_gbs": read_gbs,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS,
                     "traffic": measured_traffic(f"{tprec}_{link}_1rhs", bytes_launch),
                     "kernel": f"dslash_kernel {tprec} vectors, {link} 18-real links, 1 RHS",
                     "us_per_launch": dt * 1e6, "bytes_per_launch": bytes_launch,
                     "basis": "effective (MALL-assisted): the 295 MB of 20^3x64 FP32 links are close to the "
                              "256 MB memory-side cache, which serves part of each launch's link reads",
                     "above_mall": {"lattice": big, "how": "the same field tiled 2x2x2x2", "us_per_launch": us_big,
                                    "achieved": gbs_big, "frac": gbs_big / PEAK_HBM_GBS,
                                    "read_probe_frac": read_gbs / PEAK_HBM_GBS}},
        "paper_context": {"cg_gflops_titan_black_mixed_own_code": 46.48, "cg_gflops_titan_black_quda": 97.86,
                          "note": "other hardware, real MILC ensemble, flop convention unstated"},
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(w, fat, lng, b[0], mass, r64.stats[0]["iters"], args.cpu_seconds)
    print(json.dumps(out), flush=True)


def run_batched(args, asq, torch):
    """24 Gaussian RHS x 4 masses = 96 columns in one batch, FP16-with-norm vectors, FP32 18-real links."""
    w = synth.WORKLOADS["batched_20x20x20x64"]
    dims = w["dims"]
    half = int(np.prod(dims)) // 2
    nsrc, masses_u = w["nrhs"], list(w["masses"])
    masses = [m for m in masses_u for _ in range(nsrc)]
    ncol = len(masses)
    log(f"workload batched dims={dims} columns={ncol}")
    fat, lng = synth.make_gauge(dims, w["eps"], synth.gauge_seed(w["index"]))
    src = synth.make_sources(dims, nsrc, synth.source_seed(w["index"]))
    b = np.concatenate([src] * len(masses_u), axis=0)
    g = asq.Gauge(dims, fat, lng, precs=("f64", "f32"), recon=18)
    stream = torch.cuda.Stream()
    bd = asq.vec_to_device(b, "f64")
    mode = "mixed16" if args.mode == "mixed32" else args.mode
    work = g.workspace(ncol, mode)
    x = torch.empty_like(bd)
    steps = max(1, min(args.steps, 3))
    secs, _, last = solve_series(g, masses, bd, mode, w["tol"], steps, 1, stream, work, x)
    its = [s["iters"] for s in last.stats]
    res = [s["true_resid"] for s in last.stats]
    log(f"batched {ncol} columns: {secs:.3f} s; iters min/max {min(its)}/{max(its)}; resid max {max(res):.3e}")
    tprec = "f16" if mode == "mixed16" else ("f32" if mode == "mixed32" else "f64")
    link = "f64" if tprec == "f64" else "f32"
    dt = time_dslash(asq, g, tprec, ncol, 20, stream)
    bytes_launch = dslash_bytes_per_site(link, tprec, ncol) * half
    flops_launch = 1146.0 * half * ncol
    gbs = bytes_launch / dt / 1e9
    tf = flops_launch / dt / 1e12
    log(f"dslash {tprec} x{ncol}: {dt * 1e6:.1f} us, {gbs:.0f} GB/s, {tf:.1f} TFLOP/s")
    flops = half * sum((2 * 1146 + 72) * s["iters"] + (2 * 1146 + 36) * s["reliable_updates"] for s in last.stats)
    out = {"metric": METRIC, "workload": "batched_20x20x20x64", "value": ncol / secs, "unit": "RHS-solves/s",
           "columns": ncol, "masses": masses_u, "seconds_per_batch": secs, "mode": mode,
           "iters_min": min(its), "iters_max": max(its), "true_resid_max": max(res),
           "cg_gflops": flops / secs / 1e9,
           "dslash": {"us": dt * 1e6, "GBps": gbs, "TFLOPs": tf, "bytes_per_site": bytes_launch / half,
                      "flop_per_byte": flops_launch / bytes_launch,
                      "frac_hbm": gbs / PEAK_HBM_GBS, "frac_fp32_alu": tf / PEAK_FP32_TFLOPS,
                      "frac_fp32_packed_peak": tf / PEAK_FP32_PACKED_TFLOPS,
                      "traffic": measured_traffic(f"{tprec}_{link}_{ncol}rhs", bytes_launch)}}
    if not args.no_multishift:
        # the same 96 (mass, source) systems by shifted CG (one Krylov space per source)
        # plus per-column refinement; same tolerance, FP64 true residual per column
        srcd = asq.vec_to_device(src, "f64")
        wms = asq.empty_bytes(asq.asq_multishift_workspace_bytes(g.handle, nsrc, len(masses_u), asq.MODES[mode]))
        xm = torch.empty(len(masses_u) * srcd.numel(), dtype=torch.float64, device="cuda")
        g.solve_multishift(masses_u, srcd, mode=mode, tol=w["tol"], work=wms, x=xm, stream=stream)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rm = g.solve_multishift(masses_u, srcd, mode=mode, tol=w["tol"], work=wms, x=xm, stream=stream)
        torch.cuda.synchronize()
        tms = time.perf_counter() - t0
        if rm.rc != 0:
            raise SystemExit(f"multishift solve failed rc={rm.rc}")
        res_ms = [s["true_resid"] for s in rm.stats]
        log(f"multishift 24 sources x 4 masses: {tms:.3f} s; max resid {max(res_ms):.3e}")
        out["multishift"] = {"value": ncol / tms, "unit": "RHS-solves/s", "seconds_per_batch": tms,
                             "true_resid_max": max(res_ms), "iters_max": max(s["iters"] for s in rm.stats),
                             "speedup_vs_independent": secs / tms}
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle, extrapolated) ...")
        out["cpu_baseline"] = cpu_baseline_extrapolated(dims, fat, lng, src[0], masses_u[0], its,
                                                        args.cpu_seconds, "RHS-solves/s")
    print(json.dumps(out), flush=True)


def run_threelevel(args, asq, torch):
    """48^3 x 96, 12 RHS, m = 0.005: FP16-with-norm vectors and 16-bit 12-real links in the iteration,
    FP32 arithmetic and residual, FP64 solution and true residual."""
    w = synth.WORKLOADS["threelevel_48x48x48x96"]
    dims, mass, ncol = w["dims"], w["masses"][0], w["nrhs"]
    half = int(np.prod(dims)) // 2
    log(f"workload threelevel dims={dims} columns={ncol} (gauge generation takes a while)")
    t0 = time.perf_counter()
    fat, lng = synth.make_gauge(dims, w["eps"], synth.gauge_seed(w["index"]))
    log(f"gauge generated in {time.perf_counter() - t0:.0f} s")
    g = asq.Gauge(dims, fat, lng, precs=("f64", "f32", "f16"), recon=12)
    # one-column FP32 and FP64 Dslash on 18-real links: 6.1 and 12.2 GB, far beyond the
    # 256 MB memory-side cache, so their rate is HBM bandwidth
    g18 = asq.Gauge(dims, fat, lng, precs=("f64", "f32"), recon=18)
    del fat, lng
    if args.kernels_only:
        kernels_only_threelevel(asq, g, g18, dims, ncol)
        return
    stream0 = torch.cuda.Stream()
    above = {}
    for prec in ("f32", "f64"):
        dtp = time_dslash(asq, g18, prec, 1, 20, stream0)
        bl = dslash_bytes_per_site(prec, prec, 1) * half
        above[prec] = {"us": dtp * 1e6, "GBps": bl / dtp / 1e9, "frac_hbm": bl / dtp / 1e9 / PEAK_HBM_GBS,
                       "bytes_per_launch": bl,
                       "traffic": measured_traffic(f"{prec}_{prec}_1rhs_r18", bl, lattice="48x48x48x96")}
        log(f"above-MALL 1-RHS {prec} 18-real: {dtp * 1e6:.1f} us, {bl / dtp / 1e9:.0f} GB/s")
    g18.close()
    del g18
    b = synth.make_sources(dims, ncol, synth.source_seed(w["index"]))
    stream = torch.cuda.Stream()
    bd = asq.vec_to_device(b, "f64")
    del b
    work = g.workspace(ncol, "mixed16")
    x = torch.empty_like(bd)
    secs, _, last = solve_series(g, [mass] * ncol, bd, "mixed16", w["tol"], 1, 1, stream, work, x)
    its = [s["iters"] for s in last.stats]
    res = [s["true_resid"] for s in last.stats]
    log(f"three-level {ncol} columns: {secs:.3f} s; iters {max(its)}; resid max {max(res):.3e}")
    dt = time_dslash(asq, g, "f16", ncol, 10, stream)
    bytes_launch = dslash_bytes_per_site("f16r12", "f16", ncol) * half
    gbs = bytes_launch / dt / 1e9
    tf = 1146.0 * half * ncol / dt / 1e12
    dt1 = time_dslash(asq, g, "f16", 1, 10, stream)
    gbs1 = dslash_bytes_per_site("f16r12", "f16", 1) * half / dt1 / 1e9
    log(f"dslash f16 r12 x{ncol}: {dt * 1e6:.0f} us, {gbs:.0f} GB/s, {tf:.1f} TFLOP/s; 1 RHS {gbs1:.0f} GB/s")
    oracle_resid = None
    cpu = None
    if not args.no_oracle_check or not args.no_cpu_baseline:
        import oracle

        fat, lng = synth.make_gauge(dims, w["eps"], synth.gauge_seed(w["index"]))
        b = synth.make_sources(dims, ncol, synth.source_seed(w["index"]))
        if not args.no_oracle_check:
            xs = asq.vec_from_device(x, ncol, half, "f64")
            oracle_resid = [oracle.true_residual(dims, fat, lng, mass, b[c], xs[c]) for c in range(ncol)]
            log(f"oracle FP64 true residual of every column: max {max(oracle_resid):.3e}")
        if not args.no_cpu_baseline:
            log("cpu baseline (oracle, extrapolated) ...")
            cpu = cpu_baseline_extrapolated(dims, fat, lng, b[0], mass, its, args.cpu_seconds, "ms to 1e-10")
    traffic = measured_traffic("f16_f16r12_12rhs", bytes_launch, lattice="48x48x48x96")
    if traffic:
        log(f"counter-measured traffic {traffic / 1e9:.2f} GB per launch: {traffic / dt / 1e9:.0f} GB/s")
    out = {"metric": METRIC, "workload": "threelevel_48x48x48x96", "value": secs * 1e3, "unit": "ms to 1e-10",
           "columns": ncol, "mass": mass, "iters_max": max(its), "true_resid_max": max(res),
           "oracle_true_resid_max": max(oracle_resid) if oracle_resid else None,
           "reliable_updates": max(s["reliable_updates"] for s in last.stats),
           "dslash_12rhs": {"us": dt * 1e6, "GBps": gbs, "TFLOPs": tf, "frac_hbm": gbs / PEAK_HBM_GBS,
                            "frac_fp32_alu": tf / PEAK_FP32_TFLOPS, "bytes_per_launch": bytes_launch,
                            "traffic": traffic,
                            "traffic_GBps": traffic / dt / 1e9 if traffic else None},
           "dslash_1rhs_GBps": gbs1,
           "dslash_1rhs_18real_above_mall": above}
    if cpu:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


def serving_summary(done, trace, n_warm, lattices):
    """Load and latency figures of a served request stream.  done: one tuple per finished
    request (trace index, rc, latency s, columns, lattice index, max true residual, completion
    time s on the trace's clock); the first n_warm requests of the trace are warm-up and stay
    out of every figure.  The served rate is taken over the measured window, from the first
    measured arrival to the last measured completion; stable: served >= 0.95 offered."""
    meas = [d for d in done if d[0] >= n_warm]
    lats = np.array([d[2] for d in meas])
    rhs = sum(d[3] for d in meas)
    span = trace[-1]["arrival"] - trace[n_warm]["arrival"]
    window = max(d[6] for d in meas) - trace[n_warm]["arrival"]
    per_lat = {}
    for i in range(len(lattices)):
        li = [d[2] for d in meas if d[4] == i]
        if li:
            per_lat["x".join(map(str, lattices[i]))] = {"n": len(li), "p50_ms": float(np.percentile(li, 50) * 1e3),
                                                        "p99_ms": float(np.percentile(li, 99) * 1e3)}
    return {"value": len(meas) / window, "stable": len(meas) / window >= 0.95 * len(meas) / span,
            "requests": len(meas), "rhs_solves": rhs, "window_s": window,
            "offered_requests_per_s": len(meas) / span, "achieved_rhs_per_s": rhs / window,
            "p50_latency_ms": float(np.percentile(lats, 50) * 1e3), "p99_latency_ms": float(np.percentile(lats, 99) * 1e3),
            "failed": sum(1 for d in meas if d[1] != 0), "true_resid_max": max(d[5] for d in meas),
            "per_lattice": per_lat}


def split_parities(x, half):
    """A full-lattice canonical FP64 vector (flat: the even half's half x 6 reals, then the odd
    half's) -> (even, odd) flat views."""
    n = int(half) * 6
    if x.numel() != 2 * n:
        raise ValueError(f"a full-lattice vector of {2 * n} reals was expected, got {x.numel()}")
    return x[:n], x[n:]


def run_serving(args, asq, torch):
    """Poisson stream of solves on four resident lattices (continuous batching, HBM budget)."""
    lattices = synth.SERVING_LATTICES
    n_warm = args.serve_warmup
    trace = synth.serving_trace(args.requests + n_warm, rate=args.rate)
    mode = "mixed16" if args.mode == "mixed32" else args.mode
    # Each request's sources come from its trace seed: it draws its columns (without
    # replacement) from a bank of seeded Gaussian sources resident per lattice.
    bank_cols = 48
    gauges, banks, arrays = [], [], []
    for k, dims in enumerate(lattices):
        fat, lng = synth.make_gauge(dims, 0.3, synth.BASE_SEED + 10 + k)
        gauges.append(asq.Gauge(dims, fat, lng, precs=("f64", "f32"), recon=18))
        half = gauges[-1].half
        bank = synth.make_sources(dims, bank_cols, synth.BASE_SEED + 20 + k)
        banks.append(asq.vec_to_device(bank, "f64").view(bank_cols, half * 6))
        arrays.append((fat, lng, bank))
        del fat, lng, bank
    budget = 48 << 30
    srv = asq.Server(budget, max_streams=args.serve_streams, max_cols=args.serve_cols)
    gids = [srv.register(gg) for gg in gauges]  # tunes every batch shape before the stream starts
    torch.cuda.synchronize()
    log(f"serving {len(trace)} requests ({n_warm} warm-up), budget {budget >> 30} GiB")
    # a sample of served solutions is checked by the oracle afterwards: two per lattice
    check_ids = set()
    for li in range(len(lattices)):
        ids = [i for i, q in enumerate(trace) if q["lattice"] == li and i >= n_warm]
        check_ids.update(ids[:: max(1, len(ids) // 2)][:2])
    kept = {}
    pending = {}
    done = []
    t0 = time.perf_counter()
    k = 0
    while k < len(trace) or pending:
        now = time.perf_counter() - t0
        while k < len(trace) and trace[k]["arrival"] <= now:
            q = trace[k]
            lat = q["lattice"]
            n = q["nrhs"]
            cols = np.random.Generator(np.random.PCG64(q["seed"])).choice(bank_cols, size=n, replace=False)
            b = banks[lat][torch.as_tensor(cols, device=banks[lat].device)].reshape(-1)
            x = torch.empty_like(b)
            t = srv.submit(gids[lat], [q["mass"]] * n, b, x, mode=mode)
            pending[t] = (k, n, b, x)
            k += 1
        for t in list(pending):
            kk, n, b, x = pending[t]
            r = srv.poll(t, n)
            if r is not None:
                rc, stats, latency = r
                done.append((kk, rc, latency, n, trace[kk]["lattice"], max(s["true_resid"] for s in stats),
                             time.perf_counter() - t0))
                if kk in check_ids:
                    kept[kk] = x
                del pending[t]
        time.sleep(0.0005)
    wall = time.perf_counter() - t0
    srv.close()
    oracle_max = None
    if not args.no_oracle_check:
        import oracle

        rs = []
        for kk, x in sorted(kept.items()):
            q = trace[kk]
            dims = lattices[q["lattice"]]
            fat, lng, bank = arrays[q["lattice"]]
            n = q["nrhs"]
            half = int(np.prod(dims)) // 2
            cols = np.random.Generator(np.random.PCG64(q["seed"])).choice(bank_cols, size=n, replace=False)
            src = bank[cols]
            xs = asq.vec_from_device(x, n, half, "f64")
            rs += [oracle.true_residual(dims, fat, lng, q["mass"], src[c], xs[c]) for c in range(n)]
        oracle_max = max(rs) if rs else None
        log(f"oracle FP64 residual of {len(kept)} sampled requests ({len(rs)} columns): max {oracle_max:.3e}")
    del arrays
    out = {"metric": METRIC, "workload": "serving", "unit": "requests/s", "rate": args.rate, "mode": mode,
           "max_cols": args.serve_cols, "max_streams": args.serve_streams}
    out.update(serving_summary(done, trace, n_warm, lattices))
    out.update({"wall_s": wall, "oracle_checked_requests": len(kept), "oracle_true_resid_max": oracle_max})
    log(f"serving: {out['value']:.1f} req/s, p50 {out['p50_latency_ms']:.1f} ms, p99 {out['p99_latency_ms']:.1f} ms")
    print(json.dumps(out), flush=True)


def run_asqtad(args, asq, torch):
    """Asqtad fat and long links built on the device from 20^3 x 64 thin links (the single-solve
    workload's field), then the mixed-precision solve on them."""
    w = synth.WORKLOADS["single_20x20x20x64"]
    dims, mass, u0 = w["dims"], w["masses"][0], args.u0
    V = int(np.prod(dims))
    log(f"workload asqtad dims={dims} u0={u0} m={mass}")
    U = synth.thin_links(dims, w["eps"], synth.gauge_seed(w["index"])).reshape(V, 4, 3, 3)
    stream = torch.cuda.Stream()
    thin = asq.links_to_device(U)
    fat = torch.empty_like(thin)
    lng = torch.empty_like(thin)
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        for _ in range(max(1, args.warmup)):
            asq.build_links(dims, thin, u0, fat, lng, stream=stream)
        reps = max(3, args.steps)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            asq.build_links(dims, thin, u0, fat, lng, stream=stream)
        e1.record(stream)
    stream.synchronize()
    dt = e0.elapsed_time(e1) / 1e3 / reps
    t0 = time.perf_counter()
    plaq = asq.plaquette(dims, thin, stream=stream)
    t_plaq = time.perf_counter() - t0
    log(f"mean plaquette {plaq:.12f} (u0 = P^1/4 = {plaq ** 0.25:.6f}), {t_plaq * 1e3:.2f} ms with the host copy")
    flops = 198.0 * LINK_BUILD_PRODUCTS * 4 * V  # per call
    tf = flops / dt / 1e12
    log(f"link construction: {dt * 1e3:.3f} ms, {tf:.1f} TFLOP/s FP64 ({tf / PEAK_FP64_TFLOPS:.0%} of peak)")
    g = asq.Gauge(dims, fat, lng, precs=("f64", "f32"), recon=18, stream=stream)
    del fat, lng
    b = synth.make_sources(dims, 1, synth.source_seed(w["index"]))
    bd = asq.vec_to_device(b, "f64")
    secs, times, last = solve_series(g, [mass], bd, "mixed32", w["tol"], max(1, args.steps // 2), 1, stream)
    st = last.stats[0]
    log(f"mixed32 solve on the built links: {secs * 1e3:.1f} ms, iters={st['iters']} "
        f"resid={st['true_resid']:.3e}")
    # the full-lattice system M x = b (M = 2m + D) on the built links: even-odd
    # reduction, the even solve and the odd-site reconstruction
    bfull = synth.make_sources(dims, 2, synth.source_seed(w["index"]) + 7)  # [even half, odd half]
    bfd = torch.cat([asq.vec_to_device(bfull[0:1], "f64"), asq.vec_to_device(bfull[1:2], "f64")])
    xf = torch.empty_like(bfd)
    work_full = asq.empty_bytes(asq.asq_full_workspace_bytes(g.handle, 1, asq.MODES["mixed32"]))
    full_times = []
    rf = None
    for k in range(1 + max(1, args.steps // 3)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rf = g.solve_full([mass], bfd, mode="mixed32", work=work_full, x=xf, stream=stream)
        torch.cuda.synchronize()
        if rf.rc != 0:
            raise SystemExit(f"full solve failed rc={rf.rc}")
        if k > 0:
            full_times.append(time.perf_counter() - t0)
    sf = rf.stats[0]
    log(f"full M x = b on the built links: {np.median(full_times) * 1e3:.1f} ms, iters={sf['iters']} "
        f"|b - M x|/|b|={sf['true_resid']:.3e}")
    full_oracle = None
    if not args.no_oracle_check:
        import oracle

        log("oracle: links of every site and the full residual ...")
        ofat, olng = oracle.asqtad_links(dims, U, u0)
        half = V // 2
        xfe, xfo = split_parities(xf, half)
        xe = asq.vec_from_device(xfe, 1, half, "f64")[0]
        xo = asq.vec_from_device(xfo, 1, half, "f64")[0]
        re = bfull[0] - 2 * mass * xe - oracle.dslash(dims, ofat, olng, 0, xo)
        ro = bfull[1] - 2 * mass * xo - oracle.dslash(dims, ofat, olng, 1, xe)
        full_oracle = float(np.sqrt((np.vdot(re, re) + np.vdot(ro, ro)).real /
                                    (np.vdot(bfull[0], bfull[0]) + np.vdot(bfull[1], bfull[1])).real))
        log(f"oracle |b - M x|/|b| with its own links: {full_oracle:.3e}")
    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        oracle.lib()
        rng = np.random.Generator(np.random.PCG64(3))
        n = 4096
        t0 = time.perf_counter()
        oracle.asqtad_links(dims, U, u0, sites=rng.integers(0, V, size=n))
        per_site = (time.perf_counter() - t0) / n
        n = int(min(V // CPU_RUNS, max(1024, args.cpu_seconds / CPU_RUNS / max(per_site, 1e-9))))
        per = []
        for _ in range(CPU_RUNS):
            sites = rng.integers(0, V, size=n)
            t0 = time.perf_counter()
            oracle.asqtad_links(dims, U, u0, sites=sites)
            per.append((time.perf_counter() - t0) / n)
        full = _spread(np.asarray(per), V * 1e3)
        cpu = {"value": full["median"], "unit": "ms per link construction", "cores": oracle.num_threads(),
               "kind": "oracle", "ms_per_construction": full,
               "sample": f"oracle path sums ({oracle.build_flags()}), {CPU_RUNS} runs at {n} random sites "
                         f"of {V} each, median scaled to every site"}
        log(f"cpu baseline: {full['median'] / 1e3:.1f} s per construction on {cpu['cores']} threads")
    out = {"metric": METRIC, "workload": "asqtad_20x20x20x64", "value": dt * 1e3,
           "unit": "ms per link construction", "higher_is_better": False, "dtype": "f64", "data": "synthetic",
           "u0": u0, "plaquette": plaq, "u0_from_plaquette": plaq ** 0.25, "plaquette_ms": t_plaq * 1e3,
           "config": {"workload": "asqtad_20x20x20x64", "dims": list(dims), "eps": w["eps"]},
           "roofline": {"bound": "alu", "achieved": tf, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                        "frac": tf / PEAK_FP64_TFLOPS, "traffic": None,
                        "kernel": "asqtad_build_links: transpose, fat-link and long-link kernels (FP64), "
                                  "timed together",
                        "flops_per_call": flops, "ms_per_call": dt * 1e3},
           "solve_mixed32": {"ms": secs * 1e3, "time_to_solution": time_stats(times), "iters": st["iters"],
                             "reliable_updates": st["reliable_updates"], "true_resid": st["true_resid"],
                             "mass": mass},
           "full_solve_mixed32": {"ms": float(np.median(full_times) * 1e3), "time_to_solution": time_stats(full_times),
                                  "iters": sf["iters"], "true_resid": sf["true_resid"],
                                  "oracle_true_resid": full_oracle, "mass": mass}}
    if cpu:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


# SU(3) products per hypercube of the four-fermion operator that do not depend on the
# operator: the 256 link averages by their first step (sum over pairs of |A ^ D| = 512,
# less the 64 pairs at distance 1, whose average is the link itself) and the two
# bilinear colour matrices of each pair (4 x 256); and the contraction per operator:
# 16 x 16 corner pairs x 81 complex multiply-adds (8 flops each).
NPR_PRODUCTS_PER_HYPERCUBE = 448 + 4 * 256
NPR_FLOPS_PER_OP_HYPERCUBE = 256 * 81 * 8


def npr_flops(nz, nop):
    return nz * (198.0 * NPR_PRODUCTS_PER_HYPERCUBE + NPR_FLOPS_PER_OP_HYPERCUBE * nop)


def run_npr(args, asq, torch):
    """The one-colour four-fermion operator of Eq. (1) on the paper's 20^3 x 64 lattice shape:
    point-source propagators of two masses from the library's own full-lattice CG (FP64
    true residual 1e-10), then the FP64 contraction for 16 operators (every spin S with
    taste xi_5 in both bilinears) at every hypercube."""
    w = synth.WORKLOADS["single_20x20x20x64"]
    dims = w["dims"]
    V = int(np.prod(dims))
    half = V // 2
    nz = V // 16
    masses = (0.01, 0.05)
    ops = [(s, 15, s, 15) for s in range(16)]
    log(f"workload npr dims={dims} masses={masses} operators={len(ops)}")
    U = synth.thin_links(dims, w["eps"], synth.gauge_seed(w["index"]))
    fat, lng = synth.fat_long_from_thin(U)
    U = U.reshape(V, 4, 3, 3)
    g = asq.Gauge(dims, fat, lng, precs=("f64", "f32"), recon=18)
    stream = torch.cuda.Stream()
    # point sources at the origin (an even site, checkerboard index 0), one per colour and mass:
    # b = [even halves of the 6 columns, odd halves]
    ncol = 3 * len(masses)
    b = np.zeros((2, ncol, half, 3), dtype=np.complex128)
    for f in range(len(masses)):
        for a in range(3):
            b[0, 3 * f + a, 0, a] = 1.0
    bd = asq.vec_to_device(b.reshape(2 * ncol, half, 3), "f64")
    t0 = time.perf_counter()
    res = g.solve_full([m for m in masses for _ in range(3)], bd, mode="mixed32", stream=stream)
    torch.cuda.synchronize()
    t_prop = time.perf_counter() - t0
    if res.rc != 0:
        raise SystemExit(f"propagator solves failed rc={res.rc}")
    log(f"propagators: {ncol} full-lattice solves in {t_prop:.2f} s, max |b - M x|/|b| "
        f"{max(s['true_resid'] for s in res.stats):.2e}")
    # G_f(x)[c][a] in lexicographic site order (input construction, on the host)
    xs = asq.vec_from_device(res.x, 2 * ncol, half, "f64").reshape(2, ncol, half, 3)
    X, Y, Z, T = dims
    lex = np.arange(V)
    par = (lex % X + (lex // X) % Y + (lex // (X * Y)) % Z + lex // (X * Y * Z)) % 2
    G = []
    for f in range(len(masses)):
        Gf = np.empty((V, 3, 3), dtype=np.complex128)
        for p in (0, 1):
            sel = par == p
            Gf[sel] = xs[p, 3 * f:3 * f + 3][:, lex[sel] // 2].transpose(1, 2, 0)  # [site][c][a]
        G.append(Gf)
    props_h = [G[0], G[0], G[1], G[1]]  # chi, chibar of the light quark; of the heavier one
    thin = asq.links_to_device(U)
    props = [asq.links_to_device(x.reshape(V, 1, 3, 3)) for x in props_h]
    out = torch.empty(len(ops) * nz * 162, dtype=torch.float64, device="cuda")
    with torch.cuda.stream(stream):
        for _ in range(max(1, args.warmup)):
            asq.npr_fourfermion(dims, thin, props, ops, out=out, stream=stream)
        reps = max(3, args.steps)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            asq.npr_fourfermion(dims, thin, props, ops, out=out, stream=stream)
        e1.record(stream)
    stream.synchronize()
    dt = e0.elapsed_time(e1) / 1e3 / reps
    flops = npr_flops(nz, len(ops))
    tf = flops / dt / 1e12
    log(f"four-fermion contraction: {dt * 1e3:.3f} ms per call, {flops / 1e9:.1f} GFLOP, {tf:.1f} TFLOP/s FP64 "
        f"({tf / PEAK_FP64_TFLOPS:.0%} of peak)")
    import oracle

    rng = np.random.Generator(np.random.PCG64(5))
    zs = np.unique(rng.integers(0, nz, 24))
    got = out.view(len(ops), nz, 162)[:, torch.as_tensor(zs, device="cuda")].cpu().numpy()
    got = got.view(np.complex128).reshape(len(ops), len(zs), 81)
    want = oracle.npr_fourfermion(dims, U, props_h, ops, zs=zs).reshape(len(ops), len(zs), 81)
    err = max(float(np.abs(got[k] - want[k]).max() / np.abs(want[k]).max()) for k in range(len(ops)))
    log(f"oracle check on {len(zs)} hypercubes: max error {err:.2e} of each operator's largest entry")
    cpu = None
    if not args.no_cpu_baseline:
        n = 8
        t0 = time.perf_counter()
        oracle.npr_fourfermion(dims, U, props_h, ops, zs=np.arange(n))
        per_z = (time.perf_counter() - t0) / n
        n = int(min(nz // CPU_RUNS, max(n, args.cpu_seconds / CPU_RUNS / max(per_z, 1e-9))))
        per = []
        for _ in range(CPU_RUNS):
            zr = rng.integers(0, nz, n)
            t0 = time.perf_counter()
            oracle.npr_fourfermion(dims, U, props_h, ops, zs=zr)
            per.append((time.perf_counter() - t0) / n)
        t_all = _spread(np.asarray(per), nz)
        cpu = {"value": 1.0 / t_all["median"], "unit": "contractions/s", "cores": oracle.num_threads(),
               "kind": "oracle",
               "sample": f"oracle FP64 contraction of {len(ops)} operators ({oracle.build_flags()}), {CPU_RUNS} "
                         f"runs at {n} random hypercubes of {nz} each, median scaled to the whole lattice",
               "seconds_per_contraction": t_all}
    out_j = {"metric": METRIC, "workload": "npr_20x20x20x64", "value": 1.0 / dt, "unit": "contractions/s",
             "ms_per_contraction": dt * 1e3, "operators": len(ops), "hypercubes": nz, "dtype": "f64",
             "gflop_per_contraction": flops / 1e9,
             "roofline": {"bound": "alu", "achieved": tf, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                          "frac": tf / PEAK_FP64_TFLOPS, "traffic": None,
                          "kernel": "npr_kernel (FP64 VALU)"},
             "oracle_sampled_hypercubes": len(zs), "oracle_max_rel_error": err,
             "propagator_solves_s": t_prop,
             "paper_context": {"npr_gflops_titan_black": 113.36, "npr_gflops_gtx580": 76.19,
                               "note": "other hardware, real ensemble, the paper's code and flop convention"}}
    if cpu:
        out_j["cpu_baseline"] = cpu
    print(json.dumps(out_j), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only (the library has no multi-GPU path); use --gpus 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch

    import paper_1411_2223_amd as asq

    asq.load()
    if not args.no_cpu_baseline and not args.kernels_only:
        import oracle

        oracle.select_native_build()  # the CPU baseline runs code tuned for this host
    if args.workload == "single_20x20x20x64":
        run_single(args, asq, torch)
    elif args.workload == "batched_20x20x20x64":
        run_batched(args, asq, torch)
    elif args.workload == "threelevel_48x48x48x96":
        run_threelevel(args, asq, torch)
    elif args.workload == "asqtad_20x20x20x64":
        run_asqtad(args, asq, torch)
    elif args.workload == "npr_20x20x20x64":
        run_npr(args, asq, torch)
    else:
        run_serving(args, asq, torch)


if __name__ == "__main__":
    main()
