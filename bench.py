"""Benchmark of the even-odd asqtad CG on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload single_20x20x20x64]

A step is one complete solve of A x = b (A = 4m^2 - D_eo D_oe, even sites) to a
relative FP64 true residual of 1e-10 with the mixed-precision reliable-update
CG, on synthetic fields shaped like the paper's 20^3 x 64 lattice (inputs
already resident in HBM).  Rank 0 prints one JSON line with solves/s, the
time-to-1e-10, CG GFLOPS (1146 flops per site per Dslash), the speed-up over the
plain FP64 GPU CG, the Dslash HBM roofline (HIP events on the launch stream) and
the CPU oracle baseline on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

PEAK_HBM_GBS = 8000.0
# algorithmic bytes per output site of one half-Dslash at 1 RHS: 16 links + one
# input vector + one output vector (each input read once, the output written once)
BYTES_PER_SITE = {"f64": 16 * 144 + 2 * 48, "f32": 16 * 72 + 2 * 24, "f32r12": 16 * 48 + 2 * 24,
                  "f16": 16 * 72 + 2 * 16, "f16r12": 16 * 24 + 2 * 16}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="single_20x20x20x64")
    ap.add_argument("--mode", default="mixed32", choices=["f64", "mixed32", "mixed16"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="bound on the oracle sample")
    ap.add_argument("--dslash-launches", type=int, default=200)
    ap.add_argument("--kernels-only", action="store_true",
                    help="only launch the Dslash tiers and a 1 GiB copy probe (for hardware-counter runs)")
    return ap.parse_args()


def kernels_only(args, asq, g, dims):
    """Fixed launches for counter collection: each Dslash tier 20 times, then the copy probe."""
    import torch

    half = int(np.prod(dims)) // 2
    stream = torch.cuda.Stream()
    res = {}
    for prec in ("f32", "f64", "f16"):
        dt = time_dslash(asq, g, prec, 1, 20, stream)
        key = prec
        res[prec] = {"us": dt * 1e6, "alg_bytes": BYTES_PER_SITE[key] * half}
    n = 1 << 30
    src = torch.empty(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        asq.check(asq.asq_copy_probe(dst.data_ptr(), src.data_ptr(), n, asq.stream_ptr(stream)), "copy")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(5):
        asq.check(asq.asq_copy_probe(dst.data_ptr(), src.data_ptr(), n, asq.stream_ptr(stream)), "copy")
    e1.record(stream)
    e1.synchronize()
    dt = e0.elapsed_time(e1) * 1e-3 / 5
    res["copy"] = {"us": dt * 1e6, "bytes_read": n, "bytes_written": n, "GBps": 2 * n / dt / 1e9}
    print(json.dumps({"kernels_only": res}), flush=True)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def time_dslash(asq, g, prec, nrhs, launches, stream):
    """Average duration of one Dslash launch (HIP events on the launch stream) -> seconds."""
    import torch

    v = synth.make_sources(g.dims, nrhs, 99)
    vin = asq.vec_to_device(v, prec)
    out = torch.empty_like(vin)
    for _ in range(5):
        g.dslash(1, vin, prec, nrhs, out=out, stream=stream)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(launches):
        g.dslash(1, vin, prec, nrhs, out=out, stream=stream)
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) * 1e-3 / launches


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


def cpu_baseline(w, fat, lng, b, mass, iters_full, seconds):
    """Oracle CG on the same workload, bounded: time a prefix of iterations, scale to a full solve."""
    import oracle

    dims = w["dims"]
    oracle.lib()
    t0 = time.perf_counter()
    oracle.apply_A(dims, fat, lng, mass, b)  # one operator application to size the sample
    per_apply = time.perf_counter() - t0
    n = max(3, int(seconds / max(per_apply, 1e-6)))
    t0 = time.perf_counter()
    _, it, _, _ = oracle.cg(dims, fat, lng, mass, b, tol=w["tol"], maxiter=n)
    dt = time.perf_counter() - t0
    # the sample includes one extra operator application (its true residual)
    per_iter = max(dt - per_apply, 1e-9) / max(it, 1)
    t_solve = per_iter * iters_full
    return {"value": 1.0 / t_solve, "unit": "solves/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"oracle FP64 CG, first {it} of {iters_full} iterations at {dims[0]}^3x{dims[3]} "
                      f"({dt:.1f} s, {per_iter * 1e3:.1f} ms/iteration), scaled to the full solve",
            "seconds_per_solve": t_solve}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch

    import paper_1411_2223_amd as asq

    asq.load()
    w = synth.WORKLOADS[args.workload]
    dims, mass = w["dims"], w["masses"][0]
    half = int(np.prod(dims)) // 2
    log(f"workload {args.workload} dims={dims} m={mass} mode={args.mode}")
    fat, lng = synth.make_gauge(dims, w["eps"], synth.gauge_seed(w["index"]))
    b = synth.make_sources(dims, 1, synth.source_seed(w["index"]))
    g = asq.Gauge(dims, fat, lng, precs=("f64", "f32"), recon=18)
    if args.kernels_only:
        kernels_only(args, asq, g, dims)
        return
    stream = torch.cuda.Stream()
    bd = asq.vec_to_device(b, "f64")
    work = g.workspace(1, args.mode)
    x = torch.empty_like(bd)
    torch.cuda.synchronize()

    def step(mode, wk):
        return g.solve([mass], bd, mode=mode, tol=w["tol"], maxiter=50000, work=wk, x=x, stream=stream)

    for k in range(args.warmup):
        r = step(args.mode, work)
        log(f"warmup {k}: iters={r.stats[0]['iters']} ru={r.stats[0]['reliable_updates']} "
            f"resid={r.stats[0]['true_resid']:.3e} {r.stats[0]['seconds'] * 1e3:.1f} ms")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    last = None
    for k in range(args.steps):
        last = step(args.mode, work)
        if last.rc != 0:
            raise SystemExit(f"solve failed rc={last.rc}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    st = last.stats[0]
    log(f"timed {args.steps} solves in {elapsed:.3f} s; iters={st['iters']} ru={st['reliable_updates']} "
        f"resid={st['true_resid']:.3e}")

    # plain FP64 GPU CG at the same accuracy (speed-up reference), outside the timed region
    work64 = g.workspace(1, "f64")
    r64 = step("f64", work64)
    r64 = step("f64", work64)
    t64 = r64.stats[0]["seconds"]
    log(f"f64 CG: iters={r64.stats[0]['iters']} resid={r64.stats[0]['true_resid']:.3e} {t64 * 1e3:.1f} ms")

    # dominant kernel: the sloppy single-RHS Dslash (FP32 vectors, FP32 18-real links)
    prec_key = "f32" if args.mode == "mixed32" else ("f64" if args.mode == "f64" else "f16")
    tprec = {"mixed32": "f32", "f64": "f64", "mixed16": "f16"}[args.mode]
    dt = time_dslash(asq, g, tprec, 1, args.dslash_launches, stream)
    bytes_launch = BYTES_PER_SITE[prec_key] * half
    achieved = bytes_launch / dt / 1e9
    dt64 = time_dslash(asq, g, "f64", 1, max(20, args.dslash_launches // 4), stream)
    log(f"dslash {tprec}: {dt * 1e6:.2f} us, {achieved:.0f} GB/s; f64: {dt64 * 1e6:.2f} us, "
        f"{BYTES_PER_SITE['f64'] * half / dt64 / 1e9:.0f} GB/s")

    copy_gbs = copy_bandwidth(asq, stream)
    log(f"copy probe: {copy_gbs:.0f} GB/s")
    ms = elapsed / args.steps * 1e3
    iters = st["iters"]
    flops = half * ((2 * 1146 + 72) * iters + (2 * 1146 + 36) * st["reliable_updates"])
    out = {
        "metric": "asqtad Dslash HBM GB/s; CG time-to-1e-10 at 20^3x64; solves/s + p99 latency",
        "value": args.steps / elapsed,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.mode == "mixed32" else ("f64" if args.mode == "f64" else "f16"),
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {dims[0]}x{dims[1]}x{dims[2]}x{dims[3]} even-odd asqtad CG, "
                               f"1 RHS, m={mass}, eps={w['eps']}, tol 1e-10 true residual, {args.mode} "
                               f"reliable-update CG, FP32/FP64 18-real links",
                   "global_batch": 1, "parallelism": "single GPU"},
        "time_to_solution_ms": ms,
        "iterations": iters,
        "reliable_updates": st["reliable_updates"],
        "true_resid": st["true_resid"],
        "cg_gflops": flops / (ms * 1e-3) / 1e9,
        "f64_cg_ms": t64 * 1e3,
        "f64_cg_iterations": r64.stats[0]["iters"],
        "speedup_vs_f64_cg": t64 * 1e3 / ms,
        "dslash_gbs": achieved,
        "dslash_f64_gbs": BYTES_PER_SITE["f64"] * half / dt64 / 1e9,
        "copy_probe_gbs": copy_gbs,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": None,
                     "kernel": f"dslash_kernel {tprec} 18-real, 1 RHS", "us_per_launch": dt * 1e6,
                     "bytes_per_launch": bytes_launch},
        "paper_context": {"cg_gflops_titan_black_mixed": 46.48, "note": "other hardware, real MILC ensemble"},
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(w, fat, lng, b[0], mass, r64.stats[0]["iters"], args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
