"""Host-side checks of bench.py's command line (no GPU needed)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_unknown_workload_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--workload", "nope"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0 and "invalid choice" in r.stderr


def _bench():
    import importlib.util

    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_serving_summary_keeps_warm_up_out_of_the_window():
    # 10 warm-up requests (late completions) and 20 measured ones arriving 1 s apart, each
    # done 0.5 s after arrival: 20 served over [10 s, 29.5 s]
    bench = _bench()
    trace = [{"arrival": float(k)} for k in range(30)]
    done = [(k, 0, 0.5, 2, k % 2, 1e-11, k + 0.5) for k in range(10, 30)]
    done += [(k, 0, 40.0, 2, 0, 1e-11, k + 40.0) for k in range(10)]
    s = bench.serving_summary(done, trace, 10, [(4, 4, 4, 4), (8, 8, 8, 8)])
    assert s["requests"] == 20 and s["rhs_solves"] == 40 and s["failed"] == 0
    assert abs(s["window_s"] - 19.5) < 1e-12
    assert abs(s["value"] - 20 / 19.5) < 1e-12
    assert abs(s["offered_requests_per_s"] - 20 / 19.0) < 1e-12
    assert s["stable"]
    assert abs(s["p50_latency_ms"] - 500.0) < 1e-9
    assert s["per_lattice"]["4x4x4x4"]["n"] == 10 and s["per_lattice"]["8x8x8x8"]["n"] == 10
    # a backlog: the last measured request completes 30 s late, so less is served than offered
    done[19] = (29, 0, 30.0, 2, 1, 1e-11, 59.0)
    s = bench.serving_summary(done, trace, 10, [(4, 4, 4, 4), (8, 8, 8, 8)])
    assert abs(s["window_s"] - 49.0) < 1e-12 and not s["stable"]


def test_split_parities_takes_the_halves_of_a_flat_vector():
    import torch

    bench = _bench()
    half = 5
    x = torch.arange(2 * half * 6, dtype=torch.float64)
    e, o = bench.split_parities(x, half)
    assert torch.equal(e, x[:30]) and torch.equal(o, x[30:])
    with __import__("pytest").raises(ValueError):
        bench.split_parities(x[:-6], half)
