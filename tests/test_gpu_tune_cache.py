"""The autotuner's cache file (ASQ_TUNE_CACHE): JSON that maps each tuning key to a
launch variant; a second process takes its choices from the file without timing
again; entries naming a variant the tuner could not have chosen are ignored.  Every
variant computes the same result, so the outputs of all runs are bitwise equal.

Each run is a child process, since the library reads the file once per process.
"""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import sys
import numpy as np
import torch
sys.path.insert(0, sys.argv[1])
import paper_1411_2223_amd as asq
import synth
asq.load()
dims = (6, 4, 8, 10)
fat, lng = synth.make_gauge(dims, 0.3, 5)
g = asq.Gauge(dims, fat, lng, precs=("f64", "f32"), recon=18)
v = synth.make_sources(dims, 3, 21)
out = g.dslash(1, asq.vec_to_device(v, "f32"), "f32", 3)
res = g.solve([0.1, 0.2], asq.vec_to_device(synth.make_sources(dims, 2, 22), "f64"), mode="mixed32")
torch.cuda.synchronize()
assert res.rc == 0
np.save(sys.argv[2], np.concatenate([out.cpu().numpy().view(np.uint8).ravel(),
                                     res.x.cpu().numpy().view(np.uint8).ravel()]))
print("child done", flush=True)
"""


def _run(tmp_path, tag, cache, tune="1"):
    env = dict(os.environ, ASQ_TUNE_CACHE=str(cache), ASQ_TUNE=tune, ASQ_LOG="1")
    out = tmp_path / f"{tag}.npy"
    print(f"tune cache run {tag}", flush=True)
    r = subprocess.run([sys.executable, "-c", CHILD, ROOT, str(out)], env=env, capture_output=True, text=True,
                       timeout=300, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    tuned = [l for l in r.stderr.splitlines() if l.startswith("[asq] tune ")]
    return np.load(out), tuned


def test_tune_cache_json_roundtrip(tmp_path):
    cache = tmp_path / "tune.json"
    a, tuned_a = _run(tmp_path, "first", cache)
    assert tuned_a, "the first process times the candidates"
    table = json.loads(cache.read_text())
    assert table and all(isinstance(v, int) for v in table.values())
    for key, code in table.items():
        assert key.count("/") == 6, key
        assert code & 0xFF in (1, 2, 4, 6, 8, 12) and not code & 0x10000 and not code & 0x4000, (key, code)
        assert code >> 16 == 0, (key, code)
    b, tuned_b = _run(tmp_path, "second", cache)
    assert not tuned_b, "the second process takes every choice from the file"
    assert np.array_equal(a, b)
    # entries the tuner could not have chosen (an unbuilt width, the matrix-core form, a tile wider
    # than the batch) are ignored in favour of the built-in defaults
    bad = [3, 0x10000 | 32, 8 | (1 << 14), 12]
    cache.write_text(json.dumps({k: bad[i % len(bad)] for i, k in enumerate(table)}, indent=1))
    c, tuned_c = _run(tmp_path, "corrupt", cache)
    assert not tuned_c
    assert np.array_equal(a, c)
