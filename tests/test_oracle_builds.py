"""The oracle's two builds compute the same bits.

The benchmark's CPU baseline times a copy of the oracle compiled for the host it runs on
(-O3 -march=native); the tests load the generic -O3 build.  Both turn off FMA
contraction and neither reassociates, so a CG solve and the four-fermion contraction
must agree bit for bit.  Each build runs in a process of its own (the choice is made
before the first oracle call of a process)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

_SCRIPT = r"""
import hashlib, sys
import numpy as np
sys.path.insert(0, {root!r}); sys.path.insert(0, {tests!r})
import oracle, synth
if {native}:
    oracle.select_native_build()
dims = (4, 4, 4, 8)
fat, lng = synth.make_gauge(dims, 0.3, 11)
b = synth.make_sources(dims, 1, 12)[0]
x, it, tr, conv = oracle.cg(dims, fat, lng, 0.1, b, tol=1e-12, maxiter=500)
V = int(np.prod(dims))
U = synth.thin_links(dims, 0.4, 13).reshape(V, 4, 3, 3)
rng = np.random.Generator(np.random.PCG64(14))
G = [rng.standard_normal((V, 3, 3)) + 1j * rng.standard_normal((V, 3, 3)) for _ in range(2)]
v = oracle.npr_fourfermion(dims, U, [G[0], G[0], G[1], G[1]], [(3, 15, 3, 15), (6, 9, 5, 10)], zs=np.arange(8))
h = hashlib.sha256(np.ascontiguousarray(x).tobytes() + np.ascontiguousarray(v).tobytes()).hexdigest()
print(it, oracle.build_flags(), h)
"""


def _run(native):
    code = _SCRIPT.format(root=ROOT, tests=os.path.join(ROOT, "tests"), native=native)
    env = dict(os.environ, OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stderr[-2000:]
    return r.stdout.strip().splitlines()[-1].split()


def test_host_tuned_oracle_matches_generic_build():
    a = _run(False)
    b = _run(True)
    assert "-march=native" in " ".join(b) and "-march=native" not in " ".join(a)
    assert a[0] == b[0], "iteration counts differ"
    assert a[-1] == b[-1], "the host-tuned oracle computes different bits"
