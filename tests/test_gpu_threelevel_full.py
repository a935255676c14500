"""The 48^3 x 96 three-level workload at its full size, in the launch configuration the
bench times: eps = 0.2 links, 16-bit 12-real links and FP16-with-norm vectors in the
iteration, 12 columns, m = 0.005, tol 1e-10.

* The 12-column Dslash of that tier against the FP64 oracle on both parities, with
  the FP16 bounds of the single-Dslash tests (normwise sqrt(6) 2^-12 per column, and
  sqrt(2) 2^-12 of the column's largest entry elementwise, plus FP32 arithmetic).
* The 12-column mixed16 solve: every column's FP64 true residual, evaluated by the
  oracle's own operator on the host, at most 1e-10.

Generating the gauge field takes about a minute on the host; the module does it once.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import MAX_TOL, TOL, max_err, quantize_like_device, rel_err

pytestmark = pytest.mark.gpu

W = synth.WORKLOADS["threelevel_48x48x48x96"]


@pytest.fixture(scope="module")
def asq():
    import torch

    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_1411_2223_amd as m

    m.load()
    return m


@pytest.fixture(scope="module")
def field(asq):
    dims = W["dims"]
    print(f"\ngenerating the {dims} eps={W['eps']} gauge field", flush=True)
    fat, lng = synth.make_gauge(dims, W["eps"], synth.gauge_seed(W["index"]))
    g = asq.Gauge(dims, fat, lng, precs=("f64", "f32", "f16"), recon=12)
    yield dims, fat, lng, g
    g.close()


@pytest.mark.timeout(600)
def test_threelevel_dslash_full_size(asq, field):
    import torch

    dims, fat, lng, g = field
    ncol = W["nrhs"]
    half = int(np.prod(dims)) // 2
    for out_parity in (0, 1):
        v = synth.make_sources(dims, ncol, 200 + out_parity)
        vin = asq.vec_to_device(v, "f16")
        out = g.dslash(out_parity, vin, "f16", ncol)
        torch.cuda.synchronize()
        got = asq.vec_from_device(out, ncol, half, "f16")
        del out, vin
        ref = np.stack([oracle.dslash(dims, fat, lng, out_parity, c) for c in quantize_like_device(v, "f16")])
        err = rel_err(got, ref)
        emax = max_err(got, ref)
        print(f"48^3x96 f16 r12 x{ncol} parity={out_parity} max rel err {err.max():.3e} "
              f"max elementwise {emax.max():.3e}", flush=True)
        assert err.max() <= TOL["f16"]
        assert emax.max() <= MAX_TOL["f16"]


@pytest.mark.timeout(600)
def test_threelevel_solve_full_size(asq, field):
    import torch

    dims, fat, lng, g = field
    ncol, mass = W["nrhs"], W["masses"][0]
    b = synth.make_sources(dims, ncol, synth.source_seed(W["index"]))
    res = g.solve([mass] * ncol, asq.vec_to_device(b, "f64"), mode="mixed16", tol=W["tol"], maxiter=20000)
    torch.cuda.synchronize()
    x = asq.vec_from_device(res.x, ncol, g.half, "f64")
    r = np.array([oracle.true_residual(dims, fat, lng, mass, b[c], x[c]) for c in range(ncol)])
    its = [s["iters"] for s in res.stats]
    print(f"48^3x96 three-level iters={its} reliable updates={[s['reliable_updates'] for s in res.stats]} "
          f"oracle resid max={r.max():.3e}", flush=True)
    assert res.rc == 0
    assert all(s["converged"] for s in res.stats)
    assert np.all(r <= W["tol"])
