"""Serving loop (serve_* through the C ABI): continuous batching, admission and
result invariance.  A request's solution must be the same alone (cg_solve_batch
on that request only) and in the mix (sharing batches and the device with
other requests); the design makes it bitwise equal, and every result also meets
the oracle's FP64 true-residual bound."""
import time

import numpy as np
import pytest

import synth
from gpu_common import gauge_arrays, oracle_resid_cols

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def asq():
    import torch

    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_1411_2223_amd as m

    m.load()
    return m


def _wait(srv, tickets, timeout=60.0):
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        for t, n in tickets.items():
            if t in out:
                continue
            r = srv.poll(t, n)
            if r is not None:
                out[t] = r
        assert time.time() - t0 < timeout, "serving did not finish"
        time.sleep(0.001)
    return out


@pytest.mark.parametrize("max_cols,max_streams", [(8, 2), (4, 1)])
def test_same_alone_and_in_the_mix(asq, max_cols, max_streams):
    import torch

    lat = [((4, 4, 4, 8), 0.3, 14112223), ((6, 4, 8, 10), 0.3, 5)]
    gauges, arrays = [], []
    for dims, eps, seed in lat:
        fat, lng = gauge_arrays(dims, eps, seed)
        arrays.append((dims, fat, lng))
        gauges.append(asq.Gauge(dims, fat, lng, precs=("f64", "f32"), recon=18))
    srv = asq.Server(1 << 30, max_streams=max_streams, max_cols=max_cols)
    gids = [srv.register(g) for g in gauges]
    rng = np.random.default_rng(5)
    reqs = []
    for k in range(7):
        li = k % 2
        n = int(rng.integers(1, 4))
        masses = list(rng.uniform(0.02, 0.2, n))
        b = synth.make_sources(arrays[li][0], n, 300 + k)
        reqs.append((li, masses, b))
    # submit everything at once: requests queue, share batches and streams, and reuse freed slots
    tickets, xs = {}, {}
    for k, (li, masses, b) in enumerate(reqs):
        bd = asq.vec_to_device(b, "f64")
        x = torch.empty_like(bd)
        t = srv.submit(gids[li], masses, bd, x, mode="mixed32", delta=0.01, poll_iters=8)
        tickets[t] = len(masses)
        xs[t] = (k, bd, x)
    res = _wait(srv, tickets)
    torch.cuda.synchronize()
    for t, (rc, stats, latency) in res.items():
        k, bd, x = xs[t]
        li, masses, b = reqs[k]
        dims, fat, lng = arrays[li]
        assert rc == 0 and all(s["converged"] for s in stats) and latency > 0
        print(f"request {k}: iters {[s['iters'] for s in stats]} resid {[s['true_resid'] for s in stats]}", flush=True)
        assert all(0 < s["true_resid"] <= 1e-10 for s in stats)
        xm = asq.vec_from_device(x, len(masses), gauges[li].half, "f64")
        r = oracle_resid_cols(dims, fat, lng, masses, b, xm)
        assert np.all(r <= 1e-10)
        alone = gauges[li].solve(masses, bd, mode="mixed32", delta=0.01, poll_iters=8)  # the server's parameters
        torch.cuda.synchronize()
        xa = asq.vec_from_device(alone.x, len(masses), gauges[li].half, "f64")
        assert [s["iters"] for s in alone.stats] == [s["iters"] for s in stats]
        assert np.array_equal(xa, xm), f"request {k}: result differs alone vs in the mix"
    srv.close()


def test_admission_limits(asq):
    import torch

    dims = (4, 4, 4, 8)
    fat, lng = gauge_arrays(dims, 0.3, 14112223)
    g = asq.Gauge(dims, fat, lng, precs=("f64", "f32"), recon=18)
    # an arena too small for one batch: the request can never run
    tiny = asq.Server(1 << 16, max_streams=1, max_cols=4)
    gid = tiny.register(g)
    b = asq.vec_to_device(synth.make_sources(dims, 1, 1), "f64")
    x = torch.empty_like(b)
    with pytest.raises(asq.AsqError) as e:
        tiny.submit(gid, [0.1], b, x)
    assert e.value.code == asq.ASQ_ENOMEM
    tiny.close()
    # more columns than a batch holds
    srv = asq.Server(1 << 28, max_streams=1, max_cols=2)
    gid = srv.register(g)
    b3 = asq.vec_to_device(synth.make_sources(dims, 3, 2), "f64")
    with pytest.raises(asq.AsqError) as e:
        srv.submit(gid, [0.1, 0.1, 0.1], b3, torch.empty_like(b3))
    assert e.value.code == asq.ASQ_ENOMEM
    # a request submitted while another is running is admitted when slots free up
    b2 = asq.vec_to_device(synth.make_sources(dims, 2, 3), "f64")
    x2 = torch.empty_like(b2)
    t1 = srv.submit(gid, [0.1, 0.05], b2, x2)
    bb = asq.vec_to_device(synth.make_sources(dims, 2, 4), "f64")
    xb = torch.empty_like(bb)
    t2 = srv.submit(gid, [0.2, 0.07], bb, xb)
    res = _wait(srv, {t1: 2, t2: 2})
    assert res[t1][0] == 0 and res[t2][0] == 0
    srv.close()


def test_destroy_completes_submitted_requests(asq):
    # closing the server with requests still queued and running finishes them:
    # every x is written and meets the tolerance without a poll
    import torch

    dims = (6, 4, 8, 10)
    fat, lng = gauge_arrays(dims, 0.3, 5)
    g = asq.Gauge(dims, fat, lng, precs=("f64", "f32"), recon=18)
    srv = asq.Server(1 << 28, max_streams=1, max_cols=2)
    gid = srv.register(g)
    reqs = []
    for k in range(4):
        masses = [0.05 + 0.02 * k, 0.1]
        b = synth.make_sources(dims, 2, 400 + k)
        bd = asq.vec_to_device(b, "f64")
        x = torch.zeros_like(bd)
        srv.submit(gid, masses, bd, x, mode="mixed32")
        reqs.append((masses, b, bd, x))
    srv.close()
    torch.cuda.synchronize()
    for masses, b, bd, x in reqs:
        xm = asq.vec_from_device(x, len(masses), g.half, "f64")
        assert np.all(oracle_resid_cols(dims, fat, lng, masses, b, xm) <= 1e-10)
