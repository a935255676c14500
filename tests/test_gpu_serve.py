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


def test_mixed_block_shapes_same_as_alone(asq):
    # Requests with different poll_iters and graph settings are never batched together:
    # each joins a batch of its own block shape, so its reliable updates fall where
    # they fall alone, and its x is bitwise that of a solo solve with its parameters.
    import torch

    dims = (6, 4, 8, 10)
    fat, lng = gauge_arrays(dims, 0.3, 5)
    g = asq.Gauge(dims, fat, lng, precs=("f64", "f32"), recon=18)
    srv = asq.Server(1 << 30, max_streams=4, max_cols=4)
    gid = srv.register(g)
    shapes = [(8, True), (16, True), (8, False), (16, True), (8, True), (5, True)]
    tickets, keep = {}, {}
    for k, (poll, graph) in enumerate(shapes):
        masses = [0.03 + 0.01 * k, 0.1]
        b = synth.make_sources(dims, 2, 500 + k)
        bd = asq.vec_to_device(b, "f64")
        x = torch.empty_like(bd)
        t = srv.submit(gid, masses, bd, x, mode="mixed32", delta=0.01, poll_iters=poll, use_graph=graph)
        tickets[t] = 2
        keep[t] = (k, masses, b, bd, x, poll, graph)
    res = _wait(srv, tickets)
    torch.cuda.synchronize()
    for t, (rc, stats, latency) in res.items():
        k, masses, b, bd, x, poll, graph = keep[t]
        assert rc == 0
        xm = asq.vec_from_device(x, 2, g.half, "f64")
        alone = g.solve(masses, bd, mode="mixed32", delta=0.01, poll_iters=poll, use_graph=graph)
        torch.cuda.synchronize()
        xa = asq.vec_from_device(alone.x, 2, g.half, "f64")
        print(f"request {k} poll={poll} graph={graph}: ru {[s['reliable_updates'] for s in stats]} "
              f"alone {[s['reliable_updates'] for s in alone.stats]}", flush=True)
        assert [s["iters"] for s in alone.stats] == [s["iters"] for s in stats]
        assert np.array_equal(xa, xm), f"request {k}: result differs alone vs in the mix"
        assert np.all(oracle_resid_cols(dims, fat, lng, masses, b, xm) <= 1e-10)
    srv.close()


def test_submit_waits_for_the_producer_stream(asq):
    # b is written on a side stream behind a long queue of work and submitted without a
    # host synchronisation: the server reads it only after that stream's work.
    import torch

    dims = (6, 4, 8, 10)
    fat, lng = gauge_arrays(dims, 0.3, 5)
    g = asq.Gauge(dims, fat, lng, precs=("f64", "f32"), recon=18)
    srv = asq.Server(1 << 28, max_streams=1, max_cols=2)
    gid = srv.register(g)
    b = synth.make_sources(dims, 2, 510)
    src = asq.vec_to_device(b, "f64")
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    bd = torch.zeros_like(src)
    x = torch.empty_like(src)
    a = torch.randn(2048, 2048, device=src.device)
    with torch.cuda.stream(side):
        for _ in range(40):
            a = torch.tanh(a @ a * 1e-3)
        bd.copy_(src)
        t = srv.submit(gid, [0.05, 0.1], bd, x, mode="mixed32", stream=side)
    res = _wait(srv, {t: 2})
    torch.cuda.synchronize()
    rc, stats, _ = res[t]
    assert rc == 0 and all(s["iters"] > 0 for s in stats)
    xm = asq.vec_from_device(x, 2, g.half, "f64")
    assert np.all(oracle_resid_cols(dims, fat, lng, [0.05, 0.1], b, xm) <= 1e-10)
    srv.close()


def test_queue_full_returns_eagain(asq, monkeypatch):
    # a queue of two (ASQ_SERVE_MAX_QUEUE) behind a long request that holds the only slot:
    # the third queued request is refused with ASQ_EAGAIN, the others complete
    import torch

    monkeypatch.setenv("ASQ_SERVE_MAX_QUEUE", "2")
    dims = (16, 16, 16, 32)
    fat, lng = gauge_arrays(dims, 0.3, 77)
    g = asq.Gauge(dims, fat, lng, precs=("f64", "f32"), recon=18)
    srv = asq.Server(1 << 30, max_streams=1, max_cols=1)
    gid = srv.register(g)
    bufs = []
    tickets = {}
    # the long one: an unreachable tolerance, stopped by maxiter
    b0 = asq.vec_to_device(synth.make_sources(dims, 1, 520), "f64")
    x0 = torch.empty_like(b0)
    t0 = srv.submit(gid, [0.005], b0, x0, mode="mixed32", tol=1e-300, maxiter=20000)
    tickets[t0] = 1
    time.sleep(0.05)  # admitted by now: the queue is empty again
    for k in range(2):
        bk = asq.vec_to_device(synth.make_sources(dims, 1, 521 + k), "f64")
        xk = torch.empty_like(bk)
        tickets[srv.submit(gid, [0.1], bk, xk, mode="mixed32")] = 1
        bufs.append((bk, xk))
    b3 = asq.vec_to_device(synth.make_sources(dims, 1, 530), "f64")
    with pytest.raises(asq.AsqError) as e:
        srv.submit(gid, [0.1], b3, torch.empty_like(b3), mode="mixed32")
    assert e.value.code == asq.ASQ_EAGAIN
    res = _wait(srv, tickets, timeout=120.0)
    assert res[t0][0] == asq.ASQ_ENOCONV
    assert all(res[t][0] == 0 for t in tickets if t != t0)
    srv.close()


def test_serving_mixed16_full_size(asq):
    # the serving bench's mode on the paper's lattice shape: FP16-with-norm vectors,
    # FP32 links, continuous batching of requests of different widths; every served x
    # meets the oracle's FP64 true residual and one request is bitwise its solo solve
    import torch

    w = synth.WORKLOADS["single_20x20x20x64"]
    dims = w["dims"]
    fat, lng = gauge_arrays(dims, w["eps"], synth.gauge_seed(w["index"]))
    g = asq.Gauge(dims, fat, lng, precs=("f64", "f32"), recon=18)
    srv = asq.Server(1 << 33, max_streams=2, max_cols=4)
    gid = srv.register(g)
    tickets, keep = {}, {}
    for k, masses in enumerate([[0.02, 0.05], [0.01], [0.1, 0.03, 0.07]]):
        b = synth.make_sources(dims, len(masses), 540 + k)
        bd = asq.vec_to_device(b, "f64")
        x = torch.empty_like(bd)
        t = srv.submit(gid, masses, bd, x, mode="mixed16", poll_iters=8)
        tickets[t] = len(masses)
        keep[t] = (k, masses, b, bd, x)
    res = _wait(srv, tickets, timeout=120.0)
    torch.cuda.synchronize()
    for t, (rc, stats, latency) in res.items():
        k, masses, b, bd, x = keep[t]
        xm = asq.vec_from_device(x, len(masses), g.half, "f64")
        r = oracle_resid_cols(dims, fat, lng, masses, b, xm)
        print(f"mixed16 request {k}: iters {[s['iters'] for s in stats]} resid {r}", flush=True)
        assert rc == 0 and np.all(r <= 1e-10)
        if k == 1:
            alone = g.solve(masses, bd, mode="mixed16", poll_iters=8)
            torch.cuda.synchronize()
            assert np.array_equal(asq.vec_from_device(alone.x, 1, g.half, "f64"), xm)
    srv.close()
