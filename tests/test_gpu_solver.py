"""GPU CG solvers (cg_solve / cg_solve_batch through the C ABI) against the FP64 oracle.

Several x are correct for an iterative solver, so x is never compared with the
oracle's x elementwise: the oracle applies its own FP64 operator to the GPU's x
and the relative true residual must be <= tol (1e-10).  Plain FP64 CG must also
take the oracle's iteration count (+-2).  Batch invariance and graph/eager
equality are bitwise.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import gauge_arrays, oracle_resid_cols

pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module")
def asq():
    import torch

    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_1411_2223_amd as m

    m.load()
    return m


def _solve(asq, g, masses, b, mode, **kw):
    import torch

    bd = asq.vec_to_device(b, "f64")
    res = g.solve(masses, bd, mode=mode, **kw)
    torch.cuda.synchronize()
    x = asq.vec_from_device(res.x, len(masses), g.half, "f64")
    return x, res


@pytest.mark.parametrize("mode", ["f64", "mixed32", "mixed16"])
def test_cg_tiny_config(asq, mode):
    w = synth.WORKLOADS["tiny_4x4x4x8"]
    dims, m = w["dims"], w["masses"][0]
    fat, lng = gauge_arrays(dims, w["eps"], synth.gauge_seed(w["index"]))
    g = asq.Gauge(dims, fat, lng, precs=("f64", "f32", "f16"), recon=12)
    b = synth.make_sources(dims, 1, synth.source_seed(w["index"]))
    x, res = _solve(asq, g, [m], b, mode)
    st = res.stats[0]
    r = oracle.true_residual(dims, fat, lng, m, b[0], x[0])
    _, it_o, _, _ = oracle.cg(dims, fat, lng, m, b[0], tol=TOL)
    print(f"mode={mode} iters={st['iters']} oracle_iters={it_o} ru={st['reliable_updates']} "
          f"resid={r:.3e} gpu_resid={st['true_resid']:.3e}", flush=True)
    assert res.rc == 0 and st["converged"] == 1
    assert r <= TOL
    assert abs(st["true_resid"] - r) <= 1e-3 * r + 1e-15
    if mode == "f64":
        assert abs(st["iters"] - it_o) <= 2


@pytest.mark.parametrize("mode", ["f64", "mixed32", "mixed16"])
def test_cg_batch_columns_match_solo(asq, mode):
    dims = (6, 4, 8, 10)
    fat, lng = gauge_arrays(dims, 0.3, 5)
    g = asq.Gauge(dims, fat, lng, precs=("f64", "f32", "f16"), recon=12)
    masses = [0.05, 0.1, 0.02, 0.2, 0.07]
    b = synth.make_sources(dims, len(masses), 42)
    xb, rb = _solve(asq, g, masses, b, mode)
    r = oracle_resid_cols(dims, fat, lng, masses, b, xb)
    print(f"mode={mode} iters={[s['iters'] for s in rb.stats]} resid={r}", flush=True)
    assert rb.rc == 0
    assert np.all(r <= TOL)
    for c in (0, 3):
        xs, rs = _solve(asq, g, [masses[c]], b[c:c + 1], mode)
        assert rs.stats[0]["iters"] == rb.stats[c]["iters"]
        assert np.array_equal(xs[0], xb[c]), "column result depends on the batch"


@pytest.mark.parametrize("mode,recon", [("mixed16", 18), ("mixed16", 12), ("mixed32", 18), ("f64", 18)])
def test_batch_every_launch_variant(asq, mode, recon, monkeypatch):
    # The NORM, UPDATE and RESID epilogues of every launch variant reduce their
    # partials with the same tree: a batched solve gives bitwise the same x under
    # each forced variant (ASQ_VARIANT) as under the tuned ones.
    dims = (6, 4, 8, 10)
    fat, lng = gauge_arrays(dims, 0.3, 5)
    precs = ("f64", "f32", "f16") if recon == 12 else ("f64", "f32")
    g = asq.Gauge(dims, fat, lng, precs=precs, recon=recon)
    masses = [0.05, 0.1, 0.02, 0.2, 0.07, 0.03, 0.15, 0.05, 0.1, 0.04, 0.3, 0.06, 0.08]
    b = synth.make_sources(dims, len(masses), 43)
    x0, r0 = _solve(asq, g, masses, b, mode)
    assert r0.rc == 0
    assert np.all(oracle_resid_cols(dims, fat, lng, masses, b, x0) <= TOL)
    for cols, pipe, order, sweep, chunk in asq.VARIANTS_ALL:
        if chunk or (cols == 1 and (order > 0 or sweep)):
            # one-column tiles: the orders only permute blocks, and runs of blocks need
            # larger lattices; both are covered by the Dslash tests
            continue
        monkeypatch.setenv("ASQ_VARIANT", str(asq.variant_code(cols, pipe, order, sweep=sweep)))
        x, r = _solve(asq, g, masses, b, mode)
        print(f"mode={mode} recon={recon} variant cols={cols} pipe={pipe} order={order} sweep={sweep}", flush=True)
        assert r.rc == 0
        assert [s["iters"] for s in r.stats] == [s["iters"] for s in r0.stats]
        assert np.array_equal(x, x0), f"variant ({cols}, {pipe}, {order}) changes the solution"
    # tiles that stage their x and y neighbours in LDS
    for cols, sweep in ((1, False), (1, True), (4, True), (8, False)):
        monkeypatch.setenv("ASQ_VARIANT", str(asq.variant_code(cols, True, 0, sweep=sweep, lds=True)))
        x, r = _solve(asq, g, masses, b, mode)
        print(f"mode={mode} recon={recon} variant cols={cols} pipe=True lds=True sweep={sweep}", flush=True)
        assert r.rc == 0
        assert [s["iters"] for s in r.stats] == [s["iters"] for s in r0.stats]
        assert np.array_equal(x, x0), "the LDS window changes the solution"


@pytest.mark.parametrize("mode", ["f64", "mixed32", "mixed16"])
def test_multishift_every_mass_and_source(asq, mode):
    # One shifted CG per source carries every mass; the refinement brings each
    # (mass, source) column to the FP64 true residual, checked with the oracle.
    dims = (6, 4, 8, 10)
    fat, lng = gauge_arrays(dims, 0.3, 5)
    g = asq.Gauge(dims, fat, lng, precs=("f64", "f32", "f16"), recon=12)
    masses = [0.05, 0.02, 0.2, 0.1]  # not sorted: the smallest is found
    nsrc = 3
    b = synth.make_sources(dims, nsrc, 71)
    res = g.solve_multishift(masses, asq.vec_to_device(b, "f64"), mode=mode)
    import torch

    torch.cuda.synchronize()
    assert res.rc == 0
    x = asq.vec_from_device(res.x, len(masses) * nsrc, g.half, "f64")
    for j, m in enumerate(masses):
        for sidx in range(nsrc):
            c = j * nsrc + sidx
            r = oracle.true_residual(dims, fat, lng, m, b[sidx], x[c])
            st = res.stats[c]
            print(f"mode={mode} m={m} src={sidx} iters={st['iters']} resid={r:.3e}", flush=True)
            assert st["converged"] == 1 and r <= TOL


def test_multishift_matches_direct_solves(asq):
    # Against dense solves on 4^3 x 8 at a loose tolerance, where the shifted
    # phase does nearly all the work: every mass's error is within the condition
    # number times the tolerance, and its residual within the tolerance.
    dims = (4, 4, 4, 8)
    fat, lng = gauge_arrays(dims, 0.3, 14112223)
    g = asq.Gauge(dims, fat, lng, precs=("f64", "f32"), recon=18)
    masses = [0.1, 0.3, 0.05]
    b = synth.make_sources(dims, 2, 72)
    tol = 1e-6
    res = g.solve_multishift(masses, asq.vec_to_device(b, "f64"), mode="mixed32", tol=tol)
    assert res.rc == 0
    x = asq.vec_from_device(res.x, len(masses) * 2, g.half, "f64")
    for j, m in enumerate(masses):
        A = oracle.dense_operator(lambda v, m=m: oracle.apply_A(dims, fat, lng, m, v), g.half)
        cond = np.linalg.cond(A)
        for sidx in range(2):
            xd = np.linalg.solve(A, b[sidx].reshape(-1)).reshape(g.half, 3)
            err = np.linalg.norm(x[j * 2 + sidx] - xd) / np.linalg.norm(xd)
            r = oracle.true_residual(dims, fat, lng, m, b[sidx], x[j * 2 + sidx])
            print(f"m={m} src={sidx} resid {r:.3e} rel err vs dense {err:.3e} cond {cond:.1f}", flush=True)
            assert r <= tol
            assert err <= cond * tol


def _full_apply(dims, fat, lng, m, xe, xo):
    """M x = 2m x + D x on both parities, composed from the oracle's one-parity D."""
    return (2 * m * xe + oracle.dslash(dims, fat, lng, 0, xo), 2 * m * xo + oracle.dslash(dims, fat, lng, 1, xe))


@pytest.mark.parametrize("mode", ["f64", "mixed32", "mixed16"])
def test_full_system_solve(asq, mode):
    # M x = b on both parities (M = 2m + D) through the even-odd reduction and the
    # odd-site reconstruction: the oracle's M applied to the GPU's x leaves a
    # relative residual <= tol, and the reported residual is that one.
    dims = (6, 4, 8, 10)
    fat, lng = gauge_arrays(dims, 0.3, 5)
    g = asq.Gauge(dims, fat, lng, precs=("f64", "f32", "f16"), recon=12)
    masses = [0.1, 0.05, 0.2]
    n = len(masses)
    v = synth.make_sources(dims, 2 * n, 61)  # even halves, then odd halves
    bd = asq.vec_to_device(v, "f64")
    res = g.solve_full(masses, bd, mode=mode)
    import torch

    torch.cuda.synchronize()
    assert res.rc == 0
    x = asq.vec_from_device(res.x, 2 * n, g.half, "f64")
    for c, m in enumerate(masses):
        re, ro = _full_apply(dims, fat, lng, m, x[c], x[n + c])
        r = np.sqrt(np.sum(np.abs(v[c] - re) ** 2) + np.sum(np.abs(v[n + c] - ro) ** 2))
        r /= np.sqrt(np.sum(np.abs(v[c]) ** 2) + np.sum(np.abs(v[n + c]) ** 2))
        st = res.stats[c]
        print(f"mode={mode} m={m} iters={st['iters']} resid={r:.3e} gpu_resid={st['true_resid']:.3e}", flush=True)
        assert st["converged"] == 1 and r <= TOL
        assert abs(st["true_resid"] - r) <= 1e-3 * r + 1e-15


def test_full_system_matches_dense_solve(asq):
    # brute force on 4^3 x 8: the dense M (both parities) solved directly
    dims, m = (4, 4, 4, 8), 0.1
    fat, lng = gauge_arrays(dims, 0.3, 14112223)
    g = asq.Gauge(dims, fat, lng, precs=("f64", "f32"), recon=18)
    half = g.half
    v = synth.make_sources(dims, 2, 62)
    res = g.solve_full([m], asq.vec_to_device(v, "f64"), mode="mixed32")
    assert res.rc == 0
    x = asq.vec_from_device(res.x, 2, half, "f64")

    def apply_m(z):
        z = z.reshape(2, half, 3)
        re, ro = _full_apply(dims, fat, lng, m, z[0], z[1])
        return np.stack([re, ro])

    M = oracle.dense_operator(apply_m, 2 * half)
    xd = np.linalg.solve(M, v.reshape(-1)).reshape(2, half, 3)
    err = np.linalg.norm(x - xd) / np.linalg.norm(xd)
    print(f"dense full solve: rel err {err:.3e} cond {np.linalg.cond(M):.2e}", flush=True)
    assert err <= 1e-8


def test_graph_matches_eager(asq):
    dims = (6, 4, 8, 10)
    fat, lng = gauge_arrays(dims, 0.3, 5)
    g = asq.Gauge(dims, fat, lng, precs=("f64", "f32"), recon=18)
    b = synth.make_sources(dims, 2, 43)
    x1, r1 = _solve(asq, g, [0.05, 0.1], b, "mixed32", use_graph=True)
    x2, r2 = _solve(asq, g, [0.05, 0.1], b, "mixed32", use_graph=False)
    assert np.array_equal(x1, x2)
    assert [s["iters"] for s in r1.stats] == [s["iters"] for s in r2.stats]


def test_maxiter_and_zero_source(asq):
    dims = (4, 4, 4, 8)
    fat, lng = gauge_arrays(dims, 0.3, 14112223)
    g = asq.Gauge(dims, fat, lng, precs=("f64", "f32"), recon=18)
    b = synth.make_sources(dims, 2, 44)
    b[1] = 0
    x, res = _solve(asq, g, [0.1, 0.1], b, "mixed32", maxiter=5, poll_iters=4)
    assert res.rc == asq.ASQ_ENOCONV
    assert res.stats[0]["converged"] == 0 and res.stats[0]["status"] == asq.ASQ_ENOCONV
    assert res.stats[0]["iters"] <= 8
    assert res.stats[1]["converged"] == 1 and res.stats[1]["iters"] == 0
    assert np.all(x[1] == 0)


@pytest.mark.parametrize("mode", ["f64", "mixed32"])
def test_cg_full_size_single_rhs(asq, mode):
    # 20^3 x 64, m = 0.01, 1 RHS: the paper's lattice shape, the bench's workload
    w = synth.WORKLOADS["single_20x20x20x64"]
    dims, m = w["dims"], w["masses"][0]
    fat, lng = gauge_arrays(dims, w["eps"], synth.gauge_seed(w["index"]))
    g = asq.Gauge(dims, fat, lng, precs=("f64", "f32"), recon=18)
    b = synth.make_sources(dims, 1, synth.source_seed(w["index"]))
    x, res = _solve(asq, g, [m], b, mode, maxiter=20000)
    st = res.stats[0]
    r = oracle.true_residual(dims, fat, lng, m, b[0], x[0])
    print(f"20^3x64 mode={mode} iters={st['iters']} ru={st['reliable_updates']} resid={r:.3e} "
          f"t={st['seconds']:.3f}s gflops={st['gflops']:.1f}", flush=True)
    assert res.rc == 0 and r <= TOL


def test_cg_batched_full_size_f16(asq):
    # 20^3 x 64 with several RHS x masses, FP16-with-norm vectors, FP32 18-real links
    w = synth.WORKLOADS["batched_20x20x20x64"]
    dims = w["dims"]
    fat, lng = gauge_arrays(dims, w["eps"], synth.gauge_seed(w["index"]))
    g = asq.Gauge(dims, fat, lng, precs=("f64", "f32"), recon=18)
    masses = list(w["masses"]) * 2
    b = synth.make_sources(dims, len(masses), synth.source_seed(w["index"]))
    x, res = _solve(asq, g, masses, b, "mixed16", maxiter=20000)
    r = oracle_resid_cols(dims, fat, lng, masses, b, x)
    print(f"batched f16 iters={[s['iters'] for s in res.stats]} resid max={r.max():.3e}", flush=True)
    assert res.rc == 0 and np.all(r <= TOL)


def test_three_level_mid_size(asq):
    # the three-level tier (FP16-with-norm vectors, 16-bit 12-real links, FP32 residual, FP64 x) at
    # 16^3 x 32 with the eps = 0.2 links and m = 0.005 of the 48^3 x 96 workload, 12 columns
    dims, m, eps = (16, 16, 16, 32), 0.005, 0.2
    fat, lng = gauge_arrays(dims, eps, 77)
    g = asq.Gauge(dims, fat, lng, precs=("f64", "f32", "f16"), recon=12)
    b = synth.make_sources(dims, 12, 78)
    x, res = _solve(asq, g, [m] * 12, b, "mixed16", maxiter=20000)
    r = oracle_resid_cols(dims, fat, lng, [m] * 12, b, x)
    print(f"three-level 16^3x32 iters={[s['iters'] for s in res.stats]} resid max={r.max():.3e}", flush=True)
    assert res.rc == 0 and np.all(r <= TOL)


def test_recon12_mixed32_matches_tolerance(asq):
    # FP32 12-real links in the iteration (reconstructed in-kernel), FP64 18-real for the residual
    dims = (8, 6, 4, 12)
    fat, lng = gauge_arrays(dims, 0.2, 6)
    g = asq.Gauge(dims, fat, lng, precs=("f64", "f32"), recon=12)
    b = synth.make_sources(dims, 3, 79)
    masses = [0.01, 0.03, 0.1]
    x, res = _solve(asq, g, masses, b, "mixed32")
    r = oracle_resid_cols(dims, fat, lng, masses, b, x)
    assert res.rc == 0 and np.all(r <= TOL)


@pytest.mark.parametrize("mode,poll", [("f64", 16), ("mixed32", 16), ("mixed32", 5), ("mixed16", 7), ("mixed32", 1)])
def test_folded_scalars_match_scalar_launches(asq, mode, poll, monkeypatch):
    """Narrow batches form alpha inside D_eo and beta inside the direction update
    (alternating two state copies); with both folds switched off every scalar
    comes from the one-block reduction launch.  The sums use the same order and
    tree, so x and the iteration counts must be bitwise equal.  poll = 16 ends a
    block on the second state copy, 5 on the first, 1 folds nothing."""
    dims = (6, 4, 8, 10)
    fat, lng = gauge_arrays(dims, 0.3, 5)
    g = asq.Gauge(dims, fat, lng, precs=("f64", "f32"), recon=18)
    b = synth.make_sources(dims, 2, 47)
    masses = [0.05, 0.1]
    x1, r1 = _solve(asq, g, masses, b, mode, poll_iters=poll)
    monkeypatch.setenv("ASQ_FOLD_ALPHA", "0")
    monkeypatch.setenv("ASQ_FOLD_BETA", "0")
    x2, r2 = _solve(asq, g, masses, b, mode, poll_iters=poll)
    assert r1.rc == 0 and r2.rc == 0
    assert np.array_equal(x1, x2)
    assert [s["iters"] for s in r1.stats] == [s["iters"] for s in r2.stats]
    assert [s["reliable_updates"] for s in r1.stats] == [s["reliable_updates"] for s in r2.stats]
    for c, m in enumerate(masses):
        assert oracle.true_residual(dims, fat, lng, m, b[c], x1[c]) <= TOL


def test_mfma_variant_in_the_solver(asq, monkeypatch):
    # The matrix-core Dslash with its NORM and UPDATE epilogues, forced for a
    # mixed16 batch (FP32 18-real links): every column reaches the FP64 true
    # residual (checked by the oracle) while columns stop at different iterations.
    dims = (6, 4, 8, 10)
    fat, lng = gauge_arrays(dims, 0.3, 5)
    g = asq.Gauge(dims, fat, lng, precs=("f64", "f32"), recon=18)
    masses = [0.05, 0.1, 0.02, 0.2, 0.07, 0.03, 0.15, 0.05, 0.1, 0.04, 0.3, 0.06, 0.08, 0.5, 0.01]
    b = synth.make_sources(dims, len(masses), 44)
    monkeypatch.setenv("ASQ_VARIANT", str(asq.variant_code_mfma(0)))
    x, r = _solve(asq, g, masses, b, "mixed16")
    assert r.rc == 0
    resid = oracle_resid_cols(dims, fat, lng, masses, b, x)
    print(f"mfma solver iters={[s['iters'] for s in r.stats]} resid max={resid.max():.3e}", flush=True)
    assert np.all(resid <= TOL)
    x2, r2 = _solve(asq, g, masses, b, "mixed16")
    assert np.array_equal(x, x2)


def test_solver_rejects_bad_arguments(asq):
    # masses, tolerances, trigger and iteration limits are checked on the host before any launch
    dims = (4, 4, 4, 8)
    fat, lng = gauge_arrays(dims, 0.3, 14112223)
    g = asq.Gauge(dims, fat, lng, precs=("f64", "f32"), recon=18)
    b = asq.vec_to_device(synth.make_sources(dims, 1, 45), "f64")
    bad = [dict(masses=[0.0]), dict(masses=[-0.1]), dict(masses=[float("nan")]), dict(masses=[float("inf")]),
           dict(tol=0.0), dict(tol=float("nan")), dict(delta=1.0), dict(delta=-0.5), dict(maxiter=0),
           dict(mode="mixed16")]  # no FP16-tier links kept: the 16-bit sloppy tier falls back to FP32 links
    for kw in bad:
        args = dict(masses=[0.1], mode="mixed32")
        args.update(kw)
        masses = args.pop("masses")
        if kw.get("mode") == "mixed16":
            res = g.solve(masses, b, **args)  # valid: FP16 vectors with the FP32 links
            assert res.rc == 0
            continue
        with pytest.raises(asq.AsqError) as e:
            g.solve(masses, b, **args)
        assert e.value.code == asq.ASQ_EINVAL, kw
    # a gauge without FP64 links cannot decide on the true residual in any mode
    g32 = asq.Gauge(dims, fat, lng, precs=("f32",), recon=18)
    for mode in ("mixed32", "f64"):
        with pytest.raises(asq.AsqError) as e:
            g32.solve([0.1], b, mode=mode)
        assert e.value.code == asq.ASQ_EINVAL


def test_aliased_buffers_rejected(asq):
    # an output that shares bytes with an input or the workspace is refused on the host
    import torch

    dims = (4, 4, 4, 8)
    fat, lng = gauge_arrays(dims, 0.3, 14112223)
    g = asq.Gauge(dims, fat, lng, precs=("f64", "f32"), recon=18)
    b = asq.vec_to_device(synth.make_sources(dims, 2, 46), "f64")
    flat = b.view(-1)
    col = flat.numel() // 2  # doubles per column
    cases = {
        "dslash in place": lambda: g.dslash(1, b, "f64", 2, out=b),
        "dslash shifted": lambda: g.dslash(1, flat[:col], "f64", 1, out=flat[16 : 16 + col]),
        "solve x = b": lambda: g.solve([0.1, 0.2], b, x=b),
        "solve x inside b": lambda: g.solve([0.1], flat[:col], x=flat[col - 16 : 2 * col - 16]),
    }
    work = g.workspace(2, "mixed32")
    vb = flat.numel() * 8
    buf = asq.empty_bytes(work.numel() + vb)
    b_in_work = buf[:vb].view(torch.float64)
    b_in_work.copy_(flat)
    cases["solve b in the workspace"] = lambda: g.solve([0.1, 0.2], b_in_work, work=buf[: work.numel()])
    cases["solve x in the workspace"] = lambda: g.solve([0.1, 0.2], flat, work=buf[: work.numel()], x=b_in_work)
    xm = torch.empty(3 * flat.numel(), dtype=torch.float64, device=b.device)
    bm = xm[flat.numel() : 2 * flat.numel()]
    bm.copy_(flat)
    cases["multishift x over b"] = lambda: g.solve_multishift([0.1, 0.2, 0.3], bm, x=xm)
    bf = asq.vec_to_device(synth.make_sources(dims, 2, 47), "f64")  # even half, odd half of one column
    cases["full x = b"] = lambda: g.solve_full([0.1], bf, x=bf)
    for name, call in cases.items():
        print(f"aliased: {name}", flush=True)
        with pytest.raises(asq.AsqError) as e:
            call()
        assert e.value.code == asq.ASQ_EINVAL, name
    srv = asq.Server(1 << 26, max_streams=1, max_cols=2)
    gid = srv.register(g)
    with pytest.raises(asq.AsqError) as e:
        srv.submit(gid, [0.1, 0.2], b, b)
    assert e.value.code == asq.ASQ_EINVAL
    srv.close()
    # disjoint buffers still solve
    x, res = _solve(asq, g, [0.1, 0.2], synth.make_sources(dims, 2, 46), "mixed32")
    assert res.rc == 0


def test_binding_checks_tensor_sizes(asq):
    # the C ABI sees pointers only: the binding refuses short, host or strided tensors before a call
    import torch

    dims = (4, 4, 4, 8)
    fat, lng = gauge_arrays(dims, 0.3, 14112223)
    g = asq.Gauge(dims, fat, lng, precs=("f64", "f32"), recon=18)
    b = asq.vec_to_device(synth.make_sources(dims, 2, 48), "f64")
    flat = b.view(-1)
    cases = {
        "dslash short out": lambda: g.dslash(1, b, "f64", 2, out=flat[:100]),
        "dslash host input": lambda: g.dslash(1, b.cpu(), "f64", 2),
        "solve short x": lambda: g.solve([0.1, 0.2], b, x=flat[: flat.numel() // 2].clone()),
        "solve strided b": lambda: g.solve([0.1], flat[::2]),
        "full short b": lambda: g.solve_full([0.1, 0.2], b),
    }
    for name, call in cases.items():
        print(f"binding check: {name}", flush=True)
        with pytest.raises(asq.AsqError) as e:
            call()
        assert e.value.code == asq.ASQ_EINVAL, name


@pytest.mark.parametrize("mode,ncol", [("mixed32", 1), ("mixed32", 2), ("f64", 1), ("f64", 2)])
def test_narrow_batch_beyond_1024_site_blocks(asq, mode, ncol, monkeypatch):
    """Batches of one or two columns form alpha inside D_eo and beta inside the direction
    update only up to 1024 site blocks, where every block's re-read of all partials stays
    small; beyond (24^3 x 48: 1296 blocks of 256 sites) the scalars come from the one-block
    reduction launches whatever the fold switches say.  Both runs must give the same bits
    and the FP64 true residual."""
    import torch

    dims = (24, 24, 24, 48)
    fat, lng = gauge_arrays(dims, 0.3, 91)
    g = asq.Gauge(dims, fat, lng, precs=("f64", "f32"), recon=18)
    assert (g.half + 255) // 256 > 1024
    masses = [0.02, 0.05][:ncol]
    b = synth.make_sources(dims, ncol, 92)
    x1, r1 = _solve(asq, g, masses, b, mode)
    monkeypatch.setenv("ASQ_FOLD_ALPHA", "0")
    monkeypatch.setenv("ASQ_FOLD_BETA", "0")
    x2, r2 = _solve(asq, g, masses, b, mode)
    print(f"24^3x48 mode={mode} ncol={ncol} iters={[s['iters'] for s in r1.stats]}", flush=True)
    assert r1.rc == 0 and r2.rc == 0
    assert [s["iters"] for s in r1.stats] == [s["iters"] for s in r2.stats]
    assert np.array_equal(x1, x2), "folded scalars differ from the scalar launches"
    r = oracle_resid_cols(dims, fat, lng, masses, b, x1)
    assert np.all(r <= TOL)


def test_nan_source_column_reports_enan(asq):
    # One column's source holds a NaN: that column stops with ASQ_ENAN at its first
    # reduction, the call returns ASQ_ENAN, and every other column is bitwise its solo solve.
    dims = (6, 4, 8, 10)
    fat, lng = gauge_arrays(dims, 0.3, 5)
    g = asq.Gauge(dims, fat, lng, precs=("f64", "f32"), recon=18)
    masses = [0.05, 0.1, 0.02]
    b = synth.make_sources(dims, 3, 93)
    b[1, 17, 2] = complex(np.nan, 0.0)
    x, res = _solve(asq, g, masses, b, "mixed32")
    print(f"nan column: rc={res.rc} status={[s['status'] for s in res.stats]}", flush=True)
    assert res.rc == asq.ASQ_ENAN
    assert res.stats[1]["status"] == asq.ASQ_ENAN and res.stats[1]["converged"] == 0
    for c in (0, 2):
        assert res.stats[c]["status"] == 0 and res.stats[c]["converged"] == 1
        xs, rs = _solve(asq, g, [masses[c]], b[c:c + 1], "mixed32")
        assert rs.rc == 0 and rs.stats[0]["iters"] == res.stats[c]["iters"]
        assert np.array_equal(xs[0], x[c])
        assert oracle.true_residual(dims, fat, lng, masses[c], b[c], x[c]) <= TOL


@pytest.mark.parametrize("mode", ["mixed32", "mixed16"])
def test_mixed_cg_on_fp64_only_links(asq, mode):
    # A field kept in FP64 only: the iterated FP32 Dslash reads the FP64 18-real links and
    # rounds them to FP32 on load; every column reaches the oracle's FP64 true residual.
    dims = (6, 4, 8, 10)
    fat, lng = gauge_arrays(dims, 0.3, 5)
    g = asq.Gauge(dims, fat, lng, precs=("f64",), recon=18)
    masses = [0.05, 0.1, 0.02]
    b = synth.make_sources(dims, 3, 94)
    x, res = _solve(asq, g, masses, b, mode)
    r = oracle_resid_cols(dims, fat, lng, masses, b, x)
    print(f"fp64-only links mode={mode} iters={[s['iters'] for s in res.stats]} resid={r}", flush=True)
    assert res.rc == 0 and np.all(r <= TOL)


def test_mixed32_fp64_links_full_size(asq):
    # the 20^3 x 64 single solve with FP64-stored links and FP32 arithmetic
    w = synth.WORKLOADS["single_20x20x20x64"]
    dims, m = w["dims"], w["masses"][0]
    fat, lng = gauge_arrays(dims, w["eps"], synth.gauge_seed(w["index"]))
    g = asq.Gauge(dims, fat, lng, precs=("f64",), recon=18)
    b = synth.make_sources(dims, 1, synth.source_seed(w["index"]))
    x, res = _solve(asq, g, [m], b, "mixed32", maxiter=20000)
    st = res.stats[0]
    r = oracle.true_residual(dims, fat, lng, m, b[0], x[0])
    print(f"20^3x64 mixed32 on FP64 links iters={st['iters']} ru={st['reliable_updates']} resid={r:.3e}", flush=True)
    assert res.rc == 0 and r <= TOL


@pytest.mark.parametrize("mode", ["mixed16", "mixed32"])
def test_stalled_columns_escalate(asq, mode, monkeypatch):
    """A column whose FP64 true residual stops falling (ASQ_STALL_UPDATES reliable updates
    in a row without a drop by ASQ_STALL_DROP) continues from its x in the next tier:
    mixed16 -> mixed32 -> f64.  The host forces the condition: with an unreachable drop
    every reliable update counts as a stall, so each column hands on after two updates
    per tier and finishes in FP64.  Each column still reaches the oracle's 1e-10, the
    counters add up, and a column's result is bitwise its solo run's."""
    dims = (6, 4, 8, 10)
    fat, lng = gauge_arrays(dims, 0.3, 5)
    g = asq.Gauge(dims, fat, lng, precs=("f64", "f32", "f16"), recon=12)
    masses = [0.05, 0.1, 0.02]
    b = synth.make_sources(dims, 3, 95)
    monkeypatch.setenv("ASQ_STALL_UPDATES", "2")
    monkeypatch.setenv("ASQ_STALL_DROP", "1e100")
    x, res = _solve(asq, g, masses, b, mode, poll_iters=4)
    steps = 2 if mode == "mixed16" else 1
    print(f"escalation {mode}: {[(s['iters'], s['reliable_updates'], s['escalations'], s['final_mode']) for s in res.stats]}",
          flush=True)
    assert res.rc == 0
    for c, st in enumerate(res.stats):
        assert st["converged"] == 1 and st["escalations"] == steps and st["final_mode"] == asq.ASQ_MODE_F64
        assert oracle.true_residual(dims, fat, lng, masses[c], b[c], x[c]) <= TOL
    xs, rs = _solve(asq, g, [masses[1]], b[1:2], mode, poll_iters=4)
    assert rs.stats[0]["iters"] == res.stats[1]["iters"] and rs.stats[0]["escalations"] == steps
    assert np.array_equal(xs[0], x[1])
    # the default rule leaves an ordinary solve in its own tier
    monkeypatch.delenv("ASQ_STALL_UPDATES")
    monkeypatch.delenv("ASQ_STALL_DROP")
    x2, r2 = _solve(asq, g, masses, b, mode)
    assert r2.rc == 0 and all(s["escalations"] == 0 and s["final_mode"] == asq.MODES[mode] for s in r2.stats)
