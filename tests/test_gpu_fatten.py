"""GPU asqtad link construction (asqtad_build_links through the C ABI) against the FP64 oracle.

The oracle sums the asqtad paths one by one; the kernel evaluates nested
staples.  Both are FP64 and differ only in the order of the sums: each link
entry is a sum of at most 86 products of seven unitary-bounded matrices, so the
two agree to a few units of 1e-16 times |F| ~ 1; the bound used is 1e-13
absolute.  At the full 20^3 x 64 size the oracle computes sampled sites.
Solves on the constructed links are checked by the oracle's own operator built
from the oracle's links: relative true residual <= 1e-10.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

LINK_TOL = 1e-13


@pytest.fixture(scope="module")
def asq():
    import torch

    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_1411_2223_amd as m

    m.load()
    return m


def _gpu_links(asq, dims, U, u0):
    import torch

    thin = asq.links_to_device(U.reshape(-1, 4, 3, 3))
    fat, lng = asq.build_links(dims, thin, u0)
    torch.cuda.synchronize()

    def host(t):
        return t.cpu().numpy().view(np.complex128).reshape(-1, 4, 3, 3)

    return host(fat), host(lng)


@pytest.mark.parametrize("dims,u0", [((4, 4, 4, 4), 1.0), ((6, 6, 4, 10), 0.87), ((4, 6, 8, 6), 1.0)])
def test_links_match_oracle(asq, dims, u0):
    # (6, 6, 4, 10): 1440 sites, 22.5 blocks of 64 -- a ragged last block
    print(f"links dims={dims} u0={u0}", flush=True)
    U = synth.thin_links(dims, 0.5, seed=41)
    fat, lng = _gpu_links(asq, dims, U, u0)
    want_f, want_l = oracle.asqtad_links(dims, U.reshape(-1, 4, 3, 3), u0)
    assert np.abs(fat - want_f).max() < LINK_TOL
    assert np.abs(lng - want_l).max() < LINK_TOL


def test_links_deterministic(asq):
    dims = (6, 4, 4, 8)
    U = synth.thin_links(dims, 0.4, seed=42)
    a = _gpu_links(asq, dims, U, 0.9)
    b = _gpu_links(asq, dims, U, 0.9)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_links_full_size_sampled(asq):
    """20^3 x 64 thin links of the single-solve workload, 300 sampled sites incl. the wrap edges."""
    w = synth.WORKLOADS["single_20x20x20x64"]
    dims = w["dims"]
    print(f"links full size dims={dims}", flush=True)
    U = synth.thin_links(dims, w["eps"], synth.gauge_seed(w["index"]))
    fat, lng = _gpu_links(asq, dims, U, 1.0)
    X, Y, Z, T = dims
    V = X * Y * Z * T
    rng = np.random.Generator(np.random.PCG64(7))
    edges = [0, V - 1, X - 1, X * Y - 1, X * Y * Z - 1, (T - 1) * X * Y * Z, V - X, V // 2 + X - 1]
    sites = np.concatenate([edges, rng.integers(0, V, size=300 - len(edges))])
    want_f, want_l = oracle.asqtad_links(dims, U.reshape(-1, 4, 3, 3), 1.0, sites=sites)
    assert np.abs(fat[sites] - want_f).max() < LINK_TOL
    assert np.abs(lng[sites] - want_l).max() < LINK_TOL


@pytest.mark.parametrize("mode", ["f64", "mixed32", "mixed16"])
def test_solve_on_constructed_links(asq, mode):
    import torch

    dims, u0, mass = (8, 8, 8, 8), 0.9, 0.05
    print(f"solve on built links mode={mode}", flush=True)
    U = synth.thin_links(dims, 0.3, seed=43)
    g = asq.Gauge.from_thin(dims, U.reshape(-1, 4, 3, 3), u0)
    b = synth.make_sources(dims, 2, seed=44)
    bd = asq.vec_to_device(b, "f64")
    res = g.solve([mass, 2 * mass], bd, mode=mode)
    torch.cuda.synchronize()
    x = asq.vec_from_device(res.x, 2, g.half, "f64")
    fat, lng = oracle.asqtad_links(dims, U.reshape(-1, 4, 3, 3), u0)
    for c, m in enumerate((mass, 2 * mass)):
        assert res.stats[c]["converged"]
        assert oracle.true_residual(dims, fat, lng, m, b[c], x[c]) <= 1e-10


def test_constructed_fat_links_refuse_compression(asq):
    import torch

    dims = (4, 4, 4, 8)
    U = synth.thin_links(dims, 0.3, seed=45)
    thin = asq.links_to_device(U.reshape(-1, 4, 3, 3))
    fat, lng = asq.build_links(dims, thin, 1.0)
    torch.cuda.synchronize()
    with pytest.raises(asq.AsqError) as e:
        asq.Gauge(dims, fat, lng, precs=("f64", "f32"), recon=12)
    assert e.value.code == asq.ASQ_ENOTSU3


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (6, 6, 4, 10), (20, 20, 20, 64)])
def test_plaquette_matches_oracle(asq, dims):
    # FP64 on both sides, different summation orders: 1e-13 absolute on a mean of order 1
    eps = 0.3 if dims[0] == 20 else 0.5
    U = synth.thin_links(dims, eps, seed=46)
    thin = asq.links_to_device(U.reshape(-1, 4, 3, 3))
    p1 = asq.plaquette(dims, thin)
    p2 = asq.plaquette(dims, thin)
    want = oracle.plaquette(dims, U.reshape(-1, 4, 3, 3))
    print(f"plaquette dims={dims}: gpu {p1!r} oracle {want!r}", flush=True)
    assert p1 == p2
    assert abs(p1 - want) < 1e-13


def test_tadpole_improved_construction(asq):
    # u0 from the plaquette: the links match the oracle's at that u0 and a solve meets the tolerance
    import torch

    dims, mass = (8, 8, 8, 8), 0.05
    U = synth.thin_links(dims, 0.3, seed=47)
    u0 = oracle.plaquette(dims, U.reshape(-1, 4, 3, 3)) ** 0.25
    g = asq.Gauge.from_thin(dims, U.reshape(-1, 4, 3, 3), u0="plaquette")
    fat, lng = oracle.asqtad_links(dims, U.reshape(-1, 4, 3, 3), u0)
    b = synth.make_sources(dims, 1, seed=48)
    res = g.solve([mass], asq.vec_to_device(b, "f64"), mode="mixed32")
    torch.cuda.synchronize()
    x = asq.vec_from_device(res.x, 1, g.half, "f64")
    assert res.rc == 0
    assert oracle.true_residual(dims, fat, lng, mass, b[0], x[0]) <= 1e-10
