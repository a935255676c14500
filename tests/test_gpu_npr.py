"""GPU parity of the one-colour four-fermion operator (asqtad_npr_fourfermion through
the C ABI) against the FP64 oracle of Eq. (1).

Both sides compute in FP64 from the same links and propagators; they sum the same
terms in different orders, so each output agrees to 1e-12 of the operator's largest
entry (an FP64 sum of 256 products of 3 x 3 matrix products).  Every hypercube of
the small lattices is compared; at 20^3 x 64 a sample of hypercubes is.
"""
import ctypes

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def asq():
    import torch

    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_1411_2223_amd as m

    m.load()
    return m


def random_props(dims, seed, n=4):
    V = int(np.prod(dims))
    rng = np.random.Generator(np.random.PCG64(seed))
    return [rng.standard_normal((V, 3, 3)) + 1j * rng.standard_normal((V, 3, 3)) for _ in range(n)]


def run_gpu(asq, dims, U, G, ops):
    import torch

    V = int(np.prod(dims))
    thin = asq.links_to_device(U.reshape(V, 4, 3, 3))
    props = [asq.links_to_device(g.reshape(V, 1, 3, 3)) for g in G]  # canonical complex128 -> float64 views
    out = asq.npr_fourfermion(dims, thin, props, ops)
    out2 = asq.npr_fourfermion(dims, thin, props, ops)
    torch.cuda.synchronize()
    assert torch.equal(out, out2), "not bitwise reproducible"
    a = out.cpu().numpy().view(np.complex128)
    return a.reshape(len(ops), V // 16, 3, 3, 3, 3)


def compare(got, want, label):
    for k in range(want.shape[0]):
        scale = np.abs(want[k]).max()
        err = np.abs(got[k] - want[k]).max() / scale
        print(f"{label} op {k}: max error {err:.2e} of max |V| {scale:.3e}", flush=True)
        assert err <= TOL


ALL_OPS = [(s1, f1, s2, f2) for s1, f1, s2, f2 in
           np.random.Generator(np.random.PCG64(7)).integers(0, 16, size=(40, 4)).tolist()]


@pytest.mark.parametrize("dims,nops", [((4, 4, 4, 4), 5), ((6, 4, 4, 8), 40), ((2, 4, 6, 4), 23)])
def test_npr_every_hypercube_small(asq, dims, nops):
    # 40 operators take two launches (32 per launch) and two passes of the
    # contraction loop (21 per pass); 23 a ragged second pass
    V = int(np.prod(dims))
    U = synth.thin_links(dims, 0.5, 21) if min(dims) >= 4 else None
    if U is None:  # extents of 2 are outside the thin-link generator: random SU(3) per link
        U = synth.su3_exp(np.random.Generator(np.random.PCG64(21)).standard_normal((V * 4, 8)), 0.5)
    U = U.reshape(V, 4, 3, 3)
    G = random_props(dims, 22)
    ops = ALL_OPS[:nops]
    got = run_gpu(asq, dims, U, G, ops)
    want = oracle.npr_fourfermion(dims, U, G, ops)
    compare(got, want, f"{dims}")


def test_npr_same_propagator_four_times(asq):
    # the four propagator arguments may be one array (one flavour)
    dims = (4, 4, 4, 4)
    V = int(np.prod(dims))
    U = synth.thin_links(dims, 0.3, 23).reshape(V, 4, 3, 3)
    G = random_props(dims, 24, n=1) * 4
    ops = [(0, 0, 0, 0), (15, 15, 15, 15), (5, 10, 5, 10)]
    compare(run_gpu(asq, dims, U, G, ops), oracle.npr_fourfermion(dims, U, G, ops), "one flavour")


def test_npr_full_size_sampled(asq):
    # the paper's 20^3 x 64 lattice shape, 16 operators, sampled hypercubes
    import torch

    w = synth.WORKLOADS["single_20x20x20x64"]
    dims = w["dims"]
    V = int(np.prod(dims))
    U = synth.thin_links(dims, w["eps"], synth.gauge_seed(w["index"])).reshape(V, 4, 3, 3)
    G = random_props(dims, 25, n=2)
    G = [G[0], G[0], G[1], G[1]]
    ops = [(s, 15, s, 15) for s in range(16)]
    thin = asq.links_to_device(U)
    props = [asq.links_to_device(g.reshape(V, 1, 3, 3)) for g in G]
    out = asq.npr_fourfermion(dims, thin, props, ops)
    torch.cuda.synchronize()
    nz = V // 16
    zs = np.unique(np.concatenate([[0, nz - 1], np.random.Generator(np.random.PCG64(26)).integers(0, nz, 14)]))
    got = out.view(len(ops), nz, 162)[:, torch.as_tensor(zs, device=out.device)].cpu().numpy()
    got = got.view(np.complex128).reshape(len(ops), len(zs), 3, 3, 3, 3)
    want = oracle.npr_fourfermion(dims, U, G, ops, zs=zs)
    compare(got, want, "20^3x64 sampled")


def test_npr_rejects_bad_arguments(asq):
    import torch

    dims = (4, 4, 4, 4)
    V = int(np.prod(dims))
    thin = torch.zeros(V * 72, dtype=torch.float64, device="cuda")
    g = torch.zeros(V * 18, dtype=torch.float64, device="cuda")
    out = torch.zeros(V // 16 * 162, dtype=torch.float64, device="cuda")
    d4 = (ctypes.c_int * 4)(*dims)

    def call(ops, o=out, dd=d4, gg=g):
        op = np.ascontiguousarray(np.asarray(ops, dtype=np.int32).reshape(-1, 4))
        return asq.asqtad_npr_fourfermion(dd, thin.data_ptr(), gg.data_ptr(), g.data_ptr(), g.data_ptr(),
                                          g.data_ptr(), op.shape[0], op.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                          o.data_ptr(), None)

    assert call([(16, 0, 0, 0)]) == asq.ASQ_EINVAL
    assert call([(0, -1, 0, 0)]) == asq.ASQ_EINVAL
    assert call([(0, 0, 0, 0)], o=g) == asq.ASQ_EINVAL  # output over a propagator
    assert call([(0, 0, 0, 0)], dd=(ctypes.c_int * 4)(4, 4, 3, 4)) == asq.ASQ_EINVAL
    assert call([(0, 0, 0, 0)], gg=g[1:]) == asq.ASQ_EINVAL  # misaligned
    assert call([(0, 0, 0, 0)]) == asq.ASQ_OK
    torch.cuda.synchronize()
