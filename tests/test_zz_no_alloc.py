"""The allocation-free mean plaquette (asqtad_plaquette_noalloc through the C ABI):
its partial sums live in the library's fixed device array instead of a caller
workspace, so it must give exactly the bits of asqtad_plaquette, call after call,
also when a later call covers a smaller lattice than the one before (the array
keeps the earlier call's contents)."""
import ctypes

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def asq():
    import torch

    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_1411_2223_amd as m

    m.load()
    return m


def _fn(asq):
    return asq.asqtad_plaquette_noalloc


def _noalloc(asq, dims, thin, out):
    rc = _fn(asq)((ctypes.c_int * 4)(*dims), thin.data_ptr(), out.data_ptr(), asq.stream_ptr(None))
    asq.check(rc, "asqtad_plaquette_noalloc")


def test_noalloc_plaquette_matches_workspace_form(asq):
    import torch

    # a larger lattice first, then a smaller one: the second call must not see the
    # first call's partials left in the shared array
    cases = [((8, 8, 8, 16), 0.3, 31), ((6, 4, 4, 8), 0.5, 32), ((8, 8, 8, 16), 0.3, 31)]
    out = torch.full((4,), float("nan"), dtype=torch.float64, device="cuda")
    for k, (dims, eps, seed) in enumerate(cases):
        V = int(np.prod(dims))
        U = synth.thin_links(dims, eps, seed).reshape(V, 4, 3, 3)
        thin = asq.links_to_device(U)
        ref = asq.plaquette(dims, thin)  # the workspace form, through the C ABI
        _noalloc(asq, dims, thin, out[k:])
        torch.cuda.synchronize()
        got = float(out[k].item())
        print(f"noalloc plaquette {dims}: {got!r} vs {ref!r}", flush=True)
        assert got == ref
    # the refusals: a lattice beyond the fixed array, and an output inside the links
    # (both refused on the host, before any launch)
    f = _fn(asq)
    assert f((ctypes.c_int * 4)(64, 64, 128, 256), 1 << 24, out.data_ptr(), None) == asq.ASQ_ENOMEM
    thin = asq.links_to_device(synth.thin_links((4, 4, 4, 4), 0.3, 1).reshape(256, 4, 3, 3))
    assert f((ctypes.c_int * 4)(4, 4, 4, 4), thin.data_ptr(), thin.data_ptr() + 64, None) == asq.ASQ_EINVAL
