"""Host-side checks of the C ABI: the library loads, exports every function that
include/asqtad.h declares, and rejects bad arguments before touching the GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1411_2223_amd as asq

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "asqtad.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(asq.LIB_PATH):
        from paper_1411_2223_amd import build

        build.build()
    return asq.load()


def test_exports_match_header(lib):
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(asq.EXPORTS)


def test_strerror(lib):
    for code in (0, 1, -1, -2, -3, -4, -5, -6, -7):
        assert asq.asq_strerror(code)
    assert asq.asq_strerror(-99) == b"unknown error"


def _desc(dims=(4, 4, 4, 8), mask=3, recon=18, fs=9 / 8, ls=-1 / 24):
    return asq.asq_gauge_desc((ctypes.c_int * 4)(*dims), mask, recon, fs, ls)


def test_gauge_bytes(lib):
    d = _desc()
    half = 4 * 4 * 4 * 8 // 2
    n = asq.asq_gauge_bytes(ctypes.byref(d))
    # F64 18-real + F32 18-real copies: 16 slots x half sites x (144 + 72) bytes, then the staging
    # area of the host import (FP64 fat and long links of min(V, 16 MB / 1152 B) sites) and a flag word
    stage = min(2 * half, (16 << 20) // 1152) * 1152
    assert n >= 16 * half * (144 + 72) + stage
    assert n < 16 * half * (144 + 72) + stage + 4096
    d12 = _desc(mask=7, recon=12)
    assert asq.asq_gauge_bytes(ctypes.byref(d12)) >= 16 * half * (144 + 48 + 24)
    for bad in (_desc(dims=(5, 4, 4, 8)), _desc(dims=(2, 4, 4, 8)), _desc(mask=0), _desc(recon=15),
                _desc(mask=7, recon=12, fs=0.0)):
        assert asq.asq_gauge_bytes(ctypes.byref(bad)) == 0


def test_invalid_arguments_rejected_on_host(lib):
    h = ctypes.c_void_p()
    d = _desc(dims=(5, 4, 4, 8))
    assert asq.asq_gauge_create(ctypes.byref(d), 16, 16, 256, 1 << 20, None, ctypes.byref(h)) == asq.ASQ_EINVAL
    d = _desc()
    assert asq.asq_gauge_create(ctypes.byref(d), None, 16, 256, 1 << 20, None, ctypes.byref(h)) == asq.ASQ_EINVAL
    # misaligned storage
    assert asq.asq_gauge_create(ctypes.byref(d), 16, 16, 257, 1 << 20, None, ctypes.byref(h)) == asq.ASQ_EINVAL
    assert asq.asqtad_dslash_eo(None, 0, 0, 1, 16, 16, None) == asq.ASQ_EINVAL
    params = asq.asq_cg_params(1e-10, 100, 0, 0.1, 8, 1)
    stats = (asq.asq_cg_stats * 1)()
    m = (ctypes.c_double * 1)(0.1)
    assert asq.cg_solve_batch(None, 1, m, 16, 16, 256, 1, ctypes.byref(params), stats, None) == asq.ASQ_EINVAL
    assert asq.asq_workspace_bytes(None, 1, 0) == 0
    srv = ctypes.c_void_p()
    assert asq.serve_create(None, 1 << 20, 1, 1, ctypes.byref(srv)) == asq.ASQ_EINVAL
    assert asq.serve_create(256, 1 << 20, 0, 1, ctypes.byref(srv)) == asq.ASQ_EINVAL
    assert asq.serve_submit(None, 0, 1, m, 16, 16, ctypes.byref(params), None, None) == asq.ASQ_EINVAL
    assert asq.asq_gauge_create_device(ctypes.byref(d), None, 16, 256, 1 << 20, None,
                                       ctypes.byref(h)) == asq.ASQ_EINVAL
    # device links must be 16-byte aligned (host links need not be)
    assert asq.asq_gauge_create_device(ctypes.byref(d), 24, 16, 256, 1 << 20, None,
                                       ctypes.byref(h)) == asq.ASQ_EINVAL
    # vectors: precisions, alignment, overlap, a gauge handle
    assert asq.asq_vec_bytes(0, 10) == 480 and asq.asq_vec_bytes(1, 10) == 240 and asq.asq_vec_bytes(2, 10) == 160
    assert asq.asq_vec_bytes(3, 10) == 0
    base = 1 << 24
    assert asq.asq_vec_convert(10, 3, base, 0, base + 4096, None) == asq.ASQ_EINVAL
    assert asq.asq_vec_convert(10, 0, base + 8, 1, base + 4096, None) == asq.ASQ_EINVAL
    assert asq.asq_vec_convert(10, 0, None, 1, base + 4096, None) == asq.ASQ_EINVAL
    assert asq.asq_vec_convert(10, 0, base, 2, base + 256, None) == asq.ASQ_EINVAL  # 480 bytes overlap
    assert asq.asq_vec_convert(0, 0, base, 2, base + 4096, None) == asq.ASQ_OK  # nothing to do
    assert asq.asq_vec_to_native(None, 0, 1, base, base + 4096, None) == asq.ASQ_EINVAL
    assert asq.asq_vec_from_native(None, 0, 1, base, base + 4096, None) == asq.ASQ_EINVAL
    assert asq.serve_poll(None, 1, None, None) == asq.ASQ_EINVAL
    assert asq.asq_copy_probe(16, 16, 15, None) == asq.ASQ_EINVAL
    assert asq.asq_read_probe(16, 15, 16, None) == asq.ASQ_EINVAL
    assert asq.asq_read_probe(None, 16, 16, None) == asq.ASQ_EINVAL
    assert asq.asqtad_dslash_eo_variant(None, 0, 0, 1, 16, 16, 1, None) == asq.ASQ_EINVAL
    assert asq.cg_solve_full(None, 1, m, 16, 16, 256, 1, ctypes.byref(params), stats, None) == asq.ASQ_EINVAL
    assert asq.asq_full_workspace_bytes(None, 1, 0) == 0
    assert asq.cg_solve_multishift(None, 1, 1, m, 16, 16, 256, 1, ctypes.byref(params), stats,
                                   None) == asq.ASQ_EINVAL
    assert asq.asq_multishift_workspace_bytes(None, 1, 1, 0) == 0
    # link construction: every case fails a host check, none reaches a launch
    good = (ctypes.c_int * 4)(4, 4, 4, 4)
    bad = (ctypes.c_int * 4)(5, 4, 4, 4)
    base, step = 1 << 24, 1 << 22  # far apart: a 4^4 link array is 73728 bytes
    assert asq.asqtad_build_links(bad, base, 1.0, base + step, base + 2 * step, None) == asq.ASQ_EINVAL
    assert asq.asqtad_build_links(good, None, 1.0, base + step, base + 2 * step, None) == asq.ASQ_EINVAL
    assert asq.asqtad_build_links(None, base, 1.0, base + step, base + 2 * step, None) == asq.ASQ_EINVAL
    for u0 in (0.0, -1.0, float("nan"), float("inf")):
        assert asq.asqtad_build_links(good, base, u0, base + step, base + 2 * step, None) == asq.ASQ_EINVAL
    assert asq.asqtad_build_links(good, base + 8, 1.0, base + step, base + 2 * step, None) == asq.ASQ_EINVAL
    assert asq.asqtad_build_links(good, base, 1.0, base + 4096, base + 2 * step, None) == asq.ASQ_EINVAL
    assert asq.asqtad_build_links(good, base, 1.0, base + step, base + step + 16, None) == asq.ASQ_EINVAL
    p = ctypes.c_double(0)
    nw = asq.asqtad_plaquette_workspace_bytes(good)
    assert nw >= (256 // 256 + 1) * 8 and asq.asqtad_plaquette_workspace_bytes(bad) == 0
    assert asq.asqtad_plaquette(bad, base, base + step, nw, ctypes.byref(p), None) == asq.ASQ_EINVAL
    assert asq.asqtad_plaquette(good, None, base + step, nw, ctypes.byref(p), None) == asq.ASQ_EINVAL
    assert asq.asqtad_plaquette(good, base, base + step, nw, None, None) == asq.ASQ_EINVAL
    assert asq.asqtad_plaquette(good, base + 8, base + step, nw, ctypes.byref(p), None) == asq.ASQ_EINVAL
    assert asq.asqtad_plaquette(good, base, base + step, nw - 8, ctypes.byref(p), None) == asq.ASQ_ENOMEM
    assert asq.asqtad_plaquette(good, base, base + 4096, nw, ctypes.byref(p), None) == asq.ASQ_EINVAL
    assert asq.asqtad_plaquette(good, base + step, base + step - 64, nw, ctypes.byref(p), None) == asq.ASQ_EINVAL


def test_magic_division_formula():
    # floor(n * (floor(2^64/d) + 1) / 2^64) == n // d for the device's 32-bit site indices
    rng = np.random.default_rng(0)
    for d in list(range(2, 70)) + [96, 100, 128, 1000, 4096, 16383]:
        m = (1 << 64) // d + 1
        ns = list(range(0, 5000)) + [int(v) for v in rng.integers(0, 2**31, 2000)] + [2**31 - 1, 2**32 - 1]
        for n in ns:
            assert (n * m) >> 64 == n // d


def test_reference_f16n_encoder_follows_its_definition():
    """The tests' own FP16-with-norm encoder (the reference the library's encoder is held to,
    bit for bit on the GPU):
    the norm is the largest magnitude, the largest component encodes as +-1 exactly, values
    that are binary16 multiples of the norm survive unchanged, and the rounding error of the
    others is at most half a binary16 unit of [1/2, 1) times the norm (2^-12 nu)."""
    from gpu_common import f16n_encode, f16n_value

    rng = np.random.default_rng(1)
    v = rng.standard_normal((2, 50, 3)) + 1j * rng.standard_normal((2, 50, 3))
    h, nu = f16n_encode(v)
    comp = np.stack([v.real, v.imag], -1).astype(np.float32)
    assert np.array_equal(nu, np.abs(comp).reshape(2, 50, 6).max(-1))
    assert np.all(np.abs(h.astype(np.float32)).reshape(2, 50, 6).max(-1) == 1.0)
    w = f16n_value(h, nu)
    err = np.abs(np.stack([(w - v).real, (w - v).imag], -1)).reshape(2, 50, 6).max(-1) / nu
    # |h| < 1 rounds within half a unit of [1/2, 1): 2^-12
    assert err.max() <= 2 ** -12 * (1 + 1e-6) + 2 ** -24
    # exact cases: a site of powers of two times a common scale, and a zero site
    e = np.zeros((1, 2, 3), dtype=np.complex128)
    e[0, 0] = np.array([3.0 + 0.75j, -1.5 - 0.375j, 0.1875 + 3.0j])
    he, ne = f16n_encode(e)
    assert ne[0, 0] == 3.0 and ne[0, 1] == 0.0
    assert np.array_equal(f16n_value(he, ne), e)


def test_build_links_binding_checks_shapes(lib):
    """The binding refuses tensors of the wrong size or type before calling the library."""
    import torch

    dims = (4, 4, 4, 4)
    n = 256 * 4 * 18
    with pytest.raises(asq.AsqError):
        asq.build_links(dims, torch.zeros(n - 1, dtype=torch.float64))
    with pytest.raises(asq.AsqError):
        asq.build_links(dims, torch.zeros(n, dtype=torch.float32))
    with pytest.raises(asq.AsqError):
        asq.build_links(dims, torch.zeros(n, dtype=torch.float64), fat=torch.zeros(n + 1, dtype=torch.float64),
                        lng=torch.zeros(n, dtype=torch.float64))


def test_gauge_rejects_malformed_device_links(lib):
    """A tensor passed as links must hold V*4*18 float64 values on the GPU; checked before any call."""
    import torch

    dims = (4, 4, 4, 4)
    bad = torch.zeros(256 * 4 * 18 - 2, dtype=torch.float64)
    with pytest.raises(asq.AsqError):
        asq.Gauge(dims, bad, bad, device="cpu")
