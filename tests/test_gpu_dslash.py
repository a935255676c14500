"""GPU parity of the asqtad Dslash (asqtad_dslash_eo through the C ABI) against the FP64 oracle.

Tolerances per column: normwise relative FP64 1e-14, FP32 1e-6 (the stated
single-Dslash bound), FP16-with-norm 6.1e-4 (sqrt(6) 2^-12, from storing the output
in that tier), and the largest elementwise error relative to the column's largest
entry (gpu_common.MAX_TOL: sqrt(2) 2^-12 for FP16).  The oracle sees exactly the input values the device
reads: FP32 rounding, and the tests' own FP16-with-norm encoder, which the library's
encoder (asq_vec_convert) matches bit for bit.  Vectors cross the C ABI in the
canonical layout; the native-layout kernels the solvers launch are covered through
asq_vec_to_native / asq_vec_from_native.
"""
import numpy as np
import pytest

import synth
from gpu_common import (MAX_TOL, TOL, f16n_bytes, f16n_encode, gauge_arrays, max_err, oracle_dslash_cols,
                        quantize_like_device, rel_err)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def asq():
    import torch

    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_1411_2223_amd as m

    m.load()
    return m


# (vector tier, links): 18 / 12 reals, or 64: a field kept in FP64 only, whose FP32 and
# FP16 Dslash read the FP64 links and round them to FP32 on load
TIERS = [("f64", 18), ("f32", 18), ("f32", 12), ("f16", 18), ("f16", 12), ("f32", 64), ("f16", 64)]


def _gauge(asq, dims, eps, seed, recon):
    fat, lng = gauge_arrays(dims, eps, seed)
    if recon == 64:
        return asq.Gauge(dims, fat, lng, precs=("f64",), recon=18), fat, lng
    precs = ("f64", "f32", "f16") if recon == 12 else ("f64", "f32")
    return asq.Gauge(dims, fat, lng, precs=precs, recon=recon), fat, lng


def _check(asq, g, fat, lng, dims, prec, nrhs, seed):
    import torch

    half = int(np.prod(dims)) // 2
    for out_parity in (0, 1):
        v = synth.make_sources(dims, nrhs, seed + out_parity)
        vq = quantize_like_device(v, prec)
        vin = asq.vec_to_device(v, prec)
        # consecutive calls walk the lattice in opposite directions: the same bits either way
        out = g.dslash(out_parity, vin, prec, nrhs)
        out2 = g.dslash(out_parity, vin, prec, nrhs)
        torch.cuda.synchronize()
        assert torch.equal(out, out2), "Dslash is not bitwise reproducible"
        got = asq.vec_from_device(out, nrhs, half, prec)
        ref = oracle_dslash_cols(dims, fat, lng, out_parity, vq)
        err = rel_err(got, ref)
        emax = max_err(got, ref)
        print(f"dims={dims} prec={prec} nrhs={nrhs} parity={out_parity} max rel err {err.max():.3e} "
              f"max elementwise {emax.max():.3e}", flush=True)
        assert err.max() <= TOL[prec]
        assert emax.max() <= MAX_TOL[prec]


@pytest.mark.parametrize("prec,recon", TIERS)
@pytest.mark.parametrize("dims,eps,seed", [((4, 4, 4, 8), 0.3, 14112223), ((6, 4, 8, 10), 0.3, 5),
                                           ((8, 6, 4, 12), 0.2, 6)])
@pytest.mark.parametrize("nrhs", [1, 3, 5, 9])
def test_dslash_parity_small(asq, dims, eps, seed, prec, recon, nrhs):
    if prec == "f64" and recon == 12:
        pytest.skip("FP64 links are always 18-real")
    g, fat, lng = _gauge(asq, dims, eps, seed, recon)
    _check(asq, g, fat, lng, dims, prec, nrhs, 100 + nrhs)


@pytest.mark.parametrize("prec,recon,nrhs", [("f64", 18, 1), ("f32", 18, 1), ("f32", 12, 2), ("f16", 18, 4),
                                             ("f16", 12, 3), ("f32", 64, 1)])
def test_dslash_parity_full_size(asq, prec, recon, nrhs):
    # the paper's 20^3 x 64 lattice shape, every output site compared
    dims = (20, 20, 20, 64)
    g, fat, lng = _gauge(asq, dims, 0.3, synth.gauge_seed(1), recon)
    _check(asq, g, fat, lng, dims, prec, nrhs, 7)


@pytest.mark.parametrize("prec,recon", TIERS)
def test_every_launch_variant(asq, prec, recon):
    # Every column-tile width, hop-loop form and block order computes each column
    # with the same arithmetic in the same order: bitwise equal outputs, and the
    # oracle's tolerance.  13 columns leave a partial tile, 960 output sites a
    # ragged last block and a short last group of site blocks.
    import torch

    if prec == "f64" and recon == 12:
        pytest.skip("FP64 links are always 18-real")
    dims, nrhs = (6, 4, 8, 10), 13
    g, fat, lng = _gauge(asq, dims, 0.3, 5, recon)
    half = int(np.prod(dims)) // 2
    v = synth.make_sources(dims, nrhs, 77)
    vin = asq.vec_to_device(v, prec)
    ref_dev = g.dslash(1, vin, prec, nrhs)
    torch.cuda.synchronize()
    ref = oracle_dslash_cols(dims, fat, lng, 1, quantize_like_device(v, prec))
    got = asq.vec_from_device(ref_dev, nrhs, half, prec)
    assert rel_err(got, ref).max() <= TOL[prec]
    assert max_err(got, ref).max() <= MAX_TOL[prec]
    # the same input in the solvers' native layout
    vin_n = g.to_native(vin, prec, nrhs)
    for cols, pipe, order, sweep, chunk in asq.VARIANTS_ALL:
        if cols == 12 and prec == "f64":
            continue  # not built for FP64 vectors; refused in test_unbuilt_variant_rejected
        out = g.dslash(1, vin, prec, nrhs, variant=asq.variant_code(cols, pipe, order, sweep=sweep, chunk=chunk))
        out_n = g.dslash(1, vin_n, prec, nrhs,
                         variant=asq.variant_code(cols, pipe, order, native=True, sweep=sweep, chunk=chunk))
        back = g.from_native(out_n, prec, nrhs)
        torch.cuda.synchronize()
        v = (cols, pipe, order, sweep, chunk)
        print(f"prec={prec} recon={recon} variant {v}", flush=True)
        assert torch.equal(out, ref_dev), f"variant {v} differs from the tuned one"
        assert torch.equal(back, ref_dev), f"native variant {v} differs from canonical"


@pytest.mark.parametrize("prec", ["f32", "f16"])
def test_sweep_in_runs_of_blocks_matches_slab_order(asq, prec):
    """At 20^3 x 64 (1000 site blocks) with 8 columns, sweeps in which each XCD takes runs
    of 16, 64 or 256 blocks cover several whole groups of 8 runs and a ragged tail: every
    block order must give the bits of the slab order."""
    import torch

    dims = (20, 20, 20, 64)
    g, fat, lng = _gauge(asq, dims, 0.3, 5, 18)
    nrhs = 8
    vin_n = g.to_native(asq.vec_to_device(synth.make_sources(dims, nrhs, 79), prec), prec, nrhs)
    for cols in (1, 4, 8):
        for order in (0, 1):
            ref = g.dslash(1, vin_n, prec, nrhs, variant=asq.variant_code(cols, True, order, native=True))
            for chunk in (0, 1, 2, 3):
                got = g.dslash(1, vin_n, prec, nrhs,
                               variant=asq.variant_code(cols, True, order, native=True, sweep=True, chunk=chunk))
                torch.cuda.synchronize()
                print(f"sweep prec={prec} cols={cols} order={order} chunk={chunk}", flush=True)
                assert torch.equal(got, ref), f"sweep in runs differs: cols={cols} order={order} chunk={chunk}"


@pytest.mark.parametrize("prec,recon", [("f32", 18), ("f32", 12), ("f16", 12), ("f16", 18)])
def test_streamed_links_match(asq, prec, recon):
    """One-column launches that read their links with non-temporal loads (FP32 18- and
    12-real, 16-bit 12-real tiers) give the bits of ordinary loads, in every sweep form."""
    import torch

    dims = (20, 20, 20, 64)
    g, fat, lng = _gauge(asq, dims, 0.3, 5, recon)
    vin_n = g.to_native(asq.vec_to_device(synth.make_sources(dims, 1, 80), prec), prec, 1)
    for pipe in (False, True):
        for sweep, chunk in ((False, 0), (True, 0), (True, 2)):
            ref = g.dslash(1, vin_n, prec, 1, variant=asq.variant_code(1, pipe, 0, native=True, sweep=sweep,
                                                                        chunk=chunk))
            got = g.dslash(1, vin_n, prec, 1, variant=asq.variant_code(1, pipe, 0, native=True, sweep=sweep,
                                                                        chunk=chunk, stream=True))
            torch.cuda.synchronize()
            print(f"streamed links prec={prec} recon={recon} pipe={pipe} sweep={sweep} chunk={chunk}", flush=True)
            assert torch.equal(got, ref)
    # wider tiles and the FP64-stored tiers have no streamed form
    with pytest.raises(asq.AsqError):
        g.dslash(1, vin_n, prec, 1, variant=asq.variant_code(2, True, 0, native=True, stream=True))


@pytest.mark.parametrize("prec,recon", [("f64", 18), ("f32", 18), ("f32", 12), ("f16", 12), ("f16", 18), ("f32", 64)])
def test_lds_window_matches(asq, prec, recon):
    """Launches whose blocks stage the input records within three y-rows of their sites in
    LDS (x hops and non-wrapping y hops read there) give the bits of the plain kernel: one
    column on lattices whose window covers the whole parity (4^3x8), whose blocks are
    ragged and whose y hops wrap (6x4x8x10, 20^3x64), both parities, every sweep form,
    with ordinary and, where the tier has them, streamed links; and every column tile."""
    import torch

    for dims in ((4, 4, 4, 8), (6, 4, 8, 10), (20, 20, 20, 64)):
        g, fat, lng = _gauge(asq, dims, 0.3, 5, recon)
        vin = g.to_native(asq.vec_to_device(synth.make_sources(dims, 1, 82), prec), prec, 1)
        streams = (False,) if prec == "f64" or recon == 64 else (False, True)
        for parity in (0, 1):
            for sweep, chunk in ((False, 0), (True, 0), (True, 2)):
                kw = dict(native=True, sweep=sweep, chunk=chunk)
                ref = g.dslash(parity, vin, prec, 1, variant=asq.variant_code(1, True, 0, **kw))
                for st in streams:
                    got = g.dslash(parity, vin, prec, 1, variant=asq.variant_code(1, True, 0, stream=st, lds=True, **kw))
                    torch.cuda.synchronize()
                    print(f"lds window dims={dims} prec={prec} recon={recon} parity={parity} sweep={sweep} "
                          f"chunk={chunk} stream={st}", flush=True)
                    assert torch.equal(got, ref)
        g.close()
    # column tiles with the window: a 13-column batch (ragged last tile) in every tile
    # width, both block orders, slabs and sweeps
    dims = (6, 4, 8, 10)
    g, fat, lng = _gauge(asq, dims, 0.3, 5, recon)
    nrhs = 13
    vn = g.to_native(asq.vec_to_device(synth.make_sources(dims, nrhs, 83), prec), prec, nrhs)
    site_bytes = {"f64": 48, "f32": 24, "f16": 16}[prec]
    for cols in (2, 4, 6, 8, 12):
        if cols == 12 and prec == "f64":
            continue
        too_big = cols * (256 + 6 * (dims[0] // 2)) * site_bytes > 65536  # the window's LDS limit
        for order in (0, 1):
            for sweep, chunk in ((False, 0), (True, 1)):
                kw = dict(native=True, sweep=sweep, chunk=chunk)
                ref = g.dslash(1, vn, prec, nrhs, variant=asq.variant_code(cols, True, order, **kw))
                if too_big:
                    with pytest.raises(asq.AsqError):
                        g.dslash(1, vn, prec, nrhs, variant=asq.variant_code(cols, True, order, lds=True, **kw))
                    continue
                got = g.dslash(1, vn, prec, nrhs, variant=asq.variant_code(cols, True, order, lds=True, **kw))
                torch.cuda.synchronize()
                print(f"lds window prec={prec} recon={recon} cols={cols} order={order} sweep={sweep}", flush=True)
                assert torch.equal(got, ref)
    # no LDS form: the plain loop, streamed links beyond one column, the canonical layout
    v4 = g.to_native(asq.vec_to_device(synth.make_sources(dims, 4, 82), prec), prec, 4)
    vc = asq.vec_to_device(synth.make_sources(dims, 1, 82), prec)
    for v, n, code in ((v4, 4, asq.variant_code(4, False, 0, native=True, lds=True)),
                       (v4, 4, asq.variant_code(4, True, 0, native=True, stream=True, lds=True)),
                       (v4, 1, asq.variant_code(1, False, 0, native=True, lds=True)),
                       (vc, 1, asq.variant_code(1, True, 0, lds=True))):
        with pytest.raises(asq.AsqError):
            g.dslash(1, v, prec, n, variant=code)


def test_unbuilt_variant_rejected(asq):
    # codes outside the documented set are refused without launching
    dims = (4, 4, 4, 8)
    g, fat, lng = _gauge(asq, dims, 0.3, 14112223, 18)
    vin = asq.vec_to_device(synth.make_sources(dims, 8, 1), "f64")
    for bad in (3, 16, asq.variant_code(4) | (1 << 14), asq.variant_code(4) | (1 << 10), asq.variant_code(12),
                asq.variant_code(12, True, 2)):
        with pytest.raises(asq.AsqError) as e:
            g.dslash(1, vin, "f64", 8, variant=bad)
        assert e.value.code == asq.ASQ_EINVAL


def test_free_field_plane_wave_on_gpu(asq):
    # U = 1: D_eo D_oe on an even plane wave is -4 sum f(p)^2 (closed form, no oracle involved)
    import torch

    dims = (8, 4, 6, 10)
    fat, lng = synth.fat_long_from_thin(synth.unit_links(dims))
    g = asq.Gauge(dims, fat, lng, precs=("f64",), recon=18)
    X, Y, Z, T = dims
    lex = np.arange(np.prod(dims))
    c = np.stack([lex % X, (lex // X) % Y, (lex // (X * Y)) % Z, lex // (X * Y * Z)], 1)
    ev = c[c.sum(1) % 2 == 0]
    p = np.array([2 * np.pi * 3 / X, 2 * np.pi / Y, 2 * np.pi * 2 / Z, 5 * np.pi / T])
    f = 9 / 8 * np.sin(p) - 1 / 24 * np.sin(3 * p)
    v = (np.exp(1j * ev @ p)[:, None] * np.array([1.0, -0.5j, 0.25])[None, :])[None]
    vin = asq.vec_to_device(v, "f64")
    t = g.dslash(1, vin, "f64")
    w = g.dslash(0, t, "f64")
    torch.cuda.synchronize()
    got = asq.vec_from_device(w, 1, ev.shape[0], "f64")
    assert np.max(np.abs(got + 4 * np.sum(f**2) * v)) < 1e-12


def test_non_su3_links_rejected_for_compression(asq):
    dims = (4, 4, 4, 8)
    rng = np.random.default_rng(0)
    V = int(np.prod(dims))
    fat = rng.standard_normal((V, 4, 3, 3)) + 1j * rng.standard_normal((V, 4, 3, 3))
    with pytest.raises(asq.AsqError) as e:
        asq.Gauge(dims, fat, fat, precs=("f64", "f32"), recon=12)
    assert e.value.code == asq.ASQ_ENOTSU3
    # 18-real tiers take any links
    asq.Gauge(dims, fat, fat, precs=("f64", "f32"), recon=18)


@pytest.mark.parametrize("dims,nrhs", [((6, 4, 8, 10), 13), ((4, 4, 4, 8), 40), ((8, 6, 4, 12), 70)])
def test_mfma_variant(asq, dims, nrhs):
    # The matrix-core form (FP32 18-real links, FP16 vectors): the oracle's FP16
    # tolerance for both parities, bitwise reproducible, every block order equal.
    # 13 and 40 columns leave idle lanes in a 32-column tile; 960 and 1152 output
    # sites a ragged last block.
    import torch

    g, fat, lng = _gauge(asq, dims, 0.3, 5, 18)
    half = int(np.prod(dims)) // 2
    for out_parity in (0, 1):
        v = synth.make_sources(dims, nrhs, 81 + out_parity)
        vin = g.to_native(asq.vec_to_device(v, "f16"), "f16", nrhs)
        ref = oracle_dslash_cols(dims, fat, lng, out_parity, quantize_like_device(v, "f16"))
        outs = []
        for order in (0, 1, 2, 3, 0):
            out = g.dslash(out_parity, vin, "f16", nrhs, variant=asq.variant_code_mfma(order))
            torch.cuda.synchronize()
            outs.append(out)
        got = asq.vec_from_device(g.from_native(outs[0], "f16", nrhs), nrhs, half, "f16")
        err = rel_err(got, ref)
        print(f"mfma dims={dims} nrhs={nrhs} parity={out_parity} max rel err {err.max():.3e}", flush=True)
        assert err.max() <= TOL["f16"]
        assert max_err(got, ref).max() <= MAX_TOL["f16"]
        assert all(torch.equal(outs[0], o) for o in outs[1:])


def test_mfma_variant_only_for_its_tier(asq):
    # FP32 vectors, 12-real links and FP64 refuse the matrix-core code without launching
    dims = (4, 4, 4, 8)
    for prec, recon in (("f32", 18), ("f64", 18), ("f16", 12)):
        g, fat, lng = _gauge(asq, dims, 0.3, 14112223, recon)
        vin = asq.vec_to_device(synth.make_sources(dims, 8, 2), prec)
        with pytest.raises(asq.AsqError) as e:
            g.dslash(1, vin, prec, 8, variant=asq.variant_code_mfma(0))
        assert e.value.code == asq.ASQ_EINVAL
    # and the canonical layout refuses it for every tier
    g, fat, lng = _gauge(asq, dims, 0.3, 14112223, 18)
    vin = asq.vec_to_device(synth.make_sources(dims, 8, 2), "f16")
    with pytest.raises(asq.AsqError) as e:
        g.dslash(1, vin, "f16", 8, variant=asq.variant_code_mfma(0) & ~asq.ASQ_VARIANT_NATIVE)
    assert e.value.code == asq.ASQ_EINVAL


def _special_sources(nrhs, half, seed):
    """Random sites plus the cases an FP16-with-norm encoder can get wrong: an all-zero site,
    tiny and huge magnitudes, negative maxima, halfway cases of binary16 rounding."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((nrhs, half, 3)) + 1j * rng.standard_normal((nrhs, half, 3))
    v[0, 0] = 0
    v[0, 1] *= 1e-30
    v[0, 2] *= 1e30
    v[0, 3] = np.array([-4.0, 1.0 + 1j, 0.5j])
    # 1 + 2^-11 is a tie between two binary16 values after scaling by 1/nu = 1/2
    v[0, 4] = np.array([2.0, 1.0 + 2.0 ** -11, (1.0 + 3 * 2.0 ** -11) * 1j])
    v[0, 5] = np.array([2.0 ** -20, -(2.0 ** -21), 2.0 ** -40 + 0j])
    return v


def test_library_f16n_encoding_matches_reference_encoder(asq):
    # asq_vec_convert FP64 -> FP16-with-norm against the tests' own encoder, bit for bit,
    # and FP16 -> FP64 gives back exactly nu * h; FP64 -> FP32 rounds to nearest.
    import torch

    nrhs, half = 3, 1000
    v = _special_sources(nrhs, half, 5)
    dev = asq.vec_to_device(v, "f64")
    enc = asq.vec_convert(dev, nrhs * half, "f64", "f16")
    torch.cuda.synchronize()
    want = f16n_bytes(*f16n_encode(v))
    got = enc.cpu().numpy().view(np.uint8)[: want.size]
    bad = np.nonzero(got != want)[0]
    if bad.size:
        n = nrhs * half
        recs = sorted({int(i) // 12 if i < 12 * n else int(i - 12 * n) // 4 for i in bad})[:8]
        gh, wh = got[: 12 * n].view(np.float16).reshape(n, 6), want[: 12 * n].view(np.float16).reshape(n, 6)
        gn, wn = got[12 * n:].view(np.float32), want[12 * n:].view(np.float32)
        detail = [(r, v.reshape(n, 3)[r].tolist(), gh[r].tolist(), wh[r].tolist(), float(gn[r]), float(wn[r]))
                  for r in recs]
        raise AssertionError(f"{bad.size} bytes differ; (record, value, library halves, reference halves, "
                             f"library norm, reference norm): {detail}")
    back = asq.vec_from_device(enc, nrhs, half, "f16")
    assert np.array_equal(back, quantize_like_device(v, "f16"))
    f32 = asq.vec_convert(dev, nrhs * half, "f64", "f32")
    torch.cuda.synchronize()
    w32 = np.stack([v.real, v.imag], -1).astype(np.float32).reshape(-1)
    assert np.array_equal(f32.cpu().numpy(), w32)
    # FP32 -> FP16 encodes the same as FP64 -> FP16 (the encoder rounds to FP32 first)
    enc2 = asq.vec_convert(f32, nrhs * half, "f32", "f16")
    torch.cuda.synchronize()
    assert torch.equal(enc2, enc)


@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
def test_native_relayout_roundtrip(asq, prec):
    # canonical -> native -> canonical is the identity, and the native layout is the
    # solvers' site-fastest one (checked for FP64: colour-major structure of arrays)
    import torch

    dims, nrhs = (6, 4, 8, 10), 5
    g, fat, lng = _gauge(asq, dims, 0.3, 5, 18)
    half = g.half
    v = _special_sources(nrhs, half, 6)
    c = asq.vec_to_device(v, prec)
    n = g.to_native(c, prec, nrhs)
    back = g.from_native(n, prec, nrhs)
    torch.cuda.synchronize()
    assert torch.equal(back, c)
    if prec == "f64":
        nat = n.cpu().numpy().reshape(nrhs, 3, half, 2)
        assert np.array_equal(nat[..., 0] + 1j * nat[..., 1], v.transpose(0, 2, 1))
