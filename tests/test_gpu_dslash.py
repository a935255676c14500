"""GPU parity of the asqtad Dslash (asqtad_dslash_eo through the C ABI) against the FP64 oracle.

Tolerances (normwise relative, per column): FP64 1e-14, FP32 1e-6 (the stated
single-Dslash bound), FP16-with-norm 2e-3.  The oracle sees exactly the input
values the device reads (FP32 rounding / FP16 encoding applied on the host).
"""
import numpy as np
import pytest

import synth
from gpu_common import TOL, gauge_arrays, oracle_dslash_cols, quantize_like_device, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def asq():
    import torch

    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_1411_2223_amd as m

    m.load()
    return m


TIERS = [("f64", 18), ("f32", 18), ("f32", 12), ("f16", 18), ("f16", 12)]


def _gauge(asq, dims, eps, seed, recon):
    fat, lng = gauge_arrays(dims, eps, seed)
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
        print(f"dims={dims} prec={prec} nrhs={nrhs} parity={out_parity} max rel err {err.max():.3e}", flush=True)
        assert err.max() <= TOL[prec]


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
                                             ("f16", 12, 3)])
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
    err = rel_err(asq.vec_from_device(ref_dev, nrhs, half, prec), ref)
    assert err.max() <= TOL[prec]
    for cols, pipe, order in asq.VARIANTS_ALL:
        if cols == 12 and prec == "f64":
            continue  # not built for FP64 vectors; refused in test_unbuilt_variant_rejected
        out = g.dslash(1, vin, prec, nrhs, variant=asq.variant_code(cols, pipe, order))
        torch.cuda.synchronize()
        print(f"prec={prec} recon={recon} variant cols={cols} pipe={pipe} order={order}", flush=True)
        assert torch.equal(out, ref_dev), f"variant ({cols}, {pipe}, {order}) differs from the tuned one"


def test_unbuilt_variant_rejected(asq):
    # codes outside the documented set are refused without launching
    dims = (4, 4, 4, 8)
    g, fat, lng = _gauge(asq, dims, 0.3, 14112223, 18)
    vin = asq.vec_to_device(synth.make_sources(dims, 8, 1), "f64")
    for bad in (3, 16, asq.variant_code(4) | (1 << 14), asq.variant_code(12), asq.variant_code(12, True, 2)):
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
        vin = asq.vec_to_device(v, "f16")
        ref = oracle_dslash_cols(dims, fat, lng, out_parity, quantize_like_device(v, "f16"))
        outs = []
        for order in (0, 1, 2, 3, 0):
            out = g.dslash(out_parity, vin, "f16", nrhs, variant=asq.variant_code_mfma(order))
            torch.cuda.synchronize()
            outs.append(out)
        err = rel_err(asq.vec_from_device(outs[0], nrhs, half, "f16"), ref)
        print(f"mfma dims={dims} nrhs={nrhs} parity={out_parity} max rel err {err.max():.3e}", flush=True)
        assert err.max() <= TOL["f16"]
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
