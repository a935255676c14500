"""Shared helpers of the GPU parity tests (inputs from synth, references from oracle)."""
import functools

import numpy as np

import oracle
import synth

TOL = {"f64": 1e-14, "f32": 1e-6, "f16": 2e-3}


@functools.lru_cache(maxsize=8)
def gauge_arrays(dims, eps, seed):
    fat, lng = synth.make_gauge(dims, eps, seed)
    fat.setflags(write=False)
    lng.setflags(write=False)
    return fat, lng


def quantize_like_device(v, prec):
    """The values the device actually reads for an input given in `prec`."""
    import paper_1411_2223_amd as asq

    if prec == "f64":
        return v
    if prec == "f32":
        return v.real.astype(np.float32).astype(np.float64) + 1j * v.imag.astype(np.float32).astype(np.float64)
    return asq.decode_f16n(asq.encode_f16n(v), v.shape[0], v.shape[1])


def rel_err(a, b):
    """Normwise relative error per column of (nrhs, V/2, 3) arrays."""
    num = np.sqrt(np.sum(np.abs(a - b) ** 2, axis=(1, 2)))
    den = np.sqrt(np.sum(np.abs(b) ** 2, axis=(1, 2)))
    return num / np.where(den > 0, den, 1)


def oracle_dslash_cols(dims, fat, lng, out_parity, v):
    return np.stack([oracle.dslash(dims, fat, lng, out_parity, v[c]) for c in range(v.shape[0])])


def oracle_resid_cols(dims, fat, lng, masses, b, x):
    return np.array([oracle.true_residual(dims, fat, lng, masses[c], b[c], x[c]) for c in range(b.shape[0])])
