"""Shared helpers of the GPU parity tests (inputs from synth, references from oracle)."""
import functools

import numpy as np

import oracle
import synth

# Normwise relative error per column.  FP16-with-norm: the output is stored in that
# tier, so each real carries at most half a binary16 unit of its site's norm,
# 2^-12 nu (the inputs are quantized identically on both sides); with nu^2 at most
# the site's |psi|^2 summed over six reals that bounds the normwise error by
# sqrt(6) 2^-12 = 5.98e-4, plus FP32 arithmetic.
TOL = {"f64": 1e-14, "f32": 1e-6, "f16": 6.1e-4}
# Largest elementwise (complex) error relative to the column's largest |entry|: FP32
# rounding of sixteen 3x3 products (a few 2^-24 per product), and for FP16 the 2^-12 nu
# bound above on each of the real and imaginary parts, so sqrt(2) 2^-12 = 3.45e-4 on
# their modulus (nu, the site's largest real, is at most the column's largest modulus).
MAX_TOL = {"f64": 1e-13, "f32": 1e-5, "f16": 3.5e-4}


@functools.lru_cache(maxsize=8)
def gauge_arrays(dims, eps, seed):
    fat, lng = synth.make_gauge(dims, eps, seed)
    fat.setflags(write=False)
    lng.setflags(write=False)
    return fat, lng


def f16n_encode(v):
    """FP16-with-norm encoding written for the tests from its definition, independent of
    the library: per site and column the six reals rounded to float32, nu = their largest
    magnitude (float32), r = 1/nu correctly rounded to float32, and each real times r
    rounded once to IEEE binary16 (nearest, ties to even): the product is exact in float64
    (two 24-bit significands) and float64 -> float16 is a single rounding.  Returns (halves
    (nrhs, V/2, 3, 2) float16, nu (nrhs, V/2) float32): the canonical layout is the halves
    followed by the norms."""
    v = np.asarray(v, dtype=np.complex128)
    comp = np.stack([v.real, v.imag], axis=-1).astype(np.float32)  # (nrhs, half, 3, 2)
    nu = np.abs(comp).reshape(comp.shape[:2] + (6,)).max(axis=-1)
    with np.errstate(divide="ignore"):
        inv = np.where(nu > 0, np.float32(1.0) / nu, np.float32(0.0)).astype(np.float32)
    exact = comp.astype(np.float64) * inv.astype(np.float64)[..., None, None]
    h = exact.astype(np.float16)
    return h, nu


def f16n_value(h, nu):
    """The exact value an FP16-with-norm record represents: nu * h, complex (nrhs, V/2, 3)."""
    w = h.astype(np.float64) * nu.astype(np.float64)[..., None, None]
    return w[..., 0] + 1j * w[..., 1]


def f16n_bytes(h, nu):
    """Canonical FP16-with-norm buffer: every column's binary16 values, then every norm."""
    return np.concatenate([np.ascontiguousarray(h).view(np.uint8).reshape(-1),
                           np.ascontiguousarray(nu, dtype=np.float32).view(np.uint8).reshape(-1)])


def quantize_like_device(v, prec):
    """The values the device actually reads for an input given in `prec`."""
    if prec == "f64":
        return v
    if prec == "f32":
        return v.real.astype(np.float32).astype(np.float64) + 1j * v.imag.astype(np.float32).astype(np.float64)
    return f16n_value(*f16n_encode(v))


def max_err(a, b):
    """Largest elementwise error per column, relative to the column's largest |b| entry."""
    num = np.abs(a - b).reshape(a.shape[0], -1).max(axis=1)
    den = np.abs(b).reshape(b.shape[0], -1).max(axis=1)
    return num / np.where(den > 0, den, 1)


def rel_err(a, b):
    """Normwise relative error per column of (nrhs, V/2, 3) arrays."""
    num = np.sqrt(np.sum(np.abs(a - b) ** 2, axis=(1, 2)))
    den = np.sqrt(np.sum(np.abs(b) ** 2, axis=(1, 2)))
    return num / np.where(den > 0, den, 1)


def oracle_dslash_cols(dims, fat, lng, out_parity, v):
    return np.stack([oracle.dslash(dims, fat, lng, out_parity, v[c]) for c in range(v.shape[0])])


def oracle_resid_cols(dims, fat, lng, masses, b, x):
    return np.array([oracle.true_residual(dims, fat, lng, masses[c], b[c], x[c]) for c in range(b.shape[0])])
