"""Seeded synthetic inputs for the even-odd asqtad CG workload.

This module builds inputs only: random SU(3) thin links, the fat and long
links that the workload recipe derives from them, Gaussian sources, random
SU(3) gauge transformations and the Poisson request trace of the serving
workload.  It holds none of the operator or solver arithmetic (no staggered
phases, no boundary signs, no Dslash, no CG); both the CPU oracle and the
GPU library receive its arrays as plain inputs.

Canonical host layout (shared by every consumer):

* lexicographic site index  lex = x + X*(y + Y*(z + Z*t))
* parity (x+y+z+t) % 2, even = 0; checkerboard index of a site = lex // 2
* links: complex128 array (V, 4, 3, 3) indexed [lex, mu, row, col],
  mu = 0..3 for x, y, z, t; U_mu(x) multiplies the colour vector at x+mu
* colour vectors of one parity: complex128 (nrhs, V/2, 3) in checkerboard order

Recipe (the paper's lattices are MILC asqtad ensembles that are not
available; these fields have the same shapes): thin links
U = exp(i*eps*H) with H = sum_a h_a lambda_a / 2, h_a ~ N(0,1) drawn from
numpy's PCG64 in the C order of shape (T, Z, Y, X, 4, 8); fat = (9/8) U;
long_mu(x) = (-1/24) U_mu(x) U_mu(x+mu) U_mu(x+2mu), periodic wrap (the time
boundary sign belongs to the operator, not to the links).
"""
from __future__ import annotations

import numpy as np

FAT_COEFF = 9.0 / 8.0
LONG_COEFF = -1.0 / 24.0
BASE_SEED = 14112223


def gell_mann() -> np.ndarray:
    """The eight Gell-Mann matrices, shape (8, 3, 3), tr(l_a l_b) = 2 delta_ab."""
    lam = np.zeros((8, 3, 3), dtype=np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1] = -1j
    lam[1][1, 0] = 1j
    lam[2][0, 0] = 1
    lam[2][1, 1] = -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2] = -1j
    lam[4][2, 0] = 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2] = -1j
    lam[6][2, 1] = 1j
    lam[7][0, 0] = lam[7][1, 1] = 1 / np.sqrt(3)
    lam[7][2, 2] = -2 / np.sqrt(3)
    return lam


def su3_exp(h: np.ndarray, eps: float) -> np.ndarray:
    """exp(i*eps*H), H = sum_a h[..., a] lambda_a / 2, by Hermitian eigendecomposition."""
    lam = gell_mann()
    H = np.einsum("...a,aij->...ij", h, lam) * 0.5
    w, v = np.linalg.eigh(H)
    ph = np.exp(1j * eps * w)
    return np.einsum("...ij,...j,...kj->...ik", v, ph, v.conj())


def volume(dims) -> int:
    X, Y, Z, T = dims
    return X * Y * Z * T


def check_dims(dims) -> None:
    if len(dims) != 4 or any(int(d) != d or d < 4 or d % 2 for d in dims):
        raise ValueError(f"lattice extents must be four even integers >= 4, got {dims}")


def thin_links(dims, eps: float, seed: int) -> np.ndarray:
    """Random SU(3) thin links, complex128 (T, Z, Y, X, 4, 3, 3).

    The normals are drawn one time slice at a time; the stream is the same as
    one draw of shape (T, Z, Y, X, 4, 8) and keeps peak memory to one slice.
    """
    check_dims(dims)
    X, Y, Z, T = dims
    rng = np.random.Generator(np.random.PCG64(seed))
    U = np.empty((T, Z, Y, X, 4, 3, 3), dtype=np.complex128)
    for t in range(T):
        h = rng.standard_normal((Z, Y, X, 4, 8))
        U[t] = su3_exp(h, eps)
    return U


def _roll_mu(A: np.ndarray, shift: int, mu: int) -> np.ndarray:
    """A(x + shift*mu) for arrays shaped (T, Z, Y, X, ...), periodic."""
    axis = 3 - mu
    return np.roll(A, -shift, axis=axis)


def fat_long_from_thin(U: np.ndarray):
    """Workload recipe: fat = (9/8) U, long = (-1/24) U(x)U(x+mu)U(x+2mu).

    Returns (fat, long) as complex128 (V, 4, 3, 3) in lexicographic order.
    """
    T, Z, Y, X = U.shape[:4]
    fat = (FAT_COEFF * U).reshape(T * Z * Y * X, 4, 3, 3)
    lng = np.empty_like(U)
    for mu in range(4):
        U1 = U[..., mu, :, :]
        U2 = _roll_mu(U1, 1, mu)
        U3 = _roll_mu(U1, 2, mu)
        lng[..., mu, :, :] = LONG_COEFF * (U1 @ U2 @ U3)
    return np.ascontiguousarray(fat), np.ascontiguousarray(lng.reshape(T * Z * Y * X, 4, 3, 3))


def make_gauge(dims, eps: float, seed: int):
    """(fat, long) complex128 (V, 4, 3, 3) for the given lattice, roughness and seed."""
    return fat_long_from_thin(thin_links(dims, eps, seed))


def make_sources(dims, nrhs: int, seed: int) -> np.ndarray:
    """Gaussian complex colour vectors on even sites, complex128 (nrhs, V/2, 3).

    Real and imaginary parts are iid N(0, 1).
    """
    check_dims(dims)
    half = volume(dims) // 2
    rng = np.random.Generator(np.random.PCG64(seed))
    z = rng.standard_normal((nrhs, half, 3, 2))
    return z[..., 0] + 1j * z[..., 1]


def random_gauge_transform(dims, seed: int, eps: float = 3.0) -> np.ndarray:
    """Random SU(3) matrix per site, complex128 (V, 3, 3) in lexicographic order."""
    check_dims(dims)
    V = volume(dims)
    rng = np.random.Generator(np.random.PCG64(seed))
    h = rng.standard_normal((V, 8))
    return su3_exp(h, eps)


def unit_links(dims) -> np.ndarray:
    """Thin links all equal to the identity (the free field), (T, Z, Y, X, 4, 3, 3)."""
    check_dims(dims)
    X, Y, Z, T = dims
    U = np.zeros((T, Z, Y, X, 4, 3, 3), dtype=np.complex128)
    U[..., 0, 0] = U[..., 1, 1] = U[..., 2, 2] = 1
    return U


def gauge_transform_thin(U: np.ndarray, g: np.ndarray) -> np.ndarray:
    """U_mu(x) -> g(x) U_mu(x) g(x+mu)^dagger for thin links (T, Z, Y, X, 4, 3, 3)."""
    T, Z, Y, X = U.shape[:4]
    G = g.reshape(T, Z, Y, X, 3, 3)
    out = np.empty_like(U)
    for mu in range(4):
        Gp = _roll_mu(G, 1, mu)
        out[..., mu, :, :] = G @ U[..., mu, :, :] @ np.conj(np.swapaxes(Gp, -1, -2))
    return out


# ---------------------------------------------------------------------------
# Workload definitions.  Each entry fixes lattice, link roughness, masses,
# right-hand sides and seeds; the gauge seed is BASE_SEED + index and the
# source seed is the gauge seed + 1000.
# ---------------------------------------------------------------------------
WORKLOADS = {
    "tiny_4x4x4x8": dict(index=0, dims=(4, 4, 4, 8), eps=0.3, masses=(0.1,), nrhs=1, tol=1e-10),
    "single_20x20x20x64": dict(index=1, dims=(20, 20, 20, 64), eps=0.3, masses=(0.01,), nrhs=1, tol=1e-10),
    "batched_20x20x20x64": dict(index=2, dims=(20, 20, 20, 64), eps=0.3,
                                masses=(0.005, 0.01, 0.02, 0.05), nrhs=24, tol=1e-10),
    "threelevel_48x48x48x96": dict(index=3, dims=(48, 48, 48, 96), eps=0.2, masses=(0.005,), nrhs=12, tol=1e-10),
}

SERVING_LATTICES = ((8, 8, 8, 8), (16, 16, 16, 32), (20, 20, 20, 64), (32, 32, 32, 64))
SERVING_WEIGHTS = (0.4, 0.3, 0.2, 0.1)


def gauge_seed(index: int) -> int:
    return BASE_SEED + index


def source_seed(index: int) -> int:
    return BASE_SEED + index + 1000


def serving_trace(n: int, rate: float = 50.0, seed: int = BASE_SEED + 4, lattices=SERVING_LATTICES,
                  weights=SERVING_WEIGHTS, mass_range=(0.005, 0.1), max_rhs: int = 12):
    """Poisson request trace: list of dicts (arrival_s, lattice index, masses, nrhs, source seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate, size=n)
    arrivals = np.cumsum(gaps)
    lat = rng.choice(len(lattices), size=n, p=np.asarray(weights) / np.sum(weights))
    nrhs = rng.integers(1, max_rhs + 1, size=n)
    out = []
    for k in range(n):
        m = rng.uniform(mass_range[0], mass_range[1])
        out.append(dict(arrival=float(arrivals[k]), lattice=int(lat[k]), mass=float(m),
                        nrhs=int(nrhs[k]), seed=int(seed * 7 + k)))
    return out
