"""FP64 CPU oracle for the even-odd asqtad CG (ctypes wrapper over asqtad_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
benchmark's CPU-baseline leg.  The GPU library never imports or calls it, and it
shares no code with the HIP path.

Every function takes the canonical host arrays produced by ``synth``:
links complex128 (V, 4, 3, 3), even/odd colour vectors complex128 (V/2, 3).

Pins (tests/test_oracle.py) tie it to facts that do not come from itself:
free-field plane-wave spectrum (closed form), anti-Hermiticity of D, gauge
covariance, hand-derived point-source values, brute-force dense solves and the
finite termination of CG on an operator with few distinct eigenvalues.  The
asqtad link construction is pinned by the free-field normalisation, the closed
form for a uniform abelian flux, gauge covariance and an independent nested
staple evaluation; the plaquette by the free field, the uniform flux and gauge
invariance.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "asqtad_oracle.c")
_SRCS = (_SRC, os.path.join(_HERE, "npr_oracle.c"))
_LIB = os.path.join(_HERE, "liboracle.so")
# a copy tuned for the host it runs on, compiled in the process that asks for it
_LIB_NATIVE = os.path.join(_HERE, "liboracle_native.so")
# -std=c11 alone already turns off FMA contraction in gcc; it is spelled out so that
# the portable and the host-tuned builds round every product and sum alike
_CFLAGS = ["-O3", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared", "-fopenmp"]
_native = False

_dptr = ctypes.POINTER(ctypes.c_double)
_iptr = ctypes.POINTER(ctypes.c_int)


def build(force: bool = False) -> str:
    """Compile the oracle shared library with gcc (-O3, OpenMP, generic x86-64 code)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(os.path.getmtime(f) for f in _SRCS):
        cmd = ["gcc", *_CFLAGS, *_SRCS, "-o", _LIB + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def select_native_build() -> str:
    """Load, in place of the portable build, a copy compiled here and now with
    -O3 -march=native for the CPU this process runs on (the CPU-baseline timing uses
    it).  Same arithmetic: no FMA contraction and no reassociation in either build.
    Must be called before the first oracle call of the process."""
    global _native
    if _lib is not None:
        raise RuntimeError("the oracle library is already loaded")
    tmp = f"{_LIB_NATIVE}.tmp{os.getpid()}"
    subprocess.run(["gcc", *_CFLAGS, "-march=native", *_SRCS, "-o", tmp, "-lm"], check=True)
    os.replace(tmp, _LIB_NATIVE)
    _native = True
    return _LIB_NATIVE


def build_flags() -> str:
    """The gcc flags of the build this process loads (or will load)."""
    return " ".join(_CFLAGS + (["-march=native"] if _native else []))


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(_LIB_NATIVE if _native else build())
        L.oracle_dslash.argtypes = [_iptr, _dptr, _dptr, ctypes.c_int, _dptr, _dptr]
        L.oracle_dslash.restype = ctypes.c_int
        L.oracle_apply_A.argtypes = [_iptr, _dptr, _dptr, ctypes.c_double, _dptr, _dptr]
        L.oracle_apply_A.restype = ctypes.c_int
        L.oracle_true_residual.argtypes = [_iptr, _dptr, _dptr, ctypes.c_double, _dptr, _dptr]
        L.oracle_true_residual.restype = ctypes.c_double
        L.oracle_cg.argtypes = [_iptr, _dptr, _dptr, ctypes.c_double, _dptr, _dptr, ctypes.c_double,
                                ctypes.c_int, _iptr, _dptr, _dptr]
        L.oracle_cg.restype = ctypes.c_int
        L.oracle_asqtad_links.argtypes = [_iptr, _dptr, ctypes.c_double, ctypes.POINTER(ctypes.c_long),
                                          ctypes.c_long, _dptr, _dptr]
        L.oracle_asqtad_links.restype = ctypes.c_int
        L.oracle_plaquette.argtypes = [_iptr, _dptr]
        L.oracle_plaquette.restype = ctypes.c_double
        L.oracle_spin_taste.argtypes = [ctypes.c_int, ctypes.c_int, _dptr]
        L.oracle_spin_taste.restype = ctypes.c_int
        L.oracle_link_average.argtypes = [_iptr, _dptr, _iptr, ctypes.c_int, ctypes.c_int, _dptr]
        L.oracle_link_average.restype = ctypes.c_int
        L.oracle_npr_fourfermion.argtypes = [_iptr, _dptr, _dptr, _dptr, _dptr, _dptr, ctypes.c_int, _iptr,
                                             ctypes.POINTER(ctypes.c_long), ctypes.c_long, _dptr]
        L.oracle_npr_fourfermion.restype = ctypes.c_int
        L.oracle_num_threads.argtypes = []
        L.oracle_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _dims(dims):
    return (ctypes.c_int * 4)(*[int(d) for d in dims])


def _c128(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    if shape is not None and a.shape != tuple(shape):
        a = a.reshape(shape)
    return a


def _p(a):
    return a.ctypes.data_as(_dptr)


def _check_links(dims, fat, lng):
    V = int(np.prod(dims))
    return _c128(fat, (V, 4, 3, 3)), _c128(lng, (V, 4, 3, 3))


def dslash(dims, fat, lng, out_parity: int, vec) -> np.ndarray:
    """D restricted to sites of ``out_parity`` acting on a vector of the other parity."""
    fat, lng = _check_links(dims, fat, lng)
    half = int(np.prod(dims)) // 2
    v = _c128(vec, (half, 3))
    out = np.empty((half, 3), dtype=np.complex128)
    rc = lib().oracle_dslash(_dims(dims), _p(fat), _p(lng), int(out_parity), _p(v), _p(out))
    if rc != 0:
        raise ValueError(f"oracle_dslash failed ({rc})")
    return out


def apply_A(dims, fat, lng, mass: float, vec) -> np.ndarray:
    """(4 m^2 - D_eo D_oe) vec on even sites."""
    fat, lng = _check_links(dims, fat, lng)
    half = int(np.prod(dims)) // 2
    v = _c128(vec, (half, 3))
    out = np.empty((half, 3), dtype=np.complex128)
    rc = lib().oracle_apply_A(_dims(dims), _p(fat), _p(lng), float(mass), _p(v), _p(out))
    if rc != 0:
        raise ValueError(f"oracle_apply_A failed ({rc})")
    return out


def true_residual(dims, fat, lng, mass: float, b, x) -> float:
    """|b - A x| / |b| computed in FP64."""
    fat, lng = _check_links(dims, fat, lng)
    half = int(np.prod(dims)) // 2
    bb, xx = _c128(b, (half, 3)), _c128(x, (half, 3))
    return float(lib().oracle_true_residual(_dims(dims), _p(fat), _p(lng), float(mass), _p(bb), _p(xx)))


def cg(dims, fat, lng, mass: float, b, tol: float = 1e-10, maxiter: int = 100000, history: bool = False):
    """Plain FP64 CG from x0 = 0.  Returns (x, iters, true_resid, converged[, resid_history])."""
    fat, lng = _check_links(dims, fat, lng)
    half = int(np.prod(dims)) // 2
    bb = _c128(b, (half, 3))
    x = np.zeros((half, 3), dtype=np.complex128)
    it = ctypes.c_int(0)
    tr = ctypes.c_double(0)
    hist = np.zeros(maxiter + 1) if history else None
    rc = lib().oracle_cg(_dims(dims), _p(fat), _p(lng), float(mass), _p(bb), _p(x), float(tol), int(maxiter),
                         ctypes.byref(it), ctypes.byref(tr), _p(hist) if history else None)
    if rc < 0:
        raise ValueError(f"oracle_cg failed ({rc})")
    if history:
        return x, it.value, tr.value, rc == 0, hist[: it.value + 1]
    return x, it.value, tr.value, rc == 0


def asqtad_links(dims, thin, u0: float = 1.0, sites=None):
    """Asqtad fat and long links from thin links, as sums over paths.

    ``thin`` is complex128 with V*4*9 entries in the canonical order.  Returns
    (fat, long) complex128 (n, 4, 3, 3): every site in lexicographic order, or
    the listed ``sites`` in the given order.
    """
    V = int(np.prod(dims))
    U = _c128(thin, (V, 4, 3, 3))
    idx = None if sites is None else np.ascontiguousarray(sites, dtype=np.int64)
    n = V if idx is None else len(idx)
    fat = np.empty((n, 4, 3, 3), dtype=np.complex128)
    lng = np.empty((n, 4, 3, 3), dtype=np.complex128)
    sp = None if idx is None else idx.ctypes.data_as(ctypes.POINTER(ctypes.c_long))
    rc = lib().oracle_asqtad_links(_dims(dims), _p(U), float(u0), sp, int(n), _p(fat), _p(lng))
    if rc != 0:
        raise ValueError(f"oracle_asqtad_links failed ({rc})")
    return fat, lng


def plaquette(dims, thin) -> float:
    """Mean plaquette (1/3) Re tr of the thin links over every site and plane."""
    V = int(np.prod(dims))
    U = _c128(thin, (V, 4, 3, 3))
    p = float(lib().oracle_plaquette(_dims(dims), _p(U)))
    if p == -1.0:
        raise ValueError("oracle_plaquette: invalid extents")
    return p


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def dense_operator(apply, n_sites: int) -> np.ndarray:
    """Dense matrix of a linear map on (n_sites, 3) complex vectors, built column by column."""
    n = n_sites * 3
    M = np.empty((n, n), dtype=np.complex128)
    e = np.zeros(n, dtype=np.complex128)
    for k in range(n):
        e[k] = 1.0
        M[:, k] = apply(e.reshape(n_sites, 3)).reshape(n)
        e[k] = 0.0
    return M


# ---- NPR: the one-colour four-fermion operator of the paper's Eq. (1) ------------

def spin_taste(S: int, F: int) -> np.ndarray:
    """(gamma_S (x) xi_F)bar as a 16 x 16 complex matrix (row A, column B), from the trace
    (1/4) Tr[gamma_A^dag gamma_S gamma_B gamma_F^dag] with explicit 4 x 4 Dirac matrices."""
    out = np.empty((16, 16), dtype=np.complex128)
    if lib().oracle_spin_taste(int(S), int(F), _p(out)) != 0:
        raise ValueError("oracle_spin_taste: S and F are 4-bit masks")
    return out


def link_average(dims, thin, z, A: int, D: int) -> np.ndarray:
    """U_AD(z): the mean over every shortest path from corner A to corner D of hypercube z
    of the ordered link products; thin is complex (V, 4, 3, 3)."""
    V = int(np.prod(dims))
    U = _c128(thin, (V, 4, 3, 3))
    out = np.empty((3, 3), dtype=np.complex128)
    zc = (ctypes.c_int * 4)(*[int(v) for v in z])
    if lib().oracle_link_average(_dims(dims), _p(U), zc, int(A), int(D), _p(out)) != 0:
        raise ValueError("oracle_link_average: bad arguments")
    return out


def npr_fourfermion(dims, thin, props, ops, zs=None) -> np.ndarray:
    """V_I(z)[a1, a2, a3, a4] of Eq. (1) for operators ops = [(S1, F1, S2, F2), ...] and
    propagators props = (G1, G2, G3, G4), each complex (V, 3, 3) [site colour, source colour],
    at every hypercube (zs=None, lexicographic, zx fastest) or the listed ones.
    Returns complex (nop, nz, 3, 3, 3, 3)."""
    V = int(np.prod(dims))
    U = _c128(thin, (V, 4, 3, 3))
    G = [_c128(g, (V, 3, 3)) for g in props]
    op = np.ascontiguousarray(np.asarray(ops, dtype=np.int32).reshape(-1, 4))
    nop = op.shape[0]
    if zs is None:
        nz = V // 16
        zp = None
    else:
        zarr = np.ascontiguousarray(zs, dtype=np.int64)
        nz = len(zarr)
        zp = zarr.ctypes.data_as(ctypes.POINTER(ctypes.c_long))
    out = np.empty((nop, nz, 3, 3, 3, 3), dtype=np.complex128)
    rc = lib().oracle_npr_fourfermion(_dims(dims), _p(U), _p(G[0]), _p(G[1]), _p(G[2]), _p(G[3]), int(nop),
                                      op.ctypes.data_as(_iptr), zp, int(nz), _p(out))
    if rc != 0:
        raise ValueError(f"oracle_npr_fourfermion failed ({rc})")
    return out
