"""MI355X (gfx950) even-odd asqtad CG: Python binding of libasqtad.so.

The binding only marshals arguments: PyTorch provides device memory and the
stream, and every step of the operator and the solvers runs in the library's
HIP kernels.  There is no CPU fallback: if the library is missing, loading
fails with an error that says how to build it.

The functions named like the C ABI (``asq_gauge_create``, ``asqtad_dslash_eo``,
``cg_solve``, ``cg_solve_batch``, ``serve_*`` ...) take raw integers for device
pointers and streams, exactly as ``include/asqtad.h`` declares them.  The
classes ``Gauge`` and ``Server`` wrap them around torch tensors.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libasqtad.so")

ASQ_OK, ASQ_PENDING = 0, 1
ASQ_EINVAL, ASQ_ENOMEM, ASQ_ENOCONV, ASQ_ENOTSU3, ASQ_EHIP, ASQ_ENAN, ASQ_EAGAIN = -1, -2, -3, -4, -5, -6, -7
ASQ_F64, ASQ_F32, ASQ_F16 = 0, 1, 2
ASQ_MODE_F64, ASQ_MODE_MIXED32, ASQ_MODE_MIXED16 = 0, 1, 2
MODES = {"f64": ASQ_MODE_F64, "mixed32": ASQ_MODE_MIXED32, "mixed16": ASQ_MODE_MIXED16}
PRECS = {"f64": ASQ_F64, "f32": ASQ_F32, "f16": ASQ_F16}

FLOPS_PER_SITE_DSLASH = 1146


class asq_gauge_desc(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int * 4), ("prec_mask", ctypes.c_int), ("recon", ctypes.c_int),
                ("fat_scale", ctypes.c_double), ("long_scale", ctypes.c_double)]


class asq_cg_params(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("maxiter", ctypes.c_int), ("mode", ctypes.c_int),
                ("delta", ctypes.c_double), ("poll_iters", ctypes.c_int), ("use_graph", ctypes.c_int)]


class asq_cg_stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("reliable_updates", ctypes.c_int), ("converged", ctypes.c_int),
                ("status", ctypes.c_int), ("true_resid", ctypes.c_double), ("seconds", ctypes.c_double),
                ("gflops", ctypes.c_double), ("escalations", ctypes.c_int), ("final_mode", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class AsqError(RuntimeError):
    def __init__(self, code, where, detail=None):
        self.code = code
        if detail is None:
            detail = _lib.asq_last_error().decode() if _lib is not None else ""
        super().__init__(f"{where}: {_lib.asq_strerror(code).decode()} ({code}) {detail}")


_vp = ctypes.c_void_p
_SIGS = {
    "asq_gauge_bytes": (ctypes.c_size_t, [ctypes.POINTER(asq_gauge_desc)]),
    "asq_gauge_create": (ctypes.c_int, [ctypes.POINTER(asq_gauge_desc), _vp, _vp, _vp, ctypes.c_size_t, _vp,
                                        ctypes.POINTER(_vp)]),
    "asq_gauge_create_device": (ctypes.c_int, [ctypes.POINTER(asq_gauge_desc), _vp, _vp, _vp, ctypes.c_size_t, _vp,
                                               ctypes.POINTER(_vp)]),
    "asq_gauge_destroy": (ctypes.c_int, [_vp]),
    "asqtad_dslash_eo": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp]),
    "asqtad_dslash_eo_variant": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp, _vp,
                                                ctypes.c_int, _vp]),
    "asq_vec_bytes": (ctypes.c_size_t, [ctypes.c_int, ctypes.c_size_t]),
    "asq_vec_convert": (ctypes.c_int, [ctypes.c_size_t, ctypes.c_int, _vp, ctypes.c_int, _vp, _vp]),
    "asq_vec_to_native": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp]),
    "asq_vec_from_native": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp]),
    "asq_workspace_bytes": (ctypes.c_size_t, [_vp, ctypes.c_int, ctypes.c_int]),
    "cg_solve": (ctypes.c_int, [_vp, ctypes.c_double, _vp, _vp, _vp, ctypes.c_size_t,
                                ctypes.POINTER(asq_cg_params), ctypes.POINTER(asq_cg_stats), _vp]),
    "cg_solve_batch": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double), _vp, _vp, _vp,
                                      ctypes.c_size_t, ctypes.POINTER(asq_cg_params),
                                      ctypes.POINTER(asq_cg_stats), _vp]),
    "asq_multishift_workspace_bytes": (ctypes.c_size_t, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "cg_solve_multishift": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double), _vp,
                                           _vp, _vp, ctypes.c_size_t, ctypes.POINTER(asq_cg_params),
                                           ctypes.POINTER(asq_cg_stats), _vp]),
    "asq_full_workspace_bytes": (ctypes.c_size_t, [_vp, ctypes.c_int, ctypes.c_int]),
    "cg_solve_full": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double), _vp, _vp, _vp,
                                     ctypes.c_size_t, ctypes.POINTER(asq_cg_params),
                                     ctypes.POINTER(asq_cg_stats), _vp]),
    "serve_create": (ctypes.c_int, [_vp, ctypes.c_size_t, ctypes.c_int, ctypes.c_int, ctypes.POINTER(_vp)]),
    "serve_register_gauge": (ctypes.c_int, [_vp, _vp, ctypes.POINTER(ctypes.c_int)]),
    "serve_submit": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double), _vp, _vp,
                                    ctypes.POINTER(asq_cg_params), ctypes.POINTER(ctypes.c_uint64), _vp]),
    "serve_poll": (ctypes.c_int, [_vp, ctypes.c_uint64, ctypes.POINTER(asq_cg_stats),
                                  ctypes.POINTER(ctypes.c_double)]),
    "serve_destroy": (ctypes.c_int, [_vp]),
    "asqtad_build_links": (ctypes.c_int, [ctypes.POINTER(ctypes.c_int), _vp, ctypes.c_double, _vp, _vp, _vp]),
    "asqtad_plaquette_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(ctypes.c_int)]),
    "asqtad_plaquette": (ctypes.c_int, [ctypes.POINTER(ctypes.c_int), _vp, _vp, ctypes.c_size_t,
                                        ctypes.POINTER(ctypes.c_double), _vp]),
    "asqtad_npr_fourfermion": (ctypes.c_int, [ctypes.POINTER(ctypes.c_int), _vp, _vp, _vp, _vp, _vp, ctypes.c_int,
                                              ctypes.POINTER(ctypes.c_int), _vp, _vp]),
    "asqtad_plaquette_noalloc": (ctypes.c_int, [ctypes.POINTER(ctypes.c_int), _vp, _vp, _vp]),
    "asq_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "asq_last_error": (ctypes.c_char_p, []),
    "asq_copy_probe": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t, _vp]),
    "asq_read_probe": (ctypes.c_int, [_vp, ctypes.c_size_t, _vp, _vp]),
    "asq_read_probe_blocks": (ctypes.c_size_t, [ctypes.c_size_t]),
}

EXPORTS = tuple(_SIGS)

_lib = None


ASQ_VARIANT_NATIVE = 0x100000


def variant_code(cols: int, pipe: bool = False, order: int = 0, native: bool = False, sweep: bool = False,
                 chunk: int = 0, stream: bool = False, lds: bool = False) -> int:
    """Launch variant of asqtad_dslash_eo_variant: columns per thread (1, 2, 4, 6, 8, 12), pipelined hop
    loop, block order (0 tiles of a site block adjacent; 1, 2, 3 tile by tile in
    groups of 16, 64 or all site blocks); sweep: one global sweep instead of a slab per XCD,
    in which each XCD takes single blocks (chunk 0) or runs of 16, 64, 256 blocks (chunk 1, 2, 3);
    stream: links read with non-temporal loads (one column, FP32 and 16-bit link tiers);
    lds: each block stages the input records of its columns within three y-rows of its sites in
    LDS for its x and y hops (pipelined loop, native layout; streamed links only at one column);
    native: vectors in the solvers' native layout."""
    return (int(cols) | (0x100 if pipe else 0) | (0x200 if stream else 0) | (0x4000 if lds else 0) | (int(order) << 12)
            | ((0x8000 | (int(chunk) << 10)) if sweep else 0) | (ASQ_VARIANT_NATIVE if native else 0))


def variant_code_mfma(order: int = 0) -> int:
    """The matrix-core launch variant (FP32 18-real links with FP16 vectors only, native
    layout): 32 columns per block, with one of the four block orders."""
    return 0x10000 | 32 | (int(order) << 12) | ASQ_VARIANT_NATIVE


# Every launch variant the library builds: (cols, pipe, order, sweep, chunk).
VARIANTS_ALL = [(c, p, o, g, k) for g, ks in ((False, (0,)), (True, (0, 1, 2, 3))) for k in ks
                for o in (0, 1, 2, 3) for p in (False, True) for c in (1, 2, 4, 6, 8, 12)]


def load():
    """Load libasqtad.so (built in-tree by ``python -m paper_1411_2223_amd.build``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1411_2223_amd.build` "
                               "(there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _fn(name):
    def call(*args):
        return getattr(load(), name)(*args)

    call.__name__ = name
    return call


for _n in _SIGS:
    globals()[_n] = _fn(_n)


def check(rc, where):
    if rc < 0:
        raise AsqError(rc, where)
    return rc


# ---------------------------------------------------------------------------
# torch-side helpers (device memory and streams only)
# ---------------------------------------------------------------------------

def _torch():
    import torch

    return torch


def stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


VEC_SITE_BYTES = {"f64": 48, "f32": 24, "f16": 16}
_TORCH_DT = {"f64": "float64", "f32": "float32", "f16": "uint8"}


def _need(t, nbytes, where, name):
    """A caller tensor is checked before its pointer crosses the C ABI, which sees no
    sizes: a contiguous device tensor of at least nbytes."""
    if not getattr(t, "is_cuda", False):
        raise AsqError(ASQ_EINVAL, where, f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise AsqError(ASQ_EINVAL, where, f"{name} must be contiguous")
    have = t.numel() * t.element_size()
    if have < nbytes:
        raise AsqError(ASQ_EINVAL, where, f"{name} holds {have} bytes, {nbytes} needed")


def empty_bytes(n, device="cuda"):
    """Caller-owned device buffer of n bytes (256-byte aligned by the caching allocator)."""
    torch = _torch()
    t = torch.empty(max(int(n), 1), dtype=torch.uint8, device=device)
    assert t.data_ptr() % 256 == 0
    return t


def empty_vec(nsites, prec="f64", device="cuda"):
    """A device tensor holding nsites canonical colour-vector records of tier prec."""
    torch = _torch()
    load()
    n = asq_vec_bytes(PRECS[prec], int(nsites))
    return torch.empty(n // np.dtype(_TORCH_DT[prec]).itemsize, dtype=getattr(torch, _TORCH_DT[prec]),
                       device=device)


def vec_convert(src, nsites, src_prec, dst_prec, dst=None, stream=None):
    """dst = src converted between canonical tiers by the library (asq_vec_convert)."""
    load()
    if dst is None:
        dst = empty_vec(nsites, dst_prec, src.device)
    _need(src, nsites * VEC_SITE_BYTES[src_prec], "vec_convert", "src")
    _need(dst, nsites * VEC_SITE_BYTES[dst_prec], "vec_convert", "dst")
    check(asq_vec_convert(int(nsites), PRECS[src_prec], src.data_ptr(), PRECS[dst_prec], dst.data_ptr(),
                          stream_ptr(stream)), "asq_vec_convert")
    return dst


def vec_to_device(v, prec="f64", device="cuda", stream=None):
    """(nrhs, V/2, 3) complex host array -> device tensor in the canonical layout of tier prec.

    The complex128 array already is the canonical FP64 layout [nrhs][V/2][3][2]; it is
    uploaded as is, and the library converts it to FP32 or FP16-with-norm when asked."""
    torch = _torch()
    v = np.ascontiguousarray(np.asarray(v, dtype=np.complex128))
    if v.ndim == 2:
        v = v[None]
    t = torch.from_numpy(v.reshape(-1).view(np.float64)).to(device)
    if prec == "f64":
        return t
    return vec_convert(t, v.shape[0] * v.shape[1], "f64", prec, stream=stream)


def vec_from_device(t, nrhs, half, prec="f64", stream=None):
    """Inverse of vec_to_device: canonical device tensor -> (nrhs, V/2, 3) complex128 host array
    (FP32 and FP16 tiers widened to FP64 by the library first)."""
    torch = _torch()
    if prec != "f64":
        t = vec_convert(t, nrhs * half, prec, "f64", stream=stream)
    torch.cuda.synchronize(t.device)
    a = t.detach().cpu().numpy().view(np.float64)[: nrhs * half * 6]
    return a.view(np.complex128).reshape(nrhs, half, 3).copy()


def links_to_device(a, device="cuda"):
    """Canonical complex128 links (V, 4, 3, 3) -> a float64 device tensor of V * 4 * 18 reals."""
    torch = _torch()
    a = np.ascontiguousarray(np.asarray(a, dtype=np.complex128))
    return torch.from_numpy(a.reshape(-1).view(np.float64)).to(device)


def build_links(dims, thin_dev, u0=1.0, fat=None, lng=None, stream=None):
    """Asqtad fat and long links from thin links on the device (asqtad_build_links).

    thin_dev, fat, lng: float64 device tensors of V * 4 * 18 reals in the canonical
    layout (see links_to_device); fat and lng are allocated when not given.
    Returns (fat, lng); the work is enqueued on the stream.
    """
    torch = _torch()
    load()
    dims = tuple(int(d) for d in dims)
    n = int(np.prod(dims)) * 4 * 18
    if thin_dev.dtype != torch.float64 or thin_dev.numel() != n or not thin_dev.is_contiguous():
        raise AsqError(ASQ_EINVAL, "build_links: thin links must be a contiguous float64 tensor of V*4*18 reals")
    fat = torch.empty(n, dtype=torch.float64, device=thin_dev.device) if fat is None else fat
    lng = torch.empty(n, dtype=torch.float64, device=thin_dev.device) if lng is None else lng
    for t in (fat, lng):
        if t.dtype != torch.float64 or t.numel() != n or not t.is_contiguous():
            raise AsqError(ASQ_EINVAL, "build_links: outputs must be contiguous float64 tensors of V*4*18 reals")
    rc = asqtad_build_links((ctypes.c_int * 4)(*dims), thin_dev.data_ptr(), float(u0), fat.data_ptr(),
                            lng.data_ptr(), stream_ptr(stream))
    check(rc, "asqtad_build_links")
    return fat, lng


def plaquette(dims, thin_dev, stream=None) -> float:
    """Mean plaquette of thin links on the device (asqtad_plaquette); u0 = P ** 0.25."""
    torch = _torch()
    load()
    dims = tuple(int(d) for d in dims)
    n = int(np.prod(dims)) * 4 * 18
    if thin_dev.dtype != torch.float64 or thin_dev.numel() != n or not thin_dev.is_contiguous():
        raise AsqError(ASQ_EINVAL, "plaquette: thin links must be a contiguous float64 tensor of V*4*18 reals")
    d4 = (ctypes.c_int * 4)(*dims)
    nbytes = asqtad_plaquette_workspace_bytes(d4)
    if nbytes == 0:
        raise AsqError(ASQ_EINVAL, "asqtad_plaquette_workspace_bytes")
    work = torch.empty(nbytes, dtype=torch.uint8, device=thin_dev.device)
    p = ctypes.c_double(0)
    check(asqtad_plaquette(d4, thin_dev.data_ptr(), work.data_ptr(), nbytes, ctypes.byref(p), stream_ptr(stream)),
          "asqtad_plaquette")
    return p.value


def npr_fourfermion(dims, thin_dev, props, ops, out=None, stream=None):
    """The one-colour four-fermion operator of Eq. (1) (asqtad_npr_fourfermion): thin_dev the
    canonical links (V * 4 * 18 float64), props four float64 device tensors of V * 18 reals
    (G1..G4, [site][colour][source colour] complex), ops [(S1, F1, S2, F2), ...].  Returns out,
    float64 [nop][V/16][81][2] (indices a1 a2 a3 a4); the work is enqueued on the stream."""
    torch = _torch()
    load()
    dims = tuple(int(d) for d in dims)
    V = int(np.prod(dims))
    op = np.ascontiguousarray(np.asarray(ops, dtype=np.int32).reshape(-1, 4))
    nop = op.shape[0]
    _need(thin_dev, V * 4 * 18 * 8, "npr_fourfermion", "thin links")
    for k, g in enumerate(props):
        _need(g, V * 18 * 8, "npr_fourfermion", f"propagator {k + 1}")
    if len(props) != 4:
        raise AsqError(ASQ_EINVAL, "npr_fourfermion", "four propagators (G1, G2, G3, G4)")
    if out is None:
        out = torch.empty(nop * (V // 16) * 162, dtype=torch.float64, device=thin_dev.device)
    _need(out, nop * (V // 16) * 162 * 8, "npr_fourfermion", "out")
    rc = asqtad_npr_fourfermion((ctypes.c_int * 4)(*dims), thin_dev.data_ptr(), props[0].data_ptr(),
                                props[1].data_ptr(), props[2].data_ptr(), props[3].data_ptr(), int(nop),
                                op.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), out.data_ptr(), stream_ptr(stream))
    check(rc, "asqtad_npr_fourfermion")
    return out


@dataclass
class SolveResult:
    x: object
    stats: list
    rc: int


class Gauge:
    """A resident gauge field: canonical links uploaded, imported into device storage."""

    def __init__(self, dims, fat, lng, precs=("f64", "f32"), recon=18, fat_scale=9 / 8, long_scale=-1 / 24,
                 device="cuda", stream=None):
        torch = _torch()
        load()
        self.dims = tuple(int(d) for d in dims)
        self.half = int(np.prod(self.dims)) // 2
        self.precs = tuple(precs)
        mask = 0
        for p in precs:
            mask |= 1 << PRECS[p]
        self.desc = asq_gauge_desc((ctypes.c_int * 4)(*self.dims), mask, int(recon), float(fat_scale),
                                   float(long_scale))
        nbytes = asq_gauge_bytes(ctypes.byref(self.desc))
        if nbytes == 0:
            raise AsqError(ASQ_EINVAL, "asq_gauge_bytes")
        V = int(np.prod(self.dims))

        on_dev = [isinstance(a, torch.Tensor) for a in (fat, lng)]
        if on_dev[0] != on_dev[1]:
            raise AsqError(ASQ_EINVAL, "Gauge: fat and long links must both be host arrays or both device tensors")
        if on_dev[0]:  # already on the device (e.g. from build_links): imported in place
            for a in (fat, lng):
                if (a.dtype != torch.float64 or a.numel() != V * 4 * 18 or not a.is_contiguous()
                        or a.device.type != "cuda"):
                    raise AsqError(ASQ_EINVAL, "Gauge: device links must be contiguous float64 CUDA tensors "
                                               "of V*4*18 reals")
            ptrs = (fat.data_ptr(), lng.data_ptr())
            create = asq_gauge_create_device
        else:  # host arrays: the library copies them in
            keep = [np.ascontiguousarray(np.asarray(a, dtype=np.complex128).reshape(V, 4, 3, 3)) for a in (fat, lng)]
            ptrs = tuple(k.ctypes.data for k in keep)
            create = asq_gauge_create
        self.storage = empty_bytes(nbytes, device)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.storage.device):
            rc = create(ctypes.byref(self.desc), ptrs[0], ptrs[1], self.storage.data_ptr(), nbytes,
                        stream_ptr(stream), ctypes.byref(h))
        check(rc, create.__name__)
        self.handle = h
        self.device = device

    @classmethod
    def from_thin(cls, dims, thin, u0=1.0, precs=("f64", "f32"), device="cuda", stream=None):
        """A resident gauge field whose fat and long links are built on the device from
        canonical thin links (host array or device tensor) by asqtad_build_links.
        u0 = "plaquette" takes the tadpole factor from the mean plaquette, P ** 0.25.
        The fat links are not SU(3), so the links are kept as 18 reals."""
        torch = _torch()
        thin_d = thin if isinstance(thin, torch.Tensor) else links_to_device(thin, device)
        if isinstance(u0, str):
            if u0 != "plaquette":
                raise AsqError(ASQ_EINVAL, "from_thin: u0 is a number or 'plaquette'")
            u0 = plaquette(dims, thin_d, stream=stream) ** 0.25
        fat, lng = build_links(dims, thin_d, u0, stream=stream)
        return cls(dims, fat, lng, precs=precs, recon=18, device=device, stream=stream)

    def close(self):
        if getattr(self, "handle", None):
            asq_gauge_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def dslash(self, out_parity, vin, prec="f64", nrhs=1, out=None, stream=None, variant=None):
        """out = D_{out_parity <- other} vin on device tensors in the canonical layout of tier prec,
        with the tuned launch variant or the given one (see variant_code; a native variant takes
        vectors in the solvers' layout, see to_native)."""
        torch = _torch()
        if out is None:
            out = torch.empty_like(vin)
        nbytes = int(nrhs) * self.half * VEC_SITE_BYTES.get(prec, 0)
        _need(vin, nbytes, "dslash", "vin")
        _need(out, nbytes, "dslash", "out")
        if variant is None:
            rc = asqtad_dslash_eo(self.handle, int(out_parity), PRECS[prec], int(nrhs), vin.data_ptr(),
                                  out.data_ptr(), stream_ptr(stream))
            check(rc, "asqtad_dslash_eo")
        else:
            rc = asqtad_dslash_eo_variant(self.handle, int(out_parity), PRECS[prec], int(nrhs), vin.data_ptr(),
                                          out.data_ptr(), int(variant), stream_ptr(stream))
            check(rc, "asqtad_dslash_eo_variant")
        return out

    def to_native(self, v, prec="f64", nrhs=1, out=None, stream=None):
        """Canonical device vectors -> the solvers' native layout (asq_vec_to_native)."""
        torch = _torch()
        out = torch.empty_like(v) if out is None else out
        nbytes = int(nrhs) * self.half * VEC_SITE_BYTES[prec]
        _need(v, nbytes, "to_native", "v")
        _need(out, nbytes, "to_native", "out")
        check(asq_vec_to_native(self.handle, PRECS[prec], int(nrhs), v.data_ptr(), out.data_ptr(), stream_ptr(stream)),
              "asq_vec_to_native")
        return out

    def from_native(self, v, prec="f64", nrhs=1, out=None, stream=None):
        """Native-layout device vectors -> canonical (asq_vec_from_native)."""
        torch = _torch()
        out = torch.empty_like(v) if out is None else out
        nbytes = int(nrhs) * self.half * VEC_SITE_BYTES[prec]
        _need(v, nbytes, "from_native", "v")
        _need(out, nbytes, "from_native", "out")
        check(asq_vec_from_native(self.handle, PRECS[prec], int(nrhs), v.data_ptr(), out.data_ptr(),
                                  stream_ptr(stream)), "asq_vec_from_native")
        return out

    def default_delta(self, mode):
        """Reliable-update trigger: 0.01, or 0.1 when the FP16 tier iterates with 16-bit
        links (their rounding makes the iterated residual drift faster: at 48^3 x 96 the
        three-level solve needs 454 iterations with 0.1 and 1047 with 0.01)."""
        return 0.1 if mode == "mixed16" and "f16" in self.precs else 0.01

    def workspace(self, nrhs, mode="mixed32"):
        n = asq_workspace_bytes(self.handle, int(nrhs), MODES[mode])
        return empty_bytes(n, self.device)

    def solve(self, masses, b, mode="mixed32", tol=1e-10, maxiter=20000, delta=None, poll_iters=16, use_graph=True,
              work=None, x=None, stream=None):
        """Batched CG: b is a canonical device tensor [nrhs][V/2][3][2] float64; returns SolveResult."""
        torch = _torch()
        masses = np.atleast_1d(np.asarray(masses, dtype=np.float64))
        nrhs = len(masses)
        if work is None:
            work = self.workspace(nrhs, mode)
        if x is None:
            x = torch.empty_like(b)
        nbytes = nrhs * self.half * 48
        _need(b, nbytes, "solve", "b")
        _need(x, nbytes, "solve", "x")
        _need(work, 0, "solve", "work")
        if delta is None:
            delta = self.default_delta(mode)
        params = asq_cg_params(float(tol), int(maxiter), MODES[mode], float(delta), int(poll_iters),
                               1 if use_graph else 0)
        stats = (asq_cg_stats * nrhs)()
        m = (ctypes.c_double * nrhs)(*masses)
        rc = cg_solve_batch(self.handle, nrhs, m, b.data_ptr(), x.data_ptr(), work.data_ptr(), work.numel(),
                            ctypes.byref(params), stats, stream_ptr(stream))
        if rc < 0 and rc not in (ASQ_ENOCONV, ASQ_ENAN):  # per-column outcomes: x and stats are written
            check(rc, "cg_solve_batch")
        return SolveResult(x, [s.as_dict() for s in stats], rc)

    def solve_multishift(self, masses, b, mode="mixed32", tol=1e-10, maxiter=20000, delta=None, poll_iters=16,
                         use_graph=True, work=None, x=None, stream=None):
        """Every (mass, source) pair: b is a canonical device tensor [nsrc][V/2][3][2] float64; x is
        [nmass][nsrc][V/2][3][2] (column j * nsrc + s); returns SolveResult over those columns."""
        torch = _torch()
        masses = np.atleast_1d(np.asarray(masses, dtype=np.float64))
        nmass = len(masses)
        nsrc = b.numel() * b.element_size() // (48 * self.half)
        if nsrc < 1:
            raise AsqError(ASQ_EINVAL, "solve_multishift", "b holds less than one column")
        if work is None:
            work = empty_bytes(asq_multishift_workspace_bytes(self.handle, nsrc, nmass, MODES[mode]), self.device)
        if x is None:
            x = torch.empty(nmass * nsrc * self.half * 6, dtype=torch.float64, device=b.device)
        _need(b, nsrc * self.half * 48, "solve_multishift", "b")
        _need(x, nmass * nsrc * self.half * 48, "solve_multishift", "x")
        _need(work, 0, "solve_multishift", "work")
        if delta is None:
            delta = self.default_delta(mode)
        params = asq_cg_params(float(tol), int(maxiter), MODES[mode], float(delta), int(poll_iters),
                               1 if use_graph else 0)
        stats = (asq_cg_stats * (nmass * nsrc))()
        m = (ctypes.c_double * nmass)(*masses)
        rc = cg_solve_multishift(self.handle, nsrc, nmass, m, b.data_ptr(), x.data_ptr(), work.data_ptr(),
                                 work.numel(), ctypes.byref(params), stats, stream_ptr(stream))
        if rc < 0 and rc not in (ASQ_ENOCONV, ASQ_ENAN):  # per-column outcomes: x and stats are written
            check(rc, "cg_solve_multishift")
        return SolveResult(x, [s.as_dict() for s in stats], rc)

    def solve_full(self, masses, b, mode="mixed32", tol=1e-10, maxiter=20000, delta=None, poll_iters=16,
                   use_graph=True, work=None, x=None, stream=None):
        """M x = b on both parities (M = 2m + D): b is a canonical device tensor [2][nrhs][V/2][3][2]
        float64 (even halves, then odd halves); returns SolveResult with |b - M x| / |b| per column."""
        torch = _torch()
        masses = np.atleast_1d(np.asarray(masses, dtype=np.float64))
        nrhs = len(masses)
        if work is None:
            work = empty_bytes(asq_full_workspace_bytes(self.handle, nrhs, MODES[mode]), self.device)
        if x is None:
            x = torch.empty_like(b)
        _need(b, 2 * nrhs * self.half * 48, "solve_full", "b")
        _need(x, 2 * nrhs * self.half * 48, "solve_full", "x")
        _need(work, 0, "solve_full", "work")
        if delta is None:
            delta = self.default_delta(mode)
        params = asq_cg_params(float(tol), int(maxiter), MODES[mode], float(delta), int(poll_iters),
                               1 if use_graph else 0)
        stats = (asq_cg_stats * nrhs)()
        m = (ctypes.c_double * nrhs)(*masses)
        rc = cg_solve_full(self.handle, nrhs, m, b.data_ptr(), x.data_ptr(), work.data_ptr(), work.numel(),
                           ctypes.byref(params), stats, stream_ptr(stream))
        if rc < 0 and rc not in (ASQ_ENOCONV, ASQ_ENAN):  # per-column outcomes: x and stats are written
            check(rc, "cg_solve_full")
        return SolveResult(x, [s.as_dict() for s in stats], rc)


class Server:
    """Continuous-batching solve server over a caller-owned arena (the HBM budget)."""

    def __init__(self, arena_bytes, max_streams=4, max_cols=16, device="cuda"):
        load()
        self.arena = empty_bytes(int(arena_bytes), device)
        h = ctypes.c_void_p()
        check(serve_create(self.arena.data_ptr(), int(arena_bytes), int(max_streams), int(max_cols),
                           ctypes.byref(h)), "serve_create")
        self.handle = h
        self.gauges = []

    def register(self, gauge):
        gid = ctypes.c_int()
        check(serve_register_gauge(self.handle, gauge.handle, ctypes.byref(gid)), "serve_register_gauge")
        self.gauges.append(gauge)
        return gid.value

    def submit(self, gauge_id, masses, b, x, mode="mixed32", tol=1e-10, maxiter=20000, delta=None, poll_iters=8,
               use_graph=True, stream=None):
        """Queue a batched solve of canonical b into x; the server reads b after the work already
        enqueued on `stream` (torch's current stream by default).  Returns the ticket."""
        masses = np.atleast_1d(np.asarray(masses, dtype=np.float64))
        n = len(masses)
        if delta is None:
            delta = self.gauges[gauge_id].default_delta(mode)
        params = asq_cg_params(float(tol), int(maxiter), MODES[mode], float(delta), int(poll_iters),
                               1 if use_graph else 0)
        half = self.gauges[gauge_id].half if 0 <= gauge_id < len(self.gauges) else 0
        _need(b, n * half * 48, "serve_submit", "b")
        _need(x, n * half * 48, "serve_submit", "x")
        t = ctypes.c_uint64()
        rc = serve_submit(self.handle, int(gauge_id), n, (ctypes.c_double * n)(*masses), b.data_ptr(), x.data_ptr(),
                          ctypes.byref(params), ctypes.byref(t), stream_ptr(stream))
        check(rc, "serve_submit")
        return t.value

    def poll(self, ticket, nrhs):
        """None while pending; else (rc, per-column stats, latency seconds)."""
        stats = (asq_cg_stats * int(nrhs))()
        lat = ctypes.c_double()
        rc = serve_poll(self.handle, ctypes.c_uint64(ticket), stats, ctypes.byref(lat))
        if rc == ASQ_PENDING:
            return None
        if rc == ASQ_EINVAL:
            check(rc, "serve_poll")
        return rc, [s.as_dict() for s in stats], lat.value

    def close(self):
        if getattr(self, "handle", None):
            serve_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
