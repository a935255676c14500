"""Pins for the FP64 CPU oracle: facts fixed by the mathematics, not by the oracle.

* free-field spectrum of A = 4m^2 - D_eo D_oe against the plane-wave closed form
  4m^2 + 4 sum_mu f(p_mu)^2, f(p) = (9/8) sin p - (1/24) sin 3p, with periodic
  spatial and antiperiodic temporal momenta (dense eigvalsh and plane waves)
* hand-derived point-source values (tests/golden/point_source_free_8x8x10x12.txt)
* anti-Hermiticity D_oe = -D_eo^dagger on random links
* gauge covariance D[U^g](g psi) = g D[U] psi with random SU(3) g
* brute-force dense solves against CG, and the CG solution's covariance
* finite termination of CG on the free field (few distinct eigenvalues)
* an independent whole-lattice (shifted-array) form of D on random links
"""
import itertools
import os

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def lex_coords(dims):
    X, Y, Z, T = dims
    lex = np.arange(X * Y * Z * T)
    x = lex % X
    y = (lex // X) % Y
    z = (lex // (X * Y)) % Z
    t = lex // (X * Y * Z)
    return np.stack([x, y, z, t], axis=1)


def parity_sites(dims, parity):
    """Coordinates of the sites of one parity, in checkerboard order."""
    c = lex_coords(dims)
    sel = (c.sum(axis=1) % 2) == parity
    return c[sel]


def f_naik(p):
    return 9.0 / 8.0 * np.sin(p) - 1.0 / 24.0 * np.sin(3 * p)


def momenta(dims):
    X, Y, Z, T = dims
    px = 2 * np.pi * np.arange(X) / X
    py = 2 * np.pi * np.arange(Y) / Y
    pz = 2 * np.pi * np.arange(Z) / Z
    pt = (2 * np.arange(T) + 1) * np.pi / T
    return px, py, pz, pt


def free_even_spectrum(dims, mass):
    """Closed-form eigenvalues of A on even sites (each momentum pair p, p+pi counted once)."""
    px, py, pz, pt = momenta(dims)
    lam = []
    for a, b, c, d in itertools.product(px, py, pz, pt):
        lam.append(4 * mass**2 + 4 * (f_naik(a) ** 2 + f_naik(b) ** 2 + f_naik(c) ** 2 + f_naik(d) ** 2))
    lam = np.sort(np.array(lam))
    # p and p + (pi,pi,pi,pi) give the same even-site vector; f^2 is equal on both
    assert np.allclose(lam[0::2], lam[1::2])
    return np.repeat(lam[0::2], 3)  # three colours


def free_gauge(dims):
    return synth.fat_long_from_thin(synth.unit_links(dims))


# ---------------------------------------------------------------------------


def test_generator_su3_and_stream():
    dims = (4, 4, 4, 4)
    U = synth.thin_links(dims, 0.3, 123)
    flat = U.reshape(-1, 3, 3)
    eye = np.eye(3)
    assert np.max(np.abs(flat @ np.conj(np.swapaxes(flat, -1, -2)) - eye)) < 1e-14
    assert np.max(np.abs(np.linalg.det(flat) - 1)) < 1e-14
    lam = synth.gell_mann()
    tr = np.einsum("aij,bji->ab", lam, lam)
    assert np.allclose(tr, 2 * np.eye(8), atol=1e-15)
    # slice-by-slice draw equals one draw of the full shape
    rng = np.random.Generator(np.random.PCG64(123))
    h = rng.standard_normal((4, 4, 4, 4, 4, 8))
    assert np.array_equal(synth.su3_exp(h, 0.3), U)


def test_long_link_recipe_free_field():
    fat, lng = free_gauge((4, 4, 4, 8))
    assert np.allclose(fat, 9 / 8 * np.eye(3))
    assert np.allclose(lng, -1 / 24 * np.eye(3))


def test_naik_coefficients_closed_form():
    # f(p) = p + O(p^5): the p^3 term cancels, the p^5 coefficient is -3/40
    for p in (1e-2, 2e-2, 4e-2):
        assert abs((f_naik(p) - p) / p**5 + 3 / 40) < 1e-3
    assert abs(f_naik(np.pi / 2) - 7 / 6) < 1e-15


def test_point_source_golden():
    dims = (8, 8, 10, 12)
    fat, lng = free_gauge(dims)
    X, Y, Z, T = dims
    x0 = (1, 2, 3, 2)
    lex0 = x0[0] + X * (x0[1] + Y * (x0[2] + Z * x0[3]))
    assert sum(x0) % 2 == 0
    src = np.zeros((X * Y * Z * T // 2, 3), dtype=np.complex128)
    src[lex0 // 2, 1] = 1.0
    out = oracle.dslash(dims, fat, lng, 1, src)
    expect = np.zeros_like(out)
    rows = np.loadtxt(os.path.join(GOLDEN, "point_source_free_8x8x10x12.txt"), comments="#")
    assert rows.shape == (16, 7)
    for x, y, z, t, col, re, im in rows:
        lex = int(x) + X * (int(y) + Y * (int(z) + Z * int(t)))
        assert (int(x) + int(y) + int(z) + int(t)) % 2 == 1
        expect[lex // 2, int(col)] = re + 1j * im
    assert np.max(np.abs(out - expect)) < 1e-15


@pytest.mark.parametrize("dims", [(4, 4, 4, 8), (4, 4, 4, 4)])
def test_free_spectrum_dense(dims):
    mass = 0.1
    fat, lng = free_gauge(dims)
    half = int(np.prod(dims)) // 2
    A = oracle.dense_operator(lambda v: oracle.apply_A(dims, fat, lng, mass, v), half)
    assert np.max(np.abs(A - A.conj().T)) < 1e-13
    ev = np.linalg.eigvalsh(A)
    ref = free_even_spectrum(dims, mass)
    assert ev.shape == ref.shape
    assert np.max(np.abs(np.sort(ev) - ref)) < 1e-12


def test_free_plane_waves_nonuniform_lattice():
    dims = (6, 8, 4, 10)
    mass = 0.05
    fat, lng = free_gauge(dims)
    ev_sites = parity_sites(dims, 0)
    px, py, pz, pt = momenta(dims)
    rng = np.random.default_rng(7)
    for _ in range(6):
        p = np.array([rng.choice(px), rng.choice(py), rng.choice(pz), rng.choice(pt)])
        c = rng.standard_normal(3) + 1j * rng.standard_normal(3)
        v = np.exp(1j * ev_sites @ p)[:, None] * c[None, :]
        lam = 4 * mass**2 + 4 * np.sum(f_naik(p) ** 2)
        Av = oracle.apply_A(dims, fat, lng, mass, v)
        assert np.max(np.abs(Av - lam * v)) < 1e-12 * max(1.0, lam)


def test_free_plane_wave_full_size_lattice():
    # the 20^3 x 64 shape of the paper's workload: one plane wave
    dims = (20, 20, 20, 64)
    mass = 0.01
    fat, lng = free_gauge(dims)
    ev_sites = parity_sites(dims, 0)
    px, py, pz, pt = momenta(dims)
    p = np.array([px[3], py[7], pz[11], pt[5]])
    c = np.array([1.0, 0.5j, -0.25])
    v = np.exp(1j * ev_sites @ p)[:, None] * c[None, :]
    lam = 4 * mass**2 + 4 * np.sum(f_naik(p) ** 2)
    Av = oracle.apply_A(dims, fat, lng, mass, v)
    assert np.max(np.abs(Av - lam * v)) < 1e-12


@pytest.mark.parametrize("dims", [(4, 4, 4, 8), (6, 4, 8, 6)])
def test_anti_hermiticity(dims):
    fat, lng = synth.make_gauge(dims, 0.3, 99)
    half = int(np.prod(dims)) // 2
    rng = np.random.default_rng(1)
    phi = rng.standard_normal((half, 3)) + 1j * rng.standard_normal((half, 3))
    psi = rng.standard_normal((half, 3)) + 1j * rng.standard_normal((half, 3))
    lhs = np.vdot(phi, oracle.dslash(dims, fat, lng, 0, psi))  # <phi_e, D_eo psi_o>
    rhs = -np.vdot(oracle.dslash(dims, fat, lng, 1, phi), psi)  # -<D_oe phi_e, psi_o>
    assert abs(lhs - rhs) < 1e-14 * abs(lhs) * 10


def test_full_operator_composition():
    # M = 2m + D on both parities, composed from the one-parity D as the
    # full-system GPU tests compose it: since D is anti-Hermitian every
    # eigenvalue of M has real part 2m, and M^dag M restricted to even sites is
    # exactly A = 4m^2 - D_eo D_oe.  A transposed parity or a sign slip in the
    # composition breaks one of the two.
    dims, m = (4, 4, 4, 8), 0.07
    fat, lng = synth.make_gauge(dims, 0.3, 8)
    half = int(np.prod(dims)) // 2

    def apply_m(z):
        z = z.reshape(2, half, 3)
        return np.stack([2 * m * z[0] + oracle.dslash(dims, fat, lng, 0, z[1]),
                         2 * m * z[1] + oracle.dslash(dims, fat, lng, 1, z[0])])

    M = oracle.dense_operator(apply_m, 2 * half)
    ev = np.linalg.eigvals(M)
    assert np.max(np.abs(ev.real - 2 * m)) < 1e-12
    A = oracle.dense_operator(lambda v: oracle.apply_A(dims, fat, lng, m, v), half)
    n = half * 3
    assert np.max(np.abs((M.conj().T @ M)[:n, :n] - A)) < 1e-12


def _split(dims, g_lex, vec_full):
    """Apply per-site SU(3) g to a vector given on all sites in lexicographic order."""
    return np.einsum("sij,sj->si", g_lex, vec_full)


@pytest.mark.parametrize("dims", [(4, 4, 4, 8), (6, 4, 4, 8)])
def test_gauge_covariance(dims):
    U = synth.thin_links(dims, 0.3, 5)
    g = synth.random_gauge_transform(dims, 77)
    fat, lng = synth.fat_long_from_thin(U)
    fat_g, lng_g = synth.fat_long_from_thin(synth.gauge_transform_thin(U, g))
    V = int(np.prod(dims))
    c = lex_coords(dims)
    par = c.sum(axis=1) % 2
    rng = np.random.default_rng(3)
    for out_par in (0, 1):
        in_idx = np.nonzero(par == 1 - out_par)[0]
        out_idx = np.nonzero(par == out_par)[0]
        psi = rng.standard_normal((V // 2, 3)) + 1j * rng.standard_normal((V // 2, 3))
        g_in = g[in_idx]
        g_out = g[out_idx]
        lhs = oracle.dslash(dims, fat_g, lng_g, out_par, np.einsum("sij,sj->si", g_in, psi))
        rhs = np.einsum("sij,sj->si", g_out, oracle.dslash(dims, fat, lng, out_par, psi))
        assert np.max(np.abs(lhs - rhs)) < 1e-13


def test_dense_solve_matches_cg_config_tiny():
    w = synth.WORKLOADS["tiny_4x4x4x8"]
    dims, mass = w["dims"], w["masses"][0]
    fat, lng = synth.make_gauge(dims, w["eps"], synth.gauge_seed(w["index"]))
    b = synth.make_sources(dims, 1, synth.source_seed(w["index"]))[0]
    half = int(np.prod(dims)) // 2
    A = oracle.dense_operator(lambda v: oracle.apply_A(dims, fat, lng, mass, v), half)
    assert np.max(np.abs(A - A.conj().T)) < 1e-13
    ev = np.linalg.eigvalsh(A)
    # spectrum bounds: 4m^2 <= lambda <= 4m^2 + (8 (9/8 + 1/24))^2 for unitary thin links
    assert ev[0] >= 4 * mass**2 * (1 - 1e-12)
    assert ev[-1] <= 4 * mass**2 + (8 * (9 / 8 + 1 / 24)) ** 2
    x_dense = np.linalg.solve(A, b.reshape(-1))
    x, iters, tr, conv = oracle.cg(dims, fat, lng, mass, b, tol=1e-10)
    assert conv and tr <= 1e-10
    assert np.linalg.norm(x.reshape(-1) - x_dense) <= 1e-9 * np.linalg.norm(x_dense)
    # CG iteration bound from the condition number: sqrt(kappa)/2 ln(2/tol)
    kappa = ev[-1] / ev[0]
    assert iters <= 0.5 * np.sqrt(kappa) * np.log(2 / 1e-10) + 5


def test_cg_finite_termination_free_field():
    # free field on 4^3 x 8: 8 distinct eigenvalues, so exact CG ends in <= 8 steps
    dims = (4, 4, 4, 8)
    mass = 0.1
    fat, lng = free_gauge(dims)
    ref = free_even_spectrum(dims, mass)
    n_distinct = len(np.unique(np.round(ref, 9)))
    assert n_distinct == 8
    b = synth.make_sources(dims, 1, 11)[0]
    x, iters, tr, conv, hist = oracle.cg(dims, fat, lng, mass, b, tol=1e-12, history=True)
    assert conv and iters <= n_distinct + 1
    assert tr < 1e-11


def test_cg_solution_gauge_covariant():
    dims = (4, 4, 4, 8)
    mass = 0.1
    U = synth.thin_links(dims, 0.3, 21)
    g = synth.random_gauge_transform(dims, 22)
    fat, lng = synth.fat_long_from_thin(U)
    fat_g, lng_g = synth.fat_long_from_thin(synth.gauge_transform_thin(U, g))
    b = synth.make_sources(dims, 1, 23)[0]
    c = lex_coords(dims)
    g_e = g[(c.sum(axis=1) % 2) == 0]
    x, it1, tr1, _ = oracle.cg(dims, fat, lng, mass, b, tol=1e-12)
    xg, it2, tr2, _ = oracle.cg(dims, fat_g, lng_g, mass, np.einsum("sij,sj->si", g_e, b), tol=1e-12)
    assert np.linalg.norm(xg - np.einsum("sij,sj->si", g_e, x)) <= 1e-9 * np.linalg.norm(x)
    assert abs(it1 - it2) <= 1


def test_true_residual_of_exact_solution_and_zero_source():
    dims = (4, 4, 4, 8)
    fat, lng = synth.make_gauge(dims, 0.3, 31)
    half = int(np.prod(dims)) // 2
    b = np.zeros((half, 3), dtype=np.complex128)
    x, iters, tr, conv = oracle.cg(dims, fat, lng, 0.1, b)
    assert conv and iters == 0 and np.all(x == 0)
    rng = np.random.default_rng(0)
    x0 = rng.standard_normal((half, 3)) + 1j * rng.standard_normal((half, 3))
    b = oracle.apply_A(dims, fat, lng, 0.1, x0)
    assert oracle.true_residual(dims, fat, lng, 0.1, b, x0) < 1e-15


def test_oracle_rejects_odd_dims():
    with pytest.raises(ValueError):
        oracle.dslash((5, 4, 4, 4), np.zeros((320, 4, 3, 3)), np.zeros((320, 4, 3, 3)), 0, np.zeros((160, 3)))


def _numpy_dslash_full(dims, fat, lng, psi):
    """D on the whole lattice with whole-lattice shifts: an implementation independent of the
    oracle's site loop.  fat, lng (V, 4, 3, 3); psi (V, 3) in lexicographic order."""
    X, Y, Z, T = dims
    F = fat.reshape(T, Z, Y, X, 4, 3, 3)
    L = lng.reshape(T, Z, Y, X, 4, 3, 3)
    P = psi.reshape(T, Z, Y, X, 3)
    t, z, y, x = np.meshgrid(np.arange(T), np.arange(Z), np.arange(Y), np.arange(X), indexing="ij")
    eta = [np.ones_like(x), (-1.0) ** x, (-1.0) ** (x + y), (-1.0) ** (x + y + z)]
    out = np.zeros_like(P)
    for mu in range(4):
        axis = 3 - mu

        def shifted(A, h):
            # A(x + h mu), periodic (the fermion boundary sign is bc below)
            return np.roll(A, -h, axis=axis)

        def bc(h):
            # -1 where x + h mu leaves [0, T) in time (only for mu = t)
            if mu != 3:
                return np.ones_like(t)
            u = t + h
            return np.where((u < 0) | (u >= T), -1.0, 1.0)

        Fm, Lm = F[..., mu, :, :], L[..., mu, :, :]
        dag = lambda A: np.conj(np.swapaxes(A, -1, -2))
        term = np.einsum("...ab,...b->...a", Fm, shifted(P, 1)) * bc(1)[..., None]
        term -= np.einsum("...ab,...b->...a", dag(shifted(Fm, -1)), shifted(P, -1)) * bc(-1)[..., None]
        term += np.einsum("...ab,...b->...a", Lm, shifted(P, 3)) * bc(3)[..., None]
        term -= np.einsum("...ab,...b->...a", dag(shifted(Lm, -3)), shifted(P, -3)) * bc(-3)[..., None]
        out += eta[mu][..., None] * term
    return out.reshape(-1, 3)


@pytest.mark.parametrize("dims", [(4, 4, 4, 8), (6, 4, 4, 8)])
def test_dslash_matches_independent_numpy_form(dims):
    # random links and vectors: the oracle's per-site loop against whole-lattice shifts
    fat, lng = synth.make_gauge(dims, 0.5, 17)
    V = int(np.prod(dims))
    rng = np.random.Generator(np.random.PCG64(18))
    psi = rng.standard_normal((V, 3)) + 1j * rng.standard_normal((V, 3))
    c = lex_coords(dims)
    par = c.sum(axis=1) % 2
    for out_parity in (0, 1):
        src = psi[par == 1 - out_parity]
        got = oracle.dslash(dims, fat, lng, out_parity, src)
        # the numpy form on the whole lattice with the other parity zeroed
        masked = np.where((par == 1 - out_parity)[:, None], psi, 0)
        want = _numpy_dslash_full(dims, fat, lng, masked)[par == out_parity]
        assert np.abs(got - want).max() < 1e-13 * np.abs(want).max()


def _numpy_dense_A(dims, fat, lng, mass):
    """Dense A = 4m^2 - D_eo D_oe on even sites, built column by column from the
    whole-lattice numpy form of D above (no oracle code involved)."""
    c = lex_coords(dims)
    par = c.sum(axis=1) % 2
    V = int(np.prod(dims))
    even, odd = par == 0, par == 1
    n = V // 2 * 3
    A = np.empty((n, n), dtype=np.complex128)
    e = np.zeros((V, 3), dtype=np.complex128)
    for k in range(n):
        e[:] = 0
        e[np.nonzero(even)[0][k // 3], k % 3] = 1.0
        t = _numpy_dslash_full(dims, fat, lng, e)  # D_oe e on odd sites
        t = np.where(odd[:, None], t, 0)
        u = _numpy_dslash_full(dims, fat, lng, t)  # D_eo t on even sites
        A[:, k] = (4 * mass**2 * e - u)[even].reshape(-1)
    return A


def test_true_residual_scale_pinned_by_dense_numpy_residual():
    # The relative true residual decides every full-size solver parity test, so
    # its scale is pinned against numpy on a dense A built without the oracle:
    #   x = 0          -> exactly 1 (|b| / |b|)
    #   x = c x_dense  -> |1 - c| (b - A c x = (1 - c) b)
    #   random x       -> ||b - A x|| / ||b|| from numpy
    # A dropped square root (|r|^2/|b|^2) or a |b|^2 denominator fails each.
    dims, m = (4, 4, 4, 8), 0.1
    fat, lng = synth.make_gauge(dims, 0.3, 41)
    half = int(np.prod(dims)) // 2
    A = _numpy_dense_A(dims, fat, lng, m)
    b = synth.make_sources(dims, 1, 42)[0]
    assert oracle.true_residual(dims, fat, lng, m, b, np.zeros_like(b)) == 1.0
    x_dense = np.linalg.solve(A, b.reshape(-1)).reshape(half, 3)
    for c in (0.5, 0.9, 1.1):
        tr = oracle.true_residual(dims, fat, lng, m, b, c * x_dense)
        assert abs(tr - abs(1 - c)) <= 1e-12, (c, tr)
    rng = np.random.default_rng(43)
    for scale in (1e-3, 1.0, 1e3):
        x = scale * (rng.standard_normal((half, 3)) + 1j * rng.standard_normal((half, 3)))
        want = np.linalg.norm(b.reshape(-1) - A @ x.reshape(-1)) / np.linalg.norm(b.reshape(-1))
        got = oracle.true_residual(dims, fat, lng, m, b, x)
        assert abs(got - want) <= 1e-14 * want, (scale, got, want)
    # the scale of b cancels: the residual is relative
    tr1 = oracle.true_residual(dims, fat, lng, m, b, 0.7 * x_dense)
    tr2 = oracle.true_residual(dims, fat, lng, m, 5.0 * b, 3.5 * x_dense)
    assert abs(tr1 - 0.3) <= 1e-12 and abs(tr2 - 0.3) <= 1e-12
