"""Pins for the oracle of the paper's one-colour four-fermion operator, Eq. (1) of
the "GTX Titan Black" section: facts fixed by the algebra, not by the oracle.

* spin-taste matrices (1/4) Tr[gamma_A^dag gamma_S gamma_B gamma_F^dag]: the same in a
  second, independently written Dirac representation (numpy, Dirac-Pauli), the
  identity for S = F = 0, one entry of modulus one per row at B = A ^ S ^ F, and the
  representation property M(S, F) = M(S, 0) M(0, F)
* path-averaged links: unit links give 1; a uniform abelian field exp(i theta_mu) gives
  exp(i theta . (D - A)) on every path; one step is the link or its adjoint; the
  reverse pair is the adjoint; gauge covariance; an independent numpy recursion
* the contraction: gauge invariance; the closed form for unit links and propagators that
  are site scalars times fixed colour matrices; the exchange of the two bilinears;
  an independent numpy evaluation of the sum over corners
"""
import itertools

import numpy as np
import pytest

import oracle
import synth

# ---------------------------------------------------------------------------
# an independent Dirac representation (Dirac-Pauli, Euclidean) in numpy
# ---------------------------------------------------------------------------
_s = [np.array([[0, 1], [1, 0]], complex), np.array([[0, -1j], [1j, 0]]), np.array([[1, 0], [0, -1]], complex)]
_Z2 = np.zeros((2, 2), complex)
_I2 = np.eye(2, dtype=complex)
GAMMA_DP = [np.block([[_Z2, -1j * _s[k]], [1j * _s[k], _Z2]]) for k in range(3)] + \
           [np.block([[_I2, _Z2], [_Z2, -_I2]])]


def gamma_of(mask, gam=GAMMA_DP):
    g = np.eye(4, dtype=complex)
    for mu in range(4):
        if mask >> mu & 1:
            g = g @ gam[mu]
    return g


def spin_taste_np(S, F, gam=GAMMA_DP):
    M = np.empty((16, 16), complex)
    gS, gFd = gamma_of(S, gam), gamma_of(F, gam).conj().T
    for A in range(16):
        gAd = gamma_of(A, gam).conj().T
        for B in range(16):
            M[A, B] = 0.25 * np.trace(gAd @ gS @ gamma_of(B, gam) @ gFd)
    return M


def test_dirac_pauli_matrices_form_the_euclidean_algebra():
    for mu in range(4):
        assert np.allclose(GAMMA_DP[mu], GAMMA_DP[mu].conj().T)
        for nu in range(4):
            ac = GAMMA_DP[mu] @ GAMMA_DP[nu] + GAMMA_DP[nu] @ GAMMA_DP[mu]
            assert np.allclose(ac, 2 * (mu == nu) * np.eye(4))


def test_spin_taste_matches_a_second_representation():
    # the trace is representation independent: an error in the oracle's gamma
    # matrices (a commuting pair, a wrong sign) or in its trace formula shows here
    for S, F in itertools.product(range(16), range(16)):
        assert np.array_equal(np.round(oracle.spin_taste(S, F), 12), np.round(spin_taste_np(S, F), 12)), (S, F)


def test_spin_taste_structure():
    assert np.array_equal(oracle.spin_taste(0, 0), np.eye(16))
    for S, F in itertools.product(range(16), range(16)):
        M = oracle.spin_taste(S, F)
        assert np.abs(M.imag).max() == 0
        for A in range(16):
            row = M[A]
            nz = np.nonzero(row)[0]
            assert list(nz) == [A ^ S ^ F] and abs(row[A ^ S ^ F]) == 1.0
        assert np.array_equal(M, oracle.spin_taste(S, 0) @ oracle.spin_taste(0, F))


# ---------------------------------------------------------------------------
# path-averaged links
# ---------------------------------------------------------------------------
def lex_of(dims, c):
    X, Y, Z, T = dims
    return c[0] + X * (c[1] + Y * (c[2] + Z * c[3]))


def corner_of(z, A):
    return [2 * z[mu] + (A >> mu & 1) for mu in range(4)]


def link_avg_np(dims, U, z, A, D):
    """U_AD by its first step: (1/d) sum_mu L(A, mu) U_{A^mu, D}, written separately from the oracle."""
    if A == D:
        return np.eye(3, dtype=complex)
    diff = [mu for mu in range(4) if (A ^ D) >> mu & 1]
    acc = np.zeros((3, 3), complex)
    for mu in diff:
        if A >> mu & 1:
            L = U[lex_of(dims, corner_of(z, A ^ (1 << mu))), mu].conj().T
        else:
            L = U[lex_of(dims, corner_of(z, A)), mu]
        acc += L @ link_avg_np(dims, U, z, A ^ (1 << mu), D)
    return acc / len(diff)


def test_link_average_unit_and_abelian_fields():
    dims = (4, 4, 4, 6)
    V = int(np.prod(dims))
    U1 = synth.unit_links(dims).reshape(V, 4, 3, 3)
    theta = np.array([0.3, -0.7, 1.1, 0.45])
    Uab = np.zeros((V, 4, 3, 3), complex)
    for mu in range(4):
        Uab[:, mu] = np.exp(1j * theta[mu]) * np.eye(3)
    for z in ([0, 0, 0, 0], [1, 1, 0, 2]):
        for A, D in itertools.product(range(16), range(16)):
            assert np.allclose(oracle.link_average(dims, U1, z, A, D), np.eye(3), atol=1e-15)
            step = np.array([(D >> mu & 1) - (A >> mu & 1) for mu in range(4)])
            assert np.allclose(oracle.link_average(dims, Uab, z, A, D), np.exp(1j * theta @ step) * np.eye(3),
                               atol=1e-14), (A, D)


def test_link_average_steps_reverse_and_covariance():
    dims = (4, 4, 4, 4)
    V = int(np.prod(dims))
    U = synth.thin_links(dims, 0.6, 7).reshape(V, 4, 3, 3)
    g = synth.random_gauge_transform(dims, 8)
    Ug = synth.gauge_transform_thin(synth.thin_links(dims, 0.6, 7), g).reshape(V, 4, 3, 3)
    z = [1, 0, 1, 1]
    for A in range(16):
        for mu in range(4):
            if not A >> mu & 1:
                s = lex_of(dims, corner_of(z, A))
                assert np.array_equal(oracle.link_average(dims, U, z, A, A | 1 << mu), U[s, mu])
                assert np.allclose(oracle.link_average(dims, U, z, A | 1 << mu, A), U[s, mu].conj().T, atol=0)
    for A, D in itertools.product(range(16), range(16)):
        uad = oracle.link_average(dims, U, z, A, D)
        assert np.allclose(oracle.link_average(dims, U, z, D, A), uad.conj().T, atol=1e-15)
        assert np.allclose(uad, link_avg_np(dims, U, z, A, D), atol=1e-14)
        ga, gd = g[lex_of(dims, corner_of(z, A))], g[lex_of(dims, corner_of(z, D))]
        assert np.allclose(oracle.link_average(dims, Ug, z, A, D), ga @ uad @ gd.conj().T, atol=1e-13)


# ---------------------------------------------------------------------------
# the contraction
# ---------------------------------------------------------------------------
def random_props(dims, seed, n=4):
    V = int(np.prod(dims))
    rng = np.random.Generator(np.random.PCG64(seed))
    return [rng.standard_normal((V, 3, 3)) + 1j * rng.standard_normal((V, 3, 3)) for _ in range(n)]


def npr_np(dims, U, G, op, z):
    """The sum over the sixteen corners A, B, C, D written out with numpy's own spin-taste
    matrices and link averages."""
    S1, F1, S2, F2 = op
    M1, M2 = spin_taste_np(S1, F1), spin_taste_np(S2, F2)
    V = np.zeros((3, 3, 3, 3), complex)
    sites = [lex_of(dims, corner_of(z, A)) for A in range(16)]
    eps = [(-1) ** sum(corner_of(z, A)) for A in range(16)]
    Uav = {(A, D): link_avg_np(dims, U, z, A, D) for A in range(16) for D in range(16)}
    for A, B, C, D in itertools.product(range(16), repeat=4):
        w = M1[A, B] * M2[C, D]
        if w == 0:
            continue
        X = G[0][sites[A]].conj().T @ Uav[A, D] @ G[3][sites[D]]
        Y = G[2][sites[C]].conj().T @ Uav[C, B] @ G[1][sites[B]]
        V += w * eps[A] * eps[C] * np.einsum("ad,cb->abcd", X, Y)
    return V


def hyper_index(dims, z):
    hx, hy, hz = dims[0] // 2, dims[1] // 2, dims[2] // 2
    return z[0] + hx * (z[1] + hy * (z[2] + hz * z[3]))


OPS = [(0, 0, 0, 0), (15, 15, 15, 15), (1, 15, 2, 15), (6, 9, 6, 9), (3, 0, 12, 5)]


def test_contraction_matches_numpy_sum_over_corners():
    dims = (4, 4, 4, 4)
    V = int(np.prod(dims))
    U = synth.thin_links(dims, 0.5, 11).reshape(V, 4, 3, 3)
    G = random_props(dims, 12)
    zs = [[0, 0, 0, 0], [1, 1, 0, 1]]
    got = oracle.npr_fourfermion(dims, U, G, OPS[:3], zs=[hyper_index(dims, z) for z in zs])
    for k, op in enumerate(OPS[:3]):
        for iz, z in enumerate(zs):
            want = npr_np(dims, U, G, op, z)
            assert np.abs(got[k, iz] - want).max() <= 1e-12 * np.abs(want).max(), (op, z)


def test_contraction_gauge_invariant():
    dims = (4, 4, 4, 4)
    V = int(np.prod(dims))
    Ut = synth.thin_links(dims, 0.5, 13)
    g = synth.random_gauge_transform(dims, 14)
    U = Ut.reshape(V, 4, 3, 3)
    Ug = synth.gauge_transform_thin(Ut, g).reshape(V, 4, 3, 3)
    G = random_props(dims, 15)
    Gg = [np.einsum("sij,sjk->sik", g, x) for x in G]  # the propagators' sink index rotates
    a = oracle.npr_fourfermion(dims, U, G, OPS)
    b = oracle.npr_fourfermion(dims, Ug, Gg, OPS)
    assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()


def test_contraction_closed_form_for_unit_links_and_factorised_propagators():
    # U = 1 and G_f(x) = phi_f(x) W_f: every U_AD is 1, so
    #   V[a1, a2, a3, a4] = K (W1^dag W4)[a1, a4] (W3^dag W2)[a3, a2],
    #   K = sum_{ABCD} M1_AB M2_CD eps_A eps_C conj(phi1_A) phi4_D conj(phi3_C) phi2_B
    dims = (4, 4, 4, 4)
    V = int(np.prod(dims))
    U = synth.unit_links(dims).reshape(V, 4, 3, 3)
    rng = np.random.Generator(np.random.PCG64(16))
    phi = [rng.standard_normal(V) + 1j * rng.standard_normal(V) for _ in range(4)]
    W = [rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3)) for _ in range(4)]
    G = [phi[f][:, None, None] * W[f][None] for f in range(4)]
    z = [1, 0, 1, 0]
    got = oracle.npr_fourfermion(dims, U, G, OPS, zs=[hyper_index(dims, z)])
    sites = [lex_of(dims, corner_of(z, A)) for A in range(16)]
    eps = np.array([(-1) ** sum(corner_of(z, A)) for A in range(16)])
    P = [p[sites] for p in phi]
    colour = np.einsum("ad,cb->abcd", W[0].conj().T @ W[3], W[2].conj().T @ W[1])
    for k, (S1, F1, S2, F2) in enumerate(OPS):
        M1, M2 = spin_taste_np(S1, F1), spin_taste_np(S2, F2)
        K = np.einsum("ab,cd,a,c,a,d,c,b->", M1, M2, eps, eps, P[0].conj(), P[3], P[2].conj(), P[1])
        assert np.abs(got[k, 0] - K * colour).max() <= 1e-12 * np.abs(K * colour).max(), (S1, F1, S2, F2)


def test_contraction_exchange_of_bilinears():
    # swapping the bilinears (propagators 1,2 <-> 3,4 and the two spin-tastes)
    # permutes the source colours: V'[b1, b2, b3, b4] = V[b3, b4, b1, b2]
    dims = (4, 4, 4, 4)
    V = int(np.prod(dims))
    U = synth.thin_links(dims, 0.5, 17).reshape(V, 4, 3, 3)
    G = random_props(dims, 18)
    ops = [(3, 0, 12, 5), (1, 15, 2, 15)]
    a = oracle.npr_fourfermion(dims, U, G, ops)
    b = oracle.npr_fourfermion(dims, U, [G[2], G[3], G[0], G[1]], [(o[2], o[3], o[0], o[1]) for o in ops])
    assert np.abs(b - a.transpose(0, 1, 4, 5, 2, 3)).max() <= 1e-12 * np.abs(a).max()


def test_contraction_rejects_bad_labels():
    dims = (4, 4, 4, 4)
    V = int(np.prod(dims))
    with pytest.raises(ValueError):
        oracle.npr_fourfermion(dims, np.zeros((V, 4, 3, 3)), random_props(dims, 1), [(16, 0, 0, 0)])
