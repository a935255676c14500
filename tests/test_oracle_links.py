"""Pins for the oracle's asqtad link construction (fat and long links from thin links).

The oracle sums the asqtad paths one by one.  These tests tie it to facts that
do not come from that sum:

* free field: every path is the identity, so the fat link is the sum of the
  coefficients times the path counts (9/8 at u0 = 1) and the long link c_N
* a uniform abelian flux B in one plane: each path contributes the phase of the
  area it encloses, giving a closed form in cos(qB) and cos(2qB) per colour charge
* gauge covariance: F[U^g](x) = g(x) F[U](x) g(x+mu)^dag, L likewise with x+3mu
* an independent evaluation as nested staples, T_nu(X)(y) = U_nu(y) X(y+nu) U_nu(y+mu)^dag
  applied level by level with whole-lattice shifts
* the long link at u0 = 1 equals the workload recipe's -(1/24) U U U
"""
import numpy as np
import pytest

import oracle
import synth


def coeffs(u0):
    """(c1, c3, c5, c7, cL, cN) of the asqtad action with tadpole factor u0."""
    return (5 / 8, 1 / 16 / u0**2, 1 / 64 / u0**4, 1 / 384 / u0**6, -1 / 16 / u0**4, -1 / 24 / u0**2)


def lattice_links(U):
    """(T, Z, Y, X, 4, 3, 3) -> (V, 4, 3, 3) in lexicographic order."""
    return U.reshape(-1, 4, 3, 3)


@pytest.mark.parametrize("u0", [1.0, 0.85])
def test_free_field_normalisation(u0):
    dims = (4, 4, 4, 6)
    c1, c3, c5, c7, cL, cN = coeffs(u0)
    fat, lng = oracle.asqtad_links(dims, lattice_links(synth.unit_links(dims)), u0)
    # 1 one-link path, 6 three-staples, 24 five-staples, 48 seven-staples, 6 Lepage paths
    k = c1 + 6 * c3 + 24 * c5 + 48 * c7 + 6 * cL
    if u0 == 1.0:
        assert k == pytest.approx(9 / 8, abs=1e-15)
    eye = np.eye(3)
    assert np.abs(fat - k * eye).max() < 1e-14
    assert np.abs(lng - cN * eye).max() < 1e-15


def abelian_flux_links(dims, mu0, nu0, k):
    """U_nu0(x) = diag(exp(i q B x_mu0)), q = (1, 1, -2), B = 2 pi k / L_mu0; other links 1.

    The field strength is B in the (mu0, nu0) plane and zero elsewhere; the
    wrap of x_mu0 is smooth because B L_mu0 is a multiple of 2 pi.
    """
    X, Y, Z, T = dims
    B = 2 * np.pi * k / dims[mu0]
    q = np.array([1.0, 1.0, -2.0])
    U = synth.unit_links(dims)
    coords = np.meshgrid(np.arange(T), np.arange(Z), np.arange(Y), np.arange(X), indexing="ij")
    x_mu0 = coords[3 - mu0]
    for a in range(3):
        U[..., nu0, a, a] = np.exp(1j * q[a] * B * x_mu0)
    return U, B, q


@pytest.mark.parametrize("mu0,nu0,k,u0", [(0, 2, 1, 1.0), (3, 1, 1, 0.9), (1, 3, 2, 1.0)])
def test_uniform_abelian_flux_closed_form(mu0, nu0, k, u0):
    dims = (6, 4, 4, 8) if mu0 != 1 else (4, 6, 4, 8)
    U, B, q = abelian_flux_links(dims, mu0, nu0, k)
    c1, c3, c5, c7, cL, cN = coeffs(u0)
    fat, lng = oracle.asqtad_links(dims, lattice_links(U), u0)
    Ul = lattice_links(U)
    c, c2 = np.cos(q * B), np.cos(2 * q * B)
    # in the flux plane: a staple (or 5-, 7-staple) encloses area +-1 when it steps
    # across the plane's other axis, a Lepage path area +-2; out of the plane no
    # path encloses flux
    k_in = c1 + c3 * (4 + 2 * c) + c5 * (8 + 16 * c) + c7 * 48 * c + cL * (4 + 2 * c2)
    k_out = c1 + 6 * c3 + 24 * c5 + 48 * c7 + 6 * cL
    for mu in range(4):
        kmu = k_in if mu in (mu0, nu0) else np.full(3, k_out)
        want = Ul[:, mu] * kmu[None, None, :]  # diagonal links: scale column a by K(q_a)
        assert np.abs(fat[:, mu] - want).max() < 1e-13, mu
        # the long link along nu0 stays at fixed x_mu0: phase 3 q B x_mu0
        want_l = cN * Ul[:, mu] @ Ul[:, mu] @ Ul[:, mu]
        assert np.abs(lng[:, mu] - want_l).max() < 1e-14, mu


def shift(A, mu, s):
    """A(x + s mu) for fields shaped (T, Z, Y, X, ...)."""
    return np.roll(A, -s, axis=3 - mu)


def dag(A):
    return np.conj(np.swapaxes(A, -1, -2))


def step_link(U, d):
    """The link from y to y + d (d = +-(axis + 1)) as a field over y."""
    a = abs(d) - 1
    return U[..., a, :, :] if d > 0 else dag(shift(U[..., a, :, :], a, -1))


def staple(U, mu, d, Xf):
    """T_d(X)(y) = W_d(y) X(y + d) W_d(y + mu)^dag, W_d the link from y to y + d."""
    W = step_link(U, d)
    a, s = abs(d) - 1, (1 if d > 0 else -1)
    return W @ shift(Xf, a, s) @ dag(shift(W, mu, 1))


def nested_fat(U, u0):
    """F_mu = c1 U_mu + sum_nu T_nu(c3 U_mu + cL T_nu(U_mu) + sum_rho T_rho(c5 U_mu + c7 sum_sigma T_sigma(U_mu)))."""
    c1, c3, c5, c7, cL, _ = coeffs(u0)
    out = np.empty_like(U)
    signed = [d for a in range(4) for d in (a + 1, -(a + 1))]
    for mu in range(4):
        Um = U[..., mu, :, :]
        F = c1 * Um
        for nu in signed:
            if abs(nu) - 1 == mu:
                continue
            inner = c3 * Um + cL * staple(U, mu, nu, Um)
            for rho in signed:
                if abs(rho) - 1 in (mu, abs(nu) - 1):
                    continue
                core = c5 * Um
                for sg in signed:
                    if abs(sg) - 1 in (mu, abs(nu) - 1, abs(rho) - 1):
                        continue
                    core = core + c7 * staple(U, mu, sg, Um)
                inner = inner + staple(U, mu, rho, core)
            F = F + staple(U, mu, nu, inner)
        out[..., mu, :, :] = F
    return lattice_links(out)


@pytest.mark.parametrize("dims,u0", [((4, 4, 4, 6), 1.0), ((6, 4, 4, 4), 0.87)])
def test_nested_staple_evaluation(dims, u0):
    U = synth.thin_links(dims, 0.5, seed=31)
    fat, _ = oracle.asqtad_links(dims, lattice_links(U), u0)
    want = nested_fat(U, u0)
    assert np.abs(fat - want).max() < 1e-13 * np.abs(want).max()


def test_gauge_covariance_of_links():
    dims = (4, 6, 4, 4)
    U = synth.thin_links(dims, 0.4, seed=5)
    g = synth.random_gauge_transform(dims, seed=6)
    Ug = synth.gauge_transform_thin(U, g)
    fat, lng = oracle.asqtad_links(dims, lattice_links(U), 0.9)
    fat_g, lng_g = oracle.asqtad_links(dims, lattice_links(Ug), 0.9)
    G = g.reshape(dims[3], dims[2], dims[1], dims[0], 3, 3)
    for mu in range(4):
        g1 = shift(G, mu, 1).reshape(-1, 3, 3)
        g3 = shift(G, mu, 3).reshape(-1, 3, 3)
        g0 = g.reshape(-1, 3, 3)
        assert np.abs(fat_g[:, mu] - g0 @ fat[:, mu] @ dag(g1)).max() < 1e-13
        assert np.abs(lng_g[:, mu] - g0 @ lng[:, mu] @ dag(g3)).max() < 1e-14


def test_long_link_equals_workload_recipe_at_u0_one():
    dims = (4, 4, 6, 4)
    U = synth.thin_links(dims, 0.3, seed=8)
    _, lng = oracle.asqtad_links(dims, lattice_links(U), 1.0)
    _, want = synth.fat_long_from_thin(U)
    assert np.abs(lng - want).max() < 1e-15


def test_listed_sites_match_full_lattice():
    dims = (4, 4, 4, 6)
    U = lattice_links(synth.thin_links(dims, 0.3, seed=9))
    fat, lng = oracle.asqtad_links(dims, U, 0.95)
    sites = np.array([0, 383, 17, 200, 17])
    fs, ls = oracle.asqtad_links(dims, U, 0.95, sites=sites)
    assert np.array_equal(fs, fat[sites]) and np.array_equal(ls, lng[sites])


def test_link_construction_rejects_bad_arguments():
    dims = (4, 4, 4, 4)
    U = lattice_links(synth.unit_links(dims))
    with pytest.raises(ValueError):
        oracle.asqtad_links(dims, U, 0.0)
    with pytest.raises(ValueError):
        oracle.asqtad_links(dims, U, 1.0, sites=[0, 256])


def test_plaquette_free_field_and_flux():
    # unit links: every plaquette is the identity; a uniform flux B in one plane
    # gives (2 cos B + cos 2B) / 3 for the charges (1, 1, -2) in that plane, 1 in the others
    dims = (6, 4, 4, 8)
    assert oracle.plaquette(dims, lattice_links(synth.unit_links(dims))) == pytest.approx(1.0, abs=1e-15)
    U, B, q = abelian_flux_links(dims, 0, 2, 1)
    want = (5 + (2 * np.cos(B) + np.cos(2 * B)) / 3) / 6
    assert oracle.plaquette(dims, lattice_links(U)) == pytest.approx(want, abs=1e-14)


def test_plaquette_gauge_invariant():
    dims = (4, 6, 4, 4)
    U = synth.thin_links(dims, 0.4, seed=5)
    g = synth.random_gauge_transform(dims, seed=6)
    p = oracle.plaquette(dims, lattice_links(U))
    pg = oracle.plaquette(dims, lattice_links(synth.gauge_transform_thin(U, g)))
    assert 0.5 < p < 1.0
    assert pg == pytest.approx(p, abs=1e-13)
