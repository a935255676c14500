"""The seeded input generators against the recipe they state (CPU only).

The serving stream is a Poisson process (exponential gaps of mean 1/rate) over
the four lattices with weights 0.4/0.3/0.2/0.1, masses uniform in
[0.005, 0.1] and 1..12 right-hand sides; sources are iid N(0, 1) in each real
component; the thin links exp(i eps H) approach 1 + i eps H for small eps.
Statistical checks use 5-sigma bounds on 20 000 draws.
"""
import numpy as np
import pytest

import synth

N = 20000


@pytest.fixture(scope="module")
def trace():
    return synth.serving_trace(N, rate=50.0)


def test_serving_arrivals_are_poisson(trace):
    t = np.array([r["arrival"] for r in trace])
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert np.all(gaps > 0)
    mean = 1.0 / 50.0
    assert abs(gaps.mean() - mean) < 5 * mean / np.sqrt(N)
    # exponential: the standard deviation equals the mean, P(gap > mean) = 1/e
    assert abs(gaps.std() - mean) < 0.05 * mean
    p = np.mean(gaps > mean)
    assert abs(p - np.exp(-1)) < 5 * np.sqrt(np.exp(-1) * (1 - np.exp(-1)) / N)


def test_serving_lattice_weights_masses_and_columns(trace):
    lat = np.array([r["lattice"] for r in trace])
    for k, w in enumerate(synth.SERVING_WEIGHTS):
        f = np.mean(lat == k)
        assert abs(f - w) < 5 * np.sqrt(w * (1 - w) / N), (k, f)
    m = np.array([r["mass"] for r in trace])
    assert m.min() >= 0.005 and m.max() <= 0.1
    assert abs(m.mean() - 0.0525) < 5 * (0.095 / np.sqrt(12)) / np.sqrt(N)
    n = np.array([r["nrhs"] for r in trace])
    assert set(np.unique(n)) == set(range(1, 13))
    assert len({r["seed"] for r in trace}) == N  # every request draws its own source


def test_serving_trace_is_seeded():
    a = synth.serving_trace(50, rate=15.0, seed=3)
    assert a == synth.serving_trace(50, rate=15.0, seed=3)
    assert a != synth.serving_trace(50, rate=15.0, seed=4)


def test_sources_are_standard_complex_gaussians():
    dims = (8, 8, 8, 8)
    b = synth.make_sources(dims, 4, 11)
    assert b.shape == (4, 2048, 3) and b.dtype == np.complex128
    z = np.concatenate([b.real.ravel(), b.imag.ravel()])
    n = z.size
    assert abs(z.mean()) < 5 / np.sqrt(n)
    assert abs(z.var() - 1) < 5 * np.sqrt(2 / n)
    assert abs(np.mean(b.real * b.imag)) < 5 / np.sqrt(n / 2)  # real and imaginary parts uncorrelated
    assert np.array_equal(b, synth.make_sources(dims, 4, 11))
    assert not np.array_equal(b, synth.make_sources(dims, 4, 12))


def test_thin_links_small_eps_limit():
    # exp(i eps H) = 1 + i eps H + O(eps^2): the generator's H is sum_a h_a lambda_a / 2
    dims, eps = (4, 4, 4, 4), 1e-4
    U = synth.thin_links(dims, eps, 9).reshape(-1, 3, 3)
    rng = np.random.Generator(np.random.PCG64(9))
    h = np.stack([rng.standard_normal((4, 4, 4, 4, 8)) for _ in range(4)]).reshape(-1, 8)
    H = np.einsum("na,aij->nij", h, synth.gell_mann()) * 0.5
    lin = np.eye(3) + 1j * eps * H
    assert np.max(np.abs(U - lin)) < 10 * eps**2 * np.max(np.abs(H)) ** 2
    assert np.max(np.abs(U - lin)) > 0  # the quadratic term is there
