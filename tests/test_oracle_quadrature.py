"""Pins for the oracle's quadratures against exact integrals."""
import math

import numpy as np
import pytest

from oracle import double_gauss, azimuths, frequency_grid, directions_3d


@pytest.mark.parametrize("n_mu", [2, 4, 8, 12, 16])
def test_double_gauss_exact_on_each_hemisphere(n_mu):
    mu, w = double_gauss(n_mu)
    assert np.all(np.diff(mu) > 0) and np.all(mu != 0)
    assert abs(w.sum() - 1.0) < 1e-15
    pos = mu > 0
    # n_mu/2 Gauss nodes per hemisphere integrate degree <= n_mu - 1 exactly:
    # int_0^1 mu^p dmu = 1/(p+1), weights on (0,1) sum to 1/2.
    for p in range(n_mu):
        assert abs(2.0 * np.dot(w[pos], mu[pos] ** p) - 1.0 / (p + 1)) < 1e-14
    assert np.allclose(mu[~pos], -mu[pos][::-1], rtol=0, atol=1e-16)


def test_azimuths_cancel_low_harmonics():
    for n_az in (4, 8, 16):
        phi, w = azimuths(n_az)
        assert abs(w.sum() - 1) < 1e-15
        for m in range(1, n_az):
            assert abs(np.dot(w, np.cos(m * phi))) < 1e-14
            assert abs(np.dot(w, np.sin(m * phi))) < 1e-14


def test_directions_second_moments():
    om, w = directions_3d(8, 8)
    assert np.allclose(np.linalg.norm(om, axis=1), 1.0, atol=1e-15)
    assert abs(w.sum() - 1) < 1e-15
    second = np.einsum("o,oi,oj->ij", w, om, om)
    assert np.allclose(second, np.eye(3) / 3.0, atol=1e-15)
    assert np.allclose(om.T @ w, 0.0, atol=1e-16)


@pytest.mark.parametrize("n_nu", [5, 21, 32, 48])
def test_frequency_profile(n_nu):
    x, w, phi = frequency_grid(n_nu, 5.0)
    assert abs(np.dot(w, phi) - 1.0) < 1e-15
    # trapezoid of a Gaussian on [-5, 5]: renormalisation is tiny
    cont = np.exp(-x * x) / math.sqrt(math.pi)
    if n_nu >= 16:
        assert np.max(np.abs(phi / cont - 1.0)) < 1e-3
    assert np.allclose(phi, phi[::-1], rtol=1e-15)


def test_monochromatic_frequency():
    x, w, phi = frequency_grid(1, 5.0)
    assert x.tolist() == [0.0] and w.tolist() == [1.0] and phi.tolist() == [1.0]
