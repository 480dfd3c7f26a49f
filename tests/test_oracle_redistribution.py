"""Pins for the oracle's scattering kernels: symmetry, normalisation (photon
conservation, paper Sec. 2), PRD marginals and the dipole azimuthal average."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import (double_gauss, directions_3d, frequency_grid, dipole_1d,
                    dipole_3d, prd_frequency_kernel, legendre_phase, Problem)


def test_dipole_1d_is_azimuthal_average_of_3d():
    # average 3/4 (1 + cos^2 Theta) over the azimuth difference numerically
    mu = np.array([-0.9, -0.3, 0.2, 0.7])
    n = 4096
    dphi = (np.arange(n) + 0.5) * 2 * math.pi / n
    ref = np.zeros((4, 4))
    for i, a in enumerate(mu):
        for j, b in enumerate(mu):
            cos_t = a * b + math.sqrt(1 - a * a) * math.sqrt(1 - b * b) * np.cos(dphi)
            ref[i, j] = np.mean(0.75 * (1 + cos_t ** 2))
    assert np.allclose(dipole_1d(mu), ref, rtol=0, atol=1e-14)


@pytest.mark.parametrize("n_mu", [4, 8, 16])
def test_dipole_1d_normalised(n_mu):
    mu, w = double_gauss(n_mu)
    p = dipole_1d(mu)
    assert np.allclose(p, p.T)
    assert np.allclose(p @ w, 1.0, atol=1e-15)


def test_dipole_3d_normalised():
    om, w = directions_3d(8, 8)
    p = dipole_3d(om)
    assert np.allclose(p, p.T)
    assert np.allclose(p @ w, 1.0, atol=1e-14)


@pytest.mark.parametrize("n_nu", [5, 16, 21, 32, 48, 64])
def test_prd_marginals_and_symmetry(n_nu):
    x, w, phi = frequency_grid(n_nu, 5.0)
    p = prd_frequency_kernel(x, w, phi, 0.5, 0.5)
    assert np.allclose(p, p.T, rtol=1e-15, atol=0)
    assert np.all(p > 0)
    assert np.max(np.abs(p @ w - phi) / phi) < 1e-13
    assert abs(w @ p @ w - 1.0) < 1e-14
    # coherent part concentrates near the diagonal: at the line centre it
    # exceeds the CRD part's coupling to the far wing
    crd = np.outer(phi, phi)
    coh = (p - 0.5 * crd) / 0.5
    c = n_nu // 2
    assert coh[c, c] > coh[c, 0] * 1e3


def test_prd_zero_coherent_fraction_is_crd():
    x, w, phi = frequency_grid(21, 5.0)
    assert np.allclose(prd_frequency_kernel(x, w, phi, 0.0, 0.5), np.outer(phi, phi))


def test_legendre_phase_closed_form():
    mu = np.linspace(-1, 1, 7)
    assert np.allclose(legendre_phase(mu, [1.0]), 1.0)
    assert np.allclose(legendre_phase(mu, [1.0, 3.0]), 1 + 3 * np.outer(mu, mu))
    p2 = 0.5 * (3 * mu * mu - 1)
    assert np.allclose(legendre_phase(mu, [0, 0, 2.0]), 2 * np.outer(p2, p2))


@pytest.mark.parametrize("make", [W.slab64, lambda: W.small_box(4, 4, 8, 5)])
def test_kernel_photon_conservation_and_thermal_rows(make):
    p = Problem(make())
    # (1/s_d^2) double integral of Phi = 1 (paper Sec. 2 normalisation)
    assert abs(p.w_ray @ p.psi @ p.w_ray - 1.0) < 1e-13
    assert np.allclose(p.psi, p.psi.T)
    # rows of Mhat reproduce the line albedo: a Planckian field scatters to B
    assert np.allclose(p.mhat.sum(axis=1), p.phi_ray / p.fac_ray, rtol=1e-13)
