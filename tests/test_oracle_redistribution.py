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


# Continuum limit of the coherent kernel (pins the width convention).  With
# w2 = 0.5 the symmetric kernel c(x) exp(-2 (x - x')^2) c(x') whose marginals
# are the Doppler profile exp(-x^2)/sqrt(pi) has c(x) = A exp(-beta x^2):
# integrating over x' gives the exponent -(2 + beta) x^2 + 4 x^2 / (2 + beta),
# which equals -x^2 when alpha = 2 + beta solves alpha^2 - alpha - 4 = 0, and
# the prefactor A^2 sqrt(pi / alpha) = 1 / sqrt(pi).
_ALPHA = (1.0 + math.sqrt(17.0)) / 2.0
_BETA = _ALPHA - 2.0


def _coherent_continuum(x):
    a, b = x[:, None], x[None, :]
    return (math.sqrt(_ALPHA) / math.pi) * np.exp(-2.0 * (a - b) ** 2) \
        * np.exp(-_BETA * (a * a + b * b))


def _coherent_discrete(n_nu, x_max, width2):
    x, w, phi = frequency_grid(n_nu, x_max)
    # coherent part alone: with c = 1 the kernel is P_coh
    return x, prd_frequency_kernel(x, w, phi, 1.0, width2)


def test_coherent_continuum_kernel_has_doppler_marginals():
    # the closed form itself, by a fine quadrature of its marginal
    x = np.linspace(-9.0, 9.0, 3601)
    h = x[1] - x[0]
    k = _coherent_continuum(x)
    marg = k.sum(axis=1) * h
    phi = np.exp(-x * x) / math.sqrt(math.pi)
    inner = np.abs(x) < 4.0
    assert np.max(np.abs(marg[inner] - phi[inner]) / phi[inner]) < 1e-12


def test_prd_coherent_part_converges_to_continuum_kernel():
    # [-8, 8]: the discrete Sinkhorn-scaled kernel approaches the continuum
    # one at a rate that keeps rising under refinement (the trapezoid rule is
    # spectrally accurate for these Gaussians), down to rounding
    errs, hs = [], []
    for n_nu in (11, 16, 21, 31):
        x, p = _coherent_discrete(n_nu, 8.0, 0.5)
        c = _coherent_continuum(x)
        errs.append(np.max(np.abs(p - c)) / np.max(c))
        hs.append(16.0 / (n_nu - 1))
    orders = [math.log(errs[i] / errs[i + 1]) / math.log(hs[i] / hs[i + 1])
              for i in range(len(errs) - 1)]
    assert all(o > 4.0 for o in orders), orders
    assert orders[-1] > orders[0]
    for n_nu in (51, 101, 201):
        x, p = _coherent_discrete(n_nu, 8.0, 0.5)
        c = _coherent_continuum(x)
        assert np.max(np.abs(p - c)) / np.max(c) < 1e-13
    # the workloads' grids on [-5, 5]: 21 frequencies to 1e-6, finer ones to
    # the truncation of the profile's tails
    for n_nu, tol in ((21, 1e-6), (32, 1e-11), (48, 1e-11), (64, 1e-11)):
        x, p = _coherent_discrete(n_nu, 5.0, 0.5)
        c = _coherent_continuum(x)
        assert np.max(np.abs(p - c)) / np.max(c) < tol, n_nu


def test_prd_width_convention_is_pinned():
    # reading exp(-(x-x')^2 / w2) as exp(-(x-x')^2 / (2 w2)) (i.e. w2 = 1)
    # gives a different kernel with the same marginals: it misses the
    # continuum limit by 20 %
    for n_nu in (51, 101):
        x, p = _coherent_discrete(n_nu, 8.0, 1.0)
        c = _coherent_continuum(x)
        assert np.max(np.abs(p - c)) / np.max(c) > 0.1
