"""Angular and frequency quadratures (oracle; test infrastructure only).

Paper Sec. 5 (common 1D set-up): the inclination grid is two Gauss-Legendre
sets of N_Omega/2 nodes, one on [-1, 0) and one on (0, 1]; frequencies are
integrated with the trapezoidal rule.  Sec. 5.3: in 3D the angular grid is a
tensor product of Gauss-Legendre inclinations and equidistant azimuths.

Weights are normalised so that the direction weights sum to 1 (the 1/s_d
factor of the emissivity equation, Sec. 2), and the discrete line profile is
renormalised so that its trapezoidal integral is exactly 1.

Pins: GL exactness on polynomials, weight sums, profile normalisation
(tests/test_oracle_quadrature.py).
"""
from __future__ import annotations

import math

import numpy as np


def double_gauss(n_mu: int):
    """Double-Gauss inclinations mu (ascending, negatives first) and weights
    summing to 1 over the whole sphere (1/2 per hemisphere)."""
    if n_mu < 2 or n_mu % 2:
        raise ValueError("n_mu must be even and >= 2")
    half = n_mu // 2
    x, w = np.polynomial.legendre.leggauss(half)      # on [-1, 1], sum w = 2
    mu_pos = 0.5 * (x + 1.0)                           # on (0, 1)
    w_pos = 0.25 * w                                   # sums to 1/2
    order = np.argsort(mu_pos)
    mu_pos, w_pos = mu_pos[order], w_pos[order]
    mu = np.concatenate([-mu_pos[::-1], mu_pos])
    wt = np.concatenate([w_pos[::-1], w_pos])
    return mu, wt


def azimuths(n_az: int):
    """Equidistant azimuths (b + 1/2) 2 pi / n_az with equal weights 1/n_az."""
    b = np.arange(n_az)
    return (b + 0.5) * 2.0 * math.pi / n_az, np.full(n_az, 1.0 / n_az)


def directions_3d(n_mu: int, n_az: int):
    """Tensor-product ordinates, inclination-major: o = m * n_az + b.

    Returns (omega[n_omega, 3] unit vectors (x, y, z), weights summing to 1).
    z points up; mu = Omega_z.
    """
    mu, wmu = double_gauss(n_mu)
    az, waz = azimuths(n_az)
    om = np.zeros((n_mu * n_az, 3))
    wt = np.zeros(n_mu * n_az)
    for m in range(n_mu):
        st = math.sqrt(max(0.0, 1.0 - mu[m] * mu[m]))
        for b in range(n_az):
            o = m * n_az + b
            om[o] = (st * math.cos(az[b]), st * math.sin(az[b]), mu[m])
            wt[o] = wmu[m] * waz[b]
    return om, wt


def frequency_grid(n_nu: int, x_max: float):
    """Reduced frequencies x on [-x_max, x_max], trapezoid weights, and the
    Doppler profile exp(-x^2)/sqrt(pi) renormalised to unit discrete area.

    A single frequency (monochromatic problem) is x = 0 with weight 1 and
    profile 1.
    """
    if n_nu == 1:
        return np.zeros(1), np.ones(1), np.ones(1)
    x = np.linspace(-x_max, x_max, n_nu)
    h = x[1] - x[0]
    w = np.full(n_nu, h)
    w[0] = w[-1] = 0.5 * h
    phi = np.exp(-x * x) / math.sqrt(math.pi)
    phi = phi / np.dot(w, phi)
    return x, w, phi
