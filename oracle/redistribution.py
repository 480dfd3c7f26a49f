"""Scattering kernels (oracle; test infrastructure only).

The emissivity equation of the paper (Sec. 2) integrates a redistribution
function Phi(Omega, Omega', nu, nu') against the intensity; photon conservation
fixes its double integral to 1.  Sec. 3.3 collects its values at the ray pairs
into the symmetric block Psi (N_r x N_r).  Here Phi factorises into an angular
phase function and a frequency kernel:

* dipole phase 3/4 (1 + (Omega.Omega')^2) and its azimuthal average in 1D,
  3/8 (3 - mu^2 - mu'^2 + 3 mu^2 mu'^2), each normalised to unit mean;
* PRD frequency kernel (1 - c) phi phi^T + c P_coh, where P_coh is the
  symmetric Gaussian-coherent kernel d_i exp(-(x_i - x_j)^2 / w2) d_j whose
  discrete marginals equal phi (the positive diagonal scaling d is the unique
  fixed point of the symmetric Sinkhorn map, iterated here to convergence);
* the Legendre phase sum_l d_l P_l(mu) P_l(mu') of the monochromatic
  experiment (Sec. 5.1).

Pins: symmetry, unit quadrature normalisation, PRD marginals, 3D azimuthal
average equal to the 1D kernel (tests/test_oracle_redistribution.py).
"""
from __future__ import annotations

import numpy as np


def dipole_1d(mu: np.ndarray) -> np.ndarray:
    """Azimuth-averaged dipole phase p(mu_i, mu_j) (unit mean over mu')."""
    m2 = mu * mu
    return 0.375 * (3.0 - m2[:, None] - m2[None, :] + 3.0 * m2[:, None] * m2[None, :])


def dipole_3d(omega: np.ndarray) -> np.ndarray:
    """Dipole phase 3/4 (1 + cos^2 Theta) between all ordinate pairs."""
    c = omega @ omega.T
    return 0.75 * (1.0 + c * c)


def coherent_scaling(x: np.ndarray, w: np.ndarray, phi: np.ndarray,
                     width2: float, tol: float = 1e-15, max_iter: int = 100000):
    """Positive d with sum_j w_j d_i G_ij d_j = phi_i, G_ij = exp(-(x_i-x_j)^2/w2).

    Symmetric Sinkhorn iteration d <- sqrt(d * phi / (G W d)) from d = sqrt(phi),
    stopped when the largest relative marginal error is below ``tol`` (or it
    stalls at rounding level).
    """
    g = np.exp(-((x[:, None] - x[None, :]) ** 2) / width2)
    d = np.sqrt(phi)
    best = np.inf
    for _ in range(max_iter):
        marg = d * (g @ (w * d))
        err = np.max(np.abs(marg - phi) / phi)
        if err < tol:
            break
        if err >= best and err < 1e-13:
            break
        best = min(best, err)
        d = np.sqrt(d * phi / (g @ (w * d)))
    return d, g


def prd_frequency_kernel(x: np.ndarray, w: np.ndarray, phi: np.ndarray,
                         coh_frac: float, width2: float) -> np.ndarray:
    """(1 - c) phi phi^T + c P_coh with marginals sum_j w_j P_ij = phi_i."""
    if len(x) == 1:
        return np.ones((1, 1))
    d, g = coherent_scaling(x, w, phi, width2)
    p_coh = d[:, None] * g * d[None, :]
    return (1.0 - coh_frac) * np.outer(phi, phi) + coh_frac * p_coh


def legendre_phase(mu: np.ndarray, coeffs) -> np.ndarray:
    """sum_l d_l P_l(mu_i) P_l(mu_j) (monochromatic experiment, Sec. 5.1)."""
    pl = np.stack([np.polynomial.legendre.Legendre.basis(l)(mu)
                   for l in range(len(coeffs))])
    return np.einsum("l,li,lj->ij", np.asarray(coeffs, float), pl, pl)
