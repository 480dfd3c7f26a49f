"""Pins of the structure the factored scattering form relies on (Sec. 2
dipole phase function and frequency redistribution; Sec. 3.3 eq. Sigma):
the oracle's scattering block is the Kronecker product of its angular and
frequency parts, and the dipole kernel has exact rank 6 on any 3D ordinate
set (2 for the slab's azimuth average).  The ranks follow from writing
(O.O')^2 and 1 = |O|^2 |O'|^2 in the six quadratic monomials of O; the
checks below take the singular values of the oracle's own kernels."""
import numpy as np
import pytest

import workloads as W
from oracle import Problem, dipole_1d, dipole_3d, directions_3d, double_gauss


def _rank(a, rel=1e-12):
    s = np.linalg.svd(a, compute_uv=False)
    return int(np.sum(s > rel * s[0])), s


@pytest.mark.parametrize("n_mu,n_az", [(4, 8), (8, 8), (8, 16), (2, 4)])
def test_dipole_3d_has_rank_six(n_mu, n_az):
    omega, _ = directions_3d(n_mu, n_az)
    r, s = _rank(dipole_3d(omega))
    # never above six; one inclination per hemisphere (a single mu^2) leaves
    # the quadratic monomials dependent on the ordinates, rank 4
    assert r == (4 if n_mu == 2 else 6)
    assert s[6] < 1e-13 * s[0]


@pytest.mark.parametrize("n_mu", [2, 4, 8, 16])
def test_dipole_1d_has_rank_two(n_mu):
    mu, _ = double_gauss(n_mu)
    r, s = _rank(dipole_1d(mu))
    # the kernel depends on mu only through mu^2: with one node per
    # hemisphere both hemispheres see the same mu^2
    assert r == (1 if n_mu == 2 else 2)


@pytest.mark.parametrize("make", [W.slab64, lambda: W.small_box(6, 4, 8, 7, nz=5)])
def test_mhat_is_angular_kron_frequency(make):
    spec = make()
    p = Problem(spec)
    ang = (dipole_3d(p.omega) if spec.geom == "box" else dipole_1d(p.mu_o)) * p.w_o[None, :]
    n_nu = p.n_nu
    fac = p.fac_ray[:n_nu]
    # the frequency block from one diagonal angular block of Mhat
    fb = p.mhat[:n_nu, :n_nu] / ang[0, 0]
    assert np.allclose(np.kron(ang, fb), p.mhat, rtol=0, atol=1e-15 * np.abs(p.mhat).max())
    # and it is diag(1/(phi + r)) P_nu diag(w_nu) with P_nu symmetric
    pnu = fb * fac[:, None] / p.w_x[None, :]
    assert np.allclose(pnu, pnu.T, rtol=1e-13, atol=0)
