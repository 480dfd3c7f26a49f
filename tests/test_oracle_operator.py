"""Pins for the oracle's global operator: eps = 1 identity, thermal
equilibrium, the sqrt(eps) surface law, and the matrix-free apply against an
explicitly assembled Id - (1-eps) Sigma Lambda built from the paper's closed
forms (Sec. 3.2 entries, Sec. 3.3 block structure)."""
import numpy as np
import pytest

import workloads as W
from oracle import Problem, gmres, frequency_grid


@pytest.mark.parametrize("make", [W.slab64, lambda: W.small_box(4, 4, 8, 5, nz=6)])
def test_eps_one_is_identity(make):
    spec = make()
    spec.eps = 1.0
    p = Problem(spec)
    s = W.random_field((p.n_r, p.n_s), 1)
    assert np.array_equal(p.apply(s), s)
    b = p.rhs()
    assert np.allclose(b, spec.planck, rtol=1e-15)
    res = gmres(p.apply, b, restart=30, tol=1e-12)
    assert res["iters"] == 1 and np.allclose(res["x"], spec.planck, rtol=1e-15)


@pytest.mark.parametrize("make", [W.slab64, lambda: W.small_box(5, 4, 8, 5, nz=7)])
@pytest.mark.parametrize("eps", [1e-4, 0.3])
def test_thermal_equilibrium_is_exact_solution(make, eps):
    # Both boundaries radiate B: S = B everywhere solves the problem, whatever
    # eps and the continuum ratio (transfer of a constant source with Planckian
    # incidence returns B; scattering of B returns B).
    spec = make()
    spec.eps, spec.i_top, spec.i_bot, spec.planck = eps, 2.5, 2.5, 2.5
    p = Problem(spec)
    s = np.full((p.n_r, p.n_s), 2.5)
    assert np.allclose(p.intensity(s), 2.5, rtol=1e-14)
    r = p.rhs() - p.apply(s)
    assert np.max(np.abs(r)) < 1e-13


def _sqrt_eps_problem(nz):
    depth = np.logspace(-6, 7, nz)
    x, w, phi = frequency_grid(21, 5.0)
    psi = np.kron(np.ones((8, 8)), np.outer(phi, phi))      # isotropic CRD
    return Problem(W.ProblemSpec(geom="slab", nz=nz, depth=depth, n_mu=8, n_nu=21,
                                 r=0.0, eps=1e-2, planck=1.0, kernel="explicit",
                                 kernel_matrix=psi, i_top=0.0, i_bot=1.0))


@pytest.mark.slow
def test_sqrt_eps_surface_law():
    # Semi-infinite isothermal atmosphere, isotropic CRD scattering, no
    # continuum: the surface source function tends to sqrt(eps) B under depth
    # refinement (Eddington-Barbier / H-function identity).
    errs = []
    for nz in (50, 100, 200):
        p = _sqrt_eps_problem(nz)
        res = gmres(p.apply, p.rhs(), restart=200, tol=1e-12)
        s0 = res["x"].reshape(p.n_r, p.n_s)[:, 0]
        assert np.ptp(s0) < 1e-12                       # CRD: S independent of ray
        errs.append(s0[0] / 0.1 - 1.0)
    assert errs[0] < errs[1] < errs[2] < 0             # monotone from below
    assert abs(errs[2]) < 0.02
    assert abs(errs[1]) / abs(errs[2]) > 2.5            # ~second order


def _dense_ie_operator(p):
    """Id - diag(albedo) (Mhat x Id_Ns) Lambda, with Lambda assembled per ray
    from the implicit-Euler closed-form entries (paper Sec. 3.2), ray-major."""
    depth = p.spec.depth
    ns, nr = p.n_s, p.n_r
    lam = np.zeros((nr * ns, nr * ns))
    for k in range(nr):
        dtau = np.diff(depth) * p.fac_ray[k] / abs(p.mu_ray[k])
        blk = np.zeros((ns, ns))
        for i in range(ns):
            for j in range(ns):
                if p.mu_ray[k] < 0 and 1 <= j <= i:
                    blk[i, j] = dtau[j - 1] / np.prod(1 + dtau[j - 1:i])
                if p.mu_ray[k] > 0 and i <= j <= ns - 2:
                    blk[i, j] = dtau[j] / np.prod(1 + dtau[i:j + 1])
        lam[k * ns:(k + 1) * ns, k * ns:(k + 1) * ns] = blk
    sig = np.kron(p.mhat, np.eye(ns)) * np.tile(p.albedo, nr)[:, None]
    return np.eye(nr * ns) - sig @ lam, lam, sig


def test_matrix_free_equals_assembled_operator():
    spec = W.slab64()
    spec.nz, spec.n_mu, spec.n_nu = 7, 4, 5
    spec.depth = W.log_depth_grid(7, 1e-2, 1e2)
    spec.eps = np.linspace(0.01, 0.5, 7)                    # per-point eps
    spec.formal = "implicit_euler"
    p = Problem(spec)
    a, lam, sig = _dense_ie_operator(p)
    x = W.random_field(p.n, 4)
    assert np.allclose(p.apply(x).ravel(), a @ x, rtol=1e-13, atol=1e-14)
    # intensity form Id - Lambda Sigma has the same spectrum (Sec. 3.5)
    ai = np.eye(p.n) - lam @ sig
    assert np.allclose(p.apply_intensity_form(x).ravel(), ai @ x, rtol=1e-13, atol=1e-14)
    ev_s = np.sort_complex(np.linalg.eigvals(a))
    ev_i = np.sort_complex(np.linalg.eigvals(ai))
    assert np.allclose(ev_s, ev_i, atol=1e-10)


def test_scatter_points_is_scatter_by_columns():
    spec = W.small_box(6, 4, 8, 5, nz=5)
    p = Problem(spec)
    i = W.random_field((p.n_r, p.n_s), 9)
    full = p.scatter(i)
    parts = np.concatenate([p.scatter_points(i[:, c:c + 37], slice(c, c + 37))
                            for c in range(0, p.n_s, 37)], axis=1)
    assert np.allclose(parts, full, rtol=1e-15, atol=1e-15 * np.abs(full).max())
    idx = np.array([3, 0, p.n_s - 1])
    assert np.allclose(p.scatter_points(i[:, idx], idx), full[:, idx], rtol=1e-15,
                       atol=1e-15 * np.abs(full).max())
