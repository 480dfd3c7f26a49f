"""Pins for the oracle's Krylov solvers on small operators assembled densely."""
import numpy as np
import pytest

import workloads as W
from oracle import Problem, gmres, bicgstab


def _small_slab():
    spec = W.slab64()
    spec.nz, spec.n_mu, spec.n_nu = 12, 4, 5
    spec.depth = W.log_depth_grid(12, 1e-3, 1e3)
    spec.eps = 1e-3
    return Problem(spec)


def test_gmres_matches_direct_solve():
    p = _small_slab()
    a = p.dense()
    b = p.rhs().ravel()
    x_ref = np.linalg.solve(a, b)
    for m in (5, 30, 400):
        res = gmres(p.apply, b, restart=m, tol=1e-13)
        assert res["converged"]
        assert np.linalg.norm(res["x"] - x_ref) / np.linalg.norm(x_ref) < 1e-10


def test_gmres_iterates_are_krylov_minimisers():
    # With no restart, step j's residual equals min ||b - A x|| over K_j(A, b).
    p = _small_slab()
    a = p.dense()
    b = p.rhs().ravel()
    res = gmres(p.apply, b, restart=400, tol=1e-30, maxiter=8)
    hist = np.array(res["history"][1:9])
    kry = [b / np.linalg.norm(b)]
    for j in range(1, 9):
        q, _ = np.linalg.qr(np.stack(kry, axis=1))
        y, *_ = np.linalg.lstsq(a @ q, b, rcond=None)
        ref = np.linalg.norm(b - a @ (q @ y)) / np.linalg.norm(b)
        assert abs(hist[j - 1] - ref) <= 1e-9 * ref + 1e-15
        nxt = a @ kry[-1]
        kry.append(nxt / np.linalg.norm(nxt))
    assert np.all(np.diff(hist) <= 1e-15)


def test_bicgstab_matches_direct_solve():
    p = _small_slab()
    a = p.dense()
    b = p.rhs().ravel()
    x_ref = np.linalg.solve(a, b)
    res = bicgstab(p.apply, b, tol=1e-13)
    assert res["converged"]
    assert np.linalg.norm(res["x"] - x_ref) / np.linalg.norm(x_ref) < 1e-10


def test_zero_rhs_returns_zero():
    p = _small_slab()
    res = gmres(p.apply, np.zeros(p.n), tol=1e-8)
    assert res["iters"] == 0 and not np.any(res["x"])
    res = bicgstab(p.apply, np.zeros(p.n), tol=1e-8)
    assert res["iters"] == 0 and not np.any(res["x"])


@pytest.mark.slow
def test_iteration_counts_flat_under_refinement():
    # Theorem main4 (Sec. 4.2): clustering at 1 makes unpreconditioned GMRES
    # robust; counts on the 64-depth slab family stay within +-10 % once the
    # depth grid resolves the slab.
    counts = {}
    for nz in (64, 128):
        spec = W.slab64()
        spec.nz, spec.depth = nz, W.log_depth_grid(nz, 1e-4, 1e4)
        p = Problem(spec)
        counts[("nz", nz)] = gmres(p.apply, p.rhs(), restart=30, tol=1e-8)["iters"]
    for n_nu in (21, 41):
        spec = W.slab64()
        spec.n_nu = n_nu
        p = Problem(spec)
        counts[("nu", n_nu)] = gmres(p.apply, p.rhs(), restart=30, tol=1e-8)["iters"]
    base = counts[("nz", 64)]
    for v in counts.values():
        assert abs(v - base) <= 0.1 * base
