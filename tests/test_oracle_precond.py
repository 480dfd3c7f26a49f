"""Pins of the oracle's physics-based preconditioner (oracle/precond.py; the
Sec. 6 remark on physics-based preconditioning, with the local part of
Lambda and the scattering block of Sec. 3.3, eq. Sigma).

* The plane response D equals the diagonal of Lambda_0 assembled column by
  column from unit sources (linear short characteristics on the box and
  the slab, implicit Euler and quadratic short characteristics on the
  slab); with the first two it lies in [0, 1) (non-negative weights that
  sum to at most one along a ray), while the parabolic weights of the
  quadratic scheme may leave that range.
* The Kronecker form of P^-1 equals the dense inverse of every point's
  block P_i assembled from its definition, and inverts apply(); with
  eps = 1 the preconditioner is the identity.
* Right-preconditioned GMRES reaches the unpreconditioned solution (the
  same system, so the same solution within the solve tolerance) with a
  true residual below the tolerance, in fewer iterations.  The iteration
  counts are properties of this preconditioner, not paper values."""
import dataclasses

import numpy as np
import pytest

import workloads as W
from oracle import Problem, gmres
from oracle.precond import AliPreconditioner, direction_average, pgmres, plane_response


def _tiny_box(formal="linear_sc"):
    spec = W.small_box(4, 2, 4, 3, nz=3, ny=3)
    return dataclasses.replace(spec, formal=formal)


def _tiny_slab(formal):
    spec = W.slab64()
    depth = spec.depth[::8].copy()
    return dataclasses.replace(spec, nz=depth.size, depth=depth, n_mu=4, n_nu=5, formal=formal)


def _lambda_diagonal(op):
    """diag(Lambda_0) from unit sources, one column at a time."""
    d = np.empty(op.n)
    e = np.zeros(op.n)
    for j in range(op.n):
        e[j] = 1.0
        d[j] = op.lam(e.reshape(op.n_r, op.n_s), with_bc=False).ravel()[j]
        e[j] = 0.0
    return d.reshape(op.n_r, op.n_s)


@pytest.mark.parametrize("make", [lambda: _tiny_box("linear_sc"),
                                  lambda: _tiny_slab("linear_sc"),
                                  lambda: _tiny_slab("implicit_euler"),
                                  lambda: _tiny_slab("quadratic_sc")])
def test_plane_response_is_lambda_diagonal(make):
    op = Problem(make())
    d = plane_response(op)
    ref = _lambda_diagonal(op)
    assert np.max(np.abs(d - ref)) <= 1e-14
    if op.spec.formal != "quadratic_sc":
        assert d.min() >= 0.0 and d.max() < 1.0
    # the upwind boundary plane has no local contribution only where the
    # scheme says so; some point of every ray takes a nonzero share
    assert np.all(d.max(axis=1) > 0.0)


def test_direction_average_weights():
    op = Problem(_tiny_box())
    d = np.ones((op.n_r, op.n_s))
    assert np.allclose(direction_average(op, d), 1.0, rtol=0, atol=1e-15)
    # a ray-only pattern averages with the ordinate weights
    pat = np.repeat(np.arange(op.n_omega, dtype=float), op.n_nu)[:, None] * np.ones(op.n_s)
    want = np.dot(op.w_o, np.arange(op.n_omega)) / op.w_o.sum()
    assert np.allclose(direction_average(op, pat), want, rtol=1e-15)


@pytest.mark.parametrize("make", [_tiny_box, lambda: _tiny_slab("linear_sc")])
def test_kron_inverse_matches_dense_blocks(make):
    op = Problem(make())
    pc = AliPreconditioner(op)
    assert pc.kron
    rng = np.random.default_rng(5)
    x = rng.standard_normal((op.n_r, op.n_s))
    got = pc.apply_inverse(x)
    ref = np.stack([np.linalg.solve(pc.dense_block(i), x[:, i]) for i in range(op.n_s)], axis=1)
    # the blocks are ill-conditioned where eps is small (P_i approaches the
    # singular Id - Mhat D in optically thick points): forward error within
    # a small multiple of cond(P_i) times the rounding unit, backward error
    # at the rounding level of the solution (|P_i| is of order one)
    u = np.finfo(float).eps
    cond = np.array([np.linalg.cond(pc.dense_block(i)) for i in range(op.n_s)])
    err = np.max(np.abs(got - ref), axis=0)
    assert np.all(err <= 64 * u * cond * np.max(np.abs(ref), axis=0))
    assert np.max(np.abs(pc.apply(got) - x)) <= 64 * u * np.max(np.abs(got))
    # the angular eigenvalues: rank 2 on the slab, at most 6 in 3D (4 with
    # one inclination per hemisphere)
    assert pc.lam.size == (2 if op.geom == "slab" else 4)
    assert np.all(pc.lam > 0)


def test_explicit_kernel_uses_dense_blocks():
    spec = _tiny_box()
    n_r = Problem(spec).n_r
    spec = dataclasses.replace(spec, kernel="explicit",
                               kernel_matrix=W.random_symmetric_kernel(n_r, 3))
    op = Problem(spec)
    pc = AliPreconditioner(op)
    assert not pc.kron
    x = np.random.default_rng(6).standard_normal((op.n_r, op.n_s))
    y = pc.apply_inverse(x)
    # backward error at the rounding level of |P_i| |y_i| (this random
    # kernel is far from the physical normalisation: |P_i| of order 1e3)
    norms = np.array([np.linalg.norm(pc.dense_block(i), np.inf) for i in range(op.n_s)])
    bound = 64 * np.finfo(float).eps * norms * np.max(np.abs(y), axis=0)
    assert np.all(np.max(np.abs(pc.apply(y) - x), axis=0) <= bound)


def test_eps_one_is_identity():
    spec = dataclasses.replace(_tiny_box(), eps=1.0)
    op = Problem(spec)
    pc = AliPreconditioner(op)
    x = np.random.default_rng(7).standard_normal((op.n_r, op.n_s))
    assert np.array_equal(pc.apply_inverse(x), x)


@pytest.mark.parametrize("make,restart", [(lambda: W.small_box(6, 4, 4, 6), 30),
                                          (lambda: W.small_box(6, 4, 4, 6), 7),
                                          (W.slab64, 30)])
def test_preconditioned_gmres_same_solution_fewer_iterations(make, restart):
    op = Problem(make())
    b = op.rhs().ravel()
    # both to 1e-12: the two solutions of the same system then agree to
    # about cond(A) 1e-12 (cond(A) of order 1e4 here, eps = 1e-4)
    plain = gmres(op.apply, b, restart=restart, tol=1e-12)
    pc = AliPreconditioner(op)
    pre = pgmres(op, pc, b, restart=restart, tol=1e-12)
    assert pre["converged"] and op.residual_norm(pre["x"]) <= 1e-12
    scale = np.max(np.abs(plain["x"]))
    assert np.max(np.abs(pre["x"] - plain["x"])) <= 1e-8 * scale
    assert pre["iters"] * 2 <= plain["iters"], (pre["iters"], plain["iters"])
