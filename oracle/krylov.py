"""Krylov solvers (oracle; test infrastructure only).

The paper solves A I = b with GMRES (no restart in the 1D experiments,
restart 30 in the 3D experiment) and BiCGStab (Sec. 5 set-up, Sec. 5.3).

* gmres: restarted GMRES(m) of Saad and Schultz (1986): Arnoldi with modified
  Gram-Schmidt, Givens rotations on the Hessenberg matrix, the residual norm
  estimate |g_{j+1}|; at the end of each cycle x += V_m y and the true
  residual b - A x is recomputed; stop when it is <= tol * ||b||.
* bicgstab: van der Vorst (1992), unpreconditioned.

Both start from x0 = 0 unless given and measure the relative residual in the
2-norm.  Pins: dense least-squares minimality of each GMRES iterate on tiny
problems, agreement with numpy.linalg.solve, monotone residual estimates
within a cycle (tests/test_oracle_krylov.py).
"""
from __future__ import annotations

import math

import numpy as np


def _givens(a, b):
    if b == 0.0:
        return 1.0, 0.0
    h = math.hypot(a, b)
    return a / h, b / h


def gmres(apply, b, x0=None, restart: int = 30, tol: float = 1e-8,
          maxiter: int = 10000):
    """Restarted GMRES(m).

    Returns dict(x, iters, cycles, history, relres, converged) where history
    holds the relative residual estimate after every Arnoldi step (preceded by
    the initial relative residual of each cycle) and relres is the final true
    relative residual.
    """
    b = np.asarray(b, float).ravel()
    n = b.size
    x = np.zeros(n) if x0 is None else np.asarray(x0, float).ravel().copy()
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return dict(x=np.zeros(n), iters=0, cycles=0, history=[0.0], relres=0.0,
                    converged=True)
    history = []
    iters = 0
    cycles = 0
    r = b - apply(x).ravel()
    beta = np.linalg.norm(r)
    history.append(beta / bnorm)
    while beta / bnorm > tol and iters < maxiter:
        cycles += 1
        m = restart
        v = np.zeros((m + 1, n))
        h = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        v[0] = r / beta
        k_used = 0
        for j in range(m):
            w = apply(v[j]).ravel()
            for i in range(j + 1):                        # modified Gram-Schmidt
                h[i, j] = np.dot(v[i], w)
                w = w - h[i, j] * v[i]
            h[j + 1, j] = np.linalg.norm(w)
            breakdown = h[j + 1, j] <= 1e-14 * abs(h[j, j]) + 1e-300
            if not breakdown:
                v[j + 1] = w / h[j + 1, j]
            for i in range(j):                            # old rotations
                t1 = cs[i] * h[i, j] + sn[i] * h[i + 1, j]
                h[i + 1, j] = -sn[i] * h[i, j] + cs[i] * h[i + 1, j]
                h[i, j] = t1
            cs[j], sn[j] = _givens(h[j, j], h[j + 1, j])
            h[j, j] = cs[j] * h[j, j] + sn[j] * h[j + 1, j]
            h[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            iters += 1
            k_used = j + 1
            history.append(abs(g[j + 1]) / bnorm)
            if breakdown or abs(g[j + 1]) / bnorm <= tol or iters >= maxiter:
                break
        y = np.linalg.solve(np.triu(h[:k_used, :k_used]), g[:k_used]) \
            if k_used else np.zeros(0)
        x = x + v[:k_used].T @ y
        r = b - apply(x).ravel()
        beta = np.linalg.norm(r)
        if beta / bnorm > tol and iters < maxiter:
            history.append(beta / bnorm)
    relres = beta / bnorm
    return dict(x=x, iters=iters, cycles=cycles, history=history, relres=relres,
                converged=relres <= tol)


def bicgstab(apply, b, x0=None, tol: float = 1e-8, maxiter: int = 10000):
    """Unpreconditioned BiCGStab; returns dict(x, iters, history, relres, converged)."""
    b = np.asarray(b, float).ravel()
    n = b.size
    x = np.zeros(n) if x0 is None else np.asarray(x0, float).ravel().copy()
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return dict(x=np.zeros(n), iters=0, history=[0.0], relres=0.0, converged=True)
    r = b - apply(x).ravel()
    rhat = r.copy()
    rho = alpha = omega = 1.0
    v = np.zeros(n)
    p = np.zeros(n)
    history = [np.linalg.norm(r) / bnorm]
    it = 0
    while history[-1] > tol and it < maxiter:
        it += 1
        rho_new = np.dot(rhat, r)
        if rho_new == 0.0:
            break
        beta = (rho_new / rho) * (alpha / omega)
        p = r + beta * (p - omega * v)
        v = apply(p).ravel()
        alpha = rho_new / np.dot(rhat, v)
        s = r - alpha * v
        if np.linalg.norm(s) / bnorm <= tol:
            x = x + alpha * p
            r = s
            history.append(np.linalg.norm(r) / bnorm)
            break
        t = apply(s).ravel()
        omega = np.dot(t, s) / np.dot(t, t)
        x = x + alpha * p + omega * s
        r = s - omega * t
        rho = rho_new
        history.append(np.linalg.norm(r) / bnorm)
        if omega == 0.0:
            break
    relres = np.linalg.norm(b - apply(x).ravel()) / bnorm
    return dict(x=x, iters=it, history=history, relres=relres,
                converged=relres <= tol)
