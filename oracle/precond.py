"""Physics-based preconditioner of the source-function system (oracle; test
infrastructure only).

Sec. 6 remarks that, although the unpreconditioned Krylov solve is already
robust, a physics-based preconditioner can still cut the iteration count.
The classic physics-based choice approximates the formal solution Lambda by
its local part (accelerated Lambda iteration); here the local part is taken
plane by plane, averaged over directions, and kept together with the full
scattering block of every point (Sec. 3.3, eq. Sigma):

    D[k, i]     = (Lambda_0 1_z)[k, i] for the point i on plane z, where 1_z
                  is a unit source on plane z only (every ray).  With linear
                  short characteristics (and implicit Euler on slabs) this is
                  the diagonal of Lambda_0: a point's intensity depends on the
                  sources of its own plane only through its own source.  With
                  quadratic short characteristics it also holds the in-plane
                  neighbours' share through the upwind point's downwind term.
    Dbar[nu, i] = sum_o w_o D[(o, nu), i] / sum_o w_o
    P           = block diagonal over points of
                  P_i = Id - (1 - eps_i) Mhat diag_k(Dbar[nu(k), i]).

Right preconditioning solves A P^-1 y = b and returns x = P^-1 y; the
residual b - A P^-1 y is the residual of x, so the stopping test and the
reported residual are those of the unpreconditioned system.

For the dipole x PRD kernel Mhat is a Kronecker product P_A kron P_B of an
angular block P_A = p_dip diag(w_o) and a frequency block
P_B = diag(1/(phi + r)) P_PRD diag(w_nu), so with L_i = diag(Dbar[:, i])

    P_i = Id - (1 - eps_i) P_A kron (P_B L_i).

P_A = W^-1/2 S W^1/2 with S = W^1/2 p_dip W^1/2 symmetric; S = U Lam U^T
gives P_A = F Lam G^T with F = W^-1/2 U, G = W^1/2 U and G^T F = Id.  Only
the nonzero eigenvalues lam_q contribute (6 in 3D, 2 for the slab's azimuth
average), and

    P_i^-1 = Id + sum_q (F_q kron Id) T_iq (G_q^T kron Id),
    T_iq   = (Id - (1 - eps_i) lam_q P_B L_i)^-1 - Id    (N_nu x N_nu).

Parity: D is pinned against the diagonal of the assembled Lambda_0, the
Kronecker form of P^-1 against the dense inverse of the assembled blocks,
and preconditioned GMRES against the unpreconditioned solution
(tests/test_oracle_precond.py).
"""
from __future__ import annotations

import numpy as np

from .krylov import gmres
from .redistribution import dipole_1d, dipole_3d, prd_frequency_kernel


def plane_of_points(op) -> np.ndarray:
    """Plane index of every spatial point: z for the box (i = (z ny + y) nx
    + x), the depth index for the slab (one point per plane)."""
    sp = op.spec
    if op.geom == "box":
        return np.repeat(np.arange(sp.nz), sp.nx * sp.ny)
    return np.arange(op.n_s)


def plane_response(op) -> np.ndarray:
    """D (N_r, N_s): the intensity at every point for a unit source on its own
    plane only, one formal solution per plane (zero incoming radiation)."""
    plane = plane_of_points(op)
    d = np.zeros((op.n_r, op.n_s))
    for z in range(plane.max() + 1):
        on = plane == z
        s = np.zeros((op.n_r, op.n_s))
        s[:, on] = 1.0
        d[:, on] = op.lam(s, with_bc=False)[:, on]
    return d


def direction_average(op, d: np.ndarray) -> np.ndarray:
    """Dbar (N_nu, N_s): D averaged over the ordinates with the weights w_o."""
    w = op.w_o / op.w_o.sum()
    return np.einsum("o,ofi->fi", w, d.reshape(op.n_omega, op.n_nu, op.n_s))


class AliPreconditioner:
    """P of the module docstring for one oracle Problem (one kernel for all
    points).  apply(x) = P x from the definition; apply_inverse(x) = P^-1 x
    in the Kronecker form (dipole x PRD) or from per-point dense inverses
    (any other kernel)."""

    def __init__(self, op, d: np.ndarray | None = None):
        if op.point_class is not None:
            raise ValueError("one scattering kernel for all points")
        self.op = op
        self.d = plane_response(op) if d is None else np.asarray(d, float)
        self.dbar = direction_average(op, self.d)
        # diag_k(Dbar[nu(k), i]) as an (N_r, N_s) array
        self.dray = np.tile(self.dbar, (op.n_omega, 1))
        self.alpha = op.albedo
        self.kron = op.spec.kernel == "dipole_prd"
        if self.kron:
            self._kron_setup()
        else:
            eye = np.eye(op.n_r)
            self.inv = np.stack([np.linalg.inv(eye - self.alpha[i] * op.mhat * self.dray[None, :, i])
                                 for i in range(op.n_s)])

    def _kron_setup(self):
        op, sp = self.op, self.op.spec
        p_ang = dipole_1d(op.mu_o) if op.geom == "slab" else dipole_3d(op.omega)
        p_nu = prd_frequency_kernel(op.x, op.w_x, op.phi, sp.coh_frac, sp.coh_width2)
        self.pa = p_ang * op.w_o[None, :]
        self.pb = (1.0 / (op.phi + sp.r))[:, None] * p_nu * op.w_x[None, :]
        sw = np.sqrt(op.w_o)
        lam, u = np.linalg.eigh(sw[:, None] * p_ang * sw[None, :])
        keep = np.abs(lam) > 1e-12 * np.abs(lam).max()
        self.lam = lam[keep]
        self.f = u[:, keep] / sw[:, None]
        self.g = u[:, keep] * sw[:, None]
        eye = np.eye(op.n_nu)
        t = np.empty((op.n_s, self.lam.size, op.n_nu, op.n_nu))
        for i in range(op.n_s):
            bl = self.pb * self.dbar[None, :, i]
            for q, lq in enumerate(self.lam):
                t[i, q] = np.linalg.inv(eye - self.alpha[i] * lq * bl) - eye
        self.t = t

    def apply(self, x) -> np.ndarray:
        """P x = x - (1 - eps) Mhat (Dbar x), point by point."""
        op = self.op
        x2 = np.asarray(x, float).reshape(op.n_r, op.n_s)
        return x2 - self.alpha[None, :] * (op.mhat @ (self.dray * x2))

    def apply_inverse(self, x) -> np.ndarray:
        op = self.op
        x2 = np.asarray(x, float).reshape(op.n_r, op.n_s)
        if not self.kron:
            return np.einsum("ikl,li->ki", self.inv, x2)
        x3 = x2.reshape(op.n_omega, op.n_nu, op.n_s)
        r = np.einsum("oq,ofi->qfi", self.g, x3)          # G_q^T kron Id
        z = np.einsum("iqfg,qgi->qfi", self.t, r)         # T_iq per point
        return (x3 + np.einsum("oq,qfi->ofi", self.f, z)).reshape(op.n_r, op.n_s)

    def dense_block(self, i: int) -> np.ndarray:
        """P_i assembled from its definition (tiny problems)."""
        op = self.op
        return np.eye(op.n_r) - self.alpha[i] * op.mhat * self.dray[None, :, i]


def pgmres(op, prec: AliPreconditioner, b=None, restart: int = 30, tol: float = 1e-8,
           maxiter: int = 10000):
    """Right-preconditioned GMRES(m): GMRES on A P^-1 y = b, x = P^-1 y.
    Returns the oracle gmres dict with x replaced by the solution of A x = b."""
    b = op.rhs() if b is None else b
    out = gmres(lambda y: op.apply(prec.apply_inverse(y)), np.asarray(b, float).ravel(),
                restart=restart, tol=tol, maxiter=maxiter)
    out["x"] = prec.apply_inverse(out["x"]).ravel()
    return out
