"""Global radiative-transfer operator (oracle; test infrastructure only).

Paper Sec. 3.1: the discrete problem is I = Lambda S + I_in together with
S = Sigma I + t (eqs. RT_algebraic_form1/2).  Sec. 3.3: Sigma is block diagonal
over spatial points, Sigma = Gamma Psi W (eq. Sigma), with Psi the symmetric
kernel block, W the quadrature weights and Gamma the scattering coefficients.

Here Gamma and W carry the two-level-atom coefficients of the emissivity
equation (Sec. 2) with opacity chi_nu = k_L (phi_nu + r):

    S_k = (1 - eps_i) * sum_k' Mhat[k, k'] I_k' + t_k,
    Mhat = diag(1/(phi_nu + r)) Psi diag(w_o w_nu),
    t_k  = (eps_i phi_nu + r) B_i / (phi_nu + r).

Substituting I gives the source-function form solved by the HIP library,

    A s = s - (1 - eps) Mhat Lambda_0 s = b,   b = (1 - eps) Mhat I_bc + t,

where Lambda_0 is the formal solution with zero incoming radiation and I_bc
the intensity propagated from the boundaries with S = 0.  The paper's
intensity form (eq. RT_sys_algebraic), (Id - Lambda Sigma) I = Lambda t + I_in,
is also provided; both have the same spectrum since Lambda Sigma and
Sigma Lambda share their nonzero eigenvalues.

Vectors are ray-major (the paper's permuted ordering X~ = P X of Sec. 3.1):
index [k, i] with ray k = o * N_nu + nu (frequency fastest) and point i; in the
box i = (z * ny + y) * nx + x with z = 0 the bottom plane, in the slab i is the
depth index from the top.

Per-point kernels: Sec. 3.3 allows a different (possibly full) block
Psi_[i] at every point i.  With spec.point_class the points fall into classes,
each with its own kernel (a coherent fraction of the dipole x PRD recipe, or
an explicit matrix), and the scattering of point i uses its class's block.

Pins: eps = 1 identity, thermal equilibrium s = B, sqrt(eps) surface law,
matrix-free columns = dense assembly (tests/test_oracle_operator.py); classes
in tests/test_oracle_classes.py.
"""
from __future__ import annotations

import numpy as np

from .quadrature import double_gauss, directions_3d, frequency_grid
from .redistribution import dipole_1d, dipole_3d, prd_frequency_kernel
from .transfer import sweep_slab, sweep_box


class Problem:
    """Oracle problem built from a workloads.ProblemSpec.

    Optional overrides (used by the paper-reproduction tests):
    mu_weights  (mu, w_mu) slab inclinations and weights
    profile     (x, w_x, phi) frequency nodes, weights and profile
    """

    def __init__(self, spec, mu_weights=None, profile=None):
        self.spec = spec
        self.geom = spec.geom
        if self.geom == "slab":
            if mu_weights is None:
                mu, w_o = double_gauss(spec.n_mu)
            else:
                mu, w_o = (np.asarray(a, float) for a in mu_weights)
            self.omega = None
            self.mu_o = mu
        elif self.geom == "box":
            self.omega, w_o = directions_3d(spec.n_mu, spec.n_az)
            self.mu_o = self.omega[:, 2]
        else:
            raise ValueError(spec.geom)
        if profile is None:
            x, w_x, phi = frequency_grid(spec.n_nu, spec.x_max)
        else:
            x, w_x, phi = (np.asarray(a, float) for a in profile)
        self.x, self.w_x, self.phi = x, w_x, phi
        self.w_o = w_o
        n_om, n_nu = len(w_o), len(x)
        self.n_omega, self.n_nu = n_om, n_nu
        self.n_r = n_om * n_nu
        self.n_s = spec.n_s
        self.n = self.n_r * self.n_s
        self.w_ray = np.kron(w_o, w_x)
        self.phi_ray = np.tile(phi, n_om)
        self.fac_ray = self.phi_ray + spec.r
        self.mu_ray = np.repeat(self.mu_o, n_nu)

        def kernel_block(coh_frac=None, matrix=None):
            if spec.kernel == "dipole_prd":
                p_ang = dipole_1d(self.mu_o) if self.geom == "slab" else dipole_3d(self.omega)
                p_nu = prd_frequency_kernel(x, w_x, phi, coh_frac, spec.coh_width2)
                return np.kron(p_ang, p_nu)
            if spec.kernel == "explicit":
                psi = np.asarray(matrix, float)
                assert psi.shape == (self.n_r, self.n_r)
                return psi
            raise ValueError(spec.kernel)

        def mhat_of(psi):
            return (1.0 / self.fac_ray)[:, None] * psi * self.w_ray[None, :]

        base = spec.kernel_matrix
        if base is None and getattr(spec, "class_kernels", None) is not None:
            base = spec.class_kernels[0]       # classes without a kernel_matrix
        self.psi = kernel_block(spec.coh_frac, base)
        self.mhat = mhat_of(self.psi)
        # per-point classes: self.point_class (n_s) and one Mhat per class
        self.point_class = None
        self.mhat_classes = None
        if getattr(spec, "point_class", None) is not None:
            pc = np.asarray(spec.point_class, dtype=np.int64).reshape(-1)
            assert pc.shape == (spec.n_s,)
            if spec.kernel == "dipole_prd":
                blocks = [kernel_block(coh_frac=c) for c in spec.class_coh_frac]
            else:
                blocks = [kernel_block(matrix=m) for m in spec.class_kernels]
            assert pc.min() >= 0 and pc.max() < len(blocks)
            self.point_class = pc
            self.mhat_classes = [mhat_of(b) for b in blocks]

        eps = np.broadcast_to(np.asarray(spec.eps, float), (self.n_s,)).copy()
        bpl = np.broadcast_to(np.asarray(spec.planck, float), (self.n_s,)).copy()
        self.eps_pt, self.b_pt = eps, bpl
        self.albedo = 1.0 - eps
        self.t = ((eps[None, :] * self.phi_ray[:, None] + spec.r) * bpl[None, :]
                  / self.fac_ray[:, None])

    # ---------------------------------------------------------------- Lambda
    def lam(self, s, with_bc: bool):
        """Formal solution: intensity (N_r, N_s) for source s (N_r, N_s)."""
        s = np.asarray(s, float).reshape(self.n_r, self.n_s)
        sp = self.spec
        it = sp.i_top if with_bc else 0.0
        ib = sp.i_bot if with_bc else 0.0
        if self.geom == "slab":
            return sweep_slab(sp.depth, self.mu_ray, self.fac_ray, s, it, ib, sp.formal)
        if sp.formal not in ("linear_sc", "quadratic_sc"):
            raise ValueError("box supports linear_sc and quadratic_sc")
        out = sweep_box(sp.k_line, self.omega, self.phi + sp.r,
                        s.reshape(self.n_r, sp.nz, sp.ny, sp.nx), it, ib, sp.formal)
        return out.reshape(self.n_r, self.n_s)

    # ----------------------------------------------------------------- Sigma
    def scatter(self, intensity):
        """(1 - eps_i) * Mhat_[i] @ I: the scattering part of the source
        function (Mhat_[i] the block of point i's class, or the one Mhat)."""
        i2 = np.asarray(intensity, float).reshape(self.n_r, self.n_s)
        return self.scatter_points(i2, slice(None))

    def scatter_points(self, intensity, points):
        """scatter() for the spatial points `points` only (a slice or an
        index array; intensity holds their N_r x len(points) columns): the
        scattering block acts on each point by itself (eq. Sigma is block
        diagonal over points), so a subset of columns is the same product."""
        i2 = np.asarray(intensity, float).reshape(self.n_r, -1)
        if self.point_class is None:
            return self.albedo[None, points] * (self.mhat @ i2)
        pc = self.point_class[points]
        out = np.empty_like(i2)
        for c, m in enumerate(self.mhat_classes):
            sel = pc == c
            out[:, sel] = m @ i2[:, sel]
        return self.albedo[None, points] * out

    # -------------------------------------------------------------- operator
    def apply(self, s):
        """A s = s - (1 - eps) Mhat Lambda_0 s (source-function form)."""
        s2 = np.asarray(s, float).reshape(self.n_r, self.n_s)
        return s2 - self.scatter(self.lam(s2, with_bc=False))

    def rhs(self):
        """b = (1 - eps) Mhat I_bc + t."""
        zero = np.zeros((self.n_r, self.n_s))
        return self.scatter(self.lam(zero, with_bc=True)) + self.t

    def intensity(self, s):
        """Full intensity I = Lambda_0 s + I_bc for a source function s."""
        return self.lam(s, with_bc=True)

    def apply_intensity_form(self, intensity):
        """Paper's (Id - Lambda Sigma) I (eq. RT_sys_algebraic)."""
        i2 = np.asarray(intensity, float).reshape(self.n_r, self.n_s)
        return i2 - self.lam(self.scatter(i2), with_bc=False)

    def rhs_intensity_form(self):
        """Paper's Lambda t + I_in."""
        return self.lam(self.t, with_bc=True)

    def dense(self, form: str = "source"):
        """Assemble A column by column (tiny problems only)."""
        f = self.apply if form == "source" else self.apply_intensity_form
        a = np.zeros((self.n, self.n))
        e = np.zeros(self.n)
        for j in range(self.n):
            e[j] = 1.0
            a[:, j] = f(e).ravel()
            e[j] = 0.0
        return a

    def residual_norm(self, s, b=None):
        """Relative true residual ||b - A s||_2 / ||b||_2 in FP64."""
        b = self.rhs() if b is None else np.asarray(b, float).reshape(self.n_r, self.n_s)
        r = b - self.apply(s)
        return float(np.linalg.norm(r) / np.linalg.norm(b))
