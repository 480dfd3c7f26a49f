"""Seeded synthetic inputs shared by the oracle tests, the GPU parity tests and
the benchmark.

This module holds *inputs only*: workload recipes (sizes and physical
parameters), depth grids, the 3D opacity field, the batched-slab and
serving-stream draws, and random test vectors.  It holds none of the method's
arithmetic (no quadrature, no redistribution kernel, no formal solver, no
scattering sum): the oracle and the HIP library each compute those on their
own from the recipe.

Workloads (synthetic stand-ins for the paper's experiments; the paper's own 3D
atmosphere and atomic data are not available):

* ``slab64``   - 1D plane-parallel slab, 64 log-spaced line-centre depths in
  [1e-4, 1e4], 8 inclinations (4+4 double Gauss), 21 frequencies on [-5, 5],
  continuum ratio 1e-3, eps = 1e-4, B = 1, dipole x PRD scattering, FP64.
* ``box32``    - 3D box 32^3, periodic in x and y, 8 inclinations x 8 azimuths,
  32 frequencies, exponential + log-normal opacity field, eps = 1e-4, FP64.
* ``box64``    - 3D box 64^3, 8 inclinations x 16 azimuths, 48 frequencies,
  solved in mixed precision.
* ``batch512`` - 512 independent slabs with drawn N_z, N_nu, N_mu, eps, depth.
* ``serve``    - Poisson request stream (90 % slabs, 10 % 16^3 boxes).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, asdict
from typing import Optional

import numpy as np

SEED_BASE = 21958

# Continuous line-centre value of the unit-area Doppler profile exp(-x^2)/sqrt(pi).
# Used only to scale the generated opacity field to a target optical depth.
_PHI0_INPUT_SCALE = 1.0 / math.sqrt(math.pi)


@dataclass
class ProblemSpec:
    """Plain description of one radiative-transfer problem.

    geom        'slab' (1D plane-parallel) or 'box' (3D, periodic in x, y)
    nx, ny, nz  spatial nodes (slab: nx = ny = 1)
    depth       slab only: frequency-integrated line optical depth t at each
                node, top (index 0) to bottom; the optical depth of ray
                (mu, nu) between nodes is (phi_nu + r) * dt / |mu|
    k_line      box only: frequency-integrated line opacity per unit length,
                shape (nz, ny, nx), z index 0 = bottom plane; the box edge
                length is 1 in x, y and z
    n_mu        total inclinations (half per hemisphere, double Gauss)
    n_az        azimuths (box only; slab uses 1)
    n_nu        frequencies, equispaced on [-x_max, x_max]
    r           continuum-to-line opacity ratio
    eps         photon destruction probability: scalar or per-point array
    planck      thermal source B: scalar or per-point array
    i_top       incoming intensity at the top boundary (scalar)
    i_bot       incoming intensity at the bottom boundary (scalar)
    kernel      'dipole_prd' or 'explicit'
    kernel_matrix  explicit N_r x N_r symmetric kernel (only for 'explicit')
    coh_frac    weight of the coherent part of the PRD kernel
    coh_width2  squared width of the coherent Gaussian exp(-(x-x')^2/w2)
    formal      'linear_sc' (exponential integrator), 'implicit_euler' or
                'quadratic_sc' (parabolic source through upwind, local, downwind)
    point_class optional per-point scattering class (n_s ints in
                [0, n_classes)); each class has its own kernel block
    class_coh_frac   dipole_prd: coherent fraction of each class
    class_kernels    explicit: (n_classes, N_r, N_r) symmetric kernel per class
    """

    geom: str = "slab"
    nx: int = 1
    ny: int = 1
    nz: int = 64
    depth: Optional[np.ndarray] = None
    k_line: Optional[np.ndarray] = None
    n_mu: int = 8
    n_az: int = 1
    n_nu: int = 21
    x_max: float = 5.0
    r: float = 1e-3
    eps: object = 1e-4
    planck: object = 1.0
    i_top: float = 0.0
    i_bot: float = 1.0
    kernel: str = "dipole_prd"
    kernel_matrix: Optional[np.ndarray] = None
    coh_frac: float = 0.5
    coh_width2: float = 0.5
    formal: str = "linear_sc"
    point_class: Optional[np.ndarray] = None
    class_coh_frac: Optional[np.ndarray] = None
    class_kernels: Optional[np.ndarray] = None

    @property
    def n_classes(self) -> int:
        if self.point_class is None:
            return 1
        if self.class_kernels is not None:
            return len(self.class_kernels)
        return len(self.class_coh_frac)

    @property
    def n_s(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def n_omega(self) -> int:
        return self.n_mu * self.n_az

    @property
    def n_r(self) -> int:
        return self.n_omega * self.n_nu

    @property
    def n(self) -> int:
        return self.n_s * self.n_r


def log_depth_grid(nz: int, tau_min: float, tau_max: float) -> np.ndarray:
    """Depth grid t whose line-centre optical depths t/sqrt(pi) are
    logarithmically spaced from tau_min to tau_max, top to bottom."""
    tau_c = np.logspace(math.log10(tau_min), math.log10(tau_max), nz)
    return tau_c / _PHI0_INPUT_SCALE


def box_opacity_field(nx: int, ny: int, nz: int, seed: int,
                      tau_vertical: float = 1e4, scale_height: float = 1.0 / 8.0,
                      sigma: float = math.log(1.2)) -> np.ndarray:
    """Line opacity k_L(z, y, x) of the synthetic 3D atmosphere.

    k_L = k0 * exp(-z/H) * exp(sigma*g - sigma^2/2), g iid N(0,1) drawn from
    PCG64(seed) in C order (z, y, x); z_k = k/(nz-1), k = 0 is the bottom.
    k0 makes the continuous vertical line-centre optical depth of the box
    (line-centre profile 1/sqrt(pi)) equal to ``tau_vertical``.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    g = rng.standard_normal((nz, ny, nx))
    z = np.arange(nz) / (nz - 1)
    h = scale_height
    k0 = tau_vertical / (_PHI0_INPUT_SCALE * h * (1.0 - math.exp(-1.0 / h)))
    strat = k0 * np.exp(-z / h)
    return strat[:, None, None] * np.exp(sigma * g - 0.5 * sigma * sigma)


def slab64() -> ProblemSpec:
    """1D slab workload (64 depths, 8 mu, 21 frequencies, FP64)."""
    return ProblemSpec(geom="slab", nz=64, depth=log_depth_grid(64, 1e-4, 1e4),
                       n_mu=8, n_az=1, n_nu=21, x_max=5.0, r=1e-3, eps=1e-4,
                       planck=1.0, i_top=0.0, i_bot=1.0)


def box(n: int, n_mu: int, n_az: int, n_nu: int, seed: int,
        eps: float = 1e-4) -> ProblemSpec:
    return ProblemSpec(geom="box", nx=n, ny=n, nz=n,
                       k_line=box_opacity_field(n, n, n, seed),
                       n_mu=n_mu, n_az=n_az, n_nu=n_nu, x_max=5.0, r=1e-3,
                       eps=eps, planck=1.0, i_top=0.0, i_bot=1.0)


def box32() -> ProblemSpec:
    """3D box workload 32^3, 64 ordinates (8 mu x 8 az), 32 frequencies, FP64."""
    return box(32, 8, 8, 32, SEED_BASE + 1)


def box64() -> ProblemSpec:
    """3D box workload 64^3, 128 ordinates (8 mu x 16 az), 48 frequencies."""
    return box(64, 8, 16, 48, SEED_BASE + 2)


def small_box(n: int = 8, n_mu: int = 4, n_az: int = 8, n_nu: int = 5,
              seed: int = SEED_BASE + 11, nz: Optional[int] = None,
              ny: Optional[int] = None) -> ProblemSpec:
    """Small box with the box32 opacity recipe, for oracle-sized tests."""
    nz = n if nz is None else nz
    ny = n if ny is None else ny
    return ProblemSpec(geom="box", nx=n, ny=ny, nz=nz,
                       k_line=box_opacity_field(n, ny, nz, seed),
                       n_mu=n_mu, n_az=n_az, n_nu=n_nu, x_max=5.0, r=1e-3,
                       eps=1e-4, planck=1.0, i_top=0.0, i_bot=1.0)


def batch_slabs(count: int = 512, seed: int = SEED_BASE + 3) -> list:
    """Heterogeneous slab batch.

    N_z ~ U{32..256}, N_nu ~ U{16..64}, N_mu ~ U{8,10,12,14,16},
    eps log-uniform in [1e-6, 1e-2], total depth log-uniform in [1e2, 1e6];
    depth grid log-spaced from 1e-4 to the drawn depth.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(count):
        nz = int(rng.integers(32, 257))
        n_nu = int(rng.integers(16, 65))
        n_mu = int(rng.choice([8, 10, 12, 14, 16]))
        eps = float(10.0 ** rng.uniform(-6.0, -2.0))
        depth = float(10.0 ** rng.uniform(2.0, 6.0))
        out.append(ProblemSpec(geom="slab", nz=nz,
                               depth=log_depth_grid(nz, 1e-4, depth),
                               n_mu=n_mu, n_az=1, n_nu=n_nu, x_max=5.0,
                               r=1e-3, eps=eps, planck=1.0, i_top=0.0,
                               i_bot=1.0))
    return out


def serve_stream(duration_s: float = 60.0, rate_hz: float = 200.0,
                 slab_frac: float = 0.9, seed: int = SEED_BASE + 4) -> list:
    """Poisson request stream: list of (arrival_time_s, kind, draw_seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    while True:
        t += float(rng.exponential(1.0 / rate_hz))
        if t >= duration_s:
            break
        kind = "slab" if rng.uniform() < slab_frac else "box"
        out.append((t, kind, int(rng.integers(0, 2**31 - 1))))
    return out


def serve_request(kind: str, draw_seed: int) -> ProblemSpec:
    """The problem a serving request asks for."""
    if kind == "slab":
        return batch_slabs(1, seed=draw_seed)[0]
    return box(16, 4, 8, 24, SEED_BASE + 1 + (draw_seed % 1000))


def random_field(shape, seed: int, positive: bool = False) -> np.ndarray:
    """Seeded test vector (standard normal, or uniform in [0.5, 1.5])."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if positive:
        return rng.uniform(0.5, 1.5, size=shape)
    return rng.standard_normal(shape)


def random_symmetric_kernel(n_r: int, seed: int) -> np.ndarray:
    """Seeded symmetric positive matrix used as an explicit scattering kernel."""
    rng = np.random.Generator(np.random.PCG64(seed))
    a = rng.uniform(0.1, 1.0, size=(n_r, n_r))
    return 0.5 * (a + a.T)


def spec_dict(spec: ProblemSpec) -> dict:
    d = asdict(spec)
    for k in ("depth", "k_line", "kernel_matrix"):
        d.pop(k, None)
    return d
