"""FP64 CPU oracle for the matrix-free S_N radiative-transfer operator.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) imports, calls or links this package; only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` use
it.  It shares no code with the HIP path: quadratures, redistribution kernels,
formal solvers, the scattering sum and the Krylov solvers are all written here
independently, in plain NumPy float64, following the paper:

* ``quadrature``     - double-Gauss inclinations, equidistant azimuths,
                       trapezoidal frequencies (paper Sec. 5 set-up).
* ``redistribution`` - dipole phase functions, PRD kernel, Legendre phase of
                       the monochromatic experiment, isotropic kernels
                       (Sec. 2 emissivity equation and its normalisation,
                       Sec. 3.3, Sec. 5.1-5.2).
* ``transfer``       - formal solvers: implicit Euler (Sec. 3.2, eqs. ie_1,
                       ie_2), linear short characteristics with the exponential
                       integrator derived from the integral form of the
                       transfer equation (Sec. 2, eq. rt_integral), and the 3D
                       plane-to-plane sweep (Sec. 3.4 block structure).
* ``operator``       - the global operator in source-function form
                       s - (1-eps) Sigma Lambda s, its right-hand side, the
                       intensity form Id - Lambda Sigma (Sec. 3.1,
                       eq. RT_sys_algebraic; Sec. 3.5) and dense assembly.
* ``krylov``         - restarted GMRES (Saad-Schultz, modified Gram-Schmidt,
                       Givens rotations) and BiCGStab (van der Vorst).
* ``precond``        - the physics-based preconditioner of Sec. 6's remark:
                       the plane-local part of Lambda, averaged over
                       directions, with every point's scattering block, and
                       right-preconditioned GMRES.

Parity status per function is listed in each module header.
"""
from .quadrature import double_gauss, azimuths, frequency_grid, directions_3d
from .redistribution import (dipole_1d, dipole_3d, prd_frequency_kernel,
                             legendre_phase)
from .transfer import exp_weights, sweep_slab, sweep_box
from .operator import Problem
from .krylov import gmres, bicgstab

__all__ = [
    "double_gauss", "azimuths", "frequency_grid", "directions_3d",
    "dipole_1d", "dipole_3d", "prd_frequency_kernel", "legendre_phase",
    "exp_weights", "sweep_slab", "sweep_box", "Problem", "gmres", "bicgstab",
]
