"""GMRES iteration counts under grid refinement, on the GPU.

The spectral analysis (Sec. 4; Theorem main4 of Sec. 4.2) makes the
eigenvalues of the discrete operator cluster at 1 under refinement, so
unpreconditioned GMRES needs about the same number of iterations on finer
grids; the isotropic tests of Sec. 5 report a growth from 8 to 11 iterations
for 125x more unknowns, and the 3D runs of Sec. 5.3 (Table stellar) counts
that stay put across all discretisation parameters.  The oracle checks this
on small slabs (test_oracle_krylov); here the GPU path runs grids up to 216x
larger, in FP64 and, for the slab, in mixed precision (fp16 Sigma, FP32
Lambda, FP64 refinement; the count is then the total of inner iterations).

Criteria: angle, frequency and (log-spaced) depth refinement, counts within
10 % of the finest grid's; spatial refinement of a box whose grids resolve
its optical depth (vertical line-centre depth 10), at most 5 more iterations
from 16^3 to 48^3 (27x the unknowns).  A box whose cells are optically thick
(the box32 recipe, vertical depth 1e4) needs more iterations until the grid
resolves it; that regime is not a refinement of the same discrete behaviour.
"""
import sys

import pytest

import workloads as W
from oracle import Problem as OProblem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _solve(spec, precision="fp64", precond="none"):
    from paper_2602_21958_amd import rt
    with rt.Problem(spec) as p:
        x = torch.empty(p.n, dtype=torch.float64, device="cuda:0")
        st = p.solve(x, rtol=1e-8, restart=30, precision=precision, precond=precond)
        torch.cuda.synchronize()
        return st, x.cpu().numpy()


def _within(counts, frac):
    ref = counts[max(counts)]
    return all(abs(c - ref) <= frac * ref for c in counts.values())


def _box(n, n_mu=4, n_az=8, n_nu=8, tau=10.0):
    # stratified box (no horizontal fluctuations), the same continuous
    # atmosphere on every grid
    s = W.small_box(n, n_mu, n_az, n_nu)
    s.k_line = W.box_opacity_field(n, n, n, 0, tau_vertical=tau, sigma=0.0)
    return s


@pytest.mark.parametrize("precision", ["fp64", "fp16"])
def test_slab_counts_flat_under_depth_refinement(precision):
    counts = {}
    for nz in (64, 128, 256, 512):
        spec = W.slab64()
        spec.nz, spec.depth = nz, W.log_depth_grid(nz, 1e-4, 1e4)
        say(f"slab nz={nz} {precision}")
        st, s = _solve(spec, precision)
        assert st["converged"], st
        assert OProblem(spec).residual_norm(s) <= 1e-8
        counts[nz] = st["iters"]
    say(f"   slab {precision} iterations by N_z: {counts}")
    assert _within(counts, 0.1), counts


def test_counts_flat_under_angle_and_frequency_refinement():
    counts = {}
    for shape in ((4, 8, 8), (8, 8, 8), (4, 16, 8), (4, 8, 16), (8, 16, 16)):
        spec = _box(16, *shape, tau=100.0)
        say(f"box 16^3 mu x az x nu = {shape}")
        st, s = _solve(spec)
        assert st["converged"], st
        counts[shape] = st["iters"]
    say(f"   box iterations by (mu, az, nu): {counts}")
    assert _within(counts, 0.1), counts
    counts = {}
    for n_mu, n_nu in ((8, 21), (16, 21), (8, 81), (16, 81)):
        spec = W.slab64()
        spec.n_mu, spec.n_nu = n_mu, n_nu
        say(f"slab mu={n_mu} nu={n_nu}")
        st, s = _solve(spec)
        assert st["converged"], st
        assert OProblem(spec).residual_norm(s) <= 1e-8
        counts[(n_mu, n_nu)] = st["iters"]
    say(f"   slab iterations by (mu, nu): {counts}")
    assert _within(counts, 0.1), counts


def test_box_counts_under_spatial_refinement():
    counts = {}
    for n in (16, 32, 48):
        spec = _box(n)
        say(f"box {n}^3")
        st, s = _solve(spec)
        assert st["converged"], st
        if n <= 16:   # oracle FP64 residual (larger grids: the device FP64
            # operator, checked against the oracle by the parity tests)
            assert OProblem(spec).residual_norm(s) <= 1e-8
        counts[n] = st["iters"]
    say(f"   box iterations by n: {counts}")
    assert counts[48] - counts[16] <= 5, counts


def test_config_recipe_counts_flat_from_32_to_64():
    """The box workloads' own recipe (vertical line-centre depth 1e4, 20 %
    log-normal horizontal fluctuations, 8 mu x 8 azimuths) with 8 instead
    of 32-48 frequencies: GMRES(30) counts at 32^3, 48^3 and 64^3 within
    10 % of the finest grid's, the regime the benchmark boxes run in; with
    the preconditioner at most half of them on each grid."""
    counts, pre = {}, {}
    for n in (32, 48, 64):
        spec = W.box(n, 8, 8, 8, W.SEED_BASE + 1)
        say(f"config-recipe box {n}^3 (8 mu x 8 az x 8 nu)")
        st, s = _solve(spec)
        assert st["converged"], st
        counts[n] = st["iters"]
        del s
        st, s = _solve(spec, precond="local")
        assert st["converged"], st
        pre[n] = st["iters"]
        del s
    say(f"   config-recipe iterations by n: {counts}; preconditioned: {pre}")
    assert _within(counts, 0.1), counts
    # the physics-based preconditioner (Sec. 6 remark) keeps the local part
    # of Lambda: it cuts the count on every grid, but it is not flat under
    # refinement (thinner cells leave less of Lambda local)
    assert all(2 * pre[n] <= counts[n] for n in counts), (counts, pre)
