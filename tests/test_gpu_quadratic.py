"""GPU parity of the quadratic short-characteristics formal solver
(RT_FORMAL_QUADRATIC_SC) against the oracle's sweep of the same scheme.

Each node takes the integral form of the transfer equation over its upwind
interval with the source the parabola through the upwind, local and downwind
values (Sec. 2, eq. rt_integral; the production code's integrator, Sec. 5.3);
the last node of a ray has no downwind value and takes the linear step.
FP64: 1e-12 of the largest magnitude; FP32: per entry, a few FP32 roundings.
"""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import Problem as OProblem, gmres

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _rt():
    from paper_2602_21958_amd import rt
    return rt


def dev(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda:0")


def host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


def relerr(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(b)), 1e-300))


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def qslab(nz=64, n_mu=8, n_nu=21, tau_max=1e4, eps=1e-4):
    s = W.slab64()
    s.nz, s.n_mu, s.n_nu, s.eps = nz, n_mu, n_nu, eps
    s.depth = W.log_depth_grid(nz, 1e-4, tau_max)
    s.formal = "quadratic_sc"
    return s


CASES = {
    "slab64": lambda: qslab(),
    # one chunk of 64 lanes per ray and several chunks (the lane scan)
    "nz3_mu2_nu1": lambda: qslab(3, 2, 1, 10.0),
    "nz65_mu4_nu5": lambda: qslab(65, 4, 5),
    "nz300_mu6_nu7": lambda: qslab(300, 6, 7, 1e6),
    "thin_nz40": lambda: qslab(40, 4, 9, 1e-2),
}


@pytest.mark.parametrize("with_bc", [False, True])
@pytest.mark.parametrize("name", list(CASES))
def test_quadratic_lambda_fp64(name, with_bc):
    rt = _rt()
    spec = CASES[name]()
    say(f"quadratic lambda fp64 {name} bc={with_bc}")
    op = OProblem(spec)
    s = W.random_field(op.n, 61)
    with rt.Problem(spec) as p:
        out = torch.empty(op.n, dtype=torch.float64, device="cuda:0")
        p.apply_lambda(dev(s), out, with_bc=with_bc)
        got = host(out)
    ref = op.lam(s.reshape(op.n_r, op.n_s), with_bc=with_bc).ravel()
    e = relerr(got, ref)
    say(f"   max-relative error {e:.2e}")
    assert e < 1e-12


@pytest.mark.parametrize("name", list(CASES))
def test_quadratic_lambda_fp32(name):
    rt = _rt()
    spec = CASES[name]()
    say(f"quadratic lambda fp32 {name}")
    op = OProblem(spec)
    s = W.random_field(op.n, 62, positive=True)
    with rt.Problem(spec) as p:
        out = torch.empty(op.n, dtype=torch.float32, device="cuda:0")
        p.apply_lambda(dev(s, torch.float32), out, precision="fp32")
        got = host(out)
    s32 = s.astype(np.float32).astype(np.float64).reshape(op.n_r, op.n_s)
    ref = op.lam(s32, with_bc=False).ravel()
    # the downwind weight is negative, so an entry can be much smaller than
    # its terms: each entry carries a few FP32 roundings of the same sweep
    # taken with the weights' absolute values
    mag = _magnitude_sweep(spec, op, s32).ravel()
    edge = ref == 0
    assert np.all(got[edge] == 0)
    err = np.abs(got - ref)
    bound = 32 * 2.0 ** -24 * mag
    say(f"   worst error / bound {np.max(err[~edge] / bound[~edge]):.2e}")
    assert np.all(err <= bound)


def _magnitude_sweep(spec, op, s):
    """The quadratic sweep with every weight replaced by its absolute value
    (zero incoming radiation): a bound on the sum of the magnitudes of the
    terms behind each intensity."""
    from oracle.transfer import exp_weights, quad_weights
    dt = np.diff(np.asarray(spec.depth, float))
    dtau = dt[None, :] * (op.fac_ray[:, None] / np.abs(op.mu_ray)[:, None])
    nz = spec.nz
    out = np.zeros_like(s)
    for down in (True, False):
        rays = op.mu_ray < 0 if down else op.mu_ray > 0
        order = range(1, nz) if down else range(nz - 2, -1, -1)
        for i in order:
            iu, idn = (i - 1, i + 1) if down else (i + 1, i - 1)
            du = dtau[rays, i - 1] if down else dtau[rays, i]
            last = idn < 0 or idn >= nz
            if last:
                e, a, c = exp_weights(du)
                out[rays, i] = e * out[rays, iu] + np.abs(a) * s[rays, iu] + np.abs(c) * s[rays, i]
            else:
                dd = dtau[rays, i] if down else dtau[rays, i - 1]
                e, pu, p0, pd = quad_weights(du, dd)
                out[rays, i] = (e * out[rays, iu] + np.abs(pu) * s[rays, iu]
                                + np.abs(p0) * s[rays, i] + np.abs(pd) * s[rays, idn])
    return out


@pytest.mark.parametrize("name", ["slab64", "nz65_mu4_nu5", "nz300_mu6_nu7"])
def test_quadratic_operator_rhs_and_solve(name):
    rt = _rt()
    spec = CASES[name]()
    say(f"quadratic operator and solve {name}")
    op = OProblem(spec)
    x = W.random_field(op.n, 63)
    ref = gmres(op.apply, op.rhs().ravel(), restart=30, tol=1e-13)
    with rt.Problem(spec) as p:
        y = torch.empty(op.n, dtype=torch.float64, device="cuda:0")
        p.apply(dev(x), y)
        got = host(y)
        b = torch.empty_like(y)
        p.rhs(b)
        gotb = host(b)
        s = torch.empty_like(y)
        st = p.solve(s, rtol=1e-8)
        res = op.residual_norm(host(s))
        st2 = p.solve(s, rtol=1e-13, max_iters=4000)
        diff = np.linalg.norm(host(s) - ref["x"]) / np.linalg.norm(ref["x"])
        m = torch.empty_like(y)
        stm = p.solve(m, rtol=1e-8, precision="fp16", max_outer=40)
        resm = op.residual_norm(host(m))
    say(f"   iters {st['iters']} (oracle at 1e-13: {ref['iters']}), residual {res:.2e}, "
        f"tight diff {diff:.2e}, mixed fp16 residual {resm:.2e}")
    assert relerr(got, op.apply(x).ravel()) < 1e-12
    assert relerr(gotb, op.rhs().ravel()) < 1e-12
    assert st["converged"] and res <= 1e-8
    assert st2["converged"] and diff < 1e-10
    assert stm["converged"] and resm <= 1e-8


def test_quadratic_batch_engine():
    """Quadratic slabs of uneven sizes in one batch engine (bf16x3 operator,
    FP64 refinement): every solution meets the oracle's FP64 residual 1e-8."""
    rt = _rt()
    specs = [qslab(40, 4, 9), qslab(97, 6, 13, 1e5), qslab(150, 8, 5, 1e3)]
    probs = [rt.Problem(s) for s in specs]
    xs = [torch.empty(p.n, dtype=torch.float64, device="cuda:0") for p in probs]
    eng = rt.Batch(precision="bf16x3", hbm_budget=2 << 30, max_slots=8)
    try:
        tk = [eng.submit(p, x, restart=30, rtol=1e-8, max_outer=60) for p, x in zip(probs, xs)]
        eng.wait_all()
        for t, s, x in zip(tk, specs, xs):
            st = eng.poll(t)
            res = OProblem(s).residual_norm(host(x))
            say(f"   batch quadratic nz={s.nz}: converged={st['converged']} residual {res:.2e}")
            assert st["converged"] and res <= 1e-8
    finally:
        eng.close()
        for p in probs:
            p.close()


# ------------------------------------------------------------------ box
def qbox(n, n_mu, n_az, n_nu, nz=None, ny=None):
    s = W.small_box(n, n_mu, n_az, n_nu, nz=nz, ny=ny)
    s.formal = "quadratic_sc"
    return s


BOXES = {
    "box8": lambda: qbox(8, 4, 8, 5),
    "box_12x10x9": lambda: qbox(12, 4, 4, 3, nz=9, ny=10),
    "box16_shallow": lambda: qbox(16, 8, 8, 3, nz=6),
    # planes of 257..1024 points (two points per thread) and of more than 1024
    "box_24x20x5": lambda: qbox(24, 2, 4, 2, nz=5, ny=20),
    "box_40x36x4": lambda: qbox(40, 2, 4, 2, nz=4, ny=36),
}


@pytest.mark.parametrize("with_bc", [False, True])
@pytest.mark.parametrize("name", list(BOXES))
def test_quadratic_box_lambda_fp64(name, with_bc):
    rt = _rt()
    spec = BOXES[name]()
    say(f"quadratic box lambda fp64 {name} bc={with_bc}")
    op = OProblem(spec)
    s = W.random_field(op.n, 64)
    with rt.Problem(spec) as p:
        out = torch.empty(op.n, dtype=torch.float64, device="cuda:0")
        p.apply_lambda(dev(s), out, with_bc=with_bc)
        got = host(out)
    ref = op.lam(s.reshape(op.n_r, op.n_s), with_bc=with_bc).ravel()
    e = relerr(got, ref)
    say(f"   max-relative error {e:.2e}")
    assert e < 1e-12


def _box_magnitude_sweep(spec, op, s):
    """The box's quadratic sweep with every weight replaced by its absolute
    value (zero incoming radiation), from the oracle's stencil, interpolation
    and weight primitives."""
    from oracle.transfer import _interp, _upwind_stencil, exp_weights, quad_weights
    nz, ny, nx = spec.nz, spec.ny, spec.nx
    k = np.asarray(spec.k_line, float).reshape(nz, ny, nx)
    n_om, n_nu = op.n_omega, op.n_nu
    s = s.reshape(n_om, n_nu, nz, ny, nx)
    out = np.zeros_like(s)
    fac = (op.phi + spec.r)[:, None, None]
    for o in range(n_om):
        i0, tx, j0, ty, path = _upwind_stencil(op.omega[o], nx, ny, nz)
        d0, dtx, e0, dty, _ = _upwind_stencil(-op.omega[o], nx, ny, nz)
        up = op.omega[o, 2] > 0
        planes, step = (range(1, nz), -1) if up else (range(nz - 2, -1, -1), +1)
        for z in planes:
            zu, zd = z + step, z - step
            d = 0.5 * (_interp(k[zu], i0, tx, j0, ty) + k[z])[None] * path * fac
            iu = _interp(out[o, :, zu], i0, tx, j0, ty)
            su = _interp(s[o, :, zu], i0, tx, j0, ty)
            if 0 <= zd < nz:
                dd = 0.5 * (_interp(k[zd], d0, dtx, e0, dty) + k[z])[None] * path * fac
                sd = _interp(s[o, :, zd], d0, dtx, e0, dty)
                e, pu, p0, pd = quad_weights(d, dd)
                out[o, :, z] = (e * iu + np.abs(pu) * su + np.abs(p0) * s[o, :, z]
                                + np.abs(pd) * sd)
            else:
                e, a, c = exp_weights(d)
                out[o, :, z] = e * iu + np.abs(a) * su + np.abs(c) * s[o, :, z]
    return out.reshape(op.n_r, op.n_s)


@pytest.mark.parametrize("name", ["box8", "box_12x10x9", "box_24x20x5", "box_40x36x4"])
def test_quadratic_box_lambda_fp32(name):
    rt = _rt()
    spec = BOXES[name]()
    say(f"quadratic box lambda fp32 {name}")
    op = OProblem(spec)
    s = W.random_field(op.n, 65, positive=True)
    with rt.Problem(spec) as p:
        out = torch.empty(op.n, dtype=torch.float32, device="cuda:0")
        p.apply_lambda(dev(s, torch.float32), out, precision="fp32")
        got = host(out)
    s32 = s.astype(np.float32).astype(np.float64).reshape(op.n_r, op.n_s)
    ref = op.lam(s32, with_bc=False).ravel()
    mag = _box_magnitude_sweep(spec, op, s32).ravel()
    assert np.all(mag >= np.abs(ref) * (1 - 1e-12))
    edge = ref == 0
    assert np.all(got[edge] == 0)
    err = np.abs(got - ref)
    bound = 32 * 2.0 ** -24 * mag
    say(f"   worst error / bound {np.max(err[~edge] / bound[~edge]):.2e}")
    assert np.all(err <= bound)


@pytest.mark.parametrize("name", ["box8", "box_12x10x9"])
def test_quadratic_box_operator_and_solves(name):
    rt = _rt()
    spec = BOXES[name]()
    say(f"quadratic box operator and solves {name}")
    op = OProblem(spec)
    x = W.random_field(op.n, 66)
    ref = gmres(op.apply, op.rhs().ravel(), restart=30, tol=1e-13)
    with rt.Problem(spec) as p:
        y = torch.empty(op.n, dtype=torch.float64, device="cuda:0")
        p.apply(dev(x), y)
        got = host(y)
        b = torch.empty_like(y)
        p.rhs(b)
        gotb = host(b)
        s = torch.empty_like(y)
        st = p.solve(s, rtol=1e-13, max_iters=3000)
        diff = np.linalg.norm(host(s) - ref["x"]) / np.linalg.norm(ref["x"])
        m = torch.empty_like(y)
        stm = p.solve(m, rtol=1e-8, precision="fp16", basis_fp16=1, max_outer=40)
        resm = op.residual_norm(host(m))
    say(f"   tight diff {diff:.2e}; mixed fp16/fp16-basis: outer {stm['outer_iters']} "
        f"residual {resm:.2e}")
    assert relerr(got, op.apply(x).ravel()) < 1e-12
    assert relerr(gotb, op.rhs().ravel()) < 1e-12
    assert st["converged"] and diff < 1e-10
    assert stm["converged"] and resm <= 1e-8


def test_quadratic_box_not_in_batch_engine():
    rt = _rt()
    with rt.Problem(BOXES["box8"]()) as p:
        eng = rt.Batch(precision="fp16", hbm_budget=1 << 30, max_slots=4)
        try:
            x = torch.empty(p.n, dtype=torch.float64, device="cuda:0")
            with pytest.raises(rt.RtError) as e:
                eng.submit(p, x)
            assert e.value.code == rt.RT_E_INVALID
        finally:
            eng.close()
