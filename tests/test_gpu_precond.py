"""GPU parity of the physics-based preconditioner (rt_apply_precond,
rt_precond_local, rt_solve with precond = RT_PRECOND_LOCAL) against the
oracle's (oracle/precond.py; Sec. 6 remark on physics-based preconditioning).

Bars:
* Dbar (FP64 formal solutions of plane sources, direction averaged): within
  1e-13 of the oracle's (values in [0, 1) for the linear schemes).
* P^-1 x (16 frequencies: the FP32 tables take the one-wavefront-per-block
  product; the other cases the point-tile one): the per-point blocks are
  ill-conditioned where eps is small
  (P_i approaches the singular Id - Mhat Dbar in optically thick points), so
  the forward error is bounded by a small multiple of cond(P_i) times the
  rounding unit of the precision, per point, and so is the backward error
  |P_i (P^-1 x)_i - x_i| relative to |x_i| (stored blocks rounded to the
  precision).
* Preconditioned FP64 solves at rtol 1e-13 agree with the oracle's
  unpreconditioned solution to 1e-10 (as the plain solves do); iteration
  counts within 2 of the oracle's preconditioned GMRES and at most half of
  the plain solve's.
* Preconditioned mixed solves (dense or factored scattering): oracle-evaluated
  FP64 residual <= 1e-8.
"""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import Problem as OProblem, gmres
from oracle.precond import AliPreconditioner, direction_average, pgmres, plane_response

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _rt():
    from paper_2602_21958_amd import rt
    return rt


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda:0")


def host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


def slab(nz=64, n_mu=8, n_nu=21, formal="linear_sc"):
    s = W.slab64()
    s.nz, s.n_mu, s.n_nu, s.formal = nz, n_mu, n_nu, formal
    s.depth = W.log_depth_grid(nz, 1e-4, 1e4)
    return s


def qbox():
    s = W.small_box(8, 4, 4, 5)
    s.formal = "quadratic_sc"
    return s


SPECS = {
    "slab64": W.slab64,
    "slab_ie": lambda: slab(formal="implicit_euler"),
    "slab_qsc": lambda: slab(nz=40, n_mu=4, n_nu=9, formal="quadratic_sc"),
    "box8": lambda: W.small_box(8, 4, 8, 5),
    "box_12x10x9": lambda: W.small_box(12, 4, 4, 3, nz=9, ny=10),
    "box_qsc": qbox,
    # one inclination per hemisphere: four angular modes, not six
    "box_mu2": lambda: W.small_box(6, 2, 8, 6, nz=5),
    # frequencies a multiple of 8: the fp16-basis solves take fp16 blocks
    "box_nu16": lambda: W.small_box(8, 4, 4, 16, nz=6),
}


@pytest.mark.parametrize("name", list(SPECS))
def test_precond_local_matches_oracle(name):
    rt = _rt()
    spec = SPECS[name]()
    say(f"precond Dbar {name}")
    op = OProblem(spec)
    ref = direction_average(op, plane_response(op))
    with rt.Problem(spec) as p:
        got = p.precond_local()
    err = float(np.max(np.abs(got - ref)))
    say(f"   max |Dbar - oracle| {err:.2e}")
    assert got.shape == ref.shape
    assert err <= 1e-13
    if spec.formal != "quadratic_sc":
        assert got.min() >= 0.0 and got.max() < 1.0


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", ["slab64", "box8", "box_12x10x9", "box_mu2", "box_qsc",
                                  "box_nu16"])
def test_apply_precond_matches_oracle(name, prec):
    rt = _rt()
    spec = SPECS[name]()
    say(f"precond apply {name} {prec}")
    op = OProblem(spec)
    pc = AliPreconditioner(op)
    x = W.random_field(op.n, 41).reshape(op.n_r, op.n_s)
    ref = pc.apply_inverse(x)
    dt = torch.float64 if prec == "fp64" else torch.float32
    xin = x.astype(np.float32).astype(np.float64) if prec == "fp32" else x
    with rt.Problem(spec) as p:
        xd = dev(xin.ravel(), dt)
        y = torch.empty_like(xd)
        p.apply_precond(xd, y, precision=prec)
        got = host(y).reshape(op.n_r, op.n_s)
    ref = pc.apply_inverse(xin)
    u = np.finfo(np.float64 if prec == "fp64" else np.float32).eps
    cond = np.array([np.linalg.cond(pc.dense_block(i)) for i in range(op.n_s)])
    err = np.max(np.abs(got - ref), axis=0)
    scale = np.max(np.abs(ref), axis=0)
    worst = float(np.max(err / (cond * scale)))
    # backward error per point: stored blocks with relative error u give
    # |P_i (P_i^-1 + E) x_i - x_i| <= |P_i| u |P_i^-1| |x_i| = cond_i u |x_i|
    back = np.max(np.abs(pc.apply(got) - xin), axis=0) / np.max(np.abs(xin), axis=0)
    say(f"   forward error / (cond |ref|) {worst:.2e}, backward / cond "
        f"{float(np.max(back / cond)):.2e}")
    assert np.all(err <= 64 * u * cond * scale)
    assert np.all(back <= 64 * u * cond)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_apply_precond_unaligned_vectors(prec):
    """Vectors that are not 16-byte aligned take the one-value-per-thread
    reduction: the same sums in the same order, so the same bits as the
    16-byte path on aligned copies of the same vectors."""
    rt = _rt()
    spec = SPECS["box_12x10x9"]()
    op = OProblem(spec)
    dt = torch.float64 if prec == "fp64" else torch.float32
    x = W.random_field(op.n, 43)
    with rt.Problem(spec) as p:
        xa = dev(x, dt)
        ya = torch.empty_like(xa)
        p.apply_precond(xa, ya, precision=prec)
        xb_buf = torch.zeros(op.n + 1, dtype=dt, device="cuda:0")
        yb_buf = torch.zeros_like(xb_buf)
        xb, yb = xb_buf[1:], yb_buf[1:]   # offset by one value: not 16-byte aligned
        xb.copy_(xa)
        p.apply_precond(xb, yb, precision=prec)
        torch.cuda.synchronize()
        assert xb.data_ptr() % 16 != 0
        assert torch.equal(ya, yb)


@pytest.mark.parametrize("two_step", [1, 0])
@pytest.mark.parametrize("name", ["slab64", "box8", "box_12x10x9"])
def test_preconditioned_fp64_solve(name, two_step):
    rt = _rt()
    spec = SPECS[name]()
    say(f"precond fp64 solve {name} two_step={two_step}")
    op = OProblem(spec)
    b = op.rhs().ravel()
    ref = gmres(op.apply, b, restart=30, tol=1e-13)
    pref = pgmres(op, AliPreconditioner(op), b, restart=30, tol=1e-8)
    plain = gmres(op.apply, b, restart=30, tol=1e-8)
    with rt.Problem(spec) as p:
        x = torch.empty(op.n, dtype=torch.float64, device="cuda:0")
        st = p.solve(x, rtol=1e-8, restart=30, two_step=two_step, precond="local")
        it8 = st["iters"]
        st = p.solve(x, rtol=1e-13, restart=30, two_step=two_step, precond="local",
                     max_iters=3000)
        s = host(x)
    diff = np.linalg.norm(s - ref["x"]) / np.linalg.norm(ref["x"])
    say(f"   iters to 1e-8 {it8} (oracle preconditioned {pref['iters']}, plain "
        f"{plain['iters']}); to 1e-13 {st['iters']}, solution diff {diff:.2e}")
    assert st["converged"] and op.residual_norm(s) <= 1e-12
    assert diff < 1e-10
    assert abs(it8 - pref["iters"]) <= 2
    assert 2 * it8 <= plain["iters"]


@pytest.mark.parametrize("prec", ["fp32", "fp16", "bf16", "bf16x3"])
@pytest.mark.parametrize("name", ["slab64", "box8", "box_12x10x9", "box_nu16"])
def test_preconditioned_mixed_solve(name, prec):
    rt = _rt()
    spec = SPECS[name]()
    say(f"precond mixed {prec} {name}")
    op = OProblem(spec)
    with rt.Problem(spec) as p:
        x = torch.empty(op.n, dtype=torch.float64, device="cuda:0")
        plain = p.solve(x, rtol=1e-8, precision=prec, max_outer=40)
        st = p.solve(x, rtol=1e-8, precision=prec, precond="local", max_outer=40)
        s = host(x)
    res = op.residual_norm(s)
    say(f"   inner {st['iters']} / outer {st['outer_iters']} (plain {plain['iters']} / "
        f"{plain['outer_iters']}), oracle residual {res:.2e}")
    assert st["converged"] and res <= 1e-8
    assert st["iters"] < plain["iters"]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16"])
@pytest.mark.parametrize("name", ["slab64", "box8", "box_12x10x9"])
def test_preconditioned_factored_solve(name, prec):
    """The preconditioner with the factored scattering form: FP64 GMRES on
    the factored FP64 operator (fp64), or FP64 outer residuals in factored
    form with the inner operator the factored FP32 form (fp32) or the dense
    16-bit GEMM (fp16).  In FP64 and FP32 the step's v - u is formed in the
    factored expansion from the preconditioner's modes.  Oracle-evaluated
    FP64 residual <= 1e-8 in fewer iterations than the plain factored solve."""
    rt = _rt()
    spec = SPECS[name]()
    say(f"precond factored {prec} {name}")
    op = OProblem(spec)
    with rt.Problem(spec) as p:
        p.set_sigma("factored")
        x = torch.empty(op.n, dtype=torch.float64, device="cuda:0")
        plain = p.solve(x, rtol=1e-8, precision=prec, max_outer=40)
        st = p.solve(x, rtol=1e-8, precision=prec, precond="local", max_outer=40)
        s = host(x)
    res = op.residual_norm(s)
    say(f"   inner {st['iters']} / outer {st['outer_iters']} (plain {plain['iters']} / "
        f"{plain['outer_iters']}), oracle residual {res:.2e}")
    assert st["converged"] and res <= 1e-8
    assert st["iters"] < plain["iters"]


@pytest.mark.parametrize("two_step", [1, 0])
@pytest.mark.parametrize("name", ["slab64", "box8", "box_12x10x9", "box_nu16"])
def test_preconditioned_factored_fp16_basis(name, two_step):
    """The preconditioned FP32 operator with factored scattering on an fp16
    Krylov basis (u = P^-1 v in FP32, the step's result rounded into the
    basis at the basis scale; with 16 frequencies the preconditioner's blocks
    are taken from their fp16 copy): oracle-evaluated FP64 residual <= 1e-8,
    in fewer inner iterations than the unpreconditioned fp16-basis solve."""
    rt = _rt()
    spec = SPECS[name]()
    say(f"precond factored fp16 basis {name} two_step={two_step}")
    op = OProblem(spec)
    with rt.Problem(spec) as p:
        x = torch.empty(op.n, dtype=torch.float64, device="cuda:0")
        plain = p.solve(x, rtol=1e-8, precision="fp16", basis_fp16=1, max_outer=40,
                        two_step=two_step)
        p.set_sigma("factored")
        st = p.solve(x, rtol=1e-8, precision="fp32", precond="local", basis_fp16=1,
                     max_outer=40, two_step=two_step)
        s = host(x)
    res = op.residual_norm(s)
    say(f"   inner {st['iters']} / outer {st['outer_iters']} (plain fp16 basis "
        f"{plain['iters']} / {plain['outer_iters']}), oracle residual {res:.2e}")
    assert st["converged"] and res <= 1e-8
    assert st["iters"] < plain["iters"]


def test_precond_rejections():
    rt = _rt()
    spec = W.small_box(6, 2, 4, 3, nz=4)
    n_r = OProblem(spec).n_r
    with rt.Problem(spec) as p:
        x = torch.empty(p.n, dtype=torch.float64, device="cuda:0")
        with pytest.raises(RuntimeError):
            p.solve(x, precond="local", krylov="bicgstab")
        with pytest.raises(RuntimeError):
            p.solve(x, precond="local", precision="fp16", basis_fp16=1)
        with pytest.raises(RuntimeError):   # FP32 on an fp16 basis: factored form only
            p.solve(x, precond="local", precision="fp32", basis_fp16=1)
        with pytest.raises(RuntimeError):   # ... and preconditioned only
            p.set_sigma("factored")
            try:
                p.solve(x, precision="fp32", basis_fp16=1)
            finally:
                p.set_sigma("dense")
        with pytest.raises(RuntimeError):
            p.solve(x, precond=7)
        y = torch.empty_like(x)
        with pytest.raises(RuntimeError):
            p.apply_precond(x, y, precision="bf16")
    spec.kernel = "explicit"
    spec.kernel_matrix = W.random_symmetric_kernel(n_r, 4)
    with rt.Problem(spec) as p:
        x = torch.zeros(p.n, dtype=torch.float64, device="cuda:0")
        y = torch.empty_like(x)
        with pytest.raises(RuntimeError):
            p.apply_precond(x, y)
        with pytest.raises(RuntimeError):
            p.solve(x, precond="local")
