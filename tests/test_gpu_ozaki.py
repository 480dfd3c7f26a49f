"""GPU parity of the emulated FP64 scattering GEMM (RT_SIGMA_OZAKI: exact
int8 matrix-core products of residues of the scaled operands, rebuilt by the
Chinese remainder theorem) against the oracle's FP64 scattering.

The emulation's only roundings are the scaling of M-hat's rows and L's
columns to 51-bit integers and the final conversion, so every product is
held to 1e-14 of the largest output magnitude, like a true FP64 GEMM
(observed errors of a few 1e-16 on the FP64 path).
"""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import Problem as OProblem, gmres, frequency_grid

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


def _slab(nz, n_mu, n_nu):
    s = W.slab64()
    s.nz, s.n_mu, s.n_nu = nz, n_mu, n_nu
    s.depth = W.log_depth_grid(nz, 1e-4, 1e4)
    return s


def _explicit():
    s = _slab(21, 4, 5)
    s.kernel = "explicit"
    s.kernel_matrix = W.random_symmetric_kernel(20, 9)
    return s


CASES = {
    "slab64": W.slab64,
    "slab_nz37_mu2_nu1": lambda: _slab(37, 2, 1),
    "slab_explicit": _explicit,
    "box8": lambda: W.small_box(8, 4, 8, 5),
    "box_12x10x9": lambda: W.small_box(12, 4, 4, 3, nz=9, ny=10),
    "box_24x20x5": lambda: W.small_box(24, 2, 4, 2, nz=5, ny=20),
    "box_300rays": lambda: W.small_box(6, 4, 5, 15, nz=5),
}


@pytest.mark.parametrize("name", list(CASES))
def test_ozaki_sigma_operator_rhs(name):
    rt = _rt()
    spec = CASES[name]()
    say(f"ozaki {name}")
    op = OProblem(spec)
    L = W.random_field(op.n, 81)
    x = W.random_field(op.n, 82)
    with rt.Problem(spec) as p:
        p.set_sigma("ozaki")
        assert p.footprint().sigma_form == 2
        y = torch.empty(op.n, dtype=torch.float64, device="cuda:0")
        p.apply_sigma(dev(L), dev(x), y)
        got = host(y)
        y2 = torch.empty_like(y)
        p.apply_sigma(dev(L), None, y2)
        got2 = host(y2)
        ya = torch.empty_like(y)
        p.apply(dev(x), ya)
        gota = host(ya)
        b = torch.empty_like(y)
        p.rhs(b)
        gotb = host(b)
    sc = op.scatter(L).ravel()
    errs = (relerr(got, x - sc), relerr(got2, sc), relerr(gota, op.apply(x).ravel()),
            relerr(gotb, op.rhs().ravel()))
    say("   errors " + " ".join(f"{e:.2e}" for e in errs))
    assert max(errs) < 1e-14


@pytest.mark.parametrize("name", ["slab64", "box8", "box_12x10x9"])
def test_ozaki_fp64_solves(name):
    """FP64 GMRES with the emulated GEMM: the oracle-evaluated residual meets
    1e-8 with the dense path's iteration count (within one), and solved to
    rtol 1e-13 the solution agrees with the oracle's to 1e-10; refinement
    with an fp16 inner operator and emulated FP64 outer residuals meets 1e-8."""
    rt = _rt()
    spec = CASES[name]()
    say(f"ozaki solves {name}")
    op = OProblem(spec)
    ref = gmres(op.apply, op.rhs().ravel(), restart=30, tol=1e-13)
    with rt.Problem(spec) as p:
        xd = torch.empty(op.n, dtype=torch.float64, device="cuda:0")
        sd = p.solve(xd, rtol=1e-8)
        p.set_sigma("ozaki")
        x = torch.empty_like(xd)
        st = p.solve(x, rtol=1e-8)
        res = op.residual_norm(host(x))
        st2 = p.solve(x, rtol=1e-13, max_iters=3000)
        diff = np.linalg.norm(host(x) - ref["x"]) / np.linalg.norm(ref["x"])
        xm = torch.empty_like(x)
        stm = p.solve(xm, rtol=1e-8, precision="fp16", max_outer=30)
        resm = op.residual_norm(host(xm))
    say(f"   iters dense {sd['iters']} emulated {st['iters']}, residual {res:.2e}, tight "
        f"diff {diff:.2e}, fp16 refinement residual {resm:.2e}")
    assert st["converged"] and abs(st["iters"] - sd["iters"]) <= 1 and res <= 1e-8
    assert st2["converged"] and diff < 1e-10
    assert stm["converged"] and resm <= 1e-8


def test_ozaki_box64_uniform_field():
    """box64 (6144 rays x 262 144 points): with L = 1 the scattering is the
    closed form (1 - eps) phi_nu / (phi_nu + r) for every point (each row of
    M-hat sums to phi / (phi + r)); the emulated product holds it to 1e-13."""
    rt = _rt()
    spec = W.box64()
    say("box64 emulated Sigma, L = 1")
    _, _, phi = frequency_grid(spec.n_nu, spec.x_max)
    expect = np.tile((1.0 - spec.eps) * phi / (phi + spec.r), spec.n_mu * spec.n_az)
    with rt.Problem(spec) as p:
        p.set_sigma("ozaki")
        n_r, n_s = p.n_r, p.n_s
        L = torch.ones(n_r * n_s, dtype=torch.float64, device="cuda:0")
        y = torch.empty_like(L)
        p.apply_sigma(L, None, y)
        torch.cuda.synchronize()
        del L
        e = torch.tensor(expect, device="cuda:0")
        yv = y.view(n_r, n_s)
        err = 0.0
        for k0 in range(0, n_r, 512):
            err = max(err, ((yv[k0:k0 + 512] - e[k0:k0 + 512, None]).abs() /
                            e[k0:k0 + 512, None]).max().item())
        say(f"   max relative error {err:.3e}")
        del y, yv
        torch.cuda.empty_cache()
    assert err <= 1e-13


def test_ozaki_rejected_with_classes():
    rt = _rt()
    spec = W.small_box(6, 4, 4, 3, nz=5)
    spec.point_class = np.arange(spec.n_s) % 2
    spec.class_coh_frac = [0.1, 0.9]
    with rt.Problem(spec) as p:
        with pytest.raises(rt.RtError) as e:
            p.set_sigma("ozaki")
        assert e.value.code == rt.RT_E_INVALID
