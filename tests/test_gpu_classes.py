"""GPU parity of per-point scattering classes (Sec. 3.3: the block Psi_[i]
of eq. Sigma may differ between points) against the oracle.

Each class's columns are gathered, multiplied by the class's Mhat on the
same MFMA GEMM as the one-kernel path, and scattered back, so FP64 results
agree with the oracle to 1e-12 of the largest magnitude; FP32 to 2e-5.
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


def slab_classes():
    s = W.slab64()
    s.point_class = (np.arange(64) // 8) % 3          # depth bands
    s.class_coh_frac = [0.0, 0.5, 1.0]
    return s


def box_layer_classes():
    s = W.small_box(12, 4, 4, 3, nz=9, ny=10)
    s.point_class = np.repeat(np.arange(9) % 2, 10 * 12)
    s.class_coh_frac = [0.2, 0.9]
    return s


def box_random_classes():
    s = W.small_box(8, 4, 8, 5)
    s.point_class = np.random.default_rng(3).integers(0, 4, s.n_s)
    s.class_coh_frac = [0.0, 0.3, 0.6, 1.0]
    s.eps = np.geomspace(1e-4, 0.1, s.n_s)
    return s


def explicit_classes():
    s = W.slab64()
    s.nz, s.n_mu, s.n_nu = 37, 4, 3
    s.depth = W.log_depth_grid(37, 1e-3, 1e3)
    s.kernel = "explicit"
    s.kernel_matrix = None
    # kernels near the physical scale: a random symmetric perturbation of a
    # constant, so that the operator stays well conditioned
    n_r = 12
    s.class_kernels = np.stack([1.0 + 0.1 * W.random_symmetric_kernel(n_r, c) /
                                np.abs(W.random_symmetric_kernel(n_r, c)).max()
                                for c in (7, 8)])
    s.point_class = np.arange(37) % 2
    return s


CASES = {"slab_classes": slab_classes, "box_layer_classes": box_layer_classes,
         "box_random_classes": box_random_classes, "explicit_classes": explicit_classes}


@pytest.mark.parametrize("name", list(CASES))
def test_classes_sigma_operator_rhs_fp64(name):
    rt = _rt()
    spec = CASES[name]()
    say(f"classes fp64 {name}")
    op = OProblem(spec)
    L = W.random_field(op.n, 71)
    x = W.random_field(op.n, 72)
    with rt.Problem(spec) as p:
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
    assert max(errs) < 1e-12


@pytest.mark.parametrize("name", list(CASES))
def test_classes_sigma_fp32(name):
    rt = _rt()
    spec = CASES[name]()
    op = OProblem(spec)
    L = W.random_field(op.n, 73).astype(np.float32)
    x = W.random_field(op.n, 74).astype(np.float32)
    with rt.Problem(spec) as p:
        y = torch.empty(op.n, dtype=torch.float32, device="cuda:0")
        p.apply_sigma(dev(L, torch.float32), dev(x, torch.float32), y, precision="fp32")
        got = host(y)
    ref = x - op.scatter(L.astype(np.float64)).ravel()
    assert relerr(got, ref) < 2e-5


@pytest.mark.parametrize("name", ["slab_classes", "box_layer_classes", "box_random_classes"])
def test_classes_solves(name):
    """FP64 GMRES to the oracle's residual 1e-8 and, at rtol 1e-13, to the
    oracle's solution within 1e-10; FP32-operator refinement to 1e-8."""
    rt = _rt()
    spec = CASES[name]()
    say(f"classes solves {name}")
    op = OProblem(spec)
    ref = gmres(op.apply, op.rhs().ravel(), restart=30, tol=1e-13)
    with rt.Problem(spec) as p:
        x = torch.empty(op.n, dtype=torch.float64, device="cuda:0")
        st = p.solve(x, rtol=1e-8)
        res = op.residual_norm(host(x))
        st2 = p.solve(x, rtol=1e-13, max_iters=3000)
        diff = np.linalg.norm(host(x) - ref["x"]) / np.linalg.norm(ref["x"])
        xm = torch.empty_like(x)
        stm = p.solve(xm, rtol=1e-8, precision="fp32", max_outer=30)
        resm = op.residual_norm(host(xm))
    say(f"   iters {st['iters']}, residual {res:.2e}, tight diff {diff:.2e}, "
        f"fp32 refinement residual {resm:.2e}")
    assert st["converged"] and res <= 1e-8
    assert st2["converged"] and diff < 1e-10
    assert stm["converged"] and resm <= 1e-8


def test_classes_reject_what_they_do_not_serve():
    rt = _rt()
    spec = box_layer_classes()
    with rt.Problem(spec) as p:
        assert p.footprint().sigma_rank == 0
        x32 = torch.zeros(p.n, dtype=torch.float32, device="cuda:0")
        for prec in ("bf16", "fp16", "bf16x3"):
            with pytest.raises(rt.RtError) as e:
                p.apply(x32, torch.empty_like(x32), precision=prec)
            assert e.value.code == rt.RT_E_INVALID
        with pytest.raises(rt.RtError):
            p.set_sigma("factored")
        with pytest.raises(rt.RtError):
            p.apply_noalloc(x32, torch.empty_like(x32), precision="fp32")
        eng = rt.Batch(precision="fp64", hbm_budget=1 << 30, max_slots=4)
        try:
            with pytest.raises(rt.RtError):
                eng.submit(p, torch.empty(p.n, dtype=torch.float64, device="cuda:0"))
        finally:
            eng.close()
    bad = box_layer_classes()
    bad.point_class = bad.point_class.copy()
    bad.point_class[5] = 7
    with pytest.raises(rt.RtError) as e:
        rt.Problem(bad)
    assert e.value.code == rt.RT_E_INVALID
