"""rt_apply_operator_noalloc (the operator application that allocates no
device memory) against rt_apply_operator, through the C ABI.

Both run the same kernels on the same inputs, so their outputs must agree
bit for bit; the FP64 result is also held to the oracle at 1e-12 of the
largest magnitude.  Two calls in a row on different problems, the second
smaller than the first, check that the shared per-GPU array carries nothing
from one call into the next.
"""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import Problem as OProblem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _rt():
    from paper_2602_21958_amd import rt
    return rt


def _pair(p, x, precision):
    ya = torch.full_like(x, float("nan"))
    yb = torch.full_like(x, float("nan"))
    p.apply(x, ya, precision=precision)
    p.apply_noalloc(x, yb, precision=precision)
    torch.cuda.synchronize()
    return ya.double().cpu().numpy(), yb.double().cpu().numpy()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_noalloc_equals_apply_operator_two_calls(precision):
    rt = _rt()
    dtype = torch.float64 if precision == "fp64" else torch.float32
    # first a 16^3 box of 768 rays (3.1 M unknowns), then smaller problems
    specs = [("box16_768rays", W.box(16, 4, 8, 24, W.SEED_BASE + 1)),
             ("box_12x10x9", W.small_box(12, 4, 4, 3, nz=9, ny=10)),
             ("slab64", W.slab64())]
    for name, spec in specs:
        say(f"noalloc {precision} {name}")
        with rt.Problem(spec) as p:
            x = torch.tensor(W.random_field(p.n, 31), dtype=dtype, device="cuda:0")
            ya, yb = _pair(p, x, precision)
            assert np.array_equal(ya, yb), f"{name}: noalloc differs from rt_apply_operator"
            assert np.all(np.isfinite(yb))
            if precision == "fp64" and p.n <= 200_000:
                op = OProblem(spec)
                ref = op.apply(W.random_field(op.n, 31)).ravel()
                err = np.max(np.abs(yb - ref)) / np.max(np.abs(ref))
                say(f"   oracle max-relative error {err:.2e}")
                assert err < 1e-12


def test_noalloc_repeated_calls_after_larger_one():
    """A smaller problem right after a larger one, twice, with the stream
    still busy: the result depends only on the current call's input."""
    rt = _rt()
    big = W.box(16, 4, 8, 24, W.SEED_BASE + 1)
    small = W.small_box(8, 4, 8, 5)
    with rt.Problem(big) as pb, rt.Problem(small) as ps:
        xb = torch.tensor(W.random_field(pb.n, 41), dtype=torch.float64, device="cuda:0")
        xs = torch.tensor(W.random_field(ps.n, 42), dtype=torch.float64, device="cuda:0")
        yb = torch.empty_like(xb)
        y1 = torch.empty_like(xs)
        y2 = torch.empty_like(xs)
        ref = torch.empty_like(xs)
        ps.apply(xs, ref)
        pb.apply_noalloc(xb, yb)
        ps.apply_noalloc(xs, y1)
        pb.apply_noalloc(xb, yb)
        ps.apply_noalloc(xs, y2)
        torch.cuda.synchronize()
        r = ref.cpu().numpy()
        assert np.array_equal(y1.cpu().numpy(), r)
        assert np.array_equal(y2.cpu().numpy(), r)


def test_noalloc_rejects_what_it_cannot_serve():
    rt = _rt()
    # 64 x 64 x 17 points x 128 rays = 8 912 896 unknowns: 71.3 MB in FP64
    # (above the 64 MiB array), 35.7 MB in FP32 (served)
    spec = W.box(64, 4, 8, 4, W.SEED_BASE + 7)
    spec.nz = 17
    spec.k_line = W.box_opacity_field(64, 64, 17, W.SEED_BASE + 7)
    with rt.Problem(spec) as p:
        assert p.n == 64 * 64 * 17 * 128
        x64 = torch.zeros(p.n, dtype=torch.float64, device="cuda:0")
        y64 = torch.empty_like(x64)
        with pytest.raises(rt.RtError) as e:
            p.apply_noalloc(x64, y64, precision="fp64")
        assert e.value.code == rt.RT_E_INVALID and "above the fixed" in str(e.value)
        del x64, y64
        x32 = torch.tensor(W.random_field(p.n, 43), dtype=torch.float32, device="cuda:0")
        ya, yb = _pair(p, x32, "fp32")
        assert np.array_equal(ya, yb)
        for prec in ("bf16", "fp16", "bf16x3"):
            with pytest.raises(rt.RtError) as e:
                p.apply_noalloc(x32, torch.empty_like(x32), precision=prec)
            assert e.value.code == rt.RT_E_INVALID
        # the factored scattering form allocates its work vectors
        p.set_sigma("factored")
        with pytest.raises(rt.RtError) as e:
            p.apply_noalloc(x32, torch.empty_like(x32), precision="fp32")
        assert e.value.code == rt.RT_E_INVALID
    lib = rt.raw_lib()
    assert lib.rt_apply_operator_noalloc(None, 0, None, None, None) == rt.RT_E_INVALID
