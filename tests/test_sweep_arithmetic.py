"""Host checks of the FP64 exponential and quotient that the box sweep uses
for a step's weights (the FMA sequences of lam::exp_neg_f64 and
lam::div_f64_normal), emulated with exact decimal arithmetic and one
rounding per operation.  The constants are read from the device source, so
the test follows the kernel.  Reference values: 50-digit decimal exp and
division.  A wrong split of ln 2, a dropped Taylor term or a wrong Newton
step shows up as an error far above the bounds.
"""
import math
import os
import random
import re
from decimal import Decimal, getcontext

import pytest

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_2602_21958_amd", "csrc", "lambda_dev.h")
getcontext().prec = 50


def _const(name):
    text = open(SRC).read()
    m = re.search(r"constexpr double " + name + r" = (0x[0-9a-fp.+-]+);", text)
    assert m, name
    return float.fromhex(m.group(1))


def fma(a, b, c):
    return float(Decimal(a) * Decimal(b) + Decimal(c))


INV_FACT = [float(Decimal(1) / Decimal(math.factorial(n))) for n in range(18)]


def exp_neg(d, inv_ln2, hi, lo):
    dc = min(d, 800.0)
    mn = float(round(dc * -inv_ln2))         # rint: round half to even
    r = fma(mn, hi, dc)
    r = fma(mn, lo, r)
    p = INV_FACT[13]
    for k in range(12, -1, -1):
        p = fma(p, -r, INV_FACT[k])
    return math.ldexp(p, int(mn))


def div_normal(num, d, rel_rcp_err):
    r = (1.0 / d) * (1.0 + rel_rcp_err)       # hardware reciprocal, perturbed
    r = fma(r, fma(-d, r, 1.0), r)
    r = fma(r, fma(-d, r, 1.0), r)
    q = num * r
    return fma(fma(-d, q, num), r, q)


def test_ln2_split():
    inv_ln2, hi, lo = _const("kInvLn2"), _const("kLn2Hi"), _const("kLn2Lo")
    ln2 = Decimal(2).ln()
    assert abs(Decimal(hi) + Decimal(lo) - ln2) < Decimal("1e-29")
    # low 12 significand bits of the head are zero: n * head is exact for n < 2^12
    m, _ = math.frexp(hi)
    assert (int(m * 2 ** 53) & 0xFFF) == 0
    assert inv_ln2 == float(1 / ln2)


def test_exponential_within_one_ulp():
    inv_ln2, hi, lo = _const("kInvLn2"), _const("kLn2Hi"), _const("kLn2Lo")
    rnd = random.Random(5)
    ds = [0.5, 0.5 + 2 ** -40, math.log(2), 1.0, 2.0, 10.0, 100.0, 700.0] + \
         [math.exp(rnd.uniform(math.log(0.5), math.log(700.0))) for _ in range(1500)]
    worst = 0.0
    for d in ds:
        ref = Decimal(-d).exp()
        got = exp_neg(d, inv_ln2, hi, lo)
        worst = max(worst, float(abs((Decimal(got) - ref) / ref)))
    # 1.14e-16 measured; one Taylor term fewer gives 2.6e-16
    assert worst < 1.5e-16


def test_exponential_underflow_and_large_steps():
    inv_ln2, hi, lo = _const("kInvLn2"), _const("kLn2Hi"), _const("kLn2Lo")
    assert exp_neg(800.0, inv_ln2, hi, lo) == 0.0
    assert exp_neg(1e6, inv_ln2, hi, lo) == 0.0
    assert exp_neg(1e300, inv_ln2, hi, lo) == 0.0
    # subnormal range: absolute error below the smallest subnormal spacing
    for d in (720.0, 740.0, 744.0):
        ref = Decimal(-d).exp()
        assert abs(Decimal(exp_neg(d, inv_ln2, hi, lo)) - ref) <= Decimal(2.0 ** -1074)


@pytest.mark.parametrize("rel_rcp_err", [2.0 ** -22, -(2.0 ** -22), 1e-9, 0.0])
def test_quotient_correctly_rounded_for_sweep_operands(rel_rcp_err):
    inv_ln2, hi, lo = _const("kInvLn2"), _const("kLn2Hi"), _const("kLn2Lo")
    rnd = random.Random(7)
    worst = 0.0
    for _ in range(800):
        d = math.exp(rnd.uniform(math.log(0.5), math.log(1e6)))
        num = 1.0 - exp_neg(d, inv_ln2, hi, lo)
        ref = Decimal(num) / Decimal(d)
        got = div_normal(num, d, rel_rcp_err)
        worst = max(worst, float(abs(Decimal(got) - ref)) / math.ulp(float(ref)))
    assert worst <= 0.5 + 1e-9
