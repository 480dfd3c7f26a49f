"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs.

FP64 tolerances: single applications of Lambda, Sigma and the operator agree
to 1e-12 of the largest magnitude (rounding order only); solves are checked
by the oracle-evaluated FP64 residual and against the oracle's own GMRES
iterate.  FP32 applications agree to a few FP32 ulps (2e-5 relative).
"""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import Problem as OProblem, gmres, bicgstab

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


# ------------------------------------------------------------------ specs
def slab(nz=64, n_mu=8, n_nu=21, formal="linear_sc", eps=1e-4):
    s = W.slab64()
    s.nz, s.n_mu, s.n_nu, s.formal, s.eps = nz, n_mu, n_nu, formal, eps
    s.depth = W.log_depth_grid(nz, 1e-4, 1e4)
    return s


SLABS = {
    "slab64": lambda: W.slab64(),
    "slab_ie": lambda: slab(formal="implicit_euler"),
    "slab_nz37_mu2_nu1": lambda: slab(nz=37, n_mu=2, n_nu=1),
    "slab_nz300": lambda: slab(nz=300, n_mu=4, n_nu=7),
    "slab_eps_field": lambda: slab(nz=20, n_mu=6, n_nu=5, eps=np.linspace(1e-4, 0.5, 20)),
}

BOXES = {
    "box8": lambda: W.small_box(8, 4, 8, 5),
    "box_12x10x9": lambda: W.small_box(12, 4, 4, 3, nz=9, ny=10),
    "box16_shallow": lambda: W.small_box(16, 8, 8, 3, nz=6),
    "box_1x1x5": lambda: W.small_box(1, 2, 4, 2, nz=5, ny=1),
    # planes of 257..1024 points (two points per thread, two LDS sets) and of
    # more than 1024 (FP64: eight points per thread, one set)
    "box_24x20x5": lambda: W.small_box(24, 2, 4, 2, nz=5, ny=20),
    "box_40x36x4": lambda: W.small_box(40, 2, 4, 2, nz=4, ny=36),
}

ALL = {**SLABS, **BOXES}


@pytest.mark.parametrize("name", list(ALL))
def test_tables_match_oracle(name):
    rt = _rt()
    spec = ALL[name]()
    say(f"tables {name}")
    op = OProblem(spec)
    with rt.Problem(spec) as p:
        t = p.tables()
    assert relerr(t["mhat"], op.mhat) < 1e-13
    assert np.allclose(t["mu_ray"], op.mu_ray, rtol=0, atol=1e-15)
    assert np.allclose(t["w_ray"], op.w_ray, rtol=1e-14, atol=0)
    assert np.allclose(t["phi_ray"], op.phi_ray, rtol=1e-13, atol=0)


@pytest.mark.parametrize("with_bc", [False, True])
@pytest.mark.parametrize("name", list(ALL))
def test_lambda_fp64(name, with_bc):
    rt = _rt()
    spec = ALL[name]()
    spec.i_top, spec.i_bot = 0.3, 1.0
    say(f"lambda fp64 {name} bc={with_bc}")
    op = OProblem(spec)
    s = W.random_field(op.n, 11)
    with rt.Problem(spec) as p:
        out = torch.empty(op.n, dtype=torch.float64, device="cuda:0")
        p.apply_lambda(dev(s), out, with_bc=with_bc)
        got = host(out)
    ref = op.lam(s.reshape(op.n_r, op.n_s), with_bc=with_bc).ravel()
    assert relerr(got, ref) < 1e-12


@pytest.mark.parametrize("name", ["slab64", "box8", "box_12x10x9", "box_24x20x5", "box_40x36x4"])
def test_lambda_fp32(name):
    rt = _rt()
    spec = ALL[name]()
    say(f"lambda fp32 {name}")
    op = OProblem(spec)
    s = W.random_field(op.n, 12, positive=True)
    with rt.Problem(spec) as p:
        out = torch.empty(op.n, dtype=torch.float32, device="cuda:0")
        p.apply_lambda(dev(s, torch.float32), out, precision="fp32")
        got = host(out)
    ref = op.lam(s.astype(np.float32).astype(np.float64).reshape(op.n_r, op.n_s),
                 with_bc=False).ravel()
    # per entry: the source is positive, so every term of the recurrence is
    # positive and each intensity carries a few FP32 roundings of its own size;
    # the first node of every ray (zero incoming radiation) is exactly zero
    edge = ref == 0
    assert np.all(ref[~edge] > 0)
    assert edge.sum() == op.n_r * (op.n_s // spec.nz)
    assert np.all(got[edge] == 0)
    rel = np.abs(got[~edge] - ref[~edge]) / ref[~edge]
    say(f"   worst per-entry relative error {rel.max():.2e}")
    assert rel.max() < 2e-5


@pytest.mark.parametrize("name", list(ALL))
def test_sigma_fp64(name):
    rt = _rt()
    spec = ALL[name]()
    say(f"sigma fp64 {name}")
    op = OProblem(spec)
    L = W.random_field(op.n, 13)
    x = W.random_field(op.n, 14)
    with rt.Problem(spec) as p:
        y = torch.empty(op.n, dtype=torch.float64, device="cuda:0")
        p.apply_sigma(dev(L), dev(x), y)
        got = host(y)
        y2 = torch.empty_like(y)
        p.apply_sigma(dev(L), None, y2)
        got2 = host(y2)
    sc = op.scatter(L)
    assert relerr(got, x - sc.ravel()) < 1e-12
    assert relerr(got2, sc.ravel()) < 1e-12


@pytest.mark.parametrize("name", ["slab64", "box8", "box_12x10x9"])
def test_sigma_fp32(name):
    rt = _rt()
    spec = ALL[name]()
    say(f"sigma fp32 {name}")
    op = OProblem(spec)
    L = W.random_field(op.n, 15).astype(np.float32)
    x = W.random_field(op.n, 16).astype(np.float32)
    with rt.Problem(spec) as p:
        y = torch.empty(op.n, dtype=torch.float32, device="cuda:0")
        p.apply_sigma(dev(L, torch.float32), dev(x, torch.float32), y, precision="fp32")
        got = host(y)
    ref = x - op.scatter(L.astype(np.float64)).ravel()
    assert relerr(got, ref) < 2e-5


@pytest.mark.parametrize("name", list(ALL))
def test_operator_and_rhs_fp64(name):
    rt = _rt()
    spec = ALL[name]()
    say(f"operator fp64 {name}")
    op = OProblem(spec)
    x = W.random_field(op.n, 17)
    with rt.Problem(spec) as p:
        y = torch.empty(op.n, dtype=torch.float64, device="cuda:0")
        p.apply(dev(x), y)
        got = host(y)
        b = torch.empty_like(y)
        p.rhs(b)
        got_b = host(b)
        inten = torch.empty_like(y)
        p.intensity(dev(x), inten)
        got_i = host(inten)
    assert relerr(got, op.apply(x).ravel()) < 1e-12
    assert relerr(got_b, op.rhs().ravel()) < 1e-12
    assert relerr(got_i, op.intensity(x).ravel()) < 1e-12


def test_box32_operator_full_size():
    """The 32^3 box workload at full size (2048 rays x 32768 points)."""
    rt = _rt()
    spec = W.box32()
    say("box32 full-size operator")
    op = OProblem(spec)
    x = W.random_field(op.n, 18)
    with rt.Problem(spec) as p:
        y = torch.empty(op.n, dtype=torch.float64, device="cuda:0")
        p.apply(dev(x), y)
        got = host(y)
    ref = op.apply(x).ravel()
    assert relerr(got, ref) < 1e-12


def oracle_at_step(op, b, restart, iters):
    """The oracle's GMRES(restart) iterate after exactly `iters` Arnoldi
    steps (no stopping test): the iterate a library solve that took `iters`
    steps computes in exact arithmetic, whatever step each side's rounding
    let cross the tolerance."""
    return gmres(op.apply, b, restart=restart, tol=0.0, maxiter=iters)["x"]


@pytest.mark.parametrize("two_step", [1, 0])
@pytest.mark.parametrize("name", ["slab64", "box8"])
def test_gmres_fp64_matches_oracle(name, two_step):
    """FP64 GMRES(30) against the oracle's: Arnoldi steps in pairs (the
    default) and one at a time.  Residual estimates follow the oracle's to
    1e-8 over 20 steps; the solution is the oracle's iterate at the same
    step to 1e-9 (Gram-Schmidt rounding only)."""
    rt = _rt()
    spec = ALL[name]()
    say(f"gmres fp64 {name} two_step={two_step}")
    op = OProblem(spec)
    b = op.rhs().ravel()
    ref = gmres(op.apply, b, restart=30, tol=1e-8)
    with rt.Problem(spec) as p:
        x = torch.empty(op.n, dtype=torch.float64, device="cuda:0")
        st = p.solve(x, rtol=1e-8, restart=30, two_step=two_step)
        s = host(x)
    assert st["converged"]
    assert abs(st["iters"] - ref["iters"]) <= 1
    # residual histories agree over the first 20 steps
    h = np.array(st["history"][:20])
    hr = np.array(ref["history"][:20])
    assert np.max(np.abs(h - hr) / hr) < 1e-8
    assert op.residual_norm(s) <= 1e-8
    xr = ref["x"] if st["iters"] == ref["iters"] else oracle_at_step(op, b, 30, st["iters"])
    diff = np.linalg.norm(s - xr) / np.linalg.norm(xr)
    say(f"   iters {st['iters']} (oracle {ref['iters']}), diff to the same-step iterate "
        f"{diff:.2e}")
    assert diff < 1e-9


@pytest.mark.parametrize("restart", [30, 7])
@pytest.mark.parametrize("name", ["slab64", "box8", "box_24x20x5"])
def test_gmres_two_step_matches_oracle(name, restart):
    """FP64 GMRES with the Arnoldi steps taken in pairs (two_step: u1 = K v_j,
    u2 = K u1 orthogonalised together; an odd restart ends each cycle with
    one single step), also with short restarts, beside the one-step form.
    Same Krylov iterates in exact arithmetic: the iteration counts are within
    2 % (at least one) of the oracle's (many short cycles compound rounding
    differences near the tolerance), the oracle-evaluated residual meets
    1e-8, the residual estimates follow the oracle's to 1e-8 relative over 20
    steps, and each solution is the oracle's iterate at its own step count
    to 1e-9 on slab64 and box8.  Two iterates whose relative residuals are
    both at most 1e-8 differ by at most 2e-8 kappa(A) relative to x; the
    24x20x5 box (GMRES(30) needs 94 steps, GMRES(7) 203) is the worst
    conditioned case here, and there the library's iterates (classical
    Gram-Schmidt, in pairs or one step at a time) differ from the oracle's
    (modified Gram-Schmidt) by 1.5e-8 .. 6.8e-8, held to 2e-7.  Solved to
    rtol 1e-13 both forms agree with the oracle to 1e-10 on the same box
    (test_gmres_tight_solution_matches_oracle)."""
    rt = _rt()
    spec = ALL[name]()
    say(f"gmres two-step {name} m={restart}")
    op = OProblem(spec)
    b = op.rhs().ravel()
    ref = gmres(op.apply, b, restart=restart, tol=1e-8)
    out = {}
    with rt.Problem(spec) as p:
        for two in (1, 0):
            x = torch.empty(op.n, dtype=torch.float64, device="cuda:0")
            out[two] = (p.solve(x, rtol=1e-8, restart=restart, two_step=two), host(x))
    say(f"   iters: pairs {out[1][0]['iters']}, one step {out[0][0]['iters']}, "
        f"oracle {ref['iters']}")
    tol_it = max(1, ref["iters"] // 50)
    for two, (st, s) in out.items():
        assert st["converged"]
        assert abs(st["iters"] - ref["iters"]) <= tol_it, (two, st["iters"], ref["iters"])
        h = np.array(st["history"][:20])
        hr = np.array(ref["history"][:20])
        assert np.max(np.abs(h - hr) / hr) < 1e-8
        assert op.residual_norm(s) <= 1e-8
        xr = ref["x"] if st["iters"] == ref["iters"] else oracle_at_step(op, b, restart,
                                                                         st["iters"])
        diff = np.linalg.norm(s - xr) / np.linalg.norm(xr)
        say(f"   two_step={two}: diff to the oracle iterate at step {st['iters']}: {diff:.2e}")
        assert diff < (2e-7 if name == "box_24x20x5" else 1e-9)


@pytest.mark.parametrize("two_step", [1, 0])
@pytest.mark.parametrize("name", ["slab64", "box8", "box_24x20x5"])
def test_gmres_tight_solution_matches_oracle(name, two_step):
    """Solves at rtol 1e-13 agree with the oracle's to 1e-10 (2-norm
    relative), with the Arnoldi steps in pairs and one at a time."""
    rt = _rt()
    spec = ALL[name]()
    say(f"gmres tight {name} two_step={two_step}")
    op = OProblem(spec)
    ref = gmres(op.apply, op.rhs().ravel(), restart=30, tol=1e-13)
    assert ref["converged"]
    with rt.Problem(spec) as p:
        x = torch.empty(op.n, dtype=torch.float64, device="cuda:0")
        st = p.solve(x, rtol=1e-13, restart=30, two_step=two_step, max_iters=3000)
        s = host(x)
    diff = np.linalg.norm(s - ref["x"]) / np.linalg.norm(ref["x"])
    say(f"   iters {st['iters']} (oracle {ref['iters']}), relres {st['relres']:.2e}, "
        f"solution diff {diff:.2e}")
    assert st["converged"]
    assert diff < 1e-10


@pytest.mark.parametrize("two_step", [1, 0])
@pytest.mark.parametrize("prec", ["fp16", "bf16x3", "bf16"])
@pytest.mark.parametrize("name", ["slab64", "box8", "small_box_ragged"])
def test_mixed_refinement_fp16_basis(name, prec, two_step):
    """Refinement whose inner GMRES keeps its basis in (scaled) fp16, with the
    inner Arnoldi steps in pairs (the default) or one at a time, reaches the
    same oracle-evaluated FP64 residual as with the FP32 basis."""
    rt = _rt()
    spec = (W.small_box(12, 4, 8, 9, seed=5, nz=9, ny=10) if name == "small_box_ragged"
            else ALL[name]())
    say(f"mixed {prec} fp16 basis {name} two_step={two_step}")
    op = OProblem(spec)
    with rt.Problem(spec) as p:
        x = torch.empty(op.n, dtype=torch.float64, device="cuda:0")
        st = p.solve(x, rtol=1e-8, precision=prec, max_outer=30, basis_fp16=1,
                     two_step=two_step)
        s = host(x)
        ref = p.solve(torch.empty_like(x), rtol=1e-8, precision=prec, max_outer=30)
    res = op.residual_norm(s)
    say(f"   {prec} {name}: converged={st['converged']} outer={st['outer_iters']} "
        f"inner={st['iters']} (FP32 basis: outer={ref['outer_iters']}) residual={res:.3e}")
    if ref["converged"]:
        assert st["converged"], st
        assert res <= 1e-8
        # the basis rounding (2^-11) must not cost the refinement extra steps
        # beyond a small margin
        assert st["outer_iters"] <= ref["outer_iters"] + 2, (st, ref)
    else:
        assert prec == "bf16", ref


def test_fp16_basis_rejected_outside_16bit_operators():
    rt = _rt()
    spec = W.small_box(8, 4, 4, 4, seed=1)
    with rt.Problem(spec) as p:
        x = torch.empty(p.n, dtype=torch.float64, device="cuda:0")
        for prec in ("fp64", "fp32"):
            with pytest.raises(rt.RtError):
                p.solve(x, precision=prec, basis_fp16=1)
        eng = rt.Batch(precision="fp16", hbm_budget=1 << 30, max_slots=4)
        try:
            with pytest.raises(rt.RtError):
                eng.submit(p, x, basis_fp16=1)
        finally:
            eng.close()
    # an explicit kernel whose scattering rows sum far above 1 (here ~40/phi)
    # voids the headroom of the basis scale: refused (the problem is valid)
    bad = slab(nz=12, n_mu=2, n_nu=3)
    n_r = 2 * 3
    bad.kernel, bad.kernel_matrix = "explicit", np.full((n_r, n_r), 40.0)
    with rt.Problem(bad) as p:
        x = torch.empty(p.n, dtype=torch.float64, device="cuda:0")
        with pytest.raises(rt.RtError):
            p.solve(x, precision="fp16", basis_fp16=1)
        y = torch.empty_like(x)
        p.apply(x.fill_(1.0), y)


@pytest.mark.parametrize("prec", ["fp64", "fp16"])
def test_gmres_with_dots_fused_into_sigma(prec, monkeypatch):
    """The opt-in variant that forms the Arnoldi inner products in the Sigma
    GEMM's epilogue reaches the same FP64 residual as the default path."""
    rt = _rt()
    monkeypatch.setenv("RTSN_FUSED_DOTS", "1")
    spec = W.small_box(12, 4, 8, 9, seed=5, nz=9, ny=10)
    say(f"gmres fused dots {prec}")
    op = OProblem(spec)
    with rt.Problem(spec) as p:
        x = torch.empty(op.n, dtype=torch.float64, device="cuda:0")
        st = p.solve(x, rtol=1e-8, restart=30, precision=prec)
        s = host(x)
    assert st["converged"]
    assert op.residual_norm(s) <= 1e-8


@pytest.mark.parametrize("name,precision,basis16",
                         [("slab64", "fp64", 0), ("box8", "fp64", 0), ("slab64", "fp16", 0),
                          ("box8", "fp16", 1)])
def test_batched_status_reads_give_identical_results(name, precision, basis16, monkeypatch):
    """Reading the Arnoldi status every 4 steps (the default for small
    problems; steps past the stop are launched and discarded) gives the same
    bits, iteration counts and residual history as reading after every step."""
    rt = _rt()
    spec = ALL[name]()
    monkeypatch.setenv("RTSN_GEMM16_CFG", "2")   # one tile shape for all three problems
    out = {}
    for every in ("1", "4", "7"):
        monkeypatch.setenv("RTSN_STATUS_EVERY", every)
        with rt.Problem(spec) as p:
            x = torch.empty(p.n, dtype=torch.float64, device="cuda:0")
            st = p.solve(x, rtol=1e-8, restart=30, precision=precision, basis_fp16=basis16)
            out[every] = (st, host(x))
    say(f"status every 1/4/7 {name} {precision}: iters "
        f"{[out[e][0]['iters'] for e in out]}")
    for every in ("4", "7"):
        assert out[every][0]["iters"] == out["1"][0]["iters"]
        assert out[every][0]["outer_iters"] == out["1"][0]["outer_iters"]
        assert out[every][0]["history"] == out["1"][0]["history"]
        assert np.array_equal(out[every][1], out["1"][1])


def test_eps_one_is_one_iteration():
    rt = _rt()
    spec = W.slab64()
    spec.eps = 1.0
    say("eps=1")
    with rt.Problem(spec) as p:
        x = torch.empty(p.n, dtype=torch.float64, device="cuda:0")
        st = p.solve(x, rtol=1e-12)
        s = host(x)
    assert st["converged"] and st["iters"] == 1
    assert np.allclose(s, 1.0, rtol=1e-14)


def test_zero_rhs_gives_zero():
    rt = _rt()
    spec = W.slab64()
    say("zero rhs")
    with rt.Problem(spec) as p:
        x = torch.ones(p.n, dtype=torch.float64, device="cuda:0")
        b = torch.zeros(p.n, dtype=torch.float64, device="cuda:0")
        st = p.solve(x, b=b)
        assert st["iters"] == 0 and st["converged"]
        assert not torch.any(x).item()


@pytest.mark.parametrize("name", ["slab64", "box8", "box_12x10x9"])
def test_bicgstab_fp64(name):
    rt = _rt()
    spec = ALL[name]()
    say(f"bicgstab {name}")
    op = OProblem(spec)
    ref = bicgstab(op.apply, op.rhs().ravel(), tol=1e-8)
    with rt.Problem(spec) as p:
        x = torch.empty(op.n, dtype=torch.float64, device="cuda:0")
        st = p.solve(x, rtol=1e-8, krylov="bicgstab")
        s = host(x)
    assert st["converged"]
    assert op.residual_norm(s) <= 1e-8
    # BiCGStab's residual is not monotone and its recurrences amplify the
    # rounding of the inner products (which differ in reduction order between
    # the two implementations), so the step at which 1e-8 is first crossed
    # moves by a few iterations; the FP64 residual above is the criterion.
    assert abs(st["iters"] - ref["iters"]) <= max(2, ref["iters"] // 10)


def test_invalid_arguments_raise():
    rt = _rt()
    spec = W.slab64()
    spec.depth = spec.depth[::-1].copy()
    with pytest.raises(rt.RtError) as e:
        rt.Problem(spec)
    assert e.value.code == rt.RT_E_INVALID
    spec = W.slab64()
    spec.eps = float("nan")
    with pytest.raises(rt.RtError) as e:
        rt.Problem(spec)
    assert e.value.code == rt.RT_E_NONFINITE
    spec = W.slab64()
    with rt.Problem(spec) as p:
        x = torch.empty(p.n, dtype=torch.float64, device="cuda:0")
        with pytest.raises(rt.RtError):
            p.apply(x, x)
        with pytest.raises(rt.RtError):
            p.solve(x, restart=0)


@pytest.mark.parametrize("name", ["slab64", "box8"])
def test_mixed_fp32_refinement_reaches_fp64_residual(name):
    """FP64 iterative refinement around an FP32 inner GMRES: the oracle-evaluated
    FP64 residual of the result meets 1e-8."""
    rt = _rt()
    spec = ALL[name]()
    say(f"mixed fp32 IR {name}")
    op = OProblem(spec)
    with rt.Problem(spec) as p:
        x = torch.empty(op.n, dtype=torch.float64, device="cuda:0")
        st = p.solve(x, rtol=1e-8, precision="fp32")
        s = host(x)
    assert st["converged"], st
    assert st["outer_iters"] >= 2
    assert op.residual_norm(s) <= 1e-8


def test_profile_counts_launches():
    rt = _rt()
    spec = W.slab64()
    with rt.Problem(spec) as p:
        x = dev(W.random_field(p.n, 3))
        y = torch.empty_like(x)
        x32 = x.float()
        y32 = torch.empty_like(x32)
        p.apply_precond(x, y)        # builds the preconditioner before timing
        rt.profile_enable(True)
        for k in rt.KCLASS:
            rt.profile_read(k)
        for _ in range(3):
            p.apply(x, y)
        for prec in ("fp32", "fp16"):
            p.apply(x32, y32, precision=prec)
        p.apply_precond(x, y)
        rt.profile_enable(False)
        got = {k: rt.profile_read(k) for k in rt.KCLASS}
    # FP64 arithmetic, the lower precisions and the preconditioner are
    # counted apart
    assert got["lambda"][0] == 3 and got["sigma"][0] == 3
    assert got["lambda_lo"][0] == 2 and got["sigma_lo"][0] == 2
    assert got["precond"][0] == 1
    assert all(ms > 0 for k, (n, ms) in got.items() if k != "arnoldi")


# 16-bit scattering GEMM: bound from operand rounding.  With unit roundoff u
# of the stored operands, each product carries at most ~2u relative error, so
# |y - y_ref| <= c u (1-eps_i) (|Mhat| |L|)_{k,i} + FP32 rounding of y.
U16 = {"bf16": 2.0 ** -8, "fp16": 2.0 ** -11, "bf16x3": 2.0 ** -15}


@pytest.mark.parametrize("prec", ["bf16", "fp16", "bf16x3"])
@pytest.mark.parametrize("name", ["slab64", "slab_nz37_mu2_nu1", "box8", "box_12x10x9",
                                  "box_1x1x5"])
def test_sigma_16bit_within_rounding_bound(name, prec):
    rt = _rt()
    spec = ALL[name]()
    say(f"sigma {prec} {name}")
    op = OProblem(spec)
    L = W.random_field(op.n, 21).astype(np.float32)
    x = W.random_field(op.n, 22).astype(np.float32)
    with rt.Problem(spec) as p:
        y = torch.empty(op.n, dtype=torch.float32, device="cuda:0")
        p.apply_sigma(dev(L, torch.float32), dev(x, torch.float32), y, precision=prec)
        got = host(y).reshape(op.n_r, op.n_s)
    L64 = L.astype(np.float64).reshape(op.n_r, op.n_s)
    ref = x.astype(np.float64).reshape(op.n_r, op.n_s) - op.scatter(L64)
    absprod = op.albedo[None, :] * (np.abs(op.mhat) @ np.abs(L64))
    # fp16: entries below the fp16 subnormal range of each scaled row vanish
    floor = 0.0
    if prec == "fp16":
        rowmax = np.abs(op.mhat).max(axis=1)
        floor = (6e-8 * rowmax)[:, None] * np.abs(L64).sum(axis=0)[None, :]
    bound = 3.0 * U16[prec] * absprod + floor + 2e-7 * np.abs(ref) + 1e-30
    err = np.abs(got - ref)
    assert np.all(err <= bound), float(np.max(err / bound))


@pytest.mark.parametrize("prec", ["bf16", "fp16", "bf16x3"])
@pytest.mark.parametrize("cfg", [0, 1, 2, 3, 4])
def test_sigma_16bit_every_tile_shape(cfg, prec, monkeypatch):
    """Every candidate tile shape of the 16-bit GEMM (forced instead of tuned)
    on a ragged problem: 288 rays (not a multiple of the 64-wide K stage or
    of the 128/256-row tiles) and 1080 points (not a multiple of the column
    tiles), several K stages and row tiles."""
    rt = _rt()
    monkeypatch.setenv("RTSN_GEMM16_CFG", str(cfg))
    spec = W.small_box(12, 4, 8, 9, seed=5, nz=9, ny=10)
    say(f"sigma {prec} tile shape {cfg}")
    op = OProblem(spec)
    assert (op.n_r, op.n_s) == (288, 1080)
    L = W.random_field(op.n, 23).astype(np.float32)
    x = W.random_field(op.n, 24).astype(np.float32)
    with rt.Problem(spec) as p:
        y = torch.empty(op.n, dtype=torch.float32, device="cuda:0")
        p.apply_sigma(dev(L, torch.float32), dev(x, torch.float32), y, precision=prec)
        got = host(y).reshape(op.n_r, op.n_s)
    L64 = L.astype(np.float64).reshape(op.n_r, op.n_s)
    ref = x.astype(np.float64).reshape(op.n_r, op.n_s) - op.scatter(L64)
    absprod = op.albedo[None, :] * (np.abs(op.mhat) @ np.abs(L64))
    floor = 0.0
    if prec == "fp16":
        rowmax = np.abs(op.mhat).max(axis=1)
        floor = (6e-8 * rowmax)[:, None] * np.abs(L64).sum(axis=0)[None, :]
    bound = 3.0 * U16[prec] * absprod + floor + 2e-7 * np.abs(ref) + 1e-30
    err = np.abs(got - ref)
    assert np.all(err <= bound), float(np.max(err / bound))


@pytest.mark.parametrize("prec", ["bf16", "fp16", "bf16x3"])
@pytest.mark.parametrize("shape", [(8, 8, 8, 4, 8, 8), (8, 8, 6, 2, 4, 5), (12, 12, 9, 4, 4, 6),
                                   (40, 40, 6, 2, 4, 4)])
def test_operator_16bit_box(shape, prec):
    """Whole 16-bit operator y = x - (1-eps) Mhat Lambda x on boxes whose
    frequency count is a multiple of 4 (a k4 group of rays is one ordinate's)
    or not (k4 groups straddle two ordinates; partial last group), with planes
    of up to 1024 points (two LDS sets) and of more (one set).  Bound: 16-bit
    operand rounding of Mhat and of the FP32 Lambda output, plus the FP32
    Lambda itself."""
    rt = _rt()
    nx, ny, nz, n_mu, n_az, n_nu = shape
    spec = W.small_box(nx, n_mu, n_az, n_nu, seed=7, nz=nz, ny=ny)
    say(f"operator {prec} box {shape}")
    op = OProblem(spec)
    x = W.random_field(op.n, 25, positive=True).astype(np.float32)
    with rt.Problem(spec) as p:
        y = torch.empty(op.n, dtype=torch.float32, device="cuda:0")
        p.apply(dev(x, torch.float32), y, precision=prec)
        got = host(y)
    x64 = x.astype(np.float64)
    L = op.lam(x64.reshape(op.n_r, op.n_s), with_bc=False)
    ref = x64 - op.scatter(L).ravel()
    absprod = (op.albedo[None, :] * (np.abs(op.mhat) @ np.abs(L))).ravel()
    floor = 0.0
    if prec == "fp16":
        rowmax = np.abs(op.mhat).max(axis=1)
        floor = ((6e-8 * rowmax)[:, None] * np.abs(L).sum(axis=0)[None, :]).ravel()
    # 3u for the two operand roundings and accumulation; FP32 Lambda within
    # 2e-5 of its largest value (the FP32 Lambda test's criterion) per entry
    lam32 = 2e-5 * np.max(np.abs(L)) * (np.abs(op.mhat).sum(axis=1)[:, None] *
                                        op.albedo[None, :]).ravel()
    bound = 3.0 * U16[prec] * absprod + lam32 + floor + 2e-7 * np.abs(ref) + 1e-30
    err = np.abs(got - ref)
    assert np.all(err <= bound), float(np.max(err / bound))


@pytest.mark.parametrize("two_step", [1, 0])
@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "fp16", "bf16"])
@pytest.mark.parametrize("name", ["slab64", "box8"])
def test_mixed_refinement_per_precision(name, prec, two_step):
    """FP64 refinement around each low-precision inner operator, the inner
    Arnoldi steps in pairs (the default) and one at a time; the result is
    checked by the oracle-evaluated FP64 residual."""
    rt = _rt()
    spec = ALL[name]()
    say(f"mixed {prec} {name} two_step={two_step}")
    op = OProblem(spec)
    with rt.Problem(spec) as p:
        x = torch.empty(op.n, dtype=torch.float64, device="cuda:0")
        st = p.solve(x, rtol=1e-8, precision=prec, max_outer=30, two_step=two_step)
        s = host(x)
    res = op.residual_norm(s)
    say(f"   {prec} {name}: converged={st['converged']} outer={st['outer_iters']} "
        f"inner={st['iters']} oracle residual={res:.3e}")
    if st["converged"]:
        assert res <= 1e-8
    else:
        # a precision too coarse for this conditioning: reported, not hidden
        assert prec == "bf16", st


def test_gemm16_tuning_cache(monkeypatch, tmp_path):
    """RTSN_TUNE_CACHE: the first tuned shape is appended to the file; a new
    problem of the same shape takes the file's entry (the last one wins)
    instead of timing the candidates again."""
    rt = _rt()
    names = ["256x256 32x32x16 K64", "256x128 16x16x32 K32", "128x128 32x32x16 K32",
             "128x128 16x16x32 K64"]
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("RTSN_TUNE_CACHE", str(path))
    monkeypatch.delenv("RTSN_GEMM16_CFG", raising=False)
    spec = W.small_box(8, 4, 8, 5)
    with rt.Problem(spec) as p:
        x = torch.tensor(W.random_field(p.n, 91), dtype=torch.float32, device="cuda:0")
        y = torch.empty_like(x)
        p.apply(x, y, precision="fp16")
        torch.cuda.synchronize()
        tuned = p.gemm16_tile("fp16")
    lines = path.read_text().splitlines()
    assert len(lines) == 1
    key, cfg = lines[0].rsplit(" ", 1)
    assert names[int(cfg)] == tuned and key.split()[0].startswith("gfx")
    other = (int(cfg) + 1) % 4
    with open(path, "a") as f:
        f.write(f"{key} {other}\n")
    with rt.Problem(spec) as p:
        x = torch.tensor(W.random_field(p.n, 92), dtype=torch.float32, device="cuda:0")
        y = torch.empty_like(x)
        p.apply(x, y, precision="fp16")
        torch.cuda.synchronize()
        assert p.gemm16_tile("fp16") == names[other]
    assert len(path.read_text().splitlines()) == 2     # nothing timed, nothing appended


@pytest.mark.parametrize("prec", ["fp32", "fp16", "bf16x3"])
@pytest.mark.parametrize("name", ["slab64", "box8", "box_12x10x9"])
def test_bicgstab_mixed_refinement(name, prec):
    """BiCGStab as the inner solver of FP64 refinement (FP32 vectors, FP64
    dot products, the low-precision operator): the oracle-evaluated FP64
    residual meets 1e-8."""
    rt = _rt()
    spec = ALL[name]()
    say(f"bicgstab mixed {prec} {name}")
    op = OProblem(spec)
    with rt.Problem(spec) as p:
        x = torch.empty(op.n, dtype=torch.float64, device="cuda:0")
        st = p.solve(x, rtol=1e-8, precision=prec, krylov="bicgstab", max_outer=40,
                     restart=60)
        s = host(x)
    res = op.residual_norm(s)
    say(f"   outer {st['outer_iters']} inner {st['iters']} residual {res:.2e}")
    assert st["converged"] and res <= 1e-8
