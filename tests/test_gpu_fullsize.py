"""Full-size checks of the configurations the benchmark times, on the GPU,
through properties that hold at any size (the oracle cannot sweep 1.6e9
unknowns in a test) and through the oracle on sampled problems.

* 64^3 box (6144 rays x 262144 points), Sigma: with L = 1 every output is the
  closed form (1 - eps) phi_nu / (phi_nu + r) - the kernel's normalisation
  (Sec. 2: the dipole phase function and the redistribution function are
  normalised, so the scattering source of a uniform radiation field equals
  the fraction phi_nu / (phi_nu + r) of it that the line absorbs).
* 64^3 box, Lambda: in a horizontally uniform (stratified) atmosphere with
  s = 1 and no incoming radiation, every plane is uniform and the formal
  solution is I = 1 - exp(-tau), tau the trapezoid optical depth along the
  ray from its entry plane (integral form of the transfer equation, Sec. 2,
  for a constant source; a + c = 1 - e in each short-characteristics step).
* 64^3 box, whole 16-bit operator (fp16 / bf16 / bf16x3 Sigma on the
  16-bit Lambda output, whose fp16 scale is capped at 2^14 at this size): in
  the stratified atmosphere with x = 1, sampled points checked against the
  closed-form Lambda and the oracle's Mhat in FP64.
* 32^3 box (the benchmark workload) solved in FP64, in mixed precision with
  an fp16 Sigma and with an fp16 Krylov basis, and preconditioned (FP64; FP32
  operators with factored scattering on an fp16 basis): the oracle's FP64
  residual of each solution meets 1e-8.
* batch512 (512 slabs of the batch recipe) in one engine: every 32nd slab's
  solution checked against the oracle's FP64 residual.
"""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import Problem as OProblem
from oracle.quadrature import directions_3d, frequency_grid

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

U16 = {"bf16": 2.0 ** -8, "fp16": 2.0 ** -11, "bf16x3": 2.0 ** -15}


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _rt():
    from paper_2602_21958_amd import rt
    return rt


def test_box64_sigma_full_size_uniform_field():
    rt = _rt()
    spec = W.box64()
    say("box64 Sigma, L = 1")
    _, _, phi = frequency_grid(spec.n_nu, spec.x_max)
    n_om = spec.n_mu * spec.n_az
    expect = np.tile((1.0 - spec.eps) * phi / (phi + spec.r), n_om)   # per ray
    with rt.Problem(spec) as p:
        n_r, n_s = p.n_r, p.n_s
        assert n_r == len(expect)
        e = torch.tensor(expect, device="cuda:0")
        # bounds: FP64, rounding of 6144-term sums of positive terms; FP32
        # accumulation (about sqrt(K) u of a positive sum, with margin); the
        # 16-bit modes add the rounding of Mhat (relative u16 per entry, all
        # entries positive)
        for prec, tol in (("fp64", 1e-12), ("fp32", 1e-4), ("fp16", 2 * U16["fp16"] + 1e-4),
                          ("bf16x3", 2 * U16["bf16x3"] + 1e-4), ("bf16", 2 * U16["bf16"] + 1e-4)):
            dt = torch.float64 if prec == "fp64" else torch.float32
            L = torch.ones(n_r * n_s, dtype=dt, device="cuda:0")
            y = torch.empty_like(L)
            p.apply_sigma(L, None, y, precision=prec)
            torch.cuda.synchronize()
            del L
            yv = y.view(n_r, n_s)
            err = 0.0
            for k0 in range(0, n_r, 512):
                blk = yv[k0:k0 + 512].double()
                ek = e[k0:k0 + 512, None]
                err = max(err, ((blk - ek).abs() / ek).max().item())
                del blk
            say(f"   {prec}: max relative error {err:.3e} (bound {tol:.1e})")
            del y
            torch.cuda.empty_cache()
            assert err <= tol, (prec, err)


def _stratified_box64():
    spec = W.box64()
    spec.k_line = W.box_opacity_field(64, 64, 64, 0, sigma=0.0)
    return spec


def _closed_form_intensity(spec, rays):
    """I(k, z) = 1 - exp(-tau_k(z)) for s = 1, zero incoming radiation."""
    omega, _ = directions_3d(spec.n_mu, spec.n_az)
    _, _, phi = frequency_grid(spec.n_nu, spec.x_max)
    kz = spec.k_line[:, 0, 0]                       # uniform planes
    nz = spec.nz
    half = 0.5 * (kz[1:] + kz[:-1]) / (nz - 1)      # trapezoid k dz per interval
    out = np.zeros((len(rays), nz))
    for r, k in enumerate(rays):
        o, nu = divmod(k, spec.n_nu)
        g = (phi[nu] + spec.r) / abs(omega[o, 2])
        if omega[o, 2] > 0:     # enters at the bottom plane z = 0
            tau = np.concatenate(([0.0], np.cumsum(half))) * g
        else:                   # enters at the top plane
            tau = np.concatenate((np.cumsum(half[::-1])[::-1], [0.0])) * g
        out[r] = -np.expm1(-tau)
    return out


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-13), ("fp32", 5e-6)])
def test_box64_lambda_full_size_stratified_closed_form(prec, tol):
    rt = _rt()
    spec = _stratified_box64()
    assert np.ptp(spec.k_line[10]) == 0.0
    say(f"box64 Lambda {prec}, stratified, s = 1")
    dt = torch.float64 if prec == "fp64" else torch.float32
    with rt.Problem(spec) as p:
        n_r, n_s = p.n_r, p.n_s
        s = torch.ones(n_r * n_s, dtype=dt, device="cuda:0")
        out = torch.empty_like(s)
        p.apply_lambda(s, out, with_bc=False, precision=prec)
        torch.cuda.synchronize()
        del s
        rays = list(range(0, n_r, 97)) + [n_r - 1]
        got = out.view(n_r, spec.nz, spec.ny * spec.nx)[rays].double().cpu().numpy()
    ref = _closed_form_intensity(spec, rays)
    err = np.max(np.abs(got - ref[:, :, None]))
    say(f"   max abs error {err:.3e} over {len(rays)} rays x {n_s} points (bound {tol:.0e})")
    assert err <= tol


@pytest.mark.parametrize("prec", ["fp16", "bf16", "bf16x3"])
def test_box64_16bit_operator_full_size_sampled_points(prec):
    rt = _rt()
    spec = _stratified_box64()
    say(f"box64 {prec} operator, stratified, x = 1")
    # the oracle's Mhat for these angle and frequency grids (it does not
    # depend on the spatial grid): a 1 x 1 x 2 box with the same quadratures
    tiny = W.small_box(1, spec.n_mu, spec.n_az, spec.n_nu, nz=2, ny=1)
    tiny.x_max, tiny.r, tiny.eps = spec.x_max, spec.r, spec.eps
    op = OProblem(tiny)
    with rt.Problem(spec) as p:
        n_r, n_s = p.n_r, p.n_s
        assert p.n > 6.7e7        # fp16 Lambda output scale at its 2^14 cap
        x = torch.ones(n_r * n_s, dtype=torch.float32, device="cuda:0")
        y = torch.empty_like(x)
        p.apply(x, y, precision=prec)
        torch.cuda.synchronize()
        del x
        nxy = spec.nx * spec.ny
        # points on every plane, at varied horizontal positions
        pts = np.array([z * nxy + (z * 977 + 13) % nxy for z in range(spec.nz)])
        got = y.view(n_r, n_s)[:, torch.tensor(pts, device="cuda:0")].double().cpu().numpy()
        del y
        torch.cuda.empty_cache()
    L = _closed_form_intensity(spec, list(range(n_r)))[:, pts // nxy]   # (n_r, points)
    ref = 1.0 - (1.0 - spec.eps) * (op.mhat @ L)
    absprod = (1.0 - spec.eps) * (np.abs(op.mhat) @ np.abs(L))
    floor = 0.0
    if prec == "fp16":
        rowmax = np.abs(op.mhat).max(axis=1)
        floor = (6e-8 * rowmax)[:, None] * np.abs(L).sum(axis=0)[None, :]
    # 3u for the operand roundings and accumulation, FP32 Lambda (5e-6 of
    # its unit-bounded values, the FP32 closed-form criterion above) through
    # the row sums of Mhat, FP32 rounding of the output
    lam32 = 5e-6 * (1.0 - spec.eps) * np.abs(op.mhat).sum(axis=1)[:, None]
    bound = 3.0 * U16[prec] * absprod + lam32 + floor + 2e-7 * np.abs(ref) + 1e-30
    err = np.abs(got - ref)
    say(f"   {len(pts)} points x {n_r} rays: max error / bound {np.max(err / bound):.3f}, "
        f"max abs error {err.max():.2e}")
    assert np.all(err <= bound)


_BOX32_ORACLE = {}


def _box32_oracle():
    if "op" not in _BOX32_ORACLE:
        op = OProblem(W.box32())
        _BOX32_ORACLE["op"] = op
        _BOX32_ORACLE["b"] = op.rhs()
    return _BOX32_ORACLE["op"], _BOX32_ORACLE["b"]


@pytest.mark.parametrize("prec,basis16,pre", [("fp64", 0, ""), ("fp16", 0, ""), ("fp16", 1, ""),
                                              ("fp64", 0, "local"), ("fp32", 1, "local")])
def test_box32_full_size_solve_oracle_residual(prec, basis16, pre):
    """Full-size box32 solves, the oracle's FP64 residual of the solution:
    FP64, fp16 refinement on FP32 / fp16 bases, and preconditioned (FP64 with
    the dense scattering; FP32 operators with factored scattering on an fp16
    basis, the fastest mixed combination)."""
    rt = _rt()
    say(f"box32 full-size solve {prec} basis_fp16={basis16} precond={pre or 'none'}")
    op, b = _box32_oracle()
    with rt.Problem(W.box32()) as p:
        if pre and prec == "fp32":
            p.set_sigma("factored")
        x = torch.empty(p.n, dtype=torch.float64, device="cuda:0")
        st = p.solve(x, rtol=1e-8, restart=30, precision=prec, basis_fp16=basis16,
                     precond=pre or "none")
        s = x.cpu().numpy()
        del x
    res = op.residual_norm(s, b)
    say(f"   iters {st['iters']}, outer {st['outer_iters']}, library residual "
        f"{st['relres']:.3e}, oracle residual {res:.3e}")
    assert st["converged"], st
    assert res <= 1e-8


def test_batch512_full_size_sampled_oracle_residuals():
    rt = _rt()
    specs = W.batch_slabs(512)
    say("batch512 in one engine (bf16x3)")
    probs = [rt.Problem(s) for s in specs]
    xs = [torch.empty(p.n, dtype=torch.float64, device="cuda:0") for p in probs]
    eng = rt.Batch(precision="bf16x3", hbm_budget=64 << 30, max_slots=512)
    try:
        tk = [eng.submit(p, x, restart=30, rtol=1e-8, max_iters=4000, max_outer=200)
              for p, x in zip(probs, xs)]
        while eng.step() > 0:
            pass
        stats = [eng.poll(t) for t in tk]
    finally:
        eng.close()
    assert all(st["converged"] for st in stats)
    for i in range(0, 512, 32):
        s = xs[i].cpu().numpy()
        res = OProblem(specs[i]).residual_norm(s)
        say(f"   slab {i}: n = {probs[i].n}, iters {stats[i]['iters']}, oracle residual {res:.2e}")
        assert res <= 1e-8
    for p in probs:
        p.close()
