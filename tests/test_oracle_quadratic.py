"""Pins for the oracle's quadratic short-characteristics step: its moments
against 120-digit arithmetic, its weights against the exact integral of any
parabola, exactness of the slab sweep for sources quadratic in optical depth,
and third-order convergence on a smooth source (second order for the linear
step), from the integral form of the transfer equation (Sec. 2)."""
import decimal
import math

import numpy as np
import pytest

from oracle import double_gauss, sweep_slab
from oracle.transfer import exp_moments, quad_weights

CTX = decimal.Context(prec=120)   # the closed forms cancel ~3 log10(1/D) digits


def _dec(x):
    return CTX.create_decimal_from_float(float(x))


def _moments_decimal(d):
    with decimal.localcontext(CTX):
        D = _dec(d)
        e = (-D).exp()
        return (float(1 - e), float(1 - (1 + D) * e), float(2 - (2 + 2 * D + D * D) * e))


@pytest.mark.parametrize("d", [1e-10, 1e-6, 1e-3, 0.1, 0.4999, 0.5, 0.5001, 1.0, 3.0, 20.0,
                               700.0])
def test_exp_moments_against_high_precision(d):
    got = exp_moments(np.array([d]))
    for k, ref in enumerate(_moments_decimal(d)):
        assert abs(got[k][0] - ref) <= 4e-15 * abs(ref), (k, got[k][0], ref)


def _parabola_integral_decimal(c, du):
    """int_0^du (c0 + c1 t + c2 t^2) e^{-t} dt in 120 digits."""
    with decimal.localcontext(CTX):
        D = _dec(du)
        e = (-D).exp()
        w0 = 1 - e
        w1 = 1 - (1 + D) * e
        w2 = 2 - (2 + 2 * D + D * D) * e
        return float(_dec(c[0]) * w0 + _dec(c[1]) * w1 + _dec(c[2]) * w2)


def test_quad_weights_integrate_every_parabola():
    rng = np.random.default_rng(2)
    for _ in range(300):
        du = 10.0 ** rng.uniform(-5, 1.5)
        dd = du * 10.0 ** rng.uniform(-0.7, 0.7)     # neighbouring intervals of a smooth grid
        c = rng.normal(size=3)
        e, pu, p0, pd = quad_weights(np.array([du]), np.array([dd]))
        f = lambda t: c[0] + c[1] * t + c[2] * t * t
        got = e[0] * 0.0 + pu[0] * f(du) + p0[0] * f(0.0) + pd[0] * f(-dd)
        ref = _parabola_integral_decimal(c, du)
        scale = (abs(c[0]) + abs(c[1]) * (du + dd) + abs(c[2]) * (du + dd) ** 2) * \
            min(1.0, du)
        assert abs(got - ref) <= 1e-12 * scale, (du, dd, got, ref)
        assert abs(e[0] - math.exp(-du)) <= 2.3e-16 * math.exp(-du)


def test_quad_weights_constant_and_limits():
    du = np.logspace(-6, 2, 50)
    dd = 1.3 * du
    e, pu, p0, pd = quad_weights(du, dd)
    # a constant source integrates to 1 - e^{-D_u}
    assert np.allclose(pu + p0 + pd, -np.expm1(-du), rtol=1e-13, atol=0)
    # an optically thick upwind interval (w0 = w1 = 1, w2 = 2): psi_u =
    # (2 + D_d) / (D_u (D_u + D_d)), psi_d = (2 - D_u) / (D_d (D_u + D_d)),
    # psi_0 = 1 - psi_u - psi_d -> 1
    du, dd = 200.0, 300.0
    e, pu, p0, pd = quad_weights(np.array([du]), np.array([dd]))
    assert abs(pu[0] - (2 + dd) / (du * (du + dd))) < 1e-15
    assert abs(pd[0] - (2 - du) / (dd * (du + dd))) < 1e-15
    assert abs(p0[0] + pu[0] + pd[0] - 1.0) < 1e-15


def _rays():
    mu, _ = double_gauss(8)
    fac = (1.0, 0.3, 0.01)
    return np.repeat(mu, len(fac)), np.tile(np.asarray(fac), len(mu))


def test_quadratic_source_is_exact_in_the_slab():
    # S = a + b t + c t^2 is quadratic in optical depth along every ray; the
    # quadratic step reproduces the integral form exactly at every point but
    # the last of each ray (which takes the linear step):
    # I(T) = I_e e^{-T} + S(T) w0(T) - S'(T) w1(T) + (S''/2) w2(T) - e^{-T}...
    # written here as the exact integral of the parabola in T from the entry
    depth = np.linspace(0.0, 12.0, 49) ** 1.3
    mu_ray, fac_ray = _rays()
    a, b, c, itop, ibot = 0.4, 0.05, 0.002, 0.3, 2.0
    s = np.tile(a + b * depth + c * depth ** 2, (len(mu_ray), 1))
    out = sweep_slab(depth, mu_ray, fac_ray, s, itop, ibot, scheme="quadratic_sc")
    for k in range(len(mu_ray)):
        g = fac_ray[k] / abs(mu_ray[k])           # dT/dt
        if mu_ray[k] < 0:
            T = (depth - depth[0]) * g
            ie, t_of = itop, lambda T: depth[0] + T / g
            idx = np.arange(len(depth) - 1)       # all but the last point
        else:
            T = (depth[-1] - depth) * g
            ie, t_of = ibot, lambda T: depth[-1] - T / g
            idx = np.arange(1, len(depth))
        for i in idx:
            # exact: I_e e^{-T} + int_0^T S(t(T - u)) e^{-u} du, S a parabola in u
            Ti = T[i]
            ti = t_of(Ti)
            # S at distance u back along the ray: t = ti -+ u / g
            sg = -1.0 if mu_ray[k] < 0 else 1.0
            c0 = a + b * ti + c * ti ** 2
            c1 = sg * (b + 2 * c * ti) / g
            c2 = c / g ** 2
            w0, w1, w2 = (float(v[0]) for v in exp_moments(np.array([Ti])))
            exact = ie * math.exp(-Ti) + c0 * w0 + c1 * w1 + c2 * w2
            assert abs(out[k, i] - exact) <= 1e-12 * max(1.0, abs(exact)), (k, i)


def _sine_errors(scheme, n):
    # S(tau) = 2 + sin(tau / 3) on a single ray mu = -1, fac = 1, tau in [0, 20]
    depth = np.linspace(0.0, 20.0, n)
    s = 2.0 + np.sin(depth / 3.0)
    out = sweep_slab(depth, np.array([-1.0]), np.array([1.0]), s[None, :], 0.0, 0.0,
                     scheme=scheme)[0]
    w = 1.0 / 3.0
    tau = depth
    exact = 2.0 * (1 - np.exp(-tau)) + (np.sin(w * tau) - w * np.cos(w * tau)
                                        + w * np.exp(-tau)) / (1 + w * w)
    return np.max(np.abs(out[:-1] - exact[:-1]))


def test_quadratic_step_converges_at_third_order():
    e_q = [_sine_errors("quadratic_sc", n) for n in (21, 41, 81)]
    e_l = [_sine_errors("linear_sc", n) for n in (21, 41, 81)]
    oq = [math.log2(e_q[i] / e_q[i + 1]) for i in range(2)]
    ol = [math.log2(e_l[i] / e_l[i + 1]) for i in range(2)]
    assert all(o > 2.7 for o in oq), oq
    assert all(1.7 < o < 2.3 for o in ol), ol
    assert e_q[-1] < 0.1 * e_l[-1]


# ------------------------------------------------------------------ box
def test_quadratic_box_with_uniform_layers_equals_slab():
    # the box's quadratic sweep of a horizontally uniform problem is the
    # slab's quadratic sweep on the trapezoid-cumulated depths (both ends of
    # every ray, including the linear last step)
    import workloads as W
    from oracle import Problem
    from test_oracle_transfer import _uniform_box_and_slab
    spec, slab = _uniform_box_and_slab()
    spec.formal = slab.formal = "quadratic_sc"
    pb, ps = Problem(spec), Problem(slab)
    n_nu, nz = spec.n_nu, spec.nz
    s_slab = W.random_field((ps.n_r, nz), 3, positive=True)
    s_box = np.zeros((spec.n_mu, spec.n_az, n_nu, nz, spec.ny, spec.nx))
    s_box[:] = s_slab.reshape(spec.n_mu, n_nu, nz)[:, :, ::-1][:, None, :, :, None, None]
    ib = pb.lam(s_box.reshape(pb.n_r, pb.n_s), with_bc=True)
    i_slab = ps.lam(s_slab, with_bc=True).reshape(spec.n_mu, n_nu, nz)[:, :, ::-1]
    ib = ib.reshape(spec.n_mu, spec.n_az, n_nu, nz, spec.ny, spec.nx)
    assert np.allclose(ib, np.broadcast_to(i_slab[:, None, :, :, None, None], ib.shape),
                       rtol=1e-12, atol=1e-14)
    # and it differs from the linear sweep (the downwind values enter)
    spec.formal = "linear_sc"
    il = Problem(spec).lam(s_box.reshape(pb.n_r, pb.n_s), with_bc=True)
    assert np.max(np.abs(il.reshape(ib.shape) - ib)) > 1e-4


def test_quadratic_box_translation_and_quarter_turn():
    import workloads as W
    from oracle import Problem
    n_az = 8
    spec = W.small_box(6, 4, n_az, 3, nz=7)
    spec.formal = "quadratic_sc"
    p = Problem(spec)
    shape = (spec.n_mu, n_az, spec.n_nu, spec.nz, spec.ny, spec.nx)
    s = W.random_field(shape, 9)
    out = p.lam(s.reshape(p.n_r, -1), with_bc=True).reshape(shape)
    spec2 = W.small_box(6, 4, n_az, 3, nz=7)
    spec2.formal = "quadratic_sc"
    spec2.k_line = np.roll(spec.k_line, (3, 5), axis=(1, 2))
    out2 = Problem(spec2).lam(np.roll(s, (3, 5), axis=(4, 5)).reshape(p.n_r, -1),
                              with_bc=True).reshape(shape)
    assert np.allclose(out2, np.roll(out, (3, 5), axis=(4, 5)), rtol=1e-13, atol=1e-14)
    perm = [(n_az // 4 - 1 - b) % n_az for b in range(n_az)]
    spec3 = W.small_box(6, 4, n_az, 3, nz=7)
    spec3.formal = "quadratic_sc"
    spec3.k_line = spec.k_line.transpose(0, 2, 1).copy()
    s3 = s[:, perm].transpose(0, 1, 2, 3, 5, 4)
    out3 = Problem(spec3).lam(s3.reshape(p.n_r, -1), with_bc=True).reshape(shape)
    assert np.allclose(out3, out[:, perm].transpose(0, 1, 2, 3, 5, 4), rtol=1e-13, atol=1e-14)


def test_quadratic_box_reads_the_downwind_point():
    # A point source on plane z0 + 1 reaches plane z0 of an up-going ray only
    # through the downwind term: the node whose downwind point is the source
    # lies upstream, at the source displaced by -Omega_xy dz/mu (bilinear
    # interpolation keeps that first moment); the linear sweep gives zero.
    from oracle import directions_3d
    from oracle.transfer import sweep_box
    n, nz = 16, 9
    k = np.full((nz, n, n), 3.0)
    om, _ = directions_3d(4, 8)
    o = [i for i in range(len(om)) if om[i, 2] > 0.5][1]
    fac = np.array([1.0])
    s = np.zeros((len(om), nz, n, n))
    z0, y0, x0 = 4, 8, 8
    s[o, z0 + 1, y0, x0] = 1.0
    lin = sweep_box(k, om, fac, s)[o, z0]
    assert np.all(lin == 0)
    out = sweep_box(k, om, fac, s, scheme="quadratic_sc")[o, z0]
    dz = 1.0 / (nz - 1)
    shift = om[o, :2] * dz / om[o, 2] * n
    ys, xs = np.mgrid[0:n, 0:n]
    wsum = out.sum()
    assert wsum < 0          # the downwind weight is negative
    cx = (out * xs).sum() / wsum - x0
    cy = (out * ys).sum() / wsum - y0
    assert abs(cx + shift[0]) < 1e-12 and abs(cy + shift[1]) < 1e-12
