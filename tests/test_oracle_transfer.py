"""Pins for the oracle's formal solvers against closed forms and symmetries."""
import decimal
import math

import numpy as np
import pytest

import workloads as W
from oracle import (exp_weights, sweep_slab, sweep_box, directions_3d,
                    double_gauss, Problem)


def _weights_decimal(d):
    """a(D), c(D) in 50-digit arithmetic from e^{-D} (closed forms; every
    operation in the 50-digit context)."""
    with decimal.localcontext(decimal.Context(prec=50)):
        D = decimal.Decimal(float(d))
        e = (-D).exp()
        q = (1 - e) / D
        return float(q - e), float(1 - q)


@pytest.mark.parametrize("d", [1e-12, 1e-8, 1e-4, 1e-2, 0.1, 0.3, 0.4999, 0.5,
                               0.5001, 0.9, 2.0, 10.0, 50.0, 800.0])
def test_exp_weights_against_high_precision(d):
    e, a, c = exp_weights(np.array([d]))
    a_ref, c_ref = _weights_decimal(d)
    assert abs(e[0] - math.exp(-d)) <= 2.3e-16 * math.exp(-d)
    assert abs(a[0] - a_ref) <= 2e-15 * abs(a_ref) + 1e-300
    assert abs(c[0] - c_ref) <= 2e-15 * abs(c_ref)


def _slab_rays(n_mu=8, fac=(1.0, 0.3, 0.01)):
    mu, _ = double_gauss(n_mu)
    mu_ray = np.repeat(mu, len(fac))
    fac_ray = np.tile(np.asarray(fac), n_mu)
    return mu_ray, fac_ray


def test_pure_absorption_slab():
    # constant S = B, nothing incident at the top: I = B (1 - e^{-tau/|mu|})
    # measured from the surface; from the bottom with I_in = B, I = B.
    depth = np.concatenate([[0.0], np.logspace(-3, 2, 40)])
    mu_ray, fac_ray = _slab_rays()
    B = 1.7
    s = np.full((len(mu_ray), len(depth)), B)
    out = sweep_slab(depth, mu_ray, fac_ray, s, 0.0, B)
    tau = depth[None, :] * (fac_ray / np.abs(mu_ray))[:, None]
    down = mu_ray < 0
    exact = B * (-np.expm1(-tau[down]))
    assert np.allclose(out[down], exact, rtol=1e-14, atol=1e-300)
    assert np.allclose(out[~down], B, rtol=1e-15)


def test_linear_source_is_exact():
    # S = alpha + beta t: linear in optical depth along every ray, so the
    # linear short-characteristics step reproduces the integral form exactly:
    # I(T) = I_e e^{-T} + s_e (1 - e^{-T}) + g (T - 1 + e^{-T}) with T the
    # optical path from the entry node, s_e the source there, g = dS/dT.
    depth = np.linspace(0.0, 30.0, 61)
    mu_ray, fac_ray = _slab_rays()
    alpha, beta, itop, ibot = 0.4, 0.05, 0.3, 2.0
    s = np.tile(alpha + beta * depth, (len(mu_ray), 1))
    out = sweep_slab(depth, mu_ray, fac_ray, s, itop, ibot)
    for k in range(len(mu_ray)):
        scale = fac_ray[k] / abs(mu_ray[k])
        if mu_ray[k] < 0:
            T = (depth - depth[0]) * scale
            ie, se, g = itop, alpha + beta * depth[0], beta / scale
        else:
            T = (depth[-1] - depth) * scale
            ie, se, g = ibot, alpha + beta * depth[-1], -beta / scale
        em = np.exp(-T)
        exact = ie * em + se * (1 - em) + g * (T - 1 + em)
        assert np.allclose(out[k], exact, rtol=1e-13, atol=1e-14)


def test_implicit_euler_closed_form_entries():
    # Assemble Lambda by unit sources and compare with the product formulas
    # f_ij, f_i (mu < 0) and h_ij, h_i (mu > 0) of the paper (Sec. 3.2).
    rng = np.random.default_rng(5)
    ns = 9
    depth = np.cumsum(rng.uniform(0.05, 2.0, ns))
    mu_ray = np.array([-0.4, 0.7])
    fac_ray = np.array([1.3, 0.6])
    for k in range(2):
        dtau = np.diff(depth) * fac_ray[k] / abs(mu_ray[k])       # dtau_1..dtau_{ns-1}
        lam = np.zeros((ns, ns))
        for j in range(ns):
            s = np.zeros((2, ns))
            s[k, j] = 1.0
            lam[:, j] = sweep_slab(depth, mu_ray, fac_ray, s, 0.0, 0.0,
                                   "implicit_euler")[k]
        inc = sweep_slab(depth, mu_ray, fac_ray, np.zeros((2, ns)), 1.0, 1.0,
                         "implicit_euler")[k]
        ref = np.zeros((ns, ns))
        ref_in = np.zeros(ns)
        # 1-based indices i, j as in the paper; dtau_l is dtau[l-1]
        if mu_ray[k] < 0:
            for i in range(1, ns + 1):
                ref_in[i - 1] = 1.0 / np.prod([1 + dtau[l - 1] for l in range(1, i)])
                for j in range(2, i + 1):
                    ref[i - 1, j - 1] = dtau[j - 2] / np.prod(
                        [1 + dtau[l - 2] for l in range(j, i + 1)])
        else:
            for i in range(1, ns + 1):
                ref_in[i - 1] = 1.0 / np.prod([1 + dtau[l - 1] for l in range(i, ns)])
                for j in range(i, ns):
                    ref[i - 1, j - 1] = dtau[j - 1] / np.prod(
                        [1 + dtau[l - 1] for l in range(i, j + 1)])
        assert np.allclose(lam, ref, rtol=1e-14, atol=0)
        assert np.allclose(inc, ref_in, rtol=1e-14, atol=0)


def _uniform_box_and_slab(nz=12, n=4, n_mu=4, n_az=8, n_nu=5):
    spec = W.small_box(n, n_mu, n_az, n_nu, nz=nz)
    kz = spec.k_line[:, 0, 0].copy()
    spec.k_line = np.broadcast_to(kz[:, None, None], spec.k_line.shape).copy()
    dz = 1.0 / (nz - 1)
    # slab depth from the top: trapezoid of k_L downward
    ktop = kz[::-1]
    depth = np.concatenate([[0.0], np.cumsum(0.5 * (ktop[1:] + ktop[:-1]) * dz)])
    slab = W.ProblemSpec(geom="slab", nz=nz, depth=depth, n_mu=n_mu, n_nu=n_nu,
                         x_max=spec.x_max, r=spec.r, eps=spec.eps, planck=spec.planck,
                         i_top=spec.i_top, i_bot=spec.i_bot)
    return spec, slab


def test_box_with_uniform_layers_equals_slab():
    spec, slab = _uniform_box_and_slab()
    pb, ps = Problem(spec), Problem(slab)
    n_nu, nz = spec.n_nu, spec.nz
    # a horizontally uniform, azimuth-independent source
    s_slab = W.random_field((ps.n_r, nz), 3, positive=True)
    s_box = np.zeros((spec.n_mu, spec.n_az, n_nu, nz, spec.ny, spec.nx))
    s_view = s_slab.reshape(spec.n_mu, n_nu, nz)[:, :, ::-1]      # slab top -> box top
    s_box[:] = s_view[:, None, :, :, None, None]
    ib = pb.lam(s_box.reshape(pb.n_r, pb.n_s), with_bc=True)
    i_slab = ps.lam(s_slab, with_bc=True).reshape(spec.n_mu, n_nu, nz)[:, :, ::-1]
    ib = ib.reshape(spec.n_mu, spec.n_az, n_nu, nz, spec.ny, spec.nx)
    expect = np.broadcast_to(i_slab[:, None, :, :, None, None], ib.shape)
    assert np.allclose(ib, expect, rtol=1e-12, atol=1e-14)
    # and the whole operator: azimuthal average of the 3D dipole is the 1D one
    ab = pb.apply(s_box).reshape(ib.shape)
    a_slab = ps.apply(s_slab).reshape(spec.n_mu, n_nu, nz)[:, :, ::-1]
    assert np.allclose(ab, np.broadcast_to(a_slab[:, None, :, :, None, None], ab.shape),
                       rtol=1e-12, atol=1e-14)


def test_box_translation_equivariance():
    spec = W.small_box(6, 4, 8, 3, nz=7)
    p = Problem(spec)
    s = W.random_field((p.n_r, spec.nz, spec.ny, spec.nx), 8)
    out = p.apply(s).reshape(s.shape)
    spec2 = W.small_box(6, 4, 8, 3, nz=7)
    spec2.k_line = np.roll(spec.k_line, (3, 5), axis=(1, 2))
    p2 = Problem(spec2)
    out2 = p2.apply(np.roll(s, (3, 5), axis=(2, 3))).reshape(s.shape)
    assert np.allclose(out2, np.roll(out, (3, 5), axis=(2, 3)), rtol=1e-13, atol=1e-14)


def test_box_quarter_turn_equivariance():
    # swapping x and y maps azimuth phi to pi/2 - phi: b -> (n_az/4 - 1 - b) mod n_az
    n_az = 8
    spec = W.small_box(6, 4, n_az, 3, nz=7)
    p = Problem(spec)
    shape = (spec.n_mu, n_az, spec.n_nu, spec.nz, spec.ny, spec.nx)
    s = W.random_field(shape, 9)
    out = p.apply(s.reshape(p.n_r, -1)).reshape(shape)
    perm = [(n_az // 4 - 1 - b) % n_az for b in range(n_az)]
    spec2 = W.small_box(6, 4, n_az, 3, nz=7)
    spec2.k_line = spec.k_line.transpose(0, 2, 1).copy()
    p2 = Problem(spec2)
    s2 = s[:, perm].transpose(0, 1, 2, 3, 5, 4)
    out2 = p2.apply(s2.reshape(p.n_r, -1)).reshape(shape)
    assert np.allclose(out2, out[:, perm].transpose(0, 1, 2, 3, 5, 4), rtol=1e-13, atol=1e-14)


def test_box_point_source_moves_downstream():
    # Radiation from a point source on plane z0 reaches plane z0+1 (mu > 0)
    # centred at the source displaced by +Omega_xy dz/mu (Sec. 2: transport
    # along Omega); bilinear interpolation preserves that first moment.
    n, nz = 16, 9
    k = np.full((nz, n, n), 3.0)
    om, _ = directions_3d(4, 8)
    o = [i for i in range(len(om)) if om[i, 2] > 0.5][1]         # steep up-going ray
    fac = np.array([1.0])
    s = np.zeros((len(om), nz, n, n))
    z0, y0, x0 = 1, 8, 8
    s[o, z0, y0, x0] = 1.0
    out = sweep_box(k, om, fac, s)[o, z0 + 1]
    dz = 1.0 / (nz - 1)
    shift = om[o, :2] * dz / om[o, 2] * n            # cells
    assert np.all(np.abs(shift) < 3)
    ys, xs = np.mgrid[0:n, 0:n]
    wsum = out.sum()
    cx = (out * xs).sum() / wsum - x0
    cy = (out * ys).sum() / wsum - y0
    assert abs(cx - shift[0]) < 1e-12 and abs(cy - shift[1]) < 1e-12
