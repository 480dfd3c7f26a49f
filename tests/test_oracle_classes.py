"""Pins for per-point scattering classes in the oracle (Sec. 3.3: the block
Psi_[i] may differ from point to point; here points fall into classes, each
with its own kernel).  Checked against: the one-kernel problem, the
normalisation of every class's redistribution (thermal consistency, Sec. 2),
thermal equilibrium as an exact solution, box = slab for horizontally
uniform layers whose class depends on height, and a dense block-diagonal
assembly of the scattering operator."""
import numpy as np
import pytest

import workloads as W
from oracle import Problem


def test_one_class_is_the_plain_problem():
    for make in (W.slab64, lambda: W.small_box(5, 4, 8, 5, nz=6)):
        s1 = make()
        s2 = make()
        s2.point_class = np.zeros(s2.n_s, int)
        s2.class_coh_frac = [s2.coh_frac]
        p1, p2 = Problem(s1), Problem(s2)
        x = W.random_field(p1.n, 1)
        assert np.array_equal(p1.apply(x), p2.apply(x))
        assert np.array_equal(p1.rhs(), p2.rhs())


@pytest.mark.parametrize("geom", ["slab", "box"])
def test_every_class_is_normalised(geom):
    spec = W.slab64() if geom == "slab" else W.small_box(4, 4, 8, 7, nz=5)
    fracs = [0.0, 0.3, 1.0]
    spec.point_class = np.arange(spec.n_s) % 3
    spec.class_coh_frac = fracs
    p = Problem(spec)
    target = p.phi_ray / p.fac_ray
    for m in p.mhat_classes:
        assert np.allclose(m.sum(axis=1), target, rtol=1e-13, atol=0)
    # the classes really differ
    assert np.max(np.abs(p.mhat_classes[0] - p.mhat_classes[2])) > 1e-3 * p.mhat.max()


def test_thermal_equilibrium_with_classes():
    spec = W.small_box(5, 4, 8, 5, nz=7)
    spec.eps, spec.i_top, spec.i_bot, spec.planck = 0.01, 2.5, 2.5, 2.5
    spec.point_class = (np.arange(spec.n_s) * 7) % 4
    spec.class_coh_frac = [0.0, 0.2, 0.7, 1.0]
    p = Problem(spec)
    s = np.full((p.n_r, p.n_s), 2.5)
    assert np.max(np.abs(p.rhs() - p.apply(s))) < 1e-13


def test_box_with_layer_classes_equals_slab():
    from test_oracle_transfer import _uniform_box_and_slab
    spec, slab = _uniform_box_and_slab()
    fracs = [0.1, 0.5, 0.95]
    zc = np.arange(spec.nz) % 3                      # class of box plane z (0 = bottom)
    spec.point_class = np.repeat(zc, spec.ny * spec.nx)
    spec.class_coh_frac = fracs
    slab.point_class = zc[::-1].copy()              # slab index 0 = top
    slab.class_coh_frac = fracs
    pb, ps = Problem(spec), Problem(slab)
    n_nu, nz = spec.n_nu, spec.nz
    s_slab = W.random_field((ps.n_r, nz), 4, positive=True)
    s_box = np.zeros((spec.n_mu, spec.n_az, n_nu, nz, spec.ny, spec.nx))
    s_box[:] = s_slab.reshape(spec.n_mu, n_nu, nz)[:, :, ::-1][:, None, :, :, None, None]
    ab = pb.apply(s_box.reshape(pb.n_r, pb.n_s)).reshape(s_box.shape)
    a_slab = ps.apply(s_slab).reshape(spec.n_mu, n_nu, nz)[:, :, ::-1]
    assert np.allclose(ab, np.broadcast_to(a_slab[:, None, :, :, None, None], ab.shape),
                       rtol=1e-12, atol=1e-14)
    # and the layered problem differs from the one-kernel one
    spec.point_class = None
    a1 = Problem(spec).apply(s_box.reshape(pb.n_r, pb.n_s)).reshape(s_box.shape)
    assert np.max(np.abs(a1 - ab)) > 1e-6


def test_explicit_class_kernels_match_block_diagonal_assembly():
    spec = W.slab64()
    spec.nz, spec.n_mu, spec.n_nu = 6, 4, 3
    spec.depth = W.log_depth_grid(6, 1e-2, 1e2)
    spec.kernel = "explicit"
    n_r = 12
    spec.kernel_matrix = W.random_symmetric_kernel(n_r, 1)
    spec.class_kernels = np.stack([W.random_symmetric_kernel(n_r, s) for s in (2, 3)])
    spec.point_class = np.array([0, 1, 1, 0, 1, 0])
    spec.eps = np.linspace(0.01, 0.3, 6)
    p = Problem(spec)
    n_s = spec.n_s
    sig = np.zeros((p.n, p.n))
    for i in range(n_s):
        m = p.mhat_classes[spec.point_class[i]]
        rows = np.arange(n_r) * n_s + i
        sig[np.ix_(rows, rows)] = p.albedo[i] * m
    I = W.random_field((n_r, n_s), 5)
    ref = sig @ I.ravel()
    assert np.max(np.abs(p.scatter(I).ravel() - ref)) <= 1e-14 * np.max(np.abs(ref))
    # changing one point's class changes only that point's column
    spec2 = W.slab64()
    spec2.__dict__.update({k: getattr(spec, k) for k in spec.__dict__})
    spec2.point_class = spec.point_class.copy()
    spec2.point_class[2] = 0
    d = Problem(spec2).scatter(I) - p.scatter(I)
    assert np.all(d[:, [0, 1, 3, 4, 5]] == 0) and np.max(np.abs(d[:, 2])) > 0
