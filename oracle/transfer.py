"""Formal solvers Lambda (oracle; test infrastructure only).

Paper Sec. 3.2: along each ray r = (mu, nu) the transfer equation
dI/dtau = I - S is integrated from the incoming boundary; different rays are
independent, so Lambda is block diagonal in ray order (eq. lambda_block).

Three schemes:

* implicit Euler, exactly eqs. ie_1 / ie_2: for mu < 0 (entering at the
  surface, index 0) I_{i+1} = (I_i + dtau_i S_{i+1}) / (1 + dtau_i); for mu > 0
  (entering at the bottom) I_{i-1} = (I_i + dtau_{i-1} S_{i-1}) / (1 + dtau_{i-1}).
* linear short characteristics: the integral form of the transfer equation
  (Sec. 2, eq. rt_integral) over one interval of optical length D with S linear
  between the upwind value s_u and the local value s_0 gives
  I_0 = e^{-D} I_u + a(D) s_u + c(D) s_0,
  a(D) = (1 - e^{-D})/D - e^{-D},  c(D) = 1 - (1 - e^{-D})/D.
  For D < 0.5 a and c are summed from their Taylor series
  a = sum_{n>=1} (-1)^{n+1} n D^n/(n+1)!,  c = sum_{n>=1} (-1)^{n+1} D^n/(n+1)!
  (25 terms), avoiding the cancellation of the closed forms.
* quadratic short characteristics: the same integral with S the parabola
  through the upwind, local and downwind values.  With t the optical depth
  measured back from the local point (t = D_u at the upwind point, -D_d at
  the downwind one) and the moments w_k = int_0^{D_u} t^k e^{-t} dt,
  integrating each Lagrange basis polynomial against e^{-t} gives
  I_0 = e^{-D_u} I_u + psi_u s_u + psi_0 s_0 + psi_d s_d,
  psi_u = (w2 + D_d w1) / (D_u (D_u + D_d)),
  psi_0 = (w2 - (D_u - D_d) w1 - D_u D_d w0) / (-D_u D_d),
  psi_d = (w2 - D_u w1) / (D_d (D_u + D_d)).
  The last point of a ray has no downwind point and takes the linear step.

Optical depths: slab, dtau_i(mu, nu) = (t_{i+1} - t_i)(phi_nu + r)/|mu| with t
the frequency-integrated line optical depth (Sec. 5: tau = phi t / mu, with |mu|
since tau increases along the ray for both hemispheres).  Box: plane-to-plane
upwind interpolation (our short-characteristics counterpart of the ray
partition of Sec. 3.4): for ordinate Omega the upwind point of node
(x_i, y_j, z_k) lies on the neighbouring plane upstream, displaced horizontally
by -Omega_xy dz/|mu|; I, S and the opacity there are bilinear interpolations
with periodic wrap, and D = (k_u + k_0)/2 (phi_nu + r) dz/|mu|.

Pins: pure-absorption and linear-source closed forms, the closed-form
implicit-Euler entries f_ij, f_i, h_ij, h_i (eqs. ie_mono3-4), box = slab for a
horizontally uniform box, translation and 90-degree rotation equivariance,
downstream propagation of a point source (tests/test_oracle_transfer.py).
"""
from __future__ import annotations

import math

import numpy as np

_SERIES_BELOW = 0.5
_SERIES_TERMS = 25


def exp_weights(d: np.ndarray):
    """(e^{-D}, a(D), c(D)) of the linear short-characteristics step."""
    d = np.asarray(d, dtype=np.float64)
    e = np.exp(-d)
    small = d < _SERIES_BELOW
    ds = np.where(small, d, 0.0)
    a_ser = np.zeros_like(d)
    c_ser = np.zeros_like(d)
    power = np.ones_like(d)
    fact = 1.0
    for n in range(1, _SERIES_TERMS + 1):
        power = power * ds
        fact = fact * (n + 1)          # (n+1)!
        sign = 1.0 if n % 2 == 1 else -1.0
        a_ser += sign * n * power / fact
        c_ser += sign * power / fact
    dl = np.where(small, 1.0, d)
    one_minus_e_over_d = -np.expm1(-dl) / dl
    a = np.where(small, a_ser, one_minus_e_over_d - np.exp(-dl))
    c = np.where(small, c_ser, 1.0 - one_minus_e_over_d)
    return e, a, c


def exp_moments(d: np.ndarray):
    """(w0, w1, w2), w_k(D) = int_0^D t^k e^{-t} dt.

    Closed forms from integration by parts, w_k = k w_{k-1} - D^k e^{-D}
    (w0 = 1 - e^{-D}); for D < 0.5 the Taylor series of e^{-t} integrated
    term by term, w_k = sum_m (-1)^m D^{k+m+1} / (m! (k+m+1)) (30 terms)."""
    d = np.asarray(d, dtype=np.float64)
    small = d < _SERIES_BELOW
    ds = np.where(small, d, 0.0)
    ser = [np.zeros_like(d) for _ in range(3)]
    for k in range(3):
        fact = 1.0
        for m in range(30):
            if m:
                fact *= m
            sign = 1.0 if m % 2 == 0 else -1.0
            ser[k] = ser[k] + sign * ds ** (k + m + 1) / (fact * (k + m + 1))
    dl = np.where(small, 1.0, d)
    e = np.exp(-dl)
    w0 = -np.expm1(-dl)
    w1 = w0 - dl * e
    w2 = 2.0 * w1 - dl * dl * e
    return (np.where(small, ser[0], w0), np.where(small, ser[1], w1),
            np.where(small, ser[2], w2))


def quad_weights(du: np.ndarray, dd: np.ndarray):
    """(e^{-D_u}, psi_u, psi_0, psi_d) of the quadratic short-characteristics
    step with upwind interval D_u and downwind interval D_d."""
    du = np.asarray(du, dtype=np.float64)
    dd = np.asarray(dd, dtype=np.float64)
    w0, w1, w2 = exp_moments(du)
    psi_u = (w2 + dd * w1) / (du * (du + dd))
    psi_0 = (w2 - (du - dd) * w1 - du * dd * w0) / (-du * dd)
    psi_d = (w2 - du * w1) / (dd * (du + dd))
    return np.exp(-du), psi_u, psi_0, psi_d


def sweep_slab(depth, mu_ray, fac_ray, s, i_top=0.0, i_bot=0.0,
               scheme: str = "linear_sc"):
    """Formal solution on a slab for every ray.

    depth   (N_z,) frequency-integrated optical depth t, top (0) to bottom
    mu_ray  (N_r,) direction cosine of each ray (mu < 0 enters at the top)
    fac_ray (N_r,) phi_nu + r of each ray
    s       (N_r, N_z) source function
    i_top, i_bot  incoming intensities (scalar or (N_r,))
    returns I (N_r, N_z)
    """
    depth = np.asarray(depth, float)
    s = np.asarray(s, float)
    nr, nz = s.shape
    dt = np.diff(depth)                                       # (N_z-1,)
    dtau = dt[None, :] * (np.asarray(fac_ray)[:, None] / np.abs(mu_ray)[:, None])
    out = np.zeros((nr, nz))
    down = np.asarray(mu_ray) < 0
    up = ~down
    itop = np.broadcast_to(np.asarray(i_top, float), (nr,))
    ibot = np.broadcast_to(np.asarray(i_bot, float), (nr,))
    out[down, 0] = itop[down]
    out[up, nz - 1] = ibot[up]
    if scheme == "implicit_euler":
        for i in range(1, nz):                      # eq. ie_1
            d = dtau[down, i - 1]
            out[down, i] = (out[down, i - 1] + d * s[down, i]) / (1.0 + d)
        for i in range(nz - 2, -1, -1):             # eq. ie_2
            d = dtau[up, i]
            out[up, i] = (out[up, i + 1] + d * s[up, i]) / (1.0 + d)
    elif scheme == "linear_sc":
        for i in range(1, nz):
            e, a, c = exp_weights(dtau[down, i - 1])
            out[down, i] = e * out[down, i - 1] + a * s[down, i - 1] + c * s[down, i]
        for i in range(nz - 2, -1, -1):
            e, a, c = exp_weights(dtau[up, i])
            out[up, i] = e * out[up, i + 1] + a * s[up, i + 1] + c * s[up, i]
    elif scheme == "quadratic_sc":
        # downgoing rays: upwind i-1, downwind i+1; the last point (i = nz-1)
        # takes the linear step
        for i in range(1, nz):
            if i + 1 < nz:
                e, pu, p0, pd = quad_weights(dtau[down, i - 1], dtau[down, i])
                out[down, i] = (e * out[down, i - 1] + pu * s[down, i - 1] + p0 * s[down, i]
                                + pd * s[down, i + 1])
            else:
                e, a, c = exp_weights(dtau[down, i - 1])
                out[down, i] = e * out[down, i - 1] + a * s[down, i - 1] + c * s[down, i]
        # upgoing rays: upwind i+1, downwind i-1; the last point is i = 0
        for i in range(nz - 2, -1, -1):
            if i > 0:
                e, pu, p0, pd = quad_weights(dtau[up, i], dtau[up, i - 1])
                out[up, i] = (e * out[up, i + 1] + pu * s[up, i + 1] + p0 * s[up, i]
                              + pd * s[up, i - 1])
            else:
                e, a, c = exp_weights(dtau[up, i])
                out[up, i] = e * out[up, i + 1] + a * s[up, i + 1] + c * s[up, i]
    else:
        raise ValueError(scheme)
    return out


def _upwind_stencil(omega_o, nx, ny, nz):
    """Cell offsets and bilinear fractions of the upwind point of ordinate o."""
    mu = omega_o[2]
    dz = 1.0 / (nz - 1)
    path = dz / abs(mu)
    sx = -omega_o[0] * path * nx        # displacement in cells (dx = 1/nx)
    sy = -omega_o[1] * path * ny
    i0 = math.floor(sx)
    j0 = math.floor(sy)
    return i0, sx - i0, j0, sy - j0, path


def _interp(plane, i0, tx, j0, ty):
    """Bilinear periodic interpolation of plane[..., y, x] at (y+j0+ty, x+i0+tx)."""
    def shifted(a, b):
        return np.roll(plane, shift=(-a, -b), axis=(-2, -1))
    return ((1 - ty) * (1 - tx) * shifted(j0, i0) + (1 - ty) * tx * shifted(j0, i0 + 1)
            + ty * (1 - tx) * shifted(j0 + 1, i0) + ty * tx * shifted(j0 + 1, i0 + 1))


def sweep_box(k_line, omega, fac_nu, s, i_top=0.0, i_bot=0.0, scheme: str = "linear_sc"):
    """Plane-to-plane short-characteristics sweep in the periodic box.

    k_line (nz, ny, nx), z index 0 = bottom; omega (n_omega, 3); fac_nu (n_nu,)
    = phi_nu + r; s (n_omega*n_nu, nz, ny, nx) with ray k = o*n_nu + nu.
    Incoming intensities: i_bot enters at the bottom plane (mu > 0), i_top at
    the top plane (mu < 0).
    scheme 'linear_sc', or 'quadratic_sc': the source is also taken at the
    downwind point, on the next plane downstream displaced by +Omega_xy dz/|mu|
    (bilinear, periodic, like the upwind point), over the downwind interval
    D_d = (k_0 + k_d)/2 (phi + r) dz/|mu|; the last plane takes the linear step.
    """
    k_line = np.asarray(k_line, float)
    nz, ny, nx = k_line.shape
    n_om = omega.shape[0]
    n_nu = len(fac_nu)
    s = np.asarray(s, float).reshape(n_om, n_nu, nz, ny, nx)
    out = np.zeros_like(s)
    fac = np.asarray(fac_nu, float)[:, None, None]
    for o in range(n_om):
        i0, tx, j0, ty, path = _upwind_stencil(omega[o], nx, ny, nz)
        # the downwind point: the same displacement in the opposite direction
        d0, dtx, e0, dty, _ = _upwind_stencil(-omega[o], nx, ny, nz)
        if omega[o, 2] > 0:
            first, planes, step = 0, range(1, nz), -1
            out[o, :, first] = i_bot
        else:
            first, planes, step = nz - 1, range(nz - 2, -1, -1), +1
            out[o, :, first] = i_top
        for z in planes:
            zu = z + step
            zd = z - step
            k_up = _interp(k_line[zu], i0, tx, j0, ty)
            d = 0.5 * (k_up + k_line[z])[None] * path * fac
            i_up = _interp(out[o, :, zu], i0, tx, j0, ty)
            s_up = _interp(s[o, :, zu], i0, tx, j0, ty)
            if scheme == "quadratic_sc" and 0 <= zd < nz:
                k_dn = _interp(k_line[zd], d0, dtx, e0, dty)
                dd = 0.5 * (k_dn + k_line[z])[None] * path * fac
                s_dn = _interp(s[o, :, zd], d0, dtx, e0, dty)
                e, pu, p0, pd = quad_weights(d, dd)
                out[o, :, z] = e * i_up + pu * s_up + p0 * s[o, :, z] + pd * s_dn
            elif scheme in ("linear_sc", "quadratic_sc"):
                e, a, c = exp_weights(d)
                out[o, :, z] = e * i_up + a * s_up + c * s[o, :, z]
            else:
                raise ValueError(scheme)
    return out.reshape(n_om * n_nu, nz, ny, nx)
