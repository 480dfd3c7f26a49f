// Host-side problem set-up in FP64: quadratures, redistribution kernel,
// scattering block Mhat, upwind stencils.
//
// Paper Sec. 5 (set-up): two Gauss-Legendre sets of n_mu/2 inclinations, one
// per hemisphere; trapezoidal frequencies; Sec. 5.3: tensor product with
// equidistant azimuths in 3D.  Sec. 2: the redistribution function is
// normalised to unit double integral (photon conservation); Sec. 3.3: Psi is
// symmetric and Sigma = Gamma Psi W.
#include <algorithm>
#include <cmath>

#include "rt_internal.h"

namespace rtsn {

// Gauss-Legendre nodes/weights on [-1, 1] by Newton iteration on P_n with the
// three-term recurrence; nodes returned ascending.
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int l = 2; l <= n; ++l) {
        double p2 = ((2.0 * l - 1.0) * z * p1 - (l - 1.0) * p0) / l;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p1 = z; p0 = 1.0; }
      // P_n = p1, P_{n-1} = p0; P_n' = n (z P_n - P_{n-1}) / (z^2 - 1)
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    // recompute derivative at the converged node for the weight
    double p0 = 1.0, p1 = z;
    for (int l = 2; l <= n; ++l) {
      double p2 = ((2.0 * l - 1.0) * z * p1 - (l - 1.0) * p0) / l;
      p0 = p1;
      p1 = p2;
    }
    if (n == 1) { p1 = z; p0 = 1.0; }
    dp = n * (z * p1 - p0) / (z * z - 1.0);
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int a, int b) { return x[a] < x[b]; });
  std::vector<double> xs(n), ws(n);
  for (int i = 0; i < n; ++i) { xs[i] = x[idx[i]]; ws[i] = w[idx[i]]; }
  x.swap(xs);
  w.swap(ws);
}

// Double-Gauss inclinations, ascending, weights summing to 1.
static void double_gauss(int n_mu, std::vector<double>& mu, std::vector<double>& w) {
  int h = n_mu / 2;
  std::vector<double> gx, gw;
  gauss_legendre(h, gx, gw);
  std::vector<double> mp(h), wp(h);
  for (int i = 0; i < h; ++i) {
    mp[i] = 0.5 * (gx[i] + 1.0);
    wp[i] = 0.25 * gw[i];
  }
  mu.resize(n_mu);
  w.resize(n_mu);
  for (int i = 0; i < h; ++i) {
    mu[i] = -mp[h - 1 - i];
    w[i] = wp[h - 1 - i];
    mu[h + i] = mp[i];
    w[h + i] = wp[i];
  }
}

// Symmetric diagonal scaling d so that sum_j w_j d_i G_ij d_j = phi_i.
static std::vector<double> coherent_scaling(const std::vector<double>& x,
                                            const std::vector<double>& w,
                                            const std::vector<double>& phi,
                                            double width2) {
  const int n = (int)x.size();
  std::vector<double> g((size_t)n * n), d(n), gd(n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double dx = x[i] - x[j];
      g[(size_t)i * n + j] = std::exp(-dx * dx / width2);
    }
  for (int i = 0; i < n; ++i) d[i] = std::sqrt(phi[i]);
  double best = 1e300;
  for (int it = 0; it < 200000; ++it) {
    for (int i = 0; i < n; ++i) {
      double s = 0.0;
      for (int j = 0; j < n; ++j) s += g[(size_t)i * n + j] * (w[j] * d[j]);
      gd[i] = s;
    }
    double err = 0.0;
    for (int i = 0; i < n; ++i) err = std::max(err, std::fabs(d[i] * gd[i] - phi[i]) / phi[i]);
    if (err < 1e-15) break;
    if (err >= best && err < 1e-13) break;
    best = std::min(best, err);
    for (int i = 0; i < n; ++i) d[i] = std::sqrt(d[i] * phi[i] / gd[i]);
  }
  return d;
}

// Factors of Mhat = (P_ang diag(w_o)) (x) (diag(1/(phi + r)) P_nu diag(w_nu))
// for the dipole phase function (Sec. 2), whose angular kernel has low rank:
//   3D: 3/4 (1 + (O.O')^2) = q(O)^T C q(O') with
//       q(O) = (x^2, y^2, z^2, sqrt2 xy, sqrt2 xz, sqrt2 yz), since
//       q(O).q(O') = (O.O')^2, and 1 = |O|^2 |O'|^2 = q(O)^T E q(O') with E
//       the 3x3 block of ones on the squares; C = 3/4 (I_6 + E), rank 6;
//   1D: 3/8 (3 - m^2 - m'^2 + 3 m^2 m'^2) = (1, m^2) C (1, m'^2)^T with
//       C = 3/8 [[3, -1], [-1, 3]], rank 2.
// fq[o][q] = q(O_o)_q, fg[o][q] = w_o (C q(O_o))_q, fb = the frequency block.
static void build_factors(Tables& t, bool box, double r, const std::vector<double>& pf) {
  const int n_om = (int)t.mu_o.size(), n_nu = (int)t.x_nu.size();
  const int R = box ? 6 : 2;
  t.frank = R;
  t.fq.assign((size_t)n_om * R, 0.0);
  t.fg.assign((size_t)n_om * R, 0.0);
  double C[6][6] = {};
  if (box) {
    for (int a = 0; a < 6; ++a) C[a][a] = 0.75;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) C[a][b] += 0.75;
  } else {
    C[0][0] = C[1][1] = 0.375 * 3.0;
    C[0][1] = C[1][0] = -0.375;
  }
  const double r2 = std::sqrt(2.0);
  for (int o = 0; o < n_om; ++o) {
    double q[6];
    if (box) {
      const double x = t.om_x[o], y = t.om_y[o], z = t.mu_o[o];
      q[0] = x * x; q[1] = y * y; q[2] = z * z;
      q[3] = r2 * x * y; q[4] = r2 * x * z; q[5] = r2 * y * z;
    } else {
      q[0] = 1.0;
      q[1] = t.mu_o[o] * t.mu_o[o];
    }
    for (int a = 0; a < R; ++a) {
      double cq = 0.0;
      for (int b = 0; b < R; ++b) cq += C[a][b] * q[b];
      t.fq[(size_t)o * R + a] = q[a];
      t.fg[(size_t)o * R + a] = t.w_o[o] * cq;
    }
  }
  t.fb.assign((size_t)n_nu * n_nu, 0.0);
  for (int i = 0; i < n_nu; ++i)
    for (int j = 0; j < n_nu; ++j)
      t.fb[(size_t)i * n_nu + j] = pf[(size_t)i * n_nu + j] * t.w_nu[j] / (t.phi[i] + r);
}

void build_tables(const rt_problem_desc& desc, Tables& t) {
  const bool box = desc.geom == RT_GEOM_BOX;
  const int n_mu = desc.n_mu, n_az = box ? desc.n_az : 1, n_nu = desc.n_nu;
  const int n_om = n_mu * n_az, n_r = n_om * n_nu;

  std::vector<double> mu, wmu;
  double_gauss(n_mu, mu, wmu);
  t.mu_o.resize(n_om);
  t.w_o.resize(n_om);
  t.om_x.assign(n_om, 0.0);
  t.om_y.assign(n_om, 0.0);
  for (int m = 0; m < n_mu; ++m)
    for (int b = 0; b < n_az; ++b) {
      int o = m * n_az + b;
      double az = (b + 0.5) * 2.0 * M_PI / n_az;
      double st = std::sqrt(std::max(0.0, 1.0 - mu[m] * mu[m]));
      t.mu_o[o] = mu[m];
      t.w_o[o] = wmu[m] / n_az;
      if (box) {
        t.om_x[o] = st * std::cos(az);
        t.om_y[o] = st * std::sin(az);
      }
    }

  t.x_nu.resize(n_nu);
  t.w_nu.resize(n_nu);
  t.phi.resize(n_nu);
  if (n_nu == 1) {
    t.x_nu[0] = 0.0;
    t.w_nu[0] = 1.0;
    t.phi[0] = 1.0;
  } else {
    double h = 2.0 * desc.x_max / (n_nu - 1);
    double area = 0.0;
    for (int j = 0; j < n_nu; ++j) {
      t.x_nu[j] = -desc.x_max + h * j;
      t.w_nu[j] = (j == 0 || j == n_nu - 1) ? 0.5 * h : h;
      t.phi[j] = std::exp(-t.x_nu[j] * t.x_nu[j]) / std::sqrt(M_PI);
      area += t.w_nu[j] * t.phi[j];
    }
    for (int j = 0; j < n_nu; ++j) t.phi[j] /= area;
  }

  t.mu_ray.resize(n_r);
  t.w_ray.resize(n_r);
  t.phi_ray.resize(n_r);
  t.fac_ray.resize(n_r);
  for (int o = 0; o < n_om; ++o)
    for (int j = 0; j < n_nu; ++j) {
      int k = o * n_nu + j;
      t.mu_ray[k] = t.mu_o[o];
      t.w_ray[k] = t.w_o[o] * t.w_nu[j];
      t.phi_ray[k] = t.phi[j];
      t.fac_ray[k] = t.phi[j] + desc.r;
    }

  // Psi (kernel) then Mhat = diag(1/fac) Psi diag(w)
  t.mhat.assign((size_t)n_r * n_r, 0.0);
  if (desc.kernel == RT_KERNEL_EXPLICIT) {
    for (size_t i = 0; i < (size_t)n_r * n_r; ++i) t.mhat[i] = desc.kernel_matrix[i];
  } else {
    // frequency kernel: (1 - c) phi phi^T + c d_i G_ij d_j
    std::vector<double> pf((size_t)n_nu * n_nu);
    if (n_nu == 1) {
      pf[0] = 1.0;
    } else {
      std::vector<double> d = coherent_scaling(t.x_nu, t.w_nu, t.phi, desc.coh_width2);
      for (int i = 0; i < n_nu; ++i)
        for (int j = 0; j < n_nu; ++j) {
          double dx = t.x_nu[i] - t.x_nu[j];
          double coh = d[i] * std::exp(-dx * dx / desc.coh_width2) * d[j];
          pf[(size_t)i * n_nu + j] =
              (1.0 - desc.coh_frac) * t.phi[i] * t.phi[j] + desc.coh_frac * coh;
        }
    }
    // angular dipole kernel
    std::vector<double> pa((size_t)n_om * n_om);
    for (int a = 0; a < n_om; ++a)
      for (int b = 0; b < n_om; ++b) {
        double v;
        if (box) {
          double c = t.om_x[a] * t.om_x[b] + t.om_y[a] * t.om_y[b] + t.mu_o[a] * t.mu_o[b];
          v = 0.75 * (1.0 + c * c);
        } else {
          double m2 = t.mu_o[a] * t.mu_o[a], n2 = t.mu_o[b] * t.mu_o[b];
          v = 0.375 * (3.0 - m2 - n2 + 3.0 * m2 * n2);
        }
        pa[(size_t)a * n_om + b] = v;
      }
    for (int a = 0; a < n_om; ++a)
      for (int i = 0; i < n_nu; ++i)
        for (int b = 0; b < n_om; ++b)
          for (int j = 0; j < n_nu; ++j)
            t.mhat[(size_t)(a * n_nu + i) * n_r + (b * n_nu + j)] =
                pa[(size_t)a * n_om + b] * pf[(size_t)i * n_nu + j];
    build_factors(t, box, desc.r, pf);
  }
  for (int k = 0; k < n_r; ++k)
    for (int kp = 0; kp < n_r; ++kp)
      t.mhat[(size_t)k * n_r + kp] *= t.w_ray[kp] / t.fac_ray[k];
}

}  // namespace rtsn
