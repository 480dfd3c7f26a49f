// extern "C" entry points of librtsn (declared in include/rtsn.h), problem
// construction and operator dispatch.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "gemm16_dev.h"
#include "gemm_dev.h"
#include "krylov.h"

namespace rtsn {

static thread_local std::string g_last_error;

void fail(rt_status code, const std::string& msg) { throw RtError{code, msg}; }

void set_last_error(const std::string& msg) { g_last_error = msg; }

std::shared_mutex& capture_mutex() {
  static std::shared_mutex mu;
  return mu;
}

void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    (void)hipGetLastError();
    fail(e == hipErrorOutOfMemory ? RT_E_NOMEM : RT_E_DEVICE,
         std::string(what) + ": " + hipGetErrorString(e));
  }
}

Problem::~Problem() {
  delete ws;
  hipFree(d_mhat64);
  hipFree(d_mhat32);
  hipFree(d_a8_bf16);
  hipFree(d_a8_bf16_lo);
  hipFree(d_a8_f16);
  hipFree(d_l16);
  hipFree(d_f16_rowscale);
  hipFree(d_albedo);
  hipFree(d_thermal);
  hipFree(d_dt);
  hipFree(d_kline);
  hipFree(d_ray_mu);
  hipFree(d_ray_fac);
  hipFree(d_stencil);
  hipFree(d_lbuf);
  hipFree(d_rhs);
  hipFree(d_fq64);
  hipFree(d_fg64);
  hipFree(d_fb64);
  hipFree(d_fq32);
  hipFree(d_fg32);
  hipFree(d_fb32);
  hipFree(d_fwork);
  hipFree(d_cmhat64);
  hipFree(d_cmhat32);
  hipFree(d_cidx);
  hipFree(d_calb);
  hipFree(d_cwork);
  hipFree(d_oz_a);
  hipFree(d_oz_ea);
  hipFree(d_ozwork);
  hipFree(d_prec_dbar);
  hipFree(d_prec_F64);
  hipFree(d_prec_G64);
  hipFree(d_prec_T64);
  hipFree(d_prec_F32);
  hipFree(d_prec_G32);
  hipFree(d_prec_T32);
  hipFree(d_prec_T16);
  hipFree(d_prec_work);
}

size_t lambda_elem_bytes(int precision) {
  switch (precision) {
    case RT_PREC_FP64: return 8;
    case RT_PREC_FP32: return 4;
    case RT_PREC_BF16:
    case RT_PREC_FP16: return 2;
    case RT_PREC_BF16X3: return 4;
    default: return 8;
  }
}

int64_t l16_part_elems(const Problem& p) { return (int64_t)p.kp16 * p.np16; }

uint16_t* problem_l16(Problem& p, hipStream_t st) {
  if (!p.d_l16) {
    const size_t bytes = 2 * (size_t)l16_part_elems(p) * sizeof(uint16_t);
    RT_HIP(hipMalloc(&p.d_l16, bytes));
    RT_HIP(hipMemsetAsync(p.d_l16, 0, bytes, st));
  }
  return p.d_l16;
}

static void* problem_fwork(Problem& p, size_t elem) {
  const size_t bytes = factored_work_elems(p) * elem;
  if (bytes > p.fwork_bytes) {
    hipFree(p.d_fwork);
    p.d_fwork = nullptr;
    p.fwork_bytes = 0;
    RT_HIP(hipMalloc(&p.d_fwork, bytes));
    p.fwork_bytes = bytes;
  }
  return p.d_fwork;
}

static void* problem_cwork(Problem& p, size_t elem) {
  const size_t bytes = classes_work_elems(p) * elem;
  if (bytes > p.cwork_bytes) {
    hipFree(p.d_cwork);
    p.d_cwork = nullptr;
    p.cwork_bytes = 0;
    RT_HIP(hipMalloc(&p.d_cwork, bytes));
    p.cwork_bytes = bytes;
  }
  return p.d_cwork;
}

static void* problem_ozwork(Problem& p) {
  const size_t bytes = ozaki_work_bytes(p);
  if (bytes > p.ozwork_bytes) {
    hipFree(p.d_ozwork);
    p.d_ozwork = nullptr;
    p.ozwork_bytes = 0;
    RT_HIP(hipMalloc(&p.d_ozwork, bytes));
    p.ozwork_bytes = bytes;
  }
  return p.d_ozwork;
}

void require_one_kernel(const Problem& p, const char* what) {
  if (p.n_classes > 1)
    fail(RT_E_INVALID, std::string(what) + " is not available with per-point scattering classes");
}

void apply_sigma_f64(Problem& p, const double* L, const double* x, double* y,
                     const double* xscale, double sign, hipStream_t st, gemm::TileDots* dots) {
  if (p.n_classes > 1) {
    if (dots) fail(RT_E_INVALID, "fused Arnoldi dots need the one-kernel scattering GEMM");
    launch_sigma_classes_f64(p, L, x, y, static_cast<double*>(problem_cwork(p, sizeof(double))),
                             xscale, sign, st);
  } else if (p.sigma_form == RT_SIGMA_FACTORED) {
    if (dots) fail(RT_E_INVALID, "fused Arnoldi dots need the dense scattering GEMM");
    launch_sigma_factored_f64(p, L, x, y, static_cast<double*>(problem_fwork(p, sizeof(double))),
                              xscale, sign, st);
  } else if (p.sigma_form == RT_SIGMA_OZAKI) {
    if (dots) fail(RT_E_INVALID, "fused Arnoldi dots need the dense scattering GEMM");
    launch_sigma_ozaki(p, L, x, y, problem_ozwork(p), xscale, sign, st);
  } else {
    launch_sigma_f64(p, L, x, y, xscale, sign, st, dots);
  }
}

void apply_sigma_f32(Problem& p, const float* L, const float* x, float* y,
                     const double* xscale, double sign, hipStream_t st, gemm::TileDots* dots) {
  if (p.n_classes > 1) {
    if (dots) fail(RT_E_INVALID, "fused Arnoldi dots need the one-kernel scattering GEMM");
    launch_sigma_classes_f32(p, L, x, y, static_cast<float*>(problem_cwork(p, sizeof(float))),
                             xscale, sign, st);
  } else if (p.sigma_form == RT_SIGMA_FACTORED) {
    if (dots) fail(RT_E_INVALID, "fused Arnoldi dots need the dense scattering GEMM");
    launch_sigma_factored_f32(p, L, x, y, static_cast<float*>(problem_fwork(p, sizeof(float))),
                              xscale, sign, st);
  } else {
    launch_sigma_f32(p, L, x, y, xscale, sign, st, dots);
  }
}

void* problem_lbuf(Problem& p, size_t bytes) {
  if (bytes > p.lbuf_bytes) {
    hipFree(p.d_lbuf);
    p.d_lbuf = nullptr;
    p.lbuf_bytes = 0;
    RT_HIP(hipMalloc(&p.d_lbuf, bytes));
    p.lbuf_bytes = bytes;
  }
  return p.d_lbuf;
}

namespace {

// Round-to-nearest-even float -> bfloat16 bits (host side).
uint16_t bf16_bits(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;  // NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

float bf16_value(uint16_t b) {
  uint32_t u = (uint32_t)b << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

uint16_t f16_bits(float f) {
  _Float16 h = (_Float16)f;
  uint16_t b;
  std::memcpy(&b, &h, 2);
  return b;
}

template <typename T>
T* upload(const T* h, size_t count, int64_t& total) {
  void* d = nullptr;
  RT_HIP(hipMalloc(&d, count * sizeof(T)));
  RT_HIP(hipMemcpy(d, h, count * sizeof(T), hipMemcpyHostToDevice));
  total += (int64_t)(count * sizeof(T));
  return static_cast<T*>(d);
}

bool all_finite(const double* a, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(a[i])) return false;
  return true;
}

void validate(const rt_problem_desc& d) {
  if (d.geom != RT_GEOM_SLAB && d.geom != RT_GEOM_BOX) fail(RT_E_INVALID, "geom must be SLAB or BOX");
  if (d.nz < 2) fail(RT_E_INVALID, "nz must be >= 2");
  if (d.n_mu < 2 || (d.n_mu & 1)) fail(RT_E_INVALID, "n_mu must be even and >= 2");
  if (d.n_nu < 1) fail(RT_E_INVALID, "n_nu must be >= 1");
  if (d.n_nu > 1 && !(d.x_max > 0)) fail(RT_E_INVALID, "x_max must be > 0");
  if (!(d.r >= 0) || !std::isfinite(d.r)) fail(RT_E_INVALID, "continuum ratio r must be >= 0");
  if (d.geom == RT_GEOM_SLAB) {
    if (d.nx != 1 || d.ny != 1) fail(RT_E_INVALID, "slab needs nx = ny = 1");
    if (!d.depth) fail(RT_E_INVALID, "slab needs depth[nz]");
    if (!all_finite(d.depth, d.nz)) fail(RT_E_NONFINITE, "depth has NaN/Inf");
    for (int i = 0; i + 1 < d.nz; ++i)
      if (!(d.depth[i + 1] > d.depth[i])) fail(RT_E_INVALID, "depth must increase strictly");
    if (d.nz > 64 * 1024) fail(RT_E_INVALID, "nz too large for the slab sweep");
  } else {
    if (d.nx < 1 || d.ny < 1) fail(RT_E_INVALID, "box needs nx, ny >= 1");
    if (d.n_az < 1) fail(RT_E_INVALID, "box needs n_az >= 1");
    if (!d.k_line) fail(RT_E_INVALID, "box needs k_line[nz*ny*nx]");
    const size_t ns = (size_t)d.nx * d.ny * d.nz;
    if (!all_finite(d.k_line, ns)) fail(RT_E_NONFINITE, "k_line has NaN/Inf");
    for (size_t i = 0; i < ns; ++i)
      if (!(d.k_line[i] > 0)) fail(RT_E_INVALID, "k_line must be > 0");
    if ((int64_t)d.nx * d.ny > 4096) fail(RT_E_INVALID, "box plane larger than 4096 points");
    if (d.formal == RT_FORMAL_IMPLICIT_EULER)
      fail(RT_E_INVALID, "implicit Euler is a slab scheme");
  }
  if (d.formal != RT_FORMAL_LINEAR_SC && d.formal != RT_FORMAL_IMPLICIT_EULER &&
      d.formal != RT_FORMAL_QUADRATIC_SC)
    fail(RT_E_INVALID, "unknown formal solver");
  if (d.kernel == RT_KERNEL_EXPLICIT) {
    if (!d.kernel_matrix && d.n_classes <= 1)
      fail(RT_E_INVALID, "explicit kernel needs kernel_matrix");
  } else if (d.kernel == RT_KERNEL_DIPOLE_PRD) {
    if (!(d.coh_frac >= 0 && d.coh_frac <= 1)) fail(RT_E_INVALID, "coh_frac must be in [0,1]");
    if (!(d.coh_width2 > 0)) fail(RT_E_INVALID, "coh_width2 must be > 0");
  } else {
    fail(RT_E_INVALID, "unknown kernel");
  }
  if (!std::isfinite(d.i_top) || !std::isfinite(d.i_bot) || !std::isfinite(d.eps) ||
      !std::isfinite(d.planck))
    fail(RT_E_NONFINITE, "non-finite scalar input");
  if (d.n_classes > 1) {
    if (d.n_classes > 256) fail(RT_E_INVALID, "at most 256 scattering classes");
    if (!d.point_class) fail(RT_E_INVALID, "n_classes > 1 needs point_class");
    const size_t ns = (size_t)d.nx * d.ny * d.nz;
    for (size_t i = 0; i < ns; ++i)
      if (d.point_class[i] < 0 || d.point_class[i] >= d.n_classes)
        fail(RT_E_INVALID, "point_class out of range");
    if (d.kernel == RT_KERNEL_DIPOLE_PRD) {
      if (!d.class_coh_frac) fail(RT_E_INVALID, "dipole x PRD classes need class_coh_frac");
      for (int c = 0; c < d.n_classes; ++c)
        if (!(d.class_coh_frac[c] >= 0 && d.class_coh_frac[c] <= 1))
          fail(RT_E_INVALID, "class_coh_frac must be in [0,1]");
    } else if (!d.class_kernels) {
      fail(RT_E_INVALID, "explicit classes need class_kernels");
    }
  }
}

}  // namespace

void problem_build(Problem& p, const rt_problem_desc& d_in) {
  validate(d_in);
  // with classes, the problem's own tables (and rt_problem_tables) are class 0's
  rt_problem_desc d = d_in;
  const bool classes = d_in.n_classes > 1;
  if (classes) {
    if (d.kernel == RT_KERNEL_EXPLICIT) d.kernel_matrix = d_in.class_kernels;
    else d.coh_frac = d_in.class_coh_frac[0];
  }
  p.geom = d.geom;
  p.nx = d.nx;
  p.ny = d.ny;
  p.nz = d.nz;
  p.n_mu = d.n_mu;
  p.n_az = d.geom == RT_GEOM_BOX ? d.n_az : 1;
  p.n_nu = d.n_nu;
  p.n_omega = p.n_mu * p.n_az;
  p.n_r = p.n_omega * p.n_nu;
  p.n_s = (int64_t)p.nx * p.ny * p.nz;
  p.n = p.n_s * p.n_r;
  p.formal = d.formal;
  p.r = d.r;
  p.i_top = d.i_top;
  p.i_bot = d.i_bot;
  if (p.n_r > 16384) fail(RT_E_INVALID, "too many rays (n_mu*n_az*n_nu > 16384)");
  if (d.kernel == RT_KERNEL_EXPLICIT &&
      !all_finite(d.kernel_matrix, (size_t)p.n_r * p.n_r * (classes ? d_in.n_classes : 1)))
    fail(RT_E_NONFINITE, "kernel matrix has NaN/Inf");

  build_tables(d, p.tab);

  // per-point albedo 1 - eps and thermal source t = (eps phi + r) B / (phi + r)
  std::vector<double> eps(p.n_s), bpl(p.n_s), alb(p.n_s);
  for (int64_t i = 0; i < p.n_s; ++i) {
    eps[i] = d.eps_field ? d.eps_field[i] : d.eps;
    bpl[i] = d.planck_field ? d.planck_field[i] : d.planck;
    if (!std::isfinite(eps[i]) || !std::isfinite(bpl[i]))
      fail(RT_E_NONFINITE, "eps/planck field has NaN/Inf");
    if (eps[i] < 0 || eps[i] > 1) fail(RT_E_INVALID, "eps must be in [0, 1]");
    alb[i] = 1.0 - eps[i];
  }
  std::vector<double> therm((size_t)p.n);
  for (int k = 0; k < p.n_r; ++k) {
    const double ph = p.tab.phi_ray[k], fac = p.tab.fac_ray[k];
    for (int64_t i = 0; i < p.n_s; ++i)
      therm[(size_t)k * p.n_s + i] = (eps[i] * ph + d.r) * bpl[i] / fac;
  }

  {
    double amax = 0.0, rmax = 0.0;
    for (int64_t i = 0; i < p.n_s; ++i) amax = std::max(amax, alb[i]);
    for (int k = 0; k < p.n_r; ++k) {
      double r = 0.0;
      for (int kp = 0; kp < p.n_r; ++kp) r += std::fabs(p.tab.mhat[(size_t)k * p.n_r + kp]);
      rmax = std::max(rmax, r);
    }
    p.scatter_inf = amax * rmax;
  }

  int64_t tot = 0;
  RT_HIP(hipSetDevice(p.device));
  {
    // FP64 / FP32 copies, transposed for the MFMA GEMM: element (k, k') at
    // k' * lda + k, lda = n_r rounded up to the 128-row tile, zero rows up to
    // a multiple of 32 in k'
    const int lda = (p.n_r + gemm::MPAD - 1) / gemm::MPAD * gemm::MPAD;
    const int kp = (p.n_r + gemm::KPAD - 1) / gemm::KPAD * gemm::KPAD;
    p.lda_mhat = lda;
    const size_t sz = (size_t)kp * lda;
    std::vector<double> m64(sz, 0.0);
    std::vector<float> m32(sz, 0.f);
    for (int k = 0; k < p.n_r; ++k)
      for (int kp2 = 0; kp2 < p.n_r; ++kp2) {
        const double m = p.tab.mhat[(size_t)k * p.n_r + kp2];
        m64[(size_t)kp2 * lda + k] = m;
        m32[(size_t)kp2 * lda + k] = (float)m;
      }
    p.d_mhat64 = upload(m64.data(), sz, tot);
    p.d_mhat32 = upload(m32.data(), sz, tot);
    if (classes) {
      // one transposed Mhat per class (the same layout), the points sorted
      // by class with their albedo in that order
      const int nc = d_in.n_classes;
      p.n_classes = nc;
      p.class_mhat_stride = sz;
      std::vector<double> c64((size_t)nc * sz, 0.0);
      std::vector<float> c32((size_t)nc * sz, 0.f);
      for (int c = 0; c < nc; ++c) {
        rt_problem_desc dc = d_in;
        if (d.kernel == RT_KERNEL_EXPLICIT)
          dc.kernel_matrix = d_in.class_kernels + (size_t)c * p.n_r * p.n_r;
        else
          dc.coh_frac = d_in.class_coh_frac[c];
        Tables tc;
        build_tables(dc, tc);
        double rmax = 0.0;
        for (int k = 0; k < p.n_r; ++k) {
          double r = 0.0;
          for (int kp2 = 0; kp2 < p.n_r; ++kp2) {
            const double m = tc.mhat[(size_t)k * p.n_r + kp2];
            c64[(size_t)c * sz + (size_t)kp2 * lda + k] = m;
            c32[(size_t)c * sz + (size_t)kp2 * lda + k] = (float)m;
            r += std::fabs(m);
          }
          rmax = std::max(rmax, r);
        }
        double amax = 0.0;
        for (int64_t i = 0; i < p.n_s; ++i) amax = std::max(amax, alb[i]);
        p.scatter_inf = std::max(p.scatter_inf, amax * rmax);
      }
      p.d_cmhat64 = upload(c64.data(), c64.size(), tot);
      p.d_cmhat32 = upload(c32.data(), c32.size(), tot);
      p.class_off.assign(nc + 1, 0);
      for (int64_t i = 0; i < p.n_s; ++i) p.class_off[d_in.point_class[i] + 1]++;
      for (int c = 0; c < nc; ++c) p.class_off[c + 1] += p.class_off[c];
      std::vector<int32_t> idx(p.n_s);
      std::vector<double> calb(p.n_s);
      std::vector<int64_t> fill(p.class_off.begin(), p.class_off.end() - 1);
      for (int64_t i = 0; i < p.n_s; ++i) {
        const int64_t at = fill[d_in.point_class[i]]++;
        idx[at] = (int32_t)i;
        calb[at] = alb[i];
      }
      p.d_cidx = upload(idx.data(), idx.size(), tot);
      p.d_calb = upload(calb.data(), calb.size(), tot);
    }
  }
  {
    // 16-bit copies in the k8 layout of the MFMA GEMM (see gemm16_dev.h):
    // element (k, k') at ((k' / 8) * mp16 + k) * 8 + k' % 8, zero padded
    p.mp16 = (int)g16::round_up(p.n_r, g16::kMAlign);
    p.kp16 = (int)g16::round_up(p.n_r, g16::kKAlign);
    p.np16 = g16::round_up(p.n_s, g16::kMAlign);
    const size_t sz = (size_t)p.mp16 * p.kp16;
    std::vector<uint16_t> hi(sz, 0), lo(sz, 0), h16(sz, 0);
    std::vector<float> rs(p.n_r, 1.f);
    for (int k = 0; k < p.n_r; ++k) {
      double rmax = 0.0;
      for (int kp = 0; kp < p.n_r; ++kp)
        rmax = std::max(rmax, std::fabs(p.tab.mhat[(size_t)k * p.n_r + kp]));
      if (!(rmax > 0)) rmax = 1.0;
      rs[k] = (float)rmax;
      for (int kp = 0; kp < p.n_r; ++kp) {
        const double m = p.tab.mhat[(size_t)k * p.n_r + kp];
        const size_t at = ((size_t)(kp / 8) * p.mp16 + k) * 8 + kp % 8;
        const uint16_t h = bf16_bits((float)m);
        hi[at] = h;
        lo[at] = bf16_bits((float)(m - (double)bf16_value(h)));
        h16[at] = f16_bits((float)(m / (double)rs[k]));
      }
    }
    p.d_a8_bf16 = upload(hi.data(), sz, tot);
    p.d_a8_bf16_lo = upload(lo.data(), sz, tot);
    p.d_a8_f16 = upload(h16.data(), sz, tot);
    p.d_f16_rowscale = upload(rs.data(), rs.size(), tot);
  }
  if (p.tab.frank > 0) {
    const auto& t = p.tab;
    p.d_fq64 = upload(t.fq.data(), t.fq.size(), tot);
    p.d_fg64 = upload(t.fg.data(), t.fg.size(), tot);
    p.d_fb64 = upload(t.fb.data(), t.fb.size(), tot);
    std::vector<float> q32(t.fq.begin(), t.fq.end()), g32(t.fg.begin(), t.fg.end()),
        b32(t.fb.begin(), t.fb.end());
    p.d_fq32 = upload(q32.data(), q32.size(), tot);
    p.d_fg32 = upload(g32.data(), g32.size(), tot);
    p.d_fb32 = upload(b32.data(), b32.size(), tot);
  }
  p.d_albedo = upload(alb.data(), alb.size(), tot);
  p.d_thermal = upload(therm.data(), therm.size(), tot);
  p.d_ray_mu = upload(p.tab.mu_ray.data(), p.tab.mu_ray.size(), tot);
  p.d_ray_fac = upload(p.tab.fac_ray.data(), p.tab.fac_ray.size(), tot);
  if (p.geom == RT_GEOM_SLAB) {
    std::vector<double> dt(p.nz - 1);
    for (int i = 0; i + 1 < p.nz; ++i) dt[i] = d.depth[i + 1] - d.depth[i];
    p.d_dt = upload(dt.data(), dt.size(), tot);
  } else {
    p.d_kline = upload(d.k_line, (size_t)p.n_s, tot);
    p.stencil.resize(p.n_omega);
    const double dz = 1.0 / (p.nz - 1);
    for (int o = 0; o < p.n_omega; ++o) {
      const double mu = p.tab.mu_o[o];
      const double path = dz / std::fabs(mu);
      const double sx = -p.tab.om_x[o] * path * p.nx;
      const double sy = -p.tab.om_y[o] * path * p.ny;
      const double fx = std::floor(sx), fy = std::floor(sy);
      BoxStencil s{};
      s.i0 = (int)(((long long)fx % p.nx + p.nx) % p.nx);
      s.j0 = (int)(((long long)fy % p.ny + p.ny) % p.ny);
      s.tx = sx - fx;
      s.ty = sy - fy;
      s.path = path;
      s.w00 = (1.0 - s.ty) * (1.0 - s.tx);
      s.w01 = (1.0 - s.ty) * s.tx;
      s.w10 = s.ty * (1.0 - s.tx);
      s.w11 = s.ty * s.tx;
      s.hpath = 0.5 * path;
      s.up = mu > 0 ? 1 : 0;
      const double dx = p.tab.om_x[o] * path * p.nx;
      const double dy = p.tab.om_y[o] * path * p.ny;
      const double gx = std::floor(dx), gy = std::floor(dy);
      s.di0 = (int)(((long long)gx % p.nx + p.nx) % p.nx);
      s.dj0 = (int)(((long long)gy % p.ny + p.ny) % p.ny);
      s.dtx = dx - gx;
      s.dty = dy - gy;
      p.stencil[o] = s;
    }
    p.d_stencil = upload(p.stencil.data(), p.stencil.size(), tot);
  }
  p.bytes_problem = tot;
}

void operator_apply(Problem& p, int precision, const void* x, void* y, const double* xscale,
                    hipStream_t st, gemm::TileDots* dots) {
  const size_t n = (size_t)p.n;
  switch (precision) {
    case RT_PREC_FP64: {
      double* L = static_cast<double*>(problem_lbuf(p, n * sizeof(double)));
      launch_lambda<double, double>(p, static_cast<const double*>(x), L, false, xscale, st);
      apply_sigma_f64(p, L, static_cast<const double*>(x), static_cast<double*>(y), xscale, -1.0,
                      st, dots);
      break;
    }
    case RT_PREC_FP32: {
      float* L = static_cast<float*>(problem_lbuf(p, n * sizeof(float)));
      launch_lambda<float, float>(p, static_cast<const float*>(x), L, false, xscale, st);
      apply_sigma_f32(p, L, static_cast<const float*>(x), static_cast<float*>(y), xscale, -1.0,
                      st, dots);
      break;
    }
    case RT_PREC_BF16:
    case RT_PREC_FP16:
    case RT_PREC_BF16X3: {
      require_one_kernel(p, "a 16-bit operator");
      uint16_t* L = problem_l16(p, st);
      uint16_t* Llo = precision == RT_PREC_BF16X3 ? L + l16_part_elems(p) : nullptr;
      launch_lambda_k4(p, precision, static_cast<const float*>(x), L, Llo, xscale, st);
      launch_sigma_b16(p, precision, L, Llo, static_cast<const float*>(x), static_cast<float*>(y),
                       xscale, -1.0, st, dots);
      break;
    }
    default:
      fail(RT_E_INVALID, "unknown precision");
  }
}

void operator_apply_k(Problem& p, int precision, const void* x, void* y, const double* xscale,
                      hipStream_t st, gemm::TileDots* dots) {
  const size_t n = (size_t)p.n;
  switch (precision) {
    case RT_PREC_FP64: {
      double* L = static_cast<double*>(problem_lbuf(p, n * sizeof(double)));
      launch_lambda<double, double>(p, static_cast<const double*>(x), L, false, xscale, st);
      apply_sigma_f64(p, L, nullptr, static_cast<double*>(y), xscale, +1.0, st, dots);
      break;
    }
    case RT_PREC_FP32: {
      float* L = static_cast<float*>(problem_lbuf(p, n * sizeof(float)));
      launch_lambda<float, float>(p, static_cast<const float*>(x), L, false, xscale, st);
      apply_sigma_f32(p, L, nullptr, static_cast<float*>(y), xscale, +1.0, st, dots);
      break;
    }
    case RT_PREC_BF16:
    case RT_PREC_FP16:
    case RT_PREC_BF16X3: {
      require_one_kernel(p, "a 16-bit operator");
      uint16_t* L = problem_l16(p, st);
      uint16_t* Llo = precision == RT_PREC_BF16X3 ? L + l16_part_elems(p) : nullptr;
      launch_lambda_k4(p, precision, static_cast<const float*>(x), L, Llo, xscale, st);
      launch_sigma_b16(p, precision, L, Llo, nullptr, static_cast<float*>(y), xscale, +1.0, st,
                       dots);
      break;
    }
    default:
      fail(RT_E_INVALID, "unknown precision");
  }
}

void operator_apply_kx(Problem& p, int precision, const void* u, const void* nd, void* y,
                       const double* xscale, hipStream_t st) {
  const size_t n = (size_t)p.n;
  const bool fused = precond_fused(p, precision);
  if (!fused && !nd) fail(RT_E_INVALID, "operator_apply_kx: v - u missing");
  switch (precision) {
    case RT_PREC_FP64: {
      double* L = static_cast<double*>(problem_lbuf(p, n * sizeof(double)));
      launch_lambda<double, double>(p, static_cast<const double*>(u), L, false, xscale, st);
      if (fused)
        launch_sigma_factored_pre_f64(
            p, L, precond_modes_F<double>(p), precond_modes_z<double>(p), p.prec_rq,
            static_cast<double*>(y), static_cast<double*>(problem_fwork(p, sizeof(double))),
            xscale, st);
      else
        apply_sigma_f64(p, L, static_cast<const double*>(nd), static_cast<double*>(y), xscale,
                        +1.0, st, nullptr);
      break;
    }
    case RT_PREC_FP32: {
      float* L = static_cast<float*>(problem_lbuf(p, n * sizeof(float)));
      launch_lambda<float, float>(p, static_cast<const float*>(u), L, false, xscale, st);
      if (fused)
        launch_sigma_factored_pre_f32(
            p, L, precond_modes_F<float>(p), precond_modes_z<float>(p), p.prec_rq,
            static_cast<float*>(y), static_cast<float*>(problem_fwork(p, sizeof(float))), xscale,
            st);
      else
        apply_sigma_f32(p, L, static_cast<const float*>(nd), static_cast<float*>(y), xscale,
                        +1.0, st, nullptr);
      break;
    }
    case RT_PREC_BF16:
    case RT_PREC_FP16:
    case RT_PREC_BF16X3: {
      require_one_kernel(p, "a 16-bit operator");
      uint16_t* L = problem_l16(p, st);
      uint16_t* Llo = precision == RT_PREC_BF16X3 ? L + l16_part_elems(p) : nullptr;
      launch_lambda_k4(p, precision, static_cast<const float*>(u), L, Llo, xscale, st);
      launch_sigma_b16(p, precision, L, Llo, static_cast<const float*>(nd),
                       static_cast<float*>(y), xscale, +1.0, st, nullptr);
      break;
    }
    default:
      fail(RT_E_INVALID, "unknown precision");
  }
}

void operator_apply_kxh(Problem& p, const float* u, _Float16* y, const double* xscale,
                        float ymul, hipStream_t st) {
  if (!precond_fused(p, RT_PREC_FP32))
    fail(RT_E_INVALID, "an fp16 basis with FP32 operators needs the factored scattering");
  const size_t n = (size_t)p.n;
  float* L = static_cast<float*>(problem_lbuf(p, n * sizeof(float)));
  launch_lambda<float, float>(p, u, L, false, xscale, st);
  launch_sigma_factored_pre_h(p, L, precond_modes_F<float>(p), precond_modes_z<float>(p),
                              p.prec_rq, y, ymul,
                              static_cast<float*>(problem_fwork(p, sizeof(float))), xscale, st);
}

void operator_apply_h(Problem& p, int precision, const _Float16* x, _Float16* y,
                      const double* xscale, float ymul, hipStream_t st, bool kform) {
  if (precision != RT_PREC_BF16 && precision != RT_PREC_FP16 && precision != RT_PREC_BF16X3)
    fail(RT_E_INVALID, "an fp16 basis needs a 16-bit operator precision");
  require_one_kernel(p, "a 16-bit operator");
  uint16_t* L = problem_l16(p, st);
  uint16_t* Llo = precision == RT_PREC_BF16X3 ? L + l16_part_elems(p) : nullptr;
  launch_lambda_k4(p, precision, x, L, Llo, xscale, st);
  if (kform)
    launch_sigma_b16_h(p, precision, L, Llo, nullptr, y, ymul, xscale, +1.0, st);
  else
    launch_sigma_b16_h(p, precision, L, Llo, x, y, ymul, xscale, -1.0, st);
}

const double* physical_rhs(Problem& p, hipStream_t st) {
  const size_t n = (size_t)p.n;
  if (!p.d_rhs) RT_HIP(hipMalloc(&p.d_rhs, n * sizeof(double)));
  double* L = static_cast<double*>(problem_lbuf(p, n * sizeof(double)));
  RT_HIP(hipMemsetAsync(p.d_rhs, 0, n * sizeof(double), st));
  launch_lambda<double, double>(p, p.d_rhs, L, true, nullptr, st);
  apply_sigma_f64(p, L, p.d_thermal, p.d_rhs, nullptr, +1.0, st);
  return p.d_rhs;
}

}  // namespace rtsn

using namespace rtsn;

namespace {

template <typename F>
rt_status guarded(F&& f) {
  try {
    f();
    return RT_OK;
  } catch (const RtError& e) {
    g_last_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return RT_E_NOMEM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return RT_E_DEVICE;
  } catch (...) {
    g_last_error = "unknown error";
    return RT_E_DEVICE;
  }
}

Problem* as_problem(rt_problem p) {
  if (!p) fail(RT_E_INVALID, "null problem handle");
  Problem* q = reinterpret_cast<Problem*>(p);
  RT_HIP(hipSetDevice(q->device));
  return q;
}

void check_prec(int prec) {
  if (prec < RT_PREC_FP64 || prec > RT_PREC_BF16X3) fail(RT_E_INVALID, "unknown precision");
}

}  // namespace

extern "C" {

const char* rt_last_error(void) { return g_last_error.c_str(); }

const char* rt_gemm16_tile(rt_problem p, int precision) {
  if (!p) return "";
  const Problem* q = reinterpret_cast<const Problem*>(p);
  const int mode = precision == RT_PREC_BF16 ? 0 : precision == RT_PREC_FP16 ? 1
                   : precision == RT_PREC_BF16X3 ? 2 : -1;
  if (mode < 0) return "";
  return gemm16_config_name(q->g16_cfg[mode]);
}

int rt_version(void) { return RTSN_VERSION; }

rt_status rt_problem_create(const rt_problem_desc* desc, int device, rt_problem* out) {
  if (out) *out = nullptr;
  return guarded([&] {
    if (!desc || !out) fail(RT_E_INVALID, "null argument");
    int ndev = 0;
    RT_HIP(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) fail(RT_E_INVALID, "bad device index");
    std::shared_lock<std::shared_mutex> lk(capture_mutex());
    RT_HIP(hipSetDevice(device));
    Problem* p = new Problem();
    p->device = device;
    try {
      problem_build(*p, *desc);
    } catch (...) {
      delete p;
      throw;
    }
    *out = reinterpret_cast<rt_problem>(p);
  });
}

rt_status rt_problem_destroy(rt_problem p) {
  return guarded([&] {
    if (!p) return;
    Problem* q = reinterpret_cast<Problem*>(p);
    std::shared_lock<std::shared_mutex> lk(capture_mutex());
    RT_HIP(hipSetDevice(q->device));
    RT_HIP(hipDeviceSynchronize());
    delete q;
  });
}

rt_status rt_problem_footprint(rt_problem p, int restart, rt_problem_info* info) {
  return guarded([&] {
    Problem* q = as_problem(p);
    if (!info) fail(RT_E_INVALID, "null info");
    if (restart < 1 || restart > kMaxRestart) fail(RT_E_INVALID, "restart out of range");
    info->n_unknowns = q->n;
    info->n_rays = q->n_r;
    info->n_points = q->n_s;
    info->bytes_problem = q->bytes_problem;
    // the scattering form's work buffer, allocated by the first FP64 (or
    // FP32 factored) application of a solve
    int64_t form_work = 0;
    if (q->sigma_form == RT_SIGMA_OZAKI) form_work = (int64_t)ozaki_work_bytes(*q);
    if (q->sigma_form == RT_SIGMA_FACTORED)
      form_work = (int64_t)(factored_work_elems(*q) * sizeof(double));
    info->bytes_solve_fp64 = (int64_t)workspace_bytes(*q, restart, false, false) +
                             (int64_t)(q->n * sizeof(double)) + form_work;
    info->bytes_solve_mixed = (int64_t)workspace_bytes(*q, restart, true, false) +
                              (int64_t)(q->n * sizeof(double)) + form_work;
    info->sigma_rank = q->n_classes > 1 ? 0 : q->tab.frank;
    info->sigma_form = q->sigma_form;
  });
}

rt_status rt_problem_tables(rt_problem p, double* mhat, double* mu_ray, double* w_ray,
                            double* phi_ray) {
  return guarded([&] {
    Problem* q = as_problem(p);
    const size_t nr = (size_t)q->n_r;
    if (mhat) std::memcpy(mhat, q->tab.mhat.data(), nr * nr * sizeof(double));
    if (mu_ray) std::memcpy(mu_ray, q->tab.mu_ray.data(), nr * sizeof(double));
    if (w_ray) std::memcpy(w_ray, q->tab.w_ray.data(), nr * sizeof(double));
    if (phi_ray) std::memcpy(phi_ray, q->tab.phi_ray.data(), nr * sizeof(double));
  });
}

rt_status rt_apply_lambda(rt_problem p, int precision, const void* s, void* I, int with_bc,
                          const double* scale, void* stream) {
  return guarded([&] {
    Problem* q = as_problem(p);
    check_prec(precision);
    if (!s || !I) fail(RT_E_INVALID, "null vector");
    if (s == I) fail(RT_E_INVALID, "I must not alias s");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (precision == RT_PREC_FP64)
      launch_lambda<double, double>(*q, static_cast<const double*>(s), static_cast<double*>(I),
                                    with_bc != 0, scale, st);
    else
      launch_lambda<float, float>(*q, static_cast<const float*>(s), static_cast<float*>(I),
                                  with_bc != 0, scale, st);
  });
}

rt_status rt_apply_sigma(rt_problem p, int precision, const void* L, const void* x, void* y,
                         void* stream) {
  return guarded([&] {
    Problem* q = as_problem(p);
    check_prec(precision);
    if (!L || !y) fail(RT_E_INVALID, "null vector");
    if (L == y) fail(RT_E_INVALID, "y must not alias L");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const double sign = x ? -1.0 : +1.0;
    if (precision == RT_PREC_FP64) {
      apply_sigma_f64(*q, static_cast<const double*>(L), static_cast<const double*>(x),
                       static_cast<double*>(y), nullptr, sign, st);
    } else if (precision == RT_PREC_FP32) {
      apply_sigma_f32(*q, static_cast<const float*>(L), static_cast<const float*>(x),
                       static_cast<float*>(y), nullptr, sign, st);
    } else {
      // 16-bit operand paths take an FP32 L and round it like the operator does
      require_one_kernel(*q, "a 16-bit operator");
      uint16_t* lb = problem_l16(*q, st);
      uint16_t* lo = precision == RT_PREC_BF16X3 ? lb + l16_part_elems(*q) : nullptr;
      convert_to_k4(*q, precision, static_cast<const float*>(L), lb, lo, st);
      launch_sigma_b16(*q, precision, lb, lo, static_cast<const float*>(x), static_cast<float*>(y),
                       nullptr, sign, st);
    }
  });
}

rt_status rt_apply_operator(rt_problem p, int precision, const void* x, void* y, void* stream) {
  return guarded([&] {
    Problem* q = as_problem(p);
    check_prec(precision);
    if (!x || !y) fail(RT_E_INVALID, "null vector");
    if (x == y) fail(RT_E_INVALID, "y must not alias x");
    operator_apply(*q, precision, x, y, nullptr, static_cast<hipStream_t>(stream));
  });
}

rt_status rt_apply_operator_noalloc(rt_problem p, int precision, const void* x, void* y,
                                    void* stream) {
  return guarded([&] {
    Problem* q = as_problem(p);
    check_prec(precision);
    if (!x || !y) fail(RT_E_INVALID, "null vector");
    if (x == y) fail(RT_E_INVALID, "y must not alias x");
    operator_apply_noalloc(*q, precision, x, y, static_cast<hipStream_t>(stream));
  });
}

rt_status rt_problem_set_sigma(rt_problem p, int form) {
  return guarded([&] {
    Problem* q = as_problem(p);
    if (form != RT_SIGMA_DENSE && form != RT_SIGMA_FACTORED && form != RT_SIGMA_OZAKI)
      fail(RT_E_INVALID, "unknown scattering form");
    if (form == RT_SIGMA_OZAKI) {
      require_one_kernel(*q, "the emulated FP64 scattering GEMM");
      ozaki_prepare(*q);
    }
    if (form == RT_SIGMA_FACTORED) {
      require_one_kernel(*q, "the factored scattering form");
      if (q->tab.frank == 0)
        fail(RT_E_INVALID, "the factored scattering form needs the dipole x PRD kernel");
      if (!factored_fits(*q, sizeof(double)))
        fail(RT_E_INVALID, "too many frequencies for the factored scattering form");
    }
    // the physical right-hand side is rebuilt in the new form; the other
    // forms' work buffers are released
    RT_HIP(hipDeviceSynchronize());
    hipFree(q->d_rhs);
    q->d_rhs = nullptr;
    if (form != RT_SIGMA_OZAKI && q->d_ozwork) {
      hipFree(q->d_ozwork);
      q->d_ozwork = nullptr;
      q->ozwork_bytes = 0;
    }
    if (form != RT_SIGMA_FACTORED && q->d_fwork) {
      hipFree(q->d_fwork);
      q->d_fwork = nullptr;
      q->fwork_bytes = 0;
    }
    q->sigma_form = form;
  });
}

rt_status rt_rhs(rt_problem p, double* b, void* stream) {
  return guarded([&] {
    Problem* q = as_problem(p);
    if (!b) fail(RT_E_INVALID, "null vector");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const double* r = physical_rhs(*q, st);
    RT_HIP(hipMemcpyAsync(b, r, (size_t)q->n * sizeof(double), hipMemcpyDeviceToDevice, st));
  });
}

rt_status rt_intensity(rt_problem p, const double* s, double* I, void* stream) {
  return guarded([&] {
    Problem* q = as_problem(p);
    if (!s || !I) fail(RT_E_INVALID, "null vector");
    if (s == I) fail(RT_E_INVALID, "I must not alias s");
    launch_lambda<double, double>(*q, s, I, true, nullptr, static_cast<hipStream_t>(stream));
  });
}

rt_status rt_apply_precond(rt_problem p, int precision, const void* x, void* y, void* stream) {
  return guarded([&] {
    Problem* q = as_problem(p);
    if (precision != RT_PREC_FP64 && precision != RT_PREC_FP32)
      fail(RT_E_INVALID, "the preconditioner applies to FP64 or FP32 vectors");
    if (!x || !y) fail(RT_E_INVALID, "null vector");
    if (x == y) fail(RT_E_INVALID, "y must not alias x");
    hipStream_t st = static_cast<hipStream_t>(stream);
    precond_prepare(*q, precision == RT_PREC_FP64 ? 8 : 4, st);
    if (precision == RT_PREC_FP64) {
      double* nd = precond_nd<double>(*q);
      precond_apply<double>(*q, static_cast<const double*>(x), static_cast<double*>(y), nd, st);
    } else {
      float* nd = precond_nd<float>(*q);
      precond_apply<float>(*q, static_cast<const float*>(x), static_cast<float*>(y), nd, st);
    }
  });
}

rt_status rt_precond_local(rt_problem p, double* dbar) {
  return guarded([&] {
    Problem* q = as_problem(p);
    if (!dbar) fail(RT_E_INVALID, "null output");
    precond_prepare_local(*q, nullptr);
    RT_HIP(hipMemcpy(dbar, q->d_prec_dbar, (size_t)q->n_nu * q->n_s * sizeof(double),
                     hipMemcpyDeviceToHost));
  });
}

void rt_solver_opts_default(rt_solver_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->krylov = RT_KRYLOV_GMRES;
  o->restart = 30;
  o->max_iters = 10000;
  o->rtol = 1e-8;
  o->precision = RT_PREC_FP64;
  o->inner_rtol = 1e-3;
  o->max_outer = 50;
  o->record_history = 1;
  o->two_step = 1;
}

rt_status rt_solve(rt_problem p, const rt_solver_opts* opts, const double* b, double* x,
                   int x_is_guess, rt_solve_stats* stats, void* stream) {
  rt_status status = RT_OK;
  rt_status g = guarded([&] {
    Problem* q = as_problem(p);
    if (!x) fail(RT_E_INVALID, "null solution vector");
    rt_solver_opts o;
    if (opts) o = *opts; else rt_solver_opts_default(&o);
    if (o.krylov != RT_KRYLOV_GMRES && o.krylov != RT_KRYLOV_BICGSTAB)
      fail(RT_E_INVALID, "unknown Krylov method");
    if (o.restart < 1 || o.restart > kMaxRestart) fail(RT_E_INVALID, "restart out of range");
    if (o.max_iters < 0) fail(RT_E_INVALID, "max_iters must be >= 0");
    if (!(o.rtol > 0) || !std::isfinite(o.rtol)) fail(RT_E_INVALID, "rtol must be > 0");
    check_prec(o.precision);
    if (o.precision != RT_PREC_FP64 && !(o.inner_rtol > 0 && o.inner_rtol < 1))
      fail(RT_E_INVALID, "inner_rtol must be in (0, 1)");
    if (o.max_outer < 1) o.max_outer = 1;
    if (o.precond != RT_PRECOND_NONE && o.precond != RT_PRECOND_LOCAL)
      fail(RT_E_INVALID, "unknown preconditioner");
    // an fp16 basis: 16-bit operators without the preconditioner, or the
    // preconditioned FP32 operator with factored scattering
    const bool b16_pre = o.precision == RT_PREC_FP32 && o.precond == RT_PRECOND_LOCAL &&
                         precond_fused(*q, RT_PREC_FP32);
    if (o.basis_fp16 && o.precision != RT_PREC_BF16 && o.precision != RT_PREC_FP16 &&
        o.precision != RT_PREC_BF16X3 && !b16_pre)
      fail(RT_E_INVALID,
           "basis_fp16 needs a 16-bit operator precision, or FP32 with the preconditioner and "
           "factored scattering");
    if (o.basis_fp16 && q->scatter_inf > 2.0)
      fail(RT_E_INVALID, "basis_fp16 needs max row sum of |(1-eps) Mhat| <= 2");
    if (o.precond && o.krylov != RT_KRYLOV_GMRES)
      fail(RT_E_INVALID, "the preconditioner is a GMRES option");
    if (o.precond && o.basis_fp16 && !b16_pre)
      fail(RT_E_INVALID,
           "the preconditioner on an fp16 basis needs FP32 operators with factored scattering");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const double* bb = b ? b : physical_rhs(*q, st);
    status = solve(*q, o, bb, x, x_is_guess, stats, st);
  });
  return g != RT_OK ? g : status;
}

}  // extern "C"
