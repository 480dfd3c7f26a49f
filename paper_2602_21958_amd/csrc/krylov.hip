// Krylov building blocks on gfx950: Arnoldi (classical Gram-Schmidt) dots
// and update, Givens rotations of the Hessenberg column, cycle-end update,
// residuals and BiCGStab vector updates.
//
// The paper solves the system with restarted GMRES (Sec. 5.3: restart 30)
// and BiCGStab (Sec. 5 set-up).  Here every vector pass streams HBM once:
//  * mdot:   h_i = s_i <W_i, w> for all i <= j in one pass over w (basis
//            vectors stored unnormalised, W_i = v_i / s_i, with the scale s_i
//            kept on the device so no separate normalisation pass is needed);
//  * update: w -= sum_i (h_i s_i) W_i and ||w||^2 in one pass;
//  * givens: one workgroup turns the new Hessenberg column into a column of
//            R, updates g and writes |g_{j+1}| and 1/h_{j+1,j} on the device.
// Reductions are deterministic: a fixed grid writes per-block partial sums
// that one workgroup adds in a fixed order; accumulation is in FP64 for
// FP32 and FP64 vectors alike.
#include "rt_internal.h"
#include "krylov.h"

namespace rtsn {

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Block-reduce G accumulators; result valid in thread 0 for each g, written
// to out[g * stride].
template <int G>
__device__ __forceinline__ void block_reduce_store(double (&acc)[G], double* out, int stride,
                                                   int count) {
  __shared__ double red[G][kThreads / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int g = 0; g < G; ++g) {
    double v = wave_sum(acc[g]);
    if (lane == 0) red[g][wave] = v;
  }
  __syncthreads();
  if (threadIdx.x < G && threadIdx.x < count) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) s += red[threadIdx.x][w];
    out[(size_t)threadIdx.x * stride] = s;
  }
  __syncthreads();
}

// 16-byte vector of a basis element type (clang vector types: arrays of
// them stay in registers)
template <typename TV> struct Vec16;
template <> struct Vec16<double> {
  typedef double type __attribute__((ext_vector_type(2)));
  static constexpr int n = 2;
  static __device__ __forceinline__ double dot(type a, type b) { return a.x * b.x + a.y * b.y; }
};
template <> struct Vec16<float> {
  typedef float type __attribute__((ext_vector_type(4)));
  static constexpr int n = 4;
  static __device__ __forceinline__ double dot(type a, type b) {
    return (double)a.x * b.x + (double)a.y * b.y + (double)a.z * b.z + (double)a.w * b.w;
  }
};

// fp16 basis (stored scaled so that its entries are of order one): products
// of two halves are exact in FP32, so a 16-byte group is summed in FP32
template <> struct Vec16<_Float16> {
  typedef _Float16 type __attribute__((ext_vector_type(8)));
  static constexpr int n = 8;
  static __device__ __forceinline__ double dot(type a, type b) {
    float s = 0.f;
#pragma unroll
    for (int q = 0; q < 8; ++q) s += (float)a[q] * (float)b[q];
    return (double)s;
  }
};

// Arithmetic type of the Gram-Schmidt update: FP64 for FP64 / FP32 vectors,
// FP32 for the fp16 basis (whose own rounding is 2^-11)
template <typename TV> struct UpdAcc { using type = double; };
template <> struct UpdAcc<_Float16> { using type = float; };

// W-wide vector of the element type of x in the cycle-end update
template <typename T, int W> struct VecN {
  typedef T type __attribute__((ext_vector_type(W)));
};

// Contiguous range [b0, b1) of n items owned by this block: every pass
// streams each vector in long sequential runs per block.
__device__ __forceinline__ void block_range(int64_t n, int64_t& b0, int64_t& b1) {
  const int64_t per = (n + gridDim.x - 1) / gridDim.x;
  b0 = (int64_t)blockIdx.x * per;
  b1 = b0 + per < n ? b0 + per : n;
}

// partial[i * nb + b] = sum over block b's range of W_i[e] * w[e].  Each block
// streams one contiguous range of every vector (16-byte loads when the vector
// length keeps them aligned); this keeps each DRAM stream sequential.
template <typename TV, int G>
__global__ __launch_bounds__(kThreads) void mdot_kernel(const TV* __restrict__ V, int64_t n,
                                                        int i0, int cnt,
                                                        const TV* __restrict__ w,
                                                        double* __restrict__ partial) {
  using VT = typename Vec16<TV>::type;
  constexpr int W = Vec16<TV>::n;
  double acc[G];
#pragma unroll
  for (int g = 0; g < G; ++g) acc[g] = 0.0;
  if (n % W == 0) {
    // vector starts are 16-byte aligned: stream with 16-byte loads
    int64_t b0, b1;
    block_range(n / W, b0, b1);
    const VT* wv = reinterpret_cast<const VT*>(w);
    for (int64_t e = b0 + threadIdx.x; e < b1; e += kThreads) {
      const VT x = wv[e];
#pragma unroll
      for (int g = 0; g < G; ++g)
        if (g < cnt)
          acc[g] += Vec16<TV>::dot(reinterpret_cast<const VT*>(V + (size_t)(i0 + g) * n)[e], x);
    }
  } else {
    int64_t b0, b1;
    block_range(n, b0, b1);
    for (int64_t e = b0 + threadIdx.x; e < b1; e += kThreads) {
      const double x = (double)w[e];
#pragma unroll
      for (int g = 0; g < G; ++g)
        if (g < cnt) acc[g] += (double)V[(size_t)(i0 + g) * n + e] * x;
    }
  }
  block_reduce_store<G>(acc, partial + (size_t)i0 * gridDim.x + blockIdx.x, gridDim.x, cnt);
}

// out[i] = scale_i * sum_b partial[i * nb + b]   (one wave per i)
__global__ __launch_bounds__(kThreads) void reduce_rows_kernel(const double* __restrict__ partial,
                                                               int nb, int nrows,
                                                               const double* __restrict__ scale,
                                                               double* __restrict__ out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int i = wave; i < nrows; i += kThreads / 64) {
    double s = 0.0;
    for (int b = lane; b < nb; b += 64) s += partial[(size_t)i * nb + b];
    s = wave_sum(s);
    if (lane == 0) out[i] = scale ? scale[i] * s : s;
  }
}

// w -= sum_i coef_i W_i with coef_i = h_i * s_i; partial norm^2 of new w.
// FP64 vectors: one element per thread, grid-stride (measured fastest for
// 8-byte elements: 1.84 ms against 1.92 ms with 16-byte groups per block
// range and 2.00 ms with 16-byte groups grid-stride, box32).  FP32 and fp16
// vectors: 16-byte groups (when the vector length keeps them aligned) over
// one contiguous range per block.  Eight basis loads in flight per thread.
template <typename TV>
__global__ __launch_bounds__(kThreads) void update_kernel(const TV* __restrict__ V, int64_t n,
                                                          int cnt, const double* __restrict__ h,
                                                          const double* __restrict__ vscale,
                                                          TV* __restrict__ w,
                                                          double* __restrict__ partial) {
  using AT = typename UpdAcc<TV>::type;
  __shared__ AT coef[kMaxRestart + 1];
  for (int i = threadIdx.x; i < cnt; i += kThreads) coef[i] = (AT)(h[i] * vscale[i]);
  __syncthreads();
  using VT = typename Vec16<TV>::type;
  constexpr int W = Vec16<TV>::n;
  double nrm = 0.0;
  if constexpr (sizeof(TV) == 8) {
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < n; e += stride) {
      AT v = (AT)w[e];
      int i = 0;
      for (; i + 8 <= cnt; i += 8) {
        AT a[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] = (AT)V[(size_t)(i + u) * n + e];
#pragma unroll
        for (int u = 0; u < 8; ++u) v -= coef[i + u] * a[u];
      }
      for (; i < cnt; ++i) v -= coef[i] * (AT)V[(size_t)i * n + e];
      const TV vs = (TV)v;
      w[e] = vs;
      nrm += (double)vs * (double)vs;
    }
  } else if (n % W == 0) {
    int64_t b0, b1;
    block_range(n / W, b0, b1);
    VT* wv = reinterpret_cast<VT*>(w);
    for (int64_t e = b0 + threadIdx.x; e < b1; e += kThreads) {
      const VT x = wv[e];
      AT v[W];
#pragma unroll
      for (int q = 0; q < W; ++q) v[q] = (AT)x[q];
      int i = 0;
      for (; i + 8 <= cnt; i += 8) {
        VT a[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] = reinterpret_cast<const VT*>(V + (size_t)(i + u) * n)[e];
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
          for (int q = 0; q < W; ++q) v[q] -= coef[i + u] * (AT)a[u][q];
      }
      for (; i < cnt; ++i) {
        const VT a = reinterpret_cast<const VT*>(V + (size_t)i * n)[e];
#pragma unroll
        for (int q = 0; q < W; ++q) v[q] -= coef[i] * (AT)a[q];
      }
      VT r;
#pragma unroll
      for (int q = 0; q < W; ++q) {
        r[q] = (TV)v[q];
        nrm += (double)r[q] * (double)r[q];
      }
      wv[e] = r;
    }
  } else {
    int64_t b0, b1;
    block_range(n, b0, b1);
    for (int64_t e = b0 + threadIdx.x; e < b1; e += kThreads) {
      AT v = (AT)w[e];
      for (int i = 0; i < cnt; ++i) v -= coef[i] * (AT)V[(size_t)i * n + e];
      const TV vs = (TV)v;
      w[e] = vs;
      nrm += (double)vs * (double)vs;
    }
  }
  double a[1] = {nrm};
  block_reduce_store<1>(a, partial + blockIdx.x, 1, 1);
}

// x += sum_i coef_i W_i (coef on device, cnt <= kMaxRestart+1); the same
// access pattern as the update for each basis type.
template <typename TV, typename TX>
__global__ __launch_bounds__(kThreads) void combine_kernel(const TV* __restrict__ V, int64_t n,
                                                           int cnt, const double* __restrict__ coef_d,
                                                           TX* __restrict__ x) {
  __shared__ double coef[kMaxRestart + 1];
  for (int i = threadIdx.x; i < cnt; i += kThreads) coef[i] = coef_d[i];
  __syncthreads();
  using VT = typename Vec16<TV>::type;
  constexpr int W = Vec16<TV>::n;
  using XT = typename VecN<TX, W>::type;
  int64_t b0, b1;
  if constexpr (sizeof(TV) == 8) {
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < n; e += stride) {
      double v = (double)x[e];
      int i = 0;
      for (; i + 8 <= cnt; i += 8) {
        double a[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] = (double)V[(size_t)(i + u) * n + e];
#pragma unroll
        for (int u = 0; u < 8; ++u) v += coef[i + u] * a[u];
      }
      for (; i < cnt; ++i) v += coef[i] * (double)V[(size_t)i * n + e];
      x[e] = (TX)v;
    }
  } else if (n % W == 0) {
    block_range(n / W, b0, b1);
    XT* xv = reinterpret_cast<XT*>(x);
    for (int64_t e = b0 + threadIdx.x; e < b1; e += kThreads) {
      const XT x0 = xv[e];
      double v[W];
#pragma unroll
      for (int q = 0; q < W; ++q) v[q] = (double)x0[q];
      int i = 0;
      for (; i + 8 <= cnt; i += 8) {
        VT a[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] = reinterpret_cast<const VT*>(V + (size_t)(i + u) * n)[e];
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
          for (int q = 0; q < W; ++q) v[q] += coef[i + u] * (double)a[u][q];
      }
      for (; i < cnt; ++i) {
        const VT a = reinterpret_cast<const VT*>(V + (size_t)i * n)[e];
#pragma unroll
        for (int q = 0; q < W; ++q) v[q] += coef[i] * (double)a[q];
      }
      XT r;
#pragma unroll
      for (int q = 0; q < W; ++q) r[q] = (TX)v[q];
      xv[e] = r;
    }
  } else {
    block_range(n, b0, b1);
    for (int64_t e = b0 + threadIdx.x; e < b1; e += kThreads) {
      double v = (double)x[e];
      for (int i = 0; i < cnt; ++i) v += coef[i] * (double)V[(size_t)i * n + e];
      x[e] = (TX)v;
    }
  }
}

// r = b - ax (into r, type TR; r may alias ax), partial norm^2 of r
template <typename TB, typename TA, typename TR>
__global__ __launch_bounds__(kThreads) void residual_kernel(const TB* __restrict__ b,
                                                            const TA* ax, int64_t n, TR* r,
                                                            double* __restrict__ partial) {
  double nrm = 0.0;
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < n; e += stride) {
    const double v = (double)b[e] - (double)ax[e];
    const TR rv = (TR)v;
    r[e] = rv;
    nrm += (double)rv * (double)rv;
  }
  double a[1] = {nrm};
  block_reduce_store<1>(a, partial + blockIdx.x, 1, 1);
}

// partial norm^2 of x (and non-finite flag via NaN propagation)
template <typename T>
__global__ __launch_bounds__(kThreads) void norm_kernel(const T* __restrict__ x, int64_t n,
                                                        double* __restrict__ partial) {
  double nrm = 0.0;
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < n; e += stride) {
    const double v = (double)x[e];
    nrm += v * v;
  }
  double a[1] = {nrm};
  block_reduce_store<1>(a, partial + blockIdx.x, 1, 1);
}

// Sum partial norms: st->beta = sqrt(sum); optionally start a GMRES cycle:
// vscale[0] = 1/beta, g[0] = beta.
__global__ __launch_bounds__(64) void finish_norm_kernel(const double* __restrict__ partial,
                                                         int nb, GmresState* st, int start_cycle) {
  const int lane = threadIdx.x;
  double s = 0.0;
  for (int b = lane; b < nb; b += 64) s += partial[b];
  s = wave_sum(s);
  if (lane == 0) {
    const double beta = sqrt(s);
    st->beta = beta;
    if (start_cycle) {
      st->vscale[0] = beta > 0.0 ? 1.0 / beta : 0.0;
      st->g[0] = beta;
      for (int i = 1; i <= kMaxRestart; ++i) st->g[i] = 0.0;
      st->stop_k = 0;
    }
  }
}

// Givens step j on the Hessenberg column already in R's column j (rows
// 0..j+1; hn = |h_{j+1,j}|, the norm of the new basis vector before
// scaling): rotations, g, 1/hn as the new vector's scale, the residual
// estimate and the stop record.  The first step whose residual estimate is
// <= tol, breaks down or is not finite is recorded in stop_k, with its
// status.
__device__ void givens_step(GmresState* st, int j, double hn, double tol) {
  double* col = st->R + (size_t)j * (kMaxRestart + 1);
  const double raw_diag = col[j];
  for (int i = 0; i < j; ++i) {
    const double t1 = st->cs[i] * col[i] + st->sn[i] * col[i + 1];
    col[i + 1] = -st->sn[i] * col[i] + st->cs[i] * col[i + 1];
    col[i] = t1;
  }
  double c = 1.0, sn = 0.0;
  if (col[j + 1] != 0.0) {
    const double hh = hypot(col[j], col[j + 1]);
    c = col[j] / hh;
    sn = col[j + 1] / hh;
  }
  st->cs[j] = c;
  st->sn[j] = sn;
  col[j] = c * col[j] + sn * col[j + 1];
  col[j + 1] = 0.0;
  st->g[j + 1] = -sn * st->g[j];
  st->g[j] = c * st->g[j];
  const int breakdown = !(hn > 1e-14 * fabs(raw_diag) + 1e-300);
  st->vscale[j + 1] = breakdown ? 0.0 : 1.0 / hn;
  const double resid = fabs(st->g[j + 1]);
  const int nonfinite = !isfinite(hn) || !isfinite(resid);
  st->log[j] = resid;
  if (st->stop_k == 0) {
    st->resid = resid;
    st->breakdown = breakdown;
    st->nonfinite = nonfinite;
    if (resid <= tol || breakdown || nonfinite) st->stop_k = j + 1;
  }
}

// Givens step j: column h[0..j] (already scaled dots), h_{j+1,j} from the
// update's partial norms.
__global__ __launch_bounds__(64) void givens_kernel(const double* __restrict__ partial, int nb,
                                                    GmresState* st, int j, double tol,
                                                    double kdiag) {
  const int lane = threadIdx.x;
  double s = 0.0;
  for (int b = lane; b < nb; b += 64) s += partial[b];
  s = wave_sum(s);
  if (lane != 0) return;
  const double hn = sqrt(s);
  double* col = st->R + (size_t)j * (kMaxRestart + 1);
  if (kdiag != 0.0) {   // c A v_j = c v_j - c K v_j
    for (int i = 0; i <= j; ++i) col[i] = (i == j ? kdiag : 0.0) - st->h[i];
    col[j + 1] = -hn;
  } else {
    for (int i = 0; i <= j; ++i) col[i] = st->h[i];
    col[j + 1] = hn;
  }
  givens_step(st, j, hn, tol);
}

// ------------------------------------------------- two Arnoldi steps at once
// Steps j and j + 1 on K from u1 = K v_j and u2 = K u1 (in basis slots j + 1
// and j + 2), with one pass over the basis for the dots and one for the
// update instead of two each.  With c1 = V^T u1, c2 = V^T u2 (V = v_0..v_j,
// unit vectors), g11 = |u1|^2 and g12 = u1 . u2:
//   P1 = u1 - V c1,            v_{j+1} = P1 / |P1|,
//   nu = (g12 - c1 . c2) / (g11 - |c1|^2)     (the P1 component of u2 - V c2),
//   Z  = u2 - nu u1 - V (c2 - nu c1) = u2 - V c2 - nu P1,   v_{j+2} = Z / |Z|.
// K P1 = u2 - K V c1 = u2 - V p - c1_j P1 with p = t + c1_j c1 and
// t_l = sum_{i<j} c1_i Hk_{l,i} (K's earlier Hessenberg columns), so
//   K v_j     = V c1 + |P1| v_{j+1},
//   K v_{j+1} = V (c2 - p) / |P1| + (nu - c1_j) v_{j+1} + |Z| / |P1| v_{j+2},
// an exact identity whatever rounding nu carries; |P1| and |Z| are the
// norms of the stored vectors, summed by the update pass.  Hk is kept per
// cycle for the t of later pairs.

template <typename TV, int G>
__global__ __launch_bounds__(kThreads) void mdot2_kernel(const TV* __restrict__ V, int64_t n,
                                                         int i0, int cnt,
                                                         const TV* __restrict__ u1,
                                                         const TV* __restrict__ u2,
                                                         double* __restrict__ partial) {
  using VT = typename Vec16<TV>::type;
  constexpr int W = Vec16<TV>::n;
  double a1[G], a2[G];
#pragma unroll
  for (int g = 0; g < G; ++g) a1[g] = a2[g] = 0.0;
  if (n % W == 0) {
    int64_t b0, b1;
    block_range(n / W, b0, b1);
    const VT* x1v = reinterpret_cast<const VT*>(u1);
    const VT* x2v = reinterpret_cast<const VT*>(u2);
    for (int64_t e = b0 + threadIdx.x; e < b1; e += kThreads) {
      const VT x1 = x1v[e], x2 = x2v[e];
#pragma unroll
      for (int g = 0; g < G; ++g)
        if (g < cnt) {
          const VT v = reinterpret_cast<const VT*>(V + (size_t)(i0 + g) * n)[e];
          a1[g] += Vec16<TV>::dot(v, x1);
          a2[g] += Vec16<TV>::dot(v, x2);
        }
    }
  } else {
    int64_t b0, b1;
    block_range(n, b0, b1);
    for (int64_t e = b0 + threadIdx.x; e < b1; e += kThreads) {
      const double x1 = (double)u1[e], x2 = (double)u2[e];
#pragma unroll
      for (int g = 0; g < G; ++g)
        if (g < cnt) {
          const double v = (double)V[(size_t)(i0 + g) * n + e];
          a1[g] += v * x1;
          a2[g] += v * x2;
        }
    }
  }
  block_reduce_store<G>(a1, partial + (size_t)i0 * gridDim.x + blockIdx.x, gridDim.x, cnt);
  block_reduce_store<G>(a2, partial + (size_t)(kPairRows + i0) * gridDim.x + blockIdx.x,
                        gridDim.x, cnt);
}

// pair[] layout: [0] nu, then c1, c2, the update coefficients k1 = c1 s,
// k2 = (c2 - nu c1) s (s: the basis scales), kPairRows each.
constexpr int kPairC1 = 8, kPairC2 = kPairC1 + kPairRows, kPairK1 = kPairC2 + kPairRows,
              kPairK2 = kPairK1 + kPairRows;

__global__ __launch_bounds__(kThreads) void pair_coef_kernel(const double* __restrict__ partial,
                                                             int nb, int j,
                                                             const double* __restrict__ vscale,
                                                             double* __restrict__ pair) {
  __shared__ double c1[kPairRows], c2[kPairRows];
  __shared__ double nu_s;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int q = wave; q <= j + 1; q += kThreads / 64) {
    double s1 = 0.0, s2 = 0.0;
    for (int b = lane; b < nb; b += 64) {
      s1 += partial[(size_t)q * nb + b];
      s2 += partial[(size_t)(kPairRows + q) * nb + b];
    }
    s1 = wave_sum(s1);
    s2 = wave_sum(s2);
    if (lane == 0) {
      const double sc = q <= j ? vscale[q] : 1.0;   // row j + 1: u1 itself
      c1[q] = sc * s1;
      c2[q] = sc * s2;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double n1 = 0.0, d12 = 0.0;
    for (int q = 0; q <= j; ++q) {
      n1 += c1[q] * c1[q];
      d12 += c1[q] * c2[q];
    }
    const double b2 = c1[j + 1] - n1;   // |P1|^2 by Pythagoras (only for nu)
    const double nu = b2 > 0.0 ? (c2[j + 1] - d12) / b2 : 0.0;
    nu_s = nu;
    pair[0] = nu;
  }
  __syncthreads();
  const double nu = nu_s;
  for (int q = threadIdx.x; q <= j; q += kThreads) {
    pair[kPairC1 + q] = c1[q];
    pair[kPairC2 + q] = c2[q];
    pair[kPairK1 + q] = c1[q] * vscale[q];
    pair[kPairK2 + q] = (c2[q] - nu * c1[q]) * vscale[q];
  }
}

// u1 <- P1 = u1 - sum k1_q W_q, u2 <- Z = u2 - nu u1 - sum k2_q W_q in one
// pass over W_0..W_j; partial[b] = block b's |P1|^2, partial[nb + b] its
// |Z|^2, partial[2 nb + b] its P1 . Z (norms of the stored, rounded values).
// FP64: one element per thread, grid-stride, eight basis loads in flight;
// FP32: 16-byte groups over one contiguous range per block, FP64
// accumulation (the one-step update's access pattern for each type).
template <typename TV>
__global__ __launch_bounds__(kThreads) void update2_kernel(const TV* __restrict__ V,
                                                           int64_t n, int cnt,
                                                           const double* __restrict__ pair,
                                                           TV* __restrict__ u1,
                                                           TV* __restrict__ u2,
                                                           double* __restrict__ partial) {
  __shared__ double k1[kMaxRestart + 1], k2[kMaxRestart + 1];
  for (int i = threadIdx.x; i < cnt; i += kThreads) {
    k1[i] = pair[kPairK1 + i];
    k2[i] = pair[kPairK2 + i];
  }
  __syncthreads();
  const double nu = pair[0];
  double n1 = 0.0, nz = 0.0, pz = 0.0;
  auto finish = [&](double a, double b, double s1, double s2, TV& o1, TV& o2) {
    o1 = (TV)(a - s1);
    o2 = (TV)((b - nu * a) - s2);
    const double p1 = (double)o1, z = (double)o2;
    n1 += p1 * p1;
    nz += z * z;
    pz += p1 * z;
  };
  using VT = typename Vec16<TV>::type;
  constexpr int W = Vec16<TV>::n;
  if constexpr (sizeof(TV) == 8) {
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < n; e += stride) {
      double s1 = 0.0, s2 = 0.0;
      int i = 0;
      for (; i + 8 <= cnt; i += 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = V[(size_t)(i + u) * n + e];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          s1 += k1[i + u] * v[u];
          s2 += k2[i + u] * v[u];
        }
      }
      for (; i < cnt; ++i) {
        const double v = V[(size_t)i * n + e];
        s1 += k1[i] * v;
        s2 += k2[i] * v;
      }
      finish((double)u1[e], (double)u2[e], s1, s2, u1[e], u2[e]);
    }
  } else if (n % W == 0) {
    int64_t b0, b1;
    block_range(n / W, b0, b1);
    VT* x1v = reinterpret_cast<VT*>(u1);
    VT* x2v = reinterpret_cast<VT*>(u2);
    for (int64_t e = b0 + threadIdx.x; e < b1; e += kThreads) {
      const VT x1 = x1v[e], x2 = x2v[e];
      double s1[W], s2[W];
#pragma unroll
      for (int q = 0; q < W; ++q) s1[q] = s2[q] = 0.0;
      int i = 0;
      for (; i + 8 <= cnt; i += 8) {
        VT a[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] = reinterpret_cast<const VT*>(V + (size_t)(i + u) * n)[e];
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
          for (int q = 0; q < W; ++q) {
            s1[q] += k1[i + u] * (double)a[u][q];
            s2[q] += k2[i + u] * (double)a[u][q];
          }
      }
      for (; i < cnt; ++i) {
        const VT a = reinterpret_cast<const VT*>(V + (size_t)i * n)[e];
#pragma unroll
        for (int q = 0; q < W; ++q) {
          s1[q] += k1[i] * (double)a[q];
          s2[q] += k2[i] * (double)a[q];
        }
      }
      VT r1, r2;
#pragma unroll
      for (int q = 0; q < W; ++q) {
        TV o1, o2;
        finish((double)x1[q], (double)x2[q], s1[q], s2[q], o1, o2);
        r1[q] = o1;
        r2[q] = o2;
      }
      x1v[e] = r1;
      x2v[e] = r2;
    }
  } else {
    int64_t b0, b1;
    block_range(n, b0, b1);
    for (int64_t e = b0 + threadIdx.x; e < b1; e += kThreads) {
      double s1 = 0.0, s2 = 0.0;
      for (int i = 0; i < cnt; ++i) {
        const double v = (double)V[(size_t)i * n + e];
        s1 += k1[i] * v;
        s2 += k2[i] * v;
      }
      finish((double)u1[e], (double)u2[e], s1, s2, u1[e], u2[e]);
    }
  }
  double acc[3] = {n1, nz, pz};
  block_reduce_store<3>(acc, partial + blockIdx.x, gridDim.x, 3);
}

// rho = (P1 . Z) / |P1|^2 from the update's sums into pair[1]: nu carries the
// rounding of |u1|^2 - |c1|^2, and Z then keeps a P1 component that one-step
// Gram-Schmidt would not leave (in NumPy on the 8^3 test box: orthogonality
// 1e-4 against 3e-9 once it is removed).
__global__ __launch_bounds__(64) void pair_rho_kernel(const double* __restrict__ partial,
                                                      int nb, double* __restrict__ pair) {
  const int lane = threadIdx.x;
  double a = 0.0, c = 0.0;
  for (int b = lane; b < nb; b += 64) {
    a += partial[b];
    c += partial[2 * nb + b];
  }
  a = wave_sum(a);
  c = wave_sum(c);
  if (lane == 0) pair[1] = a > 0.0 ? c / a : 0.0;
}

// Z <- Z - rho P1 and partial[nb + b] = block b's |Z|^2 afterwards (of the
// stored values).
template <typename TV>
__global__ __launch_bounds__(kThreads) void pair_fix_kernel(const TV* __restrict__ p1,
                                                            TV* __restrict__ z, int64_t n,
                                                            const double* __restrict__ pair,
                                                            double* __restrict__ partial) {
  const double rho = pair[1];
  double nz = 0.0;
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  bool done = false;
  if constexpr (sizeof(TV) == 2) {
    // fp16 basis: 8 values per 16-byte access (basis vectors are n values
    // apart, so 16-byte aligned when n is a multiple of 8)
    using VT = typename Vec16<TV>::type;
    done = n % 8 == 0;
    const VT* pv = reinterpret_cast<const VT*>(p1);
    VT* zv = reinterpret_cast<VT*>(z);
    for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; done && e < n / 8;
         e += stride) {
      const VT a = pv[e];
      VT b = zv[e];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        b[q] = (TV)((double)b[q] - rho * (double)a[q]);
        nz += (double)b[q] * (double)b[q];
      }
      zv[e] = b;
    }
  }
  if (!done) {
    for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < n; e += stride) {
      const TV v = (TV)((double)z[e] - rho * (double)p1[e]);
      z[e] = v;
      nz += (double)v * (double)v;
    }
  }
  double acc[1] = {nz};
  block_reduce_store<1>(acc, partial + gridDim.x + blockIdx.x, 1, 1);
}

// Hessenberg columns j and j + 1 of K (kept in hk, column i at i * kPairRows)
// from the pair's dots and norms, turned into A's (kdiag e_i - h, -h_sub)
// and given to two Givens steps; the second is skipped once the first
// stopped.  sigma: the Arnoldi operator is sigma times the one that made u2
// from u1 (an fp16 basis runs Arnoldi on S K but forms u2 = K u1, which
// keeps u2 at the basis's scale): K v_{j+1} then carries sigma on c2, on
// nu + rho and on |Z|.
__global__ __launch_bounds__(64) void givens2_kernel(const double* __restrict__ partial, int nb,
                                                     GmresState* st, int j, double tol,
                                                     const double* __restrict__ pair,
                                                     double* __restrict__ hk, double kdiag,
                                                     double sigma) {
  const int lane = threadIdx.x;
  double s1 = 0.0, s2 = 0.0;
  for (int b = lane; b < nb; b += 64) {
    s1 += partial[b];
    s2 += partial[nb + b];
  }
  s1 = wave_sum(s1);
  s2 = wave_sum(s2);
  if (lane != 0) return;
  const double np1 = sqrt(s1), nz = sqrt(s2);
  const double nu = pair[0];
  const double* c1 = pair + kPairC1;
  const double* c2 = pair + kPairC2;
  double* h0 = hk + (size_t)j * kPairRows;         // K's column j
  double* h1 = hk + (size_t)(j + 1) * kPairRows;   // K's column j + 1
  for (int i = 0; i <= j; ++i) h0[i] = c1[i];
  h0[j + 1] = np1;
  double* col = st->R + (size_t)j * (kMaxRestart + 1);
  for (int i = 0; i <= j; ++i) col[i] = (i == j ? kdiag : 0.0) - h0[i];
  col[j + 1] = -np1;
  const int stopped_before = st->stop_k != 0;
  givens_step(st, j, np1, tol);
  // p = t + c1_j c1, t_l = sum_{i<j} c1_i hk_{l,i} (column i has rows 0..i+1)
  const double inv = np1 > 0.0 ? 1.0 / np1 : 0.0;
  for (int l = 0; l <= j; ++l) {
    double t = 0.0;
    for (int i = (l > 0 ? l - 1 : 0); i < j; ++i) t += c1[i] * hk[(size_t)i * kPairRows + l];
    h1[l] = (sigma * c2[l] - (t + c1[j] * c1[l])) * inv;
  }
  h1[j + 1] = sigma * (nu + pair[1]) - c1[j];   // Z's P1 part rho moved into the column
  h1[j + 2] = sigma * nz * inv;
  if (!stopped_before && st->stop_k != 0) return;   // the pair's first step ended the cycle
  col = st->R + (size_t)(j + 1) * (kMaxRestart + 1);
  for (int i = 0; i <= j + 1; ++i) col[i] = (i == j + 1 ? kdiag : 0.0) - h1[i];
  col[j + 2] = -h1[j + 2];
  givens_step(st, j + 1, h1[j + 2], tol);
  // v_{j+2} = Z / |Z|: givens_step stored 1 / h_{j+2,j+1} = |P1| / |Z|
  st->vscale[j + 2] = st->vscale[j + 2] == 0.0 ? 0.0 : 1.0 / nz;
}

// Back substitution R y = g (k x k), coef_i = y_i * vscale_i.
__global__ __launch_bounds__(64) void solve_r_kernel(GmresState* st, int k) {
  if (threadIdx.x != 0) return;
  for (int i = k - 1; i >= 0; --i) {
    double v = st->g[i];
    for (int l = i + 1; l < k; ++l) v -= st->R[(size_t)l * (kMaxRestart + 1) + i] * st->y[l];
    st->y[i] = v / st->R[(size_t)i * (kMaxRestart + 1) + i];
  }
  for (int i = 0; i < k; ++i) st->coef[i] = st->y[i] * st->vscale[i];
}

// ------------------------------------------------------------- BiCGStab
// out[c * nb + b] partials of up to 4 dot products <a_c, b_c>
template <typename T>
__global__ __launch_bounds__(kThreads) void dots4_kernel(const T* a0, const T* b0, const T* a1,
                                                         const T* b1, const T* a2, const T* b2,
                                                         const T* a3, const T* b3, int cnt,
                                                         int64_t n, double* __restrict__ partial) {
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < n; e += stride) {
    acc[0] += (double)a0[e] * (double)b0[e];
    if (cnt > 1) acc[1] += (double)a1[e] * (double)b1[e];
    if (cnt > 2) acc[2] += (double)a2[e] * (double)b2[e];
    if (cnt > 3) acc[3] += (double)a3[e] * (double)b3[e];
  }
  block_reduce_store<4>(acc, partial + blockIdx.x, gridDim.x, cnt);
}

// p = r + beta (p - omega v)
template <typename T>
__global__ __launch_bounds__(kThreads) void bicg_p_kernel(const T* __restrict__ r,
                                                          const T* __restrict__ v, T* __restrict__ p,
                                                          int64_t n, const BicgState* st) {
  const double beta = st->beta, omega = st->omega;
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < n; e += stride)
    p[e] = (T)((double)r[e] + beta * ((double)p[e] - omega * (double)v[e]));
}

// s = r - alpha v (written over r), partial ||s||^2
template <typename T>
__global__ __launch_bounds__(kThreads) void bicg_s_kernel(T* __restrict__ r, const T* __restrict__ v,
                                                          int64_t n, const BicgState* st,
                                                          double* __restrict__ partial) {
  const double alpha = st->alpha;
  double nrm = 0.0;
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < n; e += stride) {
    const T s = (T)((double)r[e] - alpha * (double)v[e]);
    r[e] = s;
    nrm += (double)s * (double)s;
  }
  double a[1] = {nrm};
  block_reduce_store<1>(a, partial + blockIdx.x, 1, 1);
}

// x += alpha p + omega s ; r = s - omega t (s stored in r), partial ||r||^2
template <typename T, typename TX>
__global__ __launch_bounds__(kThreads) void bicg_xr_kernel(TX* __restrict__ x,
                                                           const T* __restrict__ p,
                                                           T* __restrict__ r,
                                                           const T* __restrict__ t, int64_t n,
                                                           const BicgState* st, int only_alpha,
                                                           double* __restrict__ partial) {
  const double alpha = st->alpha, omega = only_alpha ? 0.0 : st->omega;
  double nrm = 0.0;
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < n; e += stride) {
    const double s = (double)r[e];
    x[e] = (TX)((double)x[e] + alpha * (double)p[e] + omega * s);
    if (!only_alpha) {
      const T rn = (T)(s - omega * (double)t[e]);
      r[e] = rn;
      nrm += (double)rn * (double)rn;
    }
  }
  double a[1] = {nrm};
  block_reduce_store<1>(a, partial + blockIdx.x, 1, 1);
}

// Scalar stages of BiCGStab on the device.
// stage 0: rho_new = <rhat, r>; beta = (rho_new/rho)(alpha/omega); rho = rho_new
// stage 1: alpha = rho / <rhat, v>
// stage 2: omega = <t, s> / <t, t>
__global__ __launch_bounds__(64) void bicg_scalar_kernel(const double* __restrict__ partial,
                                                         int nb, int stage, BicgState* st) {
  const int lane = threadIdx.x;
  double s0 = 0.0, s1 = 0.0;
  for (int b = lane; b < nb; b += 64) {
    s0 += partial[b];
    if (stage == 2) s1 += partial[nb + b];
  }
  s0 = wave_sum(s0);
  s1 = wave_sum(s1);
  if (lane != 0) return;
  if (stage == 0) {
    const double rho_new = s0;
    st->beta = (st->iter == 0) ? 0.0 : (rho_new / st->rho) * (st->alpha / st->omega);
    st->breakdown = (rho_new == 0.0 || !isfinite(rho_new));
    st->rho = rho_new;
  } else if (stage == 1) {
    st->alpha = (s0 != 0.0) ? st->rho / s0 : 0.0;
    st->breakdown = (s0 == 0.0 || !isfinite(s0));
  } else {
    st->omega = (s1 != 0.0) ? s0 / s1 : 0.0;
    st->breakdown = (s1 == 0.0 || st->omega == 0.0 || !isfinite(st->omega));
  }
}

__global__ __launch_bounds__(64) void finish_norm_simple_kernel(const double* __restrict__ partial,
                                                                int nb, double* out) {
  const int lane = threadIdx.x;
  double s = 0.0;
  for (int b = lane; b < nb; b += 64) s += partial[b];
  s = wave_sum(s);
  if (lane == 0) *out = sqrt(s);
}

template <typename TD> __device__ __forceinline__ TD cvt_from(double v) { return (TD)v; }
template <> __device__ __forceinline__ __hip_bfloat16 cvt_from<__hip_bfloat16>(double v) {
  return __float2bfloat16((float)v);
}
template <> __device__ __forceinline__ __half cvt_from<__half>(double v) {
  return __float2half((float)v);
}

template <typename TS, typename TD>
__global__ __launch_bounds__(kThreads) void convert_kernel(const TS* __restrict__ a,
                                                           TD* __restrict__ b, int64_t n,
                                                           double scale) {
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < n; e += stride)
    b[e] = cvt_from<TD>(scale * (double)a[e]);
}

__global__ __launch_bounds__(kThreads) void axpy_f64_kernel(double* __restrict__ x,
                                                            const float* __restrict__ d, int64_t n,
                                                            const double* __restrict__ scale) {
  const double s = scale ? *scale : 1.0;
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < n; e += stride)
    x[e] += s * (double)d[e];
}

int grid_for(int64_t n) {
  int64_t g = (n + kThreads - 1) / kThreads;
  return (int)(g < kReduceBlocks ? (g < 1 ? 1 : g) : kReduceBlocks);
}

// The update / norm pass streams (j+2) vectors and writes one: a larger grid
// keeps more writes in flight.
int grid_update(int64_t n) {
  int64_t g = (n + kThreads - 1) / kThreads;
  return (int)(g < 2 * kReduceBlocks ? (g < 1 ? 1 : g) : 2 * kReduceBlocks);
}

}  // namespace

// ------------------------------------------------------------------ launchers
template <typename TV>
void k_mdot(const TV* V, int64_t n, int cnt, const TV* w, double* partial, hipStream_t st) {
  const int nb = grid_for(n);
  ProfScope prof(RT_KCLASS_ARNOLDI, st);
  for (int i0 = 0; i0 < cnt; i0 += 16) {
    const int c = cnt - i0 < 16 ? cnt - i0 : 16;
    hipLaunchKernelGGL((mdot_kernel<TV, 16>), dim3(nb), dim3(kThreads), 0, st, V, n, i0, c, w,
                       partial);
  }
  RT_HIP(hipGetLastError());
}

void k_reduce_rows_nb(const double* partial, int nb, int nrows, const double* scale, double* out,
                      hipStream_t st) {
  ProfScope prof(RT_KCLASS_ARNOLDI, st);
  hipLaunchKernelGGL(reduce_rows_kernel, dim3(1), dim3(kThreads), 0, st, partial, nb, nrows,
                     scale, out);
  RT_HIP(hipGetLastError());
}

void k_reduce_rows(const double* partial, int64_t n, int nrows, const double* scale, double* out,
                   hipStream_t st) {
  hipLaunchKernelGGL(reduce_rows_kernel, dim3(1), dim3(kThreads), 0, st, partial, grid_for(n),
                     nrows, scale, out);
  RT_HIP(hipGetLastError());
}

template <typename TV>
void k_update(const TV* V, int64_t n, int cnt, const double* h, const double* vscale, TV* w,
              double* partial, hipStream_t st) {
  ProfScope prof(RT_KCLASS_ARNOLDI, st);
  hipLaunchKernelGGL((update_kernel<TV>), dim3(grid_update(n)), dim3(kThreads), 0, st, V, n, cnt,
                     h, vscale, w, partial);
  RT_HIP(hipGetLastError());
}

template <typename TV, typename TX>
void k_combine(const TV* V, int64_t n, int cnt, const double* coef, TX* x, hipStream_t st) {
  hipLaunchKernelGGL((combine_kernel<TV, TX>), dim3(grid_for(n)), dim3(kThreads), 0, st, V, n,
                     cnt, coef, x);
  RT_HIP(hipGetLastError());
}

template <typename TB, typename TA, typename TR>
void k_residual(const TB* b, const TA* ax, int64_t n, TR* r, double* partial, hipStream_t st) {
  hipLaunchKernelGGL((residual_kernel<TB, TA, TR>), dim3(grid_for(n)), dim3(kThreads), 0, st, b,
                     ax, n, r, partial);
  RT_HIP(hipGetLastError());
}

template <typename T>
void k_norm_partial(const T* x, int64_t n, double* partial, hipStream_t st) {
  hipLaunchKernelGGL((norm_kernel<T>), dim3(grid_for(n)), dim3(kThreads), 0, st, x, n, partial);
  RT_HIP(hipGetLastError());
}

void k_finish_norm(const double* partial, int64_t n, GmresState* gs, int start_cycle,
                   hipStream_t st) {
  hipLaunchKernelGGL(finish_norm_kernel, dim3(1), dim3(64), 0, st, partial, grid_for(n), gs,
                     start_cycle);
  RT_HIP(hipGetLastError());
}

void k_finish_norm_simple(const double* partial, int64_t n, double* out, hipStream_t st) {
  hipLaunchKernelGGL(finish_norm_simple_kernel, dim3(1), dim3(64), 0, st, partial, grid_for(n),
                     out);
  RT_HIP(hipGetLastError());
}

void k_givens(const double* partial, int64_t n, GmresState* gs, int j, double tol,
              hipStream_t st, double kdiag) {
  hipLaunchKernelGGL(givens_kernel, dim3(1), dim3(64), 0, st, partial, grid_update(n), gs, j,
                     tol, kdiag);
  RT_HIP(hipGetLastError());
}

template <typename TV>
void k_mdot2(const TV* V, int64_t n, int cnt, const TV* u1, const TV* u2, double* partial,
             hipStream_t st) {
  const int nb = grid_for(n);
  ProfScope prof(RT_KCLASS_ARNOLDI, st);
  for (int i0 = 0; i0 < cnt; i0 += 8) {
    const int c = cnt - i0 < 8 ? cnt - i0 : 8;
    hipLaunchKernelGGL((mdot2_kernel<TV, 8>), dim3(nb), dim3(kThreads), 0, st, V, n, i0, c, u1,
                       u2, partial);
  }
  RT_HIP(hipGetLastError());
}

void k_pair_coef(const double* partial, int64_t n, int j, const double* vscale, double* pair,
                 hipStream_t st) {
  hipLaunchKernelGGL(pair_coef_kernel, dim3(1), dim3(kThreads), 0, st, partial, grid_for(n), j,
                     vscale, pair);
  RT_HIP(hipGetLastError());
}

template <typename TV>
void k_update2(const TV* V, int64_t n, int cnt, const double* pair, TV* u1, TV* u2,
               double* partial, hipStream_t st) {
  ProfScope prof(RT_KCLASS_ARNOLDI, st);
  hipLaunchKernelGGL((update2_kernel<TV>), dim3(grid_update(n)), dim3(kThreads), 0, st, V, n,
                     cnt, pair, u1, u2, partial);
  RT_HIP(hipGetLastError());
}

template <typename TV>
void k_pair_fix(TV* p1, TV* z, int64_t n, double* pair, double* partial, hipStream_t st) {
  ProfScope prof(RT_KCLASS_ARNOLDI, st);
  hipLaunchKernelGGL(pair_rho_kernel, dim3(1), dim3(64), 0, st, partial, grid_update(n), pair);
  hipLaunchKernelGGL((pair_fix_kernel<TV>), dim3(grid_update(n)), dim3(kThreads), 0, st, p1, z,
                     n, pair, partial);
  RT_HIP(hipGetLastError());
}

void k_givens2(const double* partial, int64_t n, GmresState* gs, int j, double tol,
               const double* pair, double* hk, hipStream_t st, double kdiag, double sigma) {
  hipLaunchKernelGGL(givens2_kernel, dim3(1), dim3(64), 0, st, partial, grid_update(n), gs, j,
                     tol, pair, hk, kdiag, sigma);
  RT_HIP(hipGetLastError());
}

void k_solve_r(GmresState* gs, int k, hipStream_t st) {
  hipLaunchKernelGGL(solve_r_kernel, dim3(1), dim3(64), 0, st, gs, k);
  RT_HIP(hipGetLastError());
}

template <typename T>
void k_dots4(const T* a0, const T* b0, const T* a1, const T* b1, int cnt, int64_t n,
             double* partial, hipStream_t st) {
  hipLaunchKernelGGL((dots4_kernel<T>), dim3(grid_for(n)), dim3(kThreads), 0, st, a0, b0, a1, b1,
                     a0, b0, a0, b0, cnt, n, partial);
  RT_HIP(hipGetLastError());
}

template <typename T>
void k_bicg_p(const T* r, const T* v, T* p, int64_t n, const BicgState* bs, hipStream_t st) {
  hipLaunchKernelGGL((bicg_p_kernel<T>), dim3(grid_for(n)), dim3(kThreads), 0, st, r, v, p, n, bs);
  RT_HIP(hipGetLastError());
}

template <typename T>
void k_bicg_s(T* r, const T* v, int64_t n, const BicgState* bs, double* partial, hipStream_t st) {
  hipLaunchKernelGGL((bicg_s_kernel<T>), dim3(grid_for(n)), dim3(kThreads), 0, st, r, v, n, bs,
                     partial);
  RT_HIP(hipGetLastError());
}

template <typename T, typename TX>
void k_bicg_xr(TX* x, const T* p, T* r, const T* t, int64_t n, const BicgState* bs,
               int only_alpha, double* partial, hipStream_t st) {
  hipLaunchKernelGGL((bicg_xr_kernel<T, TX>), dim3(grid_for(n)), dim3(kThreads), 0, st, x, p, r,
                     t, n, bs, only_alpha, partial);
  RT_HIP(hipGetLastError());
}

void k_bicg_scalar(const double* partial, int64_t n, int stage, BicgState* bs, hipStream_t st) {
  hipLaunchKernelGGL(bicg_scalar_kernel, dim3(1), dim3(64), 0, st, partial, grid_for(n), stage,
                     bs);
  RT_HIP(hipGetLastError());
}

template <typename TS, typename TD>
void k_convert(const TS* a, TD* b, int64_t n, double scale, hipStream_t st) {
  hipLaunchKernelGGL((convert_kernel<TS, TD>), dim3(grid_for(n)), dim3(kThreads), 0, st, a, b, n,
                     scale);
  RT_HIP(hipGetLastError());
}

void k_axpy_f64(double* x, const float* d, int64_t n, const double* scale, hipStream_t st) {
  hipLaunchKernelGGL(axpy_f64_kernel, dim3(grid_for(n)), dim3(kThreads), 0, st, x, d, n, scale);
  RT_HIP(hipGetLastError());
}

int reduce_blocks(int64_t n) { return grid_for(n); }

// explicit instantiations
template void k_mdot<double>(const double*, int64_t, int, const double*, double*, hipStream_t);
template void k_mdot2<double>(const double*, int64_t, int, const double*, const double*, double*,
                              hipStream_t);
template void k_mdot2<float>(const float*, int64_t, int, const float*, const float*, double*,
                             hipStream_t);
template void k_update2<double>(const double*, int64_t, int, const double*, double*, double*,
                                double*, hipStream_t);
template void k_update2<float>(const float*, int64_t, int, const double*, float*, float*,
                               double*, hipStream_t);
template void k_pair_fix<double>(double*, double*, int64_t, double*, double*, hipStream_t);
template void k_pair_fix<float>(float*, float*, int64_t, double*, double*, hipStream_t);
template void k_mdot2<_Float16>(const _Float16*, int64_t, int, const _Float16*, const _Float16*,
                                double*, hipStream_t);
template void k_update2<_Float16>(const _Float16*, int64_t, int, const double*, _Float16*,
                                  _Float16*, double*, hipStream_t);
template void k_pair_fix<_Float16>(_Float16*, _Float16*, int64_t, double*, double*, hipStream_t);
template void k_mdot<float>(const float*, int64_t, int, const float*, double*, hipStream_t);
template void k_update<double>(const double*, int64_t, int, const double*, const double*, double*,
                               double*, hipStream_t);
template void k_update<float>(const float*, int64_t, int, const double*, const double*, float*,
                              double*, hipStream_t);
template void k_combine<double, double>(const double*, int64_t, int, const double*, double*,
                                        hipStream_t);
template void k_combine<float, float>(const float*, int64_t, int, const double*, float*,
                                      hipStream_t);
template void k_residual<double, double, double>(const double*, const double*, int64_t, double*,
                                                 double*, hipStream_t);
template void k_residual<double, double, float>(const double*, const double*, int64_t, float*,
                                                double*, hipStream_t);
template void k_residual<float, float, float>(const float*, const float*, int64_t, float*,
                                              double*, hipStream_t);
template void k_norm_partial<double>(const double*, int64_t, double*, hipStream_t);
template void k_norm_partial<float>(const float*, int64_t, double*, hipStream_t);
template void k_dots4<double>(const double*, const double*, const double*, const double*, int,
                              int64_t, double*, hipStream_t);
template void k_bicg_p<double>(const double*, const double*, double*, int64_t, const BicgState*,
                               hipStream_t);
template void k_bicg_s<double>(double*, const double*, int64_t, const BicgState*, double*,
                               hipStream_t);
template void k_bicg_xr<double, double>(double*, const double*, double*, const double*, int64_t,
                                        const BicgState*, int, double*, hipStream_t);
template void k_bicg_xr<float, float>(float*, const float*, float*, const float*, int64_t,
                                      const BicgState*, int, double*, hipStream_t);
template void k_dots4<float>(const float*, const float*, const float*, const float*, int,
                             int64_t, double*, hipStream_t);
template void k_bicg_p<float>(const float*, const float*, float*, int64_t, const BicgState*,
                              hipStream_t);
template void k_bicg_s<float>(float*, const float*, int64_t, const BicgState*, double*,
                              hipStream_t);
template void k_mdot<_Float16>(const _Float16*, int64_t, int, const _Float16*, double*,
                               hipStream_t);
template void k_update<_Float16>(const _Float16*, int64_t, int, const double*, const double*,
                                 _Float16*, double*, hipStream_t);
template void k_combine<_Float16, float>(const _Float16*, int64_t, int, const double*, float*,
                                         hipStream_t);
template void k_norm_partial<_Float16>(const _Float16*, int64_t, double*, hipStream_t);
template void k_convert<double, _Float16>(const double*, _Float16*, int64_t, double, hipStream_t);
template void k_convert<double, float>(const double*, float*, int64_t, double, hipStream_t);
template void k_convert<float, double>(const float*, double*, int64_t, double, hipStream_t);
template void k_convert<float, __hip_bfloat16>(const float*, __hip_bfloat16*, int64_t, double,
                                               hipStream_t);
template void k_convert<float, __half>(const float*, __half*, int64_t, double, hipStream_t);

}  // namespace rtsn
